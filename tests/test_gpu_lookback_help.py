"""The Bernoulli look-back's self-help on the GPU: a wave that waits for a
predecessor chunk that has published nothing counts that chunk itself.
The test hook makes waves do so after a single poll, so nearly every wait of
the chunk prefix sums (Sec. 4.7) takes that path, in both kernels (single-
and double-precision skips) and in G(n, p); every sample and count must still
equal the oracle's bit for bit."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu

CASES = [
    # (p, N, seed, n0)
    (0.01, 1 << 28, 41, None),     # single precision, 1024 chunks
    (0.25, 1 << 26, 42, 64),       # many short chunks: long look-back chains
    (0.5, 1 << 22, 43, 2),         # chunks of 2^12, most written in two passes
    (2.0**-11, 1 << 30, 44, None), # double precision
    (2.0**-20, 1 << 44, 45, None), # double precision, chunks clamped at 2^32
    (2.0**-24, 1 << 42, 46, None), # double precision, one wave per chunk (~256 hits)
]


@pytest.fixture
def m():
    mod = dcs()
    mod.debug_lookback_help(1)
    yield mod
    mod.debug_lookback_help(0)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_bernoulli_with_waves_counting_predecessors(ref, m, case):
    p, N, seed, n0 = CASES[case]
    kw = {} if n0 is None else {"n0": n0}
    announce(f"look-back help after 1 poll: bernoulli p={p} N={N} seed={seed} n0={n0}")
    out, cnt = m.sample_bernoulli(p, N, seed, **kw)
    m.synchronize()
    c = int(cnt.item())
    want = ref.bernoulli(p, N, seed, **kw)
    assert c == want.size
    got = to_np_u64(out[:c])
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_gnp_with_waves_counting_predecessors(ref, m):
    nv, p, seed = 1 << 14, 0.003, 46
    announce(f"look-back help after 1 poll: G(n,p) n={nv} p={p}")
    uv, cnt = m.sample_edges_gnp(nv, p, seed)
    m.synchronize()
    c = int(cnt.item())
    want = ref.edges_gnp(nv, p, seed)
    assert c == want.shape[0]
    got = uv[:c].cpu().numpy().astype(np.uint32)
    assert np.array_equal(got, want)
