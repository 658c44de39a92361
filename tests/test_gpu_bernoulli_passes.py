"""Double-precision Bernoulli chunks (p < 2^-10, Sec. 4.7's skips in FP64)
whose hits overflow the LDS position list: the first `words` positions are
written from LDS after the look-back and the rest by a second pass that
recomputes the chunk's draws.  The list size is forced through the
library's test hook (it never changes a sample); 1-1024 words select the
one-wave kernel, more the work-group kernel.  Samples and counts against the
oracle, bit for bit."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu


@pytest.fixture
def m():
    mod = dcs()
    yield mod
    mod.debug_bernoulli_list(0)


CASES = [
    # (p, N, seed, words): chunk length 2^min(32, floor(log2(4096 / p)))
    (2.0**-23, 1 << 40, 51, 64),     # one wave, 2^32 chunks of ~512 hits
    (2.0**-11, 1 << 30, 52, 8),      # one wave, 2^23 chunks of ~4096 hits
    (2.0**-20, 1 << 40, 53, 1088),   # work-group kernel, ~4096 hits per chunk
    (2.0**-23, (1 << 38) + 12345, 54, 1024),  # one wave, ragged last chunk
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_second_pass_matches_oracle(ref, m, case):
    p, N, seed, words = CASES[case]
    m.debug_bernoulli_list(words)
    announce(f"bernoulli second pass: p={p!r} N={N} seed={seed} list={words}")
    out, cnt = m.sample_bernoulli(p, N, seed)
    m.synchronize()
    want = ref.bernoulli(p, N, seed)
    c = int(cnt.item())
    assert c == want.size
    got = to_np_u64(out[:c])
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_second_pass_gnp(ref, m):
    """G(n, p) below 2^-10 with the list forced short."""
    nv, p, seed = 1 << 16, 2.0**-14, 55
    m.debug_bernoulli_list(64)
    announce(f"bernoulli second pass: G(n,p) n={nv} p={p!r} list=64")
    uv, cnt = m.sample_edges_gnp(nv, p, seed)
    m.synchronize()
    c = int(cnt.item())
    want = ref.edges_gnp(nv, p, seed)
    assert c == want.shape[0]
    assert np.array_equal(uv[:c].cpu().numpy().astype(np.uint32), want)


def test_list_size_rejected_above_limit():
    mod = dcs()
    with pytest.raises(mod.DcsError):
        mod.debug_bernoulli_list(8257)
    mod.debug_bernoulli_list(0)
