"""Sampling over an uneven universe on the GPU (paper Sec. 4.3): the
library's dcs_sample_segments, called through the C ABI, against the
oracle, bit for bit, values and per-segment counts.

Small cases compare the whole sample; the large ones compare the counts of
every segment and the values of sampled segments, each computed by the
oracle alone (its segment tree for the counts, its plain sampler under the
segment's seed for the values)."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu

FIG3_L = [20, 15, 30, 5, 17, 25, 10, 22, 18, 12, 20, 15, 20]  # 13 PEs, N = 229

CASES = [
    # (lengths, n, seed, n0)
    (FIG3_L, 50, 7, 8),
    (FIG3_L, 229, 1, 16),                                    # every element
    ([5, 0, 6], 11, 3, None),
    ([0, 0, 0, 100, 0, 0, 0, 0], 7, 4, 2),                   # all but one empty
    ([1 << 30], 50_000, 5, None),                             # one segment
    ([1 << 20] * 16, 300_000, 6, 1024),                       # K a power of two
    ([3 << 30, 1 << 40, 7, 5 << 36, 0, 1 << 33, 11 << 38], 200_000, 8, None),  # ranges > 2^32
    ([4000, 9000, 1 << 16, 70001, 12345], 80_000, 9, None),   # dense segments
    (list(range(1, 1001)), 20_000, 10, 64),                   # ragged, K = 1000
]


def _lengths_rng(K, seed, lo=8, hi=34):
    r = np.random.default_rng(seed)
    return [int(x) for x in np.exp2(r.uniform(lo, hi, K)).astype(np.uint64)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_segments_bitexact(ref, case):
    L, n, seed, n0 = CASES[case]
    m = dcs()
    kw = {} if n0 is None else {"n0": n0}
    announce(f"dcs_sample_segments case {case}: K={len(L)} N={sum(L)} n={n} seed={seed} n0={n0}")
    out, cnt = m.sample_segments(n, L, seed, **kw)
    m.synchronize()
    want, want_c = ref.sample_segments(n, L, seed, **kw)
    got = to_np_u64(out)
    assert np.array_equal(got, want), first_mismatch(got, want)
    assert np.array_equal(to_np_u64(cnt[:len(L)]), want_c)


def test_segments_counts_only(ref):
    import torch
    m = dcs()
    L = _lengths_rng(5000, 3)
    announce("dcs_sample_segments n=0 with counts")
    cnt = torch.full((len(L),), -1, dtype=torch.int64, device="cuda")
    out, cnt = m.sample_segments(0, L, 1, counts=cnt)
    m.synchronize()
    assert int(cnt.abs().sum().item()) == 0


def _oracle_segment(ref, n_i, L_i, base, seed, D, i, n0=None):
    kw = {} if n0 is None else {"n0": n0}
    s_i = ref.stream_draw64(seed, (1 << D) + i, ref.P_SEGSEED, 0, 0)
    return ref.sample(n_i, L_i, s_i, **kw) + np.uint64(base)


@pytest.mark.parametrize("K,n,seed", [(4096, 1 << 26, 11), (1 << 16, 1 << 24, 12)])
def test_segments_large(ref, K, n, seed):
    """Many ragged segments (sizes log-uniform in [2^8, 2^34]): all K counts
    against the oracle's segment tree, the values of the first, last, largest
    and 40 random segments against the oracle's plain sampler."""
    m = dcs()
    L = _lengths_rng(K, seed)
    announce(f"dcs_sample_segments large: K={K} N={sum(L)} n={n} seed={seed}")
    out, cnt = m.sample_segments(n, L, seed)
    m.synchronize()
    _, heap_cnt = ref.segment_tree(n, L, seed)
    D = max(0, (K - 1).bit_length())
    want_c = heap_cnt[(1 << D):(1 << D) + K]
    got_c = to_np_u64(cnt[:K])
    assert np.array_equal(got_c, want_c), first_mismatch(got_c, want_c)
    off = np.concatenate([[0], np.cumsum(want_c.astype(np.int64))])
    base = np.concatenate([[0], np.cumsum(np.asarray(L, dtype=np.int64))])
    r = np.random.default_rng(seed)
    pick = {0, K - 1, int(np.argmax(L))} | {int(x) for x in r.integers(0, K, 40)}
    for i in sorted(pick):
        ni = int(want_c[i])
        want = _oracle_segment(ref, ni, L[i], int(base[i]), seed, D, i)
        got = to_np_u64(out[off[i]:off[i] + ni])
        assert np.array_equal(got, want), (i, first_mismatch(got, want))
    v = to_np_u64(out)
    assert np.all(np.diff(v.astype(np.int64)) > 0) and v[0] >= 1 and int(v[-1]) <= sum(L)


def test_segments_rejects_bad_arguments():
    """Refused before anything is enqueued; the output buffer is real, so
    that a check that let a call through could not write elsewhere."""
    import ctypes
    import torch
    m = dcs()
    out = torch.zeros(16, dtype=torch.int64, device="cuda")
    p = ctypes.c_void_p(out.data_ptr())
    L = (ctypes.c_uint64 * 2)(1 << 62, 1)  # sum above the largest universe
    assert m.lib().dcs_sample_segments(1, L, 2, 1, None, p, None, None) == m.DCS_EINVAL
    L1 = (ctypes.c_uint64 * 1)(10)
    assert m.lib().dcs_sample_segments(11, L1, 1, 1, None, p, None, None) == m.DCS_EINVAL
    assert m.lib().dcs_sample_segments(1, L1, 0, 1, None, p, None, None) == m.DCS_EINVAL
    m.synchronize()
    assert int(out.abs().sum().item()) == 0
