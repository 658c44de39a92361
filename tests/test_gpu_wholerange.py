"""Whole-range Algorithm B on the GPU (paper Sec. 2, 4.7, 5): the
library's dcs_sample_wholerange, called through the C ABI, against the
oracle, bit for bit -- small and ragged cases, rho = 1 with removals, many
chunks, and the benchmarked n = 2^29 of 2^30 whole."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu

CASES = [
    # (n, N, seed, n0)
    (1 << 20, 1 << 21, 7, None),
    (1000, 1017, 5, None),              # rho = 1, 17 removals
    (65_000, 65_536, 2, None),          # rho = 1, 536 removals
    (5000, 1 << 20, 3, None),           # sparse end: rho ~ 2^-7.6
    (500_000, 1_000_003, 4, 64),        # 245 chunks of 2^12
    (1 << 24, 1 << 24, 6, None),        # n = N
    ((1 << 24) - 1, 1 << 24, 8, None),  # N - 1
    (2, 40, 9, 16),                     # tiny
    (5_000_000, 1 << 32, 10, None),     # largest N
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_wholerange_bitexact(ref, case):
    n, N, seed, n0 = CASES[case]
    m = dcs()
    kw = {} if n0 is None else {"n0": n0}
    announce(f"dcs_sample_wholerange case {case}: n={n} N={N} seed={seed} n0={n0}")
    out = m.sample_wholerange(n, N, seed, **kw)
    m.synchronize()
    want, _ = ref.sample_wholerange(n, N, seed, **kw)
    got = to_np_u64(out)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_wholerange_benchmarked_size(ref):
    """n = 2^29 of 2^30, seed 7: the whole sample against the oracle."""
    m = dcs()
    n, N, seed = 1 << 29, 1 << 30, 7
    announce(f"dcs_sample_wholerange n=2^29 N=2^30 seed={seed}")
    out = m.sample_wholerange(n, N, seed)
    m.synchronize()
    got = to_np_u64(out)
    del out
    want, attempt = ref.sample_wholerange(n, N, seed)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_wholerange_refused():
    """Refused before anything is enqueued (the output buffer is real, so
    that a check that let a call through could not write elsewhere)."""
    import ctypes
    import torch
    m = dcs()
    L = m.lib()
    out = torch.zeros(16, dtype=torch.int64, device="cuda")
    p = ctypes.c_void_p(out.data_ptr())
    assert L.dcs_sample_wholerange(1, 1 << 20, 1, None, p, None) == m.DCS_ENOTSUP
    assert L.dcs_sample_wholerange(10, (1 << 32) + 1, 1, None, p, None) == m.DCS_EINVAL
    assert L.dcs_sample_wholerange(5, 4, 1, None, p, None) == m.DCS_EINVAL
    assert L.dcs_sample_wholerange(0, 100, 1, None, None, None) == m.DCS_OK
    m.synchronize()
    assert int(out.abs().sum().item()) == 0
