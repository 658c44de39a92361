"""The allocation-free entry point (GPU): dcs_sample_noalloc, called through
the C ABI, returns what dcs_sample_ex returns for the same arguments, on two
calls in a row (the second smaller, so that the shared static scratch still
holds the first call's contents), without allocating device memory; a call
that needs more scratch than the static array holds is refused before
anything is enqueued."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu


def _noalloc(m, n, N, seed, out, stream, n0=None):
    return m.lib().dcs_sample_noalloc(n, N, seed, m._params(n0, None), m._ptr(out),
                                      m._stream_handle(stream))


def _with_workspace(m, n, N, seed, out, stream, n0=None):
    import torch
    wsb = m.workspace_size(0, n, N, n0=n0)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    rc = m.lib().dcs_sample_ex(n, N, seed, m._params(n0, None), m._ptr(out), m._ptr(ws),
                               ctypes.c_size_t(wsb), m._stream_handle(stream))
    return rc, ws


CASES = [  # (n, N, seed, n0): the second call of each pair is smaller
    ((3_000_000, 1 << 40, 11, None), (70_001, 1 << 36, 12, None)),
    ((1 << 22, 1 << 23, 5, 1024), (5_000, 9_999, 6, None)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_matches_workspace_call(first, second):
    import torch
    m = dcs()
    s = torch.cuda.current_stream()
    for k, (n, N, seed, n0) in enumerate((first, second)):
        announce(f"dcs_sample_noalloc call {k}: n={n} N={N} seed={seed} n0={n0}")
        got = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        want = torch.full((n,), -2, dtype=torch.int64, device="cuda")
        assert _noalloc(m, n, N, seed, got, s, n0) == m.DCS_OK
        rc, ws = _with_workspace(m, n, N, seed, want, s, n0)
        assert rc == m.DCS_OK
        m.synchronize(s)
        a, b = to_np_u64(got), to_np_u64(want)
        assert np.array_equal(a, b), first_mismatch(a, b)
        assert np.all(np.diff(a.astype(np.int64)) > 0) and a[0] >= 1 and a[-1] <= N
        del ws


def test_noalloc_allocates_nothing():
    import torch
    m = dcs()
    s = torch.cuda.current_stream()
    n, N = 1 << 20, 1 << 44
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    announce("dcs_sample_noalloc warm-up, then three calls with device memory watched")
    assert _noalloc(m, n, N, 1, out, s) == m.DCS_OK
    m.synchronize(s)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for seed in (2, 3, 4):
        assert _noalloc(m, n - seed, N, seed, out, s) == m.DCS_OK
    m.synchronize(s)
    free1, _ = torch.cuda.mem_get_info()
    # any workspace the library allocated would take at least 64 MiB
    assert free1 >= free0 - (8 << 20), (free0, free1)


def test_noalloc_rejects_too_large():
    import torch
    m = dcs()
    n, N = 1 << 28, 1 << 48
    assert m.workspace_size(0, n, N) > m.NOALLOC_SCRATCH_BYTES
    out = torch.empty(1, dtype=torch.int64, device="cuda")  # never written
    announce("dcs_sample_noalloc beyond the static scratch: refused")
    assert _noalloc(m, n, N, 1, out, torch.cuda.current_stream()) == m.DCS_ENOMEM
    m.synchronize()
