"""Caller workspaces and error reporting (GPU).

A workspace passed to an _ex call is only that call's scratch: whatever it
held before does not leak into the result or into dcs_synchronize, and once
the call has completed the library never reads or writes that memory again
(its error words are its own)."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu


def test_prefilled_workspace_then_reused_memory(ref):
    import torch
    m = dcs()
    n, N, seed = 50_000, 1 << 40, 5
    wsb = m.workspace_size(0, n, N)
    announce(f"caller workspace of {wsb} bytes prefilled with 0xFF")
    ws = torch.full((wsb,), 0xFF, dtype=torch.uint8, device="cuda")
    out = m.sample(n, N, seed, workspace=ws)
    m.synchronize()  # raises if a stale word were taken for a latched error
    want = ref.sample(n, N, seed)
    got = to_np_u64(out)
    assert np.array_equal(got, want), first_mismatch(got, want)
    addr = ws.data_ptr()
    del ws
    # the caching allocator hands the same block back for the same size
    reused = torch.full((wsb,), 0x5A, dtype=torch.uint8, device="cuda")
    assert reused.data_ptr() == addr, "allocator did not reuse the block (test premise)"
    torch.cuda.synchronize()
    for k in range(3):
        m.sample(4096 + k, 1 << 30, k)  # library workspace
        m.synchronize()
    assert bool((reused == 0x5A).all()), "library wrote into memory it no longer owns"


def test_prefilled_workspace_bernoulli_and_replacement(ref):
    import torch
    m = dcs()
    p, N, seed = 0.02, 1 << 22, 9
    wsb = m.workspace_size(2, 0, N, p)
    announce("Bernoulli and with-replacement calls on prefilled workspaces")
    ws = torch.full((wsb,), 0xFF, dtype=torch.uint8, device="cuda")
    out, cnt = m.sample_bernoulli(p, N, seed, workspace=ws)
    m.synchronize()
    want = ref.bernoulli(p, N, seed)
    c = int(cnt.item())
    assert c == want.size
    got = to_np_u64(out[:c])
    assert np.array_equal(got, want), first_mismatch(got, want)
    n, N2 = 30_000, 1 << 33
    ws2 = torch.full((m.workspace_size(1, n, N2),), 0xFF, dtype=torch.uint8, device="cuda")
    out2 = m.sample_replacement(n, N2, seed, workspace=ws2)
    m.synchronize()
    want2 = ref.replacement(n, N2, seed)
    got2 = to_np_u64(out2)
    assert np.array_equal(got2, want2), first_mismatch(got2, want2)


def test_synchronize_per_stream():
    """Each stream's synchronize reports only its own calls: clean calls on
    several streams, each synchronized separately, all report success."""
    import torch
    m = dcs()
    announce("calls on four streams, synchronized one by one")
    streams = [torch.cuda.Stream() for _ in range(4)]
    outs = []
    for i, s in enumerate(streams):
        wsb = m.workspace_size(0, 20_000, 1 << 36)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        with torch.cuda.stream(s):
            outs.append((m.sample(20_000, 1 << 36, i, stream=s, workspace=ws), ws))
    for s in streams:
        m.synchronize(s)
    for i, (o, _) in enumerate(outs):
        alone = m.sample(20_000, 1 << 36, i)
        m.synchronize()
        assert torch.equal(o, alone)
