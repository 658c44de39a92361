"""Serving (GPU): continuous batching with admission by output footprint.

Each request's output must equal the same request sampled alone (and the
oracle's), whatever shared its batch; admission must hold back requests until
arena space is released."""
import numpy as np
import pytest

from paper_1610_05141_amd.workloads import batched_instances, poisson_arrivals
from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu


def test_server_mix_equals_alone(ref):
    import torch
    m = dcs()
    insts = batched_instances(240, n_lo_log2=4, n_hi_log2=17, key=1234)
    reqs = [(x.n, x.N, x.seed, i % 4 == 3) for i, x in enumerate(insts)]
    announce(f"server mix, {len(reqs)} requests")
    srv = m.Server(arena_bytes=1 << 30, max_batch=32, n_streams=3, auto_release=False)
    t0 = m.Server.now() + 0.01
    arrivals = [t0 + t for t in poisson_arrivals(len(reqs), 4000.0, key=99)]
    first = srv.submit_schedule([(n, N, s, int(v)) for n, N, s, v in reqs], arrivals)
    srv.drain()
    st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["batches"] >= 2
    alone = torch.empty(max(r[0] for r in reqs), dtype=torch.int64, device="cuda")
    for i, (n, N, s, v) in enumerate(reqs):
        got = srv.result(first + i, n)
        (m.sample_replacement if v else m.sample)(n, N, s, out=alone)
        m.synchronize()
        assert torch.equal(got, alone[:n]), f"request {i} differs from sampling it alone"
        if i % 20 == 0:
            want = ref.replacement(n, N, s) if v else ref.sample(n, N, s)
            g = to_np_u64(got)
            assert np.array_equal(g, want), first_mismatch(g, want)
        srv.release(first + i)
    srv.close()


def test_server_admission_under_pressure():
    """A 2 MiB arena and requests of 8 KiB..1 MiB: later requests can only be
    admitted after earlier results are released."""
    import torch
    m = dcs()
    announce("server admission burst")
    srv = m.Server(arena_bytes=2 << 20, max_batch=8, n_streams=2, auto_release=False)
    sizes = [1 << 17, 1000, 1 << 16, 3, 1 << 17, 77777, 1 << 17, 5, 1 << 16, 1 << 17] * 3
    tickets = [srv.submit(n, 10**12 + 39, 1000 + i) for i, n in enumerate(sizes)]
    pending = dict(zip(tickets, range(len(sizes))))
    alone = torch.empty(max(sizes), dtype=torch.int64, device="cuda")
    import time
    deadline = time.time() + 60
    while pending and time.time() < deadline:
        for tk in list(pending):
            st, _, _ = srv.poll(tk)
            if st == 2:
                i = pending.pop(tk)
                got = srv.result(tk, sizes[i])
                m.sample(sizes[i], 10**12 + 39, 1000 + i, out=alone)
                m.synchronize()
                assert torch.equal(got, alone[:sizes[i]])
                srv.release(tk)
        time.sleep(0.001)
    assert not pending, f"{len(pending)} requests never completed"
    srv.close()


def test_schedule_rejects_invalid_request_and_keeps_tickets():
    """A schedule with an invalid request (n0 above 4096) is refused whole;
    a valid schedule's request i has ticket first + i even when plain
    submissions arrive while it is being fed."""
    import torch
    m = dcs()
    announce("server schedule validation and ticket order")
    srv = m.Server(arena_bytes=1 << 28, max_batch=16, n_streams=2, auto_release=False)
    bad = [(1000, 1 << 30, 1), (1000, 1 << 30, 2, 0, 5000), (1000, 1 << 30, 3)]
    t0 = m.Server.now()
    with pytest.raises(m.DcsError):
        srv.submit_schedule(bad, [t0, t0, t0])
    reqs = [(500 + 37 * i, 1 << 34, 100 + i) for i in range(40)]
    arrivals = [m.Server.now() + 0.002 * i for i in range(len(reqs))]
    first = srv.submit_schedule(reqs, arrivals)
    extra = [srv.submit(777, 1 << 20, 5000 + k) for k in range(5)]
    assert all(t >= first + len(reqs) for t in extra)
    srv.drain()
    assert srv.stats()["completed"] == len(reqs) + len(extra)
    for i, (n, N, s) in enumerate(reqs):
        got = srv.result(first + i, n)
        alone = m.sample(n, N, s)
        m.synchronize()
        assert torch.equal(got, alone), f"ticket {first + i} is not request {i}"
    for k, tk in enumerate(extra):
        got = srv.result(tk, 777)
        alone = m.sample(777, 1 << 20, 5000 + k)
        m.synchronize()
        assert torch.equal(got, alone)
    srv.close()
