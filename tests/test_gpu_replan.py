"""Leaf-job capacity overflow on the GPU: detected, recovered on the device by
the second round, and, when the second round runs out too, reported with the
later plans enlarged (the plan row of the hot path: "overflow is detected,
flagged and re-planned").

The capacity is forced through the library's test hook to just below the
number of leaf jobs of the call's canonical tree, counted from the oracle's
splits (leaves the tree kernels do not sample themselves).  Every output is
compared bit for bit with the oracle."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64
from tests.tree_jobs import jobs as tree_jobs

pytestmark = pytest.mark.gpu


@pytest.fixture
def m():
    mod = dcs()
    yield mod
    mod.debug_leaf_capacity(0, reset_boost=True)


def wor_jobs(ref, n, N, seed, n0):
    return tree_jobs(ref, 0, n, N, seed, n0=n0)


def wr_jobs(ref, n, N, seed, n0):
    return tree_jobs(ref, 1, n, N, seed, n0=n0)


WOR = [
    # (n, N, seed, n0): sparse leaves over power-of-two ranges; dense leaves
    # over ranges that are not; a range above 2^32
    (200_000, 1 << 40, 3, 64),
    (300_000, 5_000_000, 4, 256),
    (60_000, (1 << 34) + 12345, 5, 128),
]
WR = [
    (50_000, 1 << 36, 6, 128),
    (300_000, 3, 7, 4096),        # constant leaves cut into pieces
    (120_000, 1000, 8, 64),
]


def _short_caps(jobs):
    return [jobs - 1, jobs - max(2, jobs // 32)]


@pytest.mark.parametrize("case", range(len(WOR)))
def test_second_round_recovers_without_replacement(ref, m, case):
    n, N, seed, n0 = WOR[case]
    jobs = wor_jobs(ref, n, N, seed, n0)
    want = ref.sample(n, N, seed, n0=n0)
    for cap in _short_caps(jobs):
        announce(f"forced capacity {cap} of {jobs} jobs: n={n} N={N} seed={seed} n0={n0}")
        m.debug_leaf_capacity(cap)
        out = m.sample(n, N, seed, n0=n0)
        m.synchronize()
        got = to_np_u64(out)
        assert np.array_equal(got, want), (cap, first_mismatch(got, want))
    assert m.debug_leaf_capacity(0) == 1  # recovered: nothing enlarged


@pytest.mark.parametrize("case", range(len(WR)))
def test_second_round_recovers_with_replacement(ref, m, case):
    n, N, seed, n0 = WR[case]
    jobs = wr_jobs(ref, n, N, seed, n0)
    want = ref.replacement(n, N, seed, n0=n0)
    for cap in _short_caps(jobs):
        announce(f"forced capacity {cap} of {jobs} jobs (wr): n={n} N={N} seed={seed} n0={n0}")
        m.debug_leaf_capacity(cap)
        out = m.sample_replacement(n, N, seed, n0=n0)
        m.synchronize()
        got = to_np_u64(out)
        assert np.array_equal(got, want), (cap, first_mismatch(got, want))


def test_second_round_allocation_free_and_batch(ref, m):
    """The allocation-free entry point and a batch take the same rounds."""
    import torch
    n, N, seed, n0 = WOR[0]
    jobs = wor_jobs(ref, n, N, seed, n0)
    m.debug_leaf_capacity(jobs - 3)
    announce(f"forced capacity {jobs - 3} of {jobs}: dcs_sample_noalloc")
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    m.sample_noalloc(n, N, seed, out, n0=n0)
    m.synchronize()
    want = ref.sample(n, N, seed, n0=n0)
    assert np.array_equal(to_np_u64(out), want)

    insts = [(90_000, 1 << 38, 11, 128, 0), (40_000, 777_777, 12, 32, 0), (70_000, 1 << 30, 13, 128, 1)]
    total_jobs = sum(wr_jobs(ref, a, b, c, d) if v else wor_jobs(ref, a, b, c, d)
                     for a, b, c, d, v in insts)
    per = (total_jobs - 3) // len(insts)  # the batch holds len(insts) * per slots
    m.debug_leaf_capacity(per)
    specs, off = [], 0
    for a, b, c, d, v in insts:
        specs.append(m.InstanceSpec(n=a, N=b, seed=c, out_offset=off, variant=v, n0=d))
        off += a
    announce(f"forced capacity {per} per instance of {total_jobs} jobs: batch of {len(insts)}")
    bt = m.Batch(specs)
    out = torch.full((off,), -1, dtype=torch.int64, device="cuda")
    bt.run(out)
    m.synchronize()
    got = to_np_u64(out)
    for s, (a, b, c, d, v) in zip(specs, insts):
        want = ref.replacement(a, b, c, n0=d) if v else ref.sample(a, b, c, n0=d)
        g = got[s.out_offset:s.out_offset + a]
        assert np.array_equal(g, want), ((a, b, c, d, v), first_mismatch(g, want))
    bt.close()


def test_second_round_segments(ref, m):
    """An uneven universe: the jobs of all segments' trees share one array."""
    L = [3 << 20, 5_000_000, 1 << 33, 12345, 9 << 22]
    n, seed, n0 = 150_000, 21, 128
    _, heap = ref.segment_tree(n, L, seed)
    D = max(0, (len(L) - 1).bit_length())
    counts = heap[(1 << D):(1 << D) + len(L)]
    jobs = 0
    for i, (ni, Li) in enumerate(zip(counts, L)):
        si = ref.stream_draw64(seed, (1 << D) + i, ref.P_SEGSEED, 0, 0)
        if ni:
            jobs += wor_jobs(ref, int(ni), Li, si, n0)
    m.debug_leaf_capacity(jobs - 2)
    announce(f"forced capacity {jobs - 2} of {jobs} jobs: segments K={len(L)}")
    out, cnt = m.sample_segments(n, L, seed, n0=n0)
    m.synchronize()
    want, want_c = ref.sample_segments(n, L, seed, n0=n0)
    assert np.array_equal(to_np_u64(out), want)
    assert np.array_equal(to_np_u64(cnt[:len(L)]), want_c)


def test_both_rounds_short_reports_and_enlarges(ref, m):
    """Capacity far below the jobs: the second round runs out too, the call
    reports DCS_EDEVICE at synchronize, the multiplier of later expected-case
    capacities goes up, and the next call (normal plan) is exact."""
    n, N, seed, n0 = WOR[0]
    m.debug_leaf_capacity(1)
    announce("forced capacity 1: both rounds short")
    m.sample(n, N, seed, n0=n0)
    with pytest.raises(m.DcsError) as e:
        m.synchronize()
    assert e.value.code == m.DCS_EDEVICE
    assert m.debug_leaf_capacity(0) == 4
    announce("normal plan after the reported overflow")
    out = m.sample(n, N, seed, n0=n0)
    m.synchronize()
    assert np.array_equal(to_np_u64(out), ref.sample(n, N, seed, n0=n0))
