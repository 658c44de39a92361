"""Online sampling sessions on the GPU (Sec. 4.1): dcs_online_create /
dcs_online_next through the C ABI.  The parts' counts and ranks equal the
oracle's parts of the same cut; streaming the parts in runs of any length
gives the oracle's whole sample, bit for bit."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu

CASES = [
    # (variant, n, N, seed, depth, n0)
    (0, 100_000, 1 << 40, 3, 6, None),
    (0, 50_000, 123_456_789, 4, 10, 64),        # leaves above the cut, ragged ranges
    (1, 80_000, 1 << 33, 5, 8, 128),
    (0, 2000, 2500, 6, 12, 16),                  # dense, most parts empty or inside leaves
    (1, 5000, 7, 9, 5, None),                    # ranges of one element and empty ones
    (0, 70_000, (1 << 36) + 5, 10, 0, None),     # depth 0: one part
    (0, 0, 1000, 11, 4, None),                   # nothing to sample
]


def _want(ref, variant, n, N, seed, n0):
    kw = {} if n0 is None else {"n0": n0}
    return ref.replacement(n, N, seed, **kw) if variant else ref.sample(n, N, seed, **kw)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_online_parts_and_stream(ref, case):
    import torch
    m = dcs()
    variant, n, N, seed, depth, n0 = CASES[case]
    announce(f"online session case {case}: variant={variant} n={n} N={N} seed={seed} depth={depth}")
    o = m.Online(n, N, seed, depth, variant=variant, n0=n0)
    counts, ranks = o.counts()
    assert int(counts.sum()) == n
    assert np.array_equal(ranks, np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.uint64))
    kw = {} if n0 is None else {"n0": n0}
    r = np.random.default_rng(case)
    for g in sorted({0, o.parts - 1} | {int(x) for x in r.integers(0, o.parts, 12)}):
        vals, c, rk = ref.part(variant, n, N, seed, depth, g, **kw)
        assert (c, rk) == (int(counts[g]), int(ranks[g])), g
    want = _want(ref, variant, n, N, seed, n0)
    for run in (1, 7, o.parts):
        out = torch.full((max(n, 1),), -1, dtype=torch.int64, device="cuda")
        pos = 0
        for g in range(0, o.parts, run):
            k = min(run, o.parts - g)
            w = o.next(g, k, out[pos:] if pos < n else out[:0])
            pos += w
        m.synchronize()
        assert pos == n
        got = to_np_u64(out[:n])
        assert np.array_equal(got, want), (run, first_mismatch(got, want))
    o.close()


def test_online_rejects_bad_arguments():
    import torch
    m = dcs()
    o = m.Online(1000, 1 << 20, 1, 4)
    counts, _ = o.counts()
    small = torch.zeros(1, dtype=torch.int64, device="cuda")
    big = int(counts[:8].sum())
    with pytest.raises(m.DcsError) as e:
        o.next(0, 8, small)  # the parts hold more than one value
    assert e.value.code == m.DCS_ENOMEM
    with pytest.raises(m.DcsError):
        o.next(10, 7, small)  # beyond 2^4 parts
    with pytest.raises(m.DcsError):
        m.Online(10, 5, 1, 4)  # n > N
    with pytest.raises(m.DcsError):
        m.Online(10, 50, 1, 21)  # depth above the limit
    m.synchronize()
    assert int(small.item()) == 0 and big > 1
    o.close()


def test_online_full_size_stream(ref):
    """n = 2^30 of N = 2^48 (seed 7) at depth 8, in runs of 16 parts into one
    reused buffer: every run ascending and continuing the previous one, all
    runs together n values; the first and last runs' heads and tails, and a
    middle run, against the oracle's windows of the whole sample."""
    import torch
    m = dcs()
    n, N, seed, depth = 1 << 30, 1 << 48, 7, 8
    announce("online session n=2^30 N=2^48 depth 8")
    o = m.Online(n, N, seed, depth)
    counts, ranks = o.counts()
    assert int(counts.sum()) == n
    run = 16
    cap = max(int(counts[g:g + run].sum()) for g in range(0, o.parts, run))
    buf = torch.empty(cap, dtype=torch.int64, device="cuda")
    prev_last = 0
    check = {0, o.parts // 2, o.parts - run}
    for g in range(0, o.parts, run):
        w = o.next(g, run, buf)
        x = buf[:w]
        assert bool((x[1:] > x[:-1]).all().item())
        assert int(x[0].item()) > prev_last
        prev_last = int(x[-1].item())
        if g in check:
            start = int(ranks[g])
            for off in (0, w - 4096):
                want = ref.sample_window(n, N, seed, start + off, 4096)
                got = to_np_u64(x[off:off + 4096])
                assert np.array_equal(got, want), (g, off, first_mismatch(got, want))
    m.synchronize()
    assert prev_last <= N
    o.close()
