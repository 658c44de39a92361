"""Online sampling in parts (Sec. 4.1) on the GPU, through the C ABI: every
part of a cut equals the oracle's part bit for bit (values, count, rank),
the parts concatenate to the full GPU sample, a part that does not fit its
buffer writes nothing, and at the 8 GiB size sampled parts agree with the
oracle's counts, ranks and windows.
"""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu

# (n, N, seed, n0, depth, variant)
PART_CASES = [
    (1 << 20, 1 << 32, 1, 4096, 0, 0),       # depth 0: the whole sample
    (1 << 20, 1 << 32, 1, 4096, 3, 0),       # configuration 1 in 8 parts
    (200000, 1 << 30, 3, 256, 10, 0),        # leaves end most paths above the cut
    (123457, 10**9 + 7, 11, 4096, 5, 0),     # ragged ranges, void words
    (77777, 300000, 13, 64, 6, 0),           # dense leaves
    (300, 5000, 9, 4096, 2, 0),              # the root is a leaf: part 0 holds it all
    (5, 40, 7, 2, 5, 0),                     # empty nodes above the cut
    (100000, 2**40 + 3, 12, 512, 7, 0),      # range-forced depth below the cut
    (1 << 18, 1 << 40, 8, 4096, 4, 1),       # with replacement
    (3000, 7, 9, 64, 4, 1),                  # with replacement, N_v = 1 leaves
]


@pytest.mark.parametrize("n,N,seed,n0,depth,variant", PART_CASES)
def test_parts_match_oracle_and_concatenate(ref, n, N, seed, n0, depth, variant):
    import torch
    m = dcs()
    announce(f"parts n={n} N={N} seed={seed} n0={n0} depth={depth} variant={variant}")
    if variant == 0:
        full = m.sample(n, N, seed, n0=n0)
    else:
        full = m.sample_replacement(n, N, seed, n0=n0)
    buf = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
    cr = torch.zeros(2, dtype=torch.int64, device="cuda")
    pieces, rank = [], 0
    for g in range(1 << depth):
        m.sample_part(n, N, seed, depth, g, out=buf, capacity=n, count_rank=cr,
                      variant=variant, n0=n0)
        m.synchronize()
        count, r = (int(x) for x in cr.cpu())
        want, wc, wr = ref.part(variant, n, N, seed, depth, g, n0=n0)
        assert (count, r) == (wc, wr), (g, count, r, wc, wr)
        assert r == rank
        got = to_np_u64(buf[:count])
        assert np.array_equal(got, want), f"part {g}: {first_mismatch(got, want)}"
        pieces.append(got)
        rank += count
    assert rank == n
    cat = np.concatenate(pieces)
    f = to_np_u64(full)
    assert np.array_equal(cat, f), first_mismatch(cat, f)


def test_part_that_does_not_fit_writes_nothing(ref):
    import torch
    m = dcs()
    n, N, seed = 1 << 20, 1 << 32, 1
    announce("part overflow")
    _, wc, wr = ref.part(0, n, N, seed, 2, 1)
    buf = torch.full((wc - 1,), -7, dtype=torch.int64, device="cuda")
    cr = torch.zeros(2, dtype=torch.int64, device="cuda")
    m.sample_part(n, N, seed, 2, 1, out=buf, capacity=wc - 1, count_rank=cr)
    m.synchronize()
    assert [int(x) for x in cr.cpu()] == [wc, wr]
    assert bool((buf == -7).all())
    # the same part into a buffer that fits, twice in a row (workspace reuse)
    buf2 = torch.empty(wc, dtype=torch.int64, device="cuda")
    for _ in range(2):
        m.sample_part(n, N, seed, 2, 1, out=buf2, capacity=wc, count_rank=cr)
        m.synchronize()
        want, _, _ = ref.part(0, n, N, seed, 2, 1)
        got = to_np_u64(buf2)
        assert np.array_equal(got, want), first_mismatch(got, want)


def test_parts_of_the_8gib_sample(ref):
    """n = 2^30 of 2^48 cut at depth 6 (64 parts of about 128 MiB): sampled
    parts agree with the oracle's count and rank and with oracle windows of
    the full sample at their start, middle and end."""
    import torch
    m = dcs()
    n, N, seed, depth = 1 << 30, 1 << 48, 7, 6
    cap = (n >> depth) + (1 << 20)
    buf = torch.empty(cap, dtype=torch.int64, device="cuda")
    cr = torch.zeros(2, dtype=torch.int64, device="cuda")
    for g in (0, 1, 37, 63):
        announce(f"8 GiB sample, part {g} of depth {depth}")
        m.sample_part(n, N, seed, depth, g, out=buf, capacity=cap, count_rank=cr)
        m.synchronize()
        count, r = (int(x) for x in cr.cpu())
        _, wc, wr = ref.part(0, n, N, seed, depth, g, capacity=0)
        assert (count, r) == (wc, wr)
        d = buf[1:count] - buf[:count - 1]
        assert bool((d > 0).all())
        for s in (0, count // 2, count - 4096):
            want = ref.sample_window(n, N, seed, r + s, 4096)
            got = to_np_u64(buf[s:s + 4096])
            assert np.array_equal(got, want), f"part {g} at {s}: {first_mismatch(got, want)}"


@pytest.mark.parametrize("n,N,depth,index,variant", [
    (0, 100, 3, 5, 0),                   # empty sample: every part empty, rank 0
    (0, 100, 0, 0, 1),
    (200, 2**52, 45, 2**44 + 12345, 0),  # deepest cut, largest universe
    (200, 2**52, 45, 0, 0),              # its leftmost part holds the leaf above the cut
    (5000, 2**52, 40, 2**39, 1),         # with replacement, deep cut
    (30000, 2**62, 45, 2**44 + 3, 0),    # largest universe of the tree
    (30000, 2**61 + 7, 20, 77777, 1),    # with replacement above 2^53
])
def test_part_edge_cases(ref, n, N, depth, index, variant):
    import torch
    m = dcs()
    announce(f"part edge n={n} N={N} depth={depth} index={index} variant={variant}")
    buf = torch.full((max(n, 1),), -3, dtype=torch.int64, device="cuda")
    cr = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    m.sample_part(n, N, 9, depth, index, out=buf, capacity=max(n, 1), count_rank=cr,
                  variant=variant)
    m.synchronize()
    count, r = (int(x) for x in cr.cpu())
    want, wc, wr = ref.part(variant, n, N, 9, depth, index, capacity=max(n, 1))
    assert (count, r) == (wc, wr)
    got = to_np_u64(buf[:count])
    assert np.array_equal(got, want), first_mismatch(got, want)
