"""The tree plan's bounds (host logic, no GPU): the proven bound on leaf jobs
and the depth-first stack bound hold for every outcome of the random splits.
Jobs are the leaves the tree kernels do not sample themselves (sparse and
with-replacement leaves of at most 32 values they do).

Tiny universes: exhaustive worst case over every value a split can take
(the hypergeometric / binomial supports), computed here from the tree's
rules alone (Fig. 1: a node splits iff n_v >= n0, at l = floor(N_v / 2);
with replacement a range of one element is a leaf).  Larger universes,
including ranges above 2^32: the oracle's trees for many seeds.  The plan is
read through dcs_debug_plan, which does no device work."""
from functools import lru_cache

import pytest

import oracle
import paper_1610_05141_amd as dcs
from tests.tree_jobs import FILL_PIECE, INLINE_MAX, LEAF_RANGE, jobs as tree_jobs


def worst_case(variant: int, N: int, n: int, n0: int, dense_ratio: int = 16):
    """(most leaf jobs, deepest internal node) over all split outcomes."""

    @lru_cache(maxsize=None)
    def go(Nv: int, nv: int, depth: int):
        if nv == 0:
            return 0, -1
        if variant == 1 and Nv == 1:
            return -(-nv // FILL_PIECE), -1
        if nv < n0 and Nv <= LEAF_RANGE:
            if variant == 1:
                inline = nv <= INLINE_MAX
            else:
                inline = nv <= INLINE_MAX and dense_ratio * nv < Nv
            return (0 if inline else 1), -1
        l = Nv // 2
        lo = 0 if variant == 1 else max(0, nv - (Nv - l))
        hi = nv if variant == 1 else min(nv, l)
        best_jobs, best_depth = 0, depth
        for L in range(lo, hi + 1):
            ja, da = go(l, L, depth + 1)
            jb, db = go(Nv - l, nv - L, depth + 1)
            best_jobs = max(best_jobs, ja + jb)
            best_depth = max(best_depth, da, db)
        return best_jobs, best_depth

    return go(N, n, 0)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n0", [2, 3, 4, 7])
def test_bounds_hold_for_every_outcome(variant, n0):
    """Every (n, N) with N <= 40 (n <= 24 with replacement): the proven bound
    is at least the most jobs any outcome gives, the capacity at least the
    bound unless the second round is planned, and the stack covers the
    deepest internal node below the cut."""
    for N in range(1, 41):
        for n in range(1, (N if variant == 0 else 24) + 1):
            jobs, deepest = worst_case(variant, N, n, n0)
            p = dcs.debug_plan(variant, n, N, n0=n0)
            assert p["leaf_bound"] >= jobs, (variant, n, N, n0, p, jobs)
            if not p["second_round"]:
                assert p["leaf_cap"] >= jobs
            if deepest >= p["cut"]:
                # one pending right child per level from the cut down
                assert p["stack_depth"] >= deepest - p["cut"] + 1, (n, N, n0, p, deepest)


@pytest.mark.parametrize("variant", [0, 1])
def test_bounds_hold_where_the_level_count_binds(variant):
    """Larger n0 and N up to 256: here the bound comes from the count of
    internal nodes per level (2I + 1 < n), not from n, in most cases."""
    binding = 0
    for N in (64, 100, 255, 256):
        for n0 in (8, 16, 40):
            for n in range(1, 65):
                if variant == 0 and n > N:
                    continue
                jobs, _ = worst_case(variant, N, n, n0)
                p = dcs.debug_plan(variant, n, N, n0=n0)
                assert p["leaf_bound"] >= jobs, (variant, n, N, n0, p, jobs)
                binding += p["leaf_bound"] < n
    assert binding > 200


def test_bound_reached_by_adversarial_outcome():
    """The count argument is not loose by more than a factor 2 on a case
    where one outcome makes a chain of nodes that each shed one leaf."""
    jobs, _ = worst_case(0, 1 << 10, 12, 2)
    p = dcs.debug_plan(0, 12, 1 << 10, n0=2)
    assert jobs <= p["leaf_bound"] <= 2 * jobs + 1


@pytest.mark.parametrize("variant", [0, 1])
def test_bounds_hold_with_leaves_of_either_kind(variant):
    """n0 = 40 (leaves of up to 39 values, some sampled by the tree kernels,
    some jobs, dense ones among them on the narrow ranges): every outcome."""
    for N in (1 << 12, 5000, 1 << 14):
        for n in range(40, 200, 7):
            jobs, _ = worst_case(variant, N, n, 40)
            p = dcs.debug_plan(variant, n, N, n0=40)
            assert p["leaf_bound"] >= jobs, (variant, n, N, p, jobs)


@pytest.mark.parametrize("n,N,n0", [
    (1 << 16, 1 << 40, 64), (5000, (1 << 34) + 123, 16), (1 << 14, 1 << 52, 256),
    (300, (1 << 45) + 7, 4), (1 << 18, (1 << 33) - 5, 4096), (1 << 20, 1 << 24, 512),
])
def test_bounds_hold_on_oracle_trees(n, N, n0):
    """Trees of the canonical definition (the oracle's splits, 4 seeds each),
    including range-forced levels above 2^32: jobs within the bound (and the
    capacity, without the second round), depth within the stack bound."""
    p = dcs.debug_plan(0, n, N, n0=n0)
    for seed in range(4):
        internal, leaves, depth_max = oracle.tree_stats(n, N, seed, n0=n0)
        jobs = tree_jobs(oracle, 0, n, N, seed, n0=n0)
        assert jobs <= leaves
        assert jobs <= p["leaf_bound"], (seed, jobs, p)
        if not p["second_round"]:
            assert jobs <= p["leaf_cap"]
        # internal nodes sit above the deepest node; a thread's stack holds at
        # most one entry per level between the cut and the last internal level
        assert depth_max - p["cut"] <= p["stack_depth"], (seed, depth_max, p)


def test_plan_choice():
    """Affordable bounds are used as the capacity (no second round); the
    headline-sized sample keeps the expected-case capacity with the second
    round; the bound never exceeds n."""
    small = dcs.debug_plan(0, 1 << 20, 1 << 32)
    assert not small["second_round"] and small["leaf_cap"] == small["leaf_bound"]
    big = dcs.debug_plan(0, 1 << 30, 1 << 48)
    assert big["second_round"] and big["leaf_cap"] < big["leaf_bound"]
    assert big["leaf_cap"] >= 4 * (1 << 30) // 4096
    wr = dcs.debug_plan(1, 1 << 28, 1 << 40)
    assert wr["leaf_bound"] >= wr["leaf_cap"] and wr["second_round"]
    for n, N in [(1, 1), (7, 7), (1 << 10, 1 << 62), (123456, 1 << 33)]:
        p = dcs.debug_plan(0, n, N, n0=2)
        assert p["leaf_bound"] <= n
        assert p["leaf_cap"] >= p["threads"] // 64 + 1
    # sparse over a huge universe: jobs only for leaves of 33 or more values
    g = dcs.debug_plan(0, 1 << 24, (1 << 30) * ((1 << 30) - 1) // 2)
    assert g["leaf_cap"] <= (1 << 24) // 33 + 1 and not g["second_round"]
