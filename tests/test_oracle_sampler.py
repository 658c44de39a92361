"""Pins for the oracle's samplers (CPU only): brute force over every subset on
tiny universes, exact hypergeometric laws of prefix counts, the equivalence of
Algorithm H's sequential rule with the round-based rule, Bernoulli and
with-replacement laws, and the structural invariants of Sec. 3 and Sec. 4.1.
"""
import itertools
import math
from collections import Counter

import mpmath
import numpy as np
import pytest

from tests.test_oracle_primitives import _chisq_pvalue


def _subset_chisq(ref, N, n, n0, dense_ratio, seeds):
    subsets = list(itertools.combinations(range(1, N + 1), n))
    index = {s: i for i, s in enumerate(subsets)}
    obs = np.zeros(len(subsets))
    for seed in range(seeds):
        s = ref.sample(n, N, seed, n0=n0, dense_ratio=dense_ratio)
        t = tuple(int(x) for x in s)
        assert t in index, t  # sorted, distinct, in range
        obs[index[t]] += 1
    return _chisq_pvalue(obs, np.full(len(subsets), 1.0 / len(subsets)))


# (N, n, n0, dense_ratio): dense_ratio 2 forces sparse leaves on tiny ranges,
# 16 (the default) makes them dense; small n0 forces splits.
BRUTE_CASES = [
    (8, 3, 2, 16),
    (8, 3, 2, 2),
    (12, 5, 2, 2),
    (12, 5, 3, 16),
    (16, 8, 4, 16),
    (10, 9, 2, 16),
    (20, 3, 4, 2),    # one sparse leaf: Algorithm H alone
    (20, 3, 4, 16),   # one dense leaf: geometric skips + repair
    (13, 6, 8, 16),   # dense leaf with rho = 1: repair only
    (11, 4, 2, 2),    # odd sizes at every level
]


@pytest.mark.parametrize("N,n,n0,dr", BRUTE_CASES)
def test_uniform_over_all_subsets(ref, N, n, n0, dr):
    cells = math.comb(N, n)
    seeds = max(20000, 40 * cells)
    assert _subset_chisq(ref, N, n, n0, dr, seeds) > 1e-4


def test_degenerate_samples(ref):
    assert ref.sample(0, 10, 1).size == 0
    assert ref.sample(0, 0, 1).size == 0
    np.testing.assert_array_equal(ref.sample(10, 10, 3, n0=4), np.arange(1, 11, dtype=np.uint64))
    np.testing.assert_array_equal(ref.sample(5000, 5000, 3), np.arange(1, 5001, dtype=np.uint64))
    assert ref.sample(1, 1, 9).tolist() == [1]
    with pytest.raises(RuntimeError):
        ref.sample(11, 10, 1)
    with pytest.raises(RuntimeError):
        ref.sample(1, 2**62 + 1, 1)
    with pytest.raises(RuntimeError):
        ref.sample(1, 10, 1, n0=1)


def test_inclusion_marginals(ref):
    """Every element is included with probability n/N, every pair with
    n(n-1)/(N(N-1)) (uniform subsets), across sparse and dense leaves."""
    for N, n, n0, dr in [(64, 20, 4, 2), (64, 20, 4, 16), (50, 45, 4, 16)]:
        seeds = 20000
        inc = np.zeros(N + 1)
        pair = 0
        for seed in range(seeds):
            s = ref.sample(n, N, seed, n0=n0, dense_ratio=dr).astype(np.int64)
            inc[s] += 1
            pair += (1 in s) and (N in s)
        p = n / N
        z = (inc[1:] - seeds * p) / math.sqrt(seeds * p * (1 - p))
        assert np.abs(z).max() < 4.5
        pp = n * (n - 1) / (N * (N - 1))
        assert abs(pair - seeds * pp) / math.sqrt(seeds * pp * (1 - pp)) < 4.5


@pytest.mark.parametrize("n,N,n0", [(5000, 1_000_007, 256), (5000, 12_001, 256),
                                    (3000, 2**40 + 3, 512)])
def test_prefix_counts_are_hypergeometric(ref, n, N, n0):
    """Sec. 3: for ANY split position x the number of samples in 1..x is
    Hyp(n, x, N) -- tested at cut points that are not tree boundaries."""
    seeds = 1500
    cuts = [1, N // 7, N // 3 + 11, N // 2 + 1, N - N // 5, N - 2]
    counts = {x: [] for x in cuts}
    for seed in range(seeds):
        s = ref.sample(n, N, seed + 1000, n0=n0)
        for x in cuts:
            counts[x].append(int(np.searchsorted(s, x, side="right")))
    mpmath.mp.dps = 40
    lg = mpmath.loggamma
    for x in cuts:
        c = np.array(counts[x])
        mu = n * x / N
        sd = math.sqrt(max(mu * (1 - x / N) * (N - n) / (N - 1), 1e-12))
        lo = max(0, n - (N - x), int(mu - 9 * sd) - 1)
        hi = min(n, x, int(mu + 9 * sd) + 2)
        ks = np.arange(lo, hi + 1)
        base = lg(x + 1) + lg(N - x + 1) + lg(n + 1) + lg(N - n + 1) - lg(N + 1)
        pmf = np.array([float(mpmath.exp(base - lg(k + 1) - lg(x - k + 1) - lg(n - k + 1)
                                         - lg(N - x - n + k + 1))) for k in ks])
        pmf[0] += max(0.0, 1.0 - pmf.sum())  # the (negligible) mass beyond +-9 sd
        obs = np.bincount(np.clip(c, lo, hi) - lo, minlength=len(ks))
        assert _chisq_pvalue(obs, pmf) > 1e-4, x


def test_invariants_config1(ref):
    n, N = 1 << 20, 1 << 32
    s = ref.sample(n, N, 1)
    assert s.dtype == np.uint64 and s.size == n
    d = np.diff(s.astype(np.int64))
    assert (d > 0).all()
    assert int(s[0]) >= 1 and int(s[-1]) <= N
    # the sample's spread is that of a uniform subset (order statistics)
    assert abs(int(s[n // 2]) - N // 2) < 10 * N / math.sqrt(n)


def test_window_equals_slice(ref):
    n, N = 1 << 20, 1 << 32
    full = ref.sample(n, N, 1)
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = int(rng.integers(0, n))
        c = int(rng.integers(0, min(70000, n - a) + 1))
        np.testing.assert_array_equal(ref.sample_window(n, N, 1, a, c), full[a:a + c])
    np.testing.assert_array_equal(ref.sample_window(n, N, 1, n - 5, 5), full[-5:])


def test_root_split_position_and_stream(ref):
    """Fig. 1 splits 1..N at floor(N/2) and the left part receives the root's
    hypergeometric draw: the number of sampled values <= floor(N/2) equals
    Hyp(n, floor(N/2), N) from the root's stream (node id 1)."""
    for n, N, seed, n0 in [(5000, 10**6 + 7, 3, 256), (7, 21, 5, 2), (300, 2**33 + 1, 9, 64),
                           (1 << 16, (1 << 17) + 1, 4, 4096)]:
        s = ref.sample(n, N, seed, n0=n0)
        left = int(np.searchsorted(s, N // 2, side="right"))
        assert left == ref.hyp(n, N // 2, N, seed, 1)
    for n, N, seed, n0 in [(5000, 10**6 + 7, 3, 256), (9, 5, 2, 2)]:
        s = ref.replacement(n, N, seed, n0=n0)
        left = int(np.searchsorted(s, N // 2, side="right"))
        assert left == ref.binom(n, N // 2, N, seed, 1)


def test_tree_size_bound(ref):
    """Sec. 3.1: the recursion tree has at most about 2n/n0 nodes; with
    n_v < n0 leaves and halving splits its internal nodes stay below 2n/n0."""
    for n, N, n0 in [(1 << 20, 1 << 32, 4096), (1 << 30, 1 << 48, 4096), (1 << 24, 1 << 25, 4096)]:
        internal, leaves, depth = ref.tree_stats(n, N, 7, n0)
        assert internal <= 2 * n // n0
        assert leaves == internal + 1  # every internal node here has two non-empty children
        assert depth <= math.ceil(math.log2(N))


def _rounds_first_distinct(ref, seed, node_id, purpose, attempt, want, rng_size):
    """Round-based rule: draw `want - d` more non-void values per round until d
    distinct values are held (the order inside a round does not matter)."""
    have = set()
    t = 0
    while len(have) < want:
        need = want - len(have)
        got = []
        while len(got) < need:
            v = ref.range_map(ref.stream_word(seed, node_id, purpose, attempt, t), rng_size)
            t += 1
            if v >= 0:
                got.append(v)
        have.update(got)
    return sorted(have)


@pytest.mark.parametrize("n,N", [(300, 5000), (200, 2**31 + 1), (1000, 17000), (50, 801)])
def test_sparse_leaf_rounds_equal_algorithm_h(ref, n, N):
    """The key equivalence behind the parallel leaf: taking (n - d) more draws
    per round reproduces exactly the set of the first n distinct values that
    Algorithm H (Sec. 2) keeps, whatever the order inside a round."""
    for seed in (1, 2, 3):
        s = ref.sample(n, N, seed, n0=4096, dense_ratio=2)  # root is one sparse leaf
        want = _rounds_first_distinct(ref, seed, 1, 2, 0, n, N)
        assert [int(x) - 1 for x in s] == want


# --------------------------------------------------------------------------
# Bernoulli sampling (Sec. 4.7)
# --------------------------------------------------------------------------
def test_bernoulli_degenerate(ref):
    assert ref.bernoulli(0.0, 1000, 1).size == 0
    np.testing.assert_array_equal(ref.bernoulli(1.0, 1000, 1), np.arange(1, 1001, dtype=np.uint64))
    assert ref.bernoulli(0.3, 0, 1).size == 0
    with pytest.raises(RuntimeError):
        ref.bernoulli(1.5, 10, 1)


@pytest.mark.parametrize("p", [0.3, 0.01, 2.0**-10, 1e-4, 0.97])
def test_bernoulli_counts_binomial(ref, p):
    N = 1 << 22
    counts = np.array([ref.bernoulli(p, N, seed).size for seed in range(60 if p < 0.5 else 15)])
    mu, sd = N * p, math.sqrt(N * p * (1 - p))
    z = (counts - mu) / sd
    assert np.abs(z).max() < 4.5
    assert abs(z.sum() / math.sqrt(len(z))) < 4.5


@pytest.mark.parametrize("p,N", [(0.3, 9), (0.75, 8), (2.0**-11, 6)])
def test_bernoulli_all_subsets(ref, p, N):
    """Every one of the 2^N subsets appears with probability p^k (1-p)^(N-k)."""
    seeds = 60000
    obs = np.zeros(1 << N)
    for seed in range(seeds):
        mask = 0
        for v in ref.bernoulli(p, N, seed):
            mask |= 1 << (int(v) - 1)
        obs[mask] += 1
    probs = np.array([p ** bin(m).count("1") * (1 - p) ** (N - bin(m).count("1"))
                      for m in range(1 << N)])
    assert _chisq_pvalue(obs, probs) > 1e-4


@pytest.mark.parametrize("p", [0.3, 0.01, 1e-4])
def test_bernoulli_gaps_geometric(ref, p):
    """Within a chunk, gaps between hits are geometric: P(gap = g) = p(1-p)^(g-1)."""
    N = 1 << 24 if p >= 1e-3 else 1 << 28
    s = ref.bernoulli(p, N, 5).astype(np.int64)
    C = ref.bernoulli_chunk_len(p)
    same = (s[1:] - 1) // C == (s[:-1] - 1) // C
    gaps = np.diff(s)[same]
    gmax = int(np.quantile(gaps, 0.999))
    obs = np.bincount(np.clip(gaps, 1, gmax + 1) - 1, minlength=gmax + 1)
    pm = p * (1 - p) ** np.arange(gmax)
    probs = np.concatenate([pm, [(1 - p) ** gmax]])
    assert _chisq_pvalue(obs, probs) > 1e-4


def test_bernoulli_chunk_boundaries(ref):
    """Several chunks: hits are uniform over positions, across boundaries."""
    p = 0.3
    C = ref.bernoulli_chunk_len(p)
    assert C == 1 << 13
    N = 3 * C + 5
    hist = np.zeros(64)
    total = 0
    for seed in range(300):
        s = ref.bernoulli(p, N, seed).astype(np.int64)
        hist += np.bincount((s - 1) * 64 // N, minlength=64)
        total += s.size
    assert abs(total - 300 * N * p) / math.sqrt(300 * N * p * (1 - p)) < 4.5
    probs = np.array([((i + 1) * N + 63) // 64 - (i * N + 63) // 64 for i in range(64)]) / N
    assert _chisq_pvalue(hist, probs) > 1e-4


def test_bernoulli_chunk_rule(ref):
    assert ref.bernoulli_chunk_len(0.01) == 1 << 18   # 4096/0.01 = 409600
    assert ref.bernoulli_chunk_len(1.0) == 1 << 12
    assert ref.bernoulli_chunk_len(1e-12) == 1 << 32


# --------------------------------------------------------------------------
# Sampling with replacement (Sec. 4.6)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,n,n0", [(3, 4, 2), (5, 7, 4), (4, 6, 2), (2, 9, 4)])
def test_replacement_multinomial(ref, N, n, n0):
    cells = list(itertools.combinations_with_replacement(range(1, N + 1), n))
    index = {c: i for i, c in enumerate(cells)}
    probs = []
    for c in cells:
        cnt = Counter(c)
        m = math.factorial(n)
        for v in cnt.values():
            m //= math.factorial(v)
        probs.append(m / N**n)
    obs = np.zeros(len(cells))
    for seed in range(30000):
        s = tuple(int(x) for x in ref.replacement(n, N, seed, n0=n0))
        obs[index[s]] += 1
    assert _chisq_pvalue(obs, probs) > 1e-4


def test_replacement_invariants(ref):
    np.testing.assert_array_equal(ref.replacement(7, 1, 3), np.ones(7, dtype=np.uint64))
    n, N = 1 << 20, 1 << 34
    dups = []
    for seed in range(6):
        s = ref.replacement(n, N, seed).astype(np.int64)
        assert (np.diff(s) >= 0).all() and s[0] >= 1 and s[-1] <= N
        dups.append(int((np.diff(s) == 0).sum()))
    lam = n * (n - 1) / (2 * N)  # expected repeated pairs, 32
    assert abs(np.mean(dups) - lam) < 4.5 * math.sqrt(lam / len(dups))
    # marginal uniformity at a non-power-of-two range with many leaves
    N = 3 * 10**6 + 1
    s = ref.replacement(200000, N, 11, n0=512).astype(np.int64)
    obs = np.bincount((s - 1) * 50 // N, minlength=50)
    probs = np.array([((i + 1) * N + 49) // 50 - (i * N + 49) // 50 for i in range(50)]) / N
    assert _chisq_pvalue(obs, probs) > 1e-4


# Online sampling in parts (Sec. 4.1): the parts of one cut, in index order,
# concatenate to the full sample, and each rank is the number of values in
# the parts before it.  (n, N, seed, n0, depth, variant): small n0 makes
# leaves end paths above the cut (leftmost-part rule) and empty nodes occur.
PART_CASES = [
    (50000, 1 << 30, 3, 256, 0, 0),
    (50000, 1 << 30, 3, 256, 4, 0),
    (50000, 1 << 30, 3, 256, 10, 0),    # most paths end at leaves above the cut
    (3000, 3100, 5, 64, 6, 0),          # dense leaves
    (777, 10**9 + 7, 6, 16, 8, 0),      # ragged ranges
    (5, 40, 7, 2, 5, 0),                # empty nodes above the cut
    (40000, 1 << 36, 8, 512, 7, 1),     # with replacement
    (3000, 7, 9, 64, 4, 1),             # with replacement, N_v = 1 leaves
]


@pytest.mark.parametrize("n,N,seed,n0,depth,variant", PART_CASES)
def test_parts_concatenate_to_the_sample(ref, n, N, seed, n0, depth, variant):
    full = ref.sample(n, N, seed, n0=n0) if variant == 0 else ref.replacement(n, N, seed, n0=n0)
    got, rank = [], 0
    for g in range(1 << depth):
        vals, count, r = ref.part(variant, n, N, seed, depth, g, n0=n0)
        assert r == rank, (g, r, rank)
        assert len(vals) == count
        got.append(vals)
        rank += count
    assert rank == n
    assert (np.concatenate(got) == full).all()


def test_part_depth_one_is_the_root_split(ref):
    n, N, seed = 100000, 1 << 40, 11
    left = ref.hyp(n, N // 2, N, seed, 1)
    _, c0, r0 = ref.part(0, n, N, seed, 1, 0)
    vals, c1, r1 = ref.part(0, n, N, seed, 1, 1)
    assert (c0, r0, c1, r1) == (left, 0, n - left, left)
    assert int(vals.min()) > N // 2  # the right half's range N/2+1 .. N


def test_part_leaf_above_the_cut_and_overflow(ref):
    n, N, seed = 100, 1 << 20, 4
    full = ref.sample(n, N, seed)  # the root is a leaf (n < n0 = 4096)
    vals, count, rank = ref.part(0, n, N, seed, 3, 0)
    assert (count, rank) == (n, 0) and (vals == full).all()
    for g in range(1, 8):
        vals, count, rank = ref.part(0, n, N, seed, 3, g)
        assert (count, rank, len(vals)) == (0, n, 0)
    vals, count, rank = ref.part(0, n, N, seed, 0, 0, capacity=n - 1)
    assert vals is None and (count, rank) == (n, 0)


def test_part_edge_cases(ref):
    for g in range(8):
        vals, count, rank = ref.part(0, 0, 100, 1, 3, g)
        assert (count, rank, len(vals)) == (0, 0, 0)
    # the deepest cut of the largest universe: the range rule splits down to
    # depth 20 (ranges of 2^32), where these 20 values sit in leaves; the leaf
    # over range i (values i*2^32+1 .. (i+1)*2^32) goes whole to the leftmost
    # depth-45 part below it, index i*2^25, and the part after it is empty
    n, N, seed = 20, 2**52, 9
    full = ref.sample(n, N, seed).astype(np.int64)
    for i in sorted({int(v - 1) >> 32 for v in full}):
        inside = full[(full - 1) >> 32 == i]
        before = int(np.count_nonzero(((full - 1) >> 32) < i))
        vals, count, rank = ref.part(0, n, N, seed, 45, i << 25)
        assert (count, rank) == (len(inside), before)
        assert (vals.astype(np.int64) == inside).all()
        vals, count, rank = ref.part(0, n, N, seed, 45, (i << 25) + 1)
        assert (count, rank) == (0, before + len(inside))
