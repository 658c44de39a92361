"""Pins of the oracle's sampling over an uneven universe (paper Sec. 4.3,
Fig. 3): K segments (the paper's PEs) of sizes L_0..L_{K-1}, n samples of
their concatenation.  The oracle is checked against what the paper and the
mathematics fix, not against itself:

* the tree is the paper's binomial tree: PE i with k trailing zero bits is
  joined to PE i + 2^j for j < k (when that PE exists), element counts are
  summed bottom-up and sample counts split top-down (checked on Fig. 3's
  configuration, 13 PEs, n = 50, N = 229);
* the vector of per-segment counts follows the multivariate hypergeometric
  law prod C(L_i, n_i) / C(N, n) (every vector of tiny cases, chi-square);
* the sample is uniform over all C(N, n) subsets of the concatenation (brute
  force on tiny universes with empty and unequal segments);
* the number of sampled values up to a segment boundary (and inside a
  segment) is hypergeometric (large segments, moments);
* one segment is the plain sample keyed by the segment's seed, and each
  segment's block is the plain sample of its count, shifted by the elements
  before it (the identity of a segment's randomness).
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from tests.test_oracle_primitives import _chisq_pvalue

# Fig. 3: 13 PEs, N = 229 elements, n = 50 samples (the figure's L-values are
# not legible in the text, so these sizes are ours, with the same sum).
FIG3_L = [20, 15, 30, 5, 17, 25, 10, 22, 18, 12, 20, 15, 20]
FIG3_N, FIG3_n = 229, 50


def _depth(K):
    return max(0, (K - 1).bit_length())


def _span(D, K, node_id):
    """PEs of heap node `node_id`: level j, subtree a spans 2^j a .. min(2^j a + 2^j, K)-1."""
    level_from_top = node_id.bit_length() - 1
    j = D - level_from_top
    a = node_id - (1 << level_from_top)
    return (a << j), min((a << j) + (1 << j), K)


def _paper_edges(p):
    """The binomial tree of Sec. 4.3: PE i with k trailing zeros (in ceil(log p)
    bits) is connected with PEs i + 2^j, j in 0..k-1, if i + 2^j < p."""
    D = _depth(p)
    edges = set()
    for i in range(p):
        k = D if i == 0 else (i & -i).bit_length() - 1
        for j in range(k):
            if i + (1 << j) < p:
                edges.add((i, i + (1 << j)))
    return edges


def test_fig3_binomial_tree():
    assert sum(FIG3_L) == FIG3_N
    K, D = len(FIG3_L), _depth(len(FIG3_L))
    for seed in range(20):
        sums, cnt = oracle.segment_tree(FIG3_n, FIG3_L, seed)
        assert int(cnt[1]) == FIG3_n and int(sums[1]) == FIG3_N
        splits = set()
        for node in range(1, 1 << D):
            lo, hi = _span(D, K, node)
            if lo >= K:
                assert sums[node] == 0 and cnt[node] == 0
                continue
            # upward pass: the element count of the subtree
            assert int(sums[node]) == sum(FIG3_L[lo:hi])
            # downward pass: the children's counts add up, never exceed sizes
            assert int(cnt[2 * node]) + int(cnt[2 * node + 1]) == int(cnt[node])
            assert cnt[node] <= sums[node]
            rlo, _ = _span(D, K, 2 * node + 1)
            if rlo < K:
                splits.add((lo, rlo))
        # one split per edge of the paper's binomial tree, and nothing else
        assert splits == _paper_edges(K)
        assert len(splits) == K - 1
        # leaves are the segments; the sample puts counts[i] values in each
        vals, counts = oracle.sample_segments(FIG3_n, FIG3_L, seed, n0=8)
        leaf = [int(cnt[(1 << D) + i]) for i in range(K)]
        assert counts.tolist() == leaf
        bounds = np.cumsum([0] + FIG3_L)
        per = np.histogram(vals.astype(np.int64), bins=bounds + 0.5)[0]
        assert per.tolist() == leaf
        assert np.all(np.diff(vals.astype(np.int64)) > 0) and vals[0] >= 1 and vals[-1] <= FIG3_N


@pytest.mark.parametrize("L,n", [([2, 0, 3, 1, 2], 3), ([4, 1, 2], 4), ([1, 1, 1, 1, 1, 1, 1], 3)])
def test_counts_multivariate_hypergeometric(L, n):
    N = sum(L)
    vecs = [v for v in itertools.product(*[range(x + 1) for x in L]) if sum(v) == n]
    probs = [math.prod(math.comb(x, k) for x, k in zip(L, v)) / math.comb(N, n) for v in vecs]
    assert abs(sum(probs) - 1) < 1e-12
    idx = {v: i for i, v in enumerate(vecs)}
    obs = np.zeros(len(vecs))
    for seed in range(20000):
        _, c = oracle.sample_segments(n, L, seed, n0=2)
        obs[idx[tuple(int(x) for x in c)]] += 1
    assert _chisq_pvalue(obs, probs) > 1e-4


@pytest.mark.parametrize("L,n,n0", [([3, 1, 0, 4, 2], 3, 2), ([3, 3], 2, 2), ([5, 0, 0, 2, 1, 4], 4, 4)])
def test_uniform_over_all_subsets(L, n, n0):
    N = sum(L)
    cells = list(itertools.combinations(range(1, N + 1), n))
    idx = {c: i for i, c in enumerate(cells)}
    obs = np.zeros(len(cells))
    for seed in range(max(20000, 40 * len(cells))):
        v, _ = oracle.sample_segments(n, L, seed, n0=n0)
        t = tuple(int(x) for x in v)
        assert t in idx
        obs[idx[t]] += 1
    assert _chisq_pvalue(obs, np.full(len(cells), 1 / len(cells))) > 1e-4


def test_prefix_counts_hypergeometric():
    L = [3 << 30, 1 << 40, 7, 5 << 36, 0, 1 << 33, 11 << 38]
    N, n = sum(L), 6000
    bounds = np.cumsum(L)
    cuts = [int(bounds[0]), int(bounds[1]), int(bounds[3]), int(bounds[5]),
            int(bounds[1]) + (L[2] // 2), int(bounds[5]) + L[6] // 3]
    obs = {x: [] for x in cuts}
    reps = 400
    for seed in range(reps):
        v, _ = oracle.sample_segments(n, L, seed, n0=512)
        for x in cuts:
            obs[x].append(int(np.searchsorted(v, x, side="right")))
    for x in cuts:
        p = x / N
        mu = n * p
        sd = math.sqrt(n * p * (1 - p) * (N - n) / (N - 1))
        c = np.asarray(obs[x], dtype=np.float64)
        if sd > 0:
            assert abs(c.mean() - mu) < 4.5 * sd / math.sqrt(reps), (x, c.mean(), mu)
            assert 0.75 < c.var() / sd**2 < 1.3, (x, c.var(), sd**2)


def test_one_segment_is_the_plain_sample():
    for n, L0, seed in [(1000, 1 << 30, 3), (5, 9, 1), (3000, 4000, 8)]:
        v, c = oracle.sample_segments(n, [L0], seed, n0=256)
        s0 = oracle.stream_draw64(seed, 1, oracle.P_SEGSEED, 0, 0)
        assert int(c[0]) == n
        assert np.array_equal(v, oracle.sample(n, L0, s0, n0=256))


def test_blocks_are_plain_samples_of_their_counts():
    L = [1 << 20, 0, 12345, 1 << 28, 3, 77777]
    K, D = len(L), _depth(len(L))
    for seed in (1, 2):
        v, c = oracle.sample_segments(20000, L, seed, n0=1024)
        off = base = 0
        for i in range(K):
            ni = int(c[i])
            si = oracle.stream_draw64(seed, (1 << D) + i, oracle.P_SEGSEED, 0, 0)
            want = oracle.sample(ni, L[i], si, n0=1024) + np.uint64(base)
            assert np.array_equal(v[off:off + ni], want)
            off += ni
            base += L[i]


def test_degenerate_cases():
    # n = 0, n = N, all but one segment empty, K a power of two
    v, c = oracle.sample_segments(0, [5, 6], 1)
    assert v.size == 0 and c.tolist() == [0, 0]
    v, c = oracle.sample_segments(11, [5, 0, 6], 1, n0=2)
    assert v.tolist() == list(range(1, 12)) and c.tolist() == [5, 0, 6]
    v, c = oracle.sample_segments(7, [0, 0, 0, 100, 0, 0, 0, 0], 4, n0=2)
    assert c.tolist() == [0, 0, 0, 7, 0, 0, 0, 0]
    assert np.all((v >= 1) & (v <= 100)) and np.all(np.diff(v.astype(np.int64)) > 0)
    for bad in [(3, [], 1), (10, [4, 5], 1), (1, [1 << 62, 1], 1)]:
        with pytest.raises(RuntimeError):
            oracle.sample_segments(*bad)
