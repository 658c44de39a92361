"""Pins of the oracle's whole-range Algorithm B (paper Sec. 2 Algorithm B,
Sec. 4.7 skips and prefix sums, Sec. 5's GPU variant with the repair done
without a host round trip): a Bernoulli(rho) sample of the whole range,
restarted while too small, then cut down to n hits by removing a uniformly
random set of hit indices.  Checked against what the mathematics fixes:

* uniform over all C(N, n) subsets of tiny ranges, with rho < 1 (so that
  the Bernoulli part matters) and rho = 1 (repair only);
* the hit count n' of an attempt is Bin(N, rho) (moments) and every
  position is a hit with probability rho;
* the number of sampled values up to x is hypergeometric, also across many
  chunk boundaries;
* the removed hit indices are Algorithm H's first n'-n distinct values of
  the repair stream, which the GPU computes in rounds (each round draws as
  many more words as values are missing): both rules give the same set;
* n = 0, n = N, n = N - 1; unsupported ranges and densities are refused.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from tests.test_oracle_primitives import _chisq_pvalue


def _rho(n, N):
    num = n + 8 * math.isqrt(n) + 16
    return 1.0 if num >= N else num / N


@pytest.mark.parametrize("n,N", [(2, 40), (1, 30), (3, 12), (5, 9)])
def test_uniform_over_all_subsets(n, N):
    cells = list(itertools.combinations(range(1, N + 1), n))
    idx = {c: i for i, c in enumerate(cells)}
    obs = np.zeros(len(cells))
    attempts = 0
    for seed in range(max(20000, 30 * len(cells))):
        v, a = oracle.sample_wholerange(n, N, seed, n0=16)
        attempts += a
        t = tuple(int(x) for x in v)
        assert t in idx
        obs[idx[t]] += 1
    assert _chisq_pvalue(obs, np.full(len(cells), 1 / len(cells))) > 1e-4


def test_hit_count_and_marginals():
    n, N, reps = 3000, 1 << 16, 400
    rho = _rho(n, N)
    counts, incl = [], np.zeros(N)
    for seed in range(reps):
        c, pos = oracle.wholerange_hits(n, N, seed, cap=N)
        counts.append(c)
        incl[pos.astype(np.int64) - 1] += 1
    c = np.asarray(counts, dtype=np.float64)
    mu, var = N * rho, N * rho * (1 - rho)
    assert abs(c.mean() - mu) < 4.5 * math.sqrt(var / reps)
    assert 0.7 < c.var() / var < 1.4
    # per-position inclusion: binomial(reps, rho) at every position
    z = (incl - reps * rho) / math.sqrt(reps * rho * (1 - rho))
    assert abs(z.mean()) < 0.05
    assert 0.85 < z.var() < 1.15


@pytest.mark.parametrize("n,N,n0", [(5000, 1 << 20, 4096), (500_000, 1_000_003, 64)])
def test_prefix_counts_hypergeometric(n, N, n0):
    cuts = [N // 7, N // 3, N // 2 + 1, (5 * N) // 6]
    reps = 250
    obs = {x: [] for x in cuts}
    for seed in range(reps):
        v, _ = oracle.sample_wholerange(n, N, seed, n0=n0)
        assert v.size == n and np.all(np.diff(v.astype(np.int64)) > 0)
        for x in cuts:
            obs[x].append(int(np.searchsorted(v, x, side="right")))
    for x in cuts:
        p = x / N
        mu = n * p
        sd = math.sqrt(n * p * (1 - p) * (N - n) / (N - 1))
        c = np.asarray(obs[x], dtype=np.float64)
        assert abs(c.mean() - mu) < 4.5 * sd / math.sqrt(reps), (x, c.mean(), mu)
        assert 0.7 < c.var() / sd**2 < 1.4


def _rounds_removals(seed, attempt, r, count):
    """The GPU's rule: rounds of (r - d) stream words, d = distinct values so
    far (voids never count), until d = r."""
    got, t = set(), 0
    while len(got) < r:
        take = r - len(got)
        for k in range(t, t + take):
            v = oracle.range_map(oracle.stream_word(seed, 0, oracle.P_WREPAIR, attempt, k), count)
            if v >= 0:
                got.add(v)
        t += take
    return got


@pytest.mark.parametrize("n,N,seed", [(20_000, 40_000, 3), (1000, 1017, 5), (60_000, 65_536, 8)])
def test_removals_are_algorithm_h_and_rounds(n, N, seed):
    v, a = oracle.sample_wholerange(n, N, seed, n0=256)
    cnt, hits = oracle.wholerange_hits(n, N, seed, attempt=a, n0=256, cap=N)
    keep = np.isin(hits, v)
    assert int(keep.sum()) == n
    removed = set(np.nonzero(~keep)[0].tolist())
    assert removed == _rounds_removals(seed, a, cnt - n, cnt)


def test_degenerate_and_refused():
    v, _ = oracle.sample_wholerange(0, 100, 1)
    assert v.size == 0
    v, _ = oracle.sample_wholerange(100, 100, 1)
    assert v.tolist() == list(range(1, 101))
    v, _ = oracle.sample_wholerange(99, 100, 2)
    assert v.size == 99 and len(set(v.tolist())) == 99 and v.max() <= 100
    for bad in [(1, 1 << 20, 1), (10, (1 << 32) + 1, 1), (5, 4, 1), (1, 0, 1)]:
        with pytest.raises(RuntimeError):
            oracle.sample_wholerange(*bad)
