"""Pins of the oracle above N = 2^52 (the recursion tree accepts universes up
to 2^62; the paper's own experiments run at N = 2^50, Sec. 6, and random
graphs on 2^30 vertices need N near 2^59, Sec. 7).  Integers above 2^53
reach the hypergeometric and binomial deviates' doubles rounded; these
tests check against 50-digit mpmath that the deviates still follow their
exact laws there, that whole samples keep the hypergeometric law of their
prefix counts, and that edge indices up to 2^62 decode exactly."""
import math

import mpmath
import numpy as np
import pytest

import oracle
from tests.test_oracle_primitives import _chisq_pvalue, _hyp_logpmf_mp


def test_lnfact_diff_above_2_53():
    mpmath.mp.dps = 60
    rng = np.random.default_rng(5)
    pairs = [(2**62, 2**62 - 1), (2**60 + 3, 2**60 - 2**20), (2**58, 2**58 + 77)]
    for scale in (2**54, 2**58, 2**61):
        for _ in range(40):
            a = scale + int(rng.integers(0, 2**40))
            pairs.append((a, a + int(rng.integers(-2**22, 2**22))))
    for a, b in pairs:
        exact = float(mpmath.loggamma(a + 1) - mpmath.loggamma(b + 1))
        got = oracle.lnfact_diff(a, b)
        assert abs(got - exact) <= 1e-13 * max(1.0, abs(exact)), (a, b, got, exact)


@pytest.mark.parametrize("n,M,N", [(1000, 2**59, 2**60),
                                   (1 << 24, 2**59 + 12345, 2**60 + 99),
                                   (3000, 3 * 2**58, 2**60 - 1),
                                   (50_000, 2**61, 2**62)])
def test_hyp_above_2_52_against_mpmath_pmf(n, M, N):
    """Ratio-of-uniforms branch: equal-mass cells of the exact pmf."""
    mpmath.mp.dps = 50
    draws = oracle.hyp_batch(n, M, N, 11, 1, 30000).astype(np.int64)
    mu = n * M / N
    sd = math.sqrt(mu * (1 - M / N) * (N - n) / (N - 1))
    lo, hi = int(mu - 7 * sd), int(mu + 7 * sd) + 1
    step = max(1, int(sd / 200))
    ks = np.arange(lo, hi + 1, step)
    mids = ks[:-1] + (step - 1) / 2.0
    pm = np.array([float(mpmath.exp(_hyp_logpmf_mp(n, M, N, mpmath.mpf(float(k)))))
                   for k in mids]) * step
    assert abs(pm.sum() - 1) < 1e-3
    cdf = np.concatenate([[0.0], np.cumsum(pm)])
    edges = [ks[np.searchsorted(cdf, q)] for q in np.linspace(0, 1, 41)[1:-1]]
    obs = np.bincount(np.searchsorted(np.array(edges), draws, side="right"), minlength=40)
    probs = np.diff(np.concatenate([[0.0], np.interp(edges, ks, cdf), [1.0]]))
    assert _chisq_pvalue(obs, probs) > 1e-4
    assert abs((draws.mean() - mu) / (sd / math.sqrt(len(draws)))) < 4.5
    assert abs(draws.var() / sd**2 - 1) < 0.05


@pytest.mark.parametrize("n,M,N", [(12, 2**61, 2**62), (16, 2**60 + 5, 3 * 2**60)])
def test_hyp_inversion_above_2_52_exact(n, M, N):
    """Inversion branch (n <= 16): every outcome against the exact pmf."""
    mpmath.mp.dps = 60
    b = mpmath.binomial
    pmf = [float(b(M, k) * b(N - M, n - k) / b(N, n)) for k in range(n + 1)]
    draws = oracle.hyp_batch(n, M, N, 3, 1, 40000).astype(np.int64)
    assert draws.min() >= 0 and draws.max() <= n
    assert _chisq_pvalue(np.bincount(draws, minlength=n + 1), pmf) > 1e-4


@pytest.mark.parametrize("n,l,Nv", [(30_000, 2**60, 2**61 + 3), (9, 2**61, 2**62 - 1)])
def test_binomial_above_2_52(n, l, Nv):
    """The with-replacement split Bin(n, l/Nv) at the top of the range."""
    mpmath.mp.dps = 50
    p = mpmath.mpf(l) / Nv
    draws = oracle.binom_batch(n, l, Nv, 4, 1, 30000).astype(np.int64)
    if n <= 16:
        pmf = [float(mpmath.binomial(n, k) * p**k * (1 - p) ** (n - k)) for k in range(n + 1)]
        assert _chisq_pvalue(np.bincount(draws, minlength=n + 1), pmf) > 1e-4
        return
    mu, sd = float(n * p), float(mpmath.sqrt(n * p * (1 - p)))
    assert abs((draws.mean() - mu) / (sd / math.sqrt(len(draws)))) < 4.5
    assert abs(draws.var() / sd**2 - 1) < 0.05


@pytest.mark.parametrize("variant,N", [(0, 2**60 - 5), (1, 2**61 + 3)])
def test_sample_prefix_counts_above_2_52(variant, N):
    """Whole samples at N near 2^60: sorted, in range (distinct without
    replacement), and the count up to x is Hyp(n, x, N) (Bin(n, x/N) with
    replacement) in mean and variance."""
    n, reps = 3000, 300
    cuts = [N // 3, N // 2 + 1, (7 * N) // 9]
    obs = {x: [] for x in cuts}
    for seed in range(reps):
        v = (oracle.sample if variant == 0 else oracle.replacement)(n, N, seed, n0=256)
        d = np.diff(v.astype(np.uint64).astype(object))
        assert all(x > 0 for x in d) if variant == 0 else all(x >= 0 for x in d)
        assert int(v[0]) >= 1 and int(v[-1]) <= N
        for x in cuts:
            obs[x].append(int(np.searchsorted(v, np.uint64(x), side="right")))
    for x in cuts:
        p = x / N
        fpc = (N - n) / (N - 1) if variant == 0 else 1.0
        mu, sd = n * p, math.sqrt(n * p * (1 - p) * fpc)
        c = np.asarray(obs[x], dtype=np.float64)
        assert abs(c.mean() - mu) < 4.5 * sd / math.sqrt(reps)
        assert 0.7 < c.var() / sd**2 < 1.4


def test_edge_pairs_up_to_2_62():
    """Edge index k = u(u-1)/2 + v decodes exactly at the top of the range
    (u up to 3,037,000,500, where 8k + 1 exceeds 64 bits)."""
    for u in (2**30, 2**31 + 7, 3037000499, 3037000500):
        t = u * (u - 1) // 2
        if t + u - 1 >= 2**62:
            assert oracle.edge_pair(t) == (u, 0)
            continue
        assert oracle.edge_pair(t) == (u, 0)
        assert oracle.edge_pair(t + u - 1) == (u, u - 1)
        assert oracle.edge_pair(t - 1) == (u - 1, u - 2)
    k = 2**62 - 1
    u, v = oracle.edge_pair(k)
    assert u * (u - 1) // 2 + v == k and v < u


def test_gnm_on_2_30_vertices():
    """G(n, m) on 2^30 vertices (N = n(n-1)/2 near 2^59): the edges are the
    decoded sample, sorted, v < u < n; the larger end u follows P(u < x) =
    x(x-1)/2 / N."""
    nv, m, seed = 1 << 30, 200_000, 3
    e = oracle.edges_gnm(nv, m, seed).astype(np.int64)
    u, v = e[:, 0], e[:, 1]
    assert np.all(v < u) and np.all(u < nv)
    k = u * (u - 1) // 2 + v
    assert np.all(np.diff(k) > 0)
    N = nv * (nv - 1) // 2
    assert np.array_equal(k + 1, oracle.sample(m, N, seed).astype(np.int64))
    for x in (nv // 4, nv // 2, (3 * nv) // 4):
        p = x * (x - 1) / 2 / N
        cnt = int((u < x).sum())
        assert abs(cnt - m * p) < 5 * math.sqrt(m * p * (1 - p))
