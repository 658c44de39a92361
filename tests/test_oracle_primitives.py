"""Pins for the oracle's primitives (CPU only).

Each primitive is checked against something other than itself: published
known-answer vectors, an independent implementation, an exhaustive count,
arbitrary-precision arithmetic or an exact probability mass function.
"""
import math
import os
import shutil
import subprocess

import mpmath
import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((tuple(v[0:4]), tuple(v[4:6]), tuple(v[6:10])))
    return rows


# --------------------------------------------------------------------------
# Philox-4x32-10: the hash h of a subproblem identity (Sec. 3.2).
# --------------------------------------------------------------------------
def test_philox_known_answers(ref):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert ref.philox(ctr, key) == want


def test_philox_matches_torch_engine(ref, tmp_path):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = tmp_path / "philox_torch_check"
    subprocess.run(["g++", "-std=c++17", "-O1", f"-I{inc}", "-o", str(exe),
                    os.path.join(HERE, "philox_torch_check.cpp")], check=True)
    rng = np.random.default_rng(1234)
    vecs = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    vecs[0] = 0
    vecs[1] = 2**32 - 1
    inp = "\n".join(" ".join(str(int(x)) for x in row) for row in vecs) + "\n"
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    got = [tuple(int(x) for x in line.split()) for line in res.stdout.strip().splitlines()]
    assert len(got) == len(vecs)
    for row, g in zip(vecs, got):
        ctr = tuple(int(x) for x in row[:4])
        key = tuple(int(x) for x in row[4:])
        assert ref.philox(ctr, key) == g


def test_stream_layout(ref):
    """Word t is word t mod 4 of block t/4; 64-bit draw t pairs words 2(t mod 2)
    (low) and 2(t mod 2)+1 (high) of block t/2; the counter carries (block,
    purpose<<24|attempt, id_lo, id_hi) and the key the seed."""
    seed, nid, purpose, attempt = 0x0123456789ABCDEF, (1 << 40) + 77, 2, 5
    key = (seed & 0xFFFFFFFF, seed >> 32)
    for b in (0, 1, 7, 1000):
        ctr = (b, (purpose << 24) | attempt, nid & 0xFFFFFFFF, nid >> 32)
        blk = ref.philox(ctr, key)
        for j in range(4):
            assert ref.stream_word(seed, nid, purpose, attempt, 4 * b + j) == blk[j]
        for h in range(2):
            want = blk[2 * h] | (blk[2 * h + 1] << 32)
            assert ref.stream_draw64(seed, nid, purpose, attempt, 2 * b + h) == want


# --------------------------------------------------------------------------
# Uniform integer in [0, s): exact multiply-shift rejection.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("s", [3, 1000003])
def test_range_map_exhaustive(ref, s):
    """Over all 2^32 words, every value has exactly floor(2^32/s) accepted
    preimages and exactly 2^32 mod s words are void: accepted draws are exactly
    uniform."""
    counts, voids = ref.range_map_counts(s)
    assert voids == (1 << 32) % s
    assert int(counts.min()) == int(counts.max()) == (1 << 32) // s


def test_range_map_power_of_two_closed_form(ref):
    rng = np.random.default_rng(7)
    for k in (0, 1, 5, 20, 31, 32):
        s = 1 << k
        for w in rng.integers(0, 2**32, size=200):
            w = int(w)
            assert ref.range_map(w, s) == (w >> (32 - k) if k < 32 else w)
    assert ref.range_map(0, 1) == 0
    assert ref.range_map(2**32 - 1, 2**32) == 2**32 - 1


def test_range_map_void_rule(ref):
    s = 2**31 + 1  # threshold 2^31 - 1: about half the words are void
    thr = (1 << 32) % s
    # the words at the boundary: low half of w*s equal to thr (kept) and thr-1 (void)
    inv = pow(s, -1, 1 << 32)
    for low, kept in ((thr, True), (thr - 1, False)):
        w = (low * inv) % (1 << 32)
        assert (ref.range_map(w, s) >= 0) == kept
    rng = np.random.default_rng(3)
    for w in rng.integers(0, 2**32, size=2000):
        w = int(w)
        m = w * s
        want = -1 if (m & 0xFFFFFFFF) < thr else m >> 32
        assert ref.range_map(w, s) == want


# --------------------------------------------------------------------------
# Logarithms: project-written series, pinned against high-precision values.
# --------------------------------------------------------------------------
def _ulp_err32(y, x):
    exact = np.log(x.astype(np.float64))
    ulp = np.spacing(np.abs(exact).astype(np.float32)).astype(np.float64)
    return np.abs(y.astype(np.float64) - exact) / ulp


def test_log32_exhaustive_unit_interval(ref):
    """Every float in [2^-32, 1] (the range of the geometric uniforms):
    error at most 2 ulp against the double-precision logarithm."""
    worst = 0.0
    for e in range(-32, 0):
        lo = np.float32(2.0 ** e).view(np.uint32)
        bits = np.arange(int(lo), int(lo) + (1 << 23), dtype=np.uint32)
        x = bits.view(np.float32)
        worst = max(worst, float(_ulp_err32(ref.log32_batch(x), x).max()))
    assert ref.log32(1.0) == 0.0
    assert worst <= 2.0, worst


def test_log32_matches_mpmath_spot(ref):
    mpmath.mp.dps = 40
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(2**-32, 1, 300), rng.uniform(1, 1e6, 100)]).astype(np.float32)
    for x in xs:
        exact = float(mpmath.log(mpmath.mpf(float(x))))
        ulp = float(np.spacing(np.float32(abs(exact))))
        assert abs(ref.log32(float(x)) - exact) <= 2.0 * ulp


def test_log64_against_mpmath_and_numpy(ref):
    mpmath.mp.dps = 50
    rng = np.random.default_rng(12)
    x = np.concatenate([np.exp(rng.uniform(-700, 700, 400000)), rng.uniform(0.5, 2.0, 400000)])
    y = ref.log64_batch(x)
    err = np.abs(y - np.log(x)) / np.spacing(np.abs(np.log(x)))
    assert err.max() <= 3.0
    for xi in np.concatenate([x[:300], [1.0, 2.0, 0.5, 2**52 + 1.0, 1 - 2**-53, 1 + 2**-52]]):
        exact = mpmath.log(mpmath.mpf(float(xi)))
        got = ref.log64(float(xi))
        tol = 2.0 * float(np.spacing(abs(float(exact)))) if exact != 0 else 0.0
        assert abs(got - float(exact)) <= tol


def test_log1p64_against_mpmath(ref):
    mpmath.mp.dps = 50
    rng = np.random.default_rng(13)
    xs = np.concatenate([rng.uniform(-0.999, 3.0, 300), rng.uniform(-1e-6, 1e-6, 100),
                         [1e-300, -1e-17, 0.2499999, 0.25, -0.25, -0.2500001]])
    for x in xs:
        exact = float(mpmath.log1p(mpmath.mpf(float(x))))
        got = ref.log1p64(float(x))
        assert abs(got - exact) <= 4.0 * float(np.spacing(abs(exact))), (x, got, exact)


# --------------------------------------------------------------------------
# ln(a!) - ln(b!) without cancellation (the ratio-of-uniforms test statistic).
# --------------------------------------------------------------------------
def test_lnfact_diff_against_mpmath(ref):
    mpmath.mp.dps = 60
    rng = np.random.default_rng(21)
    pairs = [(0, 0), (0, 1), (1023, 1024), (1024, 1023), (5, 1_000_000),
             (2**52, 2**52 - 1), (2**47, 2**47 - 123456), (2**30, 2**30 + 17)]
    for scale in (50, 1023, 1500, 10**5, 10**9, 2**40, 2**47, 2**52 - 2**21):
        for _ in range(30):
            a = int(rng.integers(0, scale + 1))
            d = int(rng.integers(-min(a, 2**20), 2**20))
            pairs.append((a, max(0, min(a + d, 2**52))))
    for a, b in pairs:
        exact = mpmath.loggamma(a + 1) - mpmath.loggamma(b + 1)
        got = ref.lnfact_diff(a, b)
        assert abs(got - float(exact)) <= 1e-13 * max(1.0, abs(float(exact))), (a, b, got, exact)


# --------------------------------------------------------------------------
# Hypergeometric deviates (Sec. 3): exact pmf.
# --------------------------------------------------------------------------
def _hyp_pmf_exact(n, M, N):
    lo, hi = max(0, n - (N - M)), min(n, M)
    tot = math.comb(N, n)
    return lo, [math.comb(M, k) * math.comb(N - M, n - k) / tot for k in range(lo, hi + 1)]


def _chisq_pvalue(obs, probs, min_expected=5.0):
    """Pearson chi-square with tail cells pooled until each expects >= 5."""
    obs = np.asarray(obs, dtype=np.float64)
    probs = np.asarray(probs, dtype=np.float64)
    total = obs.sum()
    exp_ = probs * total
    cells_o, cells_e = [], []
    acc_o = acc_e = 0.0
    for o, e in zip(obs, exp_):
        acc_o += o
        acc_e += e
        if acc_e >= min_expected:
            cells_o.append(acc_o)
            cells_e.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 or acc_o > 0:
        if cells_e:
            cells_o[-1] += acc_o
            cells_e[-1] += acc_e
        else:
            cells_o.append(acc_o)
            cells_e.append(acc_e)
    cells_o, cells_e = np.array(cells_o), np.array(cells_e)
    chi2 = float(((cells_o - cells_e) ** 2 / cells_e).sum())
    dof = max(len(cells_o) - 1, 1)
    return float(stats.chi2.sf(chi2, dof))


HYP_CASES = [
    (5, 7, 20),         # inversion
    (16, 16, 40),       # inversion at its limit
    (17, 40, 90),       # ratio of uniforms, smallest size
    (40, 50, 120),
    (100, 500, 1000),
    (300, 200, 1000),   # M < n
    (700, 400, 1000),   # n > N/2: complement rule
    (300, 800, 1000),   # M > N/2: success/failure swap
    (900, 700, 1000),   # both flips
    (1000, 500, 1000),  # n = N exact case
    (250, 250, 501),    # odd N, M = floor(N/2)
    (3, 1, 10),
    (9, 9, 18),
]


@pytest.mark.parametrize("n,M,N", HYP_CASES)
def test_hyp_exact_pmf(ref, n, M, N):
    draws = ref.hyp_batch(n, M, N, seed=99, id0=1, count=40000).astype(np.int64)
    lo, pmf = _hyp_pmf_exact(n, M, N)
    hi = lo + len(pmf) - 1
    assert draws.min() >= lo and draws.max() <= hi
    obs = np.bincount(draws - lo, minlength=len(pmf))
    assert _chisq_pvalue(obs, pmf) > 1e-4


def test_modes_are_argmax_of_exact_pmf(ref):
    """The ratio-of-uniforms hat is centred on the mode; it must be a maximiser
    of the exact pmf (ties included), for every small parameter set."""
    for N in range(2, 41):
        for M in range(1, N // 2 + 1):
            for n in range(1, N // 2 + 1):
                lo, pmf = _hyp_pmf_exact(n, M, N)
                m = ref.hyp_mode(n, M, N)
                assert lo <= m <= lo + len(pmf) - 1
                assert pmf[m - lo] == max(pmf), (n, M, N, m)
    for Nv in range(2, 30):
        for l in range(1, Nv // 2 + 1):
            for n in range(1, 60):
                pmf = [math.comb(n, k) * l**k * (Nv - l) ** (n - k) for k in range(n + 1)]
                m = ref.bin_mode(n, l, Nv)
                assert pmf[m] == max(pmf), (n, l, Nv, m)


def test_hyp_exact_cases(ref):
    assert ref.hyp(0, 5, 10, 1, 1) == 0
    assert ref.hyp(5, 0, 10, 1, 1) == 0
    assert ref.hyp(5, 10, 10, 1, 1) == 5
    assert ref.hyp(10, 4, 10, 1, 1) == 4
    assert ref.hyp(1, 1, 2, 1, 1) in (0, 1)


def _hyp_logpmf_mp(n, M, N, k):
    lg = mpmath.loggamma
    return (lg(M + 1) - lg(k + 1) - lg(M - k + 1) + lg(N - M + 1) - lg(n - k + 1)
            - lg(N - M - n + k + 1) - lg(N + 1) + lg(n + 1) + lg(N - n + 1))


@pytest.mark.parametrize("n,M,N", [(1 << 30, 1 << 47, 1 << 48),
                                   (3_000_000, 2**41 - 1, 2**42 - 1),
                                   (4095, 2**31, 2**32)])
def test_hyp_large_universe_against_mpmath_pmf(ref, n, M, N):
    """At N up to 2^48 (the paper's experiments use N = 2^50) the deviates
    follow the exact pmf, computed with 50-digit log-gamma; binned into cells
    of equal exact probability mass."""
    mpmath.mp.dps = 50
    draws = ref.hyp_batch(n, M, N, seed=7, id0=1, count=30000).astype(np.int64)
    mu = n * M / N
    sd = math.sqrt(mu * (1 - M / N) * (N - n) / (N - 1))
    # Exact cdf on a grid by summing the pmf: use log-pmf at integer points,
    # summing exactly over k in blocks (pmf is smooth on the scale of sd).
    lo = int(mu - 7 * sd)
    hi = int(mu + 7 * sd) + 1
    step = max(1, int(sd / 200))
    ks = np.arange(lo, hi + 1, step)
    # Euler-Maclaurin: sum over a block of `step` integers ~ step * f(mid).
    mids = ks[:-1] + (step - 1) / 2.0
    pm = np.array([float(mpmath.exp(_hyp_logpmf_mp(n, M, N, mpmath.mpf(float(k)))))
                   for k in mids]) * step
    assert abs(pm.sum() - 1) < 1e-3
    cdf = np.concatenate([[0.0], np.cumsum(pm)])
    # 40 equal-mass cells
    edges = [ks[np.searchsorted(cdf, q)] for q in np.linspace(0, 1, 41)[1:-1]]
    cells = np.searchsorted(np.array(edges), draws, side="right")
    obs = np.bincount(cells, minlength=40)
    probs = np.diff(np.concatenate([[0.0], np.interp(edges, ks, cdf), [1.0]]))
    assert _chisq_pvalue(obs, probs) > 1e-4
    # Mean and variance z-tests against the exact moments.
    z_mean = (draws.mean() - mu) / (sd / math.sqrt(len(draws)))
    assert abs(z_mean) < 4.5
    assert abs(draws.var() / sd**2 - 1) < 0.05


# --------------------------------------------------------------------------
# Binomial deviates (Sec. 4.6 with-replacement split).
# --------------------------------------------------------------------------
BIN_CASES = [(5, 3, 7), (16, 5, 10), (17, 1, 2), (40, 2, 5), (100, 500, 1000),
             (1000, 3, 7), (64, 4, 9), (33, 1, 3)]


@pytest.mark.parametrize("n,l,Nv", BIN_CASES)
def test_binomial_exact_pmf(ref, n, l, Nv):
    draws = ref.binom_batch(n, l, Nv, seed=5, id0=1, count=40000).astype(np.int64)
    p = l / Nv
    pmf = [math.comb(n, k) * p**k * (1 - p) ** (n - k) for k in range(n + 1)]
    assert draws.min() >= 0 and draws.max() <= n
    obs = np.bincount(draws, minlength=n + 1)
    assert _chisq_pvalue(obs, pmf) > 1e-4


def test_binomial_large(ref):
    n, l, Nv = 1 << 28, 1 << 39, 1 << 40
    draws = ref.binom_batch(n, l, Nv, seed=7, id0=1, count=20000).astype(np.float64)
    mu, sd = n / 2, math.sqrt(n) / 2
    assert abs((draws.mean() - mu) / (sd / math.sqrt(len(draws)))) < 4.5
    assert abs(draws.var() / sd**2 - 1) < 0.05
    # odd range: p slightly below 1/2
    n, Nv = 10**7, 2**33 + 1
    l = Nv // 2
    draws = ref.binom_batch(n, l, Nv, seed=8, id0=1, count=20000).astype(np.float64)
    mu, sd = n * l / Nv, math.sqrt(n * (l / Nv) * (1 - l / Nv))
    assert abs((draws.mean() - mu) / (sd / math.sqrt(len(draws)))) < 4.5


def test_binomial_exact_cases(ref):
    assert ref.binom(0, 3, 7, 1, 1) == 0
    assert ref.binom(9, 0, 1, 1, 1) == 0
    assert ref.binom(9, 4, 4, 1, 1) == 9


def test_geometric_uniform_conversion(ref):
    """U = fp32(w+1) 2^-32 covers [2^-32, 1]; exact for w+1 <= 2^24."""
    assert ref.u32_geom(0) == 2.0**-32
    assert ref.u32_geom(2**32 - 1) == 1.0
    for w in (1, 12345, 2**24 - 1):
        assert ref.u32_geom(w) == (w + 1) * 2.0**-32
    w = 2**24 + 1  # w+1 = 2^24+2 is exact too; 2^24+3 rounds to even
    assert ref.u32_geom(w) == (w + 1) * 2.0**-32
    assert ref.u32_geom(2**24 + 2) == float(np.float32(2**24 + 4)) * 2.0**-32
