"""The oracle's pins are strong enough: each plausible mistake planted in a
copy of the oracle (on the CPU) is caught by at least one pin.

Every mutant is a one-line edit of oracle/dcs_oracle.c compiled into its own
library; the pin suite below runs against it and must report a failure,
while the unmodified oracle must pass it."""
import ctypes
import itertools
import math
import os
import subprocess
import sys

import mpmath
import numpy as np
import pytest

import oracle
from tests.test_oracle_primitives import _chisq_pvalue, _hyp_pmf_exact, _kat_rows

SRC = oracle.SRC_PATH

# (name, original text, replacement): each is a plausible slip.
MUTANTS = [
    ("philox multiplier swapped", "uint64_t prod0 = (uint64_t)0xD2511F53u * c0;",
     "uint64_t prod0 = (uint64_t)0xCD9E8D57u * c0;"),
    ("philox key bump dropped", "      k1 += 0xBB67AE85u;", "      k1 += 0u;"),
    ("range map void test <=", "if ((m & 0xFFFFFFFFULL) < threshold) return -1;",
     "if ((m & 0xFFFFFFFFULL) <= threshold) return -1;"),
    ("log series cut short", "  double p = 1.0 / 23.0;\n  p = 1.0 / 21.0 + z * p;\n  p = 1.0 / 19.0 + z * p;\n  p = 1.0 / 17.0 + z * p;",
     "  double p = 1.0 / 17.0;"),
    ("log reduction threshold", "  if (m >= REF_SQRT2) {", "  if (m >= 2.0) {"),
    ("stirling operand transposed", "double t1 = (zb - 0.5) * log1p64(d / zb);",
     "double t1 = (za - 0.5) * log1p64(d / zb);"),
    ("stirling correction sign", "return r * (1.0 / 12.0 - r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0)));",
     "return r * (1.0 / 12.0 + r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0)));"),
    ("hyp fourth term dropped", "    T = T + lnfact_diff(nmM + mode, nmM + k);\n", "\n"),
    ("hyp term sign", "    T = T + lnfact_diff(M - mode, M - k);", "    T = T - lnfact_diff(M - mode, M - k);"),
    ("hyp mode off by one", "  return muldiv_floor(n + 1, M + 1, N + 2);",
     "  return muldiv_floor(n + 1, M + 1, N + 1);"),
    ("binomial mode off by one", "  return muldiv_floor(n + 1, l, Nv);", "  return muldiv_floor(n, l, Nv);"),
    ("hyp inversion ratio index", "((double)(n - k) / (double)(N - M - n + k + 1));",
     "((double)(n - k) / (double)(N - M - n + k + 2));"),
    ("hyp complement flip", "  if (flip_n) k = M - k;", "  if (flip_n) k = n1 - k;"),
    ("hyp hat width", "  double s = REF_D1 * w + REF_D2;\n  uint64_t mode = hyp_mode(n, M, N);",
     "  double s = 0.5 * REF_D1 * w;\n  uint64_t mode = hyp_mode(n, M, N);"),
    ("binomial log-odds sign", "    double T = (double)((int64_t)k - (int64_t)mode) * lodds;",
     "    double T = (double)((int64_t)mode - (int64_t)k) * lodds;"),
    ("binomial inversion odds", "    double odds = (double)l / (double)r;", "    double odds = (double)r / (double)l;"),
    ("tree split at ceil", "  uint64_t l = Nv / 2;\n  uint64_t L = hyp(nv, l, Nv, c->seed, id);",
     "  uint64_t l = (Nv + 1) / 2;\n  uint64_t L = hyp(nv, l, Nv, c->seed, id);"),
    ("tree right offset", "return sample_r(c, 2 * id + 1, lo + l, Nv - l, nv - L, off + L, k);",
     "return sample_r(c, 2 * id + 1, lo + l - 1, Nv - l, nv - L, off + L, k);"),
    ("H keeps duplicates", "    if (h->slot[i] == v + 1) return 0;", "    if (h->slot[i] == v + 1) return 1;"),
    ("dense repair removes neighbour", "      if (j < r && rem[j] == t) { ++j; continue; }",
     "      if (j < r && rem[j] == t + 1) { ++j; continue; }"),
    ("dense first position", "    int64_t p = -1;\n    uint64_t cnt = 0;", "    int64_t p = 0;\n    uint64_t cnt = 0;"),
    ("bernoulli skip off by one", "        double np = (double)pos + (double)g + 1.0;",
     "        double np = (double)pos + (double)g + 2.0;"),
    ("geometric uniform scale", "  return x * 0x1p-32f;", "  return x * 0x1p-31f;"),
    ("segment split sizes swapped", "hyp_stream(cnt[id], Ll, Ll + Lr, seed, id, P_SEGSPLIT)",
     "hyp_stream(cnt[id], Lr, Ll + Lr, seed, id, P_SEGSPLIT)"),
    ("segment upward sum drops right subtree",
     "sums[first + a] = sums[2 * (first + a)] + sums[2 * (first + a) + 1];",
     "sums[first + a] = sums[2 * (first + a)];"),
    ("segment values not shifted", "rc = sample_r(&c, 1, base, lengths[i], ni, 0, &k);",
     "rc = sample_r(&c, 1, 0, lengths[i], ni, 0, &k);"),
    ("segments share one seed", "        c.seed = stream_draw64(&st, 0);", "        c.seed = seed;"),
    ("wholerange output off by one", "      out[o++] = pos[h] + 1;", "      out[o++] = pos[h];"),
    ("wholerange repair range short", "rc = first_distinct_sorted(&sr, r, nh, rem);",
     "rc = first_distinct_sorted(&sr, r, nh - 1, rem);"),
    ("wholerange skip gap", "      double nq = (double)q + (double)g + 1.0;",
     "      double nq = (double)q + (double)g + 2.0;"),
    ("wholerange removes neighbour", "      if (j < r && rem[j] == h) { ++j; continue; }",
     "      if (j < r && rem[j] == h + 1) { ++j; continue; }"),
    ("segment tree one level short", "  for (uint32_t j = D; j >= 1; --j) {", "  for (uint32_t j = D; j >= 2; --j) {"),
]


def _build(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", *oracle.CFLAGS, f"-I{os.path.dirname(SRC)}", "-o", str(so),
                    str(src), "-lm"], check=True)
    return oracle.configure(ctypes.CDLL(str(so)))


def pin_failures(L) -> list:
    """A quick run of the oracle pins against library L; returns the names of
    the pins that fail."""
    saved = oracle._lib
    oracle._lib = L
    bad = []
    try:
        def check(name, fn):
            try:
                ok = fn()
            except Exception:
                ok = False
            if not ok:
                bad.append(name)

        check("philox KAT", lambda: all(oracle.philox(c, k) == w for c, k, w in _kat_rows()))

        def range_rule():
            s = 2**31 + 1
            thr = (1 << 32) % s
            for w in np.random.default_rng(3).integers(0, 2**32, 3000):
                w = int(w)
                want = -1 if ((w * s) & 0xFFFFFFFF) < thr else (w * s) >> 32
                if oracle.range_map(w, s) != want:
                    return False
            # the word whose low product half equals the threshold is accepted
            w = (thr * pow(s, -1, 1 << 32)) % (1 << 32)
            return oracle.range_map(w, s) == (w * s) >> 32
        check("range map rule", range_rule)

        def logs():
            r = np.random.default_rng(12)
            x = np.concatenate([np.exp(r.uniform(-700, 700, 20000)), r.uniform(0.5, 2.0, 20000)])
            e = np.abs(oracle.log64_batch(x) - np.log(x)) / np.spacing(np.abs(np.log(x)))
            xf = np.random.default_rng(1).uniform(2**-32, 1, 20000).astype(np.float32)
            ef = np.abs(oracle.log32_batch(xf).astype(np.float64) - np.log(xf.astype(np.float64)))
            ulp = np.spacing(np.abs(np.log(xf.astype(np.float64))).astype(np.float32)).astype(np.float64)
            return e.max() <= 3 and (ef / ulp).max() <= 2
        check("logarithms", logs)

        def lnfact():
            mpmath.mp.dps = 40
            for a, b in [(5000, 4321), (2**40, 2**40 - 99999), (70, 65), (2**47, 2**47 + 3)]:
                ex = float(mpmath.loggamma(a + 1) - mpmath.loggamma(b + 1))
                if abs(oracle.lnfact_diff(a, b) - ex) > 1e-12 * max(1, abs(ex)):
                    return False
            return True
        check("lnfact diff", lnfact)

        def hyp_small():
            for n, M, N in [(5, 7, 20), (40, 50, 120), (700, 400, 1000), (300, 800, 1000)]:
                d = oracle.hyp_batch(n, M, N, 99, 1, 20000).astype(np.int64)
                lo, pmf = _hyp_pmf_exact(n, M, N)
                if d.min() < lo or d.max() > lo + len(pmf) - 1:
                    return False
                if _chisq_pvalue(np.bincount(d - lo, minlength=len(pmf)), pmf) < 1e-4:
                    return False
            return True
        check("hypergeometric pmf", hyp_small)

        def bin_small():
            for n, l, Nv in [(5, 3, 7), (40, 2, 5), (100, 500, 1000)]:
                d = oracle.binom_batch(n, l, Nv, 5, 1, 20000).astype(np.int64)
                p = l / Nv
                pmf = [math.comb(n, k) * p**k * (1 - p) ** (n - k) for k in range(n + 1)]
                if d.min() < 0 or d.max() > n:
                    return False
                if _chisq_pvalue(np.bincount(d, minlength=n + 1), pmf) < 1e-4:
                    return False
            return True
        check("binomial pmf", bin_small)

        def subsets():
            for N, n, n0, dr in [(12, 5, 2, 2), (20, 3, 4, 16), (16, 8, 4, 16), (13, 6, 8, 16)]:
                cells = list(itertools.combinations(range(1, N + 1), n))
                idx = {c: i for i, c in enumerate(cells)}
                obs = np.zeros(len(cells))
                for seed in range(max(20000, 25 * len(cells))):
                    t = tuple(int(v) for v in oracle.sample(n, N, seed, n0=n0, dense_ratio=dr))
                    if t not in idx:
                        return False
                    obs[idx[t]] += 1
                if _chisq_pvalue(obs, np.full(len(cells), 1 / len(cells))) < 1e-4:
                    return False
            return True
        check("uniform subsets", subsets)

        def modes():
            for N in range(2, 30):
                for M in range(1, N // 2 + 1):
                    for n in range(1, N // 2 + 1):
                        lo, pmf = _hyp_pmf_exact(n, M, N)
                        m = oracle.hyp_mode(n, M, N)
                        if not (lo <= m < lo + len(pmf)) or pmf[m - lo] != max(pmf):
                            return False
            for Nv in range(2, 20):
                for l in range(1, Nv // 2 + 1):
                    for n in range(1, 40):
                        pmf = [math.comb(n, k) * l**k * (Nv - l) ** (n - k) for k in range(n + 1)]
                        if pmf[oracle.bin_mode(n, l, Nv)] != max(pmf):
                            return False
            return True
        check("modes", modes)

        def split_position():
            for n, N, seed, n0 in [(5000, 10**6 + 7, 3, 256), (7, 21, 5, 2)]:
                s_ = oracle.sample(n, N, seed, n0=n0)
                if int(np.searchsorted(s_, N // 2, side="right")) != oracle.hyp(n, N // 2, N, seed, 1):
                    return False
            return True
        check("split position", split_position)

        def prefix():
            n, N = 2000, 10**6 + 7
            c = [int(np.searchsorted(oracle.sample(n, N, s, n0=128), N // 3, side="right"))
                 for s in range(600)]
            mu = n / 3
            sd = math.sqrt(n * (1 / 3) * (2 / 3) * (N - n) / (N - 1))
            return abs(np.mean(c) - mu) < 4.5 * sd / math.sqrt(len(c))
        check("prefix counts", prefix)

        def bernoulli():
            p, N = 0.3, 8
            obs = np.zeros(1 << N)
            for seed in range(20000):
                mk = 0
                for v in oracle.bernoulli(p, N, seed):
                    mk |= 1 << (int(v) - 1)
                obs[mk] += 1
            probs = [p ** bin(m).count("1") * (1 - p) ** (N - bin(m).count("1")) for m in range(1 << N)]
            s = oracle.bernoulli(0.01, 1 << 22, 5).astype(np.int64)
            gaps = np.diff(s)
            g1 = (gaps == 1).mean()
            return _chisq_pvalue(obs, probs) > 1e-4 and abs(g1 - 0.01) < 0.002
        check("bernoulli", bernoulli)

        def replacement():
            N, n = 3, 4
            cells = list(itertools.combinations_with_replacement(range(1, N + 1), n))
            idx = {c: i for i, c in enumerate(cells)}
            probs = []
            for c in cells:
                m = math.factorial(n)
                for v in set(c):
                    m //= math.factorial(c.count(v))
                probs.append(m / N**n)
            obs = np.zeros(len(cells))
            for seed in range(20000):
                t = tuple(int(v) for v in oracle.replacement(n, N, seed, n0=2))
                if t not in idx:
                    return False
                obs[idx[t]] += 1
            return _chisq_pvalue(obs, probs) > 1e-4
        check("with replacement", replacement)

        def segments():
            # per-segment counts: multivariate hypergeometric
            L, n = [2, 0, 3, 1, 2], 3
            N = sum(L)
            vecs = [v for v in itertools.product(*[range(x + 1) for x in L]) if sum(v) == n]
            probs = [math.prod(math.comb(x, k) for x, k in zip(L, v)) / math.comb(N, n)
                     for v in vecs]
            idx = {v: i for i, v in enumerate(vecs)}
            obs = np.zeros(len(vecs))
            for seed in range(8000):
                _, c = oracle.sample_segments(n, L, seed, n0=2)
                obs[idx[tuple(int(x) for x in c)]] += 1
            if _chisq_pvalue(obs, probs) < 1e-4:
                return False
            # all subsets of two equal segments
            cells = list(itertools.combinations(range(1, 7), 2))
            ci = {c: i for i, c in enumerate(cells)}
            obs = np.zeros(len(cells))
            for seed in range(6000):
                v, _ = oracle.sample_segments(2, [3, 3], seed, n0=2)
                t = tuple(int(x) for x in v)
                if t not in ci:
                    return False
                obs[ci[t]] += 1
            if _chisq_pvalue(obs, np.full(len(cells), 1 / len(cells))) < 1e-4:
                return False
            # counts add up on the paper's 13-PE example and land in their segments
            L13 = [20, 15, 30, 5, 17, 25, 10, 22, 18, 12, 20, 15, 20]
            v, c = oracle.sample_segments(50, L13, 3, n0=8)
            per = np.histogram(v.astype(np.int64), bins=np.cumsum([0] + L13) + 0.5)[0]
            return int(c.sum()) == 50 and per.tolist() == c.tolist()
        check("uneven universe", segments)

        def wholerange():
            n, N = 2, 40
            cells = list(itertools.combinations(range(1, N + 1), n))
            ci = {c: i for i, c in enumerate(cells)}
            obs = np.zeros(len(cells))
            for seed in range(12000):
                v, _ = oracle.sample_wholerange(n, N, seed, n0=16)
                t = tuple(int(x) for x in v)
                if t not in ci:
                    return False
                obs[ci[t]] += 1
            if _chisq_pvalue(obs, np.full(len(cells), 1 / len(cells))) < 1e-4:
                return False
            v, _ = oracle.sample_wholerange(30, 40, 3, n0=16)
            return v.size == 30 and len(set(v.tolist())) == 30 and 1 <= v.min() and v.max() <= 40
        check("whole-range B", wholerange)
    finally:
        oracle._lib = saved
    return bad


_RUNNER = r"""
import ctypes, sys
sys.path.insert(0, {root!r})
import oracle
from tests.test_oracle_mutants import pin_failures
L = oracle.configure(ctypes.CDLL({so!r}))
bad = pin_failures(L)
print("FAILED:" + ",".join(bad) if bad else "PASSED", flush=True)
"""


def _suite_verdict(so: str, timeout: float) -> str:
    """Run the pin suite against library `so` in a child process; a run that
    does not finish in time (e.g. a rejection loop that never accepts) is a
    failure too."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    try:
        r = subprocess.run([sys.executable, "-c", _RUNNER.format(root=root, so=so)],
                           capture_output=True, text=True, timeout=timeout)
    except subprocess.TimeoutExpired:
        return "FAILED:did not finish"
    out = r.stdout.strip().splitlines()
    if r.returncode != 0 or not out:
        return "FAILED:crashed"
    return out[-1]


def test_unmodified_oracle_passes_the_pin_suite(tmp_path):
    _build(tmp_path, "orig", open(SRC).read())
    assert _suite_verdict(str(tmp_path / "orig.so"), 300) == "PASSED"


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert old in text, f"mutation anchor not found: {name}"
    _build(tmp_path, "mut", text.replace(old, new, 1))
    verdict = _suite_verdict(str(tmp_path / "mut.so"), 60)
    assert verdict.startswith("FAILED"), f"no pin caught the planted mistake: {name}"
