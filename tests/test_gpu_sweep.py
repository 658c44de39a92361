"""Seeded random sweep of the sampling entry points on the GPU against the
oracle, bit for bit: universes from 1 to 2^62, densities from one value to
the whole range, every leaf size n0 class, both split variants, dense_ratio
at its bounds, Bernoulli p over nine decades, whole-range B and uneven
universes.  The cases are drawn once, from a fixed seed, when the module is
imported, so a failure names a reproducible case."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu

_R = np.random.default_rng(20261203)
N0S = [2, 3, 7, 16, 100, 512, 1024, 4096]


def _tree_case():
    variant = int(_R.integers(0, 2))
    N = int(min(2 ** 62, max(1, round(2 ** _R.uniform(0, 62)))))
    cap = 1 << 18
    if variant == 0:
        top = min(N, cap)
        n = int(min(top, round(2 ** _R.uniform(0, np.log2(top + 1)))))
        if _R.random() < 0.1:
            n = top  # the whole range (or as much of it as the case allows)
    else:
        n = int(round(2 ** _R.uniform(0, 18)))
    n0 = int(_R.choice(N0S))
    dr = int(_R.choice([2, 16, 64]))
    seed = int(_R.integers(0, 2 ** 63))
    return variant, n, N, seed, n0, dr


TREE = [_tree_case() for _ in range(300)] + [(0, 0, 5, 1, 16, 16), (1, 0, 1, 2, 4096, 16),
                                              (1, 1000, 1, 3, 2, 16), (0, 1, 1, 4, 2, 2)]


def _bern_case():
    lp = _R.uniform(-30, 0)
    p = float(2 ** lp)
    N = int(max(1, min(2 ** 52, round(2 ** _R.uniform(0, 52)))))
    N = int(min(N, max(1, (1 << 20) / p)))  # about a million hits at most
    return p, N, int(_R.integers(0, 2 ** 63)), int(_R.choice(N0S))


BERN = [_bern_case() for _ in range(80)]


def _wb_case():
    N = int(round(2 ** _R.uniform(10, 26)))
    rho = 2 ** _R.uniform(-9.5, 0)
    n = int(min(N, max(1, round(N * rho))))
    return n, N, int(_R.integers(0, 2 ** 63))


WB = [_wb_case() for _ in range(30)]


def _seg_case():
    K = int(_R.integers(1, 300))
    L = [int(round(2 ** _R.uniform(0, 34))) if _R.random() > 0.1 else 0 for _ in range(K)]
    if sum(L) == 0:
        L[0] = 1
    n = int(min(sum(L), round(2 ** _R.uniform(0, 18))))
    return L, n, int(_R.integers(0, 2 ** 63)), int(_R.choice(N0S))


SEGS = [_seg_case() for _ in range(30)]


@pytest.mark.parametrize("case", range(len(TREE)))
def test_sweep_tree(ref, case):
    variant, n, N, seed, n0, dr = TREE[case]
    m = dcs()
    announce(f"sweep tree {case}: variant={variant} n={n} N={N} seed={seed} n0={n0} dr={dr}")
    if variant == 0:
        out = m.sample(n, N, seed, n0=n0, dense_ratio=dr)
        m.synchronize()
        want = ref.sample(n, N, seed, n0=n0, dense_ratio=dr)
    else:
        out = m.sample_replacement(n, N, seed, n0=n0)
        m.synchronize()
        want = ref.replacement(n, N, seed, n0=n0)
    got = to_np_u64(out[:n])
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("case", range(len(BERN)))
def test_sweep_bernoulli(ref, case):
    p, N, seed, n0 = BERN[case]
    m = dcs()
    announce(f"sweep bernoulli {case}: p={p!r} N={N} seed={seed} n0={n0}")
    out, cnt = m.sample_bernoulli(p, N, seed, n0=n0)
    m.synchronize()
    want = ref.bernoulli(p, N, seed, n0=n0)
    c = int(cnt.item())
    assert c == want.size
    got = to_np_u64(out[:c])
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("case", range(len(WB)))
def test_sweep_wholerange(ref, case):
    n, N, seed = WB[case]
    m = dcs()
    announce(f"sweep whole-range B {case}: n={n} N={N} seed={seed}")
    out = m.sample_wholerange(n, N, seed)
    m.synchronize()
    want, _ = ref.sample_wholerange(n, N, seed)
    got = to_np_u64(out[:n])
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("case", range(len(SEGS)))
def test_sweep_segments(ref, case):
    L, n, seed, n0 = SEGS[case]
    m = dcs()
    announce(f"sweep segments {case}: K={len(L)} N={sum(L)} n={n} seed={seed} n0={n0}")
    out, cnt = m.sample_segments(n, L, seed, n0=n0)
    m.synchronize()
    want, want_c = ref.sample_segments(n, L, seed, n0=n0)
    got = to_np_u64(out[:n])
    assert np.array_equal(got, want), first_mismatch(got, want)
    assert np.array_equal(to_np_u64(cnt[:len(L)]), want_c)
