"""Small sparse and with-replacement leaves (at most 1024 values, ranges that
are not powers of two) run one wave per leaf in k_leaf_small.  Each case is
built so that at least 10^4 leaves of a few hundred values take that path
(the range bound N_v <= 2^32 forces the tree that deep, or n0 is small), and
the whole sample is compared with the oracle bit for bit: plain sparse
leaves, leaves dense enough that Algorithm H's repeat rounds are common, and
with-replacement leaves."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu

CASES = [
    # (variant, n, N, seed, n0): leaves of ~256 values over ranges of ~2^30
    (0, 1 << 23, 3 << 45, 21, None),
    # leaves of 512..1023 values at density ~1/20: repeats in most leaves
    (0, 12_000_000, 240_000_017, 22, 1024),
    # leaves of 200..400 values, n0 = 400
    (0, 5_000_000, 10**12 + 39, 23, 400),
    # with replacement: leaves of ~128 values over ranges of ~2^31
    (1, 1 << 22, 3 << 44, 24, None),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_small_leaves_bitexact(ref, case):
    variant, n, N, seed, n0 = CASES[case]
    m = dcs()
    kw = {} if n0 is None else {"n0": n0}
    if variant == 0:
        internal, leaves, _ = ref.tree_stats(n, N, seed, **kw)
        assert leaves >= 10_000 and 200 <= n / leaves <= 1024, (leaves, n / leaves)
    announce(f"small leaves case {case}: variant={variant} n={n} N={N} seed={seed} n0={n0}")
    f = m.sample if variant == 0 else m.sample_replacement
    out = f(n, N, seed, **kw)
    m.synchronize()
    got = to_np_u64(out)
    want = (ref.sample if variant == 0 else ref.replacement)(n, N, seed, **kw)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_small_leaf_kernel_runs(ref):
    """The one-wave kernel takes the leaves (it is timed with work) and the
    work-group kernel of the back list leaves them alone (it takes next to
    no time)."""
    m = dcs()
    n, N, seed = 1 << 23, 3 << 45, 21
    m.sample(n, N, seed)
    m.synchronize()
    m.profile_enable(True)
    m.sample(n, N, seed)
    m.synchronize()
    small_ms, small_n = m.profile_read(12)
    mixed_ms, _ = m.profile_read(5)
    m.profile_enable(False)
    assert small_n == 1 and small_ms > 0
    assert mixed_ms < small_ms


TINY = [
    # (variant, n, N, seed, n0): leaves of one to 32 values, which the tree
    # kernel samples itself (the range bound forces the tree deep, or n0 is
    # small)
    (0, 300_000, 1 << 60, 31, None),
    (0, 200_000, (1 << 58) + 12345, 32, None),   # ranges that are not powers of two
    (1, 250_000, (1 << 55) + 7, 33, None),
    (0, 60_000, 1 << 40, 34, 3),                  # n0 = 3: leaves of 1 or 2 values
    (1, 80_000, 1 << 20, 35, 4),                  # with replacement: repeats inside tiny leaves
    (0, 5_000, 1 << 16, 36, 2),                   # leaves of one value; dense ones stay jobs
    (0, 1 << 20, 1 << 40, 37, 32),                # leaves of 16..31 values
    (1, 300_000, 1 << 36, 38, 20),                # with replacement, up to 19 values
    (0, 1 << 24, 1 << 54, 40, None),              # ~4 values per leaf, tails past 10
    (0, 400_000, 3_000_000_019, 41, 33),          # up to 32 values, ranges not powers of two
]


@pytest.mark.parametrize("case", range(len(TINY)))
def test_tiny_leaves_bitexact(ref, case):
    variant, n, N, seed, n0 = TINY[case]
    m = dcs()
    kw = {} if n0 is None else {"n0": n0}
    if variant == 0:
        _, leaves, _ = ref.tree_stats(n, N, seed, **kw)
        assert n / leaves <= 32, (leaves, n / leaves)
    announce(f"tiny leaves case {case}: variant={variant} n={n} N={N} seed={seed} n0={n0}")
    f = m.sample if variant == 0 else m.sample_replacement
    out = f(n, N, seed, **kw)
    m.synchronize()
    got = to_np_u64(out)
    want = (ref.sample if variant == 0 else ref.replacement)(n, N, seed, **kw)
    assert np.array_equal(got, want), first_mismatch(got, want)
