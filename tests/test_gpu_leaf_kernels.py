"""Which leaf kernels run never changes a sample (Sec. 4.5: the result is a
function of the input alone).  A single-instance call leaves out the
specialised leaf kernels (one-wave dense, one-wave small, one-pass) whose
leaves its tree cannot plausibly hold, and the general work-group kernel then
runs any such leaf itself.  The test hook forces the choice: every kind of
leaf is sampled once by its own kernel (mask 0) and once by the general
kernel (mask 7), and by default; all against the oracle, bit for bit."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu

CASES = [
    # (variant, n, N, seed, n0): the leaf kind the case is made of
    (0, 1 << 20, 1 << 21, 61, 4096),              # dense leaves over ranges below 2^16
    (0, 200_000, 10**9 + 7, 62, 512),             # sparse leaves of 256-511 values
    (1, 200_000, 10**9 + 7, 63, 512),             # with-replacement leaves of 256-511
    (0, 1 << 20, 20 * (1 << 20) + 12345, 64, 4096),  # sparse leaves expected to repeat
    (0, 1 << 22, 1 << 40, 65, 4096),              # power-of-two ranges (front list)
    (1, 300_000, 3, 66, 4096),                    # constant leaves cut into pieces
    # around N = n n0, where a single call stops launching the one-pass kernel
    (0, 1 << 20, (1 << 31) + 11, 67, 4096),       # N = n n0 / 2: one-pass leaves
    (0, 1 << 20, 1 << 32, 68, 4096),              # N = n n0: none expected
    (0, 300_000, 300_000 * 1500 - 1, 69, 1500),   # just below n n0
]


@pytest.fixture
def m():
    mod = dcs()
    yield mod
    mod.debug_leaf_kernels(-1)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_leaf_kernel_choice_never_changes_the_sample(ref, m, case):
    variant, n, N, seed, n0 = CASES[case]
    want = ref.replacement(n, N, seed, n0=n0) if variant else ref.sample(n, N, seed, n0=n0)
    for mask in (0, 7, -1):
        m.debug_leaf_kernels(mask)
        announce(f"leaf kernels mask {mask}: variant={variant} n={n} N={N} seed={seed} n0={n0}")
        f = m.sample_replacement if variant else m.sample
        out = f(n, N, seed, n0=n0)
        m.synchronize()
        got = to_np_u64(out)
        assert np.array_equal(got, want), (mask, first_mismatch(got, want))


def test_leaf_kernel_mask_rejected_above_limit():
    mod = dcs()
    with pytest.raises(mod.DcsError):
        mod.debug_leaf_kernels(8)
    mod.debug_leaf_kernels(-1)


SESSION_CASES = [
    # (variant, n, N, seed, n0, depth): parts of samples with the leaf kinds above
    (0, 1 << 20, 1 << 21, 81, 4096, 6),               # dense leaves
    (0, 1 << 20, 20 * (1 << 20) + 12345, 82, 4096, 5),  # sparse leaves expected to repeat
    (0, 200_000, 10**9 + 7, 83, 512, 7),              # sparse leaves of 256-511 values
    (1, 200_000, 10**9 + 7, 84, 512, 4),              # with-replacement leaves
]


@pytest.mark.parametrize("case", range(len(SESSION_CASES)))
def test_leaf_kernel_choice_in_sessions(ref, m, case):
    """An online session's calls are subtrees of one sample's tree and leave
    out the same kernels as the whole sample's call; forced either way, and
    by default, every part read in runs of 3 equals the oracle's sample."""
    import torch
    variant, n, N, seed, n0, depth = SESSION_CASES[case]
    want = ref.replacement(n, N, seed, n0=n0) if variant else ref.sample(n, N, seed, n0=n0)
    for mask in (0, 7, -1):
        m.debug_leaf_kernels(mask)
        announce(f"session leaf kernels mask {mask}: variant={variant} n={n} N={N} "
                 f"seed={seed} n0={n0} depth={depth}")
        o = m.Online(n, N, seed, depth, variant=variant, n0=n0)
        buf = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        pos = 0
        for g in range(0, o.parts, 3):
            pos += o.next(g, min(3, o.parts - g), buf[pos:])
        m.synchronize()
        o.close()
        assert pos == n
        got = to_np_u64(buf)
        assert np.array_equal(got, want), (mask, first_mismatch(got, want))
