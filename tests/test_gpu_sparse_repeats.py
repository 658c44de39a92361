"""Sparse leaves whose first n_v values repeat (Algorithm H's duplicates,
Sec. 2), on the GPU against the oracle, bit for bit.

A sparse leaf of more than 1024 values with n_v^2 / (2 N_v) of at least
one (its first n_v values are expected to repeat) takes one pass over the
first W words of its stream, W = n_v plus margins for repeats and void words
(at most 4096); when fewer than n_v distinct values occur there, the repeat
rounds continue from word W.  Such leaves over power-of-two ranges leave
the power-of-two kernel for the same sampler (those of at most 1024
values for the one-wave kernel).  The cases below are chosen so that both
branches run, which `leaf_paths` checks on the CPU from the oracle's tree
and streams (the sizing rule is restated here; it decides only how much
work a leaf does, never its values)."""
import math

import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

KEYS = 4096
SMALL_MAX = 1024


def _isqrt(x: int) -> int:
    return math.isqrt(x)


def one_pass_words(nv: int, Nv: int) -> int:
    """W of the one-pass leaf (the kernel's sizing rule)."""
    thr = (1 << 32) % Nv
    r = (nv * nv) // (2 * Nv)
    base = nv + r + (r >> 2) + 4 * _isqrt(r) + 16
    full = base + ((2 * base * thr) >> 32) + 32
    return min(full, KEYS)


def leaves(ref, n, N, seed, n0, dense_ratio):
    """(id, N_v, n_v) of the sparse leaves of the canonical tree (C4, C5)."""
    out, todo = [], [(1, N, n)]
    while todo:
        node, Nv, nv = todo.pop()
        if nv == 0:
            continue
        if nv < n0 and Nv <= (1 << 32):
            if dense_ratio * nv < Nv:
                out.append((node, Nv, nv))
            continue
        l = Nv // 2
        L = ref.hyp(nv, l, Nv, seed, node)
        todo.append((2 * node, l, L))
        todo.append((2 * node + 1, Nv - l, nv - L))
    return out


def leaf_paths(ref, n, N, seed, n0, dense_ratio, limit=40):
    """Counts of one-pass leaves that finish in the pass and that continue in
    rounds, over at most `limit` one-pass leaves of the tree."""
    done = rounds = 0
    for node, Nv, nv in leaves(ref, n, N, seed, n0, dense_ratio):
        if nv <= SMALL_MAX or nv * nv < 2 * Nv:
            continue
        W = one_pass_words(nv, Nv)
        seen = set()
        for t in range(W):
            v = ref.range_map(ref.stream_word(seed, node, ref.P_LEAF, 0, t), Nv)
            if v >= 0:
                seen.add(v)
        if len(seen) >= nv:
            done += 1
        else:
            rounds += 1
        if done + rounds >= limit:
            break
    return done, rounds


CASES = [
    # (n, N, seed, n0, dense_ratio): density, so expected repeats per leaf
    (1 << 20, 20 * (1 << 20) + 12345, 41, 4096, 16),   # ~1/20: tens of repeats
    (1 << 18, 1000 * (1 << 18) + 7, 42, 4096, 16),     # ~1e-3: a few
    (1 << 18, 1300 * (1 << 18) + 3, 43, 4096, 16),     # ~7.7e-4: near the threshold
    (1 << 19, 3 * (1 << 19) + 1, 44, 4096, 2),         # 1/3: W capped, rounds follow
    (300_000, 5 * 300_000 - 11, 45, 3000, 4),          # 1/5, leaves of 1500-3000
    (200_000, 40 * 200_000 + 99, 46, 1500, 16),        # leaves just above 1024
    (1 << 20, 1 << 25, 47, 4096, 16),                  # power-of-two ranges, 1/32
    (1 << 18, 1 << 23, 48, 512, 16),                   # the same, leaves of 256-511
    (1 << 19, 1 << 22, 49, 2048, 4),                   # power-of-two ranges, 1/8
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_one_pass_paths_are_exercised(ref, case):
    """CPU only: the case has one-pass leaves; over all cases both branches
    occur (checked per case where the case is meant for it)."""
    n, N, seed, n0, dr = CASES[case]
    done, rounds = leaf_paths(ref, n, N, seed, n0, dr)
    if n0 <= SMALL_MAX:
        return  # leaves for the one-wave kernel
    assert done + rounds > 0, "no leaf takes the one-pass path"
    if case == 0:
        assert done > 0 and rounds > 0, (done, rounds)
    if case == 3:
        assert rounds > 0, (done, rounds)


def one_pass_leaves(ref, n, N, seed, n0, dense_ratio):
    """Sparse leaves of the canonical tree that the one-pass kernel takes."""
    return [(node, Nv, nv) for node, Nv, nv in leaves(ref, n, N, seed, n0, dense_ratio)
            if nv > SMALL_MAX and nv * nv >= 2 * Nv]


@pytest.mark.parametrize("n,N,seed,n0,dr", [
    (1 << 20, 1 << 32, 71, 4096, 16),
    (1 << 20, (1 << 32) + 12345, 72, 4096, 4),
    (1 << 18, 1500 * (1 << 18), 73, 1500, 16),
    (1 << 19, 3 * 4096 * (1 << 19) // 2, 74, 4096, 16),
])
def test_no_one_pass_leaf_when_N_is_at_least_n_n0(ref, n, N, seed, n0, dr):
    """CPU only: a single call with N >= n n0 does not launch the one-pass
    kernel, since such a leaf would need a count more than twice its range's
    expectation; the canonical trees agree (the general kernel would take any
    such leaf, so this decides only the work, never the sample)."""
    assert N >= n * n0
    assert one_pass_leaves(ref, n, N, seed, n0, dr) == []


def test_one_pass_leaves_below_the_threshold(ref):
    """CPU only: the check above can fail: at N = n n0 / 4 the tree has
    one-pass leaves."""
    n, n0 = 1 << 20, 4096
    assert len(one_pass_leaves(ref, n, n * n0 // 4, 75, n0, 16)) > 0


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(len(CASES)))
def test_repeating_sparse_leaves_match_oracle(ref, case):
    n, N, seed, n0, dr = CASES[case]
    m = dcs()
    announce(f"sparse repeats case {case}: n={n} N={N} seed={seed} n0={n0} dr={dr}")
    out = m.sample(n, N, seed, n0=n0, dense_ratio=dr)
    m.synchronize()
    want = ref.sample(n, N, seed, n0=n0, dense_ratio=dr)
    got = to_np_u64(out)
    assert np.array_equal(got, want), first_mismatch(got, want)
