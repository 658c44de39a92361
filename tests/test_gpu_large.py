"""Parity at the full benchmark sizes (GPU): the whole output is produced in
the launch configuration the benchmark times; the oracle recomputes sampled
windows of it on its own (visiting only the subtrees that overlap each
window), and properties that hold at any size are checked on everything.
"""
import math

import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu


def _windows(n, count, width, seed):
    rng = np.random.default_rng(seed)
    starts = [0, max(0, n - width), max(0, n // 2 - width // 2)]
    starts += [int(x) for x in rng.integers(0, max(1, n - width), size=count)]
    return [(s, min(width, n - s)) for s in starts]


def _strictly_increasing(out, lo, hi, strict=True):
    import torch
    step = 1 << 27
    n = out.numel()
    ok = True
    for a in range(0, n, step):
        b = min(n, a + step + 1)
        seg = out[a:b]
        d = seg[1:] - seg[:-1]
        ok &= bool((d > 0).all()) if strict else bool((d >= 0).all())
    return ok and int(out[0]) >= lo and int(out[-1]) <= hi


def _check_windows(ref_fn, out, wins):
    for s, c in wins:
        got = to_np_u64(out[s:s + c])
        want = ref_fn(s, c)
        assert np.array_equal(got, want), f"window {s}+{c}: {first_mismatch(got, want)}"


def test_config2a_sparse_8gib(ref):
    n, N, seed = 1 << 30, 1 << 48, 7
    m = dcs()
    announce("config 2a full size")
    out = m.sample(n, N, seed)
    m.synchronize()
    assert _strictly_increasing(out, 1, N)
    _check_windows(lambda s, c: ref.sample_window(n, N, seed, s, c), out,
                   _windows(n, 24, 1 << 15, 1))


def test_config2b_dense_4gib(ref):
    n, N, seed = 1 << 29, 1 << 30, 7
    m = dcs()
    announce("config 2b full size")
    out = m.sample(n, N, seed)
    m.synchronize()
    assert _strictly_increasing(out, 1, N)
    _check_windows(lambda s, c: ref.sample_window(n, N, seed, s, c), out,
                   _windows(n, 24, 1 << 15, 2))


def test_config3a_bernoulli(ref):
    p, N, seed = 0.01, 1 << 36, 7
    m = dcs()
    announce("config 3a Bernoulli full size")
    out, cnt = m.sample_bernoulli(p, N, seed)
    m.synchronize()
    c = int(cnt.item())
    mu, sd = N * p, math.sqrt(N * p * (1 - p))
    assert abs(c - mu) < 6 * sd
    out = out[:c]
    assert _strictly_increasing(out, 1, N)
    C = ref.bernoulli_chunk_len(p)
    n_chunks = (N + C - 1) // C
    rng = np.random.default_rng(3)
    import torch
    for j in [0, n_chunks - 4] + [int(x) for x in rng.integers(0, n_chunks - 4, 12)]:
        want = ref.bernoulli_chunks(p, N, seed, j, j + 4)
        lo = int(torch.searchsorted(out, torch.tensor([j * C + 1], device="cuda")).item())
        got = to_np_u64(out[lo:lo + want.size])
        assert np.array_equal(got, want), f"chunks {j}..{j + 3}: {first_mismatch(got, want)}"
        if lo + want.size < c:
            assert int(out[lo + want.size]) > (j + 4) * C


def test_config3b_with_replacement(ref):
    n, N, seed = 1 << 28, 1 << 40, 7
    m = dcs()
    announce("config 3b with replacement full size")
    out = m.sample_replacement(n, N, seed)
    m.synchronize()
    assert _strictly_increasing(out, 1, N, strict=False)
    _check_windows(lambda s, c: ref.replacement_window(n, N, seed, s, c), out,
                   _windows(n, 16, 1 << 15, 4))
    # repeated pairs ~ Poisson(n(n-1)/(2N)) = 2^15
    d = out[1:] - out[:-1]
    reps = int((d == 0).sum())
    lam = n * (n - 1) / (2 * N)
    assert abs(reps - lam) < 6 * math.sqrt(lam)
