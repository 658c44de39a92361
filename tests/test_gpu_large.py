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
    """The whole p = 0.01 sample of 1..2^36 and its count against the
    oracle, which recomputes it in blocks of chunks on several host threads
    (each block is independent: Sec. 4.7's subranges)."""
    from concurrent.futures import ThreadPoolExecutor
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
    per = 4096  # chunks per block: ~1.07e7 hits
    blocks = [(j, min(n_chunks, j + per)) for j in range(0, n_chunks, per)]
    cap = int(per * C * p + 12 * math.sqrt(per * C * p) + 64)
    announce(f"config 3a: oracle over all {n_chunks} chunks in {len(blocks)} blocks")
    pos = 0
    with ThreadPoolExecutor(max_workers=8) as ex:
        for (j0, j1), want in zip(blocks, ex.map(
                lambda b: ref.bernoulli_chunks(p, N, seed, b[0], b[1], capacity=cap), blocks)):
            assert want.size < cap
            got = to_np_u64(out[pos:pos + want.size])
            assert np.array_equal(got, want), f"chunks {j0}..{j1 - 1}: {first_mismatch(got, want)}"
            pos += want.size
    assert pos == c, f"oracle count {pos} != GPU count {c}"


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
