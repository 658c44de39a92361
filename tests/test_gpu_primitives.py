"""Bit-exact parity of the device primitives with the oracle (GPU)."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs

pytestmark = pytest.mark.gpu


def _run(m, op, x, x2, ytype, n, p=(0, 0, 0, 0)):
    import torch
    xd = torch.from_numpy(x).cuda()
    x2d = torch.from_numpy(x2).cuda() if x2 is not None else None
    yd = torch.empty(n, dtype=ytype, device="cuda")
    m.debug_primitive(op, xd, x2d, yd, *p)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def test_philox_blocks(ref):
    import torch
    m = dcs()
    announce("philox blocks")
    rng = np.random.default_rng(1)
    for key in [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (0xA4093822, 0x299F31D0), (7, 0)]:
        ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
        ctr[0] = 0
        ctr[1] = 0xFFFFFFFF
        y = _run(m, 8, ctr.reshape(-1).view(np.int32), None, torch.int32, 4 * 4096,
                 (key[0], key[1], 0, 0)).view(np.uint32).reshape(-1, 4)
        for i in range(0, 4096, 37):
            assert tuple(int(v) for v in y[i]) == ref.philox(tuple(int(c) for c in ctr[i]), key)


def test_log64_log1p64_bitexact(ref):
    import torch
    m = dcs()
    announce("log64/log1p64")
    rng = np.random.default_rng(2)
    x = np.concatenate([np.exp(rng.uniform(-700, 700, 500000)), rng.uniform(0.5, 2, 500000),
                        np.arange(1, 5000, dtype=np.float64), [2.0**52, 2.0**52 + 1, 1.0]])
    y = _run(m, 0, x, None, torch.float64, x.size)
    assert np.array_equal(y.view(np.uint64), ref.log64_batch(x).view(np.uint64))
    x = np.concatenate([rng.uniform(-0.999, 4, 500000), rng.uniform(-1e-9, 1e-9, 100000),
                        [0.25, -0.25, 0.2499999999, 1e-300]])
    y = _run(m, 1, x, None, torch.float64, x.size)
    assert np.array_equal(y.view(np.uint64), ref.log1p64_batch(x).view(np.uint64))


def test_log32_bitexact(ref):
    import torch
    m = dcs()
    announce("log32")
    rng = np.random.default_rng(3)
    bits = np.concatenate([
        rng.integers(int(np.float32(2.0**-32).view(np.uint32)), int(np.float32(1.0).view(np.uint32)) + 1,
                     size=4_000_000, dtype=np.int64),
        np.arange(int(np.float32(0.5).view(np.uint32)), int(np.float32(1.0).view(np.uint32)) + 1,
                  dtype=np.int64)]).astype(np.uint32)
    x = bits.view(np.float32)
    y = _run(m, 2, x, None, torch.float32, x.size)
    assert np.array_equal(y.view(np.uint32), ref.log32_batch(x).view(np.uint32))


def test_sqrt_and_division_correctly_rounded():
    """The hypergeometric setup relies on correctly rounded sqrt and
    division; the device must agree bit for bit with the host's IEEE ops."""
    import torch
    m = dcs()
    announce("sqrt/div")
    rng = np.random.default_rng(4)
    x = np.concatenate([np.exp(rng.uniform(-30, 100, 1_000_000)), rng.uniform(0, 1e6, 200000),
                        (np.arange(1, 200000, dtype=np.float64) ** 2),
                        (np.arange(1, 200000, dtype=np.float64) ** 2) + 0.5])
    y = _run(m, 3, x, None, torch.float64, x.size)
    assert np.array_equal(y.view(np.uint64), np.sqrt(x).view(np.uint64))
    a = rng.uniform(-1e6, 1e6, 1_000_000)
    b = np.exp(rng.uniform(-20, 20, 1_000_000))
    y = _run(m, 4, a, b, torch.float64, a.size)
    assert np.array_equal(y.view(np.uint64), (a / b).view(np.uint64))


def test_lnfact_diff_bitexact(ref):
    import torch
    m = dcs()
    announce("lnfact_diff")
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.integers(0, 2000, 200000), rng.integers(0, 2**52, 200000),
                        rng.integers(2**52, 2**62, 100000), rng.integers(60, 70, 1000)]).astype(np.uint64)
    d = rng.integers(-2**20, 2**20, a.size)
    b = np.clip(a.astype(np.int64) + d, 0, 2**62).astype(np.uint64)
    b[:1000] = rng.integers(0, 1100, 1000).astype(np.uint64)
    y = _run(m, 5, a, b, torch.float64, a.size)
    assert np.array_equal(y.view(np.uint64), ref.lnfact_diff_batch(a, b).view(np.uint64))


HYP = [(5, 7, 20), (16, 16, 40), (17, 40, 90), (300, 200, 1000), (700, 400, 1000),
       (900, 700, 1000), (1 << 30, 1 << 47, 1 << 48), (4095, 2**31, 2**32),
       (3_000_000, 2**41 - 1, 2**42 - 1), (1 << 20, 1 << 31, 1 << 32), (2, 2**51, 2**52),
       (1000, 2**59, 2**60), (1 << 24, 2**59 + 12345, 2**60 + 99), (12, 2**61, 2**62),
       (50_000, 3 * 2**59, 2**62 - 1)]


@pytest.mark.parametrize("n,M,N", HYP)
def test_hypergeometric_bitexact(ref, n, M, N):
    import torch
    m = dcs()
    announce(f"hyp {n} {M} {N}")
    ids = np.arange(1, 20001, dtype=np.uint64)
    y = _run(m, 6, ids, None, torch.int64, ids.size, (n, M, N, 99)).view(np.uint64)
    assert np.array_equal(y, ref.hyp_batch(n, M, N, 99, 1, ids.size))


BIN = [(5, 3, 7), (16, 5, 10), (17, 1, 2), (100, 500, 1000), (1000, 3, 7),
       (1 << 28, 1 << 39, 1 << 40), (10**7, 2**32, 2**33 + 1), (30_000, 2**60, 2**61 + 3),
       (9, 2**61, 2**62 - 1)]


@pytest.mark.parametrize("n,l,Nv", BIN)
def test_binomial_bitexact(ref, n, l, Nv):
    import torch
    m = dcs()
    announce(f"bin {n} {l} {Nv}")
    ids = np.arange(1, 20001, dtype=np.uint64)
    y = _run(m, 7, ids, None, torch.int64, ids.size, (n, l, Nv, 5)).view(np.uint64)
    assert np.array_equal(y, ref.binom_batch(n, l, Nv, 5, 1, ids.size))


def test_geometric_unit_bitexact(ref):
    import torch
    m = dcs()
    announce("geom unit")
    w = np.concatenate([np.random.default_rng(6).integers(0, 2**32, 100000, dtype=np.uint64),
                        [0, 1, 2**24 - 1, 2**24, 2**24 + 1, 2**32 - 2, 2**32 - 1]]).astype(np.uint32)
    y = _run(m, 9, w, None, torch.float32, w.size)
    want = np.array([ref.u32_geom(int(v)) for v in w], dtype=np.float32)
    assert np.array_equal(y.view(np.uint32), want.view(np.uint32))
