"""Bit-exact parity of the HIP sampler with the oracle (GPU), through the C ABI.

Full outputs are compared element by element at sizes the oracle finishes in
seconds (several leaves, ragged tails, every leaf kind); the 8 GiB
configuration is compared on windows the oracle computes on its own, plus
properties that hold at any size.
"""
import math

import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu

# (n, N, seed, n0, dense_ratio)
WOR_CASES = [
    (1 << 20, 1 << 32, 1, 4096, 16),          # configuration 1 (n = 2^20 of 2^32)
    (0, 10, 1, 4096, 16),                     # empty sample
    (1, 1, 3, 4096, 16),
    (10, 10, 3, 4, 16),                       # n = N, tiny leaves
    (5000, 5000, 2, 4096, 16),                # n = N, dense leaves with rho = 1
    (4095, 2**32, 5, 4096, 16),               # one sparse leaf, full 32-bit range
    (4095, 2**32 + 1, 5, 4096, 16),           # one split forced by the 2^32 range rule
    (300, 5000, 9, 4096, 2),                  # one sparse leaf with many duplicates
    (200, 2**31 + 1, 9, 4096, 2),             # half of all words void
    (1 << 16, (1 << 16) + 3, 4, 4096, 16),    # nearly full: dense leaves
    (1 << 20, 1 << 21, 7, 4096, 16),          # density 0.5 (configuration 2b, scaled)
    (123457, 10**9 + 7, 11, 4096, 16),        # ragged sizes everywhere
    (100000, 2**40 + 3, 12, 512, 16),         # range-forced depth, small n0
    (77777, 300000, 13, 64, 16),              # dense leaves, small n0 (many leaves)
    (50000, 2**44, 14, 4096, 16),             # very sparse
    (200, 2**52, 15, 4096, 16),               # 2^52: integers still exact in doubles
    (3, 2**52, 16, 2, 16),                    # n0 = 2, depth 50
    (1 << 22, 2**60, 25, 4096, 16),           # above 2^53: rounded conversions in the splits
    (300_000, 2**62, 26, 4096, 16),           # largest universe
    (3, 2**62 - 1, 27, 2, 16),                # n0 = 2, depth 60
    (20000, 640000, 17, 4096, 16),            # density 1/32: sparse, duplicates common
    # ~17 repeated draws per leaf over ~1500 leaves: repeats inside the last
    # sorting window of a leaf, power-of-two and other leaf ranges
    (1 << 22, 1 << 28, 21, 4096, 16),
    (1 << 22, 3 * 2**26 + 5, 22, 4096, 16),
    # dense ratio 64: dense leaves over 2^16 (one wave each) and 2^17
    # (work-group path) in one sample
    (1 << 17, 1 << 22, 23, 4096, 64),
    (3000, 3000 * 64, 24, 4096, 64),          # one dense leaf over more than 2^16
    # half of all words void: fewer than n_v values among the first 4096
    # words, so the leaf takes the general rounds from word 0
    (3000, 2**31 + 1, 25, 4096, 16),
    (1 << 18, 3 * 2**30 + 7, 26, 4096, 16),   # a third void at the root's leaves
    # density 0.49 with dense ratio 2: ~490 repeats in the first round (a full
    # re-sort round), then rounds of at most 256 new values merged in
    (2000, 4100, 27, 4096, 2),
    (3900, 7900, 28, 4096, 2),
]


@pytest.mark.parametrize("n,N,seed,n0,dr", WOR_CASES)
def test_without_replacement_matches_oracle(ref, n, N, seed, n0, dr):
    import torch
    m = dcs()
    announce(f"wor n={n} N={N} seed={seed} n0={n0} dr={dr}")
    out = m.sample(n, N, seed, n0=n0, dense_ratio=dr)
    m.synchronize()
    got = to_np_u64(out)
    want = ref.sample(n, N, seed, n0=n0, dense_ratio=dr)
    assert np.array_equal(got, want), first_mismatch(got, want)


def dense_hits(ref, seed, nv, Nv, attempt=0):
    """Bernoulli hits of the dense root leaf (node 1) of an (nv, Nv) sample,
    from the oracle's stream words and logarithm (seed finder for the test
    below)."""
    rho_num = nv + 3 * math.isqrt(nv) + 8
    rho = np.float32(rho_num) / np.float32(Nv)
    cg = np.float32(1.0 / ref.log64(1.0 - float(rho)))
    u = np.array([ref.u32_geom(ref.stream_word(seed, 1, 3, attempt, t))
                  for t in range(2 * rho_num)], dtype=np.float32)
    g = np.floor(ref.log32_batch(u) * cg).astype(np.int64)
    pos = np.cumsum(g + 1) - 1
    assert pos[-1] >= Nv, "draw more words"
    return int(np.count_nonzero(pos < Nv))


def test_dense_leaf_beyond_stored_chunks(ref):
    """One dense leaf whose hit count exceeds the 4352 positions a wave keeps
    in LDS: the chunk past them is recomputed from its start (the seeds with
    the most hits among the first 40, and one just below the bound)."""
    m = dcs()
    nv, Nv = 4095, 4095 * 16
    counts = [(dense_hits(ref, seed, nv, Nv), seed) for seed in range(1, 41)]
    counts.sort(reverse=True)
    found = [(nv, seed, c) for c, seed in counts[:3]]
    assert found[-1][2] > 4352, counts
    # a leaf whose hits just fit the stored chunks
    for seed in range(41, 400):
        c = dense_hits(ref, seed, nv, Nv)
        if 4352 - 8 <= c <= 4352:
            found.append((nv, seed, c))
            break
    assert found[-1][2] <= 4352, found
    for nv, seed, c in found:
        Nv = nv * 16
        announce(f"dense leaf nv={nv} Nv={Nv} seed={seed} hits={c}")
        out = m.sample(nv, Nv, seed)
        m.synchronize()
        got = to_np_u64(out)
        want = ref.sample(nv, Nv, seed)
        assert np.array_equal(got, want), first_mismatch(got, want)


def test_config1_invariants_and_repeatability():
    import torch
    m = dcs()
    n, N = 1 << 20, 1 << 32
    announce("config 1 repeat")
    a = m.sample(n, N, 1)
    b = torch.empty_like(a)
    m.sample(n, N, 1, out=b)
    m.synchronize()
    assert torch.equal(a, b)
    d = a[1:] - a[:-1]
    assert bool((d > 0).all())
    assert int(a[0]) >= 1 and int(a[-1]) <= N


WR_CASES = [
    (1 << 20, 1 << 34, 7, 4096),
    (1 << 20, 2**61 + 3, 8, 4096),   # above 2^53
    (5000, 2**62, 9, 64),            # largest universe
    (3000, 2**31 + 1, 10, 4096),     # half of all words void: values drawn beyond the first 4096 words
    (1 << 20, 3 * 2**40 + 5, 11, 4096),  # leaves over ranges just above 2^31 (up to half void)
    (7, 1, 3, 4096),                 # N = 1: all ones
    (1 << 18, 2, 5, 4096),           # constant leaves cut into pieces
    (100000, 3 * 10**6 + 1, 11, 512),
    (5, 3, 1, 2),
    (1 << 16, 1 << 10, 8, 4096),     # many repeats per value
    (3000, 2**45 + 1, 9, 4096),
    (4000, 8, 12, 4096),             # one leaf, 8 values: buckets of ~500 equal keys
    (4095, 5, 13, 4096),
    (3000, 2**31 + 1, 14, 4096),     # half of all words void: general rounds
    (1 << 18, 10**9 + 7, 15, 4096),  # ranges that are not powers of two
]


@pytest.mark.parametrize("n,N,seed,n0", WR_CASES)
def test_with_replacement_matches_oracle(ref, n, N, seed, n0):
    m = dcs()
    announce(f"wr n={n} N={N} seed={seed} n0={n0}")
    out = m.sample_replacement(n, N, seed, n0=n0)
    m.synchronize()
    got = to_np_u64(out)
    want = ref.replacement(n, N, seed, n0=n0)
    assert np.array_equal(got, want), first_mismatch(got, want)


BERN_CASES = [
    (0.01, 1 << 26, 7),      # p of configuration 3, smaller universe
    (0.3, 100003, 1),
    (2.0**-10, 1 << 24, 2),  # smallest single-precision p
    (1e-4, 1 << 28, 3),      # double-precision skips
    (0.97, 50000, 4),
    (0.0, 1000, 5),
    (1.0, 1000, 6),
    (0.5, 3, 7),
    # chunks of 8192 with ~4096 hits: about half hold more hits than the
    # 4096 increments a wave keeps, and recompute their last group
    (0.5, 1 << 22, 21),
    # double-precision skips over many chunks, handed out by all ticket
    # classes: chunks clamped at 2^32 with ~512 hits each, and 128 chunks
    # of 2^23 just below the single-precision threshold
    (2.0**-23, 1 << 40, 31),
    (2.0**-11, 1 << 30, 32),
]


@pytest.mark.parametrize("p,N,seed", BERN_CASES)
def test_bernoulli_matches_oracle(ref, p, N, seed):
    m = dcs()
    announce(f"bernoulli p={p} N={N} seed={seed}")
    out, cnt = m.sample_bernoulli(p, N, seed)
    m.synchronize()
    c = int(cnt.item())
    want = ref.bernoulli(p, N, seed)
    assert c == want.size
    got = to_np_u64(out[:c])
    assert np.array_equal(got, want), first_mismatch(got, want)


# Small n0: chunks clamp to 2^12 positions while only 2 n0 + 64 hits of a
# chunk stay in LDS, so most chunks take the second (direct-write) pass; the
# many short chunks also give long look-back chains.
BERN_N0_CASES = [
    (0.5, 1 << 22, 11, 2),     # 1024 chunks, ~2048 hits each, 68 held in LDS
    (0.02, 1 << 24, 12, 16),   # 4096 chunks, ~82 hits each, 96 held in LDS
    (0.25, 1 << 26, 13, 64),   # 16384 chunks, look-back over many chunks
    (2.0**-11, 1 << 26, 14, 2),  # double-precision skips, 16384 chunks
]


@pytest.mark.parametrize("p,N,seed,n0", BERN_N0_CASES)
def test_bernoulli_small_n0_matches_oracle(ref, p, N, seed, n0):
    m = dcs()
    announce(f"bernoulli p={p} N={N} seed={seed} n0={n0}")
    out, cnt = m.sample_bernoulli(p, N, seed, n0=n0)
    m.synchronize()
    c = int(cnt.item())
    want = ref.bernoulli(p, N, seed, n0=n0)
    assert c == want.size
    got = to_np_u64(out[:c])
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("p,N,seed", [(0.01, 1 << 24, 31), (0.5, 1 << 20, 32)])
def test_bernoulli_output_one_element_off_alignment(ref, p, N, seed):
    """Output that starts 8 bytes past a 16-byte boundary: the paired stores
    must fall back to single ones."""
    import torch
    m = dcs()
    announce(f"bernoulli unaligned p={p} N={N}")
    want = ref.bernoulli(p, N, seed)
    cap = want.size + 64
    buf = torch.zeros(cap + 1, dtype=torch.int64, device="cuda")
    out = buf[1:]
    assert out.data_ptr() % 16 == 8
    _, cnt = m.sample_bernoulli(p, N, seed, out=out, capacity=cap)
    m.synchronize()
    assert int(cnt.item()) == want.size
    assert int(buf[0].item()) == 0
    assert np.array_equal(to_np_u64(out[:want.size]), want)


def test_wor_output_one_element_off_alignment(ref):
    import torch
    m = dcs()
    n, N, seed = 300000, 10**9 + 7, 33
    announce("wor unaligned")
    buf = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    m.sample(n, N, seed, out=buf[1:])
    m.synchronize()
    assert int(buf[0].item()) == 0
    assert np.array_equal(to_np_u64(buf[1:]), ref.sample(n, N, seed))


def test_bernoulli_capacity_overflow_keeps_prefix(ref):
    import torch
    m = dcs()
    p, N, seed = 0.01, 1 << 24, 9
    announce("bernoulli overflow")
    want = ref.bernoulli(p, N, seed)
    cap = want.size // 2
    out = torch.zeros(cap, dtype=torch.int64, device="cuda")
    _, cnt = m.sample_bernoulli(p, N, seed, out=out, capacity=cap)
    m.synchronize()
    assert int(cnt.item()) == want.size
    assert np.array_equal(to_np_u64(out), want[:cap])


def test_invalid_arguments_rejected():
    import torch
    m = dcs()
    out = torch.empty(16, dtype=torch.int64, device="cuda")
    for args in [(11, 10, 1), (1, 2**62 + 1, 1)]:
        with pytest.raises(m.DcsError):
            m.sample(*args, out=out)
    with pytest.raises(m.DcsError):
        m.sample(4, 10, 1, out=out, n0=1)
    with pytest.raises(m.DcsError):
        m.sample_bernoulli(1.5, 10, 1, out=out)
    with pytest.raises(m.DcsError):
        m.sample_replacement(3, 0, 1, out=out)
