// dcs_device.hpp -- device primitives of the divide-and-conquer sampler
// (gfx950, HIP).  Everything here is part of the sample's definition: the
// same operations, in the same order and precision, give the same bits on
// every launch geometry.  Compile with -ffp-contract=off (no fused
// multiply-add is formed from the separate multiplies and adds written here).
//
// Contents:
//   * Philox-4x32-10 (Salmon et al., SC'11): the hash h of a subproblem's
//     identity that drives every random decision (paper Sec. 3.2).
//   * exact uniform conversions and the multiply-shift range map;
//   * logarithms by the atanh series (fixed polynomial, fixed order);
//   * ln(a!) - ln(b!) without cancellation;
//   * the hypergeometric split deviate (paper Sec. 3; Stadlober's
//     ratio-of-uniforms method) and the binomial one (Sec. 4.6).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lnfact_dev.inc"

namespace dcs {

// ---------------------------------------------------------------------------
// Stream purposes: the third component of the identity (j, k, t) hashed in
// Algorithm P (Sec. 3.2) -- which decision of a node a stream feeds.
// ---------------------------------------------------------------------------
enum Purpose : uint32_t {
  kSplit = 1,    // hypergeometric split of a without-replacement node
  kLeaf = 2,     // sparse leaf: uniform offsets (Algorithm H)
  kBern = 3,     // dense leaf: geometric skips (Algorithm B)
  kRepair = 4,   // dense leaf: hits removed by the repair step
  kBChunk = 5,   // Bernoulli sampling: geometric skips of one chunk
  kWrSplit = 6,  // binomial split of a with-replacement node
  kWrLeaf = 7,   // with-replacement leaf: uniform offsets
  kSegSplit = 8, // uneven universe: split of a subtree of segments
  kSegSeed = 9,  // uneven universe: seed of one segment's own tree
  kWChunk = 10,  // whole-range Algorithm B: skips of one chunk
  kWRepair = 11, // whole-range Algorithm B: hits removed by the repair
};

constexpr uint64_t kLeafMaxRange = 1ull << 32;

// ---------------------------------------------------------------------------
// Philox-4x32-10
// ---------------------------------------------------------------------------
struct Stream {
  uint32_t k0, k1;  // key = seed
  uint32_t c1;      // purpose << 24 | attempt
  uint32_t c2, c3;  // node id (low, high)
};

__device__ __forceinline__ Stream make_stream(uint64_t seed, uint64_t node, uint32_t purpose,
                                              uint32_t attempt) {
  Stream s;
  s.k0 = static_cast<uint32_t>(seed);
  s.k1 = static_cast<uint32_t>(seed >> 32);
  s.c1 = (purpose << 24) | (attempt & 0xFFFFFFu);
  s.c2 = static_cast<uint32_t>(node);
  s.c3 = static_cast<uint32_t>(node >> 32);
  return s;
}

// One 128-bit block: counter (block, c1, c2, c3), key (k0, k1), ten rounds.
__device__ __forceinline__ uint4 philox_block(const Stream& s, uint32_t block) {
  uint32_t x0 = block, x1 = s.c1, x2 = s.c2, x3 = s.c3;
  uint32_t k0 = s.k0, k1 = s.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 multiply-add each (v_mad_u64_u32) gives both halves
    const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * x0;
    const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * x2;
    // three-input XOR in one instruction (truth table 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pb >> 32), x1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pa >> 32), x3, k1, 0x96);
    x1 = static_cast<uint32_t>(pb);
    x3 = static_cast<uint32_t>(pa);
    x0 = n0;
    x2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(x0, x1, x2, x3);
}

__device__ __forceinline__ uint32_t pick(const uint4& v, unsigned j) {
  return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}

// Sequential reader of 64-bit draws: draw t = words 2(t&1) | 2(t&1)+1 << 32
// of block t/2.
struct Draws64 {
  Stream s;
  uint64_t t;
  uint32_t gbits = 6;  // wave mode: groups of 2^gbits lanes share a deviate
  __device__ __forceinline__ uint64_t next() {
    const uint4 b = philox_block(s, static_cast<uint32_t>(t >> 1));
    const uint64_t v = (t & 1) ? (static_cast<uint64_t>(b.z) | (static_cast<uint64_t>(b.w) << 32))
                               : (static_cast<uint64_t>(b.x) | (static_cast<uint64_t>(b.y) << 32));
    ++t;
    return v;
  }
};

// ---------------------------------------------------------------------------
// Uniform conversions
// ---------------------------------------------------------------------------
// (0,1]: ((x >> 11) + 1) 2^-53 and [0,1): (x >> 11) 2^-53 -- both exact.
__device__ __forceinline__ double unit_open0(uint64_t x) {
  return static_cast<double>((x >> 11) + 1) * 0x1p-53;
}
__device__ __forceinline__ double unit_closed0(uint64_t x) {
  return static_cast<double>(x >> 11) * 0x1p-53;
}

// Geometric uniform in [2^-32, 1]: the integer w+1 rounded to nearest float,
// times 2^-32.
__device__ __forceinline__ float geom_unit(uint32_t w) {
  const float x = (w == 0xFFFFFFFFu) ? 4294967296.0f : static_cast<float>(w + 1u);
  return x * 0x1p-32f;
}

// Range map for s in [1, 2^32]: value (w*s) >> 32, void when the low half of
// w*s is below 2^32 mod s (that threshold is passed in, precomputed per
// range).  Returns false for a void draw.
__device__ __forceinline__ bool range_map(uint32_t w, uint64_t s, uint32_t threshold,
                                          uint32_t* v) {
  const uint64_t m = static_cast<uint64_t>(w) * s;
  *v = static_cast<uint32_t>(m >> 32);
  return static_cast<uint32_t>(m) >= threshold;
}

__host__ __device__ __forceinline__ uint32_t range_threshold(uint64_t s) {
  return static_cast<uint32_t>((1ull << 32) % s);
}

// ---------------------------------------------------------------------------
// Logarithms (atanh series after reduction to [sqrt(1/2), sqrt(2))).
// ---------------------------------------------------------------------------
// ln 2 = kLn2Hi + kLn2Lo with kLn2Hi holding 32 significant bits.
constexpr double kLn2Hi = 0x1.62e42feep-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;
constexpr float kLn2HiF = 0x1.62e4p-1f;      // 16 significant bits
constexpr float kLn2LoF = 0x1.7f7d1cp-20f;
constexpr float kSqrt2F = 0x1.6a09e6p+0f;

// sum_{j=0}^{10} z^j / (2j+3), Horner from the innermost coefficient 1/23.
__device__ __forceinline__ double series64(double z) {
  double p = 1.0 / 23.0;
  p = 1.0 / 21.0 + z * p;
  p = 1.0 / 19.0 + z * p;
  p = 1.0 / 17.0 + z * p;
  p = 1.0 / 15.0 + z * p;
  p = 1.0 / 13.0 + z * p;
  p = 1.0 / 11.0 + z * p;
  p = 1.0 / 9.0 + z * p;
  p = 1.0 / 7.0 + z * p;
  p = 1.0 / 5.0 + z * p;
  return 1.0 / 3.0 + z * p;
}

// 2 atanh(s) for s = f/(2+f).
__device__ __forceinline__ double atanh2_64(double f) {
  const double s = f / (2.0 + f);
  const double z = s * s;
  const double t = s + s;
  return t + t * (z * series64(z));
}

__device__ __forceinline__ double log64(double x) {
  const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(x));
  int e = static_cast<int>((bits >> 52) & 0x7FF) - 1023;
  double m = __longlong_as_double(
      static_cast<long long>((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
  if (m >= kSqrt2) {
    m = m * 0.5;
    e += 1;
  }
  const double r = atanh2_64(m - 1.0);
  const double de = static_cast<double>(e);
  return de * kLn2Hi + (de * kLn2Lo + r);
}

__device__ __forceinline__ double log1p64(double x) {
  if (x > -0.25 && x < 0.25) return atanh2_64(x);
  return log64(1.0 + x);
}

__device__ __forceinline__ float series32(float z) {
  float p = 1.0f / 11.0f;
  p = 1.0f / 9.0f + z * p;
  p = 1.0f / 7.0f + z * p;
  p = 1.0f / 5.0f + z * p;
  return 1.0f / 3.0f + z * p;
}

// f / d for |f| < 1/2 and d in [3/2, 5/2] (the logarithm's reduced
// argument): no operand scaling or special case can arise, so a hardware
// reciprocal refined by one Newton step, the product, and one correction
// from the exact (fused) residual give the correctly rounded quotient -- for
// every f the reduction can produce, which a test checks against the
// correctly rounded division.
__device__ __forceinline__ float div_reduced(float f, float d) {
  float y = __builtin_amdgcn_rcpf(d);
  y = __builtin_fmaf(__builtin_fmaf(-d, y, 1.0f), y, y);
  const float q = f * y;
  return __builtin_fmaf(__builtin_fmaf(-q, d, f), y, q);
}

__device__ __forceinline__ float log32(float x) {
  const uint32_t bits = __float_as_uint(x);
  int e = static_cast<int>((bits >> 23) & 0xFF) - 127;
  float m = __uint_as_float((bits & 0x007FFFFFu) | 0x3F800000u);
  if (m >= kSqrt2F) {
    m = m * 0.5f;
    e += 1;
  }
  const float f = m - 1.0f;
  const float s = div_reduced(f, 2.0f + f);
  const float z = s * s;
  const float t = s + s;
  const float r = t + t * (z * series32(z));
  const float fe = static_cast<float>(e);
  return fe * kLn2HiF + (fe * kLn2LoF + r);
}

// Geometric skip floor(ln(U) * c) for U from one 32-bit word.
__device__ __forceinline__ int geom_skip32(uint32_t w, float c) {
  return static_cast<int>(floorf(log32(geom_unit(w)) * c));
}

// ---------------------------------------------------------------------------
// ln(a!) - ln(b!)
// ---------------------------------------------------------------------------
constexpr double kHalfLn2Pi = 0x1.d67f1c864beb5p-1;
constexpr uint64_t kStirlingDiffMin = 64;

__device__ __forceinline__ double lnfact_table(uint64_t k) {
  return __longlong_as_double(static_cast<long long>(dcs_lnfact_bits[k]));
}

// 1/(12 z) - 1/(360 z^3) + 1/(1260 z^5)
__device__ __forceinline__ double stirling_tail(double z) {
  const double r = 1.0 / z;
  const double r2 = r * r;
  return r * (1.0 / 12.0 - r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0)));
}

__device__ __forceinline__ double lnfact(uint64_t x) {
  if (x < DCS_LNFACT_ENTRIES) return lnfact_table(x);
  const double z = static_cast<double>(x) + 1.0;
  return (z - 0.5) * log64(z) - z + kHalfLn2Pi + stirling_tail(z);
}

__device__ __forceinline__ double lnfact_diff(uint64_t a, uint64_t b) {
  if (a == b) return 0.0;
  if (a >= kStirlingDiffMin && b >= kStirlingDiffMin) {
    const double za = static_cast<double>(a) + 1.0;
    const double zb = static_cast<double>(b) + 1.0;
    const double d = static_cast<double>(static_cast<int64_t>(a) - static_cast<int64_t>(b));
    const double t1 = (zb - 0.5) * log1p64(d / zb);
    const double t2 = d * (log64(za) - 1.0);
    const double t3 = stirling_tail(za) - stirling_tail(zb);
    return (t1 + t2) + t3;
  }
  return lnfact(a) - lnfact(b);
}

// ---------------------------------------------------------------------------
// Exact floor(x*y/z) for x, y, z < 2^53 and a quotient below 2^53 (the
// splits' modes): the FP64 quotient is within 2 of it, and 128-bit products
// correct it (a 128-bit integer division would run bit by bit).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t floor_muldiv(uint64_t x, uint64_t y, uint64_t z) {
  const unsigned __int128 p = static_cast<unsigned __int128>(x) * y;
  const double e = (static_cast<double>(x) * static_cast<double>(y)) / static_cast<double>(z);
  uint64_t q = e < 0x1p63 ? static_cast<uint64_t>(e) : (1ull << 63);
  unsigned __int128 qz = static_cast<unsigned __int128>(q) * z;
  while (qz > p) {
    --q;
    qz -= z;
  }
  while (p - qz >= z) {
    ++q;
    qz += z;
  }
  return q;
}

// ---------------------------------------------------------------------------
// Ratio-of-uniforms deviates (Stadlober 1990).
// ---------------------------------------------------------------------------
constexpr double kD1 = 0x1.b72cd3f331398p+0;  // 2 sqrt(2/e)
constexpr double kD2 = 0x1.cc3ebd3bc711ap-1;  // 3 - 2 sqrt(3/e)
constexpr uint64_t kInversionMax = 16;

// 2 ln U, computed before T so that its dependent chain overlaps T's (the
// wave waits for its slowest lane, and some lane of a wave usually needs it).
__device__ __forceinline__ double rou_log2u(double u) {
  double l = 2.0 * log64(u);
  asm volatile("" : "+v"(l));  // keep it here, not sunk into the test below
  return l;
}

// Accept/reject for 2 ln U <= T with the two squeezes; lu2 = rou_log2u(u).
__device__ __forceinline__ bool rou_accept(double u, double T, double lu2, bool* reject) {
  *reject = false;
  if (u * (4.0 - u) - 3.0 <= T) return true;
  if (u * (u - T) >= 1.0) { *reject = true; return false; }
  return lu2 <= T;
}

// Broadcast of lane j's value within each aligned quad of lanes (DPP
// quad_perm), for a double.
template <int j>
__device__ __forceinline__ double quad_lane(double x) {
  constexpr int ctrl = j | (j << 2) | (j << 4) | (j << 6);
  const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
  const uint32_t lo = static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(b), ctrl, 0xf, 0xf, false));
  const uint32_t hi = static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), ctrl, 0xf, 0xf, false));
  return __longlong_as_double(static_cast<long long>(static_cast<uint64_t>(lo) |
                                                     (static_cast<uint64_t>(hi) << 32)));
}

// The ratio-of-uniforms loop: attempt a takes draws 2a (U) and 2a+1 (V),
// i.e. Philox block a, and the deviate is the first accepted attempt.
// kWave: the lanes of a wave form aligned groups of G = 2^d.gbits lanes
// (the whole wave when gbits = 6), each group sampling one deviate, and the
// group takes its lowest accepted attempt (the same deviate, found in one
// round instead of one attempt after another).  With G >= 4 each aligned
// quad of lanes shares one attempt (quad q of a group: attempt G/4 * j + q
// in round j) and its lanes compute the attempt's ln-factorial terms side by
// side (attempt(u, v, sub, true, &k), sub = lane mod 4); with G = 2 each
// lane tries one attempt (attempt 2j + r in round j).
template <bool kWave, class Attempt>
__device__ __forceinline__ uint64_t rou_first_accepted(Draws64& d, Attempt attempt) {
  if constexpr (kWave) {
    uint32_t lane = threadIdx.x & 63u;
    asm volatile("" : "+v"(lane));
    const uint32_t size = 1u << d.gbits;
    const uint32_t r = lane & (size - 1u);
    const uint32_t base = lane - r;
    const unsigned long long gmask = d.gbits >= 6 ? ~0ull : (1ull << size) - 1ull;
    const bool quad = size >= 4;
    const uint32_t per_round = quad ? size >> 2 : size;
    const uint32_t slot = quad ? r >> 2 : r;
    for (uint32_t round = 0;; ++round) {
      const uint4 b = philox_block(d.s, round * per_round + slot);
      const double u = unit_open0(static_cast<uint64_t>(b.x) | (static_cast<uint64_t>(b.y) << 32));
      const double v = unit_closed0(static_cast<uint64_t>(b.z) | (static_cast<uint64_t>(b.w) << 32));
      uint64_t k = 0;
      const bool ok = attempt(u, v, static_cast<int>(lane & 3u), quad, &k);
      const unsigned long long m = (__ballot(ok) >> base) & gmask;
      if (m != 0) {
        const uint32_t f = static_cast<uint32_t>(__ffsll(static_cast<long long>(m)) - 1);
        uint32_t lo, hi;
        if (d.gbits >= 6) {
          lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(k), f);
          hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(k >> 32), f);
        } else {
          lo = static_cast<uint32_t>(__shfl(static_cast<int>(k), static_cast<int>(base + f)));
          hi = static_cast<uint32_t>(__shfl(static_cast<int>(k >> 32), static_cast<int>(base + f)));
        }
        return static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32);
      }
    }
  } else {
    for (;;) {
      const double u = unit_open0(d.next());
      const double v = unit_closed0(d.next());
      uint64_t k = 0;
      if (attempt(u, v, 0, false, &k)) return k;
    }
  }
}

// Hypergeometric core for 1 <= n, M <= N/2.
template <bool kWave>
__device__ __forceinline__ uint64_t hyp_core(uint64_t n, uint64_t M, uint64_t N, Draws64& d) {
  const uint64_t q = n < M ? n : M;
  const uint64_t big = n < M ? M : n;
  if (q <= kInversionMax) {
    double p0 = 1.0;
    for (uint64_t i = 0; i < q; ++i)
      p0 = p0 * (static_cast<double>(N - big - i) / static_cast<double>(N - i));
    for (;;) {
      double u = unit_open0(d.next());
      double p = p0;
      for (uint64_t k = 0;; ++k) {
        if (u <= p) return k;
        u = u - p;
        if (k == q) break;
        const double r = (static_cast<double>(M - k) / static_cast<double>(k + 1)) *
                         (static_cast<double>(n - k) / static_cast<double>(N - M - n + k + 1));
        p = p * r;
      }
    }
  }
  const double pm = static_cast<double>(M) / static_cast<double>(N);
  const double mu = static_cast<double>(n) * pm;
  const double var = (mu * (1.0 - pm)) * (static_cast<double>(N - n) / static_cast<double>(N - 1));
  const double a = mu + 0.5;
  const double w = __builtin_sqrt(var + 0.5);
  const double s = kD1 * w + kD2;
  const uint64_t mode = floor_muldiv(n + 1, M + 1, N + 2);
  const double kcap = floor(a + 16.0 * w);
  uint64_t kmax = q + 1;
  if (kcap < static_cast<double>(kmax)) kmax = static_cast<uint64_t>(kcap);
  const double kmax_d = static_cast<double>(kmax);
  const uint64_t rest = N - M - n;
  return rou_first_accepted<kWave>(d, [&](double u, double v, int sub, bool quad,
                                          uint64_t* out) {
    const double x = a + (s * (v - 0.5)) / u;
    if (x < 0.0 || x >= kmax_d) return false;  // the same in every lane of a quad
    const uint64_t k = static_cast<uint64_t>(floor(x));
    const double lu2 = rou_log2u(u);
    double T;
    if (quad) {
      // term `sub` in this lane, then the sum in the sequential order
      uint64_t ta, tb;
      if (sub == 0) {
        ta = mode;
        tb = k;
      } else if (sub == 1) {
        ta = M - mode;
        tb = M - k;
      } else if (sub == 2) {
        ta = n - mode;
        tb = n - k;
      } else {
        ta = rest + mode;
        tb = rest + k;
      }
      const double t = lnfact_diff(ta, tb);
      T = ((quad_lane<0>(t) + quad_lane<1>(t)) + quad_lane<2>(t)) + quad_lane<3>(t);
    } else {
      T = lnfact_diff(mode, k);
      T = T + lnfact_diff(M - mode, M - k);
      T = T + lnfact_diff(n - mode, n - k);
      T = T + lnfact_diff(rest + mode, rest + k);
    }
    bool rej;
    *out = k;
    return rou_accept(u, T, lu2, &rej);
  });
}

// Hyp(n, M, N): successes among n draws without replacement from N items, M
// of them successes; stream (seed, node, purpose, 0), purpose SPLIT for the
// recursion tree.  kWave: called by every lane of the wave, each aligned
// group of 2^gbits lanes with the same arguments.
template <bool kWave = false>
__device__ __forceinline__ uint64_t hypergeometric(uint64_t n, uint64_t M, uint64_t N, uint64_t seed,
                                   uint64_t node, uint32_t purpose = kSplit,
                                   uint32_t gbits = 6) {
  if (n == 0 || M == 0) return 0;
  if (M == N) return n;
  if (n == N) return M;
  Draws64 d{make_stream(seed, node, purpose, 0), 0, gbits};
  const bool flip_n = n > N - n;
  const uint64_t n1 = flip_n ? N - n : n;
  const bool flip_m = M > N - M;
  const uint64_t M1 = flip_m ? N - M : M;
  uint64_t k = hyp_core<kWave>(n1, M1, N, d);
  if (flip_m) k = n1 - k;
  if (flip_n) k = M - k;
  return k;
}

// Binomial core for 1 <= l <= Nv - l.
template <bool kWave>
__device__ __forceinline__ uint64_t binom_core(uint64_t n, uint64_t l, uint64_t Nv, Draws64& d) {
  const uint64_t r = Nv - l;
  if (n <= kInversionMax) {
    const double qv = static_cast<double>(r) / static_cast<double>(Nv);
    double p0 = 1.0;
    for (uint64_t i = 0; i < n; ++i) p0 = p0 * qv;
    const double odds = static_cast<double>(l) / static_cast<double>(r);
    for (;;) {
      double u = unit_open0(d.next());
      double p = p0;
      for (uint64_t k = 0;; ++k) {
        if (u <= p) return k;
        u = u - p;
        if (k == n) break;
        p = p * ((static_cast<double>(n - k) / static_cast<double>(k + 1)) * odds);
      }
    }
  }
  const double pp = static_cast<double>(l) / static_cast<double>(Nv);
  const double mu = static_cast<double>(n) * pp;
  const double var = mu * (1.0 - pp);
  const double a = mu + 0.5;
  const double w = __builtin_sqrt(var + 0.5);
  const double s = kD1 * w + kD2;
  const uint64_t mode = floor_muldiv(n + 1, l, Nv);
  const double kcap = floor(a + 16.0 * w);
  uint64_t kmax = n + 1;
  if (kcap < static_cast<double>(kmax)) kmax = static_cast<uint64_t>(kcap);
  const double kmax_d = static_cast<double>(kmax);
  const double lodds = log1p64(
      static_cast<double>(static_cast<int64_t>(2 * l) - static_cast<int64_t>(Nv)) /
      static_cast<double>(r));
  return rou_first_accepted<kWave>(d, [&](double u, double v, int sub, bool quad,
                                          uint64_t* out) {
    const double x = a + (s * (v - 0.5)) / u;
    if (x < 0.0 || x >= kmax_d) return false;  // the same in every lane of a quad
    const uint64_t k = static_cast<uint64_t>(floor(x));
    const double lu2 = rou_log2u(u);
    double T = static_cast<double>(static_cast<int64_t>(k) - static_cast<int64_t>(mode)) * lodds;
    if (quad) {
      // lanes 0 and 1 of the quad: one ln-factorial term each
      const double t = sub == 0 ? lnfact_diff(mode, k) : sub == 1 ? lnfact_diff(n - mode, n - k)
                                                                  : 0.0;
      T = (T + quad_lane<0>(t)) + quad_lane<1>(t);
    } else {
      T = T + lnfact_diff(mode, k);
      T = T + lnfact_diff(n - mode, n - k);
    }
    bool rej;
    *out = k;
    return rou_accept(u, T, lu2, &rej);
  });
}

// Bin(n, l/Nv) from stream (seed, node, WRSPLIT, 0).  kWave: called by
// every lane of the wave, each aligned group of 2^gbits lanes with the same
// arguments.
template <bool kWave = false>
__device__ __forceinline__ uint64_t binomial(uint64_t n, uint64_t l, uint64_t Nv, uint64_t seed,
                                             uint64_t node, uint32_t gbits = 6) {
  if (n == 0 || l == 0) return 0;
  if (l == Nv) return n;
  Draws64 d{make_stream(seed, node, kWrSplit, 0), 0, gbits};
  if (l > Nv - l) return n - binom_core<kWave>(n, Nv - l, Nv, d);
  return binom_core<kWave>(n, l, Nv, d);
}

__host__ __device__ __forceinline__ uint64_t isqrt64(uint64_t x) {
  // Integer square root by bitwise restoring method (exact).
  uint64_t r = 0;
  uint64_t bit = 1ull << 62;
  while (bit > x) bit >>= 2;
  while (bit != 0) {
    if (x >= r + bit) {
      x -= r + bit;
      r = (r >> 1) + bit;
    } else {
      r >>= 1;
    }
    bit >>= 2;
  }
  return r;
}

}  // namespace dcs
