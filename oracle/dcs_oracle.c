/*
 * dcs_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of the divide-and-conquer
 * sampler of Sanders, Lamm, Huebschle-Schneider, Schrade and Dachsbacher,
 * "Efficient Parallel Random Sampling -- Vectorized, Cache-Efficient, and
 * Online" (ACM TOMS 44(3), 2018).  It is the checker that the HIP library is
 * compared against, bit for bit.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or constant generator with the HIP path.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 * (contraction off: every floating-point operation below is rounded on its
 * own, in the order written, exactly as the canonical definition states).
 *
 * What it computes (section numbers are the paper's):
 *   - Sec. 3.1, Fig. 1 (Algorithm R): recursive split of 1..N at floor(N/2);
 *     the left count L is a hypergeometric deviate (Sec. 3, first paragraph);
 *     recursion stops below n0 (base case).
 *   - Sec. 3.2 (Algorithm P): the random decisions at a subproblem are a hash
 *     of the subproblem's identity.  Here the hash is Philox-4x32-10 keyed by
 *     the seed, with the tree-node id (root 1, children 2i and 2i+1) and a
 *     purpose tag in the counter.
 *   - Sec. 2, Algorithm H: the sparse base case keeps the first n distinct
 *     values of a stream of uniform deviates (duplicates rejected).
 *   - Sec. 2, Algorithm B, and Sec. 4.7: the dense base case takes a
 *     Bernoulli sample by geometric skips, restarts if it is too small and
 *     removes the excess at random (the removal uses Algorithm H semantics).
 *   - Sec. 4.1: output in sorted order.
 *   - Sec. 4.6: with replacement = the same recursion with binomial splits.
 *   - Sec. 4.7: Bernoulli sampling over independent subranges.
 *   - Stadlober (1990), cited in Sec. 3.1: ratio-of-uniforms hypergeometric and
 *     binomial deviates; the log-density differences are formed as sums of
 *     ln(a!) - ln(b!) terms, never as differences of absolute log-factorials.
 *
 * Parity status: every primitive is pinned by tests against published
 * known-answer vectors, mpmath, exact pmfs and brute force; the exact bits of a
 * full sample for a given seed are NOT printed in the paper (it uses a
 * different generator), so those bits are "parity unpinned" against the
 * paper and are pinned only distributionally.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "lnfact_table.h"

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Error codes (same numeric meaning as the library's, defined here anew).   */
/* ------------------------------------------------------------------------ */
enum { REF_OK = 0, REF_EINVAL = 1, REF_ENOMEM = 2, REF_EOVERFLOW = 4 };

/* Largest universe of Bernoulli sampling: chunk positions and their counts
 * stay exact in a double, and the look-back words stay few. */
#define REF_MAX_N (1ULL << 52)
/* Largest universe of the recursion tree (without and with replacement,
 * parts, segments, G(n, m)): node ids and output values stay below 2^63;
 * integers above 2^53 enter the hypergeometric deviate's doubles rounded,
 * which only perturbs its ratio-of-uniforms test at the level of the
 * rounding of its logarithms (the mode and the exact cases stay integer). */
#define REF_MAX_TREE_N (1ULL << 62)
/* A leaf's range must fit a 32-bit draw. */
#define REF_LEAF_MAX_RANGE (1ULL << 32)

/* Stream purposes (the "t" dimension of h((j,k,t)) in Sec. 3.2). */
enum {
  P_SPLIT = 1,   /* hypergeometric split of a without-replacement node */
  P_LEAF = 2,    /* sparse leaf: uniform offsets */
  P_BERN = 3,    /* dense leaf: geometric skips */
  P_REPAIR = 4,  /* dense leaf: which Bernoulli hits to remove */
  P_BCHUNK = 5,  /* Bernoulli variant: geometric skips of one chunk */
  P_WRSPLIT = 6, /* binomial split of a with-replacement node */
  P_WRLEAF = 7,  /* with-replacement leaf: uniform offsets */
  P_SEGSPLIT = 8, /* uneven universe: split of a subtree of segments */
  P_SEGSEED = 9,  /* uneven universe: the seed of one segment's own tree */
  P_WCHUNK = 10,  /* whole-range Algorithm B: skips of one chunk */
  P_WREPAIR = 11  /* whole-range Algorithm B: which hits to remove */
};

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).                       */
/* ------------------------------------------------------------------------ */
static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)prod1;
    uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)prod0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A stream = (seed, node id, purpose, attempt).  Block b of the stream is
 * Philox(counter = (b, purpose<<24 | attempt, id_lo, id_hi), key = seed). */
typedef struct {
  uint32_t key[2];
  uint32_t ctr1, ctr2, ctr3;
} stream_t;

static stream_t make_stream(uint64_t seed, uint64_t id, uint32_t purpose,
                            uint32_t attempt) {
  stream_t s;
  s.key[0] = (uint32_t)seed;
  s.key[1] = (uint32_t)(seed >> 32);
  s.ctr1 = (purpose << 24) | (attempt & 0xFFFFFFu);
  s.ctr2 = (uint32_t)id;
  s.ctr3 = (uint32_t)(id >> 32);
  return s;
}

static void stream_block(const stream_t *s, uint64_t b, uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)b, s->ctr1, s->ctr2, s->ctr3};
  philox4x32_10(ctr, s->key, w);
}

/* 32-bit word t of the stream: word (t mod 4) of block floor(t/4). */
static uint32_t stream_word(const stream_t *s, uint64_t t) {
  uint32_t w[4];
  stream_block(s, t >> 2, w);
  return w[t & 3];
}

/* 64-bit draw t: words 2(t mod 2) (low half) and 2(t mod 2)+1 (high half) of
 * block floor(t/2). */
static uint64_t stream_draw64(const stream_t *s, uint64_t t) {
  uint32_t w[4];
  stream_block(s, t >> 1, w);
  unsigned j = (unsigned)(t & 1) * 2;
  return (uint64_t)w[j] | ((uint64_t)w[j + 1] << 32);
}

/* ------------------------------------------------------------------------ */
/* Uniform conversions.                                                      */
/* ------------------------------------------------------------------------ */
/* U in (0,1]: ((x >> 11) + 1) * 2^-53, exact. */
static double u53_open0(uint64_t x) { return (double)((x >> 11) + 1) * 0x1p-53; }
/* V in [0,1): (x >> 11) * 2^-53, exact. */
static double u53_closed0(uint64_t x) { return (double)(x >> 11) * 0x1p-53; }

/* Integer in [0, s), 1 <= s <= 2^32, by multiply-shift with exact rejection
 * (Lemire 2019): m = w*s; the draw is void when (m mod 2^32) < (2^32 mod s),
 * otherwise the value is m >> 32.  Every value has exactly floor(2^32/s)
 * accepted preimages, so accepted values are exactly uniform.  Returns -1 for
 * a void draw. */
static int64_t range_map(uint32_t w, uint64_t s) {
  uint64_t m = (uint64_t)w * s;
  uint64_t threshold = (1ULL << 32) % s;
  if ((m & 0xFFFFFFFFULL) < threshold) return -1;
  return (int64_t)(m >> 32);
}

/* U in [2^-32, 1] for geometric skips, single precision: the integer w+1
 * (1..2^32) rounded to the nearest float, scaled by 2^-32 (exact). */
static float u32_geom(uint32_t w) {
  float x = (float)((uint64_t)w + 1);
  return x * 0x1p-32f;
}

/* ------------------------------------------------------------------------ */
/* Logarithms: argument reduction x = 2^e * m, m in [sqrt(1/2), sqrt(2)),    */
/* then ln m = 2 atanh(s), s = (m-1)/(m+1), as the odd power series          */
/* 2s (1 + s^2/3 + s^4/5 + ...) truncated at a fixed term, Horner in s^2.    */
/* ln 2 is split into a head with trailing zero bits (so e*head is exact)    */
/* and a tail.  Fixed operation order, no contraction.                       */
/* ------------------------------------------------------------------------ */
static double bits_to_double(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }
static uint64_t double_to_bits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }
static float bits_to_float(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t float_to_bits(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

/* ln 2 truncated to 32 significant bits, and the rest rounded to double. */
#define REF_LN2_HI 0x1.62e42feep-1            /* 0x3fe62e42fee00000 */
#define REF_LN2_LO 0x1.a39ef35793c76p-33      /* 0x3dea39ef35793c76 */
#define REF_SQRT2 0x1.6a09e667f3bcdp+0        /* nearest double to sqrt(2) */

/* Series 1/3 + z/5 + ... + z^10/23 (11 terms). */
static double atanh_tail64(double z) {
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
  p = 1.0 / 3.0 + z * p;
  return p;
}

/* ln x for a positive normal double x. */
static double log64(double x) {
  uint64_t b = double_to_bits(x);
  int e = (int)((b >> 52) & 0x7FF) - 1023;
  double m = bits_to_double((b & 0x000FFFFFFFFFFFFFULL) | 0x3FF0000000000000ULL);
  if (m >= REF_SQRT2) {
    m = m * 0.5;
    e = e + 1;
  }
  double f = m - 1.0;
  double s = f / (2.0 + f);
  double z = s * s;
  double t = 2.0 * s;
  double r = t + t * (z * atanh_tail64(z));
  double de = (double)e;
  return de * REF_LN2_HI + (de * REF_LN2_LO + r);
}

/* ln(1+x) for x > -1. */
static double log1p64(double x) {
  if (x > -0.25 && x < 0.25) {
    double s = x / (2.0 + x);
    double z = s * s;
    double t = 2.0 * s;
    return t + t * (z * atanh_tail64(z));
  }
  return log64(1.0 + x);
}

#define REF_LN2F_HI 0x1.62e4p-1f      /* 0x3f317200: ln 2 to 16 bits */
#define REF_LN2F_LO 0x1.7f7d1cp-20f   /* 0x35bfbe8e: the rest, to float */
#define REF_SQRT2F 0x1.6a09e6p+0f     /* 0x3fb504f3 */

/* Series 1/3 + z/5 + z^2/7 + z^3/9 + z^4/11 (5 terms). */
static float atanh_tail32(float z) {
  float p = 1.0f / 11.0f;
  p = 1.0f / 9.0f + z * p;
  p = 1.0f / 7.0f + z * p;
  p = 1.0f / 5.0f + z * p;
  p = 1.0f / 3.0f + z * p;
  return p;
}

/* ln x for a positive normal float x. */
static float log32(float x) {
  uint32_t b = float_to_bits(x);
  int e = (int)((b >> 23) & 0xFF) - 127;
  float m = bits_to_float((b & 0x007FFFFFu) | 0x3F800000u);
  if (m >= REF_SQRT2F) {
    m = m * 0.5f;
    e = e + 1;
  }
  float f = m - 1.0f;
  float s = f / (2.0f + f);
  float z = s * s;
  float t = 2.0f * s;
  float r = t + t * (z * atanh_tail32(z));
  float fe = (float)e;
  return fe * REF_LN2F_HI + (fe * REF_LN2F_LO + r);
}

/* ------------------------------------------------------------------------ */
/* ln(a!) - ln(b!) without cancellation.                                     */
/* ------------------------------------------------------------------------ */
#define REF_HALF_LN_2PI 0x1.d67f1c864beb5p-1 /* nearest double to ln(2 pi)/2 */

static double lnfact_small(uint64_t k) { return bits_to_double(oracle_lnfact_bits[k]); }

/* 1/(12z) - 1/(360 z^3) + 1/(1260 z^5): the Stirling correction terms. */
static double stirling_corr(double z) {
  double r = 1.0 / z;
  double r2 = r * r;
  return r * (1.0 / 12.0 - r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0)));
}

/* ln(x!) by Stirling's series, for x >= ORACLE_LNFACT_N. */
static double lnfact_stirling(uint64_t x) {
  double z = (double)x + 1.0;
  return (z - 0.5) * log64(z) - z + REF_HALF_LN_2PI + stirling_corr(z);
}

static double lnfact_any(uint64_t x) {
  return x < ORACLE_LNFACT_N ? lnfact_small(x) : lnfact_stirling(x);
}

/* Below this argument one side is small and a plain difference loses nothing
 * (ln 63! < 202); at or above it the series truncation error of each Stirling
 * term is below 1/(1680 * 64^7) < 2e-16. */
#define REF_STIRLING_DIFF_MIN 64

/* G(a,b) = ln(a!) - ln(b!).  Both arguments >= 64: the Stirling series
 * difference
 *   (b + 1/2) log1p(d / (b+1)) + d (ln(a+1) - 1) + c(a+1) - c(b+1),  d = a-b,
 * which is what ln Gamma(a+1) - ln Gamma(b+1) reduces to after the common
 * terms cancel algebraically; otherwise the difference of absolute values. */
static double lnfact_diff(uint64_t a, uint64_t b) {
  if (a == b) return 0.0;
  if (a >= REF_STIRLING_DIFF_MIN && b >= REF_STIRLING_DIFF_MIN) {
    double za = (double)a + 1.0;
    double zb = (double)b + 1.0;
    double d = (double)((int64_t)a - (int64_t)b);
    double t1 = (zb - 0.5) * log1p64(d / zb);
    double t2 = d * (log64(za) - 1.0);
    double t3 = stirling_corr(za) - stirling_corr(zb);
    return (t1 + t2) + t3;
  }
  return lnfact_any(a) - lnfact_any(b);
}

/* ------------------------------------------------------------------------ */
/* Hypergeometric deviate: number of successes among n draws without         */
/* replacement from N items of which M are successes (Sec. 3: the count of  */
/* samples that fall into the left part 1..M).                               */
/* ------------------------------------------------------------------------ */
#define REF_D1 0x1.b72cd3f331398p+0 /* nearest double to 2 sqrt(2/e)       */
#define REF_D2 0x1.cc3ebd3bc711ap-1 /* nearest double to 3 - 2 sqrt(3/e)   */
#define REF_INVERSION_MAX 16

typedef struct {
  stream_t s;
  uint64_t t; /* next 64-bit draw */
} draws_t;

static uint64_t next_draw(draws_t *d) { return stream_draw64(&d->s, d->t++); }

/* floor(x * y / z) exactly (x*y < 2^128). */
static uint64_t muldiv_floor(uint64_t x, uint64_t y, uint64_t z) {
  unsigned __int128 p = (unsigned __int128)x * y;
  return (uint64_t)(p / z);
}

/* Mode of Hyp(n, M, N): floor((n+1)(M+1)/(N+2)). */
static uint64_t hyp_mode(uint64_t n, uint64_t M, uint64_t N) {
  return muldiv_floor(n + 1, M + 1, N + 2);
}

/* Mode of Bin(n, l/Nv): floor((n+1) l / Nv). */
static uint64_t bin_mode(uint64_t n, uint64_t l, uint64_t Nv) {
  return muldiv_floor(n + 1, l, Nv);
}

/* Ratio-of-uniforms acceptance loop shared in shape by both distributions
 * (Stadlober 1990): X = a + s (V - 1/2) / U, k = floor(X), accept iff
 * U^2 <= f(k)/f(mode), i.e. 2 ln U <= T(k), with the two squeezes
 * U(4-U)-3 <= T (sure accept) and U(U-T) >= 1 (sure reject). */
static int rou_decide(double u, double T) {
  if (u * (4.0 - u) - 3.0 <= T) return 1;
  if (u * (u - T) >= 1.0) return 0;
  return 2.0 * log64(u) <= T;
}

/* Core for 1 <= n <= N/2 and 1 <= M <= N/2. */
static uint64_t hyp_core(uint64_t n, uint64_t M, uint64_t N, draws_t *dr) {
  uint64_t q = n < M ? n : M;
  uint64_t big = n < M ? M : n;
  if (q <= REF_INVERSION_MAX) {
    /* Inversion: p(0) = prod_{i<q} (N-big-i)/(N-i); then walk the pmf upward
     * with p(k+1)/p(k) = (M-k)(n-k) / ((k+1)(N-M-n+k+1)). */
    double p0 = 1.0;
    for (uint64_t i = 0; i < q; ++i) p0 = p0 * ((double)(N - big - i) / (double)(N - i));
    for (;;) {
      double u = u53_open0(next_draw(dr));
      double p = p0;
      uint64_t k = 0;
      for (;;) {
        if (u <= p) return k;
        u = u - p;
        if (k == q) break; /* rounding exhausted the support: fresh U */
        double r = ((double)(M - k) / (double)(k + 1)) *
                   ((double)(n - k) / (double)(N - M - n + k + 1));
        p = p * r;
        k = k + 1;
      }
    }
  }
  double pm = (double)M / (double)N;
  double mu = (double)n * pm;
  double var = (mu * (1.0 - pm)) * ((double)(N - n) / (double)(N - 1));
  double a = mu + 0.5;
  double w = sqrt(var + 0.5);
  double s = REF_D1 * w + REF_D2;
  uint64_t mode = hyp_mode(n, M, N);
  double kmax_d = floor(a + 16.0 * w);
  uint64_t kmax = q + 1;
  if (kmax_d < (double)kmax) kmax = (uint64_t)kmax_d;
  uint64_t nmM = N - M - n; /* >= 0 */
  for (;;) {
    double u = u53_open0(next_draw(dr));
    double v = u53_closed0(next_draw(dr));
    double x = a + (s * (v - 0.5)) / u;
    if (x < 0.0 || x >= (double)kmax) continue;
    uint64_t k = (uint64_t)floor(x);
    double T = lnfact_diff(mode, k);
    T = T + lnfact_diff(M - mode, M - k);
    T = T + lnfact_diff(n - mode, n - k);
    T = T + lnfact_diff(nmM + mode, nmM + k);
    if (rou_decide(u, T)) return k;
  }
}

/* Hyp(n, M, N) from the (seed, id, purpose) stream. */
static uint64_t hyp_stream(uint64_t n, uint64_t M, uint64_t N, uint64_t seed, uint64_t id,
                           uint32_t purpose) {
  if (n == 0 || M == 0) return 0;
  if (M == N) return n;
  if (n == N) return M;
  draws_t dr = {make_stream(seed, id, purpose, 0), 0};
  uint64_t n1 = n, M1 = M;
  int flip_n = 0, flip_m = 0;
  /* Sec. 2: for n > N/2 take the complement of the sample. */
  if (n1 > N - n1) { n1 = N - n1; flip_n = 1; }
  /* Swap the roles of successes and failures. */
  if (M1 > N - M1) { M1 = N - M1; flip_m = 1; }
  uint64_t k = hyp_core(n1, M1, N, &dr);
  if (flip_m) k = n1 - k;
  if (flip_n) k = M - k;
  return k;
}

/* Hyp(n, M, N) of a tree split: the (seed, id, SPLIT) stream. */
static uint64_t hyp(uint64_t n, uint64_t M, uint64_t N, uint64_t seed, uint64_t id) {
  return hyp_stream(n, M, N, seed, id, P_SPLIT);
}

/* Binomial deviate Bin(n, l/Nv), 1 <= l <= Nv - l, from the (seed, id,
 * WRSPLIT) stream (Sec. 4.6: the with-replacement split). */
static uint64_t bin_core(uint64_t n, uint64_t l, uint64_t Nv, draws_t *dr) {
  uint64_t r = Nv - l;
  if (n <= REF_INVERSION_MAX) {
    double qv = (double)r / (double)Nv;
    double p0 = 1.0;
    for (uint64_t i = 0; i < n; ++i) p0 = p0 * qv;
    double odds = (double)l / (double)r;
    for (;;) {
      double u = u53_open0(next_draw(dr));
      double p = p0;
      uint64_t k = 0;
      for (;;) {
        if (u <= p) return k;
        u = u - p;
        if (k == n) break;
        double rt = ((double)(n - k) / (double)(k + 1)) * odds;
        p = p * rt;
        k = k + 1;
      }
    }
  }
  double pp = (double)l / (double)Nv;
  double mu = (double)n * pp;
  double var = mu * (1.0 - pp);
  double a = mu + 0.5;
  double w = sqrt(var + 0.5);
  double s = REF_D1 * w + REF_D2;
  uint64_t mode = bin_mode(n, l, Nv);
  double kmax_d = floor(a + 16.0 * w);
  uint64_t kmax = n + 1;
  if (kmax_d < (double)kmax) kmax = (uint64_t)kmax_d;
  /* ln(l / (Nv - l)) = log1p((2l - Nv) / (Nv - l)) */
  double lodds = log1p64((double)((int64_t)(2 * l) - (int64_t)Nv) / (double)r);
  for (;;) {
    double u = u53_open0(next_draw(dr));
    double v = u53_closed0(next_draw(dr));
    double x = a + (s * (v - 0.5)) / u;
    if (x < 0.0 || x >= (double)kmax) continue;
    uint64_t k = (uint64_t)floor(x);
    double T = (double)((int64_t)k - (int64_t)mode) * lodds;
    T = T + lnfact_diff(mode, k);
    T = T + lnfact_diff(n - mode, n - k);
    if (rou_decide(u, T)) return k;
  }
}

static uint64_t bin(uint64_t n, uint64_t l, uint64_t Nv, uint64_t seed, uint64_t id) {
  if (n == 0 || l == 0) return 0;
  if (l == Nv) return n;
  draws_t dr = {make_stream(seed, id, P_WRSPLIT, 0), 0};
  if (l > Nv - l) return n - bin_core(n, Nv - l, Nv, &dr);
  return bin_core(n, l, Nv, &dr);
}

/* ------------------------------------------------------------------------ */
/* Algorithm H (Sec. 2): hash table with linear probing, addressed by the    */
/* most significant bits of the key; the first `want` distinct values of the */
/* non-void stream.  Used by the sparse leaf and by the dense leaf's repair. */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint64_t *slot; /* value+1, 0 = empty */
  uint64_t mask;
  int shift;
} htab_t;

static int ht_init(htab_t *h, uint64_t want, uint64_t range) {
  uint64_t m = 16;
  while (m < 4 * want) m <<= 1;
  h->slot = (uint64_t *)calloc(m, sizeof(uint64_t));
  if (!h->slot) return REF_ENOMEM;
  h->mask = m - 1;
  int bits = 0;
  while ((1ULL << bits) < range) ++bits; /* keys are < 2^bits */
  int lg = 0;
  while ((1ULL << lg) < m) ++lg;
  h->shift = bits > lg ? bits - lg : 0;
  return REF_OK;
}

/* Insert v; returns 1 if new. */
static int ht_insert(htab_t *h, uint64_t v) {
  uint64_t i = (v >> h->shift) & h->mask;
  for (;;) {
    if (h->slot[i] == 0) { h->slot[i] = v + 1; return 1; }
    if (h->slot[i] == v + 1) return 0;
    i = (i + 1) & h->mask;
  }
}

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* First `want` distinct non-void values in [0, range) of the u32 stream s,
 * returned sorted ascending in `vals`. */
static int first_distinct_sorted(const stream_t *s, uint64_t want, uint64_t range,
                                 uint64_t *vals) {
  htab_t h;
  if (ht_init(&h, want, range) != REF_OK) return REF_ENOMEM;
  uint64_t got = 0;
  for (uint64_t t = 0; got < want; ++t) {
    int64_t v = range_map(stream_word(s, t), range);
    if (v < 0) continue;
    if (ht_insert(&h, (uint64_t)v)) vals[got++] = (uint64_t)v;
  }
  free(h.slot);
  qsort(vals, want, sizeof(uint64_t), cmp_u64);
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Canonical parameters.                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint64_t seed;
  uint32_t n0;          /* base-case threshold: a node is split iff n_v >= n0 */
  uint32_t dense_ratio; /* a leaf is dense iff dense_ratio * n_v >= N_v */
} ctx_t;

/* The output sink: either the whole sample, or only a window [w0, w1) of it. */
typedef struct {
  uint64_t *out;
  uint64_t w0, w1;
} sink_t;

static void sink_put(const sink_t *k, uint64_t pos, uint64_t value) {
  if (pos >= k->w0 && pos < k->w1) k->out[pos - k->w0] = value;
}

static int overlaps(const sink_t *k, uint64_t off, uint64_t cnt) {
  return off < k->w1 && off + cnt > k->w0;
}

static uint64_t isqrt_u64(uint64_t x) {
  uint64_t r = (uint64_t)sqrt((double)x);
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return r;
}

/* Sparse leaf: Algorithm H on [0, Nv) with the (id, LEAF, 0) stream. */
static int leaf_sparse(const ctx_t *c, uint64_t id, uint64_t lo, uint64_t Nv,
                       uint64_t nv, uint64_t off, const sink_t *k) {
  uint64_t *vals = (uint64_t *)malloc(nv * sizeof(uint64_t));
  if (!vals) return REF_ENOMEM;
  stream_t s = make_stream(c->seed, id, P_LEAF, 0);
  int rc = first_distinct_sorted(&s, nv, Nv, vals);
  if (rc == REF_OK)
    for (uint64_t i = 0; i < nv; ++i) sink_put(k, off + i, lo + 1 + vals[i]);
  free(vals);
  return rc;
}

/* Dense leaf: Algorithm B (Sec. 2) with geometric skips (Sec. 4.7). */
static int leaf_dense(const ctx_t *c, uint64_t id, uint64_t lo, uint64_t Nv,
                      uint64_t nv, uint64_t off, const sink_t *k) {
  uint64_t rho_num = nv + 3 * isqrt_u64(nv) + 8;
  int full = rho_num >= Nv; /* rho = 1: every element is a Bernoulli hit */
  float rho = full ? 1.0f : (float)rho_num / (float)Nv;
  float cg = full ? 0.0f : (float)(1.0 / log64(1.0 - (double)rho));
  uint64_t cap = 2 * (uint64_t)c->n0 + 64;
  uint64_t *pos = (uint64_t *)malloc((cap + 1) * sizeof(uint64_t));
  uint64_t *rem = (uint64_t *)malloc((cap + 1) * sizeof(uint64_t));
  if (!pos || !rem) { free(pos); free(rem); return REF_ENOMEM; }
  int rc = REF_OK;
  for (uint32_t attempt = 0;; ++attempt) {
    stream_t sb = make_stream(c->seed, id, P_BERN, attempt);
    int64_t p = -1;
    uint64_t cnt = 0;
    for (uint64_t t = 0;; ++t) {
      int64_t g = 0;
      if (!full) {
        float u = u32_geom(stream_word(&sb, t));
        g = (int64_t)floorf(log32(u) * cg);
      }
      p = p + g + 1;
      if ((uint64_t)p >= Nv) break;
      if (cnt > cap) break; /* already too many: this attempt is rejected */
      pos[cnt++] = (uint64_t)p;
    }
    if (cnt < nv || cnt > cap) continue;
    /* Repair: remove the first (cnt - nv) distinct values of the REPAIR
     * stream mapped into [0, cnt). */
    uint64_t r = cnt - nv;
    if (r > 0) {
      stream_t sr = make_stream(c->seed, id, P_REPAIR, attempt);
      rc = first_distinct_sorted(&sr, r, cnt, rem);
      if (rc != REF_OK) break;
    }
    uint64_t j = 0, o = 0;
    for (uint64_t t = 0; t < cnt; ++t) {
      if (j < r && rem[j] == t) { ++j; continue; }
      sink_put(k, off + o, lo + 1 + pos[t]);
      ++o;
    }
    break;
  }
  free(pos);
  free(rem);
  return rc;
}

/* Algorithm R (Fig. 1): recursive divide and conquer, node = (id, lo, Nv, nv,
 * off); its sample occupies out[off .. off+nv). */
static int sample_r(const ctx_t *c, uint64_t id, uint64_t lo, uint64_t Nv, uint64_t nv,
                    uint64_t off, const sink_t *k) {
  if (nv == 0) return REF_OK;
  if (!overlaps(k, off, nv)) return REF_OK; /* nothing of it is requested */
  if (nv < c->n0 && Nv <= REF_LEAF_MAX_RANGE) {
    if ((uint64_t)c->dense_ratio * nv >= Nv) return leaf_dense(c, id, lo, Nv, nv, off, k);
    return leaf_sparse(c, id, lo, Nv, nv, off, k);
  }
  uint64_t l = Nv / 2;
  uint64_t L = hyp(nv, l, Nv, c->seed, id);
  int rc = sample_r(c, 2 * id, lo, l, L, off, k);
  if (rc != REF_OK) return rc;
  return sample_r(c, 2 * id + 1, lo + l, Nv - l, nv - L, off + L, k);
}

/* With-replacement leaf: the first nv non-void draws, sorted, repeats kept. */
static int leaf_wr(const ctx_t *c, uint64_t id, uint64_t lo, uint64_t Nv, uint64_t nv,
                   uint64_t off, const sink_t *k) {
  uint64_t *vals = (uint64_t *)malloc(nv * sizeof(uint64_t));
  if (!vals) return REF_ENOMEM;
  stream_t s = make_stream(c->seed, id, P_WRLEAF, 0);
  uint64_t got = 0;
  for (uint64_t t = 0; got < nv; ++t) {
    int64_t v = range_map(stream_word(&s, t), Nv);
    if (v >= 0) vals[got++] = (uint64_t)v;
  }
  qsort(vals, nv, sizeof(uint64_t), cmp_u64);
  for (uint64_t i = 0; i < nv; ++i) sink_put(k, off + i, lo + 1 + vals[i]);
  free(vals);
  return REF_OK;
}

/* Sec. 4.6: Algorithm R with binomial instead of hypergeometric splits. */
static int sample_wr(const ctx_t *c, uint64_t id, uint64_t lo, uint64_t Nv, uint64_t nv,
                     uint64_t off, const sink_t *k) {
  if (nv == 0) return REF_OK;
  if (!overlaps(k, off, nv)) return REF_OK;
  if (Nv == 1) {
    for (uint64_t i = 0; i < nv; ++i) sink_put(k, off + i, lo + 1);
    return REF_OK;
  }
  if (nv < c->n0 && Nv <= REF_LEAF_MAX_RANGE) return leaf_wr(c, id, lo, Nv, nv, off, k);
  uint64_t l = Nv / 2;
  uint64_t L = bin(nv, l, Nv, c->seed, id);
  int rc = sample_wr(c, 2 * id, lo, l, L, off, k);
  if (rc != REF_OK) return rc;
  return sample_wr(c, 2 * id + 1, lo + l, Nv - l, nv - L, off + L, k);
}

static int check_params(uint32_t n0, uint32_t dense_ratio) {
  if (n0 < 2 || n0 > 4096) return REF_EINVAL;
  if (dense_ratio < 2 || dense_ratio > 64) return REF_EINVAL;
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Bernoulli sampling over fixed chunks (Sec. 4.7).                          */
/* ------------------------------------------------------------------------ */
#define REF_BERN_FP32_MIN_P 0x1p-10

/* Chunk length 2^floor(log2(n0/p)) clamped to [2^12, 2^32]. */
static uint64_t bern_chunk(double p, uint32_t n0) {
  double x = (double)n0 / p;
  if (!(x < 0x1p32)) return 1ULL << 32;
  int e;
  frexp(x, &e); /* x = f 2^e, f in [0.5,1): floor(log2 x) = e-1 */
  int lg = e - 1;
  if (lg < 12) lg = 12;
  if (lg > 32) lg = 32;
  return 1ULL << lg;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points.                                                    */
/* ------------------------------------------------------------------------ */
EXPORT int dcs_ref_sample_window(uint64_t n, uint64_t N, uint64_t seed, uint32_t n0,
                                 uint32_t dense_ratio, uint64_t start, uint64_t count,
                                 uint64_t *out) {
  if (check_params(n0, dense_ratio) != REF_OK) return REF_EINVAL;
  if (N > REF_MAX_TREE_N || n > N) return REF_EINVAL;
  if (count > 0 && (out == NULL || start > n || count > n - start)) return REF_EINVAL;
  if (count == 0) return REF_OK;
  ctx_t c = {seed, n0, dense_ratio};
  sink_t k = {out, start, start + count};
  return sample_r(&c, 1, 0, N, n, 0, &k);
}

EXPORT int dcs_ref_sample(uint64_t n, uint64_t N, uint64_t seed, uint32_t n0,
                          uint32_t dense_ratio, uint64_t *out) {
  return dcs_ref_sample_window(n, N, seed, n0, dense_ratio, 0, n, out);
}

EXPORT int dcs_ref_replacement_window(uint64_t n, uint64_t N, uint64_t seed, uint32_t n0,
                                      uint64_t start, uint64_t count, uint64_t *out) {
  if (n0 < 2 || n0 > 4096) return REF_EINVAL;
  if (N > REF_MAX_TREE_N || (N == 0 && n > 0)) return REF_EINVAL;
  if (count > 0 && (out == NULL || start > n || count > n - start)) return REF_EINVAL;
  if (count == 0) return REF_OK;
  ctx_t c = {seed, n0, 16};
  sink_t k = {out, start, start + count};
  return sample_wr(&c, 1, 0, N, n, 0, &k);
}

EXPORT int dcs_ref_replacement(uint64_t n, uint64_t N, uint64_t seed, uint32_t n0,
                               uint64_t *out) {
  return dcs_ref_replacement_window(n, N, seed, n0, 0, n, out);
}

/* Online sampling in parts (Sec. 4.1: the sorted sample is produced piece
 * by piece, each piece a subrange split off by the recursion).  The parts
 * at depth d are the 2^d nodes of the tree d levels below the root, from
 * left to right; node `index` is reached by taking, at level i, the right
 * child iff bit d-1-i of index is set.  A path that meets a leaf (or an
 * empty node) above depth d stops there: the leaf's values form the part
 * whose remaining index bits are all zero, and the other parts below it
 * are empty.  *count is the part's size, *rank the number of values of the
 * full sample in earlier parts; the values are written to out[0..count)
 * when count <= capacity (REF_EOVERFLOW and nothing written otherwise). */
EXPORT int dcs_ref_part(int variant, uint64_t n, uint64_t N, uint64_t seed, uint32_t n0,
                        uint32_t dense_ratio, uint32_t depth, uint64_t index, uint64_t *out,
                        uint64_t capacity, uint64_t *count, uint64_t *rank) {
  if (count == NULL || rank == NULL) return REF_EINVAL;
  *count = 0;
  *rank = 0;
  if (variant != 0 && variant != 1) return REF_EINVAL;
  if (check_params(n0, dense_ratio) != REF_OK || N > REF_MAX_TREE_N) return REF_EINVAL;
  if (variant == 0 && n > N) return REF_EINVAL;
  if (variant == 1 && N == 0 && n > 0) return REF_EINVAL;
  if (depth > 45 || index >= (1ULL << depth)) return REF_EINVAL;
  ctx_t c = {seed, n0, dense_ratio};
  uint64_t id = 1, lo = 0, Nv = N, nv = n, off = 0;
  for (uint32_t level = 0; level < depth; ++level) {
    int leaf = variant == 1 ? (Nv == 1 || (nv < n0 && Nv <= REF_LEAF_MAX_RANGE))
                            : (nv < n0 && Nv <= REF_LEAF_MAX_RANGE);
    if (nv == 0) break; /* empty node: every part below it is empty */
    if (leaf) {
      uint64_t rest = index & ((1ULL << (depth - level)) - 1);
      if (rest != 0) { /* not the leftmost part below the leaf */
        off += nv;
        nv = 0;
      }
      break;
    }
    uint64_t l = Nv / 2;
    uint64_t L = variant == 1 ? bin(nv, l, Nv, seed, id) : hyp(nv, l, Nv, seed, id);
    if ((index >> (depth - 1 - level)) & 1) {
      id = 2 * id + 1;
      lo += l;
      Nv -= l;
      nv -= L;
      off += L;
    } else {
      id = 2 * id;
      Nv = l;
      nv = L;
    }
  }
  *count = nv;
  *rank = off;
  if (nv == 0) return REF_OK;
  if (nv > capacity) return REF_EOVERFLOW;
  if (out == NULL) return REF_EINVAL;
  /* the node's subtree writes positions off .. off+nv of the full sample */
  sink_t k = {out, off, off + nv};
  return variant == 1 ? sample_wr(&c, id, lo, Nv, nv, off, &k)
                      : sample_r(&c, id, lo, Nv, nv, off, &k);
}

/* Random graphs (Sec. 7): G(n, m) samples m of the n(n-1)/2 possible edges
 * without replacement, G(n, p) takes each with probability p.  Edge index k
 * (0-based) is the pair (u, v), v < u, with k = u(u-1)/2 + v, i.e. u is the
 * unique integer with u(u-1)/2 <= k < u(u+1)/2.  Since 8k+1 then lies in
 * [(2u-1)^2, (2u+1)^2), u = (1 + isqrt(8k+1)) / 2 (integer square root). */
/* floor(sqrt(x)) of a 128-bit integer: a double estimate, then exact
 * integer corrections. */
static uint64_t isqrt_u128(unsigned __int128 x) {
  uint64_t r = (uint64_t)sqrt((double)x);
  while ((unsigned __int128)r * r > x) --r;
  while ((unsigned __int128)(r + 1) * (r + 1) <= x) ++r;
  return r;
}

static void edge_pair(uint64_t k, uint64_t *u, uint64_t *v) {
  uint64_t r = isqrt_u128(8 * (unsigned __int128)k + 1);
  *u = (1 + r) / 2;
  *v = k - *u * (*u - 1) / 2;
}

/* max_N: the largest universe of the sampler the graph uses. */
static int edge_count(uint64_t n_vertices, uint64_t max_N, uint64_t *N) {
  if (n_vertices > (1ULL << 32)) return REF_EINVAL;
  *N = n_vertices < 2 ? 0 : n_vertices * (n_vertices - 1) / 2;
  return *N > max_N ? REF_EINVAL : REF_OK;
}

static void decode_edges(const uint64_t *vals, uint64_t count, uint32_t *uv) {
  for (uint64_t i = 0; i < count; ++i) {
    uint64_t u, v;
    edge_pair(vals[i] - 1, &u, &v);
    uv[2 * i] = (uint32_t)u;
    uv[2 * i + 1] = (uint32_t)v;
  }
}

EXPORT void dcs_ref_edge_pair(uint64_t k, uint64_t out[2]) { edge_pair(k, &out[0], &out[1]); }

EXPORT int dcs_ref_edges_gnm(uint64_t n_vertices, uint64_t m, uint64_t seed, uint32_t n0,
                             uint32_t *uv) {
  uint64_t N;
  if (edge_count(n_vertices, REF_MAX_TREE_N, &N) != REF_OK || m > N) return REF_EINVAL;
  if (m == 0) return REF_OK;
  uint64_t *vals = (uint64_t *)malloc(m * sizeof(uint64_t));
  if (!vals) return REF_ENOMEM;
  int rc = dcs_ref_sample(m, N, seed, n0, 16, vals);
  if (rc == REF_OK) decode_edges(vals, m, uv);
  free(vals);
  return rc;
}

EXPORT int dcs_ref_bernoulli(double p, uint64_t N, uint64_t seed, uint32_t n0,
                             uint64_t *out, uint64_t capacity, uint64_t *count);

EXPORT int dcs_ref_edges_gnp(uint64_t n_vertices, double p, uint64_t seed, uint32_t n0,
                             uint32_t *uv, uint64_t capacity, uint64_t *count) {
  uint64_t N;
  if (count == NULL) return REF_EINVAL;
  *count = 0;
  if (edge_count(n_vertices, REF_MAX_N, &N) != REF_OK) return REF_EINVAL;
  uint64_t *vals = (uint64_t *)malloc((capacity ? capacity : 1) * sizeof(uint64_t));
  if (!vals) return REF_ENOMEM;
  int rc = dcs_ref_bernoulli(p, N, seed, n0, vals, capacity, count);
  if (rc == REF_OK || rc == REF_EOVERFLOW)
    decode_edges(vals, *count < capacity ? *count : capacity, uv);
  free(vals);
  return rc;
}

/* Bernoulli sample of 1..N with probability p, chunks [jC, (j+1)C) sampled
 * independently with their own streams.  Writes the first `capacity` values
 * to out and the true count to *count.  Chunks [c0, c1) only when
 * chunk_lo/chunk_hi restrict it (then *count is the count of those chunks and
 * values are written from out[0]); pass chunk_hi = UINT64_MAX for all. */
EXPORT int dcs_ref_bernoulli_chunks(double p, uint64_t N, uint64_t seed, uint32_t n0,
                                    uint64_t chunk_lo, uint64_t chunk_hi,
                                    uint64_t *out, uint64_t capacity, uint64_t *count) {
  if (count == NULL) return REF_EINVAL;
  *count = 0;
  if (n0 < 2 || n0 > 4096) return REF_EINVAL;
  if (!(p >= 0.0 && p <= 1.0) || N > REF_MAX_N) return REF_EINVAL;
  if (capacity > 0 && out == NULL) return REF_EINVAL;
  uint64_t got = 0;
  if (p == 0.0 || N == 0) return REF_OK;
  if (p == 1.0) {
    for (uint64_t i = 0; i < N; ++i) {
      if (got < capacity) out[got] = i + 1;
      ++got;
    }
    *count = got;
    return got > capacity ? REF_EOVERFLOW : REF_OK;
  }
  uint64_t C = bern_chunk(p, n0);
  uint64_t nchunks = (N + C - 1) / C;
  if (chunk_hi > nchunks) chunk_hi = nchunks;
  int fp32 = p >= REF_BERN_FP32_MIN_P;
  double c64 = 1.0 / log1p64(-p);
  float c32 = (float)c64;
  for (uint64_t j = chunk_lo; j < chunk_hi; ++j) {
    uint64_t base = j * C;
    uint64_t len = (N - base) < C ? (N - base) : C;
    stream_t s = make_stream(seed, j, P_BCHUNK, 0);
    int64_t pos = -1;
    for (uint64_t t = 0;; ++t) {
      if (fp32) {
        float u = u32_geom(stream_word(&s, t));
        float g = floorf(log32(u) * c32);
        double np = (double)pos + (double)g + 1.0;
        if (np >= (double)len) break;
        pos = (int64_t)np;
      } else {
        double u = u53_open0(stream_draw64(&s, t));
        double g = floor(log64(u) * c64);
        double np = (double)pos + g + 1.0;
        if (np >= (double)len) break;
        pos = (int64_t)np;
      }
      if (got < capacity) out[got] = base + (uint64_t)pos + 1;
      ++got;
    }
  }
  *count = got;
  return got > capacity ? REF_EOVERFLOW : REF_OK;
}

EXPORT int dcs_ref_bernoulli(double p, uint64_t N, uint64_t seed, uint32_t n0,
                             uint64_t *out, uint64_t capacity, uint64_t *count) {
  return dcs_ref_bernoulli_chunks(p, N, seed, n0, 0, UINT64_MAX, out, capacity, count);
}

EXPORT uint64_t dcs_ref_bernoulli_chunk_len(double p, uint32_t n0) {
  return bern_chunk(p, n0);
}

/* Sampling over an uneven universe (Sec. 4.3, owner computes).  The
 * universe is the concatenation of K segments -- the paper's PEs 0..K-1,
 * PE i holding L_i elements -- and the sample is n distinct elements of
 * 1..N, N = L_0 + ... + L_{K-1}; segment i computes those that fall into
 * it.
 *
 * The segments form the paper's binomial tree: at level j (level 0 = the
 * segments) subtree a spans segments 2^j a .. min(2^j a + 2^j, K) - 1, and
 * its children are subtrees 2a and 2a+1 of level j-1.  Upward pass: the
 * element count of every subtree, level by level from j = 0.  Downward
 * pass: the root (level D = ceil(log2 K)) holds n; an inner node holding n'
 * gives its left subtree n_l = Hyp(n', L_l, L_l + L_r) and its right one
 * n' - n_l.  The hash input of a node (Sec. 4.3: the range of PEs it
 * represents) is its heap index 2^(D-j) + a, with the SEGSPLIT purpose; a
 * node whose right subtree lies beyond K has L_r = 0, so n_l = n' (Hyp's
 * exact case).
 *
 * Segment i then samples its n_i of L_i by Algorithm R (Fig. 1) keyed by
 * seed_i = 64-bit draw 0 of (seed, 2^D + i, SEGSEED): the hash of its own
 * leaf identity.  Its values are shifted by the elements of the segments
 * before it and follow the samples of those segments. */
#define REF_MAX_SEGMENTS (1ULL << 24)

static uint32_t ceil_log2_u64(uint64_t k) {
  uint32_t d = 0;
  while ((1ULL << d) < k) ++d;
  return d;
}

/* Both passes; sums[id] and cnt[id] for heap ids 1 .. 2^(D+1) - 1 (zeroed
 * by the caller; subtrees that start at or beyond K keep 0). */
static void segment_tree(uint64_t n, const uint64_t *L, uint64_t K, uint64_t seed, uint32_t D,
                         uint64_t *sums, uint64_t *cnt) {
  for (uint64_t a = 0; a < K; ++a) sums[(1ULL << D) + a] = L[a];
  for (uint32_t j = 1; j <= D; ++j) {
    uint64_t first = 1ULL << (D - j);
    uint64_t width = (K + (1ULL << j) - 1) >> j;
    for (uint64_t a = 0; a < width; ++a)
      sums[first + a] = sums[2 * (first + a)] + sums[2 * (first + a) + 1];
  }
  cnt[1] = n;
  for (uint32_t j = D; j >= 1; --j) {
    uint64_t first = 1ULL << (D - j);
    uint64_t width = (K + (1ULL << j) - 1) >> j;
    for (uint64_t a = 0; a < width; ++a) {
      uint64_t id = first + a;
      uint64_t Ll = sums[2 * id], Lr = sums[2 * id + 1];
      uint64_t nl = hyp_stream(cnt[id], Ll, Ll + Lr, seed, id, P_SEGSPLIT);
      cnt[2 * id] = nl;
      cnt[2 * id + 1] = cnt[id] - nl;
    }
  }
}

static int segments_check(uint64_t n, const uint64_t *lengths, uint64_t K, uint64_t *N) {
  if (K == 0 || K > REF_MAX_SEGMENTS || lengths == NULL) return REF_EINVAL;
  uint64_t total = 0;
  for (uint64_t i = 0; i < K; ++i) {
    if (lengths[i] > REF_MAX_TREE_N - total) return REF_EINVAL;
    total += lengths[i];
  }
  if (n > total) return REF_EINVAL;
  *N = total;
  return REF_OK;
}

/* The two passes alone: sums and cnt receive 2^(D+1) entries each (entry 0
 * unused), in heap order. */
EXPORT int dcs_ref_segment_tree(uint64_t n, const uint64_t *lengths, uint64_t K, uint64_t seed,
                                uint64_t *sums, uint64_t *cnt) {
  uint64_t N;
  if (segments_check(n, lengths, K, &N) != REF_OK || sums == NULL || cnt == NULL)
    return REF_EINVAL;
  uint32_t D = ceil_log2_u64(K);
  memset(sums, 0, (2ULL << D) * sizeof(uint64_t));
  memset(cnt, 0, (2ULL << D) * sizeof(uint64_t));
  segment_tree(n, lengths, K, seed, D, sums, cnt);
  return REF_OK;
}

/* The sample: out[0..n) ascending (values in 1..N); counts[i] = n_i if
 * counts is not NULL. */
EXPORT int dcs_ref_sample_segments(uint64_t n, const uint64_t *lengths, uint64_t K,
                                   uint64_t seed, uint32_t n0, uint32_t dense_ratio,
                                   uint64_t *out, uint64_t *counts) {
  uint64_t N;
  if (check_params(n0, dense_ratio) != REF_OK) return REF_EINVAL;
  if (segments_check(n, lengths, K, &N) != REF_OK) return REF_EINVAL;
  if (n > 0 && out == NULL) return REF_EINVAL;
  uint32_t D = ceil_log2_u64(K);
  uint64_t *sums = (uint64_t *)calloc(2ULL << D, sizeof(uint64_t));
  uint64_t *cnt = (uint64_t *)calloc(2ULL << D, sizeof(uint64_t));
  int rc = (sums && cnt) ? REF_OK : REF_ENOMEM;
  if (rc == REF_OK) {
    segment_tree(n, lengths, K, seed, D, sums, cnt);
    ctx_t c = {0, n0, dense_ratio};
    uint64_t base = 0, off = 0;
    for (uint64_t i = 0; rc == REF_OK && i < K; ++i) {
      uint64_t ni = cnt[(1ULL << D) + i];
      if (counts) counts[i] = ni;
      if (ni > 0) {
        stream_t st = make_stream(seed, (1ULL << D) + i, P_SEGSEED, 0);
        c.seed = stream_draw64(&st, 0);
        sink_t k = {out + off, 0, ni};
        rc = sample_r(&c, 1, base, lengths[i], ni, 0, &k);
      }
      base += lengths[i];
      off += ni;
    }
  }
  free(sums);
  free(cnt);
  return rc;
}

/* Algorithm B over the whole range (Sec. 2, with the skips and prefix sums of
 * Sec. 4.7, as the paper's GPU variant of Sec. 5 runs it, minus its host
 * round trip): n of 1..N without replacement, for 1 <= N <= 2^32 and
 * rho >= 2^-10.
 *   rho = min(1, (n + 8 isqrt(n) + 16) / N) in double;
 *   attempt a = 0, 1, ...: the Bernoulli(rho) hits of 0..N-1 by the chunks
 *     and single-precision skips of Sec. 4.7's variant (chunk j keyed by
 *     (j, WCHUNK, a)); rho = 1 makes every element a hit;
 *   accept iff n <= n' <= n + 16 isqrt(n) + 64 for the hit count n' (any
 *   rule on n' alone keeps the sample uniform), else the next attempt;
 *   remove the hits whose index (0-based, in position order) is one of the
 *   first n' - n distinct non-void values of (0, WREPAIR, a) mapped into
 *   [0, n') -- Algorithm H's rule;
 *   output the remaining positions + 1, ascending.
 * *attempt_out receives the accepted attempt. */
#define REF_WB_MIN_RHO 0x1p-10

static uint64_t wb_rho_num(uint64_t n) { return n + 8 * isqrt_u64(n) + 16; }

static int wb_check(uint64_t n, uint64_t N, double *rho) {
  if (N == 0 || N > (1ULL << 32) || n > N) return REF_EINVAL;
  uint64_t num = wb_rho_num(n);
  *rho = num >= N ? 1.0 : (double)num / (double)N;
  if (n > 0 && *rho < REF_WB_MIN_RHO) return REF_EINVAL;
  return REF_OK;
}

/* Hits of attempt a: positions into pos[0..cap) while they fit; returns n'. */
static uint64_t wb_hits(double rho, uint64_t N, uint64_t seed, uint32_t n0, uint32_t attempt,
                        uint64_t *pos, uint64_t cap) {
  uint64_t got = 0;
  if (rho >= 1.0) {
    for (uint64_t i = 0; i < N; ++i) {
      if (got < cap) pos[got] = i;
      ++got;
    }
    return got;
  }
  uint64_t C = bern_chunk(rho, n0);
  float c32 = (float)(1.0 / log1p64(-rho));
  for (uint64_t base = 0, j = 0; base < N; base += C, ++j) {
    uint64_t len = (N - base) < C ? (N - base) : C;
    stream_t s = make_stream(seed, j, P_WCHUNK, attempt);
    int64_t q = -1;
    for (uint64_t t = 0;; ++t) {
      float g = floorf(log32(u32_geom(stream_word(&s, t))) * c32);
      double nq = (double)q + (double)g + 1.0;
      if (nq >= (double)len) break;
      q = (int64_t)nq;
      if (got < cap) pos[got] = base + (uint64_t)q;
      ++got;
    }
  }
  return got;
}

EXPORT int dcs_ref_sample_wholerange(uint64_t n, uint64_t N, uint64_t seed, uint32_t n0,
                                     uint64_t *out, uint32_t *attempt_out) {
  double rho;
  if (n0 < 2 || n0 > 4096 || wb_check(n, N, &rho) != REF_OK) return REF_EINVAL;
  if (attempt_out) *attempt_out = 0;
  if (n == 0) return REF_OK;
  if (out == NULL) return REF_EINVAL;
  uint64_t hi = n + 16 * isqrt_u64(n) + 64;
  uint64_t *pos = (uint64_t *)malloc((hi + 1) * sizeof(uint64_t));
  uint64_t *rem = (uint64_t *)malloc((hi - n + 1) * sizeof(uint64_t));
  int rc = (pos && rem) ? REF_OK : REF_ENOMEM;
  for (uint32_t a = 0; rc == REF_OK; ++a) {
    uint64_t nh = wb_hits(rho, N, seed, n0, a, pos, hi + 1);
    if (nh < n || nh > hi) continue;
    uint64_t r = nh - n;
    if (r > 0) {
      stream_t sr = make_stream(seed, 0, P_WREPAIR, a);
      rc = first_distinct_sorted(&sr, r, nh, rem);
      if (rc != REF_OK) break;
    }
    uint64_t j = 0, o = 0;
    for (uint64_t h = 0; h < nh; ++h) {
      if (j < r && rem[j] == h) { ++j; continue; }
      out[o++] = pos[h] + 1;
    }
    if (attempt_out) *attempt_out = a;
    break;
  }
  free(pos);
  free(rem);
  return rc;
}

/* The hit count n' of one attempt (for the law of n'), and its first
 * min(n', cap) positions + 1. */
EXPORT int dcs_ref_wholerange_hits(uint64_t n, uint64_t N, uint64_t seed, uint32_t n0,
                                   uint32_t attempt, uint64_t *out, uint64_t cap,
                                   uint64_t *count) {
  double rho;
  if (n0 < 2 || n0 > 4096 || wb_check(n, N, &rho) != REF_OK || count == NULL) return REF_EINVAL;
  if (cap > 0 && out == NULL) return REF_EINVAL;
  uint64_t *pos = (uint64_t *)malloc((cap + 1) * sizeof(uint64_t));
  if (!pos) return REF_ENOMEM;
  *count = wb_hits(rho, N, seed, n0, attempt, pos, cap);
  for (uint64_t i = 0; i < cap && i < *count; ++i) out[i] = pos[i] + 1;
  free(pos);
  return REF_OK;
}

/* --- primitives, exported so that the tests can pin each one ----------- */
EXPORT void dcs_ref_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox4x32_10(ctr, key, out);
}
EXPORT uint32_t dcs_ref_stream_word(uint64_t seed, uint64_t id, uint32_t purpose,
                                    uint32_t attempt, uint64_t t) {
  stream_t s = make_stream(seed, id, purpose, attempt);
  return stream_word(&s, t);
}
EXPORT uint64_t dcs_ref_stream_draw64(uint64_t seed, uint64_t id, uint32_t purpose,
                                      uint32_t attempt, uint64_t t) {
  stream_t s = make_stream(seed, id, purpose, attempt);
  return stream_draw64(&s, t);
}
EXPORT int64_t dcs_ref_range_map(uint32_t w, uint64_t s) { return range_map(w, s); }
EXPORT double dcs_ref_log64(double x) { return log64(x); }
EXPORT double dcs_ref_log1p64(double x) { return log1p64(x); }
EXPORT float dcs_ref_log32(float x) { return log32(x); }
EXPORT float dcs_ref_u32_geom(uint32_t w) { return u32_geom(w); }
EXPORT double dcs_ref_lnfact_diff(uint64_t a, uint64_t b) { return lnfact_diff(a, b); }
EXPORT uint64_t dcs_ref_hyp(uint64_t n, uint64_t M, uint64_t N, uint64_t seed, uint64_t id) {
  return hyp(n, M, N, seed, id);
}
EXPORT uint64_t dcs_ref_bin(uint64_t n, uint64_t l, uint64_t Nv, uint64_t seed, uint64_t id) {
  return bin(n, l, Nv, seed, id);
}
/* The modes the ratio-of-uniforms tests are centred on (hypergeometric with
 * n, M <= N/2; binomial with l <= Nv - l). */
EXPORT uint64_t dcs_ref_hyp_mode(uint64_t n, uint64_t M, uint64_t N) { return hyp_mode(n, M, N); }
EXPORT uint64_t dcs_ref_bin_mode(uint64_t n, uint64_t l, uint64_t Nv) { return bin_mode(n, l, Nv); }

/* Tree statistics (for the node-count invariant of Sec. 3.1): counts the
 * internal nodes and the non-empty leaves of the without-replacement tree. */
static void count_nodes(const ctx_t *c, uint64_t id, uint64_t Nv, uint64_t nv,
                        uint64_t *internal, uint64_t *leaves, uint64_t *depth_max,
                        uint64_t depth) {
  if (nv == 0) return;
  if (depth > *depth_max) *depth_max = depth;
  if (nv < c->n0 && Nv <= REF_LEAF_MAX_RANGE) { ++*leaves; return; }
  ++*internal;
  uint64_t l = Nv / 2;
  uint64_t L = hyp(nv, l, Nv, c->seed, id);
  count_nodes(c, 2 * id, l, L, internal, leaves, depth_max, depth + 1);
  count_nodes(c, 2 * id + 1, Nv - l, nv - L, internal, leaves, depth_max, depth + 1);
}

EXPORT int dcs_ref_tree_stats(uint64_t n, uint64_t N, uint64_t seed, uint32_t n0,
                              uint64_t stats[3]) {
  if (n0 < 2 || n0 > 4096 || N > REF_MAX_TREE_N || n > N) return REF_EINVAL;
  ctx_t c = {seed, n0, 16};
  stats[0] = stats[1] = stats[2] = 0;
  count_nodes(&c, 1, N, n, &stats[0], &stats[1], &stats[2], 0);
  return REF_OK;
}

/* --- batch forms of the primitives (plain loops), for the pin tests ----- */
EXPORT void dcs_ref_log32_batch(const float *x, uint64_t n, float *y) {
  for (uint64_t i = 0; i < n; ++i) y[i] = log32(x[i]);
}
EXPORT void dcs_ref_log64_batch(const double *x, uint64_t n, double *y) {
  for (uint64_t i = 0; i < n; ++i) y[i] = log64(x[i]);
}
EXPORT void dcs_ref_log1p64_batch(const double *x, uint64_t n, double *y) {
  for (uint64_t i = 0; i < n; ++i) y[i] = log1p64(x[i]);
}
EXPORT void dcs_ref_lnfact_diff_batch(const uint64_t *a, const uint64_t *b, uint64_t n,
                                      double *y) {
  for (uint64_t i = 0; i < n; ++i) y[i] = lnfact_diff(a[i], b[i]);
}
EXPORT void dcs_ref_hyp_batch(uint64_t n, uint64_t M, uint64_t N, uint64_t seed,
                              uint64_t id0, uint64_t count, uint64_t *out) {
  for (uint64_t i = 0; i < count; ++i) out[i] = hyp(n, M, N, seed, id0 + i);
}
EXPORT void dcs_ref_bin_batch(uint64_t n, uint64_t l, uint64_t Nv, uint64_t seed,
                              uint64_t id0, uint64_t count, uint64_t *out) {
  for (uint64_t i = 0; i < count; ++i) out[i] = bin(n, l, Nv, seed, id0 + i);
}
/* For every one of the 2^32 words: how often each value in [0, s) is hit by
 * range_map, and how many words are void.  counts has s entries. */
EXPORT void dcs_ref_range_map_counts(uint64_t s, uint64_t *counts, uint64_t *voids) {
  uint64_t nv = 0;
  for (uint64_t w = 0; w < (1ULL << 32); ++w) {
    int64_t v = range_map((uint32_t)w, s);
    if (v < 0) ++nv; else ++counts[v];
  }
  *voids = nv;
}
