// dcs_kernels.hip -- the sampler's kernels for gfx950.
//
//   k_reset      zero a workspace control block (and store a single instance)
//   k_tree       recursion tree: each thread follows one root-to-depth-`cut`
//                path of Algorithm R, recomputing the splits on the way
//                exactly as a processing element of Algorithm P does
//                (paper Sec. 3.2, Fig. 2), then expands the subtree below by
//                a depth-first walk; every leaf becomes a self-contained job.
//   k_leaf       persistent work-groups, each taking every G-th leaf job (the
//                atomic jobs of Sec. 4.2, assigned statically so that job
//                records stream into LDS ahead of use), run the base case:
//                  sparse  Algorithm H semantics (Sec. 2): the first n_v
//                          distinct values of the node's stream, found in
//                          rounds with an LDS counting sort by most
//                          significant bits (the sorted-H idea of Sec. 4.1);
//                  dense   Algorithm B (Sec. 2): geometric skips + prefix sum
//                          (Sec. 4.7), restart on a short sample, removal of
//                          the excess by Algorithm H semantics;
//                  with replacement (Sec. 4.6): sorted draws, repeats kept.
//                The leaf's sorted values leave LDS as coalesced
//                non-temporal 64-bit stores.
//   k_bern       Bernoulli sampling over fixed chunks (Sec. 4.7), chunk
//                offsets by a decoupled look-back over an atomic ticket.
//   k_debug      elementwise primitives for bit-exact tests.
#include <type_traits>

#include "dcs_device.hpp"
#include "dcs_kernels.hpp"

namespace dcs {

// ---------------------------------------------------------------------------
// Block-wide exclusive prefix sums (one value per thread).  `scratch` holds
// BLOCK/64 words of LDS; *total receives the block sum.
// ---------------------------------------------------------------------------
// Inclusive prefix sum across the 64 lanes of a wave with DPP moves:
// row_shr 1, 2, 4, 8 inside each 16-lane row, then row_bcast15 / row_bcast31
// carry the row totals forward (lanes without a source add 0).
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x) {
  x += __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0u, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0u, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

__device__ __forceinline__ uint64_t wave_scan_incl(uint64_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// kTail = false drops the closing barrier that guards `scratch` against the
// next scan; the caller then guarantees a barrier before scratch is written
// again.
template <int BLOCK, typename T, bool kTail = true>
__device__ __forceinline__ T block_scan_excl(T v, T* scratch, T* total) {
  constexpr int kW = BLOCK / 64;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const T x = wave_scan_incl(v);
  if (lane == 63) scratch[wave] = x;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kW; ++w) {
    const T s = scratch[w];
    before += (w < wave) ? s : T(0);
    all += s;
  }
  if (kTail) __syncthreads();
  *total = all;
  return before + x - v;
}

// threadIdx.x, opaque to the optimizer: values derived from it are then
// recomputed where used instead of being hoisted out of the persistent leaf
// loop and spilled (a spill reload waits for all of the wave's outstanding
// output stores).
__device__ __forceinline__ uint32_t lane_tid() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x >> 32));
  return static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32);
}

__device__ __forceinline__ uint32_t bit_length(uint64_t x) {
  return x == 0 ? 0u : 64u - static_cast<uint32_t>(__clzll(static_cast<long long>(x)));
}

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void store_out(uint64_t* out, uint64_t v) {
  __builtin_nontemporal_store(v, out);
}

// ---------------------------------------------------------------------------
// LDS layout of a leaf work-group (32-bit words).
//   [0, kRegionA)            sparse: keys | tmp      dense: positions
//   [kRegionA, +kRegionB)    sparse: bucket counts   dense: kept | mask
//   [.., +kCacheWords)       leaf-job records read ahead
//   [.., +kScratch)          scan scratch
// ---------------------------------------------------------------------------
constexpr uint32_t kKeys = kMaxN0;                    // 4096 keys
constexpr uint32_t kDenseCap = 2 * kMaxN0 + 64;        // largest accepted n'
constexpr uint32_t kRegionA = 2 * kMaxN0 + 128;        // >= kDenseCap + 1
constexpr uint32_t kBuckets = kMaxN0;                  // most buckets used
constexpr uint32_t kBucketPad = 3;                     // one pad word per 8
// region B ends with spare words: kSpareCount counts keys of unused positions
constexpr uint32_t kSpareCount = kBuckets + (kBuckets >> kBucketPad);
constexpr uint32_t kRegionB = kSpareCount + 4;
constexpr uint32_t kMaskWords = (kDenseCap + 32) / 32 + 1;
static_assert(kKeys + kMaskWords <= kRegionB, "dense kept values + mask fit region B");
constexpr uint32_t kCacheLeaves = 32;
constexpr uint32_t kLeafWords = sizeof(Leaf) / 4;
constexpr uint32_t kCacheWords = kCacheLeaves * kLeafWords;
constexpr uint32_t kScratch = 64;
// sorted keys live in region A's first kKeys words; unused positions scatter
// to its last word
constexpr uint32_t kSpareSlot = kRegionA - 1;
static_assert(kSpareSlot >= kKeys, "spare slot lies outside the sorted keys");
constexpr uint32_t kSmemWords = kRegionA + kRegionB + kCacheWords + kScratch;
// scratch words: [0, 16) scan; 16 next-word offset; 17 duplicate flag;
// [24, 40) per-wave maxima; 48 which cached jobs the work-group runs
constexpr uint32_t kScrNext = 16, kScrDups = 17, kScrMax = 24, kScrKeep = 48;

__device__ __forceinline__ uint32_t bpad(uint32_t b) { return b + (b >> kBucketPad); }

struct LeafSmem {
  uint32_t* keys;  // kKeys
  uint32_t* tmp;   // kKeys
  uint32_t* buck;  // kRegionB (padded bucket counters)
  uint32_t* kept;  // = buck, dense
  uint32_t* mask;  // after kept, dense
  uint32_t* scr;   // kScratch
};

struct RangeInfo {
  uint64_t s;
  uint32_t thr;
  bool pow2;
  uint32_t pshift;  // pow2: value = word >> pshift (32: value 0)
};

__device__ __forceinline__ RangeInfo range_info(uint64_t s) {
  RangeInfo r;
  r.s = s;
  r.pow2 = (s & (s - 1)) == 0;
  r.pshift = r.pow2 ? 32u - (bit_length(s) - 1u) : 0u;
  r.thr = r.pow2 ? 0u : range_threshold(s);
  return r;
}

// ---------------------------------------------------------------------------
// The first `need` non-void values in [0, s) of a 32-bit stream, from word
// t0 on, delivered in stream order to sink(p, value), p = 0..need-1.
// Returns the word index just after the last value taken.  For a power-of-two
// range no word is void and value p is word t0+p.  Otherwise each round
// examines at most as many words as values are still wanted (a void costs a
// further round) and a block scan orders the survivors.
// ---------------------------------------------------------------------------
template <int B, class Sink>
__device__ uint64_t take_values(const Stream& st, uint64_t t0, uint32_t need, const RangeInfo& ri,
                                uint32_t* scr, Sink sink) {
  if (need == 0) return t0;
  if (ri.pow2) {
    const uint64_t t1 = t0 + need;
    for (uint64_t blk = (t0 >> 2) + threadIdx.x; (blk << 2) < t1; blk += B) {
      const uint4 w = philox_block(st, static_cast<uint32_t>(blk));
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint64_t t = (blk << 2) + j;
        if (t >= t0 && t < t1) {
          const uint32_t word = pick(w, j);
          sink(static_cast<uint32_t>(t - t0), ri.pshift >= 32 ? 0u : (word >> ri.pshift));
        }
      }
    }
    __syncthreads();
    return t1;
  }
  uint32_t done = 0;
  uint64_t t = t0;
  while (done < need) {
    const uint32_t want = need - done;
    const uint64_t first_blk = t >> 2;
    uint64_t last_word = t + want;
    const uint64_t reach = (first_blk + B) << 2;
    if (last_word > reach) last_word = reach;
    const uint64_t blk = first_blk + threadIdx.x;
    uint32_t v[4];
    uint32_t ok = 0;
    if ((blk << 2) < last_word) {
      const uint4 w = philox_block(st, static_cast<uint32_t>(blk));
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint64_t tj = (blk << 2) + j;
        const bool good = range_map(pick(w, j), ri.s, ri.thr, &v[j]);
        if (good && tj >= t && tj < last_word) ok |= 1u << j;
      }
    }
    uint32_t total;
    uint32_t p = done + block_scan_excl<B, uint32_t>(__popc(ok), scr, &total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (ok & (1u << j)) {
        if (p < need) {
          sink(p, v[j]);
          if (p == need - 1) scr[kScrNext] = static_cast<uint32_t>(((blk << 2) + j + 1) - t0);
        }
        ++p;
      }
    }
    done += total;
    t = last_word;
    __syncthreads();
  }
  const uint64_t next = t0 + scr[kScrNext];
  __syncthreads();
  return next;
}

// ---------------------------------------------------------------------------
// Batcher's odd-even merge sorting network for 16 inputs (63 comparators):
// sort both halves, then merge them; two sorted runs interleaved at stride r
// merge by merging their even and odd subsequences (stride 2r) and then
// comparing neighbours at distance r.
// ---------------------------------------------------------------------------
constexpr uint8_t kNet16[63][2] = {
    {0, 1},   {2, 3},   {0, 2},   {1, 3},   {1, 2},   {4, 5},   {6, 7},   {4, 6},
    {5, 7},   {5, 6},   {0, 4},   {2, 6},   {2, 4},   {1, 5},   {3, 7},   {3, 5},
    {1, 2},   {3, 4},   {5, 6},   {8, 9},   {10, 11}, {8, 10},  {9, 11},  {9, 10},
    {12, 13}, {14, 15}, {12, 14}, {13, 15}, {13, 14}, {8, 12},  {10, 14}, {10, 12},
    {9, 13},  {11, 15}, {11, 13}, {9, 10},  {11, 12}, {13, 14}, {0, 8},   {4, 12},
    {4, 8},   {2, 10},  {6, 14},  {6, 10},  {2, 4},   {6, 8},   {10, 12}, {1, 9},
    {5, 13},  {5, 9},   {3, 11},  {7, 15},  {7, 11},  {3, 5},   {7, 9},   {11, 13},
    {1, 2},   {3, 4},   {5, 6},   {7, 8},   {9, 10},  {11, 12}, {13, 14}};

// The first 19 comparators sort inputs 0..7: Batcher's network for 8.  The
// last 9 of those (and the last 25 of the 16-input network) are the final
// merge stage, which alone sorts an input whose two halves are sorted.
template <int W, bool kMergeOnly>
__device__ __forceinline__ void sort_net(uint32_t (&v)[W]) {
  static_assert(W == 8 || W == 16, "networks for 8 and 16 inputs");
  constexpr int kEnd = W == 16 ? 63 : 19;
  constexpr int kBegin = kMergeOnly ? (W == 16 ? 38 : 10) : 0;
#pragma unroll
  for (int c = kBegin; c < kEnd; ++c) {
    const uint32_t a = v[kNet16[c][0]], b = v[kNet16[c][1]];
    v[kNet16[c][0]] = min(a, b);
    v[kNet16[c][1]] = max(a, b);
  }
}

// Inclusive prefix maximum across a wave (same DPP pattern, counts >= 0).
__device__ __forceinline__ uint32_t wave_max_incl(uint32_t x) {
  x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x111, 0xf, 0xf, false)));
  x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x112, 0xf, 0xf, false)));
  x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x114, 0xf, 0xf, false)));
  x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x118, 0xf, 0xf, false)));
  x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x142, 0xa, 0xf, false)));
  x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x143, 0xc, 0xf, false)));
  return x;
}

// Sorts the W-key windows keys[off + Wi .. off + Wi + W) that start below n
// (entries past n are 0xFFFFFFFF sentinels); kMergeOnly: each window's halves
// are already sorted.  Returns, in each lane, the ballot over the lanes that
// took the same branch: nonzero in some lane of the wave iff one of its
// windows holds equal neighbours among its first n entries.
template <int B, int W, bool kMergeOnly>
__device__ __forceinline__ uint64_t window_pass(uint32_t* keys, uint32_t n, uint32_t off,
                                                uint32_t tid) {
  static_assert(W * B >= kKeys, "one window per thread");
  uint64_t dup = 0;
  const uint32_t w0 = off + W * tid;
  if (w0 < n) {
    uint4* p = reinterpret_cast<uint4*>(keys + w0);
    uint32_t v[W];
#pragma unroll
    for (int q = 0; q < W / 4; ++q) {
      const uint4 x = p[q];
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    }
    sort_net<W, kMergeOnly>(v);
#pragma unroll
    for (int q = 0; q < W / 4; ++q)
      p[q] = make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    if (w0 + W <= n) {  // the whole window lies below n
#pragma unroll
      for (int i = 0; i + 1 < W; ++i) dup |= __ballot(v[i] == v[i + 1]);
    } else {
      const uint32_t lim = n - w0;  // entries of this window below n
#pragma unroll
      for (int i = 0; i + 1 < W; ++i)
        dup |= __ballot(v[i] == v[i + 1] && static_cast<uint32_t>(i + 1) < lim);
    }
  }
  return dup;
}

// ---------------------------------------------------------------------------
// Sort of up to 4096 keys held in registers: thread tid holds the keys at
// positions 4(tid + kB) + j (j < 4); positions >= n are unused.
//   1. counting pass by most significant bits (bucket = key >> shift,
//      nb <= 4096 buckets; counters at padded indices so that each thread's
//      run of the scan falls in distinct LDS banks), LDS atomics give each
//      key its slot inside its bucket;
//   2. exclusive scan of the counts (always over 4096 buckets, the unused
//      ones zero), which also finds the largest bucket c_max;
//   3. scatter into sm.keys in bucket order;
//   4. order inside the buckets.  Sorting any window of bucket-ordered keys
//      only permutes keys within buckets, so sorting the W-key windows at Wi
//      and then those at Wi + W/2 sorts every bucket of at most W/2 + 1 keys
//      (it lies inside a window of one of the two passes), and equal keys,
//      which share a bucket, meet as neighbours inside such a window; W = 8
//      when c_max <= 5, W = 16 when c_max <= 9.  Larger
//      buckets (c_max > 9, rare) take c_max odd-even transposition rounds
//      over the whole array -- a pair that spans two buckets never swaps, so
//      each bucket is sorted after as many rounds as it has keys -- and a
//      pass comparing neighbours.  With shift = 0 a bucket holds one value:
//      nothing to order, and values repeat iff c_max >= 2.
// Result: sm.keys[0..n) ascending, equal values adjacent.  Returns nonzero
// iff some value occurs twice.  Keys of unused positions add 0 to a spare
// counter whose scanned start is a spare slot, so the passes carry no
// per-key branches.  Each key keeps its counter index | slot << 16 in one
// register between the passes.
// kLazyZero: the counters are zero on entry and are zeroed again once read
// (during the first window pass), and the sentinels and the duplicate flag
// are written after the counting barrier, so that a caller may start the next
// sort without a barrier after this sort's result has been read; otherwise
// everything is cleared on entry.
// ---------------------------------------------------------------------------
template <int B>
__device__ __forceinline__ void zero_counters(uint32_t* cnt, uint32_t tid) {
  for (uint32_t w = tid; w < kSpareCount / 4; w += B)
    reinterpret_cast<uint4*>(cnt)[w] = make_uint4(0, 0, 0, 0);
  if (tid == 0) cnt[kSpareCount] = 0;
}

constexpr uint32_t kDeadKey = 0xFFFFFFFFu;  // counter/slot word of a key left out

// kMasked: key[q] takes part iff bit q of `live` is set (n of them), wherever
// it sits; otherwise key[q] takes part iff its position 4(tid + kB) + j < n.
template <int B, bool kLazyZero = false, bool kMasked = false>
__device__ uint32_t sort_registers(const uint32_t (&key)[kKeys / B], uint32_t n, uint32_t shift,
                                   uint32_t nb, LeafSmem& sm, uint32_t live_mask = 0) {
  constexpr int kBlk = kKeys / (4 * B);
  constexpr int kPer = kBuckets / B;  // buckets per thread in the scan
  constexpr int kPairs = kKeys / (2 * B);
  static_assert(kPer >= 1 && 8 % kPer == 0, "a scan run stays inside one padded group of 8");
  (void)nb;
  const uint32_t tid = lane_tid();
  const uint32_t wave_first = tid & ~63u;
  uint32_t* cnt = sm.buck;
  uint32_t* keys = sm.keys;
  // 1. zero the counters, sentinels after the keys, count
  if (!kLazyZero) {
    zero_counters<B>(cnt, tid);
    if (tid < 24) keys[n + tid] = 0xFFFFFFFFu;
    if (tid == 0) sm.scr[kScrDups] = 0;
    __syncthreads();
  }
  uint32_t as[4 * kBlk];
#pragma unroll
  for (int k = 0; k < kBlk; ++k) {
    const uint32_t first = 4 * (wave_first + k * B);  // first key position of the wave
    if (kMasked) {
      // dead keys skip the counters and the scatter (all of them on one
      // spare word would serialize the LDS accesses of the whole wave)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = 4 * k + j;
        as[q] = kDeadKey;
        if ((live_mask >> q) & 1u) {
          const uint32_t a = bpad(key[q] >> shift);
          as[q] = a | (atomicAdd(&cnt[a], 1u) << 16);
        }
      }
    } else if (first + 256 <= n) {                    // every lane holds 4 keys
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = 4 * k + j;
        const uint32_t a = bpad(key[q] >> shift);
        as[q] = a | (atomicAdd(&cnt[a], 1u) << 16);
      }
    } else if (first < n) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = 4 * k + j;
        const bool live = 4 * (tid + k * B) + j < n;
        const uint32_t a = live ? bpad(key[q] >> shift) : kSpareCount;
        as[q] = a | (atomicAdd(&cnt[a], live ? 1u : 0u) << 16);
      }
    }
  }
  __syncthreads();
  // 2. scan: thread tid owns buckets [kPer tid, kPer tid + kPer), contiguous
  // words from bpad(kPer tid)
  if (kLazyZero) {
    if (tid < 24) keys[n + tid] = 0xFFFFFFFFu;
    if (tid == 0) sm.scr[kScrDups] = 0;
  }
  {
    uint32_t* run8 = cnt + bpad(kPer * tid);
    uint32_t c[kPer];
    uint32_t run = 0, big = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      c[k] = run8[k];
      run += c[k];
      big = max(big, c[k]);
    }
    big = wave_max_incl(big);
    if ((tid & 63) == 63) sm.scr[kScrMax + (tid >> 6)] = big;
    uint32_t total;
    uint32_t acc = block_scan_excl<B, uint32_t, false>(run, sm.scr, &total);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      run8[k] = acc;
      acc += c[k];
    }
    if (tid == 0) cnt[kSpareCount] = kSpareSlot;
  }
  __syncthreads();
  uint32_t cmax = 0;
#pragma unroll
  for (int w = 0; w < B / 64; ++w) cmax = max(cmax, sm.scr[kScrMax + w]);
  // 3. scatter in bucket order (unused positions land on the spare slot)
#pragma unroll
  for (int k = 0; k < kBlk; ++k) {
    if (kMasked) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = 4 * k + j;
        if (as[q] != kDeadKey) keys[cnt[as[q] & 0xFFFFu] + (as[q] >> 16)] = key[q];
      }
    } else if (4 * (wave_first + k * B) < n) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = 4 * k + j;
        keys[cnt[as[q] & 0xFFFFu] + (as[q] >> 16)] = key[q];
      }
    }
  }
  __syncthreads();
  // 4. order inside buckets
  if (shift == 0 || cmax <= 1) {
    if (kLazyZero) {
      zero_counters<B>(cnt, tid);
      __syncthreads();
    }
    return (shift == 0 && cmax >= 2) ? 1u : 0u;
  }
  if (kLazyZero) zero_counters<B>(cnt, tid);  // read for the last time in the scatter
  if (cmax <= 9) {
    uint64_t dup;
    // the second pass's windows are two sorted halves of first-pass windows
    if (cmax <= 5) {
      dup = window_pass<B, 8, false>(keys, n, 0, tid);
      __syncthreads();
      dup |= window_pass<B, 8, true>(keys, n, 4, tid);
    } else {
      dup = window_pass<B, 16, false>(keys, n, 0, tid);
      __syncthreads();
      dup |= window_pass<B, 16, true>(keys, n, 8, tid);
    }
    // lanes of a wave may hold ballots of different branches: any of them sets it
    if (dup) sm.scr[kScrDups] = 1;
    __syncthreads();
    return sm.scr[kScrDups];
  }
  for (uint32_t r = 0; r < cmax; ++r) {
    const uint32_t odd = r & 1u;
#pragma unroll
    for (int m = 0; m < kPairs; ++m) {
      const uint32_t i = 2 * (tid + m * B) + odd;
      if (i + 1 < n) {
        const uint32_t a = keys[i], b = keys[i + 1];
        keys[i] = min(a, b);
        keys[i + 1] = max(a, b);
      }
    }
    __syncthreads();
  }
  uint32_t dup = 0;
#pragma unroll
  for (int m = 0; m < kPairs; ++m) {
    const uint32_t i = 2 * (tid + m * B);
    if (i + 1 < n) {
      const uint32_t a = keys[i], b = keys[i + 1];
      dup |= a == b ? 1u : 0u;
      if (i + 2 < n) dup |= b == keys[i + 2] ? 1u : 0u;
    }
  }
  if (dup) sm.scr[kScrDups] = 1;
  __syncthreads();
  return sm.scr[kScrDups];
}

// Registers <- keys[0..n) in the layout sort_registers expects.
template <int B>
__device__ __forceinline__ void load_registers(uint32_t (&key)[kKeys / B], const uint32_t* keys,
                                               uint32_t n) {
  constexpr int kBlk = kKeys / (4 * B);
  const uint32_t nblk = (n + 3) >> 2;
#pragma unroll
  for (int k = 0; k < kBlk; ++k) {
    const uint32_t blk = threadIdx.x + k * B;
    if (blk < nblk) {
      const uint4 v = reinterpret_cast<const uint4*>(keys)[blk];
      key[4 * k + 0] = v.x;
      key[4 * k + 1] = v.y;
      key[4 * k + 2] = v.z;
      key[4 * k + 3] = v.w;
    }
  }
}

// keys[0..n) ascending with equal values adjacent -> the distinct values in
// keys[0..d); returns d.
template <int B>
__device__ uint32_t compact_distinct(uint32_t* keys, uint32_t* tmp, uint32_t* scr, uint32_t n) {
  constexpr int R = kKeys / B;
  const uint32_t tid = threadIdx.x;
  // contiguous runs per thread keep the scan order equal to index order
  const uint32_t per = (n + B - 1) / B;
  const uint32_t i0 = tid * per;
  uint32_t c = 0;
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t i = i0 + k;
    if (i < n && (i == 0 || keys[i] != keys[i - 1])) ++c;
  }
  uint32_t total;
  uint32_t p = block_scan_excl<B, uint32_t>(c, scr, &total);
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t i = i0 + k;
    if (i < n && (i == 0 || keys[i] != keys[i - 1])) tmp[p++] = keys[i];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = tid + r * B;
    if (i < total) keys[i] = tmp[i];
  }
  __syncthreads();
  return total;
}

// out[i] = base + 1 + vals[i] for i < n, coalesced.
template <int B>
__device__ __forceinline__ void write_sorted(uint64_t* out, uint64_t base, const uint32_t* vals,
                                             uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += B)
    store_out(out + i, base + 1 + static_cast<uint64_t>(vals[i]));
}

// Buckets for keys < range: the top 12 of the key's kb = bits(range - 1)
// bits (all of them when kb <= 12), at most 4096 buckets.
__device__ __forceinline__ void bucket_params(uint64_t range, uint32_t n, uint32_t* shift,
                                              uint32_t* nb) {
  (void)n;
  const uint32_t kb = bit_length(range - 1);
  constexpr uint32_t lb = 12;
  *shift = kb > lb ? kb - lb : 0u;
  *nb = static_cast<uint32_t>(((range - 1) >> *shift) + 1);
}


// out[i] = base + 1 + vals[i] for i < n with 16-byte stores where the
// destination allows (out is 8-byte aligned; pairs start at an even index of
// the destination).
template <int B>
__device__ __forceinline__ void write_sorted_pairs(uint64_t* out, uint64_t base,
                                                   const uint32_t* vals, uint32_t n) {
  const uint32_t s0 = static_cast<uint32_t>((reinterpret_cast<uintptr_t>(out) >> 3) & 1u);
  const uint64_t b1 = base + 1;
  const uint32_t tid = lane_tid();
  if (s0 && tid == 0 && n > 0) store_out(out, b1 + vals[0]);
  for (uint32_t e = s0 + 2 * tid; e < n; e += 2 * B) {
    if (e + 1 < n) {
      u64x2 pr;
      pr.x = b1 + vals[e];
      pr.y = b1 + vals[e + 1];
      __builtin_nontemporal_store(pr, reinterpret_cast<u64x2*>(out + e));
    } else {
      store_out(out + e, b1 + vals[e]);
    }
  }
}


// ---------------------------------------------------------------------------
// Sparse leaf: Algorithm H semantics, computed in rounds.
// ---------------------------------------------------------------------------
// Rounds after the first: keys[0..have) hold distinct values; draw the next
// (nv - have) non-void values from word t on, sort, repeat while values repeat.
template <int B, bool kLazyZero = false>
__device__ void sparse_rounds(const Stream& st, uint64_t t, uint32_t have, uint32_t nv,
                              const RangeInfo& ri, uint32_t shift, uint32_t nb, LeafSmem& sm) {
  uint32_t* keys = sm.keys;
  uint32_t key[kKeys / B];
  for (;;) {
    const uint32_t base = have;
    t = take_values<B>(st, t, nv - have, ri, sm.scr,
                       [&](uint32_t p, uint32_t v) { keys[base + p] = v; });
    load_registers<B>(key, keys, nv);
    __syncthreads();
    if (sort_registers<B, kLazyZero>(key, nv, shift, nb, sm) == 0) return;
    have = compact_distinct<B>(keys, sm.tmp, sm.scr, nv);
  }
}

// First round of a sparse or with-replacement leaf over a range that is not a
// power of two, in registers: the words t < W of the stream mapped into
// [0, N_v), W = n_v plus twice the expected number of void words among n_v,
// plus 32 (at most 4096); the first
// n_v non-void values in stream order are the live keys (bit q of *live for
// key[q]), ranked by one block scan.  Returns how many of the W words are
// non-void (below n_v the caller takes the LDS rounds instead); when it is at
// least n_v, sm.scr[kScrNext] holds the word index just after the n_v-th
// value once a barrier has passed.
template <int B>
__device__ uint32_t first_round_regs(const Stream& st, uint32_t nv, const RangeInfo& ri,
                                     uint32_t (&key)[kKeys / B], uint32_t* live, LeafSmem& sm) {
  constexpr int kBlk = kKeys / (4 * B);
  static_assert(kBlk == 2, "two 16-bit counts share one scanned word");
  const uint32_t tid = lane_tid();
  const uint64_t extra = ((2ull * nv * ri.thr) >> 32) + 32u;
  const uint32_t W = nv + extra < kKeys ? nv + static_cast<uint32_t>(extra) : kKeys;
  const uint32_t nblk = (W + 3) >> 2;
  uint32_t ok = 0;
#pragma unroll
  for (int k = 0; k < kBlk; ++k) {
    const uint32_t blk = tid + k * B;
#pragma unroll
    for (int j = 0; j < 4; ++j) key[4 * k + j] = 0;
    if (blk < nblk) {
      const uint4 w = philox_block(st, blk);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint32_t v;
        const bool good = range_map(pick(w, j), ri.s, ri.thr, &v);
        key[4 * k + j] = v;
        if (good && 4 * blk + j < W) ok |= 1u << (4 * k + j);
      }
    }
  }
  uint32_t total;
  const uint32_t packed = static_cast<uint32_t>(__popc(ok & 0xFu)) |
                          (static_cast<uint32_t>(__popc(ok >> 4)) << 16);
  const uint32_t excl = block_scan_excl<B, uint32_t>(packed, sm.scr, &total);
  const uint32_t total0 = total & 0xFFFFu;
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < kBlk; ++k) {
    const uint32_t base = k == 0 ? (excl & 0xFFFFu) : total0 + (excl >> 16);
    const uint32_t okk = (ok >> (4 * k)) & 0xFu;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t rank = base + static_cast<uint32_t>(__popc(okk & ((1u << j) - 1u)));
      if (((okk >> j) & 1u) && rank < nv) {
        m |= 1u << (4 * k + j);
        if (rank == nv - 1) sm.scr[kScrNext] = 4 * (tid + k * B) + j + 1;
      }
    }
  }
  *live = m;
  return total0 + (total >> 16);
}

// A sparse leaf whose first n_v values are expected to repeat (n_v^2 / (2 N_v)
// of at least one; see once_by_group): one pass over the first W words
// instead of repeat rounds.  W covers n_v plus margins for void words and for repeats
// (at most 4096).  Every non-void value among them is counted into its bucket
// and ranked inside the bucket by (value, word index); a value whose bucket
// holds the same value at a smaller word index repeats an earlier one.  The
// words that are first occurrences, in stream order, give the first n_v
// distinct values (Algorithm H's set); their bucket ranks are their sorted
// positions among all W words, and a scan over the positions of the kept
// ones compacts them.  When fewer than n_v distinct values occur among the W
// words, those values are sorted and the repeat rounds continue from word W.
// Returns where the sorted sample lies (sm.tmp, or sm.keys after rounds).
template <int B>
__device__ const uint32_t* leaf_sparse_once(const Stream& st, uint32_t nv, const RangeInfo& ri,
                                 uint32_t shift, uint32_t nb, LeafSmem& sm) {
  constexpr int kBlk = kKeys / (4 * B);
  constexpr int kQ = 4 * kBlk;
  constexpr int kPer = kBuckets / B;
  static_assert(kBlk == 2, "two 16-bit counts share one scanned word");
  static_assert(kPer * B == kKeys && kPer == 8, "one byte of the position bitmap per thread");
  const uint32_t tid = lane_tid();
  uint32_t* cnt = sm.buck;
  uint32_t* keys = sm.keys;
  uint16_t* widx = reinterpret_cast<uint16_t*>(sm.tmp);  // word index by bucket position
  zero_counters<B>(cnt, tid);
  // W: n_v, the expected repeats r with a margin, and twice the expected void
  // words plus 32
  const uint64_t r = (static_cast<uint64_t>(nv) * nv) / (2 * ri.s);
  const uint64_t base = nv + r + (r >> 2) + 4 * isqrt64(r) + 16;
  const uint64_t full = base + ((2 * base * ri.thr) >> 32) + 32;
  const uint32_t W = full < kKeys ? static_cast<uint32_t>(full) : kKeys;
  const uint32_t nblk = (W + 3) >> 2;
  uint32_t key[kQ];
  uint32_t ok = 0;
#pragma unroll
  for (int k = 0; k < kBlk; ++k) {
    const uint32_t blk = tid + k * B;
#pragma unroll
    for (int j = 0; j < 4; ++j) key[4 * k + j] = 0;
    if (blk < nblk) {
      const uint4 w = philox_block(st, blk);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint32_t v;
        const bool good = range_map(pick(w, j), ri.s, ri.thr, &v);
        key[4 * k + j] = v;
        if (good && 4 * blk + j < W) ok |= 1u << (4 * k + j);
      }
    }
  }
  __syncthreads();
  // 1. count into buckets; each key keeps its counter index | slot << 16
  uint32_t as[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    as[q] = 0;
    if ((ok >> q) & 1u) {
      const uint32_t a = bpad(key[q] >> shift);
      as[q] = a | (atomicAdd(&cnt[a], 1u) << 16);
    }
  }
  __syncthreads();
  // 2. exclusive scan of the counts; the word after the last bucket holds the
  // total, the end of the last bucket
  {
    uint32_t* run8 = cnt + bpad(kPer * tid);
    uint32_t c[kPer];
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      c[k] = run8[k];
      run += c[k];
    }
    uint32_t total;
    uint32_t acc = block_scan_excl<B, uint32_t, false>(run, sm.scr, &total);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      run8[k] = acc;
      acc += c[k];
    }
    if (tid == 0) cnt[kSpareCount] = total;
  }
  __syncthreads();
  // 3. scatter values and word indices in bucket order; each key keeps its
  // bucket's start | count << 13 | min(slot, 4) << 26
#pragma unroll
  for (int k = 0; k < kBlk; ++k) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = 4 * k + j;
      if ((ok >> q) & 1u) {
        const uint32_t a = as[q] & 0xFFFFu;
        const uint32_t b = key[q] >> shift;
        const uint32_t s0 = cnt[a], e0 = cnt[bpad(b + 1)];
        const uint32_t slot = as[q] >> 16;
        const uint32_t p = s0 + slot;
        keys[p] = key[q];
        widx[p] = static_cast<uint16_t>(4 * (tid + k * B) + j);
        as[q] = s0 | ((e0 - s0) << 13) | (min(slot, 4u) << 26);
      }
    }
  }
  __syncthreads();
  // the counters are dead from here on: region B's first words become the
  // bitmap of kept sorted positions (cleared before the scan's barrier below)
  uint32_t* kept_bits = cnt;
  if (tid < kKeys / 32) kept_bits[tid] = 0;
  // 4. rank inside the bucket by (value, word index); each key's register
  // then holds its sorted position among the W words.  A bucket's first four
  // entries are read at once (the words past a bucket's end lie inside region
  // A and are ignored); larger buckets continue one entry at a time.
  uint32_t rep = 0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    if ((ok >> q) & 1u) {
      const uint32_t s0 = as[q] & 0x1FFFu, c = (as[q] >> 13) & 0x1FFFu, self = as[q] >> 26;
      const uint32_t t = 4 * (tid + (q >> 2) * B) + (q & 3);
      uint32_t rk = 0, eq = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t v = keys[s0 + u];
        const bool in = static_cast<uint32_t>(u) < c;
        rk += (in && v < key[q]) ? 1u : 0u;
        eq |= (in && v == key[q]) ? (1u << u) : 0u;
      }
      for (uint32_t i = s0 + 4; i < s0 + c; ++i) {
        const uint32_t v = keys[i];
        rk += v < key[q] ? 1u : 0u;
        if (v == key[q] && widx[i] < t) {
          ++rk;
          rep |= 1u << q;
        }
      }
      eq &= ~(1u << self);  // self < 4: its own entry; self = 4: none of the four
      if (eq != 0) {        // the value occurs again among the first four
        for (uint32_t m = eq; m != 0; m &= m - 1u) {
          const uint32_t i = s0 + static_cast<uint32_t>(__ffs(m) - 1);
          if (widx[i] < t) {
            ++rk;
            rep |= 1u << q;
          }
        }
      }
      as[q] = s0 + rk;
    }
  }
  // 5. first occurrences in stream order: the first n_v of them are kept
  const uint32_t first = ok & ~rep;
  uint32_t total;
  const uint32_t packed = static_cast<uint32_t>(__popc(first & 0xFu)) |
                          (static_cast<uint32_t>(__popc(first >> 4)) << 16);
  const uint32_t excl = block_scan_excl<B, uint32_t>(packed, sm.scr, &total);
  const uint32_t total0 = total & 0xFFFFu;
  const uint32_t distinct = total0 + (total >> 16);
  const uint32_t take = distinct < nv ? distinct : nv;
  // 6. kept values to their sorted positions (every read of the bucket-order
  // arrays is behind the scan's barriers)
#pragma unroll
  for (int k = 0; k < kBlk; ++k) {
    const uint32_t b0 = k == 0 ? (excl & 0xFFFFu) : total0 + (excl >> 16);
    const uint32_t fk = (first >> (4 * k)) & 0xFu;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = 4 * k + j;
      const uint32_t sr = b0 + static_cast<uint32_t>(__popc(fk & ((1u << j) - 1u)));
      if (((fk >> j) & 1u) && sr < take) {
        const uint32_t p = as[q];
        keys[p] = key[q];
        atomicOr(&kept_bits[p >> 5], 1u << (p & 31u));
      }
    }
  }
  __syncthreads();
  // 7. compact the kept positions in order into sm.tmp
  const uint32_t byte = (kept_bits[tid >> 2] >> (8 * (tid & 3u))) & 0xFFu;
  uint32_t unused;
  uint32_t o = block_scan_excl<B, uint32_t>(static_cast<uint32_t>(__popc(byte)), sm.scr, &unused);
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if ((byte >> j) & 1u) sm.tmp[o++] = keys[8 * tid + j];
  __syncthreads();
  if (take == nv) return sm.tmp;
  // fewer than n_v distinct values among the W words: they are the rounds'
  // starting set, and the rounds continue from word W
  for (uint32_t i = tid; i < take; i += B) keys[i] = sm.tmp[i];
  __syncthreads();
  sparse_rounds<B>(st, W, take, nv, ri, shift, nb, sm);
  return keys;
}

template <int B>
__device__ void leaf_sparse(const Leaf& L, uint64_t* out, LeafSmem& sm) {
  const uint32_t nv = L.nv;
  if (nv == 0) return;
  const RangeInfo ri = range_info(L.Nv);
  uint32_t shift, nb;
  bucket_params(L.Nv, nv, &shift, &nb);
  const Stream st = make_stream(L.seed, L.id, kLeaf, 0);
  uint32_t key[kKeys / B];
  uint32_t live;
  const uint32_t got = first_round_regs<B>(st, nv, ri, key, &live, sm);
  __builtin_amdgcn_s_setprio(2);  // the sort and its rounds ahead of other work-groups
  if (got >= nv) {
    if (sort_registers<B, false, true>(key, nv, shift, nb, sm, live) != 0) {
      const uint64_t t = sm.scr[kScrNext];
      const uint32_t have = compact_distinct<B>(sm.keys, sm.tmp, sm.scr, nv);
      sparse_rounds<B>(st, t, have, nv, ri, shift, nb, sm);
    }
  } else {
    // too many void words among the first W: the general rounds from word 0
    sparse_rounds<B>(st, 0, 0, nv, ri, shift, nb, sm);
  }
  __builtin_amdgcn_s_setprio(0);
  write_sorted_pairs<B>(out + L.off, L.lo, sm.keys, nv);
}

// Sparse leaves of more than kSmallMax values whose first n_v values are
// expected to repeat (n_v^2 >= 2 N_v, any range) run in k_leaf_once, in one
// pass; k_leaf_mixed skips them, so that its own leaf bodies keep their
// registers.
template <int B>
__device__ void leaf_once(const Leaf& L, uint64_t* out, LeafSmem& sm) {
  const uint32_t nv = L.nv;
  const RangeInfo ri = range_info(L.Nv);
  uint32_t shift, nb;
  bucket_params(L.Nv, nv, &shift, &nb);
  const Stream st = make_stream(L.seed, L.id, kLeaf, 0);
  __builtin_amdgcn_s_setprio(2);  // the passes ahead of other work-groups
  const uint32_t* sorted = leaf_sparse_once<B>(st, nv, ri, shift, nb, sm);
  __builtin_amdgcn_s_setprio(0);
  write_sorted_pairs<B>(out + L.off, L.lo, sorted, nv);
}

// Sparse or with-replacement leaf on a power-of-two range (no word is void):
// the first round's n_v words go from Philox straight into registers; for a
// sparse leaf the general rounds take over only if a value repeats (a
// with-replacement leaf keeps repeats).
template <int B>
__device__ void leaf_sparse_pow2(const Leaf& L, uint64_t* out, LeafSmem& sm) {
  constexpr int kBlk = kKeys / (4 * B);
  const uint32_t tid = lane_tid();
  const uint32_t nv = L.nv;
  const uint32_t kb = bit_length(L.Nv) - 1;        // range = 2^kb, 1 <= kb <= 32
  const uint32_t pshift = 32u - kb;                 // value = word >> pshift
  uint32_t shift, nb;
  bucket_params(L.Nv, nv, &shift, &nb);
  const bool wr = (L.flags & 3u) == kKindWr;
  const Stream st = make_stream(L.seed, L.id, wr ? kWrLeaf : kLeaf, 0);
  const uint32_t nblk = (nv + 3) >> 2;
  uint32_t key[kKeys / B];
#pragma unroll
  for (int k = 0; k < kBlk; ++k) {
    const uint32_t blk = tid + k * B;  // tid is opaque: no Philox round is hoisted
    if (blk < nblk) {
      const uint4 w = philox_block(st, blk);
      key[4 * k + 0] = w.x >> pshift;
      key[4 * k + 1] = w.y >> pshift;
      key[4 * k + 2] = w.z >> pshift;
      key[4 * k + 3] = w.w >> pshift;
    }
  }
  // The sort is a chain of barrier-separated LDS phases; at raised issue
  // priority its waves go ahead of other work-groups' Philox and store
  // instructions, so a work-group spends less time waiting at its barriers
  // (the stores and the next leaf's draws fill the gaps).
  __builtin_amdgcn_s_setprio(2);
  const uint32_t dups = sort_registers<B, true>(key, nv, shift, nb, sm);
  __builtin_amdgcn_s_setprio(0);
  if (dups != 0 && !wr) {
    const uint32_t have = compact_distinct<B>(sm.keys, sm.tmp, sm.scr, nv);
    sparse_rounds<B, true>(st, nv, have, nv, range_info(L.Nv), shift, nb, sm);
  }
  write_sorted_pairs<B>(out + L.off, L.lo, sm.keys, nv);
}

// With-replacement leaf: the first n_v non-void draws, sorted, repeats kept.
template <int B>
__device__ void leaf_wr(const Leaf& L, uint64_t* out, LeafSmem& sm) {
  const uint32_t nv = L.nv;
  if (nv == 0) return;
  const RangeInfo ri = range_info(L.Nv);
  uint32_t shift, nb;
  bucket_params(L.Nv, nv, &shift, &nb);
  const Stream st = make_stream(L.seed, L.id, kWrLeaf, 0);
  uint32_t key[kKeys / B];
  uint32_t live;
  const uint32_t got = first_round_regs<B>(st, nv, ri, key, &live, sm);
  __builtin_amdgcn_s_setprio(2);  // the sort ahead of other work-groups
  if (got >= nv) {
    sort_registers<B, false, true>(key, nv, shift, nb, sm, live);
  } else {
    uint32_t* keys = sm.keys;
    take_values<B>(st, 0, nv, ri, sm.scr, [&](uint32_t p, uint32_t v) { keys[p] = v; });
    load_registers<B>(key, keys, nv);
    __syncthreads();
    sort_registers<B>(key, nv, shift, nb, sm);
  }
  __builtin_amdgcn_s_setprio(0);
  write_sorted_pairs<B>(out + L.off, L.lo, sm.keys, nv);
}

// ---------------------------------------------------------------------------
// Dense leaf: Algorithm B with geometric skips and repair.
// ---------------------------------------------------------------------------
template <int B>
__device__ void leaf_dense(const Leaf& L, uint64_t* out, LeafSmem& sm) {
  const uint32_t tid = lane_tid();
  const uint32_t nv = L.nv;
  const uint32_t Nv = static_cast<uint32_t>(L.Nv);  // < 64 * 4096 here
  const uint32_t n0 = L.flags >> 8;
  const uint32_t rho_num = nv + 3u * static_cast<uint32_t>(isqrt64(nv)) + 8u;
  const bool full = rho_num >= Nv;
  float cg = 0.0f;
  if (!full) {
    const float rho = static_cast<float>(rho_num) / static_cast<float>(Nv);
    cg = static_cast<float>(1.0 / log64(1.0 - static_cast<double>(rho)));
  }
  const uint32_t cap = 2u * n0 + 64u;
  uint32_t* pos = sm.keys;  // region A: up to kDenseCap + 1 positions
  for (uint32_t attempt = 0;; ++attempt) {
    uint32_t hits;  // n'
    if (full) {
      hits = Nv;
    } else {
      // Hit k sits at 0-based position q_k - 1, q_k = sum_{i<=k} (skip_i + 1);
      // each round takes 4 draws per thread in stream order and one scan.
      // A skip is below 2^24 and Nv + round sums stay far below 2^32.
      const Stream st = make_stream(L.seed, L.id, kBern, attempt);
      uint32_t last = 0;  // q of the previous round's last draw
      uint32_t count = 0;
      for (uint32_t blk0 = 0;; blk0 += B) {
        const uint4 w = philox_block(st, blk0 + tid);
        uint32_t inc[4];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          inc[j] = static_cast<uint32_t>(geom_skip32(pick(w, j), cg)) + 1u;
          sum += inc[j];
        }
        uint32_t total;
        const uint32_t q0 = last + block_scan_excl<B, uint32_t>(sum, sm.scr, &total);
        uint32_t q = q0, in = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          q += inc[j];
          if (q <= Nv) {
            ++in;
            const uint32_t idx = count + 4u * tid + j;  // stream index = hit index
            if (idx <= cap) pos[idx] = q - 1;
          }
        }
        if (last + total <= Nv) {  // every draw of the round is a hit
          count += 4u * B;
          last += total;
          if (count > cap) break;
          continue;
        }
        // hits are a prefix of the round: the one thread that starts in range
        // and holds the first miss reports how many
        if (in < 4 && q0 <= Nv) sm.scr[kScrNext] = 4u * tid + in;
        __syncthreads();
        count += sm.scr[kScrNext];
        __syncthreads();
        break;
      }
      hits = count;
      if (hits < nv || hits > cap) continue;
    }
    // Repair: remove the first (hits - nv) distinct values of the REPAIR
    // stream mapped into [0, hits); a value counts when its bit was clear.
    const uint32_t r = hits - nv;
    const uint32_t mwords = (hits + 31) / 32;
    for (uint32_t i = tid; i < mwords; i += B) sm.mask[i] = 0;
    if (tid == 0) sm.scr[kScrDups] = 0;
    __syncthreads();
    if (r > 0) {
      const Stream sr = make_stream(L.seed, L.id, kRepair, attempt);
      const RangeInfo ri = range_info(hits);
      uint64_t t = 0;
      for (uint32_t have = 0; have < r;) {
        t = take_values<B>(sr, t, r - have, ri, sm.scr, [&](uint32_t, uint32_t v) {
          const uint32_t bit = 1u << (v & 31);
          if (!(atomicOr(&sm.mask[v >> 5], bit) & bit)) atomicAdd(&sm.scr[kScrDups], 1u);
        });
        have = sm.scr[kScrDups];  // take_values ends with a barrier
        __syncthreads();
      }
    }
    // Compact the kept hits (ascending position) into kept[0..nv).
    const uint32_t per = (hits + B - 1) / B;
    const uint32_t i0 = tid * per;
    uint32_t c = 0;
    for (uint32_t k = 0; k < per; ++k) {
      const uint32_t i = i0 + k;
      if (i < hits && !((sm.mask[i >> 5] >> (i & 31)) & 1u)) ++c;
    }
    uint32_t total;
    uint32_t o = block_scan_excl<B, uint32_t>(c, sm.scr, &total);
    for (uint32_t k = 0; k < per; ++k) {
      const uint32_t i = i0 + k;
      if (i < hits && !((sm.mask[i >> 5] >> (i & 31)) & 1u)) sm.kept[o++] = full ? i : pos[i];
    }
    __syncthreads();
    write_sorted_pairs<B>(out + L.off, L.lo, sm.kept, nv);
    break;
  }
}

// ---------------------------------------------------------------------------
// Dense leaf, one wave per leaf (same sample as leaf_dense).
// ---------------------------------------------------------------------------
// Leaves whose range fits 16-bit positions are taken by k_leaf_dense, one
// wave each with no barrier; the work-group leaf loop skips them.  With the
// default dense ratio (16) and n0 <= 4096 that is every dense leaf.
constexpr uint32_t kWaveMaxRange = 1u << 16;
constexpr uint32_t kWaveChunk = 256;                             // draws per chunk
constexpr uint32_t kWaveListChunks = 17;                         // chunks kept in LDS
constexpr uint32_t kWaveList = kWaveChunk * kWaveListChunks;     // 4352 positions
constexpr uint32_t kWaveMaskWords = (kDenseCap + 1 + 31) / 32 + 1;
constexpr uint32_t kWaveBases = kDenseCap / kWaveChunk + 2;

__device__ __forceinline__ bool dense_by_wave(const Leaf& L) {
  return (L.flags & 3u) == kKindDense && L.Nv <= kWaveMaxRange;
}

__device__ __forceinline__ uint32_t lane_rank(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

// Chunk c of the skip stream: lane l holds draws 256c + 4l + j (j < 4), the
// words of Philox block 64c + l.  On return q[j] is the 1-based position
// reached after draw j (the hit, if q[j] <= Nv, sits at q[j] - 1) and the
// result is the chunk's total advance.
__device__ __forceinline__ uint32_t skip_chunk(const Stream& st, uint32_t c, uint32_t lane,
                                               float cg, uint32_t q_base, uint32_t q[4]) {
  const uint4 w = philox_block(st, c * (kWaveChunk / 4) + lane);
  uint32_t inc[4];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    inc[j] = static_cast<uint32_t>(geom_skip32(pick(w, j), cg)) + 1u;
    sum += inc[j];
  }
  const uint32_t incl = wave_scan_incl(sum);
  uint32_t x = q_base + incl - sum;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    x += inc[j];
    q[j] = x;
  }
  return __builtin_amdgcn_readlane(incl, 63);
}

// The chunk's four positions q[j] - 1 as 16-bit values (entries past the
// last hit are never read).
__device__ __forceinline__ void put_chunk(uint16_t* dst, const uint32_t q[4]) {
  uint2 v;
  v.x = ((q[0] - 1u) & 0xFFFFu) | ((q[1] - 1u) << 16);
  v.y = ((q[2] - 1u) & 0xFFFFu) | ((q[3] - 1u) << 16);
  *reinterpret_cast<uint2*>(dst) = v;
}

// One wave samples one dense leaf (Algorithm B, Sec. 2, with geometric skips,
// Sec. 4.7): hit positions as 16-bit values (chunks beyond kWaveListChunks
// are recomputed from their start position when they are written out), the
// repair's removed hit indices as a bit mask, and the kept hits written with
// consecutive lanes on consecutive outputs.
__device__ void leaf_dense_wave(const Leaf& L, uint64_t* out, uint16_t* list, uint32_t* mask,
                                uint32_t* bases) {
  const uint32_t lane = lane_tid();
  const uint32_t nv = L.nv;
  const uint32_t Nv = static_cast<uint32_t>(L.Nv);
  const uint32_t n0 = L.flags >> 8;
  const uint32_t rho_num = nv + 3u * static_cast<uint32_t>(isqrt64(nv)) + 8u;
  const bool full = rho_num >= Nv;
  float cg = 0.0f;
  if (!full) {
    const float rho = static_cast<float>(rho_num) / static_cast<float>(Nv);
    cg = static_cast<float>(1.0 / log64(1.0 - static_cast<double>(rho)));
  }
  const uint32_t cap = 2u * n0 + 64u;
  for (uint32_t attempt = 0;; ++attempt) {
    const Stream st = make_stream(L.seed, L.id, kBern, attempt);
    uint32_t cnt = 0;  // n'
    if (full) {
      cnt = Nv;
    } else {
      uint32_t q_base = 0;
      for (uint32_t c = 0;; ++c) {
        uint32_t q[4];
        if (lane == 0) bases[c] = q_base;
        const uint32_t adv = skip_chunk(st, c, lane, cg, q_base, q);
        uint32_t in = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) in += q[j] <= Nv ? 1u : 0u;
        if (c < kWaveListChunks) put_chunk(list + c * kWaveChunk + 4u * lane, q);
        // hits are a prefix of the chunk: whole lanes, then one partial lane
        const unsigned long long whole = __ballot(in == 4u);
        const uint32_t nw = static_cast<uint32_t>(__popcll(whole));
        const uint32_t got =
            nw == 64u ? kWaveChunk : 4u * nw + __builtin_amdgcn_readlane(in, nw);
        cnt += got;
        q_base += adv;
        if (got < kWaveChunk || cnt > cap) break;
      }
      if (cnt < nv || cnt > cap) continue;
    }
    // Repair: remove the first (cnt - nv) distinct values of the REPAIR
    // stream mapped into [0, cnt).  Words are taken 64 at a time in stream
    // order (lane m holds word 64 j + m of a 256-word Philox round), so the
    // r-th new value is found with a ballot.
    const uint32_t r = cnt - nv;
    const uint32_t mwords = (cnt + 31u) / 32u;
    for (uint32_t i = lane; i < mwords; i += 64u) mask[i] = 0u;
    if (r > 0) {
      const Stream sr = make_stream(L.seed, L.id, kRepair, attempt);
      const uint32_t thr = range_threshold(cnt);
      uint32_t have = 0;
      for (uint32_t it = 0; have < r; ++it) {
        const uint4 w4 = philox_block(sr, it * 64u + lane);
        for (uint32_t j = 0; j < 4u && have < r; ++j) {
          const int src = static_cast<int>(16u * j + (lane >> 2));
          const uint32_t x0 = __shfl(w4.x, src), x1 = __shfl(w4.y, src);
          const uint32_t x2 = __shfl(w4.z, src), x3 = __shfl(w4.w, src);
          const uint32_t cmp = lane & 3u;
          const uint32_t word = cmp == 0 ? x0 : (cmp == 1 ? x1 : (cmp == 2 ? x2 : x3));
          uint32_t v;
          const bool ok = range_map(word, cnt, thr, &v);
          const uint32_t bit = 1u << (v & 31u);
          uint32_t* mw = mask + (v >> 5);
          const bool fresh = ok && !(*mw & bit);
          const uint32_t old = fresh ? atomicOr(mw, bit) : 0u;
          // equal fresh values in one step: the lowest lane is the first
          unsigned long long raced = __ballot(fresh && (old & bit));
          bool later = false;
          while (raced) {
            const uint32_t s = static_cast<uint32_t>(__ffsll(static_cast<long long>(raced)) - 1);
            const uint32_t vs = __builtin_amdgcn_readlane(v, s);
            const unsigned long long same = __ballot(fresh && v == vs);
            const uint32_t first = static_cast<uint32_t>(__ffsll(static_cast<long long>(same)) - 1);
            later = later || (fresh && v == vs && lane != first);
            raced &= ~same;
          }
          const bool firsts = fresh && !later;
          const unsigned long long F = __ballot(firsts);
          const uint32_t need = r - have;
          // values past the r-th are not removed: take their bits back
          if (firsts && lane_rank(F) >= need) atomicAnd(mw, ~bit);
          const uint32_t nf = static_cast<uint32_t>(__popcll(F));
          have += nf < need ? nf : need;
        }
      }
    }
    // Kept hits in order, consecutive lanes on consecutive outputs (exactly
    // nv of them; the bound only keeps the stores inside the leaf's part).
    uint64_t* const o0 = out + L.off;
    uint32_t done = 0;
    const uint64_t b1 = L.lo + 1;
    constexpr uint32_t kSpare = (kWaveListChunks - 1) * kWaveChunk;  // recomputed chunks
    // One chunk per step: lane l takes hits k0 + 64s + l (s < 4), so the
    // chunk's LDS reads issue together.
    for (uint32_t k0 = 0; k0 < cnt; k0 += kWaveChunk) {
      const uint32_t c = k0 / kWaveChunk;
      uint32_t sbase = k0;  // list index of hit k0
      if (!full && c >= kWaveListChunks) {
        uint32_t q[4];
        skip_chunk(st, c, lane, cg, bases[c], q);
        put_chunk(list + kSpare + 4u * lane, q);
        sbase = kSpare;
      }
      uint32_t pos[4], rm[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint32_t k = k0 + 64u * t + lane;
        // every index stays inside the list and the mask; values past the
        // last hit are read but never stored
        pos[t] = full ? k : static_cast<uint32_t>(list[sbase + 64u * t + lane]);
        const uint32_t w = k >> 5;
        rm[t] = mask[w < kWaveMaskWords ? w : kWaveMaskWords - 1];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint32_t k = k0 + 64u * t + lane;
        const bool kept = k < cnt && !((rm[t] >> (k & 31u)) & 1u);
        const unsigned long long K = __ballot(kept);
        const uint32_t at = done + lane_rank(K);
        if (kept && at < nv) store_out(o0 + at, b1 + pos[t]);
        done += static_cast<uint32_t>(__popcll(K));
      }
    }
    break;
  }
}

// Constant leaf of a with-replacement tree: N_v = 1, every draw is lo+1.
// ---------------------------------------------------------------------------
// Small sparse and with-replacement leaves, one wave per leaf.
// ---------------------------------------------------------------------------
// Sparse and with-replacement leaves of the back list (ranges that are not
// powers of two) with at most kSmallMax values are taken by k_leaf_small,
// one wave each with no barrier: the same values as leaf_sparse / leaf_wr
// (the first n_v non-void values of the leaf's stream, for a sparse leaf
// Algorithm H's distinct ones by rounds), ranked in stream order by wave
// scans, sorted by a counting pass over kSmallBuckets buckets and the
// Batcher windows, and written with consecutive lanes on consecutive
// outputs.  The work-group leaf loop skips them.
constexpr uint32_t kSmallKpl = 16;                     // keys per lane
constexpr uint32_t kSmallMax = 64 * kSmallKpl;         // 1024 values
constexpr uint32_t kSmallBucketBits = 10;
constexpr uint32_t kSmallBuckets = 1u << kSmallBucketBits;
static_assert(kSmallBuckets == kSmallMax, "one bucket per key slot");
// counter of bucket b at spad(b): one pad word per 16, so that lane l's
// run of 16 counters (words 17 l .. 17 l + 15) spans 16 distinct banks
__device__ __forceinline__ uint32_t spad(uint32_t b) { return b + (b >> 4); }
constexpr uint32_t kSmallCnt = kSmallBuckets + kSmallBuckets / 16;
constexpr uint32_t kSmallKeys = kSmallMax + 32;        // keys, then sentinels

__device__ __forceinline__ bool small_by_wave(const Leaf& L) {
  const uint32_t kind = L.flags & 3u;
  return (kind == kKindSparse || kind == kKindWr) && L.nv <= kSmallMax;
}

// Back-list jobs of k_leaf_once (both rounds): sparse leaves of more than
// kSmallMax values with n_v^2 >= 2 N_v, i.e. at least one repeat expected
// among their first n_v values.
__device__ __forceinline__ bool once_by_group(const Leaf& L) {
  return (L.flags & 3u) == kKindSparse && L.nv > kSmallMax &&
         static_cast<uint64_t>(L.nv) * L.nv >= 2 * L.Nv;
}

// The first `need` non-void values in [0, s) of the 32-bit stream from word
// t0 on, in stream order, into dst[0..need), by one wave: lane l maps the
// words of Philox block (t >> 2) + l, a wave scan ranks the non-void ones.
// Returns the word index just after the last value taken.
__device__ uint64_t take_wave(const Stream& st, uint64_t t0, uint32_t need, const RangeInfo& ri,
                              uint32_t* dst, uint32_t lane) {
  uint32_t done = 0;
  uint64_t t = t0, after = t0;
  while (done < need) {
    const uint64_t blk = (t >> 2) + lane;
    const uint4 w = philox_block(st, static_cast<uint32_t>(blk));
    uint32_t v[4], ok = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bool good = true;
      if (ri.pow2)
        v[j] = ri.pshift >= 32 ? 0u : (pick(w, j) >> ri.pshift);
      else
        good = range_map(pick(w, j), ri.s, ri.thr, &v[j]);
      if (good && 4 * blk + j >= t) ok |= 1u << j;
    }
    const uint32_t c = static_cast<uint32_t>(__popc(ok));
    const uint32_t incl = wave_scan_incl(c);
    uint32_t p = done + incl - c;
    bool has_last = false;
    uint64_t last = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if ((ok >> j) & 1u) {
        if (p < need) dst[p] = v[j];
        if (p == need - 1) {
          has_last = true;
          last = 4 * blk + j + 1;
        }
        ++p;
      }
    }
    const unsigned long long m = __ballot(has_last);
    if (m != 0) {
      const uint32_t f = static_cast<uint32_t>(__ffsll(static_cast<long long>(m)) - 1);
      after = static_cast<uint64_t>(__builtin_amdgcn_readlane(static_cast<uint32_t>(last), f)) |
              (static_cast<uint64_t>(__builtin_amdgcn_readlane(static_cast<uint32_t>(last >> 32), f))
               << 32);
    }
    done += __builtin_amdgcn_readlane(incl, 63);
    t = ((t >> 2) + 64) << 2;
  }
  return after;
}

// W-key windows at off + W i of keys[0..n) (sentinels follow n); merge: each
// window's halves are already sorted.  True iff some window holds equal
// neighbours below n.
template <int W, bool kMerge>
__device__ __forceinline__ bool wave_windows(uint32_t* keys, uint32_t n, uint32_t off,
                                             uint32_t lane) {
  bool dup = false;
  for (uint32_t w0 = off + W * lane; w0 < n; w0 += 64 * W) {
    uint4* p = reinterpret_cast<uint4*>(keys + w0);
    uint32_t v[W];
#pragma unroll
    for (int q = 0; q < W / 4; ++q) {
      const uint4 x = p[q];
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    }
    sort_net<W, kMerge>(v);
#pragma unroll
    for (int q = 0; q < W / 4; ++q)
      p[q] = make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    const uint32_t lim = n - w0;
#pragma unroll
    for (int i = 0; i + 1 < W; ++i)
      dup = dup || (v[i] == v[i + 1] && static_cast<uint32_t>(i + 1) < lim);
  }
  return __ballot(dup) != 0;
}

// keys[0..n) ascending by one wave (n <= kSmallMax, keys >> shift below
// kSmallBuckets); returns true iff a value repeats.  Counting pass by
// key >> shift (LDS atomics give each key its slot in its bucket), scan of
// the counts (lane l owns buckets 16 l .. 16 l + 15), scatter back into
// keys, then the Batcher windows of the work-group sort (8-key windows and
// merge windows shifted by 4 when no bucket holds more than 5 keys, 16-key
// ones up to 9), else odd-even transposition rounds.
__device__ bool wave_sort(uint32_t* keys, uint32_t n, uint32_t shift, uint32_t* cnt,
                          uint32_t lane) {
  for (uint32_t w = lane; w < kSmallCnt / 4; w += 64)
    reinterpret_cast<uint4*>(cnt)[w] = make_uint4(0, 0, 0, 0);
  uint32_t kk[kSmallKpl], as[kSmallKpl];
#pragma unroll
  for (uint32_t q = 0; q < kSmallKpl; ++q) {
    const uint32_t i = 64 * q + lane;
    kk[q] = 0;
    as[q] = ~0u;
    if (i < n) {
      kk[q] = keys[i];
      const uint32_t b = spad(kk[q] >> shift);
      as[q] = b | (atomicAdd(&cnt[b], 1u) << 16);
    }
  }
  {
    uint32_t* run = cnt + spad(kSmallKpl * lane);
    uint32_t c[kSmallKpl];
    uint32_t sum = 0, big = 0;
#pragma unroll
    for (uint32_t m = 0; m < kSmallKpl; ++m) {
      c[m] = run[m];
      sum += c[m];
      big = max(big, c[m]);
    }
    const uint32_t incl = wave_scan_incl(sum);
    uint32_t acc = incl - sum;
#pragma unroll
    for (uint32_t m = 0; m < kSmallKpl; ++m) {
      run[m] = acc;
      acc += c[m];
    }
    big = __builtin_amdgcn_readlane(wave_max_incl(big), 63);
    if (lane < 24) keys[n + lane] = 0xFFFFFFFFu;
#pragma unroll
    for (uint32_t q = 0; q < kSmallKpl; ++q)
      if (as[q] != ~0u) keys[cnt[as[q] & 0xFFFFu] + (as[q] >> 16)] = kk[q];
    if (shift == 0 || big <= 1) return shift == 0 && big >= 2;
    if (big <= 5) {
      const bool d = wave_windows<8, false>(keys, n, 0, lane);
      return wave_windows<8, true>(keys, n, 4, lane) || d;
    }
    if (big <= 9) {
      const bool d = wave_windows<16, false>(keys, n, 0, lane);
      return wave_windows<16, true>(keys, n, 8, lane) || d;
    }
    for (uint32_t r = 0; r < big; ++r) {
      for (uint32_t i = 2 * lane + (r & 1u); i + 1 < n; i += 128) {
        const uint32_t a = keys[i], b = keys[i + 1];
        keys[i] = min(a, b);
        keys[i + 1] = max(a, b);
      }
    }
  }
  bool dup = false;
  for (uint32_t i = lane; i + 1 < n; i += 64) dup = dup || keys[i] == keys[i + 1];
  return __ballot(dup) != 0;
}

// keys[0..n) ascending with equal values adjacent -> the distinct values in
// keys[0..d); returns d (one wave; every key is read before any is moved).
__device__ uint32_t compact_wave(uint32_t* keys, uint32_t n, uint32_t lane) {
  uint32_t kk[kSmallKpl];
  uint32_t keep = 0;
#pragma unroll
  for (uint32_t q = 0; q < kSmallKpl; ++q) {
    const uint32_t i = 64 * q + lane;
    kk[q] = 0;
    if (i < n) {
      kk[q] = keys[i];
      if (i == 0 || keys[i - 1] != kk[q]) keep |= 1u << q;
    }
  }
  uint32_t d = 0;
#pragma unroll
  for (uint32_t q = 0; q < kSmallKpl; ++q) {
    const unsigned long long m = __ballot((keep >> q) & 1u);
    if ((keep >> q) & 1u) keys[d + lane_rank(m)] = kk[q];
    d += static_cast<uint32_t>(__popcll(m));
  }
  return d;
}

__device__ void leaf_small_wave(const Leaf& L, uint64_t* out, uint32_t* keys, uint32_t* cnt) {
  const uint32_t lane = lane_tid();
  const uint32_t nv = L.nv;
  const bool wr = (L.flags & 3u) == kKindWr;
  const RangeInfo ri = range_info(L.Nv);
  const uint32_t kb = bit_length(L.Nv - 1);
  const uint32_t shift = kb > kSmallBucketBits ? kb - kSmallBucketBits : 0u;
  const Stream st = make_stream(L.seed, L.id, wr ? kWrLeaf : kLeaf, 0);
  uint64_t t = take_wave(st, 0, nv, ri, keys, lane);
  bool dups = wave_sort(keys, nv, shift, cnt, lane);
  while (dups && !wr) {  // Algorithm H's rounds (sparse leaves only)
    const uint32_t have = compact_wave(keys, nv, lane);
    t = take_wave(st, t, nv - have, ri, keys + have, lane);
    dups = wave_sort(keys, nv, shift, cnt, lane);
  }
  const uint64_t b1 = L.lo + 1;
  uint64_t* o = out + L.off;
  for (uint32_t i = lane; i < nv; i += 64) store_out(o + i, b1 + keys[i]);
}

template <int B>
__device__ void leaf_fill(const Leaf& L, uint64_t* out) {
  uint64_t* o = out + L.off;
  for (uint32_t i = threadIdx.x; i < L.nv; i += B) store_out(o + i, L.lo + 1);
}

// Jobs handed over in a round (front list count in the low 32 bits, back
// list count in the high 32 bits): those granted slots.
__device__ __forceinline__ uint64_t job_counts(const Control* ctl, int round) {
  const unsigned long long g = round ? ctl->granted2 : ctl->granted;
  return g != ~0ull ? g : (round ? ctl->leaf_counts2 : ctl->leaf_counts);
}

// Persistent leaf loop: job i of the class's list goes to work-group
// i mod G, whose job records are read kCacheLeaves at a time into LDS.
// kListFront: the front list (sparse and with-replacement leaves over
// power-of-two ranges, except sparse ones expected to repeat) with only that
// leaf body compiled in, so that the hot path keeps its values in registers.
// kListBack: the back list with every other leaf body, leaving to the
// one-wave kernels and to k_leaf_once the jobs they take, except the kinds in
// `takes` (kTakesDense / kTakesSmall / kTakesOnce: that kernel is not
// launched); round2: the second round's jobs (back list only, every kind
// but those of k_leaf_once, which it takes too when kTakesOnce is set).
// kListOnce: the back list's jobs of once_by_group, both rounds.
constexpr int kListFront = 0, kListBack = 1, kListOnce = 2;

template <int B, int kList>
__device__ __forceinline__ void leaf_loop(const Leaf* __restrict__ leaves, uint64_t leaf_cap,
                                          uint64_t* out, Control* ctl, int round2 = 0,
                                          uint32_t takes = 0) {
  constexpr bool kPow2 = kList == kListFront;
  __shared__ uint32_t smem[kSmemWords];
  LeafSmem sm;
  sm.keys = smem;
  sm.tmp = smem + kKeys;
  sm.buck = smem + kRegionA;
  sm.kept = sm.buck;
  sm.mask = sm.buck + kKeys;
  uint32_t* cache = smem + kRegionA + kRegionB;
  sm.scr = cache + kCacheWords;
  const uint64_t counts = uniform64(job_counts(ctl, round2));
  const uint64_t front = counts & 0xFFFFFFFFull, back = counts >> 32;
  if (front + back > leaf_cap) {
    // cannot happen (granted slots sum to at most the capacity): report it
    // and sample nothing
    if (kList == kListBack && blockIdx.x == 0 && threadIdx.x == 0)
      atomicOr(ctl->err, kErrLeafCapacity);
    return;
  }
  const uint64_t n_leaves = kPow2 ? front : back;
  const uint64_t G = gridDim.x;
  if (kPow2) {
    // the power-of-two leaf sorts leave the bucket counters zeroed behind them
    zero_counters<B>(sm.buck, threadIdx.x);
    __syncthreads();
  }
  uint32_t keep = ~0u;  // bit s: cached job s is run here (not by k_leaf_dense)
  for (uint64_t j = 0;; ++j) {
    const uint64_t i = blockIdx.x + j * G;
    if (i >= n_leaves) break;
    const uint32_t slot = static_cast<uint32_t>(j % kCacheLeaves);
    if (slot == 0) {
      // read the next kCacheLeaves job records of this work-group into LDS;
      // skipped jobs end without a barrier, so wait until every thread has
      // read the previous record
      if constexpr (!kPow2) __syncthreads();
      const uint32_t tid = threadIdx.x;
      if (tid < kCacheLeaves * 3) {
        const uint32_t which = tid / 3, part = tid % 3;
        const uint64_t li = i + static_cast<uint64_t>(which) * G;
        if (li < n_leaves) {
          const Leaf* rec = kPow2 ? leaves + li : leaves + (leaf_cap - 1 - li);
          const uint4 v = reinterpret_cast<const uint4*>(rec)[part];
          reinterpret_cast<uint4*>(cache + which * kLeafWords)[part] = v;
        }
      }
      __syncthreads();
      if constexpr (!kPow2) {
        if (tid < 64) {
          bool run = false;
          if (tid < kCacheLeaves && i + static_cast<uint64_t>(tid) * G < n_leaves) {
            Leaf c;
            const uint32_t* r = cache + tid * kLeafWords;
            c.Nv = static_cast<uint64_t>(r[4]) | (static_cast<uint64_t>(r[5]) << 32);
            c.nv = r[10];
            c.flags = r[11];
            if (kList == kListOnce)
              run = once_by_group(c);
            else
              run = (!once_by_group(c) || (takes & kTakesOnce)) &&
                    (round2 || ((!dense_by_wave(c) || (takes & kTakesDense)) &&
                                (!small_by_wave(c) || (takes & kTakesSmall))));
          }
          const unsigned long long m = __ballot(run);
          if (tid == 0) sm.scr[kScrKeep] = static_cast<uint32_t>(m);
        }
        __syncthreads();
        keep = __builtin_amdgcn_readfirstlane(sm.scr[kScrKeep]);
        if (keep == 0) {  // the whole group is other kernels'
          j += kCacheLeaves - 1;
          continue;
        }
      }
    }
    if (!kPow2 && !((keep >> slot) & 1u)) continue;  // another kernel's
    Leaf L;
    {
      const uint4* c = reinterpret_cast<const uint4*>(cache + slot * kLeafWords);
      const uint4 a = c[0], b = c[1], d = c[2];
      L.id = static_cast<uint64_t>(a.x) | (static_cast<uint64_t>(a.y) << 32);
      L.lo = static_cast<uint64_t>(a.z) | (static_cast<uint64_t>(a.w) << 32);
      L.Nv = static_cast<uint64_t>(b.x) | (static_cast<uint64_t>(b.y) << 32);
      L.off = static_cast<uint64_t>(b.z) | (static_cast<uint64_t>(b.w) << 32);
      L.seed = static_cast<uint64_t>(d.x) | (static_cast<uint64_t>(d.y) << 32);
      L.nv = d.z;
      L.flags = d.w;
      // every lane read the same record: make that explicit so the job's
      // parameters live in scalar registers
      L.id = uniform64(L.id);
      L.lo = uniform64(L.lo);
      L.Nv = uniform64(L.Nv);
      L.off = uniform64(L.off);
      L.seed = uniform64(L.seed);
      L.nv = __builtin_amdgcn_readfirstlane(L.nv);
      L.flags = __builtin_amdgcn_readfirstlane(L.flags);
    }
    if constexpr (kPow2) {
      // No barrier after the leaf: the next leaf's first LDS writes (counting
      // atomics into zeroed counters) do not touch what this leaf's output
      // pass still reads, and its sentinels and flag wait for the counting
      // barrier, which every thread reaches only after its output pass.
      leaf_sparse_pow2<B>(L, out, sm);
    } else if constexpr (kList == kListOnce) {
      leaf_once<B>(L, out, sm);
      __syncthreads();
    } else {
      switch (L.flags & 3u) {
        case kKindSparse: leaf_sparse<B>(L, out, sm); break;
        case kKindDense: leaf_dense<B>(L, out, sm); break;
        case kKindWr: leaf_wr<B>(L, out, sm); break;
        default: leaf_fill<B>(L, out); break;
      }
      __syncthreads();
    }
  }
}

template <int B>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(6))) void k_leaf_pow2(
    const Leaf* __restrict__ leaves, uint64_t leaf_cap, uint64_t* out, Control* ctl) {
  leaf_loop<B, kListFront>(leaves, leaf_cap, out, ctl);
}

template <int B>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(6))) void k_leaf_mixed(
    const Leaf* __restrict__ leaves, uint64_t leaf_cap, uint64_t* out, Control* ctl, int round2,
    uint32_t takes) {
  leaf_loop<B, kListBack>(leaves, leaf_cap, out, ctl, round2, takes);
}

template <int B>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(6))) void k_leaf_once(
    const Leaf* __restrict__ leaves, uint64_t leaf_cap, uint64_t* out, Control* ctl, int round2) {
  leaf_loop<B, kListOnce>(leaves, leaf_cap, out, ctl, round2);
}

// Dense leaves of the back list, one wave (and work-group) per leaf: back job
// i goes to wave i mod G; other jobs are left to k_leaf_mixed.
__global__ __launch_bounds__(64) void k_leaf_dense(const Leaf* __restrict__ leaves,
                                                   uint64_t leaf_cap, uint64_t* out, Control* ctl) {
  __shared__ __align__(16) uint16_t list[kWaveList];
  __shared__ uint32_t mask[kWaveMaskWords];
  __shared__ uint32_t bases[kWaveBases];
  const uint64_t counts = uniform64(job_counts(ctl, 0));
  const uint64_t front = counts & 0xFFFFFFFFull, back = counts >> 32;
  if (front + back > leaf_cap) return;  // reported by k_leaf_mixed
  for (uint64_t i = blockIdx.x; i < back; i += gridDim.x) {
    const Leaf* rec = leaves + (leaf_cap - 1 - i);
    Leaf L;
    L.id = uniform64(rec->id);
    L.lo = uniform64(rec->lo);
    L.Nv = uniform64(rec->Nv);
    L.off = uniform64(rec->off);
    L.seed = uniform64(rec->seed);
    L.nv = __builtin_amdgcn_readfirstlane(rec->nv);
    L.flags = __builtin_amdgcn_readfirstlane(rec->flags);
    if (!dense_by_wave(L) || L.nv == 0) continue;
    leaf_dense_wave(L, out, list, mask, bases);
  }
}

// Small sparse and with-replacement leaves of the back list, one wave (and
// work-group) per leaf: back job i goes to wave i mod G.
__global__ __launch_bounds__(64) void k_leaf_small(const Leaf* __restrict__ leaves,
                                                   uint64_t leaf_cap, uint64_t* out, Control* ctl) {
  __shared__ __align__(16) uint32_t keys[kSmallKeys];
  __shared__ __align__(16) uint32_t cnt[kSmallCnt];
  const uint64_t counts = uniform64(job_counts(ctl, 0));
  const uint64_t front = counts & 0xFFFFFFFFull, back = counts >> 32;
  if (front + back > leaf_cap) return;  // reported by k_leaf_mixed
  for (uint64_t i = blockIdx.x; i < back; i += gridDim.x) {
    const Leaf* rec = leaves + (leaf_cap - 1 - i);
    Leaf L;
    L.nv = __builtin_amdgcn_readfirstlane(rec->nv);
    L.flags = __builtin_amdgcn_readfirstlane(rec->flags);
    if (!small_by_wave(L) || L.nv == 0) continue;
    L.id = uniform64(rec->id);
    L.lo = uniform64(rec->lo);
    L.Nv = uniform64(rec->Nv);
    L.off = uniform64(rec->off);
    L.seed = uniform64(rec->seed);
    leaf_small_wave(L, out, keys, cnt);
  }
}

// ---------------------------------------------------------------------------
// Tree kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool is_leaf(const Node& v, const Instance& I) {
  if (I.variant == 1 && v.Nv == 1) return true;
  return v.nv < I.n0 && v.Nv <= kLeafMaxRange;
}

// kWave: aligned groups of 2^gbits lanes split the same node together.
template <bool kWave = false>
__device__ __forceinline__ uint64_t split_left(const Node& v, const Instance& I,
                                               uint32_t gbits = 6) {
  const uint64_t l = v.Nv >> 1;
  return I.variant == 1 ? binomial<kWave>(v.nv, l, v.Nv, I.seed, v.id, gbits)
                        : hypergeometric<kWave>(v.nv, l, v.Nv, I.seed, v.id, kSplit, gbits);
}

// Leaves of at most kInlineMax values, sparse or with replacement, are
// sampled by the tree thread that reaches them, straight into the output:
// the values the leaf kernels would give (the first n_v distinct non-void
// values of the leaf's word stream mapped into [0, N_v), or with replacement
// its first n_v non-void values with repeats, ascending), without a job.
// The thread keeps them sorted in its own LDS row (insertion: a repeat is
// the value just below its place).
constexpr uint32_t kInlineStride = kInlineMax + 1;  // rows start in distinct banks
constexpr uint32_t kTreeBlock = 256;

__device__ __forceinline__ bool leaf_inline_kind(const Node& v, const Instance& I) {
  if (v.nv > kInlineMax) return false;
  if (I.variant == 1) return v.Nv != 1;  // constant leaves stay jobs
  return static_cast<uint64_t>(I.dense_ratio) * v.nv < v.Nv;  // sparse (dense stay jobs)
}

__device__ void leaf_inline(const Node& v, const Instance& I, uint64_t* out, uint32_t* row) {
  const bool wr = I.variant == 1;
  const Stream st = make_stream(I.seed, v.id, wr ? kWrLeaf : kLeaf, 0);
  const uint32_t thr = range_threshold(v.Nv);
  const uint32_t nv = static_cast<uint32_t>(v.nv);
  uint32_t have = 0;
  for (uint64_t blk = 0; have < nv; ++blk) {
    const uint4 w = philox_block(st, blk);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t x;
      if (have >= nv || !range_map(pick(w, j), v.Nv, thr, &x)) continue;
      uint32_t p = have;
      while (p > 0 && row[p - 1] > x) --p;
      if (!wr && p > 0 && row[p - 1] == x) continue;  // a repeat: not a new value
      for (uint32_t i = have; i > p; --i) row[i] = row[i - 1];
      row[p] = x;
      ++have;
    }
  }
  uint64_t* o = out + I.out_offset + v.off;
  const uint64_t b1 = v.lo + 1;
  for (uint32_t i = 0; i < nv; ++i) store_out(o + i, b1 + row[i]);
}

// Hand leaf v over as a job (round 0: front or back list by kind; round 1:
// back list).  The job's slots are granted iff the slots asked for so far,
// these included, fit the capacity; returns whether they were.
__device__ __forceinline__ bool emit(const Node& v, const Instance& I, Leaf* leaves, uint64_t cap,
                                     Control* ctl, int round) {
  uint32_t kind;
  if (I.variant == 1)
    kind = v.Nv == 1 ? kKindFill : kKindWr;
  else
    kind = static_cast<uint64_t>(I.dense_ratio) * v.nv >= v.Nv ? kKindDense : kKindSparse;
  uint64_t pieces = 1;
  if (kind == kKindFill && v.nv > kFillPiece) pieces = (v.nv + kFillPiece - 1) / kFillPiece;
  // sparse and with-replacement leaves over a power-of-two range fill the
  // job array from the front, everything else from the back; the leaf
  // kernel of the other class reports the two lists meeting.  Sparse leaves
  // whose values are expected to repeat (n_v^2 >= 2 N_v) go to the back,
  // where the one-pass sampler finds the repeats.
  const bool front = round == 0 && (v.Nv & (v.Nv - 1)) == 0 &&
                     (kind == kKindWr || (kind == kKindSparse && v.nv * v.nv < 2 * v.Nv));
  // One counter word (front jobs in its low half, back jobs in its high
  // half) and one atomic per wave for the jobs of one slot each: the lanes
  // take the counter values a sequence of single increments in lane order
  // would have returned.  Constant leaves cut into several pieces take an
  // atomic of their own.
  unsigned long long* counter = round == 0 ? &ctl->leaf_counts : &ctl->leaf_counts2;
  const bool single = pieces == 1;
  const unsigned long long mf = __ballot(single && front);
  const unsigned long long mb = __ballot(single && !front);
  unsigned long long old = 0;
  if ((mf | mb) != 0) {
    const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<long long>(mf | mb)) - 1);
    unsigned long long at0 = 0;
    if ((threadIdx.x & 63u) == leader)
      at0 = atomicAdd(counter, static_cast<unsigned long long>(__popcll(mf)) +
                                   (static_cast<unsigned long long>(__popcll(mb)) << 32));
    at0 = static_cast<unsigned long long>(
              __builtin_amdgcn_readlane(static_cast<uint32_t>(at0), leader)) |
          (static_cast<unsigned long long>(
               __builtin_amdgcn_readlane(static_cast<uint32_t>(at0 >> 32), leader)) << 32);
    old = at0 + lane_rank(mf) + (static_cast<unsigned long long>(lane_rank(mb)) << 32);
  }
  if (!single) old = atomicAdd(counter, static_cast<unsigned long long>(pieces) << 32);
  const uint64_t asked = (old & 0xFFFFFFFFull) + (old >> 32);  // slots before this job
  if (asked + pieces > cap) {
    // the one job that crosses the capacity records the granted counts
    if (asked <= cap) (round == 0 ? ctl->granted : ctl->granted2) = old;
    return false;
  }
  const uint64_t base = front ? (old & 0xFFFFFFFFull) : (old >> 32);
  for (uint64_t j = 0; j < pieces; ++j) {
    if (base + j >= cap) {  // cannot happen: granted slots sum to at most cap
      atomicOr(ctl->err, kErrLeafCapacity);
      return true;
    }
    const uint64_t at = front ? base + j : cap - 1 - (base + j);
    Leaf L;
    L.id = v.id;
    L.lo = v.lo;
    L.Nv = v.Nv;
    L.off = I.out_offset + v.off + j * kFillPiece;
    L.seed = I.seed;
    L.nv = static_cast<uint32_t>(pieces == 1 ? v.nv
                                             : ((j + 1 < pieces) ? kFillPiece : v.nv - j * kFillPiece));
    L.flags = kind | (I.n0 << 8);
    leaves[at] = L;
  }
  return true;
}

// emit, and when the job array is full: in round 0 with a redo bitmap, mark
// tree thread t for the second round; otherwise latch the capacity error.
// row: this thread's LDS row of kInlineStride words.
__device__ __forceinline__ bool emit_or_mark(const Node& v, const Instance& I, Leaf* leaves,
                                             uint64_t cap, Control* ctl, int round, uint32_t* redo,
                                             uint64_t t, uint32_t* row) {
  if (leaf_inline_kind(v, I)) {
    leaf_inline(v, I, ctl->out, row);
    return true;
  }
  if (emit(v, I, leaves, cap, ctl, round)) return true;
  if (round == 0 && redo != nullptr)
    atomicOr(&redo[t >> 5], 1u << (t & 31u));
  else
    atomicOr(ctl->err, kErrLeafCapacity);
  return false;
}

__device__ __forceinline__ uint32_t find_instance(const Instance* inst, uint32_t n_inst,
                                                  uint64_t t, bool top) {
  uint32_t lo = 0, hi = n_inst;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((top ? inst[mid].top_base : inst[mid].thread_base) <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// Walk levels [d0, d1) of Algorithm P from node v along the bits of g (bit
// d1-1-d chooses the child at depth d).  Returns false when the walk ended
// early at a leaf or an empty node (the leaf is emitted by the path whose
// remaining bits are zero).  kWave: the 64 lanes of a wave walk one path
// together (lane 0 emits) and share each split's rejection attempts.
// kGroups (d1 - d0 = 6, lane l walking g with low bits l from one shared
// node): at depth d the lanes whose paths agree above bit d1-1-d hold the
// same node, an aligned group of 2^(d1-d) lanes that share its split's
// rejection attempts.  emit_or_mark's round, redo, t and row apply to the
// leaf it may emit.
template <bool kWave = false, bool kGroups = false>
__device__ __forceinline__ bool walk_path(Node& v, uint32_t d0, uint32_t d1, uint64_t g,
                                          const Instance& I, Leaf* leaves, uint64_t leaf_cap,
                                          Control* ctl, uint32_t* row, int round = 0,
                                          uint32_t* redo = nullptr, uint64_t t = 0) {
  for (uint32_t d = d0; d < d1; ++d) {
    if (v.nv == 0) return false;
    if (is_leaf(v, I)) {
      const uint32_t below = d1 - d;
      if ((g & ((1ull << below) - 1)) == 0 && (!kWave || (threadIdx.x & 63u) == 0))
        emit_or_mark(v, I, leaves, leaf_cap, ctl, round, redo, t, row);
      return false;
    }
    const uint64_t L = kGroups ? split_left<true>(v, I, d1 - d) : split_left<kWave>(v, I);
    const uint64_t l = v.Nv >> 1;
    if ((g >> (d1 - 1 - d)) & 1) {
      v = Node{2 * v.id + 1, v.lo + l, v.Nv - l, v.nv - L, v.off + L};
    } else {
      v = Node{2 * v.id, v.lo, l, L, v.off};
    }
  }
  return true;
}

// The root of part `part` of a sample cut at depth dp (Sec. 4.1, online
// sampling): the depth-dp node on the path that the bits of `part` choose,
// most significant first.  A path that ends above dp at a leaf gives that
// leaf to the leftmost part below it (the remaining bits all zero) and
// leaves the other parts empty, with rank after the leaf's values; an empty
// node gives an empty part.  On return v.nv is the part's count and v.off
// its rank (values of the sample in earlier parts); returns false when the
// part is a leaf above dp or empty.  kWave: the wave's 64 lanes walk this
// path together (sharing each split's rejection attempts).
template <bool kWave = true>
__device__ __forceinline__ bool part_root(Node& v, uint32_t dp, uint64_t part,
                                          const Instance& I) {
  for (uint32_t d = 0; d < dp; ++d) {
    if (v.nv == 0) return false;
    if (is_leaf(v, I)) {
      const uint32_t below = dp - d;
      if ((part & ((1ull << below) - 1)) != 0) {
        v.off += v.nv;
        v.nv = 0;
      }
      return false;
    }
    const uint64_t L = split_left<kWave>(v, I);
    const uint64_t l = v.Nv >> 1;
    if ((part >> (dp - 1 - d)) & 1) {
      v = Node{2 * v.id + 1, v.lo + l, v.Nv - l, v.nv - L, v.off + L};
    } else {
      v = Node{2 * v.id, v.lo, l, L, v.off};
    }
  }
  return true;
}

// One wave per top path (top_threads paths, 64 lanes each): the splits
// above the frontier form the longest chain of the tree, and a wave finds
// each split's accepted attempt in one round of 64.  In part mode every
// path first walks to the part's root (the same splits on every path),
// the first path reports the part's count and rank, and offsets below
// count from the part's first value.
__global__ __launch_bounds__(kTreeBlock) void k_tree_top(const Instance* __restrict__ inst,
                                                  uint32_t n_inst, uint64_t top_threads,
                                                  Node* frontier, Leaf* leaves, uint64_t leaf_cap,
                                                  Control* ctl, uint64_t* part_out) {
  const uint64_t t = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (t >= top_threads) return;  // whole waves
  __shared__ uint32_t inl[kTreeBlock * kInlineStride];
  uint32_t* row = inl + threadIdx.x * kInlineStride;
  const Instance I = inst[find_instance(inst, n_inst, t, true)];
  const uint64_t g = t - I.top_base;
  const bool lane0 = (threadIdx.x & 63u) == 0;
  Node v{I.root ? I.root : 1, I.base, I.N, I.n, 0};
  uint32_t d0 = 0;
  if (part_out != nullptr) {
    const bool inner = part_root(v, I.part_depth, I.part, I);
    if (g == 0 && lane0) {
      part_out[0] = v.nv;
      part_out[1] = v.off;
    }
    v.off = 0;
    if (v.nv > I.part_cap) v.nv = 0;  // the caller's buffer is too small
    if (!inner) {
      if (v.nv > 0 && g == 0 && lane0)
        emit_or_mark(v, I, leaves, leaf_cap, ctl, 0, nullptr, 0, row);
      v.nv = 0;
    }
    d0 = I.part_depth;
  }
  if (v.nv > 0 && !walk_path<true>(v, d0, I.top_cut, g, I, leaves, leaf_cap, ctl, row)) v.nv = 0;
  if (lane0) frontier[t] = v;
}

__global__ __launch_bounds__(kTreeBlock) void k_tree(const Instance* __restrict__ inst, uint32_t n_inst,
                                              uint64_t total_threads,
                                              const Node* __restrict__ frontier, Leaf* leaves,
                                              uint64_t leaf_cap, Node* stacks,
                                              uint32_t stack_depth, Control* ctl, uint32_t* redo,
                                              int round) {
  __shared__ uint32_t inl[kTreeBlock * kInlineStride];
  uint32_t* row = inl + threadIdx.x * kInlineStride;
  const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total_threads) return;
  if (round == 1 && ((redo[t >> 5] >> (t & 31u)) & 1u) == 0) return;
  const uint32_t ii = find_instance(inst, n_inst, t, false);
  const Instance I = inst[ii];
  const uint64_t g = t - I.thread_base;
  const uint32_t rest = I.cut - I.top_cut;  // levels below the frontier
  Node v = frontier[I.top_base + (g >> rest)];
  const uint64_t gl = g & ((1ull << rest) - 1);
  // Algorithm P: the rest of the path to this thread's depth-`cut` node.
  // When the wave's 64 lanes are the 64 paths below one frontier node, the
  // lanes on a common node share its split's rejection attempts.
  const bool grouped =
      __ballot(rest == 6 && gl == (threadIdx.x & 63u) &&
               ii == __builtin_amdgcn_readfirstlane(ii)) == ~0ull;
  if (v.nv == 0) return;
  if (grouped ? !walk_path<false, true>(v, 0, rest, gl, I, leaves, leaf_cap, ctl, row, round,
                                        redo, t)
              : !walk_path(v, 0, rest, gl, I, leaves, leaf_cap, ctl, row, round, redo, t))
    return;
  // Depth-first expansion of the subtree (Algorithm R below depth `cut`).
  // Entry k of thread t's stack is stacks[k * total_threads + t], so that the
  // pushes of a wave's threads at one level share cache lines.
  Node* stk = stacks + t;
  uint32_t sp = 0;
  for (;;) {
    for (;;) {
      if (v.nv == 0) break;
      if (is_leaf(v, I)) {
        if (!emit_or_mark(v, I, leaves, leaf_cap, ctl, round, redo, t, row)) return;
        break;
      }
      const uint64_t L = split_left(v, I);
      const uint64_t l = v.Nv >> 1;
      const Node right{2 * v.id + 1, v.lo + l, v.Nv - l, v.nv - L, v.off + L};
      if (right.nv > 0) {
        if (sp == stack_depth) {
          atomicOr(ctl->err, kErrStackDepth);
          return;
        }
        stk[static_cast<uint64_t>(sp++) * total_threads] = right;
      }
      v = Node{2 * v.id, v.lo, l, L, v.off};
    }
    if (sp == 0) break;
    v = stk[static_cast<uint64_t>(--sp) * total_threads];
  }
}

// Online sampling (Sec. 4.1): the roots of all parts of a depth-dp cut at
// once, one thread per part walking its own path from the root (part_root's
// rule for leaves above the cut and for empty nodes), so that later calls
// sample parts from their roots without recomputing the splits above.
__global__ __launch_bounds__(256) void k_part_roots(Instance I, uint32_t dp, uint64_t parts,
                                                    Node* roots) {
  const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= parts) return;
  Node v{1, I.base, I.N, I.n, 0};
  part_root<false>(v, dp, g, I);
  roots[g] = v;
}

// Uneven universe (Sec. 4.3): thread i follows the binomial tree of the K
// segments from the root (level D) down to segment i.  At level j the
// subtree holding segment i is a = i >> j (segments a 2^j .. min(a 2^j + 2^j,
// K) - 1, heap id 2^(D-j) + a); its left subtree takes Hyp(n', L_l, L_l + L_r)
// of its n' samples, keyed by that id with the SEGSPLIT purpose.  Every path
// recomputes the splits above it, which are the same on every path (Sec. 3.2:
// decisions keyed by the node's identity), and sums the left counts it
// passes: the segment's output offset.  Element counts of subtrees come from
// the segments' bases (prefix sums the host stored).  The segment's own tree
// is keyed by 64-bit draw 0 of (seed, 2^D + i, SEGSEED).
__global__ __launch_bounds__(256) void k_segments(Instance* inst, uint64_t K, uint32_t D,
                                                  uint64_t n, uint64_t N, uint64_t seed,
                                                  uint64_t* counts) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= K) return;
  uint64_t nv = n, off = 0;
  for (uint32_t j = D; j >= 1; --j) {
    const uint64_t a = i >> j;
    const uint64_t first = a << j;
    const uint64_t mid = first + (1ull << (j - 1));
    const uint64_t end = first + (1ull << j);
    const uint64_t p_first = inst[first].base;
    const uint64_t p_mid = mid < K ? inst[mid].base : N;
    const uint64_t p_end = end < K ? inst[end].base : N;
    const uint64_t Ll = p_mid - p_first;
    const uint64_t all = p_end - p_first;
    const uint64_t nl = hypergeometric(nv, Ll, all, seed, (1ull << (D - j)) + a, kSegSplit);
    if ((i >> (j - 1)) & 1) {
      nv -= nl;
      off += nl;
    } else {
      nv = nl;
    }
  }
  const uint4 b = philox_block(make_stream(seed, (1ull << D) + i, kSegSeed, 0), 0);
  inst[i].n = nv;
  inst[i].seed = static_cast<uint64_t>(b.x) | (static_cast<uint64_t>(b.y) << 32);
  inst[i].out_offset = off;
  if (counts != nullptr) counts[i] = nv;
}

__device__ inline void start_control(Control* ctl, unsigned int* err) {
  ctl->leaf_counts = 0;
  ctl->granted = ~0ull;
  ctl->leaf_counts2 = 0;
  ctl->granted2 = ~0ull;
  ctl->out = nullptr;
  ctl->bern_count = 0;
  ctl->error = 0;
  ctl->err = err != nullptr ? err : &ctl->error;
}

__global__ void k_reset(Control* ctl, Instance single, int has_single, Instance* table,
                        unsigned int* err, uint32_t* redo, uint64_t redo_words, uint64_t* out) {
  const uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (uint64_t i = i0; i < redo_words; i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    redo[i] = 0;
  if (i0 == 0) {
    start_control(ctl, err);
    ctl->out = out;
    if (has_single) table[0] = single;
  }
}

// launch_zero runs 256-thread blocks; the first one clears every ticket word
static_assert(kTicketWords <= 256, "one thread per ticket word in k_zero's first block");
__global__ void k_zero(Control* ctl, unsigned long long* status, uint64_t n,
                       unsigned long long* tickets, unsigned int* err) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    status[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x < kTicketWords) tickets[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) start_control(ctl, err);
}

// ---------------------------------------------------------------------------
// Bernoulli chunks (Sec. 4.7).
// ---------------------------------------------------------------------------
constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagIncl = 2ull << 62;
constexpr unsigned long long kValueMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 26;

// Double-precision Bernoulli chunks (p < 2^-10), one work-group per chunk:
// one pass over the chunk's geometric stream.  Hit k of the chunk sits at
// 1-based offset q_k = sum_{i<=k} (skip_i + 1); draws are taken in (round,
// thread, draw) order, so each round's offsets come from one block scan.  Hits
// k < lds_cap go to pos[] when write == false; when write == true, hits
// k >= lds_cap are written straight to out (the chunk held more hits than LDS).
// Skips are capped at 2^33 (anything that long ends the chunk).  Returns the
// chunk's hit count.
__device__ uint64_t bern_pass(const Stream& st, uint64_t len, double c64, uint32_t* pos,
                              uint32_t lds_cap, bool write, uint64_t* out, uint64_t out_first,
                              uint64_t capacity, uint64_t base, uint64_t* scr64, uint32_t* ends) {
  constexpr int B = kBernBlock;
  constexpr uint32_t per = 2u;
  const uint32_t tid = threadIdx.x;
  const uint64_t lim = len;
  uint64_t last = 0;  // offset of the previous round's last draw
  uint64_t count = 0;
  for (uint32_t blk0 = 0;; blk0 += B) {
    const uint4 w = philox_block(st, blk0 + tid);
    uint64_t inc[per];
    uint64_t sum = 0;
    const uint64_t d0 = static_cast<uint64_t>(w.x) | (static_cast<uint64_t>(w.y) << 32);
    const uint64_t d1 = static_cast<uint64_t>(w.z) | (static_cast<uint64_t>(w.w) << 32);
#pragma unroll
    for (uint32_t j = 0; j < per; ++j) {
      const double g = floor(log64(unit_open0(j ? d1 : d0)) * c64);
      const double gc = g < 0x1p33 ? g : 0x1p33;
      inc[j] = static_cast<uint64_t>(gc) + 1;
      sum += inc[j];
    }
    uint64_t total;
    const uint64_t q0 = last + block_scan_excl<B, uint64_t>(sum, scr64, &total);
    uint64_t q = q0;
    const bool all_in = last + total <= lim;
    const uint64_t first_idx = count + per * tid;
    uint32_t in = 0;
#pragma unroll
    for (uint32_t j = 0; j < per; ++j) {
      q += inc[j];
      if (q <= lim) {
        const uint64_t idx = first_idx + j;
        if (!write) {
          if (idx < lds_cap) pos[idx] = static_cast<uint32_t>(q - 1);
        } else if (idx >= lds_cap && out_first + idx < capacity) {
          store_out(out + out_first + idx, base + static_cast<uint64_t>(q));
        }
        ++in;
      }
    }
    if (all_in) {
      count += per * B;
      last += total;
      continue;
    }
    // Offsets increase strictly, so exactly one thread starts in range and
    // holds the chunk's first out-of-range draw; it reports the count.
    if (in < per && q0 <= lim) *ends = per * tid + in;
    __syncthreads();
    count += *ends;
    __syncthreads();
    break;
  }
  return count;
}

// The hit count of a double-precision chunk (bern_pass's draws: 64-bit draw
// 2b + j is word pair j of Philox block b; hit k while the running position
// stays within len), counted by one wave, 128 draws per step.  The positions
// are exact integers, so this count equals bern_pass's whatever the grouping.
__device__ uint64_t bern_count64_wave(const Stream& st, uint64_t len, double c64, uint32_t lane) {
  uint64_t last = 0, count = 0;
  for (uint32_t blk0 = 0;; blk0 += 64) {
    const uint4 w = philox_block(st, blk0 + lane);
    const uint64_t d0 = static_cast<uint64_t>(w.x) | (static_cast<uint64_t>(w.y) << 32);
    const uint64_t d1 = static_cast<uint64_t>(w.z) | (static_cast<uint64_t>(w.w) << 32);
    uint64_t inc[2];
#pragma unroll
    for (uint32_t j = 0; j < 2; ++j) {
      const double g = floor(log64(unit_open0(j ? d1 : d0)) * c64);
      const double gc = g < 0x1p33 ? g : 0x1p33;
      inc[j] = static_cast<uint64_t>(gc) + 1;
    }
    const uint64_t sum = inc[0] + inc[1];
    const uint64_t incl = wave_scan_incl(sum);
    const uint64_t total = __shfl(incl, 63, 64);
    const uint64_t q1 = last + incl - sum + inc[0];
    const uint64_t q2 = q1 + inc[1];
    const uint32_t in = (q1 <= len ? 1u : 0u) + (q2 <= len ? 1u : 0u);
    if (last + total <= len) {
      count += 128;
      last += total;
      continue;
    }
    const unsigned long long whole = __ballot(in == 2u);
    const uint32_t nw = static_cast<uint32_t>(__popcll(whole));
    return count + 2ull * nw + (nw < 64 ? static_cast<uint32_t>(__shfl(in, nw, 64)) : 0u);
  }
}

// Decoupled look-back (one wave): chunk j's exclusive prefix is the sum of the
// aggregates of its predecessors back to the nearest one that has published an
// inclusive prefix.  Each step reads 64 predecessors at once.  Returns the
// exclusive prefix in every lane; lane 0 publishes j's inclusive prefix.
// A status word carries its whole message (flag and value in one 64-bit
// atomic), so relaxed agent-scope atomics suffice; release/acquire would add
// a write-back and an invalidation of the whole L2 per access.
// A predecessor that has published nothing after help_polls polls (its wave
// may not be running: another kernel can hold the GPU) has its hit count
// computed by this wave instead, count_of(i), a function of the chunk alone
// (Sec. 4.7: chunks are independent); the count is offered to other waves
// (compare-and-swap, only over an empty word) and the look-back goes on, so
// it ends whatever runs beside it.  From then on the wave helps at once.
template <class CountOf>
__device__ uint64_t bern_lookback(unsigned long long* status, uint64_t j, uint64_t cnt,
                                  Control* ctl, uint32_t help_polls, CountOf count_of) {
  const uint32_t lane = threadIdx.x & 63;
  if (j == 0) {
    if (lane == 0)
      __hip_atomic_store(&status[0], kFlagIncl | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0)
    __hip_atomic_store(&status[j], kFlagAgg | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint64_t acc = 0;
  long long top = static_cast<long long>(j) - 1;
  uint32_t spins = 0;
  bool helping = false;
  // this lane's predecessor counted by this wave (valid while `helped` is
  // set, for the current window of 64)
  bool helped = false;
  uint64_t own = 0;
  for (;;) {
    const long long i = top - static_cast<long long>(lane);
    // Positions before chunk 0 read as an inclusive prefix of 0.
    unsigned long long s =
        i >= 0 ? __hip_atomic_load(&status[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
               : kFlagIncl;
    if (helped && (s & ~kValueMask) == 0) s = kFlagAgg | own;
    const unsigned long long flag = s & ~kValueMask;
    const unsigned long long incl = __ballot(flag == kFlagIncl);
    const unsigned long long none = __ballot(flag == 0);
    const uint32_t first = incl ? static_cast<uint32_t>(__builtin_ctzll(incl)) : 64u;
    const unsigned long long upto = first >= 63 ? ~0ull : ((2ull << first) - 1);
    if (none & upto) {
      if (helping || ++spins > help_polls) {
        helping = true;
        // the nearest predecessor without a word
        const uint32_t h = static_cast<uint32_t>(__builtin_ctzll(none & upto));
        const uint64_t ih = static_cast<uint64_t>(top) - h;
        const uint64_t c = count_of(ih);
        if (lane == h) {
          helped = true;
          own = c;
          unsigned long long expect = 0;
          __hip_atomic_compare_exchange_strong(&status[ih], &expect, kFlagAgg | c,
                                               __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        }
        continue;
      }
      if (spins > kSpinLimit) {  // unreachable while help_polls < kSpinLimit
        if (lane == 0) atomicOr(ctl->err, kErrSpinLimit);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    uint64_t v = lane <= first ? static_cast<uint64_t>(s & kValueMask) : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    acc += v;
    if (first < 64) break;
    top -= 64;
    helped = false;
  }
  if (lane == 0)
    __hip_atomic_store(&status[j], kFlagIncl | (acc + cnt), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  return acc;
}

// Chunks are handed out as in k_bern_wave: n_cls counters kTicketStride
// words apart, work-group class c = blockIdx mod n_cls taking chunks c,
// c + n_cls, ... in order (one shared counter serializes the hand-out at
// about one chunk per same-address atomic); a chunk held up is counted by
// the waiting look-back itself.
__global__ __launch_bounds__(kBernBlock) void k_bern(uint64_t N, uint64_t seed, uint64_t chunk,
                                                     uint64_t n_chunks, double c64,
                                                     unsigned long long* status, uint64_t* out,
                                                     uint64_t capacity, uint64_t* count_dev,
                                                     Control* ctl, uint32_t lds_cap,
                                                     unsigned long long* tickets,
                                                     uint32_t n_cls, uint32_t help_polls) {
  extern __shared__ uint32_t pos[];  // lds_cap offsets (dynamic)
  __shared__ uint64_t scr64[8];
  __shared__ uint32_t ends;
  __shared__ unsigned long long cur, excl;
  const uint32_t cls = blockIdx.x % n_cls;
  unsigned long long* const ticket = tickets + cls * kTicketStride;
  for (;;) {
    if (threadIdx.x == 0) cur = cls + atomicAdd(ticket, 1ull) * n_cls;
    __syncthreads();
    const unsigned long long j = cur;
    __syncthreads();
    if (j >= n_chunks) break;
    const uint64_t base = j * chunk;
    const uint64_t len = (N - base) < chunk ? (N - base) : chunk;
    const Stream st = make_stream(seed, j, kBChunk, 0);
    const uint64_t cnt =
        bern_pass(st, len, c64, pos, lds_cap, false, out, 0, capacity, base, scr64, &ends);
    if (threadIdx.x < 64) {
      const uint64_t acc = bern_lookback(status, j, cnt, ctl, help_polls, [&](uint64_t i) {
        const uint64_t bi = i * chunk;
        return bern_count64_wave(make_stream(seed, i, kBChunk, 0),
                                 (N - bi) < chunk ? (N - bi) : chunk, c64, threadIdx.x & 63u);
      });
      if (threadIdx.x == 0) {
        excl = acc;
        if (j == n_chunks - 1) {
          *count_dev = acc + cnt;
          ctl->bern_count = acc + cnt;
        }
      }
    }
    __syncthreads();
    const uint64_t first = excl;
    const uint64_t held = cnt < lds_cap ? cnt : lds_cap;
    for (uint64_t i = threadIdx.x; i < held; i += kBernBlock)
      if (first + i < capacity) store_out(out + first + i, base + static_cast<uint64_t>(pos[i]) + 1);
    if (cnt > lds_cap)
      bern_pass(st, len, c64, pos, lds_cap, true, out, first, capacity, base, scr64, &ends);
    __syncthreads();
  }
}

// One wave's pass over a double-precision chunk: the draws and positions of
// bern_pass (64-bit draws 2b and 2b+1 of Philox block b; lane l takes block
// 64r + l in round r, so the positions grow with lane and draw).  First pass
// (out == nullptr): positions - 1 of hits below lds_cap go to pos[] and the
// hit count is returned; second pass: the hits from lds_cap on are written
// to out[first + k] as base + position.
__device__ uint64_t bern64_pass(const Stream& st, uint64_t len, double c64, uint32_t lane,
                                uint32_t* pos, uint32_t lds_cap, uint64_t* out, uint64_t first,
                                uint64_t capacity, uint64_t base) {
  uint64_t last = 0, count = 0;
  for (uint32_t blk0 = 0;; blk0 += 64) {
    const uint4 w = philox_block(st, blk0 + lane);
    const uint64_t d0 = static_cast<uint64_t>(w.x) | (static_cast<uint64_t>(w.y) << 32);
    const uint64_t d1 = static_cast<uint64_t>(w.z) | (static_cast<uint64_t>(w.w) << 32);
    uint64_t inc[2];
#pragma unroll
    for (uint32_t j = 0; j < 2; ++j) {
      const double g = floor(log64(unit_open0(j ? d1 : d0)) * c64);
      const double gc = g < 0x1p33 ? g : 0x1p33;
      inc[j] = static_cast<uint64_t>(gc) + 1;
    }
    const uint64_t sum = inc[0] + inc[1];
    const uint64_t incl = wave_scan_incl(sum);
    const uint64_t total = uniform64(__shfl(incl, 63, 64));
    const uint64_t q[2] = {last + incl - sum + inc[0], last + incl};
    const uint64_t idx0 = count + 2ull * lane;
#pragma unroll
    for (uint32_t j = 0; j < 2; ++j) {
      if (q[j] <= len) {
        const uint64_t idx = idx0 + j;
        if (out == nullptr) {
          if (idx < lds_cap) pos[idx] = static_cast<uint32_t>(q[j] - 1);
        } else if (idx >= lds_cap && first + idx < capacity) {
          store_out(out + first + idx, base + q[j]);
        }
      }
    }
    if (last + total <= len) {
      count += 128;
      last += total;
      continue;
    }
    // hits are a prefix of the round's draws (positions increase)
    const uint32_t in = (q[0] <= len ? 1u : 0u) + (q[1] <= len ? 1u : 0u);
    const unsigned long long whole = __ballot(in == 2u);
    const uint32_t nw = static_cast<uint32_t>(__popcll(whole));
    return count + 2ull * nw + (nw < 64 ? static_cast<uint32_t>(__shfl(in, nw, 64)) : 0u);
  }
}

// Double-precision Bernoulli chunks that expect few hits (chunks clamped at
// 2^32 for small p), one wave per chunk and no barrier: the hits of k_bern's
// definition, the first lds_cap positions kept in LDS while the look-back
// runs, the rest recomputed when written; consecutive lanes write
// consecutive outputs.
__global__ __launch_bounds__(64) void k_bern64_wave(uint64_t N, uint64_t seed, uint64_t chunk,
                                                    uint64_t n_chunks, double c64,
                                                    unsigned long long* status, uint64_t* out,
                                                    uint64_t capacity, uint64_t* count_dev,
                                                    Control* ctl, uint32_t lds_cap,
                                                    unsigned long long* tickets, uint32_t n_cls,
                                                    uint32_t help_polls) {
  extern __shared__ uint32_t pos[];  // lds_cap positions - 1 (dynamic)
  const uint32_t lane = lane_tid();
  const uint32_t cls = blockIdx.x % n_cls;
  unsigned long long* const ticket = tickets + cls * kTicketStride;
  for (;;) {
    uint64_t jt = 0;
    if (lane == 0) jt = atomicAdd(ticket, 1ull);
    const uint64_t j = cls + uniform64(jt) * n_cls;
    if (j >= n_chunks) break;
    const uint64_t base = j * chunk;
    const uint64_t len = (N - base) < chunk ? (N - base) : chunk;
    const Stream st = make_stream(seed, j, kBChunk, 0);
    const uint64_t cnt = bern64_pass(st, len, c64, lane, pos, lds_cap, nullptr, 0, 0, 0);
    const uint64_t first = bern_lookback(status, j, cnt, ctl, help_polls, [&](uint64_t i) {
      const uint64_t bi = i * chunk;
      return bern_count64_wave(make_stream(seed, i, kBChunk, 0),
                               (N - bi) < chunk ? (N - bi) : chunk, c64, lane);
    });
    if (lane == 0 && j == n_chunks - 1) {
      *count_dev = first + cnt;
      ctl->bern_count = first + cnt;
    }
    const uint64_t held = cnt < lds_cap ? cnt : lds_cap;
    for (uint64_t i = lane; i < held; i += 64)
      if (first + i < capacity) store_out(out + first + i, base + static_cast<uint64_t>(pos[i]) + 1);
    if (cnt > lds_cap) bern64_pass(st, len, c64, lane, pos, lds_cap, out, first, capacity, base);
  }
}

// Single-precision Bernoulli chunks (p >= 2^-10), one wave per chunk and no
// barrier: chunk j's hits are its draws up to the one that passes the chunk
// end (Sec. 4.7's skips).  The wave keeps each 256-draw group of the first
// kBernWaveGroups as 16-bit values: the positions relative to the group's
// start when the group advances less than 2^16, else the increments (below
// 22.2/p + 1 < 2^16), rebuilt by wave scans when written; later groups are
// recomputed when written.  It publishes its count for the look-back and
// writes consecutive lanes on consecutive outputs.
constexpr uint32_t kBernWaveGroup = 256;                     // draws per group
constexpr uint32_t kBernWaveGroups = 15;                     // groups kept in LDS
constexpr uint32_t kBernWaveList = kBernWaveGroup * kBernWaveGroups;

// Increments of draw group c (lane l: draws 256c + 4l + j) into dst, and
// their wave-wide inclusive prefix over lanes.
__device__ __forceinline__ uint32_t bern_group(const Stream& st, uint32_t c, uint32_t lane,
                                               float c32, uint32_t inc[4]) {
  const uint4 w = philox_block(st, c * (kBernWaveGroup / 4) + lane);
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    inc[j] = static_cast<uint32_t>(geom_skip32(pick(w, j), c32)) + 1u;
    sum += inc[j];
  }
  return sum;
}

__device__ __forceinline__ void put_incs(uint16_t* dst, const uint32_t inc[4]) {
  uint2 v;
  v.x = inc[0] | (inc[1] << 16);
  v.y = inc[2] | (inc[3] << 16);
  *reinterpret_cast<uint2*>(dst) = v;
}

// The hit count of a single-precision chunk, counted by one wave exactly as
// k_bern_wave counts its own chunk (without keeping the positions).
__device__ uint32_t bern_count32_wave(const Stream& st, uint32_t len, float c32, uint32_t lane) {
  uint32_t q_base = 0, cnt = 0;
  for (uint32_t c = 0;; ++c) {
    uint32_t inc[4];
    const uint32_t sum = bern_group(st, c, lane, c32, inc);
    const uint32_t incl = wave_scan_incl(sum);
    uint32_t r = incl - sum, in = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      r += inc[k];
      in += q_base + r <= len ? 1u : 0u;
    }
    const unsigned long long whole = __ballot(in == 4u);
    const uint32_t nw = static_cast<uint32_t>(__popcll(whole));
    const uint32_t got = nw == 64u ? kBernWaveGroup : 4u * nw + __builtin_amdgcn_readlane(in, nw);
    cnt += got;
    q_base += __builtin_amdgcn_readlane(incl, 63);
    if (got < kBernWaveGroup) return cnt;
  }
}

__global__ __launch_bounds__(64) void k_bern_wave(uint64_t N, uint64_t seed, uint64_t chunk,
                                                  uint64_t n_chunks, float c32,
                                                  unsigned long long* status, uint64_t* out,
                                                  uint64_t capacity, uint64_t* count_dev,
                                                  Control* ctl, unsigned long long* tickets,
                                                  uint32_t n_cls, uint32_t help_polls) {
  __shared__ __align__(16) uint16_t list[kBernWaveList];
  __shared__ uint32_t gbase[kBernWaveGroups + 1];  // position before group c (c <= 15)
  const uint32_t lane = lane_tid();
  constexpr uint32_t kSpare = (kBernWaveGroups - 1) * kBernWaveGroup;  // recomputed groups
  // Chunks are handed out by n_cls counters, 256 bytes apart: this wave's
  // class c = blockIdx mod n_cls takes chunks c, c + n_cls, ... in order.
  // Same-address atomics serialize, so one shared counter would cap the
  // chunk rate; with n_cls coprime to the 8 XCDs that work-groups alternate
  // over, any n_cls work-groups on one XCD cover every class.  When a chunk
  // is held up anyway (its class has no running wave because another kernel
  // holds the GPU), the look-back counts it itself (bern_lookback).
  const uint32_t cls = blockIdx.x % n_cls;
  unsigned long long* const ticket = tickets + cls * kTicketStride;
  for (;;) {
    uint64_t jt = 0;
    if (lane == 0) jt = atomicAdd(ticket, 1ull);
    const uint64_t j = cls + uniform64(jt) * n_cls;
    if (j >= n_chunks) break;
    const uint64_t base = j * chunk;
    const uint32_t len = static_cast<uint32_t>((N - base) < chunk ? (N - base) : chunk);
    const Stream st = make_stream(seed, j, kBChunk, 0);
    // hits: the draws whose running position stays within the chunk
    uint32_t q_base = 0, cnt = 0;
    uint32_t rel_groups = 0;  // bit c: group c holds relative positions
    for (uint32_t c = 0;; ++c) {
      uint32_t inc[4];
      const uint32_t sum = bern_group(st, c, lane, c32, inc);
      const uint32_t incl = wave_scan_incl(sum);
      const uint32_t adv = __builtin_amdgcn_readlane(incl, 63);
      uint32_t rel[4];
      uint32_t r = incl - sum, in = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        r += inc[k];
        rel[k] = r;
        in += q_base + r <= len ? 1u : 0u;
      }
      if (c <= kBernWaveGroups && lane == 0) gbase[c] = q_base;
      if (c < kBernWaveGroups) {
        const bool as_rel = adv < 0x10000u;
        put_incs(list + c * kBernWaveGroup + 4u * lane, as_rel ? rel : inc);
        rel_groups |= (as_rel ? 1u : 0u) << c;
      }
      const unsigned long long whole = __ballot(in == 4u);
      const uint32_t nw = static_cast<uint32_t>(__popcll(whole));
      const uint32_t got = nw == 64u ? kBernWaveGroup : 4u * nw + __builtin_amdgcn_readlane(in, nw);
      cnt += got;
      q_base += adv;
      if (got < kBernWaveGroup) break;
    }
    const uint64_t first = bern_lookback(status, j, cnt, ctl, help_polls, [&](uint64_t i) {
      const uint64_t bi = i * chunk;
      return static_cast<uint64_t>(bern_count32_wave(
          make_stream(seed, i, kBChunk, 0),
          static_cast<uint32_t>((N - bi) < chunk ? (N - bi) : chunk), c32, lane));
    });
    if (lane == 0 && j == n_chunks - 1) {
      *count_dev = first + cnt;
      ctl->bern_count = first + cnt;
    }
    // one 256-draw group per step: lane l takes hits k0 + 64s + l (s < 4);
    // qb: position before the group
    uint32_t qrun = 0;  // position before the next recomputed group
    for (uint32_t k0 = 0; k0 < cnt; k0 += kBernWaveGroup) {
      const uint32_t c = k0 / kBernWaveGroup;
      uint32_t sbase = k0;  // list index of hit k0
      bool as_rel = false;
      uint32_t qb;
      if (c < kBernWaveGroups) {
        qb = gbase[c];
        as_rel = (rel_groups >> c) & 1u;
      } else {
        if (c == kBernWaveGroups) qrun = gbase[c];
        uint32_t inc[4];
        const uint32_t sum = bern_group(st, c, lane, c32, inc);
        put_incs(list + kSpare + 4u * lane, inc);
        qb = qrun;
        qrun += __builtin_amdgcn_readlane(wave_scan_incl(sum), 63);
        sbase = kSpare;
      }
      uint32_t v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint32_t k = k0 + 64u * t + lane;
        // list indices stay inside the list; values past the last hit are
        // dropped here
        const uint32_t x = list[sbase + 64u * t + lane];
        v[t] = k < cnt ? x : 0u;
      }
      if (as_rel) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const uint32_t k = k0 + 64u * t + lane;
          if (k < cnt && first + k < capacity) store_out(out + first + k, base + qb + v[t]);
        }
      } else {
        uint32_t incl[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) incl[t] = wave_scan_incl(v[t]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const uint32_t k = k0 + 64u * t + lane;
          if (k < cnt && first + k < capacity) store_out(out + first + k, base + qb + incl[t]);
          qb += __builtin_amdgcn_readlane(incl[t], 63);
        }
      }
    }
  }
}

__global__ void k_bern_fill(uint64_t N, uint64_t* out, uint64_t capacity, uint64_t* count_dev) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  const uint64_t lim = N < capacity ? N : capacity;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < lim; i += stride)
    store_out(out + i, i + 1);
  if (blockIdx.x == 0 && threadIdx.x == 0) *count_dev = N;
}

// ---------------------------------------------------------------------------
// Whole-range Algorithm B (Sec. 2's Algorithm B over all of 0..N-1 with the
// skips and prefix sums of Sec. 4.7, as Sec. 5's GPU variant runs it, with
// the removal of the excess hits done on the device instead of the host).
// One attempt is three launches: a count pass (one wave per chunk, skips
// only), one work-group that scans the chunk counts, decides acceptance,
// draws the removed hit indices in rounds into a bitmap and scans the
// per-chunk removal counts, and a write pass that recomputes each chunk and
// writes its kept hits at their final places.
// ---------------------------------------------------------------------------
constexpr int kWbMidBlock = 1024;

__global__ void k_wb_zero(Control* ctl, WbBuffers b, unsigned int* err) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  const uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (uint64_t i = i0; i < b.words; i += stride) b.bitmap[i] = 0;
  for (uint64_t i = i0; i < b.rem_blocks; i += stride) b.rem[i] = 0;
  if (i0 == 0) {
    b.state->accepted = 0;
    b.state->hits = 0;
    b.state->pending = 0;
    b.state->fresh = 0;
    start_control(ctl, err);
  }
}

// Count pass: chunk j's hits counted 256 draws at a time exactly as
// k_bern_wave counts them (chunks dealt statically, one wave each).
__global__ __launch_bounds__(64) void k_wb_count(uint64_t N, uint64_t seed, uint64_t chunk,
                                                 uint64_t n_chunks, float c32, int full,
                                                 uint32_t attempt, WbBuffers b) {
  if (b.state->accepted != 0) return;  // an earlier attempt was accepted
  const uint32_t lane = lane_tid();
  for (uint64_t j = blockIdx.x; j < n_chunks; j += gridDim.x) {
    const uint64_t base = j * chunk;
    const uint32_t len = static_cast<uint32_t>((N - base) < chunk ? (N - base) : chunk);
    if (full) {
      if (lane == 0) b.cnt[j] = len;
      continue;
    }
    const Stream st = make_stream(seed, j, kWChunk, attempt);
    uint32_t q_base = 0, cnt = 0;
    for (uint32_t c = 0;; ++c) {
      uint32_t inc[4];
      const uint32_t sum = bern_group(st, c, lane, c32, inc);
      const uint32_t incl = wave_scan_incl(sum);
      uint32_t r = incl - sum, in = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        r += inc[k];
        in += q_base + r <= len ? 1u : 0u;
      }
      const unsigned long long whole = __ballot(in == 4u);
      const uint32_t nw = static_cast<uint32_t>(__popcll(whole));
      const uint32_t got = nw == 64u ? kBernWaveGroup : 4u * nw + __builtin_amdgcn_readlane(in, nw);
      cnt += got;
      q_base += __builtin_amdgcn_readlane(incl, 63);
      if (got < kBernWaveGroup) break;
    }
    if (lane == 0) b.cnt[j] = cnt;
  }
}

// The scan / acceptance / repair step of an attempt.  The chunk counts'
// exclusive prefix (each chunk's first hit index) and the hit total come
// from a tiled scan (k_wb_tile_sums, k_wb_mid, k_wb_tile_apply); k_wb_mid
// also takes the acceptance test and marks an accepted attempt pending.  The
// removed hit indices are the first r = n' - n distinct non-void values of
// the (0, WREPAIR, attempt) words mapped into [0, n'), found in rounds (each
// round takes as many more words as values are missing; a word adds at most
// one new value, so the rounds stop exactly where the sequential rule does);
// a value is new iff its bitmap bit was clear, and then its block's removal
// count goes up.  k_wb_repair1 (many work-groups) takes the first round,
// words [0, r): the bitmap makes the set of new values and their count
// independent of the order of the words' atomics.  k_wb_finish (one
// work-group) takes the later rounds from word r and marks the attempt
// accepted; a second tiled scan (k_wb_tile_sums, k_wb_rem_top,
// k_wb_tile_apply) turns the removal counts per block into their exclusive
// prefix before the write pass.

// Per-tile sums of x[0..count) (tile = one work-group of kWbMidBlock
// threads, 4 entries each).  after = 0: runs while no attempt is accepted;
// after = 1: runs for the accepted attempt `attempt`.
__global__ __launch_bounds__(kWbMidBlock) void k_wb_tile_sums(const uint32_t* x, uint64_t count,
                                                              uint64_t* sums, WbBuffers b,
                                                              uint32_t attempt, int after) {
  __shared__ uint64_t scr[kWbMidBlock / 64];
  static_assert(kWbTile == 4 * kWbMidBlock, "four entries per thread");
  if (after ? b.state->accepted != attempt + 1 : b.state->accepted != 0) return;
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kWbTile + 4u * threadIdx.x;
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += i + k < count ? x[i + k] : 0u;
  uint64_t total;
  (void)block_scan_excl<kWbMidBlock, uint64_t, false>(s, scr, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// y[i] = exclusive prefix of x at i: the tile's own scan plus its sum's
// prefix (sums already scanned).  after = 0: the attempt that passed the
// acceptance test; after = 1: the accepted attempt.  x may be y.
template <typename TOut>
__global__ __launch_bounds__(kWbMidBlock) void k_wb_tile_apply(const uint32_t* x, TOut* y,
                                                               uint64_t count,
                                                               const uint64_t* sums, WbBuffers b,
                                                               uint32_t attempt, int after) {
  __shared__ uint64_t scr[kWbMidBlock / 64];
  if (after ? b.state->accepted != attempt + 1
            : (b.state->accepted != 0 || b.state->pending != attempt + 1))
    return;
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kWbTile + 4u * threadIdx.x;
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = i + k < count ? x[i + k] : 0u;
  const uint64_t s = static_cast<uint64_t>(v[0]) + v[1] + v[2] + v[3];
  uint64_t total;
  uint64_t run = sums[blockIdx.x] + block_scan_excl<kWbMidBlock, uint64_t, false>(s, scr, &total);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i + k < count) y[i + k] = static_cast<TOut>(run);
    run += v[k];
  }
}

// Exclusive scan of sums[0..tiles) in place (one work-group, tiles <=
// kWbMidBlock); returns the total in every thread.
__device__ uint64_t wb_scan_sums(uint64_t* sums, uint32_t tiles, uint64_t* scr) {
  const uint32_t tid = threadIdx.x;
  const uint64_t v = tid < tiles ? sums[tid] : 0;
  uint64_t total;
  const uint64_t e = block_scan_excl<kWbMidBlock, uint64_t>(v, scr, &total);
  if (tid < tiles) sums[tid] = e;
  return total;
}

// Scan of the chunks' tile sums and the acceptance test (one work-group);
// an accepted attempt is marked pending with its hit count.
__global__ __launch_bounds__(kWbMidBlock) void k_wb_mid(uint64_t n, uint32_t tiles,
                                                        uint32_t attempt, int last, WbBuffers b,
                                                        Control* ctl) {
  __shared__ uint64_t scr[kWbMidBlock / 64];
  if (b.state->accepted != 0) return;
  const uint32_t tid = threadIdx.x;
  const uint64_t hits = wb_scan_sums(b.tsum, tiles, scr);
  const uint64_t hi = n + 16 * isqrt64(n) + 64;
  if (hits < n || hits > hi) {  // the same decision in every thread
    if (last && tid == 0) atomicOr(ctl->err, kErrRestartLimit);
    return;
  }
  if (tid == 0) {
    b.state->hits = hits;
    b.state->pending = attempt + 1;
  }
}

// Scan of the removal counts' tile sums for the accepted attempt.
__global__ __launch_bounds__(kWbMidBlock) void k_wb_rem_top(uint32_t tiles, uint32_t attempt,
                                                            WbBuffers b) {
  __shared__ uint64_t scr[kWbMidBlock / 64];
  if (b.state->accepted != attempt + 1) return;
  (void)wb_scan_sums(b.tsum + kWbMaxTiles, tiles, scr);
}

// The first repair round of a pending attempt over the whole grid; each wave
// adds its count of new values to state->fresh.
__global__ __launch_bounds__(256) void k_wb_repair1(uint64_t n, uint64_t seed, uint32_t attempt,
                                                    WbBuffers b) {
  if (b.state->accepted != 0 || b.state->pending != attempt + 1) return;
  const uint64_t hits = b.state->hits;
  const uint64_t r = hits - n;
  const Stream st = make_stream(seed, 0, kWRepair, attempt);
  const uint32_t thr = range_threshold(hits);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  uint32_t fresh = 0;
  for (uint64_t blk = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; (blk << 2) < r;
       blk += stride) {
    const uint4 w = philox_block(st, static_cast<uint32_t>(blk));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t tk = (blk << 2) + k;
      uint32_t v;
      if (tk < r && range_map(pick(w, k), hits, thr, &v)) {
        const unsigned long long bit = 1ull << (v & 63u);
        const unsigned long long old = atomicOr(&b.bitmap[v >> 6], bit);
        if ((old & bit) == 0) {
          ++fresh;
          atomicAdd(&b.rem[v >> kWbRemShift], 1u);
        }
      }
    }
  }
  const uint32_t sum = __builtin_amdgcn_readlane(wave_scan_incl(fresh), 63);
  if ((threadIdx.x & 63u) == 0 && sum != 0)
    atomicAdd(&b.state->fresh, static_cast<unsigned long long>(sum));
}

__global__ __launch_bounds__(kWbMidBlock) void k_wb_finish(uint64_t n, uint64_t seed,
                                                           uint32_t attempt, WbBuffers b) {
  __shared__ uint64_t scr[kWbMidBlock / 64];
  if (b.state->accepted != 0 || b.state->pending != attempt + 1) return;
  const uint32_t tid = threadIdx.x;
  const uint64_t hits = b.state->hits;
  const uint64_t r = hits - n;
  uint64_t d = b.state->fresh;  // new values of the first round, words [0, r)
  if (d < r) {
    const Stream st = make_stream(seed, 0, kWRepair, attempt);
    const uint32_t thr = range_threshold(hits);
    uint64_t t = r;
    while (d < r) {
      const uint64_t t1 = t + (r - d);
      uint64_t fresh = 0;
      for (uint64_t blk = (t >> 2) + tid; (blk << 2) < t1; blk += kWbMidBlock) {
        const uint4 w = philox_block(st, static_cast<uint32_t>(blk));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint64_t tk = (blk << 2) + k;
          uint32_t v;
          if (tk >= t && tk < t1 && range_map(pick(w, k), hits, thr, &v)) {
            const unsigned long long bit = 1ull << (v & 63u);
            const unsigned long long old = atomicOr(&b.bitmap[v >> 6], bit);
            if ((old & bit) == 0) {
              ++fresh;
              atomicAdd(&b.rem[v >> kWbRemShift], 1u);
            }
          }
        }
      }
      uint64_t total;
      (void)block_scan_excl<kWbMidBlock, uint64_t>(fresh, scr, &total);
      d += total;
      t = t1;
    }
  }
  if (tid == 0) b.state->accepted = attempt + 1;  // the removal counts are final
}

// Write pass: chunk j again, group by group.  Its hits have global indices
// off[j] .. ; the removals before its first hit are the prefix of its
// index block plus the bitmap bits between the block's start and off[j]
// (at most 2^kWbRemShift / 64 words).  Hit g, unless removed, goes to output
// index g - (removals before g); a group's kept hits are staged in LDS in
// order and stored with consecutive lanes on consecutive outputs.
__global__ __launch_bounds__(64) void k_wb_write(uint64_t N, uint64_t seed, uint64_t chunk,
                                                 uint64_t n_chunks, float c32, int full,
                                                 uint32_t attempt, WbBuffers b, uint64_t* out) {
  __shared__ uint64_t stage[kBernWaveGroup];
  if (b.state->accepted != attempt + 1) return;  // not this attempt's sample
  const uint32_t lane = lane_tid();
  for (uint64_t j = blockIdx.x; j < n_chunks; j += gridDim.x) {
    const uint64_t base = j * chunk;
    const uint32_t len = static_cast<uint32_t>((N - base) < chunk ? (N - base) : chunk);
    const uint64_t g0 = b.off[j];
    // removals before g0: whole blocks, then the words of g0's block below g0
    const uint64_t blk0 = g0 >> kWbRemShift;
    uint64_t before = 0;
    const uint64_t w_first = (blk0 << kWbRemShift) >> 6, w_end = g0 >> 6;  // words [w_first, w_end)
    for (uint64_t w = w_first + lane; w < w_end; w += 64)
      before += static_cast<uint64_t>(__popcll(b.bitmap[w]));
    if (lane == 0 && (g0 & 63u) != 0)
      before += static_cast<uint64_t>(__popcll(b.bitmap[w_end] & ~(~0ull << (g0 & 63u))));
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) before += __shfl_xor(before, d, 64);
    before += b.state->hits > g0 ? b.rem[blk0] : 0u;
    uint64_t o = g0 - before;  // output index of the chunk's next kept hit
    const Stream st = make_stream(seed, j, kWChunk, attempt);
    uint32_t q_base = 0;
    for (uint32_t c = 0;; ++c) {
      uint32_t inc[4] = {1u, 1u, 1u, 1u};
      uint32_t sum = 4u;
      if (!full) sum = bern_group(st, c, lane, c32, inc);
      const uint32_t incl = wave_scan_incl(sum);
      uint32_t rel[4];
      uint32_t r = incl - sum, in = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        r += inc[k];
        rel[k] = r;
        in += q_base + r <= len ? 1u : 0u;
      }
      // removal bits of this lane's hits 256c + 4 lane + k (consecutive
      // indices: at most two bitmap words)
      const uint64_t gl = g0 + kBernWaveGroup * c + 4u * lane;
      uint32_t keep = 0;
      if (in > 0) {
        const unsigned long long w0 = b.bitmap[gl >> 6];
        const uint32_t sh = static_cast<uint32_t>(gl & 63u);
        unsigned long long bits = w0 >> sh;
        if (sh > 60u && in > 64u - sh) bits |= b.bitmap[(gl >> 6) + 1] << (64u - sh);
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k)
          if (k < in && ((bits >> k) & 1ull) == 0) keep |= 1u << k;
      }
      const uint32_t nk = static_cast<uint32_t>(__popc(keep));
      const uint32_t kincl = wave_scan_incl(nk);
      uint32_t slot = kincl - nk;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((keep >> k) & 1u) stage[slot++] = base + q_base + rel[k];
      const uint32_t kept = __builtin_amdgcn_readlane(kincl, 63);
#pragma unroll
      for (uint32_t t = 0; t < 4; ++t) {
        const uint32_t idx = 64u * t + lane;
        if (idx < kept) store_out(out + o + idx, stage[idx]);
      }
      o += kept;
      const unsigned long long whole = __ballot(in == 4u);
      q_base += __builtin_amdgcn_readlane(incl, 63);
      if (__popcll(whole) < 64) break;
    }
  }
}

// ---------------------------------------------------------------------------
// Diagnostics kernel.
// ---------------------------------------------------------------------------
__global__ void k_debug(int op, const void* x, const void* x2, void* y, uint64_t count,
                        uint64_t p0, uint64_t p1, uint64_t p2, uint64_t p3) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  switch (op) {
    case 0: static_cast<double*>(y)[i] = log64(static_cast<const double*>(x)[i]); break;
    case 1: static_cast<double*>(y)[i] = log1p64(static_cast<const double*>(x)[i]); break;
    case 2: static_cast<float*>(y)[i] = log32(static_cast<const float*>(x)[i]); break;
    case 3: static_cast<double*>(y)[i] = __builtin_sqrt(static_cast<const double*>(x)[i]); break;
    case 4:
      static_cast<double*>(y)[i] =
          static_cast<const double*>(x)[i] / static_cast<const double*>(x2)[i];
      break;
    case 5:
      static_cast<double*>(y)[i] = lnfact_diff(static_cast<const uint64_t*>(x)[i],
                                               static_cast<const uint64_t*>(x2)[i]);
      break;
    case 6:
      static_cast<uint64_t*>(y)[i] =
          hypergeometric(p0, p1, p2, p3, static_cast<const uint64_t*>(x)[i]);
      break;
    case 7:
      static_cast<uint64_t*>(y)[i] = binomial(p0, p1, p2, p3, static_cast<const uint64_t*>(x)[i]);
      break;
    case 8: {
      const uint32_t* c = static_cast<const uint32_t*>(x) + 4 * i;
      Stream s;
      s.k0 = static_cast<uint32_t>(p0);
      s.k1 = static_cast<uint32_t>(p1);
      s.c1 = c[1];
      s.c2 = c[2];
      s.c3 = c[3];
      const uint4 b = philox_block(s, c[0]);
      uint32_t* o = static_cast<uint32_t*>(y) + 4 * i;
      o[0] = b.x; o[1] = b.y; o[2] = b.z; o[3] = b.w;
      break;
    }
    case 9:
      static_cast<float*>(y)[i] = geom_unit(static_cast<const uint32_t*>(x)[i]);
      break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// The library's error words (zero at load; see error_slots).
static __device__ unsigned int g_err_slots[kErrSlots];

hipError_t error_slots(unsigned int** out) {
  return hipGetSymbolAddress(reinterpret_cast<void**>(out), HIP_SYMBOL(g_err_slots));
}

hipError_t launch_reset(Control* ctl, const Instance* single, Instance* table, unsigned int* err,
                        uint32_t* redo, uint64_t redo_words, uint64_t* out, hipStream_t stream) {
  Instance one{};
  if (single) one = *single;
  if (redo == nullptr) redo_words = 0;
  uint64_t blocks = (redo_words + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_reset, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, ctl, one,
                     single ? 1 : 0, table, err, redo, redo_words, out);
  return hipGetLastError();
}

hipError_t launch_zero(Control* ctl, unsigned long long* status, uint64_t n,
                       unsigned long long* tickets, unsigned int* err, hipStream_t stream) {
  uint64_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, ctl, status, n,
                     tickets, err);
  return hipGetLastError();
}

int leaf_occupancy() {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, reinterpret_cast<const void*>(k_leaf_mixed<kLeafBlock>), kLeafBlock, 0) != hipSuccess ||
      occ <= 0)
    occ = 2;
  return occ;
}

int small_occupancy() {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, reinterpret_cast<const void*>(k_leaf_small), 64, 0) != hipSuccess ||
      occ <= 0)
    occ = 8;
  return occ;
}

hipError_t launch_leaf_small(const Leaf* leaves, uint64_t leaf_cap, uint64_t* out, Control* ctl,
                             uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_leaf_small, dim3(grid), dim3(64), 0, stream, leaves, leaf_cap, out, ctl);
  return hipGetLastError();
}

int dense_occupancy() {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, reinterpret_cast<const void*>(k_leaf_dense), 64, 0) != hipSuccess ||
      occ <= 0)
    occ = 8;
  return occ;
}

int bern_wave_occupancy() {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, reinterpret_cast<const void*>(k_bern_wave), 64, 0) != hipSuccess ||
      occ <= 0)
    occ = 8;
  return occ;
}

int bern64_wave_occupancy(uint32_t lds_cap) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, reinterpret_cast<const void*>(k_bern64_wave), 64,
          static_cast<size_t>(lds_cap) * sizeof(uint32_t)) != hipSuccess ||
      occ <= 0)
    occ = 1;
  return occ;
}

int bern_occupancy(uint32_t lds_cap) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, reinterpret_cast<const void*>(k_bern), kBernBlock,
          static_cast<size_t>(lds_cap) * sizeof(uint32_t)) != hipSuccess ||
      occ <= 0)
    occ = 1;
  return occ;
}

hipError_t launch_tree_top(const Instance* inst, uint32_t n_inst, uint64_t top_threads,
                           Node* frontier, Leaf* leaves, uint64_t leaf_cap, Control* ctl,
                           uint64_t* part_out, hipStream_t stream) {
  if (top_threads == 0) return hipSuccess;
  const uint64_t blocks = (top_threads * 64 + kTreeBlock - 1) / kTreeBlock;  // one wave per path
  hipLaunchKernelGGL(k_tree_top, dim3(static_cast<uint32_t>(blocks)), dim3(kTreeBlock), 0, stream, inst,
                     n_inst, top_threads, frontier, leaves, leaf_cap, ctl, part_out);
  return hipGetLastError();
}

hipError_t launch_tree(const Instance* inst, uint32_t n_inst, uint64_t total_threads,
                       const Node* frontier, Leaf* leaves, uint64_t leaf_cap, Node* stacks,
                       uint32_t stack_depth, Control* ctl, uint32_t* redo, int round,
                       hipStream_t stream) {
  if (total_threads == 0) return hipSuccess;
  if (round != 0 && redo == nullptr) return hipErrorInvalidValue;
  const uint64_t blocks = (total_threads + kTreeBlock - 1) / kTreeBlock;
  hipLaunchKernelGGL(k_tree, dim3(static_cast<uint32_t>(blocks)), dim3(kTreeBlock), 0, stream, inst,
                     n_inst, total_threads, frontier, leaves, leaf_cap, stacks, stack_depth, ctl,
                     redo, round);
  return hipGetLastError();
}

hipError_t launch_leaf(int which, const Leaf* leaves, uint64_t leaf_cap, uint64_t* out,
                       Control* ctl, uint32_t grid, hipStream_t stream, uint32_t takes) {
  if (which == kLeafFront)
    hipLaunchKernelGGL(k_leaf_pow2<kLeafBlock>, dim3(grid), dim3(kLeafBlock), 0, stream, leaves,
                       leaf_cap, out, ctl);
  else if (which == kLeafBack)
    hipLaunchKernelGGL(k_leaf_mixed<kLeafBlock>, dim3(grid), dim3(kLeafBlock), 0, stream, leaves,
                       leaf_cap, out, ctl, 0, takes);
  else if (which == kLeafOnce)
    hipLaunchKernelGGL(k_leaf_once<kLeafBlock>, dim3(grid), dim3(kLeafBlock), 0, stream, leaves,
                       leaf_cap, out, ctl, 0);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_leaf_round2(const Leaf* leaves, uint64_t leaf_cap, uint64_t* out, Control* ctl,
                              uint32_t grid, hipStream_t stream, uint32_t takes) {
  hipLaunchKernelGGL(k_leaf_mixed<kLeafBlock>, dim3(grid), dim3(kLeafBlock), 0, stream, leaves,
                     leaf_cap, out, ctl, 1, takes & kTakesOnce);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || (takes & kTakesOnce)) return e;
  hipLaunchKernelGGL(k_leaf_once<kLeafBlock>, dim3(grid), dim3(kLeafBlock), 0, stream, leaves,
                     leaf_cap, out, ctl, 1);
  return hipGetLastError();
}

hipError_t launch_part_roots(const Instance& I, uint32_t depth, Node* roots, hipStream_t stream) {
  const uint64_t parts = 1ull << depth;
  const uint64_t blocks = (parts + 255) / 256;
  hipLaunchKernelGGL(k_part_roots, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, I,
                     depth, parts, roots);
  return hipGetLastError();
}

hipError_t launch_leaf_dense(const Leaf* leaves, uint64_t leaf_cap, uint64_t* out, Control* ctl,
                             uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_leaf_dense, dim3(grid), dim3(64), 0, stream, leaves, leaf_cap, out, ctl);
  return hipGetLastError();
}

hipError_t launch_bernoulli(double p, uint64_t N, uint64_t seed, uint64_t chunk, uint64_t n_chunks,
                            int fp32, double c64, float c32, unsigned long long* status,
                            uint64_t* out, uint64_t capacity, uint64_t* count_dev, Control* ctl,
                            unsigned long long* tickets, uint32_t grid, uint32_t lds_cap,
                            uint32_t help_polls, hipStream_t stream) {
  (void)p;
  const uint32_t n_cls = grid < kTicketClasses ? grid : kTicketClasses;
  if (fp32 == kBernFp32Wave)
    hipLaunchKernelGGL(k_bern_wave, dim3(grid), dim3(64), 0, stream, N, seed, chunk, n_chunks, c32,
                       status, out, capacity, count_dev, ctl, tickets, n_cls, help_polls);
  else if (fp32 == kBernFp64Wave)
    hipLaunchKernelGGL(k_bern64_wave, dim3(grid), dim3(64),
                       static_cast<size_t>(lds_cap) * sizeof(uint32_t), stream, N, seed, chunk,
                       n_chunks, c64, status, out, capacity, count_dev, ctl, lds_cap, tickets,
                       n_cls, help_polls);
  else
    hipLaunchKernelGGL(k_bern, dim3(grid), dim3(kBernBlock),
                       static_cast<size_t>(lds_cap) * sizeof(uint32_t), stream, N, seed, chunk,
                       n_chunks, c64, status, out, capacity, count_dev, ctl, lds_cap, tickets,
                       n_cls, help_polls);
  return hipGetLastError();
}

hipError_t launch_segments(Instance* inst, uint64_t K, uint32_t D, uint64_t n, uint64_t N,
                           uint64_t seed, uint64_t* counts, hipStream_t stream) {
  const uint64_t blocks = (K + 255) / 256;
  hipLaunchKernelGGL(k_segments, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, inst,
                     K, D, n, N, seed, counts);
  return hipGetLastError();
}

hipError_t launch_wb_zero(Control* ctl, const WbBuffers& b, uint64_t n_chunks, unsigned int* err,
                          hipStream_t stream) {
  (void)n_chunks;
  const uint64_t most = b.words > b.rem_blocks ? b.words : b.rem_blocks;
  uint64_t blocks = (most + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_wb_zero, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, ctl, b,
                     err);
  return hipGetLastError();
}

hipError_t launch_wb_count(uint64_t N, uint64_t seed, uint64_t chunk, uint64_t n_chunks, float c32,
                           int full, uint32_t attempt, const WbBuffers& b, uint32_t grid,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_wb_count, dim3(grid), dim3(64), 0, stream, N, seed, chunk, n_chunks, c32,
                     full, attempt, b);
  return hipGetLastError();
}

hipError_t launch_wb_mid(uint64_t n, uint64_t seed, uint64_t n_chunks, uint32_t attempt, int last,
                         const WbBuffers& b, Control* ctl, uint32_t repair_grid,
                         hipStream_t stream) {
  const uint64_t ct = wb_tiles(n_chunks), rt = wb_tiles(b.rem_blocks);
  if (ct == 0 || ct > kWbMaxTiles || rt == 0 || rt > kWbMaxTiles) return hipErrorInvalidValue;
  const dim3 blk(kWbMidBlock);
  hipLaunchKernelGGL(k_wb_tile_sums, dim3(static_cast<uint32_t>(ct)), blk, 0, stream, b.cnt,
                     n_chunks, b.tsum, b, attempt, 0);
  hipLaunchKernelGGL(k_wb_mid, dim3(1), blk, 0, stream, n, static_cast<uint32_t>(ct), attempt,
                     last, b, ctl);
  hipLaunchKernelGGL(k_wb_tile_apply<uint64_t>, dim3(static_cast<uint32_t>(ct)), blk, 0, stream,
                     b.cnt, b.off, n_chunks, b.tsum, b, attempt, 0);
  hipLaunchKernelGGL(k_wb_repair1, dim3(repair_grid), dim3(256), 0, stream, n, seed, attempt, b);
  hipLaunchKernelGGL(k_wb_finish, dim3(1), blk, 0, stream, n, seed, attempt, b);
  hipLaunchKernelGGL(k_wb_tile_sums, dim3(static_cast<uint32_t>(rt)), blk, 0, stream, b.rem,
                     b.rem_blocks, b.tsum + kWbMaxTiles, b, attempt, 1);
  hipLaunchKernelGGL(k_wb_rem_top, dim3(1), blk, 0, stream, static_cast<uint32_t>(rt), attempt, b);
  hipLaunchKernelGGL(k_wb_tile_apply<uint32_t>, dim3(static_cast<uint32_t>(rt)), blk, 0, stream,
                     b.rem, b.rem, b.rem_blocks, b.tsum + kWbMaxTiles, b, attempt, 1);
  return hipGetLastError();
}

hipError_t launch_wb_write(uint64_t N, uint64_t seed, uint64_t chunk, uint64_t n_chunks, float c32,
                           int full, uint32_t attempt, const WbBuffers& b, uint64_t* out,
                           uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_wb_write, dim3(grid), dim3(64), 0, stream, N, seed, chunk, n_chunks, c32,
                     full, attempt, b, out);
  return hipGetLastError();
}

int wb_occupancy() {
  int a = 0, b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &a, reinterpret_cast<const void*>(k_wb_count), 64, 0) != hipSuccess || a <= 0)
    a = 8;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &b, reinterpret_cast<const void*>(k_wb_write), 64, 0) != hipSuccess || b <= 0)
    b = 8;
  return a < b ? a : b;
}

hipError_t launch_bernoulli_fill(uint64_t N, uint64_t* out, uint64_t capacity, uint64_t* count_dev,
                                 hipStream_t stream) {
  hipLaunchKernelGGL(k_bern_fill, dim3(1024), dim3(256), 0, stream, N, out, capacity, count_dev);
  return hipGetLastError();
}

hipError_t launch_debug(int op, const void* x, const void* x2, void* y, uint64_t count,
                        uint64_t p0, uint64_t p1, uint64_t p2, uint64_t p3, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  const uint64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_debug, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, op, x,
                     x2, y, count, p0, p1, p2, p3);
  return hipGetLastError();
}

}  // namespace dcs
