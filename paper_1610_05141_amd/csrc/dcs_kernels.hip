// dcs_kernels.hip -- the sampler's kernels for gfx950.
//
//   k_reset      zero a workspace control block
//   k_tree       recursion tree: each thread follows one root-to-depth-`cut`
//                path of Algorithm R, recomputing the splits on the way
//                exactly as a processing element of Algorithm P does
//                (paper Sec. 3.2, Fig. 2), then expands the subtree below by
//                a depth-first walk; every leaf becomes a job.
//   k_leaf       persistent work-groups take leaf jobs from an atomic ticket
//                (the atomic jobs of Sec. 4.2) and run the base case:
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
#include "dcs_device.hpp"
#include "dcs_kernels.hpp"

namespace dcs {

// ---------------------------------------------------------------------------
// Small block-wide helpers (kLeafBlock threads = 4 waves of 64).
// ---------------------------------------------------------------------------
constexpr int kWaves = kLeafBlock / 64;

// Exclusive prefix sum over the block of one value per thread; *total gets
// the block sum.  `scratch` holds kWaves words of LDS.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* scratch,
                                                    uint32_t* total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) scratch[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t s = scratch[w];
    before += (w < wave) ? s : 0u;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

__device__ __forceinline__ uint64_t block_scan_excl64(uint64_t v, uint64_t* scratch,
                                                      uint64_t* total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) scratch[wave] = x;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint64_t s = scratch[w];
    before += (w < wave) ? s : 0ull;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

__device__ __forceinline__ uint32_t bit_length(uint64_t x) {
  return x == 0 ? 0u : 64u - static_cast<uint32_t>(__clzll(static_cast<long long>(x)));
}

// ---------------------------------------------------------------------------
// LDS layout of a leaf work-group (32-bit words).
//   [0, kRegionA)           sparse: keys | tmp      dense: positions
//   [kRegionA, +kRegionB)   sparse: bucket counts   dense: kept values
//   then mask words and a little scratch.
// ---------------------------------------------------------------------------
constexpr uint32_t kKeys = kMaxN0;                   // 4096 keys
constexpr uint32_t kDenseCap = 2 * kMaxN0 + 64;       // largest accepted n'
constexpr uint32_t kRegionA = 2 * kMaxN0 + 128;       // >= kDenseCap + 1
constexpr uint32_t kRegionB = kMaxN0;                 // buckets / kept values
constexpr uint32_t kMaskWords = (kDenseCap + 32) / 32 + 1;
constexpr uint32_t kSmemWords = kRegionA + kRegionB + kMaskWords + 32;

struct LeafSmem {
  uint32_t* keys;   // kKeys
  uint32_t* tmp;    // kKeys
  uint32_t* buck;   // kRegionB
  uint32_t* mask;   // kMaskWords
  uint32_t* scr;    // 32 words of scratch
};

// ---------------------------------------------------------------------------
// The first `need` non-void values of a 32-bit stream in [0, s), starting at
// word t0, delivered in stream order to sink(p, value) for p = 0..need-1.
// Returns the word index just after the last value taken.  Only as many
// words as could still be needed are generated (no voids assumed); a void
// costs one more round.
// ---------------------------------------------------------------------------
template <class Sink>
__device__ uint64_t take_values(const Stream& st, uint64_t t0, uint32_t need, uint64_t s,
                                uint32_t thr, bool pow2, uint32_t pshift, uint32_t* scr,
                                Sink sink) {
  if (need == 0) return t0;
  uint32_t done = 0;
  uint64_t t = t0;  // next word to examine
  uint64_t next = t0;
  while (done < need) {
    const uint32_t want = need - done;
    const uint64_t first_blk = t >> 2;
    // words [t, last_word) are examined this round: at most the blocks the
    // work-group covers, and no more words than values still wanted
    uint64_t last_word = t + want;
    const uint64_t reach = (first_blk + kLeafBlock) << 2;
    if (last_word > reach) last_word = reach;
    const uint64_t blk = first_blk + threadIdx.x;
    uint32_t v[4];
    uint32_t ok = 0;  // bit j: word j of this block is a value in range
    if ((blk << 2) < last_word) {
      const uint4 w = philox_block(st, static_cast<uint32_t>(blk));
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint64_t tj = (blk << 2) + j;
        const uint32_t word = pick(w, j);
        bool good;
        if (pow2) {
          v[j] = pshift >= 32 ? 0u : (word >> pshift);
          good = true;
        } else {
          good = range_map(word, s, thr, &v[j]);
        }
        if (good && tj >= t && tj < last_word) ok |= 1u << j;
      }
    }
    const uint32_t cnt = __popc(ok);
    uint32_t total;
    uint32_t p = done + block_scan_excl(cnt, scr, &total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (ok & (1u << j)) {
        if (p < need) {
          sink(p, v[j]);
          if (p == need - 1) scr[8] = static_cast<uint32_t>(((blk << 2) + j + 1) - t0);
        }
        ++p;
      }
    }
    done += total;
    t = last_word;
    __syncthreads();
  }
  next = t0 + scr[8];
  __syncthreads();
  return next;
}

// ---------------------------------------------------------------------------
// Counting sort of keys[0..n) by their top bits, then exact ranking inside
// each bucket; keys[] ends sorted ascending with equal values adjacent.
// Returns the number of entries equal to an earlier one (duplicates).
// shift: key >> shift is the bucket, nb buckets.
// ---------------------------------------------------------------------------
__device__ uint32_t bucket_sort(uint32_t* keys, uint32_t* tmp, uint32_t* buck, uint32_t* scr,
                                uint32_t n, uint32_t shift, uint32_t nb) {
  constexpr int R = kKeys / kLeafBlock;  // 16 keys per thread at most
  const uint32_t tid = threadIdx.x;
  for (uint32_t b = tid; b < nb; b += kLeafBlock) buck[b] = 0;
  if (tid == 0) scr[9] = 0;
  __syncthreads();
  uint32_t key[R];
  uint32_t slot[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = tid + r * kLeafBlock;
    if (i < n) {
      key[r] = keys[i];
      slot[r] = atomicAdd(&buck[key[r] >> shift], 1u);
    }
  }
  __syncthreads();
  // exclusive scan of the bucket counts: thread tid owns a contiguous run
  const uint32_t per = (nb + kLeafBlock - 1) / kLeafBlock;
  const uint32_t b0 = tid * per;
  uint32_t run = 0;
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t b = b0 + k;
    if (b < nb) run += buck[b];
  }
  uint32_t total;
  uint32_t acc = block_scan_excl(run, scr, &total);
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t b = b0 + k;
    if (b < nb) {
      const uint32_t c = buck[b];
      buck[b] = acc;
      acc += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = tid + r * kLeafBlock;
    if (i < n) tmp[buck[key[r] >> shift] + slot[r]] = key[r];
  }
  __syncthreads();
  uint32_t dups = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = tid + r * kLeafBlock;
    if (i < n) {
      const uint32_t x = tmp[i];
      const uint32_t b = x >> shift;
      const uint32_t s = buck[b];
      const uint32_t e = (b + 1 < nb) ? buck[b + 1] : n;
      uint32_t lt = 0, eq = 0;
      for (uint32_t j = s; j < e; ++j) {
        const uint32_t y = tmp[j];
        lt += (y < x) ? 1u : 0u;
        eq += (y == x && j < i) ? 1u : 0u;
      }
      keys[s + lt + eq] = x;
      dups += eq ? 1u : 0u;
    }
  }
  if (dups) atomicAdd(&scr[9], dups);
  __syncthreads();
  const uint32_t d = scr[9];
  __syncthreads();
  return d;
}

// keys[0..n) sorted with equal values adjacent -> distinct values in
// keys[0..d); returns d.
__device__ uint32_t compact_distinct(uint32_t* keys, uint32_t* tmp, uint32_t* scr, uint32_t n) {
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (n + kLeafBlock - 1) / kLeafBlock;
  const uint32_t i0 = tid * per;
  uint32_t c = 0;
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t i = i0 + k;
    if (i < n && (i == 0 || keys[i] != keys[i - 1])) ++c;
  }
  uint32_t total;
  uint32_t p = block_scan_excl(c, scr, &total);
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t i = i0 + k;
    if (i < n && (i == 0 || keys[i] != keys[i - 1])) tmp[p++] = keys[i];
  }
  __syncthreads();
  for (uint32_t i = tid; i < total; i += kLeafBlock) keys[i] = tmp[i];
  __syncthreads();
  return total;
}

__device__ __forceinline__ void store_out(uint64_t* out, uint64_t v) {
  __builtin_nontemporal_store(v, out);
}

// Write base + 1 + vals[i] for i < n, coalesced.
__device__ __forceinline__ void write_sorted(uint64_t* out, uint64_t base, const uint32_t* vals,
                                             uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += kLeafBlock)
    store_out(out + i, base + 1 + static_cast<uint64_t>(vals[i]));
}

struct RangeInfo {
  uint64_t s;
  uint32_t thr;
  bool pow2;
  uint32_t pshift;  // for pow2: value = word >> pshift
};

__device__ __forceinline__ RangeInfo range_info(uint64_t s) {
  RangeInfo r;
  r.s = s;
  r.pow2 = (s & (s - 1)) == 0;
  r.pshift = r.pow2 ? 32u - (bit_length(s) - 1u) : 0u;
  r.thr = r.pow2 ? 0u : range_threshold(s);
  return r;
}

// Bucket parameters for keys < range and about n keys.
__device__ __forceinline__ void bucket_params(uint64_t range, uint32_t n, uint32_t* shift,
                                              uint32_t* nb) {
  const uint32_t kb = bit_length(range - 1);
  uint32_t lb = bit_length(n > 1 ? n - 1 : 1);
  if (lb < 6) lb = 6;
  if (lb > 12) lb = 12;
  *shift = kb > lb ? kb - lb : 0u;
  const uint64_t used = ((range - 1) >> *shift) + 1;
  *nb = static_cast<uint32_t>(used);
}

// ---------------------------------------------------------------------------
// Sparse leaf: Algorithm H semantics.
// ---------------------------------------------------------------------------
__device__ void leaf_sparse(const Leaf& L, const Instance& I, uint64_t* out, LeafSmem& sm) {
  const uint32_t nv = static_cast<uint32_t>(L.nv);
  const RangeInfo ri = range_info(L.Nv);
  uint32_t shift, nb;
  bucket_params(L.Nv, nv, &shift, &nb);
  const Stream st = make_stream(I.seed, L.id, kLeaf, 0);
  uint32_t have = 0;
  uint64_t t = 0;
  uint32_t* keys = sm.keys;
  for (;;) {
    const uint32_t base = have;
    t = take_values(st, t, nv - have, ri.s, ri.thr, ri.pow2, ri.pshift, sm.scr,
                    [&](uint32_t p, uint32_t v) { keys[base + p] = v; });
    const uint32_t dups = bucket_sort(keys, sm.tmp, sm.buck, sm.scr, nv, shift, nb);
    if (dups == 0) break;
    have = compact_distinct(keys, sm.tmp, sm.scr, nv);
  }
  write_sorted(out + I.out_offset + L.off, L.lo, keys, nv);
}

// With-replacement leaf: the first n_v non-void draws, sorted, repeats kept.
__device__ void leaf_wr(const Leaf& L, const Instance& I, uint64_t* out, LeafSmem& sm) {
  const uint32_t nv = static_cast<uint32_t>(L.nv);
  const RangeInfo ri = range_info(L.Nv);
  uint32_t shift, nb;
  bucket_params(L.Nv, nv, &shift, &nb);
  const Stream st = make_stream(I.seed, L.id, kWrLeaf, 0);
  uint32_t* keys = sm.keys;
  take_values(st, 0, nv, ri.s, ri.thr, ri.pow2, ri.pshift, sm.scr,
              [&](uint32_t p, uint32_t v) { keys[p] = v; });
  bucket_sort(keys, sm.tmp, sm.buck, sm.scr, nv, shift, nb);
  write_sorted(out + I.out_offset + L.off, L.lo, keys, nv);
}

// ---------------------------------------------------------------------------
// Dense leaf: Algorithm B with geometric skips and repair.
// ---------------------------------------------------------------------------
__device__ void leaf_dense(const Leaf& L, const Instance& I, uint64_t* out, LeafSmem& sm) {
  const uint32_t tid = threadIdx.x;
  const uint32_t nv = static_cast<uint32_t>(L.nv);
  const uint32_t Nv = static_cast<uint32_t>(L.Nv);  // < 16 * 4096 here
  const uint32_t rho_num = nv + 3u * static_cast<uint32_t>(isqrt64(nv)) + 8u;
  const bool full = rho_num >= Nv;
  float cg = 0.0f;
  if (!full) {
    const float rho = static_cast<float>(rho_num) / static_cast<float>(Nv);
    cg = static_cast<float>(1.0 / log64(1.0 - static_cast<double>(rho)));
  }
  const uint32_t cap = 2u * I.n0 + 64u;
  uint32_t* pos = sm.keys;  // region A: up to kDenseCap + 1 positions
  uint32_t* kept = sm.buck; // region B: n_v kept values
  for (uint32_t attempt = 0;; ++attempt) {
    uint32_t hits;  // n'
    if (full) {
      hits = Nv;
    } else {
      const Stream st = make_stream(I.seed, L.id, kBern, attempt);
      int64_t last = -1;  // position of the last word of the previous round
      uint32_t count = 0;
      for (uint32_t blk0 = 0;; blk0 += kLeafBlock) {
        const uint4 w = philox_block(st, blk0 + tid);
        int32_t inc[4];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          inc[j] = geom_skip32(pick(w, j), cg) + 1;
          sum += static_cast<uint32_t>(inc[j]);
        }
        uint32_t total;
        const uint32_t before = block_scan_excl(sum, sm.scr, &total);
        int64_t p = last + static_cast<int64_t>(before);
        uint32_t in = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          p += inc[j];
          if (p < static_cast<int64_t>(Nv)) {
            ++in;
            const uint32_t idx = count + 4u * tid + j;  // stream index t = hit index
            if (idx <= cap) pos[idx] = static_cast<uint32_t>(p);
          }
        }
        // hits of this round: positions below Nv form a prefix of the round
        uint32_t tot_in;
        block_scan_excl(in, sm.scr, &tot_in);
        count += tot_in;
        last += static_cast<int64_t>(total);
        if (tot_in < 4u * kLeafBlock || count > cap) break;
      }
      hits = count;
      if (hits < nv || hits > cap) continue;
    }
    // Repair: remove the first (hits - nv) distinct values of the REPAIR
    // stream mapped into [0, hits).
    const uint32_t r = hits - nv;
    const uint32_t mwords = (hits + 31) / 32;
    for (uint32_t i = tid; i < mwords; i += kLeafBlock) sm.mask[i] = 0;
    __syncthreads();
    if (r > 0) {
      const Stream sr = make_stream(I.seed, L.id, kRepair, attempt);
      const RangeInfo ri = range_info(hits);
      uint32_t have = 0;
      uint64_t t = 0;
      for (;;) {
        t = take_values(sr, t, r - have, ri.s, ri.thr, ri.pow2, ri.pshift, sm.scr,
                        [&](uint32_t, uint32_t v) { atomicOr(&sm.mask[v >> 5], 1u << (v & 31)); });
        __syncthreads();
        uint32_t c = 0;
        for (uint32_t i = tid; i < mwords; i += kLeafBlock) c += __popc(sm.mask[i]);
        uint32_t total;
        block_scan_excl(c, sm.scr, &total);
        have = total;
        if (have == r) break;
      }
    }
    // Compact the kept hits (ascending position) into kept[0..nv).
    const uint32_t per = (hits + kLeafBlock - 1) / kLeafBlock;
    const uint32_t i0 = tid * per;
    uint32_t c = 0;
    for (uint32_t k = 0; k < per; ++k) {
      const uint32_t i = i0 + k;
      if (i < hits && !((sm.mask[i >> 5] >> (i & 31)) & 1u)) ++c;
    }
    uint32_t total;
    uint32_t o = block_scan_excl(c, sm.scr, &total);
    for (uint32_t k = 0; k < per; ++k) {
      const uint32_t i = i0 + k;
      if (i < hits && !((sm.mask[i >> 5] >> (i & 31)) & 1u)) kept[o++] = full ? i : pos[i];
    }
    __syncthreads();
    write_sorted(out + I.out_offset + L.off, L.lo, kept, nv);
    break;
  }
}

// Constant leaf of a with-replacement tree: N_v = 1, every draw is lo+1.
__device__ void leaf_fill(const Leaf& L, const Instance& I, uint64_t* out) {
  uint64_t* o = out + I.out_offset + L.off;
  for (uint64_t i = threadIdx.x; i < L.nv; i += kLeafBlock) store_out(o + i, L.lo + 1);
}

__global__ __launch_bounds__(kLeafBlock) void k_leaf(const Instance* __restrict__ inst,
                                                     const Leaf* __restrict__ leaves,
                                                     uint64_t leaf_cap, uint64_t* out,
                                                     Control* ctl) {
  __shared__ uint32_t smem[kSmemWords];
  __shared__ unsigned long long cur;
  LeafSmem sm;
  sm.keys = smem;
  sm.tmp = smem + kKeys;
  sm.buck = smem + kRegionA;
  sm.mask = smem + kRegionA + kRegionB;
  sm.scr = smem + kRegionA + kRegionB + kMaskWords;
  const unsigned long long n_leaves =
      ctl->leaf_count < leaf_cap ? ctl->leaf_count : static_cast<unsigned long long>(leaf_cap);
  for (;;) {
    if (threadIdx.x == 0) cur = atomicAdd(&ctl->leaf_ticket, 1ull);
    __syncthreads();
    const unsigned long long i = cur;
    __syncthreads();
    if (i >= n_leaves) break;
    const Leaf L = leaves[i];
    const Instance I = inst[L.inst];
    if (I.variant == 1) {
      if (L.Nv == 1)
        leaf_fill(L, I, out);
      else
        leaf_wr(L, I, out, sm);
    } else if (static_cast<uint64_t>(I.dense_ratio) * L.nv >= L.Nv) {
      leaf_dense(L, I, out, sm);
    } else {
      leaf_sparse(L, I, out, sm);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Tree kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool is_leaf(const Node& v, const Instance& I) {
  if (I.variant == 1 && v.Nv == 1) return true;
  return v.nv < I.n0 && v.Nv <= kLeafMaxRange;
}

__device__ __forceinline__ uint64_t split_left(const Node& v, const Instance& I) {
  const uint64_t l = v.Nv >> 1;
  return I.variant == 1 ? binomial(v.nv, l, v.Nv, I.seed, v.id)
                        : hypergeometric(v.nv, l, v.Nv, I.seed, v.id);
}

__device__ __forceinline__ void emit(const Node& v, uint32_t inst_idx, Leaf* leaves,
                                     uint64_t cap, Control* ctl) {
  uint64_t pieces = 1;
  if (v.Nv == 1 && v.nv > kFillPiece) pieces = (v.nv + kFillPiece - 1) / kFillPiece;
  const unsigned long long base = atomicAdd(&ctl->leaf_count, static_cast<unsigned long long>(pieces));
  for (uint64_t j = 0; j < pieces; ++j) {
    if (base + j >= cap) {
      atomicOr(&ctl->error, kErrLeafCapacity);
      return;
    }
    Leaf L;
    L.id = v.id;
    L.lo = v.lo;
    L.Nv = v.Nv;
    L.off = v.off + j * kFillPiece;
    L.nv = (pieces == 1) ? v.nv : ((j + 1 < pieces) ? kFillPiece : v.nv - j * kFillPiece);
    L.inst = inst_idx;
    L.pad = 0;
    leaves[base + j] = L;
  }
}

__global__ __launch_bounds__(256) void k_tree(const Instance* __restrict__ inst, uint32_t n_inst,
                                              uint64_t total_threads, Leaf* leaves,
                                              uint64_t leaf_cap, Node* stacks,
                                              uint32_t stack_depth, Control* ctl) {
  const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total_threads) return;
  uint32_t lo = 0, hi = n_inst;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (inst[mid].thread_base <= t) lo = mid; else hi = mid;
  }
  const Instance I = inst[lo];
  const uint64_t g = t - I.thread_base;
  Node v{1, 0, I.N, I.n, 0};
  // Algorithm P: the path to this thread's depth-`cut` node.
  for (uint32_t d = 0; d < I.cut; ++d) {
    if (v.nv == 0) return;
    if (is_leaf(v, I)) {
      const uint32_t below = I.cut - d;
      if ((g & ((1ull << below) - 1)) == 0) emit(v, lo, leaves, leaf_cap, ctl);
      return;
    }
    const uint64_t L = split_left(v, I);
    const uint64_t l = v.Nv >> 1;
    if ((g >> (I.cut - 1 - d)) & 1) {
      v = Node{2 * v.id + 1, v.lo + l, v.Nv - l, v.nv - L, v.off + L};
    } else {
      v = Node{2 * v.id, v.lo, l, L, v.off};
    }
  }
  // Depth-first expansion of the subtree (Algorithm R below depth `cut`).
  Node* stk = stacks + t * stack_depth;
  uint32_t sp = 0;
  for (;;) {
    for (;;) {
      if (v.nv == 0) break;
      if (is_leaf(v, I)) {
        emit(v, lo, leaves, leaf_cap, ctl);
        break;
      }
      const uint64_t L = split_left(v, I);
      const uint64_t l = v.Nv >> 1;
      const Node right{2 * v.id + 1, v.lo + l, v.Nv - l, v.nv - L, v.off + L};
      if (right.nv > 0) {
        if (sp == stack_depth) {
          atomicOr(&ctl->error, kErrStackDepth);
          return;
        }
        stk[sp++] = right;
      }
      v = Node{2 * v.id, v.lo, l, L, v.off};
    }
    if (sp == 0) break;
    v = stk[--sp];
  }
}

__global__ void k_reset(Control* ctl, Instance single, int has_single, Instance* table) {
  if (threadIdx.x == 0) {
    ctl->leaf_count = 0;
    ctl->leaf_ticket = 0;
    ctl->chunk_ticket = 0;
    ctl->bern_count = 0;
    if (has_single) table[0] = single;
  }
}

__global__ void k_zero(Control* ctl, unsigned long long* status, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    status[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->leaf_count = 0;
    ctl->leaf_ticket = 0;
    ctl->chunk_ticket = 0;
    ctl->bern_count = 0;
  }
}

// ---------------------------------------------------------------------------
// Bernoulli chunks (Sec. 4.7).
// ---------------------------------------------------------------------------
constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagIncl = 2ull << 62;
constexpr unsigned long long kValueMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 26;

// One pass over the chunk's geometric stream.  Hits i < lds_cap go to pos[]
// when write == false; when write == true, hits i >= lds_cap are written
// straight to out (the chunk held more hits than LDS).  Returns the count.
__device__ uint64_t bern_pass(const Stream& st, uint64_t len, int fp32, double c64, float c32,
                              uint32_t* pos, uint32_t lds_cap, bool write, uint64_t* out,
                              uint64_t out_first, uint64_t capacity, uint64_t base,
                              uint64_t* scr64, uint32_t* scr) {
  const uint32_t tid = threadIdx.x;
  int64_t last = -1;
  uint64_t count = 0;
  const uint32_t per = fp32 ? 4u : 2u;
  for (uint32_t blk0 = 0;; blk0 += kLeafBlock) {
    const uint4 w = philox_block(st, blk0 + tid);
    uint64_t inc[4];
    uint64_t sum = 0;
    if (fp32) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        inc[j] = static_cast<uint64_t>(geom_skip32(pick(w, j), c32)) + 1;
        sum += inc[j];
      }
    } else {
      const uint64_t d0 = static_cast<uint64_t>(w.x) | (static_cast<uint64_t>(w.y) << 32);
      const uint64_t d1 = static_cast<uint64_t>(w.z) | (static_cast<uint64_t>(w.w) << 32);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double g = floor(log64(unit_open0(j ? d1 : d0)) * c64);
        const double gc = g < 0x1p33 ? g : 0x1p33;  // anything >= 2^33 ends the chunk
        inc[j] = static_cast<uint64_t>(gc) + 1;
        sum += inc[j];
      }
      inc[2] = inc[3] = 0;
    }
    uint64_t total;
    const uint64_t before = block_scan_excl64(sum, scr64, &total);
    int64_t p = last + static_cast<int64_t>(before);
    uint32_t in = 0;
    for (uint32_t j = 0; j < per; ++j) {
      p += static_cast<int64_t>(inc[j]);
      if (p < static_cast<int64_t>(len)) {
        const uint64_t idx = count + per * tid + j;
        if (!write) {
          if (idx < lds_cap) pos[idx] = static_cast<uint32_t>(p);
        } else if (idx >= lds_cap && out_first + idx < capacity) {
          store_out(out + out_first + idx, base + static_cast<uint64_t>(p) + 1);
        }
        ++in;
      }
    }
    uint32_t tot_in;
    block_scan_excl(in, scr, &tot_in);
    count += tot_in;
    last += static_cast<int64_t>(total);
    if (tot_in < per * kLeafBlock) break;
  }
  return count;
}

__global__ __launch_bounds__(kLeafBlock) void k_bern(uint64_t N, uint64_t seed, uint64_t chunk,
                                                     uint64_t n_chunks, int fp32, double c64,
                                                     float c32, unsigned long long* status,
                                                     uint64_t* out, uint64_t capacity,
                                                     uint64_t* count_dev, Control* ctl,
                                                     uint32_t lds_cap) {
  __shared__ uint32_t pos[kRegionA + kRegionB];
  __shared__ uint32_t scr[32];
  __shared__ uint64_t scr64[8];
  __shared__ unsigned long long cur, excl;
  for (;;) {
    if (threadIdx.x == 0) cur = atomicAdd(&ctl->chunk_ticket, 1ull);
    __syncthreads();
    const unsigned long long j = cur;
    __syncthreads();
    if (j >= n_chunks) break;
    const uint64_t base = j * chunk;
    const uint64_t len = (N - base) < chunk ? (N - base) : chunk;
    const Stream st = make_stream(seed, j, kBChunk, 0);
    const uint64_t cnt = bern_pass(st, len, fp32, c64, c32, pos, lds_cap, false, out, 0,
                                   capacity, base, scr64, scr);
    if (threadIdx.x == 0) {
      unsigned long long acc = 0;
      if (j == 0) {
        __hip_atomic_store(&status[0], kFlagIncl | cnt, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(&status[j], kFlagAgg | cnt, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        long long i = static_cast<long long>(j) - 1;
        uint32_t spins = 0;
        while (i >= 0) {
          const unsigned long long s =
              __hip_atomic_load(&status[i], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          const unsigned long long flag = s & ~kValueMask;
          if (flag == 0) {
            if (++spins > kSpinLimit) {
              atomicOr(&ctl->error, kErrSpinLimit);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          acc += s & kValueMask;
          if (flag == kFlagIncl) break;
          --i;
        }
        __hip_atomic_store(&status[j], kFlagIncl | (acc + cnt), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      excl = acc;
      if (j == n_chunks - 1) {
        *count_dev = acc + cnt;
        ctl->bern_count = acc + cnt;
      }
    }
    __syncthreads();
    const uint64_t first = excl;
    const uint64_t held = cnt < lds_cap ? cnt : lds_cap;
    for (uint64_t i = threadIdx.x; i < held; i += kLeafBlock)
      if (first + i < capacity) store_out(out + first + i, base + static_cast<uint64_t>(pos[i]) + 1);
    if (cnt > lds_cap)
      bern_pass(st, len, fp32, c64, c32, pos, lds_cap, true, out, first, capacity, base, scr64, scr);
    __syncthreads();
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
hipError_t launch_reset(Control* ctl, const Instance* single, Instance* table, hipStream_t stream) {
  Instance one{};
  if (single) one = *single;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, ctl, one, single ? 1 : 0, table);
  return hipGetLastError();
}

hipError_t launch_zero(Control* ctl, unsigned long long* status, uint64_t n, hipStream_t stream) {
  uint64_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, ctl, status, n);
  return hipGetLastError();
}

int leaf_occupancy() {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_leaf),
                                                   kLeafBlock, 0) != hipSuccess || occ <= 0)
    occ = 2;
  return occ;
}

hipError_t launch_tree(const Instance* inst, uint32_t n_inst, uint64_t total_threads,
                       Leaf* leaves, uint64_t leaf_cap, Node* stacks, uint32_t stack_depth,
                       Control* ctl, hipStream_t stream) {
  if (total_threads == 0) return hipSuccess;
  const uint64_t blocks = (total_threads + 255) / 256;
  hipLaunchKernelGGL(k_tree, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, inst,
                     n_inst, total_threads, leaves, leaf_cap, stacks, stack_depth, ctl);
  return hipGetLastError();
}

hipError_t launch_leaf(const Instance* inst, const Leaf* leaves, uint64_t leaf_cap, uint64_t* out,
                       Control* ctl, uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_leaf, dim3(grid), dim3(kLeafBlock), 0, stream, inst, leaves, leaf_cap, out,
                     ctl);
  return hipGetLastError();
}

hipError_t launch_bernoulli(double p, uint64_t N, uint64_t seed, uint64_t chunk, uint64_t n_chunks,
                            int fp32, double c64, float c32, unsigned long long* status,
                            uint64_t* out, uint64_t capacity, uint64_t* count_dev, Control* ctl,
                            uint32_t grid, uint32_t lds_cap, hipStream_t stream) {
  (void)p;
  hipLaunchKernelGGL(k_bern, dim3(grid), dim3(kLeafBlock), 0, stream, N, seed, chunk, n_chunks,
                     fp32, c64, c32, status, out, capacity, count_dev, ctl, lds_cap);
  return hipGetLastError();
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
