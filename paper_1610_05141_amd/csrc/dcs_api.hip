// dcs_api.hip -- host runtime behind include/dcs.h: argument checks, the
// per-call plan (Algorithm P cut depth, DFS stack bound, leaf capacity),
// workspace management, kernel launches, batching with hipGraph replay,
// kernel timing and latched device errors.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/dcs.h"
#include "dcs_host.hpp"
#include "dcs_kernels.hpp"

namespace dcs {
namespace host {

using dcs::Control;
using dcs::Instance;
using dcs::Leaf;
using dcs::Node;

constexpr uint32_t kDefaultN0 = 4096;
constexpr uint32_t kDefaultDenseRatio = 16;
constexpr uint32_t kMaxCut = 20;
constexpr size_t kAlign = 256;
// A leaf's range must fit a 32-bit draw (the tree splits larger ranges).
constexpr uint64_t kLeafRange = 1ull << 32;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace of dcs_sample_noalloc: one copy of this array per device, held
// from the library's load until the process ends.  Host code never passes
// its name to a kernel (on the host it is only a stand-in for the symbol):
// device_ctx looks up each device's address once with hipGetSymbolAddress,
// and calls use that address.
static __device__ __align__(256) unsigned char scratch[DCS_NOALLOC_SCRATCH_BYTES];

uint32_t floor_log2(uint64_t x) { return x == 0 ? 0 : 63u - static_cast<uint32_t>(__builtin_clzll(x)); }

uint64_t ceil_div_pow2(uint64_t N, uint32_t d) {
  if (d >= 64) return N ? 1 : 0;
  const uint64_t m = (1ull << d) - 1;
  return (N >> d) + ((N & m) ? 1 : 0);
}


int32_t read_params(const dcs_params* p, Params* out) {
  out->n0 = kDefaultN0;
  out->dense_ratio = kDefaultDenseRatio;
  if (p == nullptr) return DCS_OK;
  if (p->struct_size != sizeof(dcs_params)) return DCS_EINVAL;
  if (p->n0 != 0) out->n0 = p->n0;
  if (p->dense_ratio != 0) out->dense_ratio = p->dense_ratio;
  if (out->n0 < 2 || out->n0 > dcs::kMaxN0) return DCS_EINVAL;
  if (out->dense_ratio < 2 || out->dense_ratio > 64) return DCS_EINVAL;
  return DCS_OK;
}


uint64_t sat_add(uint64_t a, uint64_t b) { return a + b < a ? ~0ull : a + b; }

// Leaf jobs of the canonical tree, bounded for every outcome of its random
// splits.  Every leaf is a non-empty child of an internal node or the root,
// so there are at most 2 I + 1 leaves, and at most n (each holds a value).
// I counts internal nodes level by level: at depth d at most 2^d nodes, and
// at most n, are non-empty; where no range exceeds 2^32 a node splits only
// if it holds n0 or more values, and at most n / n0 such nodes are disjoint.
// Without replacement that needs N_v >= n_v >= n0, with replacement
// N_v >= 2, which ends the levels at depth d_last.  Jobs: leaves the tree
// kernels do not sample themselves, plus the extra pieces of constant
// leaves (at most n / kFillPiece).  Without replacement, when no leaf can
// span dense_ratio * kInlineMax elements or fewer (leaves lie at depth
// d_last + 1 or above, so they span at least floor(N / 2^(d_last + 1))),
// every leaf of at most kInlineMax values is sparse and sampled by the tree,
// so jobs hold at least kInlineMax + 1 values each: at most
// n / (kInlineMax + 1) of them.
uint64_t leaf_bound(uint64_t n, uint64_t N, uint32_t n0, uint32_t dense_ratio, uint32_t variant) {
  if (n == 0) return 0;
  const uint64_t need = variant == 0 ? n0 : 2;
  uint64_t internal = 0;
  uint32_t d = 0;
  for (; d < 64; ++d) {
    const uint64_t widest = ceil_div_pow2(N, d);
    const bool forced = widest > kLeafRange;
    if (!forced && widest < need) break;
    const uint64_t nodes = d < 63 ? (1ull << d) : ~0ull;
    internal = sat_add(internal, std::min(nodes, forced ? n : n / n0));
  }
  uint64_t jobs = sat_add(sat_add(internal, internal), 1);
  if (variant == 1) jobs = sat_add(jobs, n / dcs::kFillPiece);
  jobs = std::min(jobs, n);
  const uint64_t narrowest = d >= 63 ? 0 : (N >> d);  // leaves are at depth <= d
  if (variant == 0 && narrowest > static_cast<uint64_t>(dense_ratio) * dcs::kInlineMax)
    jobs = std::min(jobs, n / (dcs::kInlineMax + 1));
  return jobs;
}

// A capacity below the proven bound is used once the bound needs more than
// this many jobs (48 MiB of job records) and more than 4x the expected-case
// capacity.
constexpr uint64_t kProvenJobs = 1ull << 20;
// Test hook (dcs_debug_leaf_capacity): a fixed capacity with the second
// round, 0 = off.  Multiplier of the expected-case capacity, raised after a
// call latched a capacity error.
std::atomic<uint64_t> g_debug_leaf_cap{0};
std::atomic<uint32_t> g_cap_boost{1};
// Test hook (dcs_debug_lookback_help): polls before a Bernoulli look-back
// counts a silent predecessor itself, 0 = the default.
std::atomic<uint32_t> g_debug_help_polls{0};
// Test hook (dcs_debug_bernoulli_list): LDS positions per double-precision
// chunk (0: from the chunk's expected hits).
std::atomic<uint32_t> g_debug_bern_list{0};
// Test hook (dcs_debug_leaf_kernels): forced mixed_takes mask, or -1.
std::atomic<int32_t> g_debug_takes{-1};

void leaf_capacity_exceeded() {
  uint32_t b = g_cap_boost.load();
  while (b < 64 && !g_cap_boost.compare_exchange_weak(b, b * 4)) {
  }
}

// Capacity from the expected-case estimate and the proven bound (see
// make_plan); *second: the launch needs the second round.
uint64_t choose_capacity(uint64_t expected, uint64_t proven, uint64_t top_threads, bool* second) {
  const uint64_t debug_cap = g_debug_leaf_cap.load();
  const uint64_t boosted = expected * g_cap_boost.load();
  uint64_t cap;
  *second = false;
  if (debug_cap != 0) {
    cap = debug_cap;
    *second = true;
  } else if (proven <= std::max(kProvenJobs, 4 * boosted)) {
    cap = proven;
  } else {
    cap = boosted;
    *second = true;
  }
  // the top kernel's leaves (at most one per top path) always fit
  return std::max<uint64_t>(cap, top_threads + 1);
}

// variant 0: without replacement, 1: with replacement.
Plan make_plan(uint64_t n, uint64_t N, uint32_t n0, uint32_t dense_ratio, uint32_t variant,
               int32_t cut_bias) {
  Plan pl;
  if (n == 0) return pl;
  // Algorithm P cut: depth-`cut` subtrees hold about 2*n0 samples.
  uint32_t cut = 0;
  if (n >= 4ull * n0) cut = floor_log2(n / (2ull * n0));
  // Leaves need N_v <= 2^32: every node above that depth is internal.
  uint32_t forced = 0;
  while (ceil_div_pow2(N, forced) > kLeafRange) ++forced;
  const uint32_t by_count = floor_log2(n) + 1;
  cut = std::max(cut, std::min(forced, by_count));
  const int64_t biased = static_cast<int64_t>(cut) + cut_bias;
  cut = static_cast<uint32_t>(std::max<int64_t>(0, biased));
  // At most 2^18 threads, except where the range bound forces the tree so
  // deep that its leaves hold at most kInlineMax values on average: there
  // the threads' depth-first walks through the forced levels take the time,
  // and from n = 2^23 on up to 2^20 threads (about 16 values each) shorten
  // them by more than the splits above the cut that every extra level
  // repeats once more.
  const uint32_t lg = floor_log2(n);
  const bool deep_sparse = forced > 0 && (forced >= 64 || (n >> forced) <= dcs::kInlineMax);
  const uint32_t max_cut = deep_sparse ? std::min(kMaxCut, std::max(18u, lg > 4 ? lg - 4 : 0u)) : 18u;
  cut = std::min(cut, max_cut);
  pl.cut = cut;
  pl.threads = 1ull << cut;
  // the top kernel computes the frontier one wave (64 threads, 6 levels)
  // above the cut, so that each top-level split is computed once per wave
  pl.top_cut = cut > 6 ? cut - 6 : 0;
  pl.top_threads = 1ull << pl.top_cut;
  // Deepest possible internal node: its range must reach n0 (without
  // replacement: n_v <= N_v) or 2 (with replacement), or exceed 2^32.  The
  // depth-first walk below the cut holds at most one pending right child
  // per level, so this stack bound is never exceeded.
  const uint64_t need_range = variant == 0 ? std::min<uint64_t>(n0, kLeafRange + 1) : 2;
  uint32_t d_int = 0;
  while (d_int < 63 && ceil_div_pow2(N, d_int + 1) >= need_range) ++d_int;
  pl.stack_depth = (d_int + 2 > cut) ? d_int + 2 - cut : 2;
  // Leaf capacity.  Expected case: the tree has about 1.5 n/n0 leaves (at
  // most n/n0 internal nodes per level, halving sizes); range-forced levels
  // add at most min(n, 2^(forced+1)) small leaves; constant pieces of
  // N_v = 1 leaves.  The proven bound is used where it is affordable;
  // otherwise the expected-case capacity with the second round (tree
  // threads whose leaves found the job array full run again into the
  // emptied array), which only a deviation far beyond the expected leaf
  // count would exhaust too.
  uint64_t cap = 4 * ((n + n0 - 1) / n0) + 64;
  cap += std::min<uint64_t>(n, forced >= 62 ? n : (2ull << forced));
  if (variant == 1) cap += n / dcs::kFillPiece + std::min<uint64_t>(N, 4 * (n / n0) + 4) + 2;
  pl.leaf_cap = choose_capacity(cap, leaf_bound(n, N, n0, dense_ratio, variant), pl.top_threads,
                                &pl.second_round);
  return pl;
}


TreeLayout tree_layout(uint32_t n_inst, uint64_t leaf_cap, uint64_t threads, uint32_t stack_depth,
                       uint64_t top_threads, bool second_round) {
  TreeLayout L;
  size_t o = 0;
  L.ctl = o;
  o = align_up(o + sizeof(Control));
  L.inst = o;
  o = align_up(o + sizeof(Instance) * std::max<uint32_t>(n_inst, 1));
  L.leaves = o;
  o = align_up(o + sizeof(Leaf) * leaf_cap);
  L.stacks = o;
  o = align_up(o + sizeof(Node) * threads * stack_depth);
  L.frontier = o;
  o = align_up(o + sizeof(Node) * std::max<uint64_t>(top_threads, 1));
  L.redo = o;
  L.redo_words = second_round ? (threads + 31) / 32 : 0;
  o = align_up(o + sizeof(uint32_t) * L.redo_words);
  L.total = o;
  return L;
}

struct BernPlan {
  uint64_t chunk = 0, n_chunks = 0;
  int fp32 = 1;
  double c64 = 0;
  float c32 = 0;
};

double host_log1p_series(double x);

// Chunk length 2^floor(log2(n0/p)) clamped to [2^12, 2^32].
uint64_t bern_chunk_len(double p, uint32_t n0) {
  const double x = static_cast<double>(n0) / p;
  if (!(x < 4294967296.0)) return 1ull << 32;
  int e;
  frexp(x, &e);
  int lg = e - 1;
  lg = std::max(lg, 12);
  lg = std::min(lg, 32);
  return 1ull << lg;
}

// ---- host copies of the library's double-precision log (for the Bernoulli
// constant c = 1/ln(1-p), computed once per call on the host) ---------------
constexpr double kLn2HiH = 0x1.62e42feep-1;
constexpr double kLn2LoH = 0x1.a39ef35793c76p-33;
constexpr double kSqrt2H = 0x1.6a09e667f3bcdp+0;

double host_atanh2(double f) {
  const double s = f / (2.0 + f);
  const double z = s * s;
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
  const double t = s + s;
  return t + t * (z * p);
}

double host_log(double x) {
  uint64_t b;
  memcpy(&b, &x, 8);
  int e = static_cast<int>((b >> 52) & 0x7FF) - 1023;
  const uint64_t mb = (b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
  double m;
  memcpy(&m, &mb, 8);
  if (m >= kSqrt2H) {
    m = m * 0.5;
    e += 1;
  }
  const double r = host_atanh2(m - 1.0);
  const double de = static_cast<double>(e);
  return de * kLn2HiH + (de * kLn2LoH + r);
}

double host_log1p_series(double x) {
  if (x > -0.25 && x < 0.25) return host_atanh2(x);
  return host_log(1.0 + x);
}

// ---- device context -------------------------------------------------------

std::mutex g_mu;
std::vector<DeviceCtx> g_dev;
bool g_profile = false;
std::vector<Timing> g_timings;
uint32_t g_prof_mask = ~0u;                        // kinds that are timed
std::vector<std::vector<hipEvent_t>> g_event_pool;  // per device, reused events

hipEvent_t pooled_event(int dev) {
  if (static_cast<int>(g_event_pool.size()) <= dev) g_event_pool.resize(dev + 1);
  auto& pool = g_event_pool[dev];
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void release_timings() {
  for (Timing& t : g_timings) {
    g_event_pool[t.dev].push_back(t.a);
    g_event_pool[t.dev].push_back(t.b);
  }
  g_timings.clear();
}
// kinds: 0 reset, 1 tree, 2 leaf stage (all leaf kernels), 3 Bernoulli,
// 4 leaf kernel of the power-of-two list, 5 work-group leaf kernel of
// the rest, 6 one-wave dense leaf kernel, 7 edge-index decoding, 8 splits
// of the segments of an uneven universe, 9 / 10 / 11 whole-range
// Algorithm B: count passes / scan and repair / write passes, 12 one-wave
// leaf kernel of the small sparse and with-replacement leaves
constexpr int kProfKinds = 14;
double g_prof_ms[kProfKinds] = {};
uint64_t g_prof_n[kProfKinds] = {};

int32_t hip_status(hipError_t e) { return e == hipSuccess ? DCS_OK : DCS_EHIP; }

int32_t device_ctx(DeviceCtx** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DCS_EHIP;
  if (static_cast<int>(g_dev.size()) <= dev) g_dev.resize(dev + 1);
  DeviceCtx& c = g_dev[dev];
  if (!c.init) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DCS_EHIP;
    c.cus = prop.multiProcessorCount;
    c.leaf_occupancy = dcs::leaf_occupancy();
    c.bern_wave_occupancy = dcs::bern_wave_occupancy();
    c.wb_occupancy = dcs::wb_occupancy();
    c.small_occupancy = dcs::small_occupancy();
    c.dense_occupancy = dcs::dense_occupancy();
    if (const char* e = getenv("DCS_LEAF_GRID")) c.leaf_grid = atoll(e);
    if (dcs::error_slots(&c.err_slots) != hipSuccess || c.err_slots == nullptr) return DCS_EHIP;
    if (hipGetSymbolAddress(&c.noalloc_scratch, HIP_SYMBOL(scratch)) != hipSuccess ||
        c.noalloc_scratch == nullptr)
      return DCS_EHIP;
    c.init = true;
  }
  *out = &c;
  return DCS_OK;
}

unsigned int* error_word(DeviceCtx* c, void* stream) {
  auto it = c->err_slot_of.find(stream);
  if (it != c->err_slot_of.end()) return c->err_slots + it->second;
  // slot 0: the null stream; 1 .. kErrSlots-2: other streams in order of
  // first use; kErrSlots-1: shared by every stream after those
  int slot = 0;
  if (stream != nullptr) {
    const int used = static_cast<int>(c->err_slot_of.size() - c->err_slot_of.count(nullptr));
    slot = std::min(1 + used, dcs::kErrSlots - 1);
  }
  c->err_slot_of[stream] = slot;
  return c->err_slots + slot;
}

// ---- tuning table ------------------------------------------------------------
Tune g_tune[2][kTuneClasses];

uint32_t size_class(uint64_t n) { return n ? 63u - static_cast<uint32_t>(__builtin_clzll(n)) : 0u; }

Tune tune_for(uint32_t variant, uint64_t n) { return g_tune[variant ? 1 : 0][size_class(n)]; }

int32_t cut_bias_for(uint32_t variant, uint64_t n) {
  static const char* env = getenv("DCS_CUT_BIAS");
  return env ? atoi(env) : tune_for(variant, n).cut_bias;
}

uint32_t leaf_wgs_for(const DeviceCtx* c, uint32_t variant, uint64_t n) {
  const uint32_t occ = static_cast<uint32_t>(std::max(1, c->leaf_occupancy));
  const uint32_t w = tune_for(variant, n).leaf_wgs_per_cu;
  return w == 0 ? occ : std::min(w, occ);
}

// Library-owned workspace of at least `bytes` (grown on demand).
int32_t own_workspace(DeviceCtx* c, size_t bytes, void** ws) {
  if (c->ws_bytes < bytes) {
    if (c->ws) {
      if (hipDeviceSynchronize() != hipSuccess) return DCS_EHIP;
      if (hipFree(c->ws) != hipSuccess) return DCS_EHIP;
      c->ws = nullptr;
      c->ws_bytes = 0;
    }
    size_t grow = std::max(bytes, static_cast<size_t>(64) << 20);
    if (hipMalloc(&c->ws, grow) != hipSuccess) return DCS_ENOMEM;
    c->ws_bytes = grow;
  }
  *ws = c->ws;
  return DCS_OK;
}

// Copies `bytes` from host memory to `dst` on stream `s` through the
// device's pinned staging buffer (grown on demand), so that the caller's
// memory is free again when this returns and the copy stays asynchronous.
int32_t stage_upload(DeviceCtx* c, const void* src, size_t bytes, void* dst, hipStream_t s) {
  if (c->stage_done != nullptr && hipEventSynchronize(c->stage_done) != hipSuccess) return DCS_EHIP;
  if (c->stage_bytes < bytes) {
    if (c->stage != nullptr && hipHostFree(c->stage) != hipSuccess) return DCS_EHIP;
    c->stage = nullptr;
    c->stage_bytes = 0;
    const size_t grow = std::max(bytes, static_cast<size_t>(1) << 20);
    if (hipHostMalloc(&c->stage, grow, hipHostMallocDefault) != hipSuccess) return DCS_ENOMEM;
    c->stage_bytes = grow;
  }
  if (c->stage_done == nullptr &&
      hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming) != hipSuccess)
    return DCS_EHIP;
  memcpy(c->stage, src, bytes);
  if (hipMemcpyAsync(dst, c->stage, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipEventRecord(c->stage_done, s) != hipSuccess)
    return DCS_EHIP;
  return DCS_OK;
}

void timing_begin(int kind, hipStream_t s, Timing* t) {
  t->a = t->b = nullptr;
  if (!g_profile || !((g_prof_mask >> kind) & 1u)) return;
  if (hipGetDevice(&t->dev) != hipSuccess) return;
  t->kind = kind;
  t->a = pooled_event(t->dev);
  t->b = pooled_event(t->dev);
  if (t->a == nullptr || t->b == nullptr) {
    if (t->a) g_event_pool[t->dev].push_back(t->a);
    if (t->b) g_event_pool[t->dev].push_back(t->b);
    t->a = t->b = nullptr;
    return;
  }
  (void)hipEventRecord(t->a, s);
}

void timing_end(hipStream_t s, Timing* t) {
  if (t->a == nullptr) return;
  (void)hipEventRecord(t->b, s);
  g_timings.push_back(*t);
}

// Leaf kinds that no leaf of a single instance's tree can have except by a
// deviation of its counts from their expectations by tens of standard
// deviations; their kernels are then not launched and k_leaf_mixed runs any
// such leaf itself (the sample never depends on this).  A leaf's parent held
// n0 or more values or a range above 2^32.  Dense leaves (dense_ratio n_v >=
// N_v) then need some range of at most 2 dense_ratio n0 elements at density
// 1/(2 dense_ratio), 64 times the sample's (kept below 1/(128 dense_ratio)).
// Leaves of at most 1024 values need, when the range-forced levels end with
// nodes of 2 n0 or more values and n0 = 4096, a split of such a node to leave
// a quarter of its expected share.  One-pass leaves (n_v^2 >= 2 N_v with
// 1024 < n_v < n0) exist only for n0 > 1025; when N >= n n0, the expected
// count n N_v / N of such a leaf's range is at most n_v^2 / (2 n0) < n_v / 2,
// so n_v lies more than n_v / 2 above it: over sqrt(n_v / 2) > 22 standard
// deviations.
uint32_t mixed_takes(const Instance& I) {
  uint32_t forced = 0;
  while (ceil_div_pow2(I.N, forced) > kLeafRange) ++forced;
  const unsigned __int128 n = I.n, N = I.N;
  uint32_t takes = 0;
  if (I.variant == 1 || (I.n0 >= 1024 && n * 128u * I.dense_ratio < N)) takes |= dcs::kTakesDense;
  if (I.n0 >= 4096 && (I.n >> forced) >= 2ull * I.n0) takes |= dcs::kTakesSmall;
  if (I.variant == 1 || I.n0 <= 1025 || n * I.n0 <= N) takes |= dcs::kTakesOnce;
  return takes;
}

// Enqueue reset + tree + leaf for the instances already in the workspace.
int32_t run_tree_pipeline(DeviceCtx* c, void* ws, const TreeLayout& L, const Instance* single,
                          uint32_t n_inst, uint64_t threads, uint64_t top_threads,
                          uint64_t leaf_cap, uint32_t stack_depth, uint64_t* out, hipStream_t s,
                          unsigned int* err, uint32_t leaf_wgs_per_cu, uint64_t* part_out,
                          const Instance* whole) {
  if (leaf_cap >= dcs::kMaxLeafJobs) return DCS_ENOMEM;
  char* base = static_cast<char*>(ws);
  Control* ctl = reinterpret_cast<Control*>(base + L.ctl);
  Instance* inst = reinterpret_cast<Instance*>(base + L.inst);
  Leaf* leaves = reinterpret_cast<Leaf*>(base + L.leaves);
  Node* stacks = reinterpret_cast<Node*>(base + L.stacks);
  Node* frontier = reinterpret_cast<Node*>(base + L.frontier);
  uint32_t* redo = L.redo_words ? reinterpret_cast<uint32_t*>(base + L.redo) : nullptr;
  Timing t0{}, t1{}, t2{};
  timing_begin(0, s, &t0);
  hipError_t e = dcs::launch_reset(ctl, single, inst, err, redo, L.redo_words, out, s);
  timing_end(s, &t0);
  if (e != hipSuccess) return DCS_EHIP;
  timing_begin(1, s, &t1);
  e = dcs::launch_tree_top(inst, n_inst, top_threads, frontier, leaves, leaf_cap, ctl, part_out,
                           s);
  if (e == hipSuccess)
    e = dcs::launch_tree(inst, n_inst, threads, frontier, leaves, leaf_cap, stacks, stack_depth,
                         ctl, redo, 0, s);
  timing_end(s, &t1);
  if (e != hipSuccess) return DCS_EHIP;
  uint64_t want = static_cast<uint64_t>(c->cus) * std::max<uint32_t>(1, leaf_wgs_per_cu);
  if (c->leaf_grid > 0) want = static_cast<uint64_t>(c->leaf_grid);
  want = std::max<uint64_t>(1, std::min<uint64_t>(want, leaf_cap));
  // batches launch every leaf kernel; a single instance, or the parts of
  // one sample, skip those whose kinds the sample's tree cannot plausibly hold
  if (whole == nullptr && single != nullptr && n_inst == 1) whole = single;
  uint32_t takes = whole != nullptr ? mixed_takes(*whole) : 0u;
  const int32_t forced_takes = g_debug_takes.load();
  if (forced_takes >= 0 && whole != nullptr) takes = static_cast<uint32_t>(forced_takes);
  Timing t4{}, t5{};
  timing_begin(2, s, &t2);
  timing_begin(4, s, &t4);
  e = dcs::launch_leaf(dcs::kLeafFront, leaves, leaf_cap, out, ctl, static_cast<uint32_t>(want),
                       s);
  timing_end(s, &t4);
  if (e == hipSuccess) {
    timing_begin(5, s, &t5);
    e = dcs::launch_leaf(dcs::kLeafBack, leaves, leaf_cap, out, ctl, static_cast<uint32_t>(want),
                         s, takes);
    timing_end(s, &t5);
  }
  Timing t13{};
  if (e == hipSuccess && !(takes & dcs::kTakesOnce)) {
    timing_begin(13, s, &t13);
    e = dcs::launch_leaf(dcs::kLeafOnce, leaves, leaf_cap, out, ctl, static_cast<uint32_t>(want),
                         s);
    timing_end(s, &t13);
  }
  Timing t6{};
  if (e == hipSuccess && !(takes & dcs::kTakesDense)) {
    uint64_t waves = static_cast<uint64_t>(c->cus) * std::max(1, c->dense_occupancy);
    if (c->leaf_grid > 0) waves = static_cast<uint64_t>(c->leaf_grid) * (dcs::kLeafBlock / 64);
    waves = std::max<uint64_t>(1, std::min<uint64_t>(waves, leaf_cap));
    timing_begin(6, s, &t6);
    e = dcs::launch_leaf_dense(leaves, leaf_cap, out, ctl, static_cast<uint32_t>(waves), s);
    timing_end(s, &t6);
  }
  Timing t12{};
  if (e == hipSuccess && !(takes & dcs::kTakesSmall)) {
    uint64_t waves = static_cast<uint64_t>(c->cus) * std::max(1, c->small_occupancy);
    if (c->leaf_grid > 0) waves = static_cast<uint64_t>(c->leaf_grid) * (dcs::kLeafBlock / 64);
    waves = std::max<uint64_t>(1, std::min<uint64_t>(waves, leaf_cap));
    timing_begin(12, s, &t12);
    e = dcs::launch_leaf_small(leaves, leaf_cap, out, ctl, static_cast<uint32_t>(waves), s);
    timing_end(s, &t12);
  }
  // Second round: the tree threads marked in `redo` run again into the
  // emptied job array, and one work-group pass samples their leaves (both
  // return at once when nothing was marked).
  if (e == hipSuccess && redo != nullptr)
    e = dcs::launch_tree(inst, n_inst, threads, frontier, leaves, leaf_cap, stacks, stack_depth,
                         ctl, redo, 1, s);
  if (e == hipSuccess && redo != nullptr)
    e = dcs::launch_leaf_round2(leaves, leaf_cap, out, ctl, static_cast<uint32_t>(want), s,
                                takes);
  timing_end(s, &t2);
  if (e != hipSuccess) return DCS_EHIP;
  return DCS_OK;
}

std::mutex& lock() { return g_mu; }

// noalloc: run in this device's static scratch array (DCS_ENOMEM if the
// call needs more); the call then allocates no device memory.
int32_t sample_tree(uint32_t variant, uint64_t n, uint64_t N, uint64_t seed, const dcs_params* params,
                    uint64_t* out, void* workspace, size_t ws_bytes, void* stream,
                    bool noalloc = false) {
  Params P;
  if (read_params(params, &P) != DCS_OK) return DCS_EINVAL;
  if (N > DCS_MAX_UNIVERSE) return DCS_EINVAL;
  if (variant == 0 && n > N) return DCS_EINVAL;
  if (variant == 1 && N == 0 && n > 0) return DCS_EINVAL;
  if (n > 0 && out == nullptr) return DCS_EINVAL;
  if (n == 0) return DCS_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  const Plan pl = make_plan(n, N, P.n0, P.dense_ratio, variant, cut_bias_for(variant, n));
  const TreeLayout L =
      tree_layout(1, pl.leaf_cap, pl.threads, pl.stack_depth, pl.top_threads, pl.second_round);
  void* ws = workspace;
  if (noalloc) {
    if (L.total > DCS_NOALLOC_SCRATCH_BYTES) return DCS_ENOMEM;
    ws = c->noalloc_scratch;
  } else if (ws == nullptr) {
    rc = own_workspace(c, L.total, &ws);
    if (rc) return rc;
  } else if (ws_bytes < L.total) {
    return DCS_ENOMEM;
  }
  Instance I{};
  I.n = n;
  I.N = N;
  I.seed = seed;
  I.out_offset = 0;
  I.thread_base = 0;
  I.top_base = 0;
  I.n0 = P.n0;
  I.dense_ratio = P.dense_ratio;
  I.variant = variant;
  I.cut = pl.cut;
  I.top_cut = pl.top_cut;
  return run_tree_pipeline(c, ws, L, &I, 1, pl.threads, pl.top_threads, pl.leaf_cap,
                           pl.stack_depth, out, static_cast<hipStream_t>(stream),
                           error_word(c, stream), leaf_wgs_for(c, variant, n));
}

struct BernLayout {
  size_t ctl = 0, tickets = 0, status = 0, total = 0;
};

// Whole-range Algorithm B: control block | state | chunk counts (u32) |
// chunk offsets (u64) | removal counts per block of hit indices (u32) |
// removal bitmap (u64 words).
struct WbLayout {
  size_t ctl = 0, state = 0, cnt = 0, off = 0, rem = 0, bitmap = 0, tsum = 0, total = 0;
};

WbLayout wb_layout(uint64_t n_chunks, uint64_t rem_blocks, uint64_t words) {
  WbLayout L;
  size_t o = 0;
  L.ctl = o;
  o = align_up(o + sizeof(Control));
  L.state = o;
  o = align_up(o + sizeof(dcs::WbState));
  L.cnt = o;
  o = align_up(o + sizeof(uint32_t) * n_chunks);
  L.off = o;
  o = align_up(o + sizeof(uint64_t) * n_chunks);
  L.rem = o;
  o = align_up(o + sizeof(uint32_t) * rem_blocks);
  L.bitmap = o;
  o = align_up(o + sizeof(uint64_t) * words);
  L.tsum = o;
  o = align_up(o + sizeof(uint64_t) * dcs::kWbTileSums);
  L.total = o;
  return L;
}

uint64_t isqrt_host(uint64_t x) {
  uint64_t r = static_cast<uint64_t>(sqrt(static_cast<double>(x)));
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return r;
}

BernLayout bern_layout(uint64_t n_chunks) {
  BernLayout L;
  size_t o = 0;
  L.ctl = o;
  o = align_up(o + sizeof(Control));
  L.tickets = o;
  o = align_up(o + sizeof(unsigned long long) * dcs::kTicketWords);
  L.status = o;
  o = align_up(o + sizeof(unsigned long long) * n_chunks);
  L.total = o;
  return L;
}

}  // namespace host
}  // namespace dcs

using namespace dcs::host;
using dcs::Control;
using dcs::Instance;
using dcs::Leaf;
using dcs::Node;

extern "C" {

int32_t dcs_sample(uint64_t n, uint64_t N, uint64_t seed, uint64_t* out_dev, void* stream) {
  return sample_tree(0, n, N, seed, nullptr, out_dev, nullptr, 0, stream);
}

int32_t dcs_sample_ex(uint64_t n, uint64_t N, uint64_t seed, const dcs_params* params,
                      uint64_t* out_dev, void* workspace, size_t ws_bytes, void* stream) {
  return sample_tree(0, n, N, seed, params, out_dev, workspace, ws_bytes, stream);
}

int32_t dcs_sample_noalloc(uint64_t n, uint64_t N, uint64_t seed, const dcs_params* params,
                           uint64_t* out_dev, void* stream) {
  return sample_tree(0, n, N, seed, params, out_dev, nullptr, 0, stream, true);
}

int32_t dcs_sample_replacement(uint64_t n, uint64_t N, uint64_t seed, uint64_t* out_dev,
                               void* stream) {
  return sample_tree(1, n, N, seed, nullptr, out_dev, nullptr, 0, stream);
}

int32_t dcs_sample_replacement_ex(uint64_t n, uint64_t N, uint64_t seed, const dcs_params* params,
                                  uint64_t* out_dev, void* workspace, size_t ws_bytes,
                                  void* stream) {
  return sample_tree(1, n, N, seed, params, out_dev, workspace, ws_bytes, stream);
}

int32_t dcs_sample_part(int32_t variant, uint64_t n, uint64_t N, uint64_t seed,
                        const dcs_params* params, uint32_t depth, uint64_t index,
                        uint64_t* out_dev, uint64_t capacity, uint64_t* count_rank_dev,
                        void* stream) {
  Params P;
  if (read_params(params, &P) != DCS_OK) return DCS_EINVAL;
  if (variant != 0 && variant != 1) return DCS_EINVAL;
  if (N > DCS_MAX_UNIVERSE) return DCS_EINVAL;
  if (variant == 0 && n > N) return DCS_EINVAL;
  if (variant == 1 && N == 0 && n > 0) return DCS_EINVAL;
  if (depth > DCS_MAX_PART_DEPTH || index >= (1ull << depth)) return DCS_EINVAL;
  if (count_rank_dev == nullptr || (capacity > 0 && out_dev == nullptr)) return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  // Plan the part's subtree for at most min(n, capacity) values over the
  // largest range a depth-`depth` node can have (ranges halve with the
  // right child taking the odd element); at least one top path runs, so
  // that the count and rank are always written.
  const uint64_t range = ceil_div_pow2(N, depth);
  uint64_t np = std::min(n, capacity);
  if (variant == 0) np = std::min(np, range);
  np = std::max<uint64_t>(np, 1);
  const Plan pl = make_plan(np, std::max<uint64_t>(range, 1), P.n0, P.dense_ratio,
                            static_cast<uint32_t>(variant),
                            cut_bias_for(static_cast<uint32_t>(variant), np));
  const TreeLayout L =
      tree_layout(1, pl.leaf_cap, pl.threads, pl.stack_depth, pl.top_threads, pl.second_round);
  void* ws = nullptr;
  rc = own_workspace(c, L.total, &ws);
  if (rc) return rc;
  Instance I{};
  I.n = n;
  I.N = N;
  I.seed = seed;
  I.n0 = P.n0;
  I.dense_ratio = P.dense_ratio;
  I.variant = static_cast<uint32_t>(variant);
  I.cut = depth + pl.cut;
  I.top_cut = depth + pl.top_cut;
  I.part_depth = depth;
  I.part = index;
  I.part_cap = capacity;
  return run_tree_pipeline(c, ws, L, &I, 1, pl.threads, pl.top_threads, pl.leaf_cap,
                           pl.stack_depth, out_dev, static_cast<hipStream_t>(stream),
                           error_word(c, stream),
                           leaf_wgs_for(c, static_cast<uint32_t>(variant), np), count_rank_dev);
}

int32_t dcs_sample_segments(uint64_t n, const uint64_t* lengths, uint64_t K, uint64_t seed,
                            const dcs_params* params, uint64_t* out_dev, uint64_t* counts_dev,
                            void* stream) {
  Params P;
  if (read_params(params, &P) != DCS_OK) return DCS_EINVAL;
  if (K == 0 || K > DCS_MAX_SEGMENTS || lengths == nullptr) return DCS_EINVAL;
  uint64_t N = 0;
  for (uint64_t i = 0; i < K; ++i) {
    if (lengths[i] > DCS_MAX_UNIVERSE - N) return DCS_EINVAL;
    N += lengths[i];
  }
  if (n > N || (n > 0 && out_dev == nullptr)) return DCS_EINVAL;
  if (n == 0 && counts_dev == nullptr) return DCS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  uint32_t D = 0;
  while ((1ull << D) < K) ++D;
  // Plan every segment for its expected count (at least one tree thread for
  // any segment that may hold samples).  The plan only spreads the work: the
  // DFS below each segment's cut follows the actual count, its stack bound
  // depends on the segment's range alone, and the leaf capacity bounds the
  // leaves of all segments together (at most 4 n/n0 + 5 per non-empty
  // segment, plus the leaves of levels forced by ranges above 2^32).
  std::vector<Instance> tab(K);
  uint64_t tb = 0, tt = 0, forced_leaves = 0, nonempty = 0, proven = 0;
  uint32_t stack_depth = 1;
  uint64_t base = 0;
  for (uint64_t i = 0; i < K; ++i) {
    Instance& I = tab[i];
    I = Instance{};
    I.N = lengths[i];
    I.base = base;
    I.n0 = P.n0;
    I.dense_ratio = P.dense_ratio;
    I.thread_base = tb;
    I.top_base = tt;
    base += lengths[i];
    if (n == 0 || lengths[i] == 0) continue;
    const double m = static_cast<double>(n) *
                     (static_cast<double>(lengths[i]) / static_cast<double>(N));
    const uint64_t est = std::max<uint64_t>(1, std::min<uint64_t>(lengths[i], static_cast<uint64_t>(m)));
    const Plan pl = make_plan(est, lengths[i], P.n0, P.dense_ratio, 0, cut_bias_for(0, est));
    I.cut = pl.cut;
    I.top_cut = pl.top_cut;
    tb += pl.threads;
    tt += pl.top_threads;
    stack_depth = std::max(stack_depth, pl.stack_depth);
    uint32_t forced = 0;
    while (ceil_div_pow2(lengths[i], forced) > kLeafRange) ++forced;
    if (forced > 0) forced_leaves += std::min<uint64_t>(n, 2ull << forced);
    ++nonempty;
    // a segment holds at most min(n, L_i) values
    proven = sat_add(proven,
                     leaf_bound(std::min(n, lengths[i]), lengths[i], P.n0, P.dense_ratio, 0));
  }
  bool second = false;
  const uint64_t leaf_cap = choose_capacity(
      4 * ((n + P.n0 - 1) / P.n0) + 64 + 5 * nonempty + std::min<uint64_t>(n, forced_leaves),
      std::min(proven, n), tt, &second);
  const TreeLayout L = tree_layout(static_cast<uint32_t>(K), leaf_cap, tb, stack_depth, tt, second);
  void* ws = nullptr;
  rc = own_workspace(c, L.total, &ws);
  if (rc) return rc;
  Instance* inst = reinterpret_cast<Instance*>(static_cast<char*>(ws) + L.inst);
  rc = stage_upload(c, tab.data(), sizeof(Instance) * K, inst, s);
  if (rc) return rc;
  Timing t8{};
  timing_begin(8, s, &t8);
  hipError_t e = dcs::launch_segments(inst, K, D, n, N, seed, counts_dev, s);
  timing_end(s, &t8);
  if (e != hipSuccess) return DCS_EHIP;
  if (n == 0) return DCS_OK;
  return run_tree_pipeline(c, ws, L, nullptr, static_cast<uint32_t>(K), tb, tt, leaf_cap,
                           stack_depth, out_dev, s, error_word(c, stream),
                           leaf_wgs_for(c, 0, n));
}

int32_t dcs_sample_wholerange(uint64_t n, uint64_t N, uint64_t seed, const dcs_params* params,
                              uint64_t* out_dev, void* stream) {
  Params P;
  if (read_params(params, &P) != DCS_OK) return DCS_EINVAL;
  if (N == 0 || N > (1ull << 32) || n > N || (n > 0 && out_dev == nullptr)) return DCS_EINVAL;
  const uint64_t num = n + 8 * isqrt_host(n) + 16;
  const int full = num >= N ? 1 : 0;
  const double rho = full ? 1.0 : static_cast<double>(num) / static_cast<double>(N);
  if (n > 0 && rho < 0x1p-10) return DCS_ENOTSUP;
  if (n == 0) return DCS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  const uint64_t chunk = bern_chunk_len(rho, P.n0);
  const uint64_t n_chunks = (N + chunk - 1) / chunk;
  const uint64_t hi = n + 16 * isqrt_host(n) + 64;  // most hits an accepted attempt has
  const uint64_t words = (hi + 63) / 64;
  const uint64_t rem_blocks = (hi >> dcs::kWbRemShift) + 1;
  const WbLayout L = wb_layout(n_chunks, rem_blocks, words);
  void* ws = nullptr;
  rc = own_workspace(c, L.total, &ws);
  if (rc) return rc;
  char* base = static_cast<char*>(ws);
  Control* ctl = reinterpret_cast<Control*>(base + L.ctl);
  dcs::WbBuffers b;
  b.state = reinterpret_cast<dcs::WbState*>(base + L.state);
  b.cnt = reinterpret_cast<uint32_t*>(base + L.cnt);
  b.off = reinterpret_cast<uint64_t*>(base + L.off);
  b.rem = reinterpret_cast<uint32_t*>(base + L.rem);
  b.rem_blocks = rem_blocks;
  b.bitmap = reinterpret_cast<unsigned long long*>(base + L.bitmap);
  b.words = words;
  b.tsum = reinterpret_cast<uint64_t*>(base + L.tsum);
  const float c32 = full ? 0.0f : static_cast<float>(1.0 / host_log1p_series(-rho));
  const uint32_t grid = static_cast<uint32_t>(std::max<uint64_t>(
      1, std::min<uint64_t>(n_chunks, static_cast<uint64_t>(c->cus) * c->wb_occupancy)));
  // the first repair round's words (at most hi - n) over 256-thread groups,
  // four words per thread
  const uint32_t repair_grid = static_cast<uint32_t>(std::max<uint64_t>(
      1, std::min<uint64_t>(static_cast<uint64_t>(c->cus) * 4, (hi - n + 1023) / 1024)));
  hipError_t e = dcs::launch_wb_zero(ctl, b, n_chunks, error_word(c, stream), s);
  // Two attempts are enqueued; the second one's kernels return at once when
  // the first is accepted (a rejection has probability below about 1e-11).
  for (uint32_t a = 0; a < 2 && e == hipSuccess; ++a) {
    Timing t9{}, t10{}, t11{};
    timing_begin(9, s, &t9);
    e = dcs::launch_wb_count(N, seed, chunk, n_chunks, c32, full, a, b, grid, s);
    timing_end(s, &t9);
    if (e != hipSuccess) break;
    timing_begin(10, s, &t10);
    e = dcs::launch_wb_mid(n, seed, n_chunks, a, a == 1 ? 1 : 0, b, ctl, repair_grid, s);
    timing_end(s, &t10);
    if (e != hipSuccess) break;
    timing_begin(11, s, &t11);
    e = dcs::launch_wb_write(N, seed, chunk, n_chunks, c32, full, a, b, out_dev, grid, s);
    timing_end(s, &t11);
  }
  return hip_status(e);
}

uint64_t dcs_bernoulli_capacity_hint(double p, uint64_t N) {
  if (!(p >= 0.0 && p <= 1.0)) return 0;
  const double m = static_cast<double>(N) * p;
  const double v = m * (1.0 - p);
  double cap = m + 10.0 * sqrt(v) + 64.0;
  if (cap > static_cast<double>(N)) cap = static_cast<double>(N);
  return static_cast<uint64_t>(cap);
}

int32_t dcs_sample_bernoulli_ex(double p, uint64_t N, uint64_t seed, const dcs_params* params,
                                uint64_t* out_dev, uint64_t capacity, uint64_t* count_dev,
                                void* workspace, size_t ws_bytes, void* stream) {
  Params P;
  if (read_params(params, &P) != DCS_OK) return DCS_EINVAL;
  if (!(p >= 0.0 && p <= 1.0) || N > DCS_MAX_BERNOULLI_UNIVERSE) return DCS_EINVAL;
  if (count_dev == nullptr || (capacity > 0 && out_dev == nullptr)) return DCS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  if (p == 0.0 || N == 0) {
    return hip_status(hipMemsetAsync(count_dev, 0, sizeof(uint64_t), s));
  }
  if (p == 1.0) return hip_status(dcs::launch_bernoulli_fill(N, out_dev, capacity, count_dev, s));
  const uint64_t chunk = bern_chunk_len(p, P.n0);
  const uint64_t n_chunks = (N + chunk - 1) / chunk;
  const BernLayout L = bern_layout(n_chunks);
  void* ws = workspace;
  if (ws == nullptr) {
    rc = own_workspace(c, L.total, &ws);
    if (rc) return rc;
  } else if (ws_bytes < L.total) {
    return DCS_ENOMEM;
  }
  char* base = static_cast<char*>(ws);
  Control* ctl = reinterpret_cast<Control*>(base + L.ctl);
  unsigned long long* status = reinterpret_cast<unsigned long long*>(base + L.status);
  unsigned long long* tickets = reinterpret_cast<unsigned long long*>(base + L.tickets);
  const double c64 = 1.0 / host_log1p_series(-p);
  const float c32 = static_cast<float>(c64);
  const int fp32 = p >= 0x1p-10 ? 1 : 0;
  Timing t0{}, t1{};
  timing_begin(0, s, &t0);
  hipError_t e = dcs::launch_zero(ctl, status, n_chunks, tickets, error_word(c, stream), s);
  timing_end(s, &t0);
  if (e != hipSuccess) return DCS_EHIP;
  // LDS offsets per double-precision chunk: 2 n0 + 64, or fewer when a full
  // chunk expects fewer hits (chunks clamped at 2^32 for small p); a chunk
  // with more hits writes the rest in a second pass, so this choice never
  // changes the sample, only how many work-groups stay resident.  The grid
  // never exceeds the resident work-groups (the look-back needs them all).
  uint32_t lds_cap = 2 * P.n0 + 64;
  if (!fp32) {
    const double m = static_cast<double>(chunk) * p;
    const double want = m + 10.0 * sqrt(m) + 64.0;
    if (want < static_cast<double>(lds_cap))
      lds_cap = (static_cast<uint32_t>(want) + 63u) & ~63u;
  }
  const uint32_t forced_list = g_debug_bern_list.load();
  if (!fp32 && forced_list != 0) lds_cap = forced_list;
  // chunks expecting few hits (a short LDS list) take one wave each
  const int kind = fp32 ? dcs::kBernFp32Wave
                        : (lds_cap <= dcs::kBern64WaveMaxList ? dcs::kBernFp64Wave
                                                              : dcs::kBernFp64Group);
  const uint64_t occ = static_cast<uint64_t>(
      kind == dcs::kBernFp32Wave   ? c->bern_wave_occupancy
      : kind == dcs::kBernFp64Wave ? dcs::bern64_wave_occupancy(lds_cap)
                                   : dcs::bern_occupancy(lds_cap));
  const uint32_t grid = static_cast<uint32_t>(
      std::max<uint64_t>(1, std::min<uint64_t>(n_chunks, static_cast<uint64_t>(c->cus) * occ)));
  timing_begin(3, s, &t1);
  const uint32_t help = g_debug_help_polls.load();
  e = dcs::launch_bernoulli(p, N, seed, chunk, n_chunks, kind, c64, c32, status, out_dev, capacity,
                            count_dev, ctl, tickets, grid, lds_cap,
                            help != 0 ? help : dcs::kHelpPolls, s);
  timing_end(s, &t1);
  if (e != hipSuccess) return DCS_EHIP;
  return DCS_OK;
}

int32_t dcs_sample_bernoulli(double p, uint64_t N, uint64_t seed, uint64_t* out_dev,
                             uint64_t capacity, uint64_t* count_dev, void* stream) {
  return dcs_sample_bernoulli_ex(p, N, seed, nullptr, out_dev, capacity, count_dev, nullptr, 0,
                                 stream);
}

int32_t dcs_workspace_size(int32_t variant, uint64_t n, uint64_t N, double p_for_bernoulli,
                           const dcs_params* params, size_t* bytes) {
  Params P;
  if (bytes == nullptr || read_params(params, &P) != DCS_OK) return DCS_EINVAL;
  if (N > DCS_MAX_UNIVERSE) return DCS_EINVAL;
  if (variant == 0 || variant == 1) {
    if (variant == 0 && n > N) return DCS_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    const Plan pl = make_plan(n, N, P.n0, P.dense_ratio, static_cast<uint32_t>(variant),
                              cut_bias_for(static_cast<uint32_t>(variant), n));
    *bytes = tree_layout(1, pl.leaf_cap, pl.threads, pl.stack_depth, pl.top_threads,
                         pl.second_round).total;
    return DCS_OK;
  }
  if (variant == 2) {
    const double p = p_for_bernoulli;
    if (!(p >= 0.0 && p <= 1.0) || N > DCS_MAX_BERNOULLI_UNIVERSE) return DCS_EINVAL;
    if (p == 0.0 || p == 1.0 || N == 0) {
      *bytes = align_up(sizeof(Control));
      return DCS_OK;
    }
    const uint64_t chunk = bern_chunk_len(p, P.n0);
    *bytes = bern_layout((N + chunk - 1) / chunk).total;
    return DCS_OK;
  }
  return DCS_EINVAL;
}

// ---- batch ----------------------------------------------------------------
}  // extern "C"

struct dcs_batch {
  std::vector<Instance> host;
  uint64_t threads = 0, top_threads = 0, leaf_cap = 0, total_out = 0;
  uint32_t stack_depth = 1;
  bool second_round = false;
  TreeLayout layout;
  void* ws = nullptr;
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t* graph_out = nullptr;
  hipStream_t graph_stream = nullptr;
};

extern "C" {

int32_t dcs_batch_create(const dcs_instance* instances, uint32_t count, dcs_batch** batch,
                         uint32_t* bad_index) {
  if (batch == nullptr || (count > 0 && instances == nullptr) || count == 0) return DCS_EINVAL;
  *batch = nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  auto* b = new dcs_batch();
  uint64_t tb = 0, tt = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const dcs_instance& d = instances[i];
    dcs_params pp{sizeof(dcs_params), d.n0, d.dense_ratio, 0};
    Params P;
    const bool ok = read_params(&pp, &P) == DCS_OK && d.N <= DCS_MAX_UNIVERSE && d.variant <= 1 &&
                    !(d.variant == 0 && d.n > d.N) && !(d.variant == 1 && d.N == 0 && d.n > 0);
    if (!ok) {
      if (bad_index) *bad_index = i;
      delete b;
      return DCS_EINVAL;
    }
    const Plan pl =
        make_plan(d.n, d.N, P.n0, P.dense_ratio, d.variant, cut_bias_for(d.variant, d.n));
    Instance I{};
    I.n = d.n;
    I.N = d.N;
    I.seed = d.seed;
    I.out_offset = d.out_offset;
    I.thread_base = tb;
    I.top_base = tt;
    I.n0 = P.n0;
    I.dense_ratio = P.dense_ratio;
    I.variant = d.variant;
    I.cut = pl.cut;
    I.top_cut = pl.top_cut;
    tb += pl.threads;
    tt += pl.threads ? pl.top_threads : 0;
    b->leaf_cap += pl.leaf_cap;
    b->second_round = b->second_round || pl.second_round;
    b->stack_depth = std::max(b->stack_depth, pl.stack_depth);
    b->total_out += d.n;
    b->host.push_back(I);
  }
  b->threads = tb;
  b->top_threads = tt;
  b->layout = tree_layout(count, b->leaf_cap, b->threads, b->stack_depth, b->top_threads,
                          b->second_round);
  if (hipGetDevice(&b->device) != hipSuccess || hipMalloc(&b->ws, b->layout.total) != hipSuccess) {
    delete b;
    return DCS_ENOMEM;
  }
  char* base = static_cast<char*>(b->ws);
  if (hipMemset(base + b->layout.ctl, 0, sizeof(Control)) != hipSuccess ||
      hipMemcpy(base + b->layout.inst, b->host.data(), sizeof(Instance) * count,
                hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(b->ws);
    delete b;
    return DCS_EHIP;
  }
  *batch = b;
  return DCS_OK;
}

uint64_t dcs_batch_total(const dcs_batch* batch) { return batch ? batch->total_out : 0; }

int32_t dcs_batch_run(dcs_batch* b, uint64_t* out_dev, int32_t use_graph, void* stream) {
  if (b == nullptr || out_dev == nullptr) return DCS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  const uint32_t n_inst = static_cast<uint32_t>(b->host.size());
  unsigned int* err = error_word(c, stream);
  if (!use_graph || g_profile) {
    return run_tree_pipeline(c, b->ws, b->layout, nullptr, n_inst, b->threads, b->top_threads,
                             b->leaf_cap, b->stack_depth, out_dev, s, err,
                             leaf_wgs_for(c, 0, b->total_out));
  }
  if (s == nullptr) return DCS_EINVAL;  // capture needs a real stream
  // the captured reset names the output and the stream's error word:
  // capture again when either changes
  if (b->exec == nullptr || b->graph_out != out_dev || b->graph_stream != s) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    if (b->graph) {
      (void)hipGraphDestroy(b->graph);
      b->graph = nullptr;
    }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return DCS_EHIP;
    rc = run_tree_pipeline(c, b->ws, b->layout, nullptr, n_inst, b->threads, b->top_threads,
                           b->leaf_cap, b->stack_depth, out_dev, s, err,
                           leaf_wgs_for(c, 0, b->total_out));
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (rc != DCS_OK) return rc;
    if (e != hipSuccess) return DCS_EHIP;
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) return DCS_EHIP;
    b->graph_out = out_dev;
    b->graph_stream = s;
  }
  return hip_status(hipGraphLaunch(b->exec, s));
}

int32_t dcs_batch_destroy(dcs_batch* b) {
  if (b == nullptr) return DCS_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ws) (void)hipFree(b->ws);
  delete b;
  return DCS_OK;
}

// ---- online sampling -------------------------------------------------------
}  // extern "C"

struct dcs_online {
  int32_t variant = 0;
  uint64_t n = 0, N = 0, seed = 0;
  Params P;
  uint32_t depth = 0;
  std::vector<Node> roots;  // part g: its root node, off = its rank
  std::vector<Instance> tab;
};

extern "C" {

int32_t dcs_online_create(int32_t variant, uint64_t n, uint64_t N, uint64_t seed,
                          const dcs_params* params, uint32_t depth, void* stream,
                          dcs_online** online) {
  if (online == nullptr) return DCS_EINVAL;
  *online = nullptr;
  Params P;
  if (read_params(params, &P) != DCS_OK) return DCS_EINVAL;
  if (variant != 0 && variant != 1) return DCS_EINVAL;
  if (N > DCS_MAX_UNIVERSE || depth > DCS_MAX_ONLINE_DEPTH) return DCS_EINVAL;
  if (variant == 0 && n > N) return DCS_EINVAL;
  if (variant == 1 && N == 0 && n > 0) return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  auto* o = new dcs_online();
  o->variant = variant;
  o->n = n;
  o->N = N;
  o->seed = seed;
  o->P = P;
  o->depth = depth;
  const uint64_t parts = 1ull << depth;
  o->roots.assign(parts, Node{0, 0, 0, 0, 0});
  if (n > 0) {
    Instance I{};
    I.n = n;
    I.N = N;
    I.seed = seed;
    I.n0 = P.n0;
    I.dense_ratio = P.dense_ratio;
    I.variant = static_cast<uint32_t>(variant);
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    rc = own_workspace(c, sizeof(Node) * parts, &ws);
    if (rc == DCS_OK) {
      Node* dev = static_cast<Node*>(ws);
      if (dcs::launch_part_roots(I, depth, dev, s) != hipSuccess ||
          hipMemcpyAsync(o->roots.data(), dev, sizeof(Node) * parts, hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        rc = DCS_EHIP;
    }
    if (rc) {
      delete o;
      return rc;
    }
  }
  *online = o;
  return DCS_OK;
}

int32_t dcs_online_counts(const dcs_online* o, uint64_t first, uint64_t count, uint64_t* counts,
                          uint64_t* ranks) {
  if (o == nullptr || first > o->roots.size() || count > o->roots.size() - first) return DCS_EINVAL;
  for (uint64_t i = 0; i < count; ++i) {
    const Node& v = o->roots[first + i];
    if (counts) counts[i] = v.nv;
    if (ranks) ranks[i] = v.off;
  }
  return DCS_OK;
}

int32_t dcs_online_next(dcs_online* o, uint64_t first, uint64_t count, uint64_t* out_dev,
                        uint64_t capacity, uint64_t* written, void* stream) {
  if (o == nullptr || first > o->roots.size() || count > o->roots.size() - first) return DCS_EINVAL;
  uint64_t total = 0;
  for (uint64_t i = 0; i < count; ++i) total += o->roots[first + i].nv;
  if (written) *written = total;
  if (total > capacity) return DCS_ENOMEM;
  if (total == 0) return DCS_OK;
  if (out_dev == nullptr) return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  // every non-empty part is an instance rooted at its node of the whole tree
  const uint64_t rank0 = o->roots[first].off;
  std::vector<Instance>& tab = o->tab;
  tab.clear();
  uint64_t tb = 0, tt = 0, leaf_cap = 0;
  uint32_t stack_depth = 1;
  bool second = false;
  const uint32_t v = static_cast<uint32_t>(o->variant);
  for (uint64_t i = 0; i < count; ++i) {
    const Node& r = o->roots[first + i];
    if (r.nv == 0) continue;
    const Plan pl = make_plan(r.nv, r.Nv, o->P.n0, o->P.dense_ratio, v, cut_bias_for(v, r.nv));
    Instance I{};
    I.n = r.nv;
    I.N = r.Nv;
    I.base = r.lo;
    I.root = r.id;
    I.seed = o->seed;
    I.out_offset = r.off - rank0;
    I.thread_base = tb;
    I.top_base = tt;
    I.n0 = o->P.n0;
    I.dense_ratio = o->P.dense_ratio;
    I.variant = v;
    I.cut = pl.cut;
    I.top_cut = pl.top_cut;
    tb += pl.threads;
    tt += pl.top_threads;
    leaf_cap += pl.leaf_cap;
    second = second || pl.second_round;
    stack_depth = std::max(stack_depth, pl.stack_depth);
    tab.push_back(I);
  }
  const uint32_t n_inst = static_cast<uint32_t>(tab.size());
  const TreeLayout L = tree_layout(n_inst, leaf_cap, tb, stack_depth, tt, second);
  void* ws = nullptr;
  rc = own_workspace(c, L.total, &ws);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = stage_upload(c, tab.data(), sizeof(Instance) * n_inst, static_cast<char*>(ws) + L.inst, s);
  if (rc) return rc;
  // the parts are subtrees of the whole sample's tree
  Instance whole{};
  whole.n = o->n;
  whole.N = o->N;
  whole.seed = o->seed;
  whole.n0 = o->P.n0;
  whole.dense_ratio = o->P.dense_ratio;
  whole.variant = v;
  return run_tree_pipeline(c, ws, L, nullptr, n_inst, tb, tt, leaf_cap, stack_depth, out_dev, s,
                           error_word(c, stream), leaf_wgs_for(c, v, total), nullptr, &whole);
}

int32_t dcs_online_destroy(dcs_online* o) {
  delete o;
  return DCS_OK;
}

// ---- status, timing, diagnostics -------------------------------------------
int32_t dcs_synchronize(void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return DCS_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  // this stream's error word: everything its calls latched since the last
  // synchronize (read and cleared in stream order, after the stream's work)
  unsigned int* word = error_word(c, stream);
  unsigned int any = 0;
  if (hipMemcpyAsync(&any, word, sizeof(any), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DCS_EHIP;
  if (any != 0 && (hipMemsetAsync(word, 0, sizeof(unsigned int), s) != hipSuccess ||
                   hipStreamSynchronize(s) != hipSuccess))
    return DCS_EHIP;
  // both rounds of a call ran out of job slots: plan larger capacities
  if (any & dcs::kErrLeafCapacity) leaf_capacity_exceeded();
  if (g_profile) {
    for (Timing& t : g_timings) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
        g_prof_ms[t.kind] += ms;
        g_prof_n[t.kind] += 1;
      }
    }
    release_timings();
  }
  return any ? DCS_EDEVICE : DCS_OK;
}

const char* dcs_status_string(int32_t st) {
  switch (st) {
    case DCS_OK: return "ok";
    case DCS_EINVAL: return "invalid argument";
    case DCS_ENOMEM: return "workspace too small or device allocation failed";
    case DCS_EHIP: return "HIP runtime error";
    case DCS_EOVERFLOW: return "Bernoulli count exceeds capacity";
    case DCS_EDEVICE: return "a kernel latched an error (capacity bound exceeded)";
    case DCS_ENOTSUP: return "not supported";
    default: return "unknown status";
  }
}

int32_t dcs_tune_set(int32_t variant, uint32_t log2_n, int32_t cut_bias, uint32_t leaf_wgs_per_cu) {
  if ((variant != 0 && variant != 1) || log2_n >= kTuneClasses || cut_bias < -16 || cut_bias > 16 ||
      leaf_wgs_per_cu > 64)
    return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  g_tune[variant][log2_n] = Tune{cut_bias, leaf_wgs_per_cu};
  return DCS_OK;
}

int32_t dcs_tune_get(int32_t variant, uint32_t log2_n, int32_t* cut_bias,
                     uint32_t* leaf_wgs_per_cu) {
  if ((variant != 0 && variant != 1) || log2_n >= kTuneClasses || cut_bias == nullptr ||
      leaf_wgs_per_cu == nullptr)
    return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  *cut_bias = g_tune[variant][log2_n].cut_bias;
  *leaf_wgs_per_cu = g_tune[variant][log2_n].leaf_wgs_per_cu;
  return DCS_OK;
}

int32_t dcs_tune_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& row : g_tune)
    for (auto& t : row) t = Tune{};
  return DCS_OK;
}

int32_t dcs_debug_plan(int32_t variant, uint64_t n, uint64_t N, const dcs_params* params,
                       uint64_t* info) {
  Params P;
  if (info == nullptr || (variant != 0 && variant != 1) || read_params(params, &P) != DCS_OK ||
      N > DCS_MAX_UNIVERSE || (variant == 0 && n > N) || (variant == 1 && N == 0 && n > 0))
    return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  const uint32_t v = static_cast<uint32_t>(variant);
  const Plan pl = make_plan(n, N, P.n0, P.dense_ratio, v, cut_bias_for(v, n));
  info[0] = pl.cut;
  info[1] = pl.threads;
  info[2] = pl.stack_depth;
  info[3] = pl.leaf_cap;
  info[4] = leaf_bound(n, N, P.n0, P.dense_ratio, v);
  info[5] = pl.second_round ? 1 : 0;
  return DCS_OK;
}

int32_t dcs_debug_lookback_help(uint32_t polls) {
  g_debug_help_polls.store(polls);
  return DCS_OK;
}

int32_t dcs_debug_leaf_kernels(int32_t mask) {
  if (mask > 7) return DCS_EINVAL;
  g_debug_takes.store(mask < 0 ? -1 : mask);
  return DCS_OK;
}

int32_t dcs_debug_bernoulli_list(uint32_t words) {
  if (words > 2 * dcs::kMaxN0 + 64) return DCS_EINVAL;
  g_debug_bern_list.store(words);
  return DCS_OK;
}

int32_t dcs_debug_leaf_capacity(uint64_t capacity, int32_t reset_boost, uint32_t* boost) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (capacity >= dcs::kMaxLeafJobs) return DCS_EINVAL;
  g_debug_leaf_cap.store(capacity);
  if (boost != nullptr) *boost = g_cap_boost.load();
  if (reset_boost) g_cap_boost.store(1);
  return DCS_OK;
}

int32_t dcs_profile_enable(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  release_timings();
  for (int i = 0; i < kProfKinds; ++i) {
    g_prof_ms[i] = 0;
    g_prof_n[i] = 0;
  }
  g_profile = enable != 0;
  return DCS_OK;
}

int32_t dcs_profile_kinds(uint32_t mask) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof_mask = mask;
  return DCS_OK;
}

int32_t dcs_profile_read(int32_t kind, double* total_ms, uint64_t* launches) {
  if (kind < 0 || kind >= kProfKinds || total_ms == nullptr || launches == nullptr) return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  *total_ms = g_prof_ms[kind];
  *launches = g_prof_n[kind];
  return DCS_OK;
}

int32_t dcs_debug_primitive(int32_t op, const void* x_dev, const void* x2_dev, void* y_dev,
                            uint64_t count, uint64_t p0, uint64_t p1, uint64_t p2, uint64_t p3,
                            void* stream) {
  if (op < 0 || op > 9 || (count > 0 && (x_dev == nullptr || y_dev == nullptr))) return DCS_EINVAL;
  if ((op == 4 || op == 5) && count > 0 && x2_dev == nullptr) return DCS_EINVAL;
  return hip_status(dcs::launch_debug(op, x_dev, x2_dev, y_dev, count, p0, p1, p2, p3,
                                      static_cast<hipStream_t>(stream)));
}

}  // extern "C"
