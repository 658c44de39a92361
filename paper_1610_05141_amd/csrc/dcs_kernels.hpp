// dcs_kernels.hpp -- device data layout and kernel launch helpers shared by
// the kernels and the host runtime of the sampler library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dcs {

// One instance of the sampling problem (single call: one entry; batch: many).
struct Instance {
  uint64_t n;           // sample size (without / with replacement)
  uint64_t N;           // universe 1..N
  uint64_t seed;
  uint64_t out_offset;  // first output element of this instance
  uint64_t thread_base; // first tree-kernel thread of this instance
  uint64_t top_base;    // first top-kernel thread (= its first frontier slot)
  uint32_t n0;
  uint32_t dense_ratio;
  uint32_t variant;     // 0 without replacement, 1 with replacement
  uint32_t cut;         // Algorithm P depth: 2^cut tree threads
  uint32_t top_cut;     // depth of the frontier the top kernel computes (<= cut)
  // Part mode (part_depth > 0): only the subtree of the depth-part_depth
  // node `part` is sampled, with offsets counted from its first value; cut
  // and top_cut then count from the root and include part_depth.
  uint32_t part_depth;
  uint64_t part;
  uint64_t part_cap;    // nothing is sampled if the part holds more values
  // Elements before this instance's range: its root covers base+1 .. base+N
  // (0 except for the segments of an uneven universe and online parts).
  uint64_t base;
  // Node id of the instance's root in the tree of its seed: 0 stands for 1,
  // the whole tree; an online part's subtree keeps the id its root has in
  // the whole sample's tree, so its splits and leaves are the same.
  uint64_t root;
};

// A recursion-tree node (Fig. 1): node id (root 1, children 2i, 2i+1), the
// range lo+1 .. lo+Nv, the sample count nv and the output offset off of its
// part of the (sorted) sample.
struct Node {
  uint64_t id, lo, Nv, nv, off;
};

// A leaf job for the leaf kernel, self-contained: the node, its instance's
// seed, the absolute output offset of its first value, and its kind.
struct Leaf {
  uint64_t id, lo, Nv;
  uint64_t off;   // absolute: instance output offset + node offset
  uint64_t seed;
  uint32_t nv;    // < n0 <= 4096, or <= kFillPiece for constant pieces
  uint32_t flags; // kind (bits 0-1) | n0 << 8
};
static_assert(sizeof(Leaf) == 48, "leaf record layout");

// Leaf kinds.
constexpr uint32_t kKindSparse = 0;  // Algorithm H semantics
constexpr uint32_t kKindDense = 1;   // Algorithm B with repair
constexpr uint32_t kKindWr = 2;      // with replacement: sorted draws
constexpr uint32_t kKindFill = 3;    // with replacement, N_v = 1: constant

// Control block at the start of a workspace.
struct Control {
  // leaf jobs appended by the tree kernels: low 32 bits count the sparse and
  // with-replacement leaves over power-of-two ranges (filled from the front
  // of the job array),
  // high 32 bits all others (filled from the back); one 64-bit atomic
  // serves both.  Jobs that did not fit count too (see `granted`).
  unsigned long long leaf_counts;
  // where the kernels latch error bits (kErr*): a library-owned word of the
  // launch stream, or `error` below when the caller reads the block itself
  // (the serving loop); set by k_reset / k_zero at the start of every call
  unsigned int* err;
  // ~0, or leaf_counts just before the first job whose slots did not fit:
  // a job gets its slots iff the slots asked for up to it (front and back
  // together, in the order of the atomic) fit the capacity, so the granted
  // jobs are those counted here and they never overlap.  Every tree thread
  // stops at its first job that does not fit, so the counts stay far below
  // 2^32 (capacity plus threads).
  unsigned long long granted;
  unsigned int error;              // this call's own error bits (see `err`)
  unsigned int pad;
  unsigned long long bern_count;   // Bernoulli: total hits (copied to the caller)
  // second round (tree threads whose leaves did not all get a slot, run
  // again): its jobs, all on the back list, as leaf_counts and granted
  unsigned long long leaf_counts2;
  unsigned long long granted2;
  // the call's output (tree calls): the tree kernels write leaves of a few
  // values themselves
  uint64_t* out;
};
static_assert(sizeof(Control) == 64, "control block layout");

// Library-owned error words, one per stream that has launched work (the
// last one shared by streams beyond kErrSlots - 1), per device: kept in
// device memory the library owns, so that nothing outside a call's own
// buffers is ever written after the call, and read and cleared by
// dcs_synchronize for its stream only.
constexpr int kErrSlots = 64;
// Device address of this device's error words (call with the device current).
hipError_t error_slots(unsigned int** out);

constexpr unsigned kErrLeafCapacity = 1u;   // more leaves than the workspace holds
constexpr unsigned kErrStackDepth = 2u;     // tree deeper than the planned stack
constexpr unsigned kErrSpinLimit = 4u;      // Bernoulli look-back waited too long
constexpr unsigned kErrLeafTooLarge = 8u;   // a leaf exceeds the kernel's LDS bound
constexpr unsigned kErrRestartLimit = 16u;  // whole-range B: no attempt accepted

constexpr uint64_t kMaxLeafJobs = 1ull << 31;  // keeps the two halves of leaf_counts apart
constexpr int kLeafBlock = 512;             // threads of a leaf work-group
constexpr int kBernBlock = 256;             // threads of a Bernoulli work-group
constexpr uint32_t kMaxN0 = 4096;           // largest n0 (LDS bound of a leaf)
constexpr uint64_t kFillPiece = 1ull << 16; // constant-fill leaves are cut to this
// Sparse and with-replacement leaves of at most this many values are
// sampled by the tree kernels themselves (no job record).
constexpr uint32_t kInlineMax = 32;
// Bernoulli chunks (both kernels) are handed out by kTicketClasses
// counters (7: coprime to the 8 XCDs), kTicketStride words apart.
constexpr uint32_t kTicketClasses = 7;
constexpr uint32_t kTicketStride = 32;
constexpr uint32_t kTicketWords = kTicketClasses * kTicketStride;

// Kernel launchers (defined in dcs_kernels.hip).
// Start a call on a control block: zero its counters and its own error word
// and point its kernels' error latch at `err` (nullptr: at the block's own
// error word); if `single` is non-null, also store that instance as entry 0
// of the instance table.
// redo (may be null): the second round's bitmap over tree threads, redo_words
// 32-bit words, zeroed here too.  out: the call's output.
hipError_t launch_reset(Control* ctl, const Instance* single, Instance* table, unsigned int* err,
                        uint32_t* redo, uint64_t redo_words, uint64_t* out, hipStream_t stream);
// launch_reset for a Bernoulli call plus zeroing of its look-back status words
// and its kTicketWords chunk counters.
hipError_t launch_zero(Control* ctl, unsigned long long* status, uint64_t n,
                       unsigned long long* tickets, unsigned int* err, hipStream_t stream);
// Resident leaf work-groups per compute unit.
int leaf_occupancy();
// Resident k_leaf_dense work-groups (one wave each) per compute unit.
int dense_occupancy();
// Resident k_leaf_small work-groups (one wave each) per compute unit.
int small_occupancy();
// Resident work-groups per compute unit of the double-precision Bernoulli
// kernel holding lds_cap offsets in LDS, and of the one-wave
// single-precision one.
int bern_occupancy(uint32_t lds_cap);
int bern64_wave_occupancy(uint32_t lds_cap);
int bern_wave_occupancy();
// Top of the tree: 2^top_cut threads per instance walk to the depth-top_cut
// frontier (written to `frontier`, one slot per top thread).
// part_out (part mode only, else null): receives the part's count and rank.
hipError_t launch_tree_top(const Instance* inst, uint32_t n_inst, uint64_t top_threads,
                           Node* frontier, Leaf* leaves, uint64_t leaf_cap, Control* ctl,
                           uint64_t* part_out, hipStream_t stream);
// Below the frontier.  redo == null: a leaf that finds the job array full
// latches kErrLeafCapacity.  Otherwise round 0 marks its thread in the redo
// bitmap instead (the thread stops; the leaves it did hand over are sampled
// by the first leaf pass), and round 1 runs only the marked threads again,
// from their frontier node, into the emptied job array (every job on the
// back list), latching kErrLeafCapacity if that does not fit either.  A
// leaf's values go to fixed places of the output, so a leaf handed over in
// both rounds is written twice with the same values.
hipError_t launch_tree(const Instance* inst, uint32_t n_inst, uint64_t total_threads,
                       const Node* frontier, Leaf* leaves, uint64_t leaf_cap, Node* stacks,
                       uint32_t stack_depth, Control* ctl, uint32_t* redo, int round,
                       hipStream_t stream);
// Work-group leaf kernels: kLeafFront = the front list (sparse and
// with-replacement leaves over power-of-two ranges, except sparse ones
// expected to repeat); kLeafBack = the back list's jobs that no other kernel
// takes; kLeafOnce = the back list's sparse leaves of more than 1024 values
// with n_v^2 >= 2 N_v (one-pass sampler).
constexpr int kLeafFront = 0, kLeafBack = 1, kLeafOnce = 2;
// Kinds that k_leaf_mixed runs itself because their own kernel is not
// launched (never changes a sample): dense leaves over ranges up to 2^16,
// sparse and with-replacement leaves of at most 1024 values, the one-pass
// sparse leaves.
constexpr uint32_t kTakesDense = 1, kTakesSmall = 2, kTakesOnce = 4;
hipError_t launch_leaf(int which, const Leaf* leaves, uint64_t leaf_cap, uint64_t* out,
                       Control* ctl, uint32_t grid, hipStream_t stream, uint32_t takes = 0);
// The second round's jobs (all on the back list, every kind run by the
// work-group kernels of the back list; k_leaf_once's too when `takes` has
// kTakesOnce, which then is not launched); returns at once when round 0
// handed over every leaf.
hipError_t launch_leaf_round2(const Leaf* leaves, uint64_t leaf_cap, uint64_t* out, Control* ctl,
                              uint32_t grid, hipStream_t stream, uint32_t takes = 0);
// Dense leaves of the back list whose range fits 16-bit positions, one wave
// per leaf (k_leaf_mixed skips them).
hipError_t launch_leaf_dense(const Leaf* leaves, uint64_t leaf_cap, uint64_t* out, Control* ctl,
                             uint32_t grid, hipStream_t stream);
// Sparse and with-replacement leaves of the back list with at most 1024
// values, one wave per leaf (k_leaf_mixed skips them).
hipError_t launch_leaf_small(const Leaf* leaves, uint64_t leaf_cap, uint64_t* out, Control* ctl,
                             uint32_t grid, hipStream_t stream);
// Bernoulli chunk kernels: kBernFp64Group = k_bern (double-precision skips,
// one work-group per chunk), kBernFp32Wave = k_bern_wave (p >= 2^-10),
// kBernFp64Wave = k_bern64_wave (double precision, one wave per chunk, for
// chunks whose expected hits fit a small LDS list).
constexpr int kBernFp64Group = 0, kBernFp32Wave = 1, kBernFp64Wave = 2;
// Largest LDS position list (32-bit words) for which the one-wave
// double-precision kernel is chosen.
constexpr uint32_t kBern64WaveMaxList = 1024;
hipError_t launch_bernoulli(double p, uint64_t N, uint64_t seed, uint64_t chunk,
                            uint64_t n_chunks, int fp32, double c64, float c32,
                            unsigned long long* status, uint64_t* out, uint64_t capacity,
                            uint64_t* count_dev, Control* ctl, unsigned long long* tickets,
                            uint32_t grid, uint32_t lds_cap, uint32_t help_polls,
                            hipStream_t stream);
// Polls of a Bernoulli look-back on a chunk that has published nothing
// before the waiting wave counts that chunk itself.
constexpr uint32_t kHelpPolls = 4096;
// Online sampling: the 2^depth part roots of instance I's depth-`depth` cut
// (node with off = the part's rank; an empty part has nv = 0, a leaf above
// the cut goes whole to the leftmost part below it).
hipError_t launch_part_roots(const Instance& I, uint32_t depth, Node* roots, hipStream_t stream);
// Uneven universe: fills count, seed and output offset of the K segment
// instances (their base and N set) from the splits of the binomial tree of
// depth D over them; counts (may be null) receives the K counts.
hipError_t launch_segments(Instance* inst, uint64_t K, uint32_t D, uint64_t n, uint64_t N,
                           uint64_t seed, uint64_t* counts, hipStream_t stream);
// Whole-range Algorithm B: the state word of a call (attempt + 1 once an
// attempt is accepted, else 0) and its accepted hit count.
struct WbState {
  unsigned long long accepted;  // attempt + 1 once accepted and repaired
  unsigned long long hits;
  unsigned long long pending;   // attempt + 1 once it passed the acceptance test
  unsigned long long fresh;     // new values found by the first repair round
};
// Removal counts are kept per block of 2^kWbRemShift hit indices.
constexpr uint32_t kWbRemShift = 12;
// Workspace of one call: per-chunk hit counts (u32) and their exclusive
// prefix (u64); removal counts per block of hit indices (u32, turned into
// their exclusive prefix); the removal bitmap over hit indices (u64 words).
struct WbBuffers {
  WbState* state;
  uint32_t* cnt;
  uint64_t* off;
  uint32_t* rem;
  uint64_t rem_blocks;
  unsigned long long* bitmap;
  uint64_t words;
  uint64_t* tsum;  // kWbTileSums per-tile sums: the chunk counts', then the removal counts'
};
// The scans of the chunk counts and of the removal counts run over tiles of
// kWbTile entries: per-tile sums on the whole grid, their scan in one
// work-group, then each tile's scan offset by its sum's prefix.
constexpr uint32_t kWbTile = 4096;
constexpr uint32_t kWbMaxTiles = 512;  // per scan: up to 2^21 entries
constexpr uint32_t kWbTileSums = 2 * kWbMaxTiles;
// Zero the state, removal counts and bitmap; start the control block.
hipError_t launch_wb_zero(Control* ctl, const WbBuffers& b, uint64_t n_chunks, unsigned int* err,
                          hipStream_t stream);
// Attempt `attempt`: count pass, then the one-work-group scan / acceptance /
// repair, then the write pass (each returns at once if an earlier attempt
// was accepted).  full: rho = 1 (every element a hit).  last: latch
// kErrRestartLimit if this attempt is rejected too.
hipError_t launch_wb_count(uint64_t N, uint64_t seed, uint64_t chunk, uint64_t n_chunks, float c32,
                           int full, uint32_t attempt, const WbBuffers& b, uint32_t grid,
                           hipStream_t stream);
hipError_t launch_wb_mid(uint64_t n, uint64_t seed, uint64_t n_chunks, uint32_t attempt, int last,
                         const WbBuffers& b, Control* ctl, uint32_t repair_grid,
                         hipStream_t stream);
// Tiles a scan of `count` entries takes (at most kWbMaxTiles).
inline uint64_t wb_tiles(uint64_t count) { return (count + kWbTile - 1) / kWbTile; }
hipError_t launch_wb_write(uint64_t N, uint64_t seed, uint64_t chunk, uint64_t n_chunks, float c32,
                           int full, uint32_t attempt, const WbBuffers& b, uint64_t* out,
                           uint32_t grid, hipStream_t stream);
// Resident one-wave work-groups per compute unit of the count and write passes.
int wb_occupancy();
hipError_t launch_bernoulli_fill(uint64_t N, uint64_t* out, uint64_t capacity,
                                 uint64_t* count_dev, hipStream_t stream);
hipError_t launch_debug(int op, const void* x, const void* x2, void* y, uint64_t count,
                        uint64_t p0, uint64_t p1, uint64_t p2, uint64_t p3, hipStream_t stream);

}  // namespace dcs
