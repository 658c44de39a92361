// dcs_host.hpp -- host-side planning and launch helpers shared by the C ABI
// implementation (dcs_api.hip) and the serving loop (dcs_server.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "../../include/dcs.h"
#include "dcs_kernels.hpp"

namespace dcs {
namespace host {

struct Params {
  uint32_t n0, dense_ratio;
};

// Validates dcs_params (NULL = defaults).
int32_t read_params(const dcs_params* p, Params* out);

// Per-instance plan: Algorithm P cut depth, tree threads, DFS stack bound and
// leaf-job capacity.
struct Plan {
  uint32_t cut = 0;
  uint64_t threads = 0;
  uint32_t top_cut = 0;      // frontier depth computed by the top kernel
  uint64_t top_threads = 0;  // 2^top_cut (0 for an empty instance)
  uint32_t stack_depth = 1;
  uint64_t leaf_cap = 0;
  // leaf_cap below the proven bound on the leaf jobs: the launch adds the
  // second round for tree threads whose leaves did not all fit
  bool second_round = false;
};
Plan make_plan(uint64_t n, uint64_t N, uint32_t n0, uint32_t dense_ratio, uint32_t variant,
               int32_t cut_bias);
// Leaf jobs of the tree of (n, N, n0, dense_ratio, variant) for every
// outcome of its random splits.
uint64_t leaf_bound(uint64_t n, uint64_t N, uint32_t n0, uint32_t dense_ratio, uint32_t variant);
// After a call latched a capacity error: later plans take larger capacities.
void leaf_capacity_exceeded();

// Workspace layout of a tree launch (byte offsets).  redo_words > 0: the
// second round's bitmap over tree threads (redo_words 32-bit words).
struct TreeLayout {
  size_t ctl = 0, inst = 0, leaves = 0, stacks = 0, frontier = 0, redo = 0, total = 0;
  uint64_t redo_words = 0;
};
TreeLayout tree_layout(uint32_t n_inst, uint64_t leaf_cap, uint64_t threads, uint32_t stack_depth,
                       uint64_t top_threads, bool second_round);

struct DeviceCtx {
  bool init = false;
  int cus = 256;
  int leaf_occupancy = 2;
  int bern_wave_occupancy = 8;
  int dense_occupancy = 8;
  int wb_occupancy = 8;
  int small_occupancy = 8;
  // launch-geometry overrides (never change the sample): DCS_LEAF_GRID sets
  // the number of leaf work-groups, DCS_CUT_BIAS shifts the Algorithm P cut;
  // when set they take precedence over the tuning table
  int64_t leaf_grid = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // device address of this device's copy of the allocation-free entry
  // point's static scratch array (hipGetSymbolAddress at set-up)
  void* noalloc_scratch = nullptr;
  // pinned host buffer for instance tables uploaded by single calls, and the
  // event after its last copy (waited for before it is written again)
  void* stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_done = nullptr;
  // the library's error words on this device (kErrSlots of them) and the
  // stream each one serves; slot 0 is the null stream's, the last one is
  // shared by streams beyond the others
  unsigned int* err_slots = nullptr;
  std::map<void*, int> err_slot_of;
};

// Error word of `stream` on the current device (assigned on first use);
// caller holds lock().
unsigned int* error_word(DeviceCtx* c, void* stream);

// Tuned launch geometry of a size class (variant, floor(log2 n)), set through
// dcs_tune_set; never changes a sample.
struct Tune {
  int32_t cut_bias = 0;          // added to the Algorithm P cut depth
  uint32_t leaf_wgs_per_cu = 0;  // leaf work-groups per compute unit, 0 = occupancy
};
constexpr uint32_t kTuneClasses = 64;
// Entry for an instance of n samples (caller holds lock()).
Tune tune_for(uint32_t variant, uint64_t n);
// Cut bias for an instance: the DCS_CUT_BIAS override, else the table's
// (caller holds lock()).
int32_t cut_bias_for(uint32_t variant, uint64_t n);
// Leaf work-groups per compute unit for a launch whose largest class is
// (variant, n): the table's, clamped to the kernel's occupancy.
uint32_t leaf_wgs_for(const DeviceCtx* c, uint32_t variant, uint64_t n);

// The library lock (guards the per-device contexts, the latched-error
// registry and kernel timing).
std::mutex& lock();
// Context of the current device (creates it on first use); caller holds lock().
int32_t device_ctx(DeviceCtx** out);
// Enqueue reset + tree + leaf on `s` for the instances in the workspace
// (`single` != NULL: store that one instance first); the kernels latch
// errors at `err` (nullptr: the workspace's own control block); caller
// holds lock().
// Leaf work-groups: DCS_LEAF_GRID if set, else cus * leaf_wgs_per_cu (both
// leaf kernels use it).
// whole: an instance whose canonical tree holds every leaf of the launch
// (the sample whose parts the instances are); with `single` it decides which
// specialised leaf kernels can be left out.
int32_t run_tree_pipeline(DeviceCtx* c, void* ws, const TreeLayout& L, const Instance* single,
                          uint32_t n_inst, uint64_t threads, uint64_t top_threads,
                          uint64_t leaf_cap, uint32_t stack_depth, uint64_t* out, hipStream_t s,
                          unsigned int* err, uint32_t leaf_wgs_per_cu,
                          uint64_t* part_out = nullptr, const Instance* whole = nullptr);

// Kernel timing with pooled HIP events on the launch stream (dcs_profile_*):
// kinds as listed at dcs_profile_read; caller holds lock().
struct Timing {
  int kind;
  int dev;
  hipEvent_t a, b;  // a == nullptr: this launch is not timed
};
void timing_begin(int kind, hipStream_t s, Timing* t);
void timing_end(hipStream_t s, Timing* t);
}  // namespace host
}  // namespace dcs
