// Private host-side state of a library context and the helpers the host
// translation units share.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "tc.h"
#include "tc_internal.h"

namespace tci {

constexpr int kRing = 16;
// Bytes of each ring slot's pinned and device table buffers, allocated when
// the context is created: the tables of a render of up to about a thousand
// views, or an edit list with about 80 KiB of SET patches, fit without
// growing a slot.
constexpr size_t kSlotBytes = 256 << 10;
// Pyramid levels the dirty update after edits computes per launch, all from
// the level below the group: a node then combines at most 8 x 8 nodes of
// that level, a window entry at most 8 x 8.
constexpr int32_t kUpdateGroup = 3;

// A pinned host buffer and a device buffer of the same size, reused across
// calls, plus a device-only split queue (never uploaded, so it has no host
// mirror); `ev` marks the end of the last copy and kernels that used them.
struct Slot {
  void* host = nullptr;
  void* dev = nullptr;
  size_t cap = 0;
  uint4* queue = nullptr;
  uint32_t qcap = 0;
  // two split queue counters for renders whose tables travel in the
  // kernels' arguments, used in turn: a render counts in ctr[ctr_turn] and
  // clears ctr[1 - ctr_turn] for the slot's next such render (both zero at
  // allocation; ctr_dirty: a launch failed on the way, clear both first)
  uint32_t* ctr = nullptr;
  int ctr_turn = 0;
  bool ctr_dirty = false;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

tc_status fail(tc_context* c, tc_status st, const char* fmt, ...);
tc_status hip_fail(tc_context* c, hipError_t e, const char* what);
tc_status set_device(tc_context* ctx);
// The next ring slot, once its last use has completed, with table buffers of
// at least `bytes` (a slot grows only for tables beyond kSlotBytes).
tc_status acquire(tc_context* ctx, size_t bytes, Slot** out);
tc_status release(tc_context* ctx, Slot* s, hipStream_t st);
// Allocate every ring slot's buffers and a split queue of `qcap` entries per
// slot (at context creation, and again when TC_OPT_SPLIT_QUEUE grows).
tc_status ring_alloc(tc_context* ctx, uint32_t qcap);
// Device and pinned allocations, counted per context (tc_get_option of
// TC_INFO_ALLOCATIONS).
hipError_t dev_alloc(tc_context* ctx, void** p, size_t bytes);
hipError_t host_alloc(tc_context* ctx, void** p, size_t bytes);

// check_edits / make_view_plan (tc_plan.h) with the context's knobs, the
// reason of a failure going to the context's error message.
tc_status validate_edits(tc_context* ctx, const tc_edit* edits, int32_t n,
                         size_t* patch_bytes);
// Enqueue the edits of `plan` (uploaded at dev) on the map at `map`, then
// the dirty update of its pyramid, window levels and, if vx is given, of
// the voxel occupancy pyramid at vox.  The update also clears
// zero[0 .. nzero) (a captured frame's render counters) before it ends.
hipError_t enqueue_edits(const tci_map& d, uint32_t* map, const char* dev,
                         const EditPlan& plan, hipStream_t s,
                         const tci_voxels* vx = nullptr, uint32_t* vox = nullptr,
                         uint64_t* zero = nullptr, int32_t nzero = 0);
// The 64-bit counters at plan.off_counter that enqueue_render clears before
// its kernels unless told they are zero already: 0, 1 or 2.
int32_t render_counter_words(const tc_context* ctx, const ViewPlan& plan);
// (Re)build the context's voxel occupancy pyramid for its map and
// TC_OPT_VOXEL_SHAPE (freeing it when the shape is 0); synchronises s.
tc_status build_voxels(tc_context* ctx, hipStream_t s);

tc_status plan_views(tc_context* ctx, const tc_view* views, int32_t n,
                     ViewPlan& plan, bool allow_split = true);
// `kev`, if given, receives event records before the traversal kernel,
// after it and after the split pass (the last only when that pass runs).
// With counters_zeroed the queue counters at plan.off_counter were uploaded
// as zeros with the tables (bytes [0, plan.off_queue)), so no kernel clears
// them; a captured frame, which replays, clears them itself.  `queue` holds
// the split queue (plan.qcap entries); nullptr: it follows the tables at
// dev + plan.off_queue.  With `inl` (hierarchical mode, no read counting)
// the tables travel in the kernels' arguments instead of at dev, and the
// queue length is the counter at qctr, which must be zero, and the render
// clears the counter at qzero.
hipError_t enqueue_render(tc_context* ctx, const tci_map& d, const char* dev,
                          const ViewPlan& plan, void* out, hipStream_t s,
                          hipEvent_t* kev = nullptr, bool* split_ran = nullptr,
                          bool counters_zeroed = false, uint4* queue = nullptr,
                          const tci_inline* inl = nullptr, uint32_t* qctr = nullptr,
                          uint32_t* qzero = nullptr);

tci_render_opts render_opts(const tc_context* c);

// Look up, once per device, the device address of the scratch array of
// tc_render_views_noalloc (tc_noalloc.hip); tc_create calls it.
tc_status noalloc_setup(tc_context* ctx);

}  // namespace tci

struct tc_context {
  int device = 0;
  int num_cu = 256;
  std::string err;
  // map
  int32_t W = 0, H = 0;
  uint32_t* map = nullptr;  // all levels
  size_t map_words = 0;
  tci_map desc{};
  uint64_t map_generation = 0;  // bumped by every tc_load_columns (and
                                // voxel pyramid rebuild)
  // voxel occupancy pyramid (render mode 5), built when vox_shape != 0
  int32_t vox_shape = 0;        // v | vz << 8 (cells, height units), 0: none
  uint32_t* vox = nullptr;
  size_t vox_words = 0;
  tci_voxels vdesc{};
  // staging ring (allocated by tc_create)
  tci::Slot ring[tci::kRing];
  int ring_next = 0;
  uint64_t allocs = 0;  // device and pinned allocations made so far
  // options
  int32_t render_mode = 0;
  int32_t start_level = 2;
  int32_t max_level = TCI_MAX_LEVELS - 1;
  int32_t xcd_remap = 64;
  int32_t persist_waves = 16;
  int32_t refill_min = 16;
  int32_t refill_iters = 16;
  int32_t count_reads = 0;
  int32_t tile_order = 2;
  int32_t packet_width = 8;
  int32_t boost = 0;
  int32_t split_budget = 120;
  int32_t beam_passes = 6;
  int32_t split_waves = 4;
  int32_t split_queue = 1 << 17;
  int32_t inline_tables = 1;   // TC_OPT_INLINE_TABLES
  int32_t march_steps = 128;
  int32_t march_bisect = 4;
  int32_t march_far = 600;
  unsigned long long* d_count = nullptr;
  // TC_OPT_KERNEL_TIMING: events of the last timed render call
  int32_t kernel_timing = 0;
  // markers on the stream before the traversal, between the kernels and
  // after the split pass (kev[0..2]); or, for calls whose kernels carry
  // their own events (kev_attached), each kernel's start and end (kev[0..1]
  // the traversal, kev[2..3] the split pass)
  hipEvent_t kev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool kev_valid = false, kev_split = false, kev_attached = false;
  // a running server owns the map (tc_server.cpp)
  void* server = nullptr;
};

#define TC_HIP(call, what)                                        \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) return tci::hip_fail(ctx, e_, what);    \
  } while (0)
