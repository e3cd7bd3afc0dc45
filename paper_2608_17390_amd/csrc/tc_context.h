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

// A pinned host buffer and a device buffer of the same size, reused across
// calls; `ev` marks the end of the last copy and kernels that used it.
struct Slot {
  void* host = nullptr;
  void* dev = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

// Layout of an uploaded edit list: descriptors, per-level node rectangles
// of the dirty update, and SET patch bytes.
struct EditPlan {
  int32_t n = 0;
  int32_t top = 0;
  size_t off_edits = 0, off_rects = 0, off_patch = 0, total = 0;
  int32_t max_w = 1, max_h = 1;
  std::vector<int32_t> nrect, rmw, rmh;   // per level 0..top
};

// Device tables of a render call: views, packet prefix and queue counter.
struct ViewPlan {
  int32_t n = 0;
  int64_t rays = 0, npkt = 0;
  size_t off_views = 0, off_prefix = 0, off_counter = 0, off_rows = 0, total = 0;
  size_t off_queue = 0;
  uint32_t qcap = 0;           // split queue capacity (0: no split pass)
  int32_t qwaves = 1;          // waves per queued ray in the split pass
  std::vector<tci_view> views;
  std::vector<int64_t> prefix;
  std::vector<int32_t> rows;   // tile rows of every view, longest walks first
};

tc_status fail(tc_context* c, tc_status st, const char* fmt, ...);
tc_status hip_fail(tc_context* c, hipError_t e, const char* what);
tc_status set_device(tc_context* ctx);
tc_status acquire(tc_context* ctx, size_t bytes, Slot** out);
tc_status release(tc_context* ctx, Slot* s, hipStream_t st);

tc_status validate_edits(tc_context* ctx, const tc_edit* edits, int32_t n,
                         size_t* patch_bytes);
// Fill `plan` and write the upload image of the edit list to `host`
// (plan.total bytes; call plan_edits with host == nullptr to size it).
void plan_edits(const tci_map& d, const tc_edit* edits, int32_t n,
                size_t patch_bytes, char* host, EditPlan& plan);
hipError_t enqueue_edits(const tci_map& d, uint32_t* map, const char* dev,
                         const EditPlan& plan, hipStream_t s);

// With allow_split false the plan has no split queue (qcap 0), whatever
// the context's split budget.
tc_status plan_views(tc_context* ctx, const tc_view* views, int32_t n,
                     ViewPlan& plan, bool allow_split = true);
void write_views(const ViewPlan& plan, char* host);
// `kev`, if given, receives event records before the traversal kernel,
// after it and after the split pass (the last only when that pass runs).
// With counters_zeroed the queue counters at plan.off_counter were uploaded
// as zeros with the tables (bytes [0, plan.off_queue)), so no kernel clears
// them; a captured frame, which replays, clears them itself.
hipError_t enqueue_render(tc_context* ctx, const tci_map& d, const char* dev,
                          const ViewPlan& plan, void* out, hipStream_t s,
                          hipEvent_t* kev = nullptr, bool* split_ran = nullptr,
                          bool counters_zeroed = false);

tci_render_opts render_opts(const tc_context* c);

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
  uint64_t map_generation = 0;  // bumped by every tc_load_columns
  // staging ring
  tci::Slot ring[tci::kRing];
  int ring_next = 0;
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
  int32_t boost = 0;
  int32_t split_budget = 128;
  int32_t beam_passes = 4;
  int32_t split_waves = 4;
  int32_t split_queue = 1 << 17;
  int32_t march_steps = 128;
  int32_t march_bisect = 4;
  int32_t march_far = 600;
  unsigned long long* d_count = nullptr;
  // TC_OPT_KERNEL_TIMING: events of the last timed render call
  int32_t kernel_timing = 0;
  hipEvent_t kev[3] = {nullptr, nullptr, nullptr};
  bool kev_valid = false, kev_split = false;
  // a running server owns the map (tc_server.cpp)
  void* server = nullptr;
};

#define TC_HIP(call, what)                                        \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) return tci::hip_fail(ctx, e_, what);    \
  } while (0)
