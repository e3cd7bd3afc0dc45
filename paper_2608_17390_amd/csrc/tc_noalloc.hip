// tc_render_views_noalloc: tc_render_views for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid allocation).  The per-call device tables (views, packet
// prefix, tile-row order, the split pass's queue counters and its queue)
// live in one file-scope device array, `scratch`, instead of a staging
// slot's device buffer; the call allocates nothing: it writes the tables
// into a pinned buffer of the staging ring (allocated by tc_create and
// never grown here, since the tables are limited to its size) and uploads
// them with one stream-ordered copy.
//
// Every call on a GPU shares that GPU's array.  Calls on one stream are
// ordered, so they do not interfere; calls that overlap on one GPU (other
// streams, other contexts on the same device, other host threads) race on
// the array and must not be issued.  The array keeps the last call's
// contents; the queue counters are uploaded as zeros with the tables on
// every call, and the queue itself is written before it is read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>

#include "tc_context.h"

namespace {

// The tables of one call: at most kNoAllocTables bytes, the size of a
// staging slot (about 2,000 views of a typical mix), then the split queue
// (65,536 entries of 16 bytes): 1.25 MiB per device in all.
constexpr size_t kNoAllocTables = tci::kSlotBytes;
constexpr size_t kNoAllocQueue = 65536;
constexpr size_t kNoAllocBytes = kNoAllocTables + kNoAllocQueue * tci::kQueueEntry;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

namespace tci {

// Called by tc_create with the context's device current: looks the array's
// device address up once per device (the array's name is not a device
// address in host code).
tc_status noalloc_setup(tc_context* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return fail(ctx, TC_INVALID_ARG, "tc_create: device index beyond %d", kMaxDevices - 1);
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch[ctx->device]) return TC_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_fail(ctx, e, "hipGetSymbolAddress(scratch)");
  g_scratch[ctx->device] = p;
  return TC_OK;
}

}  // namespace tci

extern "C" tc_status tc_render_views_noalloc(tc_context* ctx, const tc_view* views, int32_t n,
                                             tc_hit* out_device, void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (!ctx->map) return tci::fail(ctx, TC_NO_MAP, "tc_render_views_noalloc: no map loaded");
    if (ctx->server)
      return tci::fail(ctx, TC_INVALID_ARG, "tc_render_views_noalloc: a server owns the map");
    if (!out_device)
      return tci::fail(ctx, TC_INVALID_ARG, "tc_render_views_noalloc: out is NULL");
    if (ctx->render_mode == 5 && !ctx->vox)
      return tci::fail(ctx, TC_INVALID_ARG,
                       "tc_render_views_noalloc: render mode 5 needs TC_OPT_VOXEL_SHAPE");
    tci::ViewPlan plan;
    tc_status st = tci::plan_views(ctx, views, n, plan);
    if (st) return st;
    if (plan.off_queue > kNoAllocTables)
      return tci::fail(ctx, TC_INVALID_ARG,
                       "tc_render_views_noalloc: the tables of %d views take %zu bytes, more "
                       "than the %zu this entry point holds", n, plan.off_queue, kNoAllocTables);
    void* dev;
    {
      std::lock_guard<std::mutex> g(g_mu);
      dev = g_scratch[ctx->device];
    }
    if (!dev)
      return tci::fail(ctx, TC_DEVICE_ERROR, "tc_render_views_noalloc: no scratch address");
    st = tci::set_device(ctx);
    if (st) return st;
    // the split queue takes the rest of the array; longer queues are cut
    // (the rays beyond it finish in the first pass, with the same result)
    const size_t qoff = kNoAllocTables;
    plan.qcap = (uint32_t)std::min<size_t>(plan.qcap, kNoAllocQueue);
    // a ring slot's pinned buffer holds at least kSlotBytes, so acquire()
    // does not grow it; it waits for the slot's previous use
    tci::Slot* slot = nullptr;
    st = tci::acquire(ctx, plan.off_queue, &slot);
    if (st) return st;
    tci::write_views(plan, (char*)slot->host);
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(dev, slot->host, plan.off_queue, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = tci::enqueue_render(ctx, ctx->desc, (const char*)dev, plan, out_device, s, nullptr,
                              nullptr, true, (uint4*)((char*)dev + qoff));
    const tc_status rs = tci::release(ctx, slot, s);
    if (e != hipSuccess) return tci::hip_fail(ctx, e, "tc_render_views_noalloc");
    return rs;
  } catch (...) {
    return tci::fail(ctx, TC_OUT_OF_MEMORY, "tc_render_views_noalloc: host allocation failed");
  }
}
