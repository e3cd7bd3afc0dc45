// Host runtime of the library: the C ABI declared in include/tc.h.
//
// Owns the device copy of the map (packed columns plus the min/max pyramid,
// one allocation), validates every call before enqueueing anything (with
// the planning layer of tc_plan.cpp), stages
// small per-call tables (views, edit lists) through a ring of pinned host
// buffers with matching device buffers, and launches the kernels of
// tc_map.hip and tc_render.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tc_context.h"

using tci::fail;
using tci::hip_fail;
using tci::set_device;

namespace {

std::string g_create_error;

}  // namespace

namespace tci {

tc_status fail(tc_context* c, tc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

tc_status hip_fail(tc_context* c, hipError_t e, const char* what) {
  return fail(c, e == hipErrorOutOfMemory ? TC_OUT_OF_MEMORY : TC_DEVICE_ERROR,
              "%s: %s", what, hipGetErrorString(e));
}

tc_status set_device(tc_context* ctx) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  return TC_OK;
}

hipError_t dev_alloc(tc_context* ctx, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) ctx->allocs++;
  return e;
}

hipError_t host_alloc(tc_context* ctx, void** p, size_t bytes) {
  hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
  if (e == hipSuccess) ctx->allocs++;
  return e;
}

tc_status ring_alloc(tc_context* ctx, uint32_t qcap) {
  for (Slot& s : ctx->ring) {
    if (s.pending) {
      TC_HIP(hipEventSynchronize(s.ev), "hipEventSynchronize(staging)");
      s.pending = false;
    }
    if (!s.ev) TC_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming), "hipEventCreate");
    if (!s.host) TC_HIP(host_alloc(ctx, &s.host, kSlotBytes), "hipHostMalloc(staging)");
    if (!s.dev) {
      TC_HIP(dev_alloc(ctx, &s.dev, kSlotBytes), "hipMalloc(staging)");
      s.cap = kSlotBytes;
    }
    if (!s.ctr) {
      TC_HIP(dev_alloc(ctx, (void**)&s.ctr, 16), "hipMalloc(queue counters)");
      TC_HIP(hipMemset(s.ctr, 0, 16), "hipMemset(queue counters)");
    }
    if (s.qcap < qcap) {
      if (s.queue) {
        (void)hipFree(s.queue);
        s.queue = nullptr;
        s.qcap = 0;
      }
      TC_HIP(dev_alloc(ctx, (void**)&s.queue, sizeof(uint4) * (size_t)qcap),
             "hipMalloc(split queue)");
      s.qcap = qcap;
    }
  }
  return TC_OK;
}

tc_status acquire(tc_context* ctx, size_t bytes, Slot** out) {
  Slot& s = ctx->ring[ctx->ring_next];
  ctx->ring_next = (ctx->ring_next + 1) % kRing;
  if (s.pending) {
    TC_HIP(hipEventSynchronize(s.ev), "hipEventSynchronize(staging)");
    s.pending = false;
  }
  if (s.cap < bytes) {
    // tables beyond kSlotBytes: the slot grows (the only allocation a call
    // can make after tc_create)
    size_t cap = (bytes + 4095) & ~(size_t)4095;
    if (s.host) { (void)hipHostFree(s.host); s.host = nullptr; }
    if (s.dev) { (void)hipFree(s.dev); s.dev = nullptr; }
    s.cap = 0;
    TC_HIP(host_alloc(ctx, &s.host, cap), "hipHostMalloc(staging)");
    TC_HIP(dev_alloc(ctx, &s.dev, cap), "hipMalloc(staging)");
    s.cap = cap;
  }
  *out = &s;
  return TC_OK;
}

tc_status release(tc_context* ctx, Slot* s, hipStream_t st) {
  TC_HIP(hipEventRecord(s->ev, st), "hipEventRecord(staging)");
  s->pending = true;
  return TC_OK;
}

tc_status validate_edits(tc_context* ctx, const tc_edit* edits, int32_t n,
                         size_t* patch_bytes) {
  return check_edits(edits, n, patch_bytes, &ctx->err);
}

tc_status plan_views(tc_context* ctx, const tc_view* views, int32_t n, ViewPlan& p,
                     bool allow_split) {
  PlanOpts o;
  o.packet_width = ctx->packet_width;
  o.render_mode = ctx->render_mode;
  o.split_budget = ctx->split_budget;
  o.split_queue = ctx->split_queue;
  o.split_waves = ctx->split_waves;
  return make_view_plan(o, views, n, p, allow_split, &ctx->err);
}

tci_render_opts render_opts(const tc_context* c) {
  tci_render_opts o;
  o.start_level = c->start_level;
  o.max_level = c->max_level;
  o.xcd_remap = c->xcd_remap;
  o.refill_min = c->refill_min;
  o.refill_iters = c->refill_iters;
  o.tile_order = c->tile_order;
  o.rows = nullptr;
  o.boost = c->boost;
  o.split_budget = 0;
  o.beam_passes = c->beam_passes;
  o.qcap = 0;
  o.queue = nullptr;
  o.qcount = nullptr;
  o.qzero = nullptr;
  o.split_waves = 1;
  o.count = c->count_reads ? c->d_count : nullptr;
  o.march_far = (float)c->march_far;
  o.march_steps = c->march_steps;
  o.march_bisect = c->march_bisect;
  return o;
}

hipError_t enqueue_edits(const tci_map& d, uint32_t* map, const char* dev,
                         const EditPlan& p, hipStream_t s, const tci_voxels* vx,
                         uint32_t* vox, uint64_t* zero, int32_t nzero) {
  hipError_t e = tci_launch_edits((const tci_edit*)(dev + p.off_edits), p.n,
                                  (const int32_t*)(dev + p.off_olap), p.olap_all,
                                  (const uint8_t*)(dev + p.off_patch), map, d.lv[0],
                                  d.W, d.H, p.max_w, p.max_h, s);
  const int32_t* rects = (const int32_t*)(dev + p.off_rects);
  // upward in groups of kUpdateGroup levels, one launch each: the dirty
  // nodes of levels s + 1 .. e and the window entries of levels s .. e - 1
  // (the top group: s .. e) whose 2 x 2 node block meets an edited node,
  // all computed from level s (each launch is a node of its own in a
  // captured frame, and a few microseconds however little it does)
  if (p.top == 0 && e == hipSuccess)
    e = tci_launch_update_window(d, map, 0, rects, p.nrect[0], p.rmw[0] + 1, p.rmh[0] + 1, s,
                                 zero, nzero);
  for (int32_t s0 = 0; s0 < p.top && e == hipSuccess; s0 += kUpdateGroup) {
    const int32_t e0 = std::min(s0 + kUpdateGroup, p.top);
    const bool last = e0 == p.top;
    // lanes of the largest job: a node of level L takes 2^(L - s0) lanes,
    // a window entry 2^(L - s0 + 1)
    int64_t lanes = 1;
    for (int32_t L = s0; L <= e0; ++L) {
      if (L > s0) lanes = std::max<int64_t>(lanes, ((int64_t)p.rmw[L] * p.rmh[L]) << (L - s0));
      if (L < e0 || last)
        lanes = std::max<int64_t>(lanes, ((int64_t)(p.rmw[L] + 1) * (p.rmh[L] + 1)) << (L - s0 + 1));
    }
    e = tci_launch_update_group(d, map, s0, e0, last, rects, p.n, p.nrect[0], lanes, s,
                                last ? zero : nullptr, last ? nzero : 0);
  }
  // and the voxel tiles over the edited cells, level by level upward
  if (vx && vox) {
    tci_map dm = d;
    dm.base = map;
    for (int32_t k = 0; k < vx->levels && e == hipSuccess; ++k)
      e = tci_launch_voxel_level(dm, *vx, vox, k, rects, p.nrect[0], s);
  }
  return e;
}

tc_status build_voxels(tc_context* ctx, hipStream_t s) {
  if (ctx->vox) {
    TC_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    (void)hipFree(ctx->vox);
    ctx->vox = nullptr;
    ctx->vox_words = 0;
    ctx->vdesc = tci_voxels{};
    ctx->map_generation++;   // frames captured with the old pyramid are stale
  }
  if (!ctx->vox_shape || !ctx->map) return TC_OK;
  int32_t vl = 0, vzl = 0;
  while ((1 << vl) < (ctx->vox_shape & 0xFF)) ++vl;
  while ((1 << vzl) < (ctx->vox_shape >> 8)) ++vzl;
  size_t words = 0;
  tci_voxels vx = layout_voxels(ctx->W, ctx->H, vl, vzl, &words);
  uint32_t* vox = nullptr;
  TC_HIP(dev_alloc(ctx, (void**)&vox, words * 4), "hipMalloc(voxels)");
  vx.base = vox;
  hipError_t e = hipSuccess;
  for (int32_t k = 0; k < vx.levels && e == hipSuccess; ++k)
    e = tci_launch_voxel_level(ctx->desc, vx, vox, k, nullptr, 0, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(vox);
    return hip_fail(ctx, e, "build of the voxel occupancy pyramid");
  }
  ctx->vox = vox;
  ctx->vox_words = words;
  ctx->vdesc = vx;
  ctx->map_generation++;
  return TC_OK;
}

int32_t render_counter_words(const tc_context* ctx, const ViewPlan& p) {
  if (ctx->render_mode == 3) return 0;
  if (ctx->render_mode == 2) return 1;
  return p.qcap > 0 ? 2 : 0;
}

hipError_t enqueue_render(tc_context* ctx, const tci_map& d, const char* dev,
                          const ViewPlan& p, void* out, hipStream_t s,
                          hipEvent_t* kev, bool* split_ran, bool counters_zeroed,
                          uint4* queue, const tci_inline* inl, uint32_t* qctr,
                          uint32_t* qzero) {
  tci_render_opts o = render_opts(ctx);
  if (inl) {
    // tables in the kernels' arguments (hierarchical mode without read
    // counting only); the queue counters are the slot's two, used in turn
    o.rows = nullptr;
    o.qzero = qzero;
    // (kev: the kernels carry their own start and end events, kev[0..1]
    // the traversal and kev[2..3] the split pass)
    if (split_ran) *split_ran = false;
    if (p.qcap > 0) {
      o.split_budget = ctx->split_budget;
      o.qcap = p.qcap;
      o.queue = queue;
      o.qcount = qctr;
      o.split_waves = p.qwaves;
    }
    hipError_t e = tci_launch_render_inline(d, p.n, p.npkt, out, o, *inl, s,
                                            kev ? kev[0] : nullptr, kev ? kev[1] : nullptr);
    if (p.qcap > 0) {
      const int32_t nb = (int32_t)std::max<int64_t>(
          1, std::min<int64_t>(ctx->num_cu * 16, ((int64_t)p.qcap * p.qwaves + 3) / 4));
      if (e == hipSuccess)
        e = tci_launch_split(d, nullptr, o, out, nb, s, inl, kev ? kev[2] : nullptr,
                             kev ? kev[3] : nullptr);
      if (split_ran) *split_ran = true;
    }
    return e;
  }
  o.rows = (const int32_t*)(dev + p.off_rows);
  const tci_view* dv = (const tci_view*)(dev + p.off_views);
  const int64_t* pre = (const int64_t*)(dev + p.off_prefix);
  auto mark = [&](int i) { return kev ? hipEventRecord(kev[i], s) : hipSuccess; };
  if (split_ran) *split_ran = false;
  if (ctx->render_mode == 3) {
    hipError_t e = mark(0);
    if (e == hipSuccess) e = tci_launch_march(d, dv, p.n, pre, p.npkt, out, o, s);
    if (e == hipSuccess) e = mark(1);
    return e;
  }
  if (ctx->render_mode == 2) {
    uint64_t* counter = (uint64_t*)(dev + p.off_counter);
    hipError_t e = counters_zeroed ? hipSuccess : tci_launch_zero_u64(counter, 1, s);
    int64_t blocks = (int64_t)ctx->num_cu * ctx->persist_waves / 4;
    blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, (p.npkt + 3) / 4));
    if (e == hipSuccess) e = mark(0);
    if (e == hipSuccess)
      e = tci_launch_render_persistent(d, dv, p.n, pre, p.npkt, out, counter,
                                       (int32_t)blocks, o, s);
    if (e == hipSuccess) e = mark(1);
    return e;
  }
  if (p.qcap > 0) {
    uint64_t* counters = (uint64_t*)(dev + p.off_counter);
    o.split_budget = ctx->split_budget;
    o.qcap = p.qcap;
    o.queue = queue ? queue : (uint4*)(dev + p.off_queue);
    o.qcount = (uint32_t*)(counters + 1);
    o.split_waves = p.qwaves;
    hipError_t e = counters_zeroed ? hipSuccess : tci_launch_zero_u64(counters, 2, s);
    if (e == hipSuccess) e = mark(0);
    if (e == hipSuccess)
      e = tci_launch_render(d, dv, p.n, pre, p.npkt, out, 0, o, s);
    if (e == hipSuccess) e = mark(1);
    const int32_t nb = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>(ctx->num_cu * 16, ((int64_t)p.qcap * p.qwaves + 3) / 4));
    // (4 / qwaves queued rays per block of 4 waves)
    if (e == hipSuccess) e = tci_launch_split(d, dv, o, out, nb, s);
    if (e == hipSuccess) e = mark(2);
    if (split_ran) *split_ran = true;
    return e;
  }
  hipError_t e = mark(0);
  if (e == hipSuccess && ctx->render_mode == 5)
    e = tci_launch_render(d, dv, p.n, pre, p.npkt, out, 3, o, s, &ctx->vdesc);
  else if (e == hipSuccess)
    e = tci_launch_render(d, dv, p.n, pre, p.npkt, out,
                          ctx->render_mode == 1 ? 1 : (ctx->render_mode == 4 ? 2 : 0), o, s);
  if (e == hipSuccess) e = mark(1);
  return e;
}

}  // namespace tci

extern "C" {

tc_status tc_create(int hip_device, tc_context** out) {
  if (!out) {
    g_create_error = "tc_create: out is NULL";
    return TC_INVALID_ARG;
  }
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) {
    g_create_error = std::string("tc_create: no HIP device: ") + hipGetErrorString(e);
    return TC_DEVICE_ERROR;
  }
  if (hip_device < 0 || hip_device >= n) {
    g_create_error = "tc_create: device index out of range";
    return TC_INVALID_ARG;
  }
  tc_context* ctx = new (std::nothrow) tc_context();
  if (!ctx) {
    g_create_error = "tc_create: out of host memory";
    return TC_OUT_OF_MEMORY;
  }
  ctx->device = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess ||
      hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount,
                            hip_device) != hipSuccess) {
    g_create_error = "tc_create: cannot query the device";
    delete ctx;
    return TC_DEVICE_ERROR;
  }
  // the staging ring and its split queues: after this, renders allocate
  // nothing unless their tables outgrow a slot; and the device address of
  // tc_render_views_noalloc's scratch array
  if (tci::ring_alloc(ctx, (uint32_t)ctx->split_queue) != TC_OK ||
      tci::noalloc_setup(ctx) != TC_OK) {
    g_create_error = "tc_create: " + ctx->err;
    tc_destroy(ctx);
    return TC_OUT_OF_MEMORY;
  }
  g_create_error.clear();
  *out = ctx;
  return TC_OK;
}

void tc_destroy(tc_context* ctx) {
  if (!ctx) return;
  if (ctx->server) (void)tc_server_stop((tc_server*)ctx->server);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (tci::Slot& s : ctx->ring) {
    if (s.ev) (void)hipEventDestroy(s.ev);
    if (s.host) (void)hipHostFree(s.host);
    if (s.dev) (void)hipFree(s.dev);
    if (s.queue) (void)hipFree(s.queue);
    if (s.ctr) (void)hipFree(s.ctr);
  }
  if (ctx->map) (void)hipFree(ctx->map);
  if (ctx->vox) (void)hipFree(ctx->vox);
  if (ctx->d_count) (void)hipFree(ctx->d_count);
  for (hipEvent_t& e : ctx->kev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

const char* tc_last_error(const tc_context* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

tc_status tc_load_columns(tc_context* ctx, int32_t W, int32_t H,
                          const uint8_t* floor_top, const uint8_t* slab_bottom,
                          const uint8_t* slab_top, size_t row_stride,
                          void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (ctx->server) return fail(ctx, TC_INVALID_ARG, "tc_load_columns: a server owns the map");
    if (W < 1 || H < 1 || W > TC_MAX_DIM || H > TC_MAX_DIM ||
        (int64_t)W * H > TC_MAX_CELLS)
      return fail(ctx, TC_INVALID_ARG, "tc_load_columns: bad map size %dx%d", W, H);
    if (!floor_top || !slab_bottom || !slab_top)
      return fail(ctx, TC_INVALID_ARG, "tc_load_columns: null array");
    if (row_stride < (size_t)W)
      return fail(ctx, TC_INVALID_ARG, "tc_load_columns: row_stride < W");
    int32_t bx = 0, by = 0;
    if (!tci::columns_valid(floor_top, slab_bottom, slab_top, W, H, row_stride, &bx, &by))
      return fail(ctx, TC_INVALID_ARG,
                  "tc_load_columns: column (%d,%d) violates B==0 => T==0, "
                  "B>0 => B>F and T>=B", bx, by);
    tc_status st = set_device(ctx);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;

    size_t words = 0;
    tci_map d = tci::layout_map(W, H, &words);
    uint32_t* map = nullptr;
    uint8_t* planes = nullptr;
    TC_HIP(tci::dev_alloc(ctx, (void**)&map, words * 4), "hipMalloc(map)");
    hipError_t e = tci::dev_alloc(ctx, (void**)&planes, (size_t)3 * W * H);
    if (e != hipSuccess) {
      (void)hipFree(map);
      return hip_fail(ctx, e, "hipMalloc(load staging)");
    }
    d.base = map;
    const uint8_t* src[3] = {floor_top, slab_bottom, slab_top};
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
      e = hipMemcpy2DAsync(planes + (size_t)k * W * H, W, src[k], row_stride, W,
                           H, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = tci_launch_repack(planes, W, H, map, d.lv[0], s);
    for (int32_t L = 1; L <= d.top && e == hipSuccess; ++L)
      e = tci_launch_build_level(d, map, L, s);
    for (int32_t L = 0; L <= d.top && e == hipSuccess; ++L)
      e = tci_launch_build_window(d, map, L, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(planes);
    if (e != hipSuccess) {
      (void)hipFree(map);
      return hip_fail(ctx, e, "tc_load_columns");
    }
    if (ctx->map) {
      (void)hipDeviceSynchronize();
      (void)hipFree(ctx->map);
    }
    ctx->map = map;
    ctx->map_generation++;
    ctx->map_words = words;
    ctx->desc = d;
    ctx->W = W;
    ctx->H = H;
    // the voxel occupancy pyramid of the new map, if one is asked for
    if (ctx->vox_shape || ctx->vox) return tci::build_voxels(ctx, s);
    return TC_OK;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_load_columns: host allocation failed");
  }
}

tc_status tc_apply_edit(tc_context* ctx, const tc_edit* edits, int32_t n,
                        void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_apply_edit: no map loaded");
    if (ctx->server) return fail(ctx, TC_INVALID_ARG, "tc_apply_edit: a server owns the map");
    size_t patch_bytes = 0;
    tc_status st = tci::validate_edits(ctx, edits, n, &patch_bytes);
    if (st) return st;
    if (n == 0) return TC_OK;
    st = set_device(ctx);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    tci::EditPlan plan;
    tci::plan_edits(ctx->desc, edits, n, patch_bytes, nullptr, plan);
    tci::Slot* slot = nullptr;
    st = tci::acquire(ctx, plan.total, &slot);
    if (st) return st;
    tci::plan_edits(ctx->desc, edits, n, patch_bytes, (char*)slot->host, plan);
    hipError_t e = hipMemcpyAsync(slot->dev, slot->host, plan.total, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = tci::enqueue_edits(ctx->desc, ctx->map, (const char*)slot->dev, plan, s,
                             ctx->vox ? &ctx->vdesc : nullptr, ctx->vox);
    st = tci::release(ctx, slot, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "tc_apply_edit");
    return st;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_apply_edit: host allocation failed");
  }
}

tc_status tc_render_views(tc_context* ctx, const tc_view* views, int32_t n,
                          tc_hit* out_device, void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_render_views: no map loaded");
    if (ctx->server) return fail(ctx, TC_INVALID_ARG, "tc_render_views: a server owns the map");
    if (!out_device) return fail(ctx, TC_INVALID_ARG, "tc_render_views: out is NULL");
    if (ctx->render_mode == 5 && !ctx->vox)
      return fail(ctx, TC_INVALID_ARG, "tc_render_views: render mode 5 needs TC_OPT_VOXEL_SHAPE");
    tci::ViewPlan plan;
    tc_status st = tci::plan_views(ctx, views, n, plan);
    if (st) return st;
    st = set_device(ctx);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t* kev = nullptr;
    if (ctx->kernel_timing) {
      for (hipEvent_t& ev : ctx->kev)
        if (!ev) TC_HIP(hipEventCreate(&ev), "hipEventCreate");
      kev = ctx->kev;
    }
    tci::Slot* slot = nullptr;
    st = tci::acquire(ctx, plan.off_queue, &slot);
    if (st) return st;
    tci::write_views(plan, (char*)slot->host);
    hipError_t e = hipSuccess;
    bool split_ran = false;
    const bool inl_used = ctx->inline_tables && ctx->render_mode == 0 && !ctx->count_reads &&
                          plan.off_counter <= (size_t)kInlineBytes;
    if (inl_used) {
      // a small call: its tables travel in the kernels' arguments, so
      // nothing is uploaded before the render
      tci_inline t;
      t.off_prefix = (uint32_t)plan.off_prefix;
      t.off_rows = (uint32_t)plan.off_rows;
      std::memcpy(t.words, slot->host, plan.off_counter);
      if (slot->ctr_dirty) e = tci_launch_zero_u64((uint64_t*)slot->ctr, 1, s);
      const int turn = slot->ctr_turn;
      if (e == hipSuccess)
        e = tci::enqueue_render(ctx, ctx->desc, nullptr, plan, out_device, s, kev, &split_ran,
                                true, slot->queue, &t, slot->ctr + turn, slot->ctr + 1 - turn);
      // (a call with no packets launches no render, so nothing clears the
      // other counter: clear both before the slot's next such call)
      slot->ctr_dirty = e != hipSuccess || plan.npkt < 1;
      slot->ctr_turn = 1 - turn;
    } else {
      // tables and zeroed queue counters in one upload; the split queue is
      // the slot's device-only buffer (plan.qcap <= TC_OPT_SPLIT_QUEUE <= its
      // size)
      e = hipMemcpyAsync(slot->dev, slot->host, plan.off_queue, hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = tci::enqueue_render(ctx, ctx->desc, (const char*)slot->dev, plan, out_device, s,
                                kev, &split_ran, true, slot->queue);
    }
    if (kev) {
      ctx->kev_valid = e == hipSuccess && plan.npkt > 0;
      ctx->kev_split = split_ran;
      ctx->kev_attached = inl_used;
    }
    tc_status rs = tci::release(ctx, slot, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "tc_render_views");
    return rs;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_render_views: host allocation failed");
  }
}

tc_status tc_shade_views(tc_context* ctx, const tc_view* views, int32_t n,
                         const tc_hit* hits_device, const tc_shade_params* params,
                         uint32_t* rgba_device, void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_shade_views: no map loaded");
    if (ctx->server) return fail(ctx, TC_INVALID_ARG, "tc_shade_views: a server owns the map");
    if (!hits_device || !rgba_device || !params || !params->palette)
      return fail(ctx, TC_INVALID_ARG, "tc_shade_views: null pointer");
    const tc_shade_params& p = *params;
    bool any = false;
    for (int c = 0; c < 3; ++c) {
      if (p.light[c] < -TC_MAX_DIR || p.light[c] > TC_MAX_DIR)
        return fail(ctx, TC_INVALID_ARG, "tc_shade_views: light component out of range");
      any |= p.light[c] != 0;
    }
    if (!any) return fail(ctx, TC_INVALID_ARG, "tc_shade_views: zero light direction");
    if (!(p.fog_far > 0.0f) || !std::isfinite(p.fog_far))
      return fail(ctx, TC_INVALID_ARG, "tc_shade_views: bad fog_far");
    if (!(p.ambient >= 0.0f && p.ambient <= 1.0f) ||
        !(p.cave_ambient >= 0.0f && p.cave_ambient <= 1.0f))
      return fail(ctx, TC_INVALID_ARG, "tc_shade_views: ambient outside 0..1");
    tci::ViewPlan plan;
    tc_status st = tci::plan_views(ctx, views, n, plan, false);
    if (st) return st;
    st = set_device(ctx);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t off_pal = (plan.off_queue + 255) & ~(size_t)255;
    const size_t total = off_pal + 512 * sizeof(uint32_t);
    tci::Slot* slot = nullptr;
    st = tci::acquire(ctx, total, &slot);
    if (st) return st;
    tci::write_views(plan, (char*)slot->host);
    memcpy((char*)slot->host + off_pal, p.palette, 512 * sizeof(uint32_t));
    const char* dev = (const char*)slot->dev;
    hipError_t e = hipMemcpyAsync(slot->dev, slot->host, total, hipMemcpyHostToDevice, s);
    tci_shade sh;
    for (int c = 0; c < 3; ++c) sh.light[c] = p.light[c];
    sh.ambient = p.ambient;
    sh.cave_ambient = p.cave_ambient;
    sh.fog_far = p.fog_far;
    sh.sky_rgba = p.sky_rgba;
    sh.fog_rgba = p.fog_rgba;
    sh.palette = (const uint32_t*)(dev + off_pal);
    tci_render_opts o = tci::render_opts(ctx);
    o.rows = (const int32_t*)(dev + plan.off_rows);
    hipEvent_t* kev = nullptr;
    if (ctx->kernel_timing) {
      for (hipEvent_t& ev : ctx->kev)
        if (!ev && e == hipSuccess) e = hipEventCreate(&ev);
      kev = ctx->kev;
    }
    if (e == hipSuccess && kev) e = hipEventRecord(kev[0], s);
    if (e == hipSuccess)
      e = tci_launch_shade(ctx->desc, (const tci_view*)(dev + plan.off_views), plan.n,
                           (const int64_t*)(dev + plan.off_prefix), plan.npkt, hits_device,
                           rgba_device, sh, o, s);
    if (e == hipSuccess && kev) e = hipEventRecord(kev[1], s);
    if (kev) {
      ctx->kev_valid = e == hipSuccess;
      ctx->kev_split = false;
      ctx->kev_attached = false;
    }
    tc_status rs = tci::release(ctx, slot, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "tc_shade_views");
    return rs;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_shade_views: host allocation failed");
  }
}

tc_status tc_set_option(tc_context* ctx, int32_t key, int64_t value) {
  if (!ctx) return TC_INVALID_ARG;
  ctx->err.clear();
  switch (key) {
    case TC_OPT_RENDER_MODE:
      if (value < 0 || value > 5) break;
      ctx->render_mode = (int32_t)value;
      return TC_OK;
    case TC_OPT_VOXEL_SHAPE: {
      const int64_t v = value & 0xFF, vz = value >> 8;
      const bool pow2 = (v == 1 || v == 2 || v == 4 || v == 8) &&
                        (vz == 1 || vz == 2 || vz == 4 || vz == 8);
      if (value != 0 && !pow2) break;
      if (ctx->server) return fail(ctx, TC_INVALID_ARG, "tc_set_option: a server owns the map");
      if (set_device(ctx)) return TC_DEVICE_ERROR;
      ctx->vox_shape = (int32_t)value;
      return tci::build_voxels(ctx, nullptr);
    }
    case TC_OPT_START_LEVEL:
      if (value < 0 || value >= TCI_MAX_LEVELS) break;
      ctx->start_level = (int32_t)value;
      return TC_OK;
    case TC_OPT_MAX_LEVEL:
      if (value < 0 || value >= TCI_MAX_LEVELS) break;
      ctx->max_level = (int32_t)value;
      return TC_OK;
    case TC_OPT_XCD_REMAP:
      if (value < 0 || value > 4096) break;
      ctx->xcd_remap = (int32_t)value;
      return TC_OK;
    case TC_OPT_PERSIST_WAVES:
      if (value < 4 || value > 64) break;
      ctx->persist_waves = (int32_t)value;
      return TC_OK;
    case TC_OPT_REFILL_MIN:
      if (value < 1 || value > 64) break;
      ctx->refill_min = (int32_t)value;
      return TC_OK;
    case TC_OPT_REFILL_ITERS:
      if (value < 1 || value > 4096) break;
      ctx->refill_iters = (int32_t)value;
      return TC_OK;
    case TC_OPT_SPLIT_BUDGET:
      if (value < 0 || value > (1 << 20)) break;
      ctx->split_budget = (int32_t)value;
      return TC_OK;
    case TC_OPT_SPLIT_WAVES:
      if (value != 1 && value != 2 && value != 4) break;
      ctx->split_waves = (int32_t)value;
      return TC_OK;
    case TC_OPT_BEAM_PASSES:
      if (value < 0 || value > 64) break;
      ctx->beam_passes = (int32_t)value;
      return TC_OK;
    case TC_OPT_SPLIT_QUEUE: {
      if (value < 1 || value > (1 << 24)) break;
      // every ring slot holds a queue of this many entries
      if (set_device(ctx)) return TC_DEVICE_ERROR;
      tc_status st = tci::ring_alloc(ctx, (uint32_t)value);
      if (st) return st;
      ctx->split_queue = (int32_t)value;
      return TC_OK;
    }
    case TC_OPT_INLINE_TABLES:
      if (value < 0 || value > 1) break;
      ctx->inline_tables = (int32_t)value;
      return TC_OK;
    case TC_OPT_MARCH_STEPS:
      if (value < 1 || value > 65536) break;
      ctx->march_steps = (int32_t)value;
      return TC_OK;
    case TC_OPT_MARCH_BISECT:
      if (value < 0 || value > 64) break;
      ctx->march_bisect = (int32_t)value;
      return TC_OK;
    case TC_OPT_MARCH_FAR:
      if (value < 1 || value > (1 << 20)) break;
      ctx->march_far = (int32_t)value;
      return TC_OK;
    case TC_OPT_KERNEL_TIMING:
      if (value < 0 || value > 1) break;
      ctx->kernel_timing = (int32_t)value;
      ctx->kev_valid = false;
      return TC_OK;
    case TC_OPT_PRIORITY_BOOST:
      if (value < 0 || value > (1 << 20)) break;
      ctx->boost = (int32_t)value;
      return TC_OK;
    case TC_OPT_TILE_ORDER:
      if (value < 0 || value > 2) break;
      ctx->tile_order = (int32_t)value;
      return TC_OK;
    case TC_OPT_PACKET_WIDTH:
      if (value != 4 && value != 8 && value != 16 && value != 32) break;
      ctx->packet_width = (int32_t)value;
      return TC_OK;
    case TC_OPT_COUNT_READS:
      if (value < 0 || value > 1) break;
      if (value && !ctx->d_count) {
        if (set_device(ctx)) return TC_DEVICE_ERROR;
        hipError_t e = tci::dev_alloc(ctx, (void**)&ctx->d_count, sizeof(unsigned long long));
        if (e == hipSuccess) e = hipMemset(ctx->d_count, 0, sizeof(unsigned long long));
        if (e != hipSuccess) return hip_fail(ctx, e, "tc_set_option(count)");
      }
      ctx->count_reads = (int32_t)value;
      return TC_OK;
    default:
      return fail(ctx, TC_INVALID_ARG, "tc_set_option: unknown key %d", key);
  }
  return fail(ctx, TC_INVALID_ARG, "tc_set_option: value %lld out of range for key %d",
              (long long)value, key);
}

tc_status tc_get_option(const tc_context* ctx, int32_t key, int64_t* value) {
  if (!ctx || !value) return TC_INVALID_ARG;
  switch (key) {
    case TC_OPT_RENDER_MODE: *value = ctx->render_mode; return TC_OK;
    case TC_OPT_START_LEVEL: *value = ctx->start_level; return TC_OK;
    case TC_OPT_MAX_LEVEL: *value = ctx->max_level; return TC_OK;
    case TC_OPT_XCD_REMAP: *value = ctx->xcd_remap; return TC_OK;
    case TC_OPT_PERSIST_WAVES: *value = ctx->persist_waves; return TC_OK;
    case TC_OPT_REFILL_MIN: *value = ctx->refill_min; return TC_OK;
    case TC_OPT_REFILL_ITERS: *value = ctx->refill_iters; return TC_OK;
    case TC_OPT_COUNT_READS: *value = ctx->count_reads; return TC_OK;
    case TC_OPT_TILE_ORDER: *value = ctx->tile_order; return TC_OK;
    case TC_OPT_PACKET_WIDTH: *value = ctx->packet_width; return TC_OK;
    case TC_OPT_VOXEL_SHAPE: *value = ctx->vox_shape; return TC_OK;
    case TC_OPT_PRIORITY_BOOST: *value = ctx->boost; return TC_OK;
    case TC_OPT_SPLIT_BUDGET: *value = ctx->split_budget; return TC_OK;
    case TC_OPT_SPLIT_QUEUE: *value = ctx->split_queue; return TC_OK;
    case TC_OPT_INLINE_TABLES: *value = ctx->inline_tables; return TC_OK;
    case TC_OPT_BEAM_PASSES: *value = ctx->beam_passes; return TC_OK;
    case TC_OPT_SPLIT_WAVES: *value = ctx->split_waves; return TC_OK;
    case TC_OPT_KERNEL_TIMING: *value = ctx->kernel_timing; return TC_OK;
    case TC_OPT_MARCH_STEPS: *value = ctx->march_steps; return TC_OK;
    case TC_OPT_MARCH_BISECT: *value = ctx->march_bisect; return TC_OK;
    case TC_OPT_MARCH_FAR: *value = ctx->march_far; return TC_OK;
    case TC_INFO_ALLOCATIONS: *value = (int64_t)ctx->allocs; return TC_OK;
    default: return TC_INVALID_ARG;
  }
}

static tc_status read_level_rows(tc_context* ctx, const tci_level& l, int32_t ty0, int32_t ty1,
                                 std::vector<uint32_t>& buf, hipStream_t s) {
  size_t row_words = (size_t)l.tiles_x * 64;
  size_t n = row_words * (size_t)(ty1 - ty0 + 1);
  buf.resize(n);
  TC_HIP(hipMemcpyAsync(buf.data(), ctx->map + l.off + row_words * ty0, n * 4,
                        hipMemcpyDeviceToHost, s), "hipMemcpyAsync(read)");
  TC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize(read)");
  return TC_OK;
}

tc_status tc_read_columns(tc_context* ctx, int32_t x0, int32_t y0, int32_t w,
                          int32_t h, uint8_t* floor_top, uint8_t* slab_bottom,
                          uint8_t* slab_top, void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_read_columns: no map loaded");
    if (w < 1 || h < 1 || x0 < 0 || y0 < 0 || x0 + w > ctx->W || y0 + h > ctx->H)
      return fail(ctx, TC_INVALID_ARG, "tc_read_columns: rectangle outside the map");
    if (!floor_top || !slab_bottom || !slab_top)
      return fail(ctx, TC_INVALID_ARG, "tc_read_columns: null output");
    tc_status st = set_device(ctx);
    if (st) return st;
    std::vector<uint32_t> buf;
    int32_t ty0 = y0 >> 3, ty1 = (y0 + h - 1) >> 3;
    st = read_level_rows(ctx, ctx->desc.lv[0], ty0, ty1, buf, (hipStream_t)hip_stream);
    if (st) return st;
    tci_level l = ctx->desc.lv[0];
    l.off = 0;
    for (int32_t j = 0; j < h; ++j)
      for (int32_t i = 0; i < w; ++i) {
        int32_t x = x0 + i, y = y0 + j;
        uint32_t v = buf[tci_tile_index(l, x, y - ty0 * 8)];
        size_t o = (size_t)j * w + i;
        floor_top[o] = v & 0xFF;
        slab_bottom[o] = (v >> 8) & 0xFF;
        slab_top[o] = (v >> 16) & 0xFF;
      }
    return TC_OK;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_read_columns: host allocation failed");
  }
}

tc_status tc_pyramid_info(const tc_context* ctx, int32_t* levels) {
  if (!ctx || !levels) return TC_INVALID_ARG;
  if (!ctx->map) return TC_NO_MAP;
  *levels = ctx->desc.top;
  return TC_OK;
}

tc_status tc_pyramid_dims(const tc_context* ctx, int32_t level, int32_t* w, int32_t* h) {
  if (!ctx || !w || !h) return TC_INVALID_ARG;
  if (!ctx->map) return TC_NO_MAP;
  if (level < 0 || level > ctx->desc.top) return TC_INVALID_ARG;
  *w = ctx->desc.lv[level].w;
  *h = ctx->desc.lv[level].h;
  return TC_OK;
}

tc_status tc_read_pyramid(tc_context* ctx, int32_t level, uint32_t* out, void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_read_pyramid: no map loaded");
    if (level < 1 || level > ctx->desc.top || !out)
      return fail(ctx, TC_INVALID_ARG, "tc_read_pyramid: bad level %d", level);
    tc_status st = set_device(ctx);
    if (st) return st;
    tci_level l = ctx->desc.lv[level];
    std::vector<uint32_t> buf;
    st = read_level_rows(ctx, l, 0, (l.h - 1) >> 3, buf, (hipStream_t)hip_stream);
    if (st) return st;
    l.off = 0;
    for (int32_t j = 0; j < l.h; ++j)
      for (int32_t i = 0; i < l.w; ++i) out[(size_t)j * l.w + i] = buf[tci_tile_index(l, i, j)];
    return TC_OK;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_read_pyramid: host allocation failed");
  }
}

tc_status tc_read_window(tc_context* ctx, int32_t level, uint32_t* out, void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_read_window: no map loaded");
    if (level < 0 || level > ctx->desc.top || !out)
      return fail(ctx, TC_INVALID_ARG, "tc_read_window: bad level %d", level);
    tc_status st = set_device(ctx);
    if (st) return st;
    tci_level l = ctx->desc.wl[level];
    std::vector<uint32_t> buf;
    st = read_level_rows(ctx, l, 0, (l.h - 1) >> 3, buf, (hipStream_t)hip_stream);
    if (st) return st;
    l.off = 0;
    for (int32_t j = 0; j < l.h; ++j)
      for (int32_t i = 0; i < l.w; ++i) out[(size_t)j * l.w + i] = buf[tci_tile_index(l, i, j)];
    return TC_OK;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_read_window: host allocation failed");
  }
}

tc_status tc_voxel_dims(const tc_context* ctx, int32_t level, int32_t* nx, int32_t* ny,
                        int32_t* nz, int32_t* levels) {
  if (!ctx || !nx || !ny || !nz) return TC_INVALID_ARG;
  if (!ctx->vox) return TC_NO_MAP;
  if (level < 0 || level >= ctx->vdesc.levels) return TC_INVALID_ARG;
  const tci_vlevel& l = ctx->vdesc.lv[level];
  *nx = l.nx;
  *ny = l.ny;
  *nz = l.nz;
  if (levels) *levels = ctx->vdesc.levels;
  return TC_OK;
}

tc_status tc_read_voxels(tc_context* ctx, int32_t level, uint8_t* out, void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (!ctx->vox) return fail(ctx, TC_NO_MAP, "tc_read_voxels: no voxel occupancy pyramid");
    if (level < 0 || level >= ctx->vdesc.levels || !out)
      return fail(ctx, TC_INVALID_ARG, "tc_read_voxels: bad level %d", level);
    tc_status st = set_device(ctx);
    if (st) return st;
    const tci_vlevel& l = ctx->vdesc.lv[level];
    const size_t words = (size_t)l.tiles_x * l.tiles_y * l.tiles_z * 16;
    std::vector<uint32_t> buf(words);
    hipStream_t s = (hipStream_t)hip_stream;
    TC_HIP(hipMemcpyAsync(buf.data(), ctx->vox + l.off, words * 4, hipMemcpyDeviceToHost, s),
           "hipMemcpyAsync(read)");
    TC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize(read)");
    for (int32_t z = 0; z < l.nz; ++z)
      for (int32_t y = 0; y < l.ny; ++y)
        for (int32_t x = 0; x < l.nx; ++x) {
          uint32_t m = 0;
          for (int b = 0; b < 3; ++b)
            m |= (((uint32_t)(x >> b) & 1u) << (3 * b)) | (((uint32_t)(y >> b) & 1u) << (3 * b + 1)) |
                 (((uint32_t)(z >> b) & 1u) << (3 * b + 2));
          const size_t t = ((size_t)((z >> 3) * l.tiles_y + (y >> 3)) * l.tiles_x + (x >> 3)) * 16;
          out[((size_t)z * l.ny + y) * l.nx + x] = (uint8_t)((buf[t + (m >> 5)] >> (m & 31)) & 1u);
        }
    return TC_OK;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_read_voxels: host allocation failed");
  }
}

tc_status tc_read_occupancy(tc_context* ctx, int32_t level, uint64_t* out, void* hip_stream) {
  if (!ctx) return TC_INVALID_ARG;
  try {
    ctx->err.clear();
    if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_read_occupancy: no map loaded");
    if (level < 1 || level > ctx->desc.top || !out)
      return fail(ctx, TC_INVALID_ARG, "tc_read_occupancy: bad level %d", level);
    tc_status st = set_device(ctx);
    if (st) return st;
    tci_level k = ctx->desc.mk[level];
    const size_t words = (size_t)k.tiles_x * ((k.h + 7) >> 3) * 128;
    std::vector<uint32_t> buf(words);
    hipStream_t s = (hipStream_t)hip_stream;
    TC_HIP(hipMemcpyAsync(buf.data(), ctx->map + k.off, words * 4, hipMemcpyDeviceToHost, s),
           "hipMemcpyAsync(read)");
    TC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize(read)");
    k.off = 0;
    for (int32_t j = 0; j < k.h; ++j)
      for (int32_t i = 0; i < k.w; ++i) {
        const uint32_t w = tci_mask_index(k, i, j);
        out[(size_t)j * k.w + i] = (uint64_t)buf[w] | ((uint64_t)buf[w + 1] << 32);
      }
    return TC_OK;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_read_occupancy: host allocation failed");
  }
}

tc_status tc_read_counters(tc_context* ctx, uint64_t* reads, void* hip_stream) {
  if (!ctx || !reads) return TC_INVALID_ARG;
  ctx->err.clear();
  *reads = 0;
  if (!ctx->d_count) return TC_OK;
  tc_status st = set_device(ctx);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  unsigned long long v = 0;
  TC_HIP(hipMemcpyAsync(&v, ctx->d_count, sizeof(v), hipMemcpyDeviceToHost, s),
         "hipMemcpyAsync(counter)");
  TC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize(counter)");
  TC_HIP(hipMemsetAsync(ctx->d_count, 0, sizeof(v), s), "hipMemsetAsync(counter)");
  TC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize(counter)");
  *reads = v;
  return TC_OK;
}

tc_status tc_read_kernel_times(tc_context* ctx, float* ms) {
  if (!ctx) return TC_INVALID_ARG;
  ctx->err.clear();
  if (!ms) return fail(ctx, TC_INVALID_ARG, "tc_read_kernel_times: ms is NULL");
  if (!ctx->kev_valid)
    return fail(ctx, TC_INVALID_ARG, "tc_read_kernel_times: no timed render since timing was enabled");
  tc_status st = set_device(ctx);
  if (st) return st;
  // markers: kev[0] | traversal | kev[1] | split pass | kev[2]; attached:
  // each kernel's own start and end, kev[0..1] and kev[2..3]
  const int a = ctx->kev_attached ? 1 : 0;
  const int last = ctx->kev_split ? 2 + a : 1;
  TC_HIP(hipEventSynchronize(ctx->kev[last]), "hipEventSynchronize");
  TC_HIP(hipEventElapsedTime(&ms[0], ctx->kev[0], ctx->kev[1]), "hipEventElapsedTime");
  ms[1] = 0.0f;
  if (ctx->kev_split)
    TC_HIP(hipEventElapsedTime(&ms[1], ctx->kev[1 + a], ctx->kev[2 + a]), "hipEventElapsedTime");
  return TC_OK;
}

tc_status tc_map_bytes(const tc_context* ctx, uint64_t* bytes) {
  if (!ctx || !bytes) return TC_INVALID_ARG;
  if (!ctx->map) return TC_NO_MAP;
  *bytes = (uint64_t)ctx->map_words * 4;
  return TC_OK;
}

}  // extern "C"
