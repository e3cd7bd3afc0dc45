// Host runtime of the library: the C ABI declared in include/tc.h.
//
// Owns the device copy of the map (packed columns plus the min/max pyramid,
// one allocation), validates every call before enqueueing anything, stages
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

bool columns_valid(const uint8_t* F, const uint8_t* B, const uint8_t* T,
                   int32_t w, int32_t h, size_t stride, int32_t* bad_x,
                   int32_t* bad_y) {
  for (int32_t y = 0; y < h; ++y) {
    const uint8_t* f = F + (size_t)y * stride;
    const uint8_t* b = B + (size_t)y * stride;
    const uint8_t* t = T + (size_t)y * stride;
    for (int32_t x = 0; x < w; ++x) {
      bool ok = b[x] == 0 ? t[x] == 0 : (b[x] > f[x] && t[x] >= b[x]);
      if (!ok) {
        *bad_x = x;
        *bad_y = y;
        return false;
      }
    }
  }
  return true;
}

int32_t top_level(int32_t W, int32_t H) {
  int32_t m = std::max(W, H), L = 0;
  while ((1 << L) < m) ++L;
  return L;
}

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

tc_status acquire(tc_context* ctx, size_t bytes, Slot** out) {
  Slot& s = ctx->ring[ctx->ring_next];
  ctx->ring_next = (ctx->ring_next + 1) % kRing;
  if (s.pending) {
    TC_HIP(hipEventSynchronize(s.ev), "hipEventSynchronize(staging)");
    s.pending = false;
  }
  if (s.cap < bytes) {
    size_t cap = std::max<size_t>(bytes, 64 << 10);
    cap = (cap + 4095) & ~(size_t)4095;
    if (s.host) { (void)hipHostFree(s.host); s.host = nullptr; }
    if (s.dev) { (void)hipFree(s.dev); s.dev = nullptr; }
    s.cap = 0;
    TC_HIP(hipHostMalloc(&s.host, cap, hipHostMallocDefault), "hipHostMalloc(staging)");
    TC_HIP(hipMalloc(&s.dev, cap), "hipMalloc(staging)");
    s.cap = cap;
  }
  if (!s.ev) TC_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming), "hipEventCreate");
  *out = &s;
  return TC_OK;
}

tc_status release(tc_context* ctx, Slot* s, hipStream_t st) {
  TC_HIP(hipEventRecord(s->ev, st), "hipEventRecord(staging)");
  s->pending = true;
  return TC_OK;
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
  o.split_waves = 1;
  o.count = c->count_reads ? c->d_count : nullptr;
  o.march_far = (float)c->march_far;
  o.march_steps = c->march_steps;
  o.march_bisect = c->march_bisect;
  return o;
}

tc_status validate_edits(tc_context* ctx, const tc_edit* edits, int32_t n,
                         size_t* patch_bytes) {
  if (n < 0 || n > 65536) return fail(ctx, TC_INVALID_ARG, "edits: bad n %d", n);
  if (n > 0 && !edits) return fail(ctx, TC_INVALID_ARG, "edits: list is NULL");
  size_t pb = 0;
  for (int32_t i = 0; i < n; ++i) {
    const tc_edit& e = edits[i];
    if (e.kind == TC_EDIT_SET) {
      if (e.w < 1 || e.h < 1 || e.w > TC_MAX_DIM || e.h > TC_MAX_DIM)
        return fail(ctx, TC_INVALID_ARG, "edits: edit %d bad size", i);
      if (!e.floor_top || !e.slab_bottom || !e.slab_top)
        return fail(ctx, TC_INVALID_ARG, "edits: edit %d null patch", i);
      int32_t bx, by;
      if (!columns_valid(e.floor_top, e.slab_bottom, e.slab_top, e.w, e.h, e.w, &bx, &by))
        return fail(ctx, TC_INVALID_ARG,
                    "edits: edit %d patch cell (%d,%d) violates the column "
                    "invariants", i, bx, by);
      pb += (size_t)3 * e.w * e.h;
    } else if (e.kind == TC_EDIT_CRATER) {
      if (e.w < 1 || e.w > 4096 || e.h != e.w)
        return fail(ctx, TC_INVALID_ARG, "edits: edit %d bad crater size", i);
      if (e.depth < 0 || e.depth > 255)
        return fail(ctx, TC_INVALID_ARG, "edits: edit %d bad crater depth", i);
    } else {
      return fail(ctx, TC_INVALID_ARG, "edits: edit %d bad kind %d", i, e.kind);
    }
    if ((int64_t)e.x0 + e.w > INT32_MAX || (int64_t)e.y0 + e.h > INT32_MAX ||
        e.x0 < -(1 << 28) || e.y0 < -(1 << 28))
      return fail(ctx, TC_INVALID_ARG, "edits: edit %d rectangle overflows", i);
  }
  *patch_bytes = pb;
  return TC_OK;
}

void plan_edits(const tci_map& d, const tc_edit* edits, int32_t n,
                size_t patch_bytes, char* host, EditPlan& p) {
  const int32_t top = d.top;
  p.n = n;
  p.top = top;
  p.off_edits = 0;
  p.off_rects = (sizeof(tci_edit) * (size_t)n + 15) & ~(size_t)15;
  p.off_patch = p.off_rects + sizeof(int32_t) * 4 * (size_t)n * (size_t)std::max(top, 1);
  p.total = p.off_patch + patch_bytes;
  p.nrect.assign(top + 1, 0);
  p.rmw.assign(top + 1, 1);
  p.rmh.assign(top + 1, 1);
  p.max_w = p.max_h = 1;
  tci_edit* he = host ? (tci_edit*)(host + p.off_edits) : nullptr;
  int32_t* hr = host ? (int32_t*)(host + p.off_rects) : nullptr;
  uint8_t* hp = host ? (uint8_t*)(host + p.off_patch) : nullptr;
  size_t po = 0;
  for (int32_t i = 0; i < n; ++i) {
    const tc_edit& e = edits[i];
    if (he) {
      tci_edit& o = he[i];
      o.kind = e.kind;
      o.x0 = e.x0;
      o.y0 = e.y0;
      o.w = e.w;
      o.h = e.h;
      o.depth = e.depth;
      o.data_off = (int64_t)po;
    }
    if (e.kind == TC_EDIT_SET) {
      size_t m = (size_t)e.w * e.h;
      if (hp) {
        memcpy(hp + po, e.floor_top, m);
        memcpy(hp + po + m, e.slab_bottom, m);
        memcpy(hp + po + 2 * m, e.slab_top, m);
      }
      po += 3 * m;
    }
    int32_t x0 = std::max(e.x0, 0), y0 = std::max(e.y0, 0);
    int32_t x1 = std::min(e.x0 + e.w, d.W), y1 = std::min(e.y0 + e.h, d.H);
    if (x0 >= x1 || y0 >= y1) continue;
    p.max_w = std::max(p.max_w, x1 - x0);
    p.max_h = std::max(p.max_h, y1 - y0);
    for (int32_t L = 1; L <= top; ++L) {
      int32_t r[4] = {x0 >> L, y0 >> L, (x1 - 1) >> L, (y1 - 1) >> L};
      if (hr) memcpy(hr + 4 * ((size_t)(L - 1) * n + p.nrect[L]), r, sizeof(r));
      p.rmw[L] = std::max(p.rmw[L], r[2] - r[0] + 1);
      p.rmh[L] = std::max(p.rmh[L], r[3] - r[1] + 1);
      p.nrect[L]++;
    }
  }
}

hipError_t enqueue_edits(const tci_map& d, uint32_t* map, const char* dev,
                         const EditPlan& p, hipStream_t s) {
  hipError_t e = tci_launch_edits((const tci_edit*)(dev + p.off_edits), p.n,
                                  (const uint8_t*)(dev + p.off_patch), map, d.lv[0],
                                  d.W, d.H, p.max_w, p.max_h, s);
  for (int32_t L = 1; L <= p.top && e == hipSuccess; ++L)
    e = tci_launch_update_level(d, map, L,
                                (const int32_t*)(dev + p.off_rects) + 4 * (size_t)(L - 1) * p.n,
                                p.nrect[L], p.rmw[L], p.rmh[L], s);
  return e;
}

tc_status plan_views(tc_context* ctx, const tc_view* views, int32_t n, ViewPlan& p,
                     bool allow_split) {
  if (n < 1 || !views) return fail(ctx, TC_INVALID_ARG, "render: no views");
  p.n = n;
  p.views.resize(n);
  p.prefix.resize((size_t)n + 1);
  int64_t out = 0, pk = 0;
  for (int32_t i = 0; i < n; ++i) {
    const tc_view& v = views[i];
    if (v.width < 1 || v.height < 1 || v.width > 16384 || v.height > 16384)
      return fail(ctx, TC_INVALID_ARG, "render: view %d bad size %dx%d", i, v.width, v.height);
    if (v.flags != 0) return fail(ctx, TC_INVALID_ARG, "render: view %d flags != 0", i);
    for (int cx = 0; cx < 2; ++cx)
      for (int cy = 0; cy < 2; ++cy) {
        int64_t a = cx ? 2 * (int64_t)v.width - 1 : 1;
        int64_t b = cy ? 2 * (int64_t)v.height - 1 : 1;
        for (int c = 0; c < 3; ++c) {
          int64_t O = (int64_t)v.o0[c] + a * v.o_px[c] + b * v.o_py[c];
          int64_t D = (int64_t)v.d0[c] + a * v.d_px[c] + b * v.d_py[c];
          if (O < INT32_MIN || O > INT32_MAX)
            return fail(ctx, TC_INVALID_ARG, "render: view %d origin overflows int32", i);
          if (D < -TC_MAX_DIR || D > TC_MAX_DIR)
            return fail(ctx, TC_INVALID_ARG, "render: view %d |direction| > 2^23-1", i);
        }
      }
    tci_view& o = p.views[i];
    o.w = v.width;
    o.h = v.height;
    for (int c = 0; c < 3; ++c) {
      o.o0[c] = v.o0[c]; o.opx[c] = v.o_px[c]; o.opy[c] = v.o_py[c];
      o.d0[c] = v.d0[c]; o.dpx[c] = v.d_px[c]; o.dpy[c] = v.d_py[c];
    }
    o.tiles_x = (v.width + 7) >> 3;
    o.small_steps = 1;
    for (int c = 0; c < 3; ++c)
      for (int32_t st : {v.o_px[c], v.o_py[c], v.d_px[c], v.d_py[c]})
        if (st <= -(1 << 22) || st >= (1 << 22)) o.small_steps = 0;
    o.out_base = out;
    o.pkt_base = pk;
    o.rows_off = (int64_t)p.rows.size();
    // tile rows ordered by how level the ray through the row's centre is:
    // near-horizontal rays take the longest walks, so their packets start
    // first and do not trail the launch
    {
      const int32_t ty_n = (v.height + 7) >> 3;
      std::vector<std::pair<double, int32_t>> key((size_t)ty_n);
      const int64_t a = v.width;  // 2 * (width / 2) + 1, rounded
      for (int32_t ty = 0; ty < ty_n; ++ty) {
        const int64_t b = 2 * (int64_t)std::min(ty * 8 + 4, v.height - 1) + 1;
        const double dx = (double)v.d0[0] + (double)a * v.d_px[0] + (double)b * v.d_py[0];
        const double dy = (double)v.d0[1] + (double)a * v.d_px[1] + (double)b * v.d_py[1];
        const double dz = (double)v.d0[2] + (double)a * v.d_px[2] + (double)b * v.d_py[2];
        const double hz = std::sqrt(dx * dx + dy * dy);
        key[ty] = {hz > 0 ? std::fabs(dz) / hz : 1e30, ty};
      }
      std::stable_sort(key.begin(), key.end(),
                       [](const std::pair<double, int32_t>& x,
                          const std::pair<double, int32_t>& y) { return x.first < y.first; });
      for (auto& k : key) p.rows.push_back(k.second);
    }
    p.prefix[i] = pk;
    out += (int64_t)v.width * v.height;
    pk += (int64_t)o.tiles_x * ((v.height + 7) >> 3);
  }
  p.prefix[n] = pk;
  if (out > ((int64_t)1 << 31))
    return fail(ctx, TC_INVALID_ARG, "render: more than 2^31 rays");
  p.rays = out;
  p.npkt = pk;
  p.off_views = 0;
  p.off_prefix = (sizeof(tci_view) * (size_t)n + 15) & ~(size_t)15;
  p.off_rows = (p.off_prefix + sizeof(int64_t) * ((size_t)n + 1) + 15) & ~(size_t)15;
  p.off_counter = (p.off_rows + sizeof(int32_t) * p.rows.size() + 15) & ~(size_t)15;
  // the split queue follows the counters (device only, never uploaded)
  p.qcap = (allow_split && ctx->render_mode == 0 && ctx->split_budget > 0)
               ? (uint32_t)std::min<int64_t>(out, ctx->split_queue) : 0;
  p.off_queue = p.off_counter + 64;
  p.qwaves = ctx->split_waves;
  p.total = p.off_queue + sizeof(uint4) * (size_t)p.qcap;
  return TC_OK;
}

void write_views(const ViewPlan& p, char* host) {
  memcpy(host + p.off_views, p.views.data(), sizeof(tci_view) * (size_t)p.n);
  memcpy(host + p.off_prefix, p.prefix.data(), sizeof(int64_t) * ((size_t)p.n + 1));
  memcpy(host + p.off_rows, p.rows.data(), sizeof(int32_t) * p.rows.size());
  memset(host + p.off_counter, 0, 64);
}

hipError_t enqueue_render(tc_context* ctx, const tci_map& d, const char* dev,
                          const ViewPlan& p, void* out, hipStream_t s,
                          hipEvent_t* kev, bool* split_ran, bool counters_zeroed) {
  tci_render_opts o = render_opts(ctx);
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
    o.queue = (uint4*)(dev + p.off_queue);
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
  if (e == hipSuccess)
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
  }
  if (ctx->map) (void)hipFree(ctx->map);
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
    if (!columns_valid(floor_top, slab_bottom, slab_top, W, H, row_stride, &bx, &by))
      return fail(ctx, TC_INVALID_ARG,
                  "tc_load_columns: column (%d,%d) violates B==0 => T==0, "
                  "B>0 => B>F and T>=B", bx, by);
    tc_status st = set_device(ctx);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;

    // level layout
    tci_map d{};
    d.W = W;
    d.H = H;
    d.top = top_level(W, H);
    size_t words = 0;
    for (int32_t L = 0; L < TCI_MAX_LEVELS; ++L) {
      tci_level& l = d.lv[L];
      if (L > d.top) {
        l = tci_level{0, 0, 0, 0};
        continue;
      }
      l.w = (int32_t)(((int64_t)W + (1 << L) - 1) >> L);
      l.h = (int32_t)(((int64_t)H + (1 << L) - 1) >> L);
      l.tiles_x = (l.w + 7) >> 3;
      l.off = (uint32_t)words;
      words += (size_t)l.tiles_x * ((l.h + 7) >> 3) * 64;
    }
    // occupancy masks of levels 1..top after the pyramid, 2 words a node
    for (int32_t L = 0; L < TCI_MAX_LEVELS; ++L) {
      tci_level& k = d.mk[L];
      k = tci_level{0, 0, 0, 0};
      if (L < 1 || L > d.top) continue;
      k = d.lv[L];
      k.off = (uint32_t)words;
      words += (size_t)k.tiles_x * ((k.h + 7) >> 3) * 128;
    }
    uint32_t* map = nullptr;
    uint8_t* planes = nullptr;
    TC_HIP(hipMalloc(&map, words * 4), "hipMalloc(map)");
    hipError_t e = hipMalloc(&planes, (size_t)3 * W * H);
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
    if (e == hipSuccess) e = tci::enqueue_edits(ctx->desc, ctx->map, (const char*)slot->dev, plan, s);
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
    st = tci::acquire(ctx, plan.total, &slot);
    if (st) return st;
    tci::write_views(plan, (char*)slot->host);
    // tables and zeroed queue counters in one upload
    hipError_t e = hipMemcpyAsync(slot->dev, slot->host, plan.off_queue,
                                  hipMemcpyHostToDevice, s);
    bool split_ran = false;
    if (e == hipSuccess)
      e = tci::enqueue_render(ctx, ctx->desc, (const char*)slot->dev, plan, out_device, s,
                              kev, &split_ran, true);
    if (kev) {
      ctx->kev_valid = e == hipSuccess;
      ctx->kev_split = split_ran;
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
      if (value < 0 || value > 4) break;
      ctx->render_mode = (int32_t)value;
      return TC_OK;
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
    case TC_OPT_SPLIT_QUEUE:
      if (value < 1 || value > (1 << 26)) break;
      ctx->split_queue = (int32_t)value;
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
    case TC_OPT_COUNT_READS:
      if (value < 0 || value > 1) break;
      if (value && !ctx->d_count) {
        if (set_device(ctx)) return TC_DEVICE_ERROR;
        hipError_t e = hipMalloc(&ctx->d_count, sizeof(unsigned long long));
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
    case TC_OPT_PRIORITY_BOOST: *value = ctx->boost; return TC_OK;
    case TC_OPT_SPLIT_BUDGET: *value = ctx->split_budget; return TC_OK;
    case TC_OPT_SPLIT_QUEUE: *value = ctx->split_queue; return TC_OK;
    case TC_OPT_BEAM_PASSES: *value = ctx->beam_passes; return TC_OK;
    case TC_OPT_SPLIT_WAVES: *value = ctx->split_waves; return TC_OK;
    case TC_OPT_KERNEL_TIMING: *value = ctx->kernel_timing; return TC_OK;
    case TC_OPT_MARCH_STEPS: *value = ctx->march_steps; return TC_OK;
    case TC_OPT_MARCH_BISECT: *value = ctx->march_bisect; return TC_OK;
    case TC_OPT_MARCH_FAR: *value = ctx->march_far; return TC_OK;
    default: return TC_INVALID_ARG;
  }
}

static tc_status read_level_rows(tc_context* ctx, int32_t L, int32_t ty0, int32_t ty1,
                                 std::vector<uint32_t>& buf, hipStream_t s) {
  const tci_level& l = ctx->desc.lv[L];
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
    st = read_level_rows(ctx, 0, ty0, ty1, buf, (hipStream_t)hip_stream);
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
    st = read_level_rows(ctx, level, 0, (l.h - 1) >> 3, buf, (hipStream_t)hip_stream);
    if (st) return st;
    l.off = 0;
    for (int32_t j = 0; j < l.h; ++j)
      for (int32_t i = 0; i < l.w; ++i) out[(size_t)j * l.w + i] = buf[tci_tile_index(l, i, j)];
    return TC_OK;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_read_pyramid: host allocation failed");
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
  const int last = ctx->kev_split ? 2 : 1;
  TC_HIP(hipEventSynchronize(ctx->kev[last]), "hipEventSynchronize");
  TC_HIP(hipEventElapsedTime(&ms[0], ctx->kev[0], ctx->kev[1]), "hipEventElapsedTime");
  ms[1] = 0.0f;
  if (ctx->kev_split)
    TC_HIP(hipEventElapsedTime(&ms[1], ctx->kev[1], ctx->kev[2]), "hipEventElapsedTime");
  return TC_OK;
}

tc_status tc_map_bytes(const tc_context* ctx, uint64_t* bytes) {
  if (!ctx || !bytes) return TC_INVALID_ARG;
  if (!ctx->map) return TC_NO_MAP;
  *bytes = (uint64_t)ctx->map_words * 4;
  return TC_OK;
}

}  // extern "C"
