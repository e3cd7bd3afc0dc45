// Captured frames and the render autotuner.
//
// A frame is one HIP graph holding, in stream order, the edit kernel, the
// dirty-node pyramid update of every level and the render of all views
// (plus, in persistent mode, the queue-counter reset), with its tables
// resident in device memory.  Replaying it is a single hipGraphLaunch.  The
// paper renders and times each frame in isolation with nothing overlapping
// (Section 7); a frame here batches many views and shadow passes instead.
//
// The autotuner times tc_render_views over a grid of the render knobs
// (traversal mode, start level, packet order, XCD grouping, split pass,
// persistent queue parameters, beam passes, packet shape, pyramid depth)
// on the caller's views and keeps the fastest setting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "tc_context.h"

using tci::fail;
using tci::hip_fail;

struct tc_frame {
  tc_context* ctx = nullptr;
  uint64_t generation = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* dev = nullptr;
  int64_t rays = 0;
};

namespace {

void frame_free(tc_frame* f) {
  if (!f) return;
  if (f->exec) (void)hipGraphExecDestroy(f->exec);
  if (f->graph) (void)hipGraphDestroy(f->graph);
  if (f->dev) (void)hipFree(f->dev);
  delete f;
}

struct Knobs {
  int32_t mode, start, order, remap, waves, rmin, riters, split, beam, pwidth, maxl;
};

void apply_knobs(tc_context* c, const Knobs& k) {
  c->render_mode = k.mode;
  c->start_level = k.start;
  c->tile_order = k.order;
  c->xcd_remap = k.remap;
  c->persist_waves = k.waves;
  c->refill_min = k.rmin;
  c->refill_iters = k.riters;
  c->split_budget = k.split;
  c->beam_passes = k.beam;
  c->packet_width = k.pwidth;
  c->max_level = k.maxl;
}

Knobs read_knobs(const tc_context* c) {
  return Knobs{c->render_mode, c->start_level, c->tile_order, c->xcd_remap,
               c->persist_waves, c->refill_min, c->refill_iters, c->split_budget,
               c->beam_passes, c->packet_width, c->max_level};
}

}  // namespace

extern "C" {

tc_status tc_frame_create(tc_context* ctx, const tc_view* views, int32_t nviews,
                          const tc_edit* edits, int32_t nedits,
                          tc_hit* out_device, void* hip_stream,
                          tc_frame** out) {
  if (!ctx) return TC_INVALID_ARG;
  if (!out) return fail(ctx, TC_INVALID_ARG, "tc_frame_create: out is NULL");
  *out = nullptr;
  tc_frame* f = nullptr;
  hipStream_t cs = nullptr;
  try {
    ctx->err.clear();
    if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_frame_create: no map loaded");
    if (ctx->server) return fail(ctx, TC_INVALID_ARG, "tc_frame_create: a server owns the map");
    if (!out_device) return fail(ctx, TC_INVALID_ARG, "tc_frame_create: out is NULL");
    if (ctx->render_mode == 5 && !ctx->vox)
      return fail(ctx, TC_INVALID_ARG, "tc_frame_create: render mode 5 needs TC_OPT_VOXEL_SHAPE");
    tci::ViewPlan vp;
    tc_status st = tci::plan_views(ctx, views, nviews, vp);
    if (st) return st;
    size_t patch_bytes = 0;
    st = tci::validate_edits(ctx, edits, nedits, &patch_bytes);
    if (st) return st;
    tci::EditPlan ep;
    tci::plan_edits(ctx->desc, edits, nedits, patch_bytes, nullptr, ep);
    st = tci::set_device(ctx);
    if (st) return st;
    const size_t off_e = (vp.total + 255) & ~(size_t)255;
    const size_t total = off_e + (nedits > 0 ? ep.total : 0);
    std::vector<char> host(total, 0);
    tci::write_views(vp, host.data());
    if (nedits > 0) tci::plan_edits(ctx->desc, edits, nedits, patch_bytes, host.data() + off_e, ep);

    f = new tc_frame();
    f->ctx = ctx;
    f->generation = ctx->map_generation;
    f->rays = vp.rays;
    hipError_t e = tci::dev_alloc(ctx, &f->dev, total);
    if (e == hipSuccess)
      e = hipMemcpyAsync(f->dev, host.data(), total, hipMemcpyHostToDevice,
                         (hipStream_t)hip_stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = hipSuccess;
      // with edits, their last launch clears the render's counters (one
      // node fewer in the graph)
      const int32_t nz = nedits > 0 ? tci::render_counter_words(ctx, vp) : 0;
      if (nedits > 0)
        le = tci::enqueue_edits(ctx->desc, ctx->map, (const char*)f->dev + off_e, ep, cs,
                                ctx->vox ? &ctx->vdesc : nullptr, ctx->vox,
                                (uint64_t*)((char*)f->dev + vp.off_counter), nz);
      if (le == hipSuccess)
        le = tci::enqueue_render(ctx, ctx->desc, (const char*)f->dev, vp, out_device, cs,
                                 nullptr, nullptr, nz > 0);
      e = hipStreamEndCapture(cs, &f->graph);
      if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&f->exec, f->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
      frame_free(f);
      return hip_fail(ctx, e, "tc_frame_create");
    }
    *out = f;
    return TC_OK;
  } catch (...) {
    if (cs) (void)hipStreamDestroy(cs);
    frame_free(f);
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_frame_create: host allocation failed");
  }
}

tc_status tc_frame_launch(tc_frame* f, void* hip_stream) {
  if (!f) return TC_INVALID_ARG;
  tc_context* ctx = f->ctx;
  ctx->err.clear();
  if (ctx->map_generation != f->generation || !ctx->map)
    return fail(ctx, TC_INVALID_ARG, "tc_frame_launch: the map was reloaded since capture");
  if (ctx->server) return fail(ctx, TC_INVALID_ARG, "tc_frame_launch: a server owns the map");
  tc_status st = tci::set_device(ctx);
  if (st) return st;
  TC_HIP(hipGraphLaunch(f->exec, (hipStream_t)hip_stream), "hipGraphLaunch");
  return TC_OK;
}

tc_status tc_frame_rays(const tc_frame* f, int64_t* rays) {
  if (!f || !rays) return TC_INVALID_ARG;
  *rays = f->rays;
  return TC_OK;
}

void tc_frame_destroy(tc_frame* f) {
  if (!f) return;
  (void)hipSetDevice(f->ctx->device);
  (void)hipDeviceSynchronize();
  frame_free(f);
}

tc_status tc_autotune(tc_context* ctx, const tc_view* views, int32_t n,
                      tc_hit* out_device, int32_t reps, void* hip_stream,
                      tc_tune_result* best) {
  if (!ctx) return TC_INVALID_ARG;
  if (!best) return fail(ctx, TC_INVALID_ARG, "tc_autotune: best is NULL");
  if (reps < 1 || reps > 1000) return fail(ctx, TC_INVALID_ARG, "tc_autotune: bad reps");
  try {
    ctx->err.clear();
    if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_autotune: no map loaded");
    if (ctx->render_mode == 3)
      return fail(ctx, TC_INVALID_ARG, "tc_autotune: tunes the exact render modes only");
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<Knobs> cand;
    const Knobs cur = read_knobs(ctx);
    for (int32_t split : {0, 120})
      for (int32_t order : {0, 1, 2})
        for (int32_t remap : {0, 8, 64})
          for (int32_t start : {1, 2, 3, 4})
            cand.push_back(Knobs{0, start, order, remap, cur.waves, cur.rmin, cur.riters, split,
                                 cur.beam, cur.pwidth, cur.maxl});
    std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
    for (auto& e : ev) TC_HIP(hipEventCreate(&e), "hipEventCreate");
    auto time_knobs = [&](const Knobs& k, float* med) -> tc_status {
      apply_knobs(ctx, k);
      tc_status st = tc_render_views(ctx, views, n, out_device, hip_stream);
      if (st) return st;
      std::vector<float> ms((size_t)reps);
      for (int32_t r = 0; r < reps; ++r) {
        TC_HIP(hipEventRecord(ev[2 * r], s), "hipEventRecord");
        st = tc_render_views(ctx, views, n, out_device, hip_stream);
        if (st) return st;
        TC_HIP(hipEventRecord(ev[2 * r + 1], s), "hipEventRecord");
      }
      TC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
      for (int32_t r = 0; r < reps; ++r)
        TC_HIP(hipEventElapsedTime(&ms[r], ev[2 * r], ev[2 * r + 1]), "hipEventElapsedTime");
      std::nth_element(ms.begin(), ms.begin() + reps / 2, ms.end());
      *med = ms[reps / 2];
      return TC_OK;
    };
    Knobs bk = cur;
    float bms = 1e30f;
    int32_t tried = 0;
    tc_status st = TC_OK;
    for (const Knobs& k : cand) {
      float m;
      st = time_knobs(k, &m);
      if (st) break;
      ++tried;
      if (m < bms) { bms = m; bk = k; }
    }
    // persistent packet queue around the best traversal setting
    for (int32_t waves : {8, 16, 32})
      for (int32_t rmin : {8, 16, 32})
        for (int32_t riters : {16, 64}) {
          if (st) break;
          Knobs k{2, bk.start, bk.order, bk.remap, waves, rmin, riters, bk.split, bk.beam,
                  bk.pwidth, bk.maxl};
          float m;
          st = time_knobs(k, &m);
          if (st) break;
          ++tried;
          if (m < bms) { bms = m; bk = k; }
        }
    // the packet beam start of the one-thread-per-pixel modes, around the
    // best setting
    if (!st && bk.mode == 0)
      for (int32_t beam : {0, 2, 4, 6, 8}) {
        if (beam == bk.beam) continue;
        Knobs k = bk;
        k.beam = beam;
        float m;
        st = time_knobs(k, &m);
        if (st) break;
        ++tried;
        if (m < bms) { bms = m; bk = k; }
      }
    // the packet shape (its width; height 64 / width) and the pyramid depth
    // (the highest level a walk climbs to), each around the best setting
    const auto try_knob = [&](Knobs k) {
      float m;
      st = time_knobs(k, &m);
      if (st) return;
      ++tried;
      if (m < bms) { bms = m; bk = k; }
    };
    for (int32_t pwidth : {4, 8, 16, 32}) {
      if (st || pwidth == bk.pwidth) continue;
      Knobs k = bk;
      k.pwidth = pwidth;
      try_knob(k);
    }
    // the split budget, around the best setting when it splits at all
    if (!st && bk.mode == 0 && bk.split > 0)
      for (int32_t split : {96, 112, 128, 160}) {
        if (st) break;
        Knobs k = bk;
        k.split = split;
        try_knob(k);
      }
    const int32_t top = ctx->desc.top;
    const auto try_maxl = [&]() {
      for (int32_t maxl : {top, top - 2, top - 4, 5}) {
        if (st || maxl < 1 || maxl == std::min(bk.maxl, top)) continue;
        Knobs k = bk;
        k.maxl = maxl;
        try_knob(k);
      }
    };
    try_maxl();
    // a second pass over every knob of the one-thread-per-pixel mode, one at
    // a time around the best setting: each stage above held the knobs of the
    // stages after it at their starting values
    if (!st && bk.mode == 0) {
      const auto sweep = [&](int32_t Knobs::*f, std::initializer_list<int32_t> vals) {
        for (int32_t v : vals) {
          if (st || bk.*f == v) continue;
          Knobs k = bk;
          k.*f = v;
          try_knob(k);
        }
      };
      sweep(&Knobs::start, {1, 2, 3, 4});
      sweep(&Knobs::order, {0, 1, 2});
      sweep(&Knobs::remap, {0, 8, 64});
      sweep(&Knobs::split, {0, 96, 112, 120, 128, 160});
      sweep(&Knobs::beam, {0, 2, 4, 6, 8});
      sweep(&Knobs::pwidth, {4, 8, 16, 32});
      try_maxl();
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (st) {
      apply_knobs(ctx, cur);
      return st;
    }
    apply_knobs(ctx, bk);
    best->render_mode = bk.mode;
    best->start_level = bk.start;
    best->tile_order = bk.order;
    best->xcd_remap = bk.remap;
    best->persist_waves = bk.waves;
    best->refill_min = bk.rmin;
    best->refill_iters = bk.riters;
    best->split_budget = bk.split;
    best->beam_passes = bk.beam;
    best->packet_width = bk.pwidth;
    best->max_level = bk.maxl;
    best->ms = bms;
    best->tried = tried;
    return TC_OK;
  } catch (...) {
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_autotune: host allocation failed");
  }
}

}  // extern "C"
