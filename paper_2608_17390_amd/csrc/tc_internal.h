// Internal declarations shared by the host runtime and the kernels of the
// library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tc_plan.h"  // level, map, view and edit records

__host__ __device__ inline uint32_t tci_tile_index(const tci_level& L,
                                                   int32_t i, int32_t j) {
  return L.off + ((uint32_t)((j >> 3) * L.tiles_x + (i >> 3)) << 6) +
         (uint32_t)((j & 7) << 3) + (uint32_t)(i & 7);
}

// Word index of the low word of node (i, j)'s occupancy mask.
__host__ __device__ inline uint32_t tci_mask_index(const tci_level& M,
                                                   int32_t i, int32_t j) {
  return M.off + ((uint32_t)((j >> 3) * M.tiles_x + (i >> 3)) << 7) +
         ((((uint32_t)(j & 7) << 3) + (uint32_t)(i & 7)) << 1);
}

// Render tuning.
struct tci_render_opts {
  int32_t start_level;
  int32_t max_level;
  int32_t xcd_remap;
  int32_t refill_min;
  int32_t refill_iters;
  int32_t tile_order;          // packets in a view: 0 row-major, 1 column-major,
                               // 2 tile rows in the order of a row table
  const int32_t* rows;         // row table of order 2
  int32_t boost;               // iterations before a wave raises its priority
                               // (0: never)
  int32_t split_budget;        // hierarchical mode: steps before a ray is
                               // handed to the split pass (0: never)
  int32_t beam_passes;         // hierarchical modes: search passes of the
                               // packet beam start (0: rays start at the eye)
  uint32_t qcap;               // capacity of the split queue
  uint4* queue;                // split queue: (view, pixel index, first
                               // dominant-axis cell line still to walk, 0)
  uint32_t* qcount;            // split queue length
  uint32_t* qzero;             // if set: a queue counter to clear (the one the
                               // next render of the same ring slot uses)
  int32_t split_waves;         // waves of one block the split pass gives
                               // each queued ray (1, 2 or 4)
  unsigned long long* count;   // if set: add each ray's node/cell reads
  float march_far;             // sampled march: far limit along each ray
  int32_t march_steps;         // sampled march: forward samples
  int32_t march_bisect;        // sampled march: bisection steps
};

// A render call's tables (view records, packet prefix and tile-row table,
// laid out as in the device table: views at byte 0) carried by value in a
// kernel's arguments, for calls whose tables fit in kInlineBytes.
constexpr int32_t kInlineBytes = 1536;
struct tci_inline {
  uint32_t off_prefix;         // byte offset of the packet prefix in words
  uint32_t off_rows;           // byte offset of the tile-row table
  uint64_t words[kInlineBytes / 8];
};

// Shading parameters (the device copy of tc_shade_params).
struct tci_shade {
  int32_t light[3];            // integer direction toward the light
  float ambient, cave_ambient, fog_far;
  uint32_t sky_rgba, fog_rgba;
  const uint32_t* palette;     // 512 RGBA entries in device memory
};

// ---- launchers (return hipError_t of the launch) -------------------------
hipError_t tci_launch_repack(const uint8_t* planes, int32_t W, int32_t H,
                             uint32_t* base, tci_level l0, hipStream_t s);
hipError_t tci_launch_build_level(const tci_map& m, uint32_t* base, int32_t L,
                                  hipStream_t s);
// Edits in list order (olap: the overlap lists of the uploaded edit plan;
// olap_all: test every edit against every other instead).
hipError_t tci_launch_edits(const tci_edit* edits, int32_t n, const int32_t* olap,
                            bool olap_all, const uint8_t* patch, uint32_t* base,
                            tci_level l0, int32_t W, int32_t H,
                            int32_t max_w, int32_t max_h, hipStream_t s);
// One launch per group of levels s + 1 .. e after edits: recompute the
// nodes (and occupancy masks) of those levels over their rectangles and the
// window entries of levels s .. e - 1, with wtop s .. e, over theirs
// (entries x0 - 1 .. x1, y0 - 1 .. y1), all from level s, which must be up
// to date (e - s <= 3).  The launch also clears zero[0 .. nzero) (nzero <=
// 256), or a launch of its own does if there is nothing to update.  rects holds
// nr rectangles per level (x0, y0, x1, y1 inclusive, in that level's node
// coordinates), level L's at rects + 4 * (L * stride + r); max_lanes bounds
// the lanes of any one rectangle job (2^(L - s) per node of level L,
// 2^(L - s + 1) per window entry).
hipError_t tci_launch_update_group(const tci_map& m, uint32_t* base, int32_t s, int32_t e,
                                   bool wtop, const int32_t* rects, int32_t stride, int32_t nr,
                                   int64_t max_lanes, hipStream_t st, uint64_t* zero = nullptr,
                                   int32_t nzero = 0);

// Window level L from level L (all entries), and its entries whose node
// block meets one of the level-L rectangles (x0, y0, x1, y1 inclusive):
// entries x0 - 1 .. x1, y0 - 1 .. y1, the largest spanning max_w x max_h.
hipError_t tci_launch_build_window(const tci_map& m, uint32_t* base, int32_t L,
                                   hipStream_t s);
// The same launch also clears zero[0 .. nzero) (nzero <= 256), or, with no
// rectangle, a launch of its own does.
hipError_t tci_launch_update_window(const tci_map& m, uint32_t* base, int32_t L,
                                    const int32_t* rects, int32_t nrect, int32_t max_w,
                                    int32_t max_h, hipStream_t s, uint64_t* zero = nullptr,
                                    int32_t nzero = 0);

// Render: views on the device, one thread per pixel.  flat: 0 the
// hierarchical walk, 1 the flat walk, 2 the hierarchical walk with the
// occupancy masks, 3 the walk over the voxel occupancy pyramid *vx.
hipError_t tci_launch_render(const tci_map& m, const tci_view* views,
                             int32_t nviews, const int64_t* pkt_prefix,
                             int64_t npkt, void* out, int32_t flat,
                             const tci_render_opts& o, hipStream_t s,
                             const tci_voxels* vx = nullptr);
// Voxel occupancy pyramid level k: every word (rects null), or the words of
// the tiles over each of the nrect clipped cell rectangles (x0, y0, x1, y1
// inclusive) of an edit list.  Level k > 0 reads level k - 1.
hipError_t tci_launch_voxel_level(const tci_map& m, const tci_voxels& vx, uint32_t* vox,
                                  int32_t k, const int32_t* rects, int32_t nrect,
                                  hipStream_t s);
// Render: persistent waves pulling 64-ray packets from a queue counter.
hipError_t tci_launch_render_persistent(const tci_map& m,
                                        const tci_view* views, int32_t nviews,
                                        const int64_t* pkt_prefix,
                                        int64_t npkt, void* out,
                                        uint64_t* counter, int32_t nblocks,
                                        const tci_render_opts& o,
                                        hipStream_t s);
hipError_t tci_launch_zero_u64(uint64_t* p, int32_t n, hipStream_t s);
// Shade: per pixel, the colour of its hit record (with a shadow ray).
hipError_t tci_launch_shade(const tci_map& m, const tci_view* views, int32_t nviews,
                            const int64_t* pkt_prefix, int64_t npkt, const void* hits,
                            uint32_t* rgba, const tci_shade& sh, const tci_render_opts& o,
                            hipStream_t s);
// Render: the sampled march (RAYMARCH), one thread per pixel.
hipError_t tci_launch_march(const tci_map& m, const tci_view* views,
                            int32_t nviews, const int64_t* pkt_prefix,
                            int64_t npkt, void* out, const tci_render_opts& o,
                            hipStream_t s);
// Second pass of a hierarchical render: walk every queued long ray as 64
// segments in parallel, one wave per ray.
// With ev_start / ev_stop, the kernel records its own start and end in them
// (the events travel with its dispatch instead of as markers on the stream).
hipError_t tci_launch_split(const tci_map& m, const tci_view* views,
                            const tci_render_opts& o, void* out, int32_t nblocks,
                            hipStream_t s, const tci_inline* t = nullptr,
                            hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// The hierarchical render (no read counting) of a call whose tables travel
// in the kernel's arguments (t; the split pass then takes t as well).
hipError_t tci_launch_render_inline(const tci_map& m, int32_t nviews, int64_t npkt, void* out,
                                    const tci_render_opts& o, const tci_inline& t,
                                    hipStream_t s, hipEvent_t ev_start = nullptr,
                                    hipEvent_t ev_stop = nullptr);
