/*
 * tc -- ray casting of editable two-layer height-column terrain on MI355X.
 *
 * C ABI of the library.  Plain pointers and sizes only.
 *
 * The problem (paper, Section 1: the three system constraints; Section 2:
 * the data): a map of W x H columns, each holding a floor interval and, on
 * some columns, an upper slab; every ray must find the first solid point it
 * meets, and a bounded edit of heights and slab metadata must be visible on
 * the next render without reloading or rebuilding the level.
 *
 * Geometry (the solid set is the paper's SOLID predicate, Section 3.1):
 *   world x = east (map width W), y = north (map height H), z = up;
 *   column (x, y) covers the closed square [x, x+1] x [y, y+1];
 *   it is solid for z <= F (floor, unbounded below) and, when B > 0, for
 *   B <= z <= T (upper slab).  Heights are integers 0..255.  Nothing is
 *   solid outside the map.
 *
 * Rays use Q16 fixed-point origins (S = 65536 per cell) and integer
 * directions.  The hit of a ray is the first point of the cell walk that
 * starts in floor(O / S), tests each cell over the closed parameter interval
 * the ray spends in it, and, when an x and a y boundary are crossed at the
 * same instant, steps x first.  Results are bit-exact: the same integers in
 * give the same hit word out, on any launch shape.
 *
 * Threading: a context is used by one host thread at a time.  Calls that
 * take a stream enqueue work on it and return without waiting for the GPU
 * unless stated otherwise; results are ready when the stream's work up to
 * that point completes.  A stream argument of NULL is HIP's null stream.
 *
 * Errors: every call returns a tc_status.  On failure no work has been
 * enqueued and the context state is unchanged (except where stated); the
 * message is available from tc_last_error().  No call aborts or throws.
 */
#ifndef TC_H
#define TC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tc_status;
#define TC_OK 0
#define TC_INVALID_ARG (-1)
#define TC_OUT_OF_MEMORY (-2)
#define TC_NO_MAP (-3)
#define TC_DEVICE_ERROR (-4)
#define TC_OVER_BUDGET (-5)
#define TC_TIMEOUT (-6)

#define TC_S 65536                 /* fixed-point cells per unit */
#define TC_MAX_DIM 16384           /* max W and H */
#define TC_MAX_CELLS (1 << 27)     /* max W * H */
#define TC_MAX_DIR ((1 << 23) - 1) /* max |direction component| */

/* Hit record (8 bytes).  word: bits 0-26 cell index y*W + x, bits 27-29
 * face, bit 30 layer (0 floor, 1 slab).  A miss is word 0xFFFFFFFF with
 * depth +inf.  depth is the Euclidean distance from the ray origin in world
 * units (float); 0 for TC_FACE_INSIDE.  Misses keep the cleared far depth
 * and hits carry the reconstructed depth (Section 3.1). */
typedef struct tc_hit {
  uint32_t word;
  float depth;
} tc_hit;

#define TC_MISS 0xFFFFFFFFu
#define TC_FACE_TOP 1    /* +Z: floor top or slab top, ray descending */
#define TC_FACE_UNDER 2  /* -Z: slab underside, ray ascending */
#define TC_FACE_WMX 3    /* wall facing -X, ray moving +x */
#define TC_FACE_WPX 4    /* wall facing +X, ray moving -x */
#define TC_FACE_WMY 5    /* wall facing -Y, ray moving +y */
#define TC_FACE_WPY 6    /* wall facing +Y, ray moving -y */
#define TC_FACE_INSIDE 7 /* ray origin inside solid */

/* A view: width x height pixels, rows top-down.  Pixel (px, py) casts
 *   O = o0 + (2px+1) o_px + (2py+1) o_py     (Q16 fixed point)
 *   D = d0 + (2px+1) d_px + (2py+1) d_py     (integers)
 * in 64-bit arithmetic.  A pinhole camera has o_px = o_py = 0; an
 * orthographic pass (e.g. a directional shadow pass) has d_px = d_py = 0.
 * Every pixel's O must fit in int32 and every |D_c| must be <= TC_MAX_DIR
 * (both are linear in px, py, so the library checks the four corners).
 * flags must be 0. */
typedef struct tc_view {
  int32_t width, height;
  int32_t o0[3], o_px[3], o_py[3];
  int32_t d0[3], d_px[3], d_py[3];
  uint32_t flags;
} tc_view;

/* An edit (Section 2: the renderer receives a dirty rectangle and the
 * modified rows; Section 4.4: the dig operation removes altitude and the
 * upper layer inside a crater).
 *   TC_EDIT_SET:    overwrite [x0, x0+w) x [y0, y0+h) with the host patch
 *                   floor_top / slab_bottom / slab_top (each w*h bytes,
 *                   row-major, copied before tc_apply_edit returns).  The
 *                   patch must satisfy the column invariants of
 *                   tc_load_columns.  depth is ignored.
 *   TC_EDIT_CRATER: w == h == s (1..4096), depth 0..255.  For patch cell
 *                   (i, j): r2 = (2i+1-s)^2 + (2j+1-s)^2, R2 = s^2; if
 *                   r2 < R2 the floor drops by floor(depth (R2-r2) / R2),
 *                   saturating at 0, and the slab is removed.  Pointers are
 *                   ignored.
 * Rectangles may hang over the map edge; they are clipped. */
#define TC_EDIT_SET 1
#define TC_EDIT_CRATER 2
typedef struct tc_edit {
  int32_t kind;
  int32_t x0, y0, w, h;
  int32_t depth;
  const uint8_t *floor_top, *slab_bottom, *slab_top;
} tc_edit;

typedef struct tc_context tc_context;

/* Create a context on HIP device `hip_device`.  *out receives the handle.
 * Errors: TC_INVALID_ARG (null out, bad device), TC_DEVICE_ERROR. */
tc_status tc_create(int hip_device, tc_context **out);

/* Destroy a context: waits for its outstanding work, then frees every
 * device and pinned buffer it owns.  NULL is a no-op. */
void tc_destroy(tc_context *ctx);

/* Message of the last failed call on this context ("" if none).  Owned by
 * the context, valid until the next call on it.  With a NULL context:
 * the message of the last failed tc_create. */
const char *tc_last_error(const tc_context *ctx);

/* Load a map (Section 2: height and metadata arrays).  Host arrays,
 * row-major with element (x, y) at y * row_stride + x (row_stride >= W),
 * are copied before return; the caller keeps ownership.  Builds the packed
 * tiled columns and the min/max pyramid on `hip_stream` and replaces any
 * previous map.  Validation (TC_INVALID_ARG, state unchanged):
 *   1 <= W, H <= TC_MAX_DIM, W * H <= TC_MAX_CELLS, non-null arrays, and per
 *   cell  B == 0 => T == 0  and  B > 0 => B > F and T >= B. */
tc_status tc_load_columns(tc_context *ctx, int32_t W, int32_t H,
                          const uint8_t *floor_top, const uint8_t *slab_bottom,
                          const uint8_t *slab_top, size_t row_stride,
                          void *hip_stream);

/* Apply n edits in array order (Section 2; Section 4.4), then update only
 * the pyramid nodes over the edited rectangles.  Stream-ordered: every later
 * render on the same stream sees the edits; the result is byte-identical to
 * loading the edited map from scratch.  Validation of the whole list happens
 * before anything is enqueued: kind, crater size and depth, SET pointers and
 * patch invariants (TC_INVALID_ARG), n in 0..65536, a map must be loaded
 * (TC_NO_MAP). */
tc_status tc_apply_edit(tc_context *ctx, const tc_edit *edits, int32_t n,
                        void *hip_stream);

/* Render n views (Section 3.1: one ray per pixel) into out_device, a
 * device buffer of sum(width*height) tc_hit records owned by the caller:
 * views concatenated in order, each row-major with rows top-down.  No host
 * synchronisation.  Errors before launch: TC_NO_MAP; TC_INVALID_ARG for
 * n < 1, null pointers, a view with width or height < 1 or > 16384, flags
 * != 0, |D| > TC_MAX_DIR or O outside int32 at a corner pixel, or more than
 * 2^31 rays in total. */
tc_status tc_render_views(tc_context *ctx, const tc_view *views, int32_t n,
                          tc_hit *out_device, void *hip_stream);

/* tc_render_views for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): same arguments, results and errors, and it allocates
 * nothing.  Its per-call tables and the split pass's queue live in a
 * library-owned device array of 1.25 MiB per GPU, held until the process
 * ends: the tables may take at most 256 KiB (about 2,000 views; more gives
 * TC_INVALID_ARG), and at most 65,536 long rays go to the split pass (the
 * rest finish in the first pass, with the same results).  Every call on a
 * GPU shares that GPU's array: calls on one stream are ordered, but calls
 * that overlap on one GPU (other streams, contexts or threads) race and must
 * not be issued. */
tc_status tc_render_views_noalloc(tc_context *ctx, const tc_view *views, int32_t n,
                                  tc_hit *out_device, void *hip_stream);

/* ---- shading ------------------------------------------------------------
 * The shared shading stage of the paper's methods (Section 3: one palette,
 * diffuse lighting with a height-field gradient normal, a shadow term and
 * fog; Section 3.5: cave ambient), applied to the hit records of an exact
 * render.  The paper gives no formulas; this is the library's definition.
 * Per pixel, with the ray (O, D) of its view and its hit record:
 *   miss        sky_rgba (also for a record naming no map cell, face 0,
 *               or a face the ray cannot have crossed)
 *   hit         cell (x, y), face, layer; column (F, B, T); h = T on the
 *               slab layer, else F
 *   time        t = tn / td by face: top (Oz - h S) / -Dz; underside
 *               (B S - Oz) / Dz; wall facing -X (x S - Ox) / Dx, facing +X
 *               (Ox - (x+1) S) / -Dx, and likewise in y; inside 0 / 1
 *   distance    q * len * 2^-16, q = (float)((double)tn / (double)td),
 *               len = sqrtf(((float)Dx*Dx + (float)Dy*Dy) + (float)Dz*Dz)
 *   normal      top face: n = (-gx, -gy, 1) / sqrtf((gx*gx + gy*gy) + 1),
 *               gx = (float)(s(x+1, y) - s(x-1, y)) * 0.5, gy likewise, over
 *               the hit layer's surface s (floor: F; slab: T where the
 *               column has a slab, else the hit column's T), neighbours
 *               clamped to the map; underside (0, 0, -1); walls their
 *               outward axis; inside (0, 0, 1)
 *   light       l = L / sqrtf(((float)Lx*Lx + (float)Ly*Ly) + (float)Lz*Lz);
 *               lambert = (nx*lx + ny*ly) + nz*lz
 *   shadow      if lambert > 0 and not inside: an exact ray from
 *               P = O + floor(tn * D / td) (fixed point, per component),
 *               moved one unit (2^-16 cell) out through the hit face, along
 *               L; lit iff it meets nothing
 *   intensity   I = fminf(a + (lit ? lambert : 0), 1), a = cave_ambient for
 *               a floor hit on a column with a slab, else ambient
 *   colour      per channel c = (float)albedo * I, albedo =
 *               palette[layer * 256 + h]; f = fminf(distance / fog_far, 1);
 *               c = c + ((float)fog - c) * f; byte (uint8)(c + 0.5); alpha 255
 * Single precision, one IEEE operation at a time in this order, no fused
 * multiply-add: the output is reproducible bit for bit. */
typedef struct tc_shade_params {
  int32_t light[3];        /* integer direction toward the light, |c| <=
                              TC_MAX_DIR, not all 0 */
  float ambient;           /* 0..1 */
  float cave_ambient;      /* 0..1 */
  float fog_far;           /* > 0: distance of complete fog */
  uint32_t sky_rgba;       /* R | G << 8 | B << 16 | A << 24 */
  uint32_t fog_rgba;
  const uint32_t *palette; /* host, 512 RGBA entries: floor top at height h,
                              then slab top at height h; copied */
} tc_shade_params;

/* Shade n views whose hit records (tc_render_views of the same views on the
 * current map, in any exact render mode) are in hits_device, into
 * rgba_device (one uint32 per pixel, same order), owned by the caller.
 * The shadow rays use the exact walk and the context's render knobs.
 * Errors: as tc_render_views for the views; TC_INVALID_ARG for null
 * pointers, a zero or too long light direction, fog_far <= 0 or not
 * finite, ambient terms outside 0..1. */
tc_status tc_shade_views(tc_context *ctx, const tc_view *views, int32_t n,
                         const tc_hit *hits_device, const tc_shade_params *params,
                         uint32_t *rgba_device, void *hip_stream);

/* ---- options ---------------------------------------------------------- */
/* Tuning knobs of the render path.  Each takes effect for later calls. */
#define TC_OPT_RENDER_MODE 1   /* 0 hierarchical (default), 1 flat walk,
                                  2 persistent packet queue, 4 hierarchical
                                  with occupancy masks, 5 the voxel-
                                  accelerated march over the voxel
                                  occupancy pyramid (TC_OPT_VOXEL_SHAPE; all
                                  five exact and bit-identical); 3 the
                                  sampled march below */
#define TC_OPT_VOXEL_SHAPE 21  /* voxels of the occupancy pyramid of render
                                  mode 5 (Section 3.2: one bit per voxel in
                                  Morton-ordered 8x8x8 tiles, each level the
                                  union of its eight children): v | vz << 8
                                  for voxels of v x v cells by vz height
                                  units, v and vz in 1, 2, 4, 8; 0 (default)
                                  keeps no pyramid.  Setting it builds the
                                  pyramid for the loaded map (synchronous);
                                  tc_load_columns rebuilds it and edits
                                  update the tiles over edited cells and
                                  their ancestors.  Frames captured before a
                                  change are stale; a server refuses to start
                                  while a pyramid is kept */
#define TC_OPT_START_LEVEL 2   /* pyramid level a ray starts at from its
                                  origin (default 2); clamped to the top
                                  level.  Walks the packet beam or the split
                                  pass start on a cell line begin at level 0 */
#define TC_OPT_MAX_LEVEL 3     /* highest level a ray ascends to (default
                                  top level) */
#define TC_OPT_XCD_REMAP 4     /* G > 0: each XCD runs G consecutive blocks
                                  of 2 packets at a time (L2 locality);
                                  0: hardware round-robin (default 64) */
#define TC_OPT_PERSIST_WAVES 5 /* waves per CU of the persistent launch
                                  (default 8) */
#define TC_OPT_REFILL_MIN 6    /* persistent mode: idle lanes that trigger a
                                  refill (1..64, default 16) */
#define TC_OPT_REFILL_ITERS 7  /* persistent mode: traversal iterations
                                  between refill checks (default 16) */
#define TC_OPT_COUNT_READS 8   /* 1: renders add the number of pyramid nodes
                                  and cells each ray reads to a context
                                  counter (diagnostic; default 0) */
#define TC_OPT_PACKET_WIDTH 20 /* shape of the 64-pixel packet (one wave) the
                                  one-thread-per-pixel modes cast together:
                                  its width in pixels, 4, 8, 16 or 32 (height
                                  64 / width; default 8).  The packet beam
                                  bounds the packet's rays, so the shape sets
                                  how tight its boxes are */
#define TC_OPT_TILE_ORDER 9    /* order of the pixel packets within a view:
                                  0 row-major, 1 column-major, 2 tile rows
                                  sorted so the rows whose rays are closest
                                  to horizontal (the longest walks) start
                                  first (default 2) */
#define TC_OPT_PRIORITY_BOOST 10 /* one-thread-per-pixel modes: a wave raises
                                    its issue priority after this many,
                                    twice and four times as many traversal
                                    steps, so long walks do not trail the
                                    launch (0: never; default 0) */
#define TC_OPT_SPLIT_BUDGET 11   /* hierarchical mode: a ray still walking
                                    after this many steps is finished by a
                                    second pass that walks 64 runs of its
                                    path per wave in parallel (4 waves by
                                    default), each from the exact state the
                                    walk enters it with (0: no second pass;
                                    default 120) */
#define TC_OPT_SPLIT_QUEUE 12    /* most rays the second pass takes per call;
                                    further long rays finish in the first
                                    pass (1..2^24, default 131072; every slot
                                    of the staging ring holds a device queue
                                    of this many 16-byte entries) */
#define TC_OPT_SPLIT_WAVES 18    /* waves of one block the second pass gives
                                    each long ray: its remaining path is cut
                                    into 64 runs per wave, each walked by one
                                    lane from the exact state the walk enters
                                    it with; the earliest run with a hit gives
                                    the record (1, 2 or 4; default 4) */
#define TC_OPT_BEAM_PASSES 17    /* render modes 0, 4 and 5: before walking,
                                    the 64 rays of each pixel packet find a
                                    common start parameter t such that none
                                    of them meets solid in [0, t], by testing
                                    bounding boxes of the packet's ray bundle
                                    over 64 intervals at a time against the
                                    window levels of the min/max pyramid
                                    (one entry per box), at most this many
                                    times (Section 3.2's skip of empty space,
                                    for a bundle); each ray then walks exactly
                                    from the last cell line it enters before
                                    t, so results are unchanged (0: rays start
                                    at the eye; 0..64, default 6) */
/* Render mode 3 is the paper's sampled ray march (Section 3.1, RAYMARCH),
 * not an exact cast.  Per pixel the segment from the eye ends at the far
 * limit (TC_OPT_MARCH_FAR world units along the ray) or where the ray
 * reaches z = 0, whichever is first; TC_OPT_MARCH_STEPS points spaced
 * uniformly inside it are tested in order with the SOLID predicate; the
 * first solid one and the one before it (or the eye) are refined by
 * TC_OPT_MARCH_BISECT halvings and the solid end is the hit.  The end point
 * is never tested, so a ray with no solid sample is a miss.  All arithmetic
 * is IEEE single precision, one rounding per operation:
 *   o = (float)O * 2^-16, d = (float)D, len = sqrt((dx*dx + dy*dy) + dz*dz),
 *   t_end = far / len, then min(t_end, -oz / dz) if dz < 0,
 *   dt = t_end / (steps + 1), sample i at t = (float)i * dt,
 *   point = o + t * d, midpoint (ta + tb) * 0.5, depth = tb * len,
 * so results are reproducible bit for bit.  A hit word holds the column of
 * the final point, face 0 (TC_FACE_SAMPLED) and the layer whose interval
 * holds it.  A sample can step over a feature thinner than its spacing:
 * that is the method's quality/cost trade-off (Section 3.1). */
#define TC_FACE_SAMPLED 0
#define TC_OPT_MARCH_STEPS 14    /* forward samples, 1..65536 (default 128) */
#define TC_OPT_MARCH_BISECT 15   /* bisection steps, 0..64 (default 4) */
#define TC_OPT_MARCH_FAR 16      /* far limit in world units, 1..2^20
                                    (default 600, Section 5) */
#define TC_OPT_KERNEL_TIMING 13  /* 1: tc_render_views and tc_shade_views
                                    time each kernel with HIP events, read
                                    back by
                                    tc_read_kernel_times (diagnostic;
                                    default 0) */
#define TC_OPT_INLINE_TABLES 22  /* 1: a tc_render_views call in the
                                    hierarchical mode (no read counting) whose
                                    view records, packet prefix and tile-row
                                    table fit in 1536 bytes passes them in
                                    the kernels' arguments, so no upload
                                    precedes its render; 0: every call
                                    uploads its tables (default 1; results
                                    are identical) */
/* Read-only (tc_get_option): the number of device and pinned host
 * allocations the context has made since tc_create, its frames' included.
 * tc_create allocates the staging ring (16 slots of table buffers and split
 * queues) up front, so tc_render_views, tc_apply_edit and tc_shade_views
 * allocate nothing unless their tables outgrow a slot (256 KiB) or
 * TC_OPT_SPLIT_QUEUE grows. */
#define TC_INFO_ALLOCATIONS 19
tc_status tc_set_option(tc_context *ctx, int32_t key, int64_t value);
tc_status tc_get_option(const tc_context *ctx, int32_t key, int64_t *value);

/* ---- batched frames ---------------------------------------------------- */
/* A frame: n edits (applied in order, then the dirty-node pyramid update)
 * followed by the render of nviews views into out_device, captured once
 * into a HIP graph with its tables copied to device memory, and replayed
 * with one graph launch.  Every launch applies the edits again (a crater
 * list digs deeper each frame) and renders the edited map.  The render
 * knobs in force at creation are baked in.  A frame is tied to the map it
 * was created on: after tc_load_columns, tc_frame_launch fails with
 * TC_INVALID_ARG.  Validation as for tc_apply_edit and tc_render_views.
 * The paper renders each frame in isolation with nothing overlapping
 * (Section 7); a frame batches views, shadow passes and edits instead. */
typedef struct tc_frame tc_frame;
tc_status tc_frame_create(tc_context *ctx, const tc_view *views, int32_t nviews,
                          const tc_edit *edits, int32_t nedits,
                          tc_hit *out_device, void *hip_stream, tc_frame **out);
/* Enqueue one replay of the frame on hip_stream (no host synchronisation). */
tc_status tc_frame_launch(tc_frame *frame, void *hip_stream);
/* Total rays of the frame's views. */
tc_status tc_frame_rays(const tc_frame *frame, int64_t *rays);
/* Wait for the device, then free the graph and tables.  NULL is a no-op. */
void tc_frame_destroy(tc_frame *frame);

/* ---- autotuning ----------------------------------------------------------- */
/* Time tc_render_views on these views (reps timed calls per setting, median)
 * over a grid of the render knobs -- traversal mode, start level, packet
 * order, XCD grouping, split budget (0 or 120), and the persistent queue's
 * waves per CU, refill threshold and refill interval, then the packet beam
 * passes (0, 2, 4, 6 or 8) of the best one-thread-per-pixel setting, then the
 * packet shape (width 4, 8, 16 or 32), the split budget (96, 112, 128 or 160, when
 * the best setting splits) and the pyramid depth (TC_OPT_MAX_LEVEL: the top
 * level, two and four below it, or 5) around the best setting; when the best
 * setting is the one-thread-per-pixel mode, a second pass then varies each of
 * its knobs (start level, packet order, XCD grouping, split budget 0, 96,
 * 112, 120, 128 or 160, beam passes, packet width, pyramid depth) once more, one
 * at a time, around the best setting -- then keep the fastest setting on the
 * context and report it.  Results are those of
 * tc_render_views for every setting (bit-identical); only the time differs.  Synchronises
 * hip_stream.  The paper picks each method's knob by a sweep on a fixed
 * fixture (Section 5.6); this tunes on the caller's workload. */
typedef struct tc_tune_result {
  int32_t render_mode, start_level, tile_order, xcd_remap;
  int32_t persist_waves, refill_min, refill_iters;
  float ms;      /* median time per call of the chosen setting */
  int32_t tried; /* settings timed */
  int32_t split_budget;
  int32_t beam_passes;
  int32_t packet_width; /* TC_OPT_PACKET_WIDTH */
  int32_t max_level;    /* TC_OPT_MAX_LEVEL: the pyramid depth walks use */
} tc_tune_result;
tc_status tc_autotune(tc_context *ctx, const tc_view *views, int32_t n,
                      tc_hit *out_device, int32_t reps, void *hip_stream,
                      tc_tune_result *best);

/* ---- request server -------------------------------------------------------
 * Keeps the map resident and serves view and edit requests submitted from
 * any thread (Section 2: edits are gameplay operations that must show up
 * without a reload; Section 7: the paper's frames run one at a time).  A
 * server thread admits requests strictly in submission order; a view is
 * admitted once its hit buffer fits in a device pool of budget_bytes (the
 * in-flight budget), and admitted views are launched together, up to
 * max_batch_views per render, on one of `streams` streams, so work that
 * arrives while other batches run overlaps them on the device (a batch
 * starts beside one in flight once at least two views wait; a lone view
 * waits for the batch in flight, as in a FIFO).  Batches use
 * the context's render mode and knobs; the split pass of the hierarchical
 * mode runs for batches of at most two views and is off for larger ones.  A view sees exactly the edits submitted before
 * it: the map is kept in two version buffers, and an edit is applied to the
 * buffer not holding the newest version, once no batch reads it, after that
 * buffer replays the previous edit (a replay the server starts on its own as
 * soon as no batch reads that buffer, so an edit usually waits only for its
 * own update); starting a server copies the map once
 * into the second buffer.  While a server runs it owns the map:
 * tc_load_columns, tc_apply_edit, tc_render_views and frames on the context
 * fail with TC_INVALID_ARG, and the render knobs must not change.
 * tc_server_stop drains all submitted work and leaves the newest map
 * version in the context. */
typedef struct tc_server tc_server;
#define TC_SERVER_AUTO_RELEASE 1u /* free a view's hit buffer when it is done
                                     (its result is discarded) */
tc_status tc_server_start(tc_context *ctx, uint64_t budget_bytes,
                          int32_t max_batch_views, int32_t streams,
                          uint32_t flags, tc_server **out);
/* Queue a view; *id identifies it.  TC_OVER_BUDGET if its hit buffer alone
 * exceeds the budget; validation as for tc_render_views. */
tc_status tc_server_submit_view(tc_server *s, const tc_view *view, uint64_t *id);
/* Queue an edit list (applied in order, as tc_apply_edit); SET patches are
 * copied before return. */
tc_status tc_server_submit_edit(tc_server *s, const tc_edit *edits, int32_t n,
                                uint64_t *id);
/* State of a request: 0 queued, 1 on the device, 2 done; latency from
 * submission to observed completion in seconds (-1 until done). */
tc_status tc_server_poll(tc_server *s, uint64_t id, int32_t *state,
                         double *latency_s);
/* tc_server_poll of n requests at once, under one lock: states[i] and (if
 * latencies_s is not NULL) latencies_s[i] for ids[i].  All ids are checked
 * first; an unknown one gives TC_INVALID_ARG with nothing written. */
tc_status tc_server_poll_many(tc_server *s, const uint64_t *ids, int32_t n,
                              int32_t *states, double *latencies_s);
/* Block until the request is done (TC_OK) or timeout_s passes (TC_TIMEOUT). */
tc_status tc_server_wait(tc_server *s, uint64_t id, double timeout_s);
/* Device pointer to a finished view's hit records (width*height, rows
 * top-down), valid until tc_server_release. */
tc_status tc_server_result(tc_server *s, uint64_t id, const tc_hit **device_ptr,
                           int64_t *records);
/* Copy a finished view's hit records to host memory (`records` entries;
 * must equal width*height).  Synchronous. */
tc_status tc_server_read(tc_server *s, uint64_t id, tc_hit *host_dst,
                         int64_t records);
/* Forget a finished request and return its hit buffer to the pool. */
tc_status tc_server_release(tc_server *s, uint64_t id);
typedef struct tc_server_stats {
  uint64_t batches, edits, views, rays;
  uint64_t peak_bytes;   /* largest pool use seen */
  uint64_t bytes_in_use;
  double queue_s;        /* sum over finished views of submission -> launch
                            (admission, batching and the host's launch path) */
  double run_s;          /* sum over finished views of launch -> observed
                            completion (GPU time and completion polling) */
} tc_server_stats;
tc_status tc_server_get_stats(tc_server *s, tc_server_stats *out);
/* Finish every submitted request, stop the thread and free the server. */
tc_status tc_server_stop(tc_server *s);

/* ---- inspection (tests, checkpoints) ---------------------------------- */
/* Copy the w x h rectangle at (x0, y0) of the current map into host arrays
 * (row-major, w bytes per row).  Synchronises `hip_stream`.  The rectangle
 * must lie inside the map. */
tc_status tc_read_columns(tc_context *ctx, int32_t x0, int32_t y0, int32_t w,
                          int32_t h, uint8_t *floor_top, uint8_t *slab_bottom,
                          uint8_t *slab_top, void *hip_stream);

/* Number of pyramid levels above the cells (level 1 .. tc_levels), and the
 * node grid of a level: ceil(W / 2^L) x ceil(H / 2^L). */
tc_status tc_pyramid_info(const tc_context *ctx, int32_t *levels);
tc_status tc_pyramid_dims(const tc_context *ctx, int32_t level, int32_t *w,
                          int32_t *h);

/* Copy pyramid level L (1..levels) into host memory as row-major uint32
 * nodes fmax | smin << 8 | smax << 16, where over the node's block of
 * cells fmax = max F, smin = min B of two-layer cells (255 if none), smax =
 * max T of two-layer cells (0 if none).  Synchronises `hip_stream`. */
tc_status tc_read_pyramid(tc_context *ctx, int32_t level, uint32_t *out,
                          void *hip_stream);

/* Copy window level `level` (0..levels) into host memory, row-major, dims
 * as tc_pyramid_dims: entry (i, j) holds fmax | smin << 8 | smax << 16 over
 * the cells of the 2^(L+1) x 2^(L+1) square whose corner is node (i, j)'s
 * corner, clipped to the map (Section 3.2: a conservative bound of a region
 * from the hierarchy).  The packet beam tests a box narrower than a level-L
 * node against one entry.  Synchronises `hip_stream`. */
tc_status tc_read_window(tc_context *ctx, int32_t level, uint32_t *out, void *hip_stream);

/* Copy the occupancy masks of pyramid level `level` (1..levels) to `out`,
 * row-major, dims as tc_pyramid_dims.  Bit k of a node's mask is set iff
 * the slab interval [B, T] of some column of its 2^L x 2^L block meets the
 * closed height band [4k, 4k + 4] (Section 3.2: a conservative occupancy
 * hierarchy whose levels are unions of their children).  Render mode 4
 * skips a node whose slabs the ray passes between.  Synchronises
 * `hip_stream`. */
tc_status tc_read_occupancy(tc_context *ctx, int32_t level, uint64_t *out,
                            void *hip_stream);

/* The voxel occupancy pyramid of render mode 5 (when TC_OPT_VOXEL_SHAPE is
 * set): voxel counts of level `level` (0 the finest) and, if `levels` is
 * not NULL, the number of levels.  TC_NO_MAP when there is no pyramid. */
tc_status tc_voxel_dims(const tc_context *ctx, int32_t level, int32_t *nx, int32_t *ny,
                        int32_t *nz, int32_t *levels);
/* Copy voxel level `level` into host memory as one byte (0 or 1) per
 * voxel, indexed [z][y][x] (z fastest-varying last: out[(z ny + y) nx + x]).
 * Level 0: bit set iff a column of the voxel's footprint has solid in its
 * closed height range; level k: the union of its eight children.
 * Synchronises `hip_stream`. */
tc_status tc_read_voxels(tc_context *ctx, int32_t level, uint8_t *out, void *hip_stream);

/* Read and reset the counter of TC_OPT_COUNT_READS: the number of
 * pyramid nodes and cells read by all rays rendered since the last reset
 * (the shading pass adds its hit columns, gradient neighbours and the
 * nodes and cells of its shadow rays).
 * Synchronises `hip_stream`.  0 if counting was never enabled. */
tc_status tc_read_counters(tc_context *ctx, uint64_t *reads, void *hip_stream);

/* Durations in milliseconds of the kernels of the most recent
 * tc_render_views or tc_shade_views call made with TC_OPT_KERNEL_TIMING on,
 * measured with HIP events: ms[0] the traversal kernel (any render mode) or
 * the shading kernel, ms[1] the split pass (0 when it did not run).  A call
 * whose tables travel in the kernels' arguments (TC_OPT_INLINE_TABLES) has
 * the events attached to its kernels' dispatches, so they time each kernel
 * from its start to its end; other calls record them on the stream between
 * the kernels, so a duration also holds the kernel's dispatch.  `ms` holds 2
 * floats.  Waits for those events.  TC_INVALID_ARG if no timed call was
 * made since timing was switched on. */
tc_status tc_read_kernel_times(tc_context *ctx, float *ms);

/* Device bytes held by the map: packed columns plus every pyramid level,
 * occupancy mask level and window level. */
tc_status tc_map_bytes(const tc_context *ctx, uint64_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
