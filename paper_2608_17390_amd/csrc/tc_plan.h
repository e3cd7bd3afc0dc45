// Host-side planning of the library's calls: validation of column planes,
// views and edit lists, the layout of the map's levels in one allocation,
// and the layout of the tables a render or an edit call uploads.  Nothing
// here touches HIP, so the file also builds with a plain C++ compiler (the
// sanitizer test builds it with g++ and AddressSanitizer / UBSan).  Not
// part of the C ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "tc.h"

#define TCI_MAX_LEVELS 16  // level 0 = cells, levels 1..15 = pyramid

// One level of the map in HBM.  Level 0 holds packed columns
// F | B << 8 | T << 16; levels >= 1 hold nodes fmax | smin << 8 | smax << 16.
// Every level is tiled in 8 x 8 blocks of 32-bit words (256 bytes, one
// wave's worth of coalesced reads): element (i, j) lives at
//   off + (((j >> 3) * tiles_x + (i >> 3)) << 6) + ((j & 7) << 3) + (i & 7).
struct tci_level {
  uint32_t off;      // offset in words from the start of the map buffer
  int32_t w, h;      // elements per row / rows
  int32_t tiles_x;   // ceil(w / 8)
};

// Occupancy masks: for every pyramid node of levels 1..top, 64 bits over
// height, bit k set iff the slab interval [B, T] of some column of the node
// meets the closed band [4k, 4k + 4].  They refine the node's slab test:
// a ray whose height range over the node meets no set band passes between
// the slabs.  Stored in the same allocation after the pyramid, tiled 8 x 8
// like the levels, two 32-bit words (low, high) per node.
//
// Window levels: for every level L = 0..top, entry (i, j) holds fmax, smin
// and smax over the cells of the 2^(L+1) square whose corner is node
// (i, j)'s, i.e. the combine of level-L nodes (i..i+1, j..j+1) that exist.
// A box narrower than a level-L node overlaps at most two nodes per axis,
// all inside the window of the first, so the packet beam tests a box with
// one load.  Same dimensions and tiling as level L, one word an entry,
// stored after the masks.
struct tci_map {
  const uint32_t* base;           // all levels, one allocation
  tci_level lv[TCI_MAX_LEVELS];
  tci_level mk[TCI_MAX_LEVELS];   // occupancy mask levels 1..top (off in words)
  tci_level wl[TCI_MAX_LEVELS];   // window levels 0..top (off in words)
  int32_t W, H;
  int32_t top;                    // highest stored level (0 if none)
};

// The voxel occupancy pyramid of the voxel-accelerated march (Section 3.2):
// voxels of 2^v_log2 x 2^v_log2 cells by 2^vz_log2 height units; a bit of
// the finest level (k = 0) is set when a column of the voxel's footprint has
// solid in its closed height range, and each higher level is the union of
// its eight children, up to a single voxel.  Every level is stored in
// Morton-ordered 8 x 8 x 8 tiles of 512 bits (16 words): tile (tx, ty, tz)
// at word off + ((tz * tiles_y + ty) * tiles_x + tx) * 16, voxel (x, y, z)
// of the tile at bit m = x0 | y0 << 1 | z0 << 2 | x1 << 3 | y1 << 4 | z1 << 5
// | x2 << 6 | y2 << 7 | z2 << 8 (the bits of x & 7, y & 7, z & 7
// interleaved) of the tile, i.e. bit m & 31 of word m >> 5.  One allocation,
// apart from the map.
struct tci_vlevel {
  uint32_t off;                 // word offset of the level
  int32_t nx, ny, nz;           // voxels per axis
  int32_t tiles_x, tiles_y, tiles_z;
};
struct tci_voxels {
  const uint32_t* base;
  int32_t v_log2, vz_log2;      // voxel footprint and height, as powers of two
  int32_t levels;               // levels 0 .. levels - 1
  tci_vlevel lv[TCI_MAX_LEVELS];
};

// Device copy of a view plus the first ray index of the view and the
// first 64-ray packet of the view.
struct tci_view {
  int32_t w, h;
  int32_t o0[3], opx[3], opy[3];
  int32_t d0[3], dpx[3], dpy[3];
  int32_t tiles_x;     // packets per row of packets: ceil(w / packet width)
  int32_t small_steps; // every per-pixel step (opx, opy, dpx, dpy) below 2^22
                       // in magnitude: twice one is a 24-bit operand
  int32_t pw_log2;     // log2 of the packet width in pixels (2..5); a packet
                       // (one wave) is 2^pw_log2 x 2^(6 - pw_log2) pixels
  int64_t out_base;    // first output record of the view
  int64_t pkt_base;    // first 8x8 packet of the view
  int64_t rows_off;    // packet order 2: offset of the view's tile-row
                       // permutation in the row table
};

// Device edit descriptor; SET data lives at data_off in the patch buffer
// as three planes of w*h bytes (F, then B, then T).
struct tci_edit {
  int32_t kind;
  int32_t x0, y0, w, h;
  int32_t depth;
  int64_t data_off;
};

namespace tci {

// Bytes of one split queue entry (view, pixel, first line, 0).
constexpr size_t kQueueEntry = 16;

// Layout of an uploaded edit list: descriptors, the clipped rectangle of
// every edit on every level 0..top (level L's at rects + 4 (L n + k)), the
// overlap lists, and SET patch bytes.  Overlap lists: int32 start[n + 1]
// then the lists, edit i's (the other edits whose clipped rectangle meets
// its own, ascending) at start[i] .. start[i + 1] - 1 after start[n]; with
// olap_all set (too many candidates to list) every edit tests every other
// and the lists are empty.
struct EditPlan {
  int32_t n = 0;
  int32_t top = 0;
  size_t off_edits = 0, off_rects = 0, off_olap = 0, off_patch = 0, total = 0;
  int32_t max_w = 1, max_h = 1;
  bool olap_all = false;
  std::vector<int32_t> nrect, rmw, rmh;   // per level 0..top
  std::vector<int32_t> olap;              // start[n + 1], then the lists
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

// The render knobs a view plan depends on.
struct PlanOpts {
  int32_t packet_width = 8;    // pixels across a 64-pixel packet: 4, 8, 16 or 32
  int32_t render_mode = 0;
  int32_t split_budget = 0;
  int32_t split_queue = 0;
  int32_t split_waves = 1;
};

// Column invariants of a w x h patch of planes with row stride `stride`:
// B == 0 => T == 0, B > 0 => B > F and T >= B.  On failure the first bad
// cell is stored in (bad_x, bad_y).
bool columns_valid(const uint8_t* F, const uint8_t* B, const uint8_t* T, int32_t w,
                   int32_t h, size_t stride, int32_t* bad_x, int32_t* bad_y);

// Level layout of the voxel occupancy pyramid of a W x H map (base null);
// *words receives the size of its allocation in 32-bit words.
tci_voxels layout_voxels(int32_t W, int32_t H, int32_t v_log2, int32_t vz_log2, size_t* words);

// Highest pyramid level of a W x H map: ceil(log2(max(W, H))).
int32_t top_level(int32_t W, int32_t H);

// Level layout of a W x H map (cells, pyramid levels 1..top, the occupancy
// masks of levels 1..top, then the window levels 0..top); base is left null.  *words receives
// the size of the allocation in 32-bit words.
tci_map layout_map(int32_t W, int32_t H, size_t* words);

// Validate an edit list (TC_OK, or TC_INVALID_ARG with the reason in *err)
// and sum the bytes of its SET patches.
tc_status check_edits(const tc_edit* edits, int32_t n, size_t* patch_bytes,
                      std::string* err);
// Fill `plan` and write the upload image of the edit list to `host`
// (plan.total bytes; call plan_edits with host == nullptr to size it).
void plan_edits(const tci_map& d, const tc_edit* edits, int32_t n,
                size_t patch_bytes, char* host, EditPlan& plan);

// Validate n views and lay out their tables.  With allow_split false the
// plan has no split queue (qcap 0), whatever the split budget.
tc_status make_view_plan(const PlanOpts& o, const tc_view* views, int32_t n,
                         ViewPlan& plan, bool allow_split, std::string* err);
// Write the tables (bytes [0, plan.off_queue)) to `host`.
void write_views(const ViewPlan& plan, char* host);

}  // namespace tci
