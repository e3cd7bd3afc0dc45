// Map maintenance kernels: column repack, pyramid build, ordered edits and
// the dirty-node pyramid update.
//
// The pyramid is the maximum-mipmap structure cited in Section 1.1,
// extended to the two solid intervals of a column: a node of level L covers
// a 2^L x 2^L block of cells and keeps the largest floor top (fmax), the
// smallest slab bottom (smin) and the largest slab top (smax) of the block.
// A ray whose height range over the node's time span stays above fmax and
// either above smax or below smin cannot meet solid in the block.
//
// Beside each node, a 64-bit occupancy mask over height (bit k: a slab of
// the block meets the band [4k, 4k + 4]) is the union of its children's,
// as the paper's occupancy pyramid takes the union of its children
// (Section 3.2); it is built and updated with the node.
//
// Window levels (one per level, used by the packet beam's box test) hold,
// per node, the combine of its 2 x 2 node neighbourhood on the same level;
// they are built after the levels and, after edits, updated for the entries
// whose neighbourhood meets an edited node.
//
// Edits follow Section 2 (a dirty rectangle with new heights and slab
// metadata) and Section 4.4 (the dig crater).  Only the nodes above the
// edited rectangles are recomputed, from the same 2x2 reduction as the full
// build, so the updated pyramid is byte-identical to a rebuild.
#include "tc_internal.h"

namespace {

constexpr int kEditSet = 1;

__device__ inline uint32_t cell_to_node(uint32_t c) {
  // packed column F | B << 8 | T << 16 -> node fmax | smin << 8 | smax << 16
  uint32_t F = c & 0xFF, B = (c >> 8) & 0xFF, T = (c >> 16) & 0xFF;
  return B ? (F | (B << 8) | (T << 16)) : (F | (255u << 8));
}

__device__ inline uint32_t node_merge(uint32_t a, uint32_t b) {
  uint32_t f = max(a & 0xFF, b & 0xFF);
  uint32_t lo = min((a >> 8) & 0xFF, (b >> 8) & 0xFF);
  uint32_t hi = max((a >> 16) & 0xFF, (b >> 16) & 0xFF);
  return f | (lo << 8) | (hi << 16);
}

// Node (i, j) of level L from its up-to-four children at level L-1.
__device__ inline uint32_t reduce_node(const tci_map& m, const uint32_t* base,
                                       int32_t L, int32_t i, int32_t j) {
  const tci_level& c = m.lv[L - 1];
  uint32_t acc = 0u | (255u << 8);  // empty: fmax 0, smin 255, smax 0
  #pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    #pragma unroll
    for (int di = 0; di < 2; ++di) {
      int32_t ci = 2 * i + di, cj = 2 * j + dj;
      if (ci < c.w && cj < c.h) {
        uint32_t v = base[tci_tile_index(c, ci, cj)];
        acc = node_merge(acc, L == 1 ? cell_to_node(v) : v);
      }
    }
  }
  return acc;
}

__global__ void repack_kernel(const uint8_t* __restrict__ planes, int32_t W,
                              int32_t H, uint32_t* __restrict__ base,
                              tci_level l0) {
  // one thread per word of the tiled level-0 array
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t ntiles = (int64_t)l0.tiles_x * ((H + 7) >> 3);
  if (k >= ntiles * 64) return;
  int32_t tile = (int32_t)(k >> 6), e = (int32_t)(k & 63);
  int32_t x = (tile % l0.tiles_x) * 8 + (e & 7);
  int32_t y = (tile / l0.tiles_x) * 8 + (e >> 3);
  uint32_t v = 0;
  if (x < W && y < H) {
    size_t idx = (size_t)y * W + x;
    size_t plane = (size_t)W * H;
    uint32_t F = planes[idx], B = planes[plane + idx], T = planes[2 * plane + idx];
    v = F | (B << 8) | (T << 16);
  }
  base[l0.off + k] = v;
}

// Occupancy bands of one column's slab [B, T]: bits (B + 3) / 4 - 1 ..
// T / 4, the bands [4k, 4k + 4] that meet it (none without a slab).
__device__ inline uint64_t cell_mask(uint32_t c) {
  const uint32_t B = (c >> 8) & 0xFF, T = (c >> 16) & 0xFF;
  if (!B) return 0;
  const uint32_t lo = (B + 3) / 4 - 1, hi = T / 4;
  return (~0ull >> (63 - hi)) & (~0ull << lo);
}

// Occupancy mask of node (i, j) of level L: the union of its children's.
__device__ inline uint64_t reduce_mask(const tci_map& m, const uint32_t* base,
                                       int32_t L, int32_t i, int32_t j) {
  const tci_level& c = m.lv[L - 1];
  uint64_t acc = 0;
  #pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    #pragma unroll
    for (int di = 0; di < 2; ++di) {
      int32_t ci = 2 * i + di, cj = 2 * j + dj;
      if (ci < c.w && cj < c.h) {
        if (L == 1) {
          acc |= cell_mask(base[tci_tile_index(c, ci, cj)]);
        } else {
          const uint32_t k = tci_mask_index(m.mk[L - 1], ci, cj);
          acc |= (uint64_t)base[k] | ((uint64_t)base[k + 1] << 32);
        }
      }
    }
  }
  return acc;
}

__device__ inline void store_mask(const tci_map& m, uint32_t* base, int32_t L,
                                  int32_t i, int32_t j, uint64_t v) {
  const uint32_t k = tci_mask_index(m.mk[L], i, j);
  base[k] = (uint32_t)v;
  base[k + 1] = (uint32_t)(v >> 32);
}

__global__ void build_level_kernel(tci_map m, uint32_t* __restrict__ base,
                                   int32_t L) {
  const tci_level& l = m.lv[L];
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)l.tiles_x * ((l.h + 7) >> 3) * 64;
  if (k >= total) return;
  int32_t tile = (int32_t)(k >> 6), e = (int32_t)(k & 63);
  int32_t i = (tile % l.tiles_x) * 8 + (e & 7);
  int32_t j = (tile / l.tiles_x) * 8 + (e >> 3);
  uint32_t v = 0;
  uint64_t mask = 0;
  if (i < l.w && j < l.h) {
    v = reduce_node(m, base, L, i, j);
    mask = reduce_mask(m, base, L, i, j);
  }
  base[l.off + k] = v;
  store_mask(m, base, L, i, j, mask);
}

__device__ inline bool covers(const tci_edit& e, int32_t x, int32_t y) {
  return x >= e.x0 && x < e.x0 + e.w && y >= e.y0 && y < e.y0 + e.h;
}

// Apply edit e to a packed column at cell (x, y) inside e's rectangle.
__device__ inline uint32_t apply_one(const tci_edit& e,
                                     const uint8_t* __restrict__ patch,
                                     uint32_t col, int32_t x, int32_t y) {
  int32_t i = x - e.x0, j = y - e.y0;
  if (e.kind == kEditSet) {
    int64_t n = (int64_t)e.w * e.h;
    int64_t o = e.data_off + (int64_t)j * e.w + i;
    uint32_t F = patch[o], B = patch[o + n], T = patch[o + 2 * n];
    return F | (B << 8) | (T << 16);
  }
  // crater of size s = w = h <= 4096 and depth <= 255: r2 < 2^25 and
  // depth (R2 - r2) < 2^32, so 32-bit arithmetic is exact
  const int32_t s = e.w;
  const int32_t a = 2 * i + 1 - s, b = 2 * j + 1 - s;
  const uint32_t r2 = (uint32_t)(a * a) + (uint32_t)(b * b), R2 = (uint32_t)(s * s);
  if (r2 >= R2) return col;
  const uint32_t drop = ((uint32_t)e.depth * (R2 - r2)) / R2;
  const uint32_t F = col & 0xFF;
  return F > drop ? F - drop : 0u;  // slab removed: B = T = 0
}

// grid.x = edit index; threads stride over that edit's clipped rectangle.
// A cell is owned by the first edit that covers it; the owner applies all
// covering edits in list order, so the result is the sequential one and no
// two threads write the same cell.  Only the edits whose rectangles meet
// this edit's can cover its cells: olap lists them (start[n + 1], then the
// ascending lists), or with `all` every edit is tested.
__global__ void edits_kernel(const tci_edit* __restrict__ edits, int32_t n,
                             const int32_t* __restrict__ olap, int32_t all,
                             const uint8_t* __restrict__ patch,
                             uint32_t* __restrict__ base, tci_level l0,
                             int32_t W, int32_t H) {
  const int32_t ei = blockIdx.x;
  const tci_edit e = edits[ei];
  const int32_t x0 = max(e.x0, 0), y0 = max(e.y0, 0);
  const int32_t x1 = min(e.x0 + e.w, W), y1 = min(e.y0 + e.h, H);
  if (x0 >= x1 || y0 >= y1) return;
  const int32_t lb = all ? 0 : olap[ei], lc = all ? n : olap[ei + 1] - lb;
  const int32_t* lst = olap + n + 1 + lb;
  // (a clipped rectangle holds at most 2^28 cells)
  const int32_t cw = x1 - x0, cells = cw * (y1 - y0);
  for (int32_t k = blockIdx.y * blockDim.x + threadIdx.x; k < cells;
       k += gridDim.y * blockDim.x) {
    const int32_t x = x0 + k % cw, y = y0 + k / cw;
    bool owned = true;
    for (int32_t t = 0; t < lc; ++t) {
      const int32_t p = all ? t : lst[t];
      if (p >= ei) break;
      if (covers(edits[p], x, y)) {
        owned = false;
        break;
      }
    }
    if (!owned) continue;
    const uint32_t idx = tci_tile_index(l0, x, y);
    uint32_t col = apply_one(e, patch, base[idx], x, y);
    for (int32_t t = 0; t < lc; ++t) {
      const int32_t q = all ? t : lst[t];
      if (q > ei && covers(edits[q], x, y)) col = apply_one(edits[q], patch, col, x, y);
    }
    base[idx] = col;
  }
}

// Window entry (i, j) of level L: the combine of level-L nodes (i..i+1,
// j..j+1) that exist (level 0: the cells, as nodes).
__device__ inline uint32_t window_entry(const tci_map& m, const uint32_t* base, int32_t L,
                                        int32_t i, int32_t j) {
  const tci_level& l = m.lv[L];
  uint32_t acc = 0u | (255u << 8);  // empty: fmax 0, smin 255, smax 0
  #pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    #pragma unroll
    for (int di = 0; di < 2; ++di) {
      const int32_t ni = i + di, nj = j + dj;
      if (ni < l.w && nj < l.h) {
        const uint32_t v = base[tci_tile_index(l, ni, nj)];
        acc = node_merge(acc, L == 0 ? cell_to_node(v) : v);
      }
    }
  }
  return acc;
}

__global__ void build_window_kernel(tci_map m, uint32_t* __restrict__ base, int32_t L) {
  const tci_level& w = m.wl[L];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)w.tiles_x * ((w.h + 7) >> 3) * 64;
  if (k >= total) return;
  const int32_t tile = (int32_t)(k >> 6), e = (int32_t)(k & 63);
  const int32_t i = (tile % w.tiles_x) * 8 + (e & 7);
  const int32_t j = (tile / w.tiles_x) * 8 + (e >> 3);
  base[w.off + k] = (i < w.w && j < w.h) ? window_entry(m, base, L, i, j) : 0u;
}

// grid.x = rectangle index: entries x0 - 1 .. x1, y0 - 1 .. y1 (clipped to
// the level) of the level-L rectangle, the entries whose 2 x 2 node block
// meets it.  The first block also clears zero[0 .. nzero) (a captured
// frame's render counters: one launch fewer in the frame).
__global__ void update_window_kernel(tci_map m, uint32_t* __restrict__ base, int32_t L,
                                     const int32_t* __restrict__ rects, uint64_t* zero,
                                     int32_t nzero) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && (int32_t)threadIdx.x < nzero) zero[threadIdx.x] = 0;
  const int32_t* r = rects + 4 * blockIdx.x;
  const tci_level& w = m.wl[L];
  const int32_t x0 = max(r[0] - 1, 0), y0 = max(r[1] - 1, 0);
  const int32_t x1 = min(r[2], w.w - 1), y1 = min(r[3], w.h - 1);
  if (x0 > x1 || y0 > y1) return;
  const int32_t rw = x1 - x0 + 1;
  const int64_t n = (int64_t)rw * (y1 - y0 + 1);
  for (int64_t k = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.y * blockDim.x) {
    const int32_t i = x0 + (int32_t)(k % rw), j = y0 + (int32_t)(k / rw);
    base[tci_tile_index(w, i, j)] = window_entry(m, base, L, i, j);
  }
}

// One row of a block of level-s nodes: the combine (fmax, smin, smax) of
// nodes x0 <= x < x0 + S of row y, clipped to the level (level 0: the
// cells, as nodes), and with kMask the union of their occupancy masks; an
// empty combine if the row lies outside the block (in false).  The S loads
// are unrolled so that they are in flight together.
template <int S, bool kMask>
__device__ inline uint32_t reduce_row(const tci_map& m, const uint32_t* base, int32_t s,
                                      int32_t x0, int32_t y, bool in, uint64_t& mk) {
  const tci_level& c = m.lv[s];
  const int32_t nx = in ? min(S, c.w - x0) : 0;
  uint32_t v[S];
  uint2 mw[kMask ? S : 1];
#pragma unroll
  for (int dx = 0; dx < S; ++dx) {
    v[dx] = dx < nx ? base[tci_tile_index(c, x0 + dx, y)] : 0u;
    if constexpr (kMask) {
      mw[dx] = ((dx < nx) & (s > 0)) ? *reinterpret_cast<const uint2*>(
                                           base + tci_mask_index(m.mk[s], x0 + dx, y))
                                     : make_uint2(0u, 0u);
    }
  }
  uint32_t acc = 0u | (255u << 8);  // empty: fmax 0, smin 255, smax 0
  mk = 0;
#pragma unroll
  for (int dx = 0; dx < S; ++dx) {
    if (dx >= nx) continue;
    if (s == 0) {
      acc = node_merge(acc, cell_to_node(v[dx]));
      if constexpr (kMask) mk |= cell_mask(v[dx]);
    } else {
      acc = node_merge(acc, v[dx]);
      if constexpr (kMask) mk |= (uint64_t)mw[dx].x | ((uint64_t)mw[dx].y << 32);
    }
  }
  return acc;
}

// The items (nodes, or window entries) x0..x1, y0..y1 of one rectangle job
// of level L = s + k, each the combine of its S x S block of level-s nodes
// (S = 2^k for a node, 2^(k + 1) for a window entry's 2 x 2 node block).
// Both combines are associative, so an item of any level above s is the
// combine over its block of level-s nodes.  S consecutive lanes take one
// item, one block row each, and fold their rows together with cross-lane
// exchanges, so an item waits on one round of loads.
template <int S, bool kNode>
__device__ inline void group_job(const tci_map& m, uint32_t* base, int32_t s, int32_t L,
                                 int32_t x0, int32_t y0, int32_t x1, int32_t y1) {
  const int32_t k = L - s, rw = x1 - x0 + 1;
  const int64_t n = (int64_t)rw * (y1 - y0 + 1) * S;
  const tci_level& src = m.lv[s];
  // (blockDim.x is a multiple of S, so the S lanes of an item are aligned
  // and leave or stay in the loop together)
  for (int64_t q = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.y * blockDim.x) {
    const int64_t item = q / S;
    const int32_t row = (int32_t)(q % S);
    const int32_t i = x0 + (int32_t)(item % rw), j = y0 + (int32_t)(item / rw);
    const int32_t bx = i << k, by = (j << k) + row;
    uint64_t mk;
    uint32_t acc = reduce_row<S, kNode>(m, base, s, bx, by, by < src.h, mk);
#pragma unroll
    for (int o = 1; o < S; o <<= 1) {
      acc = node_merge(acc, (uint32_t)__shfl_xor((int)acc, o, S));
      if constexpr (kNode) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)mk, o, S);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(mk >> 32), o, S);
        mk |= (uint64_t)lo | ((uint64_t)hi << 32);
      }
    }
    if (row == 0) {
      if constexpr (kNode) {
        base[tci_tile_index(m.lv[L], i, j)] = acc;
        store_mask(m, base, L, i, j, mk);
      } else {
        base[tci_tile_index(m.wl[L], i, j)] = acc;
      }
    }
  }
}

// One launch per group of levels after edits, reading only level s, which
// the launch before finished (level 0, the cells, for the first group):
// blocks [0, (e - s) nr) recompute the dirty nodes and masks of levels
// s + 1 .. e; the blocks after them the dirty window entries of levels
// s .. e - 1, and with wtop of level e too (the top group).  Job j of either
// kind is level (first level) + j / nr, rectangle j % nr; the rectangles of
// level L (x0, y0, x1, y1 inclusive, in level-L node coordinates) are at
// rects + 4 (L stride + r).  Every output depends on level s alone, so no
// job waits for another, and a level's rectangles may overlap (two threads
// then write the same value).  Groups of at most 3 levels keep blocks at
// most 8 x 8 nodes for a node (k <= 3) and 16 x 16 for a window entry.  The
// first block also clears zero[0 .. nzero) (a captured frame's render
// counters, in the top group).
__global__ void update_group_kernel(tci_map m, uint32_t* __restrict__ base, int32_t s,
                                    int32_t e, int32_t wtop, const int32_t* __restrict__ rects,
                                    int32_t stride, int32_t nr, uint64_t* zero, int32_t nzero) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && (int32_t)threadIdx.x < nzero) zero[threadIdx.x] = 0;
  const int32_t nl = (e - s) * nr;
  const bool node_job = (int32_t)blockIdx.x < nl;
  const int32_t job = node_job ? (int32_t)blockIdx.x : (int32_t)blockIdx.x - nl;
  const int32_t L = (node_job ? s + 1 : s) + job / nr;
  const int32_t* r = rects + 4 * ((size_t)L * stride + job % nr);
  const int32_t k = L - s;
  int32_t x0 = r[0], y0 = r[1], x1 = r[2], y1 = r[3];
  if (node_job) {
    if (k == 1) group_job<2, true>(m, base, s, L, x0, y0, x1, y1);
    else if (k == 2) group_job<4, true>(m, base, s, L, x0, y0, x1, y1);
    else group_job<8, true>(m, base, s, L, x0, y0, x1, y1);
    return;
  }
  // entries x0 - 1 .. x1, y0 - 1 .. y1: those whose node block meets the
  // rectangle
  const tci_level& w = m.wl[L];
  x0 = max(x0 - 1, 0);
  y0 = max(y0 - 1, 0);
  x1 = min(x1, w.w - 1);
  y1 = min(y1, w.h - 1);
  if (x0 > x1 || y0 > y1) return;
  if (k == 0) group_job<2, false>(m, base, s, L, x0, y0, x1, y1);
  else if (k == 1) group_job<4, false>(m, base, s, L, x0, y0, x1, y1);
  else if (k == 2) group_job<8, false>(m, base, s, L, x0, y0, x1, y1);
  else group_job<16, false>(m, base, s, L, x0, y0, x1, y1);
}

__global__ void zero_u64_kernel(uint64_t* p, int32_t n) {
  int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
}

inline int32_t blocks_for(int64_t items, int32_t per, int32_t cap) {
  int64_t b = (items + per - 1) / per;
  if (b < 1) b = 1;
  return (int32_t)(b > cap ? cap : b);
}

}  // namespace

hipError_t tci_launch_repack(const uint8_t* planes, int32_t W, int32_t H,
                             uint32_t* base, tci_level l0, hipStream_t s) {
  int64_t words = (int64_t)l0.tiles_x * ((H + 7) >> 3) * 64;
  int32_t blocks = blocks_for(words, 256, 1 << 30);
  hipLaunchKernelGGL(repack_kernel, dim3(blocks), dim3(256), 0, s, planes, W,
                     H, base, l0);
  return hipGetLastError();
}

hipError_t tci_launch_build_level(const tci_map& m, uint32_t* base, int32_t L,
                                  hipStream_t s) {
  const tci_level& l = m.lv[L];
  int64_t words = (int64_t)l.tiles_x * ((l.h + 7) >> 3) * 64;
  int32_t blocks = blocks_for(words, 256, 1 << 30);
  hipLaunchKernelGGL(build_level_kernel, dim3(blocks), dim3(256), 0, s, m,
                     base, L);
  return hipGetLastError();
}

hipError_t tci_launch_edits(const tci_edit* edits, int32_t n, const int32_t* olap,
                            bool olap_all, const uint8_t* patch, uint32_t* base,
                            tci_level l0, int32_t W, int32_t H,
                            int32_t max_w, int32_t max_h, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int32_t gy = blocks_for((int64_t)max_w * max_h, 256, 64);
  hipLaunchKernelGGL(edits_kernel, dim3(n, gy), dim3(256), 0, s, edits, n, olap,
                     (int32_t)olap_all, patch, base, l0, W, H);
  return hipGetLastError();
}

hipError_t tci_launch_build_window(const tci_map& m, uint32_t* base, int32_t L,
                                   hipStream_t s) {
  const tci_level& w = m.wl[L];
  const int64_t words = (int64_t)w.tiles_x * ((w.h + 7) >> 3) * 64;
  const int32_t blocks = blocks_for(words, 256, 1 << 30);
  hipLaunchKernelGGL(build_window_kernel, dim3(blocks), dim3(256), 0, s, m, base, L);
  return hipGetLastError();
}

hipError_t tci_launch_update_window(const tci_map& m, uint32_t* base, int32_t L,
                                    const int32_t* rects, int32_t nrect, int32_t max_w,
                                    int32_t max_h, hipStream_t s, uint64_t* zero,
                                    int32_t nzero) {
  if (nrect <= 0) return nzero > 0 ? tci_launch_zero_u64(zero, nzero, s) : hipSuccess;
  const int32_t gy = blocks_for((int64_t)max_w * max_h, 256, 64);
  hipLaunchKernelGGL(update_window_kernel, dim3(nrect, gy), dim3(256), 0, s, m, base, L, rects,
                     zero, nzero);
  return hipGetLastError();
}

hipError_t tci_launch_update_group(const tci_map& m, uint32_t* base, int32_t s, int32_t e,
                                   bool wtop, const int32_t* rects, int32_t stride, int32_t nr,
                                   int64_t max_lanes, hipStream_t st, uint64_t* zero,
                                   int32_t nzero) {
  if (nr <= 0 || e <= s) return nzero > 0 ? tci_launch_zero_u64(zero, nzero, st) : hipSuccess;
  const int32_t gy = blocks_for(max_lanes, 256, 64);
  hipLaunchKernelGGL(update_group_kernel, dim3((2 * (e - s) + (wtop ? 1 : 0)) * nr, gy),
                     dim3(256), 0, st, m, base, s, e, (int32_t)wtop, rects, stride, nr, zero,
                     nzero);
  return hipGetLastError();
}

hipError_t tci_launch_zero_u64(uint64_t* p, int32_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s,
                     p, n);
  return hipGetLastError();
}
