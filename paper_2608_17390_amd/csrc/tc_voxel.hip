// The voxel occupancy pyramid of the voxel-accelerated march (Section 3.2):
// build and incremental update.
//
// The finest level holds one bit per voxel of 2^v x 2^v cells by 2^vz
// height units: set when a column of the footprint has solid in the
// voxel's closed height range (a floor (-inf, F] meets [z0, z1] iff
// z0 <= F; a slab [B, T] iff B <= z1 and T >= z0).  Each higher level is
// the union of its eight children.  Levels are stored in Morton-ordered
// 8 x 8 x 8 tiles (tc_plan.h); one thread computes one 32-bit word, so no
// two threads write the same word and no atomics are needed.
//
// Parents from children: the 32 voxels of parent word w (Morton indices
// 32 w .. 32 w + 31 of the parent tile) have as children the 256 voxels of
// Morton indices 256 w .. 256 w + 255 of the 16 x 16 x 16 block of child
// voxels under the parent tile, because interleaving nests: the children
// of the parent at in-tile index m are 8 m .. 8 m + 7.  The block's index
// splits into a child tile (its top three bits, the tile's offset in the
// 2 x 2 x 2 block of child tiles) and an index in that tile, so those 256
// children are the 8 consecutive words 8 (w & 1) .. 8 (w & 1) + 7 of child
// tile (w >> 1), and parent bit j is set iff byte j of them is nonzero.
//
// After edits, the words of every tile over an edited rectangle are
// recomputed from the edited columns, level by level upward.
#include "tc_internal.h"

namespace {

// Voxel (x, y, z) of its tile -> in-tile Morton index (x, y, z < 8).
__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b)
    m |= (((x >> b) & 1u) << (3 * b)) | (((y >> b) & 1u) << (3 * b + 1)) |
         (((z >> b) & 1u) << (3 * b + 2));
  return m;
}

// Bit of finest-level voxel (X, Y, Z): a column of the footprint with solid
// in [Z 2^vz, (Z + 1) 2^vz].
__device__ __forceinline__ bool leaf_bit(const tci_map& m, const uint32_t* map, int32_t v_log2,
                                         int32_t vz_log2, int32_t X, int32_t Y, int32_t Z) {
  const int32_t z0 = Z << vz_log2, z1 = (Z + 1) << vz_log2;
  const int32_t x0 = X << v_log2, y0 = Y << v_log2;
  const int32_t x1 = min(x0 + (1 << v_log2), m.W), y1 = min(y0 + (1 << v_log2), m.H);
  for (int32_t y = y0; y < y1; ++y)
    for (int32_t x = x0; x < x1; ++x) {
      const uint32_t c = map[tci_tile_index(m.lv[0], x, y)];
      const int32_t F = c & 0xFF, B = (c >> 8) & 0xFF, T = (c >> 16) & 0xFF;
      if (z0 <= F || (B > 0 && B <= z1 && T >= z0)) return true;
    }
  return false;
}

// Word `w` (0..15) of tile (tx, ty, tz) of level k, from the columns (k = 0)
// or from level k - 1.
__device__ uint32_t voxel_word(const tci_map& m, const uint32_t* map, const tci_voxels& vx,
                               uint32_t* vox, int32_t k, int32_t tx, int32_t ty, int32_t tz,
                               int32_t w) {
  const tci_vlevel& l = vx.lv[k];
  uint32_t bits = 0;
  if (k == 0) {
    for (int32_t j = 0; j < 32; ++j) {
      const uint32_t mi = (uint32_t)(w * 32 + j);
      uint32_t x = 0, y = 0, z = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        x |= ((mi >> (3 * b)) & 1u) << b;
        y |= ((mi >> (3 * b + 1)) & 1u) << b;
        z |= ((mi >> (3 * b + 2)) & 1u) << b;
      }
      const int32_t X = tx * 8 + (int32_t)x, Y = ty * 8 + (int32_t)y, Z = tz * 8 + (int32_t)z;
      if (X < l.nx && Y < l.ny && Z < l.nz &&
          leaf_bit(m, map, vx.v_log2, vx.vz_log2, X, Y, Z))
        bits |= 1u << j;
    }
    return bits;
  }
  // the 2 x 2 x 2 child tiles under this tile; child tile (w >> 1) of them
  const tci_vlevel& c = vx.lv[k - 1];
  const int32_t o = w >> 1;
  const int32_t ctx = 2 * tx + (o & 1), cty = 2 * ty + ((o >> 1) & 1), ctz = 2 * tz + (o >> 2);
  if (ctx >= c.tiles_x || cty >= c.tiles_y || ctz >= c.tiles_z) return 0;
  const uint32_t* cw = vox + c.off + ((size_t)((ctz * c.tiles_y + cty) * c.tiles_x + ctx)) * 16 +
                       8 * (w & 1);
#pragma unroll
  for (int32_t q = 0; q < 8; ++q) {
    const uint32_t v = cw[q];
#pragma unroll
    for (int32_t b = 0; b < 4; ++b)
      if ((v >> (8 * b)) & 0xFFu) bits |= 1u << (4 * q + b);
  }
  return bits;
}

// One thread per word of the tiles [tx0, tx1] x [ty0, ty1] x (all tz) of
// level k; grid.y = rectangle (edit) index when rects is given, else the
// whole level.
__global__ void voxel_words_kernel(tci_map m, const uint32_t* __restrict__ map, tci_voxels vx,
                                   uint32_t* vox, int32_t k, const int32_t* __restrict__ rects) {
  const tci_vlevel& l = vx.lv[k];
  int32_t tx0 = 0, ty0 = 0, tx1 = l.tiles_x - 1, ty1 = l.tiles_y - 1;
  if (rects) {
    // the edit's clipped cell rectangle -> tiles of level k
    const int32_t* r = rects + 4 * blockIdx.y;
    const int32_t sh = vx.v_log2 + k + 3;
    tx0 = r[0] >> sh;
    ty0 = r[1] >> sh;
    tx1 = min(r[2] >> sh, l.tiles_x - 1);
    ty1 = min(r[3] >> sh, l.tiles_y - 1);
  }
  const int32_t ntx = tx1 - tx0 + 1, nty = ty1 - ty0 + 1;
  const int64_t words = (int64_t)ntx * nty * l.tiles_z * 16;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = (int32_t)(i & 15);
    int64_t t = i >> 4;
    const int32_t tx = tx0 + (int32_t)(t % ntx);
    t /= ntx;
    const int32_t ty = ty0 + (int32_t)(t % nty);
    const int32_t tz = (int32_t)(t / nty);
    vox[l.off + ((size_t)((tz * l.tiles_y + ty) * l.tiles_x + tx)) * 16 + w] =
        voxel_word(m, map, vx, vox, k, tx, ty, tz, w);
  }
}

}  // namespace

hipError_t tci_launch_voxel_level(const tci_map& m, const tci_voxels& vx, uint32_t* vox,
                                  int32_t k, const int32_t* rects, int32_t nrect,
                                  hipStream_t s) {
  if (rects && nrect <= 0) return hipSuccess;
  const tci_vlevel& l = vx.lv[k];
  const int64_t words = (int64_t)l.tiles_x * l.tiles_y * l.tiles_z * 16;
  int64_t blocks = (words + 255) / 256;
  if (rects) blocks = blocks < 64 ? blocks : 64;      // per rectangle: a few tiles
  blocks = blocks < 1 ? 1 : (blocks > (1 << 20) ? (1 << 20) : blocks);
  hipLaunchKernelGGL(voxel_words_kernel, dim3((uint32_t)blocks, rects ? nrect : 1), dim3(256), 0,
                     s, m, m.base, vx, vox, k, rects);
  return hipGetLastError();
}
