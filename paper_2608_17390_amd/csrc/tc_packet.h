// Device helpers shared by the render kernels: view lookup, the pixel of a
// lane in an 8 x 8 packet, XCD-aware block order and the hit store.
#pragma once

#include "tc_internal.h"

namespace tcp {

// View containing packet p: largest v with pkt_prefix[v] <= p.
__device__ __forceinline__ int32_t find_view(const int64_t* pkt_prefix,
                                             int32_t nviews, int64_t p) {
  int32_t lo = 0, hi = nviews - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (pkt_prefix[mid] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Tile (the packet's block of 2^pw_log2 x 2^(6 - pw_log2) pixels) of packet
// `t` of a view; packets run row-major (order 0), column-major (order 1) or
// by the view's tile-row table (order 2).  A view holds at most about 2^22
// packets, so 32-bit arithmetic suffices.
__device__ __forceinline__ void packet_tile(const tci_view& v, int64_t t64,
                                            int32_t order, const int32_t* rows,
                                            int32_t& tx, int32_t& ty) {
  const uint32_t t = (uint32_t)t64;
  if (order == 2) {
    tx = (int32_t)(t % (uint32_t)v.tiles_x);
    ty = rows[v.rows_off + t / (uint32_t)v.tiles_x];
  } else if (order == 1) {
    const int32_t ph = 6 - v.pw_log2;
    const uint32_t tiles_y = (uint32_t)(v.h + (1 << ph) - 1) >> ph;
    tx = (int32_t)(t / tiles_y);
    ty = (int32_t)(t % tiles_y);
  } else {
    tx = (int32_t)(t % (uint32_t)v.tiles_x);
    ty = (int32_t)(t / (uint32_t)v.tiles_x);
  }
}

// Pixel of ray `k` (0..63, row-major in the packet's block) of packet `t`.
__device__ __forceinline__ void packet_pixel(const tci_view& v, int64_t t,
                                             int32_t k, int32_t order,
                                             const int32_t* rows,
                                             int32_t& px, int32_t& py) {
  int32_t tx, ty;
  packet_tile(v, t, order, rows, tx, ty);
  const int32_t pw = v.pw_log2;
  px = (tx << pw) + (k & ((1 << pw) - 1));
  py = (ty << (6 - pw)) + (k >> pw);
}

// Logical block of hardware block b.  Consecutive hardware blocks go to
// different XCDs (block r of a group of 8G runs on XCD r % 8); with G > 0
// each XCD gets G consecutive logical blocks of the group, so neighbouring
// packets share one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb, int32_t G) {
  if (G > 0) {
    const int64_t group = 8 * (int64_t)G;
    if (b < (nb / group) * group) {
      const int64_t g = b / group, r = b - g * group;
      b = g * group + (r & 7) * G + (r >> 3);
    }
  }
  return b;
}

__device__ __forceinline__ void store_hit(void* out, int64_t idx,
                                          uint32_t word, float depth) {
  uint2 h;
  h.x = word;
  h.y = __float_as_uint(depth);
  reinterpret_cast<uint2*>(out)[idx] = h;
}

}  // namespace tcp
