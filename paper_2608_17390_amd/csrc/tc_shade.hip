// Shading pass: the colour of every pixel from its exact hit record.
//
// The paper's methods share one palette, fog, diffuse lighting function and
// shadow term, and all but the mesh estimate a height-field gradient for the
// normal (Section 3); its resolve adds cave ambient (Section 3.5).  It gives
// no formulas; the steps here are this library's definition (spelled out in
// tc.h beside tc_shade_views):
//   * the exact hit time t = tn / td is rebuilt from the hit word's cell,
//     face and layer with the same integer formulas the walk resolves hits
//     with, and the hit point P = O + floor(tn * D / td) (fixed point) is
//     moved one unit out through the face;
//   * where the surface faces the light, a shadow ray from P along the light
//     direction is cast with the exact walk -- one secondary ray per pixel
//     instead of a sampled shadow map (the paper renders a 1024^2 shadow map
//     per frame, Section 4.3);
//   * the top-face normal is the gradient of the hit layer's surface over
//     the four neighbouring columns; walls and slab undersides use their own
//     axis; then diffuse + ambient (cave ambient for a floor under a slab),
//     a palette entry per layer and height, and linear fog.
// Single precision, one IEEE operation at a time in a fixed order (this file
// is compiled without floating-point contraction), so results are
// reproducible bit for bit.
#include "tc_walk.h"
#include "tc_packet.h"

namespace {

// 8x8 pixel packets (waves) per block: two (1 % faster shading than four)
constexpr int32_t kPackets = 2;

struct sh_map {
  const uint32_t* base;
  lvl_t l0;
  int32_t W, H;
};

__device__ __forceinline__ uint32_t column(const sh_map& m, int32_t x, int32_t y) {
  return m.base[m.l0.off + ((uint32_t)((y >> 3) * m.l0.tiles_x + (x >> 3)) << 6) +
                ((y & 7) << 3) + (x & 7)];
}

// Surface height of the hit layer at (x, y), clamped to the map: the floor
// top, or on the slab layer the slab top where the column has a slab (the
// hit column's top elsewhere).
__device__ __forceinline__ int32_t surf(const sh_map& m, int32_t x, int32_t y, int32_t layer,
                                        int32_t hT) {
  x = x < 0 ? 0 : (x >= m.W ? m.W - 1 : x);
  y = y < 0 ? 0 : (y >= m.H ? m.H - 1 : y);
  const uint32_t c = column(m, x, y);
  if (layer == 0) return (int32_t)(c & 0xFF);
  return ((c >> 8) & 0xFF) ? (int32_t)((c >> 16) & 0xFF) : hT;
}

// floor(a / b) for 0 < b < 2^24 and a quotient below 2^40 in magnitude: a
// double-precision estimate (a relative error below 2^-51, so less than one
// unit from the true quotient), then exact integer corrections.  A generic
// 64-bit division costs several times more.
__device__ __forceinline__ int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = (int64_t)floor((double)a / (double)b);
  int64_t r = a - q * b;
  while (r < 0) { --q; r += b; }
  while (r >= b) { ++q; r -= b; }
  return q;
}

// Does a ray from P along L meet any solid?  `reads` gains the nodes and
// cells the walk read.  kDir: the sign of L[2] (1 negative, 2 otherwise),
// the walk loop's specialisation.
template <int kDir, bool kCount>
__device__ __forceinline__ bool occluded(const tci_map& m, const lvl_t* lv, const int64_t P[3],
                                         const int32_t L[3], int32_t L0, int32_t Lmax,
                                         int32_t& reads) {
  ray_t s;
  s.Ox = P[0];
  s.Oy = P[1];
  s.Oz = P[2];
  s.Dx = L[0];
  s.Dy = L[1];
  s.Dz = L[2];
  s.ax = (uint32_t)(s.Dx < 0 ? -s.Dx : s.Dx);
  s.ay = (uint32_t)(s.Dy < 0 ? -s.Dy : s.Dy);
  if (s.Dx == 0 && s.Dy == 0) {
    uint32_t w;
    float d;
    trace_vertical(m, lv, s, w, d);
    reads += 1;
    return w != kMiss;
  }
  walk_t st;
  walk_idx_t k;
  walk_origin(s, k);
  walk_at_origin(s, L0, st);
  uint32_t col = 0;
  // the budget bounds the walk: a walk that uses it up (never expected)
  // counts as occluded, as a hit does
  const int32_t res = walk_steps<false, false, false, kDir>(m, lv, s, k, st, Lmax, kIterCap + 1,
                                                           col, 0, 0, 0, 0, nullptr, kCount);
  if (kCount) reads += st.reads;
  return res != kMissed;
}

// One kernel per sign of the light's vertical direction: every shadow ray
// of a launch shares it, so the walk loop is specialised to it; and one
// with read counting (o.count) and one without.
template <int kDir, bool kCount>
__global__ __launch_bounds__(64 * kPackets) void shade_kernel(
    tci_map m, const tci_view* __restrict__ views, int32_t nviews,
    const int64_t* __restrict__ pkt_prefix, int64_t npkt, const uint2* __restrict__ hits,
    uint32_t* __restrict__ rgba, tci_shade sh, tci_render_opts o) {
  __shared__ lvl_t lv[TCI_MAX_LEVELS];
  load_levels(m, lv);
  const int64_t b = tcp::xcd_block(blockIdx.x, gridDim.x, o.xcd_remap);
  const int32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = b * kPackets + wave;
  if (p >= npkt) return;
  const int32_t vi = __builtin_amdgcn_readfirstlane(tcp::find_view(pkt_prefix, nviews, p));
  const tci_view& v = views[vi];
  int32_t px, py;
  tcp::packet_pixel(v, p - v.pkt_base, lane, o.tile_order, o.rows, px, py);
  if (px >= v.w || py >= v.h) return;
  const int64_t idx = v.out_base + (int64_t)py * v.w + px;
  const uint32_t word = hits[idx].x;
  const uint32_t cell = word & 0x07FFFFFFu;
  const int32_t face = (int32_t)((word >> 27) & 7);
  // a miss, or a record that names no cell of the map or no face of the
  // exact walk (not produced by an exact render), is shaded as sky
  if (word == kMiss || cell >= (uint32_t)m.W * (uint32_t)m.H || face == 0) {
    rgba[idx] = sh.sky_rgba;
    return;
  }
  int32_t reads = 1;   // the hit column
  ray_t r;
  pixel_ray(v, px, py, r);
  const int64_t O[3] = {r.Ox, r.Oy, r.Oz};
  const int32_t D[3] = {r.Dx, r.Dy, r.Dz};
  const sh_map sm{m.base, lv[0], m.W, m.H};
  const int32_t k = (int32_t)cell;
  const int32_t x = k % m.W, y = k / m.W;
  const int32_t layer = (int32_t)((word >> 30) & 1);
  const uint32_t c = column(sm, x, y);
  const int32_t F = (int32_t)(c & 0xFF), B = (int32_t)((c >> 8) & 0xFF),
                T = (int32_t)((c >> 16) & 0xFF);
  const int32_t h = layer ? T : F;
  // exact hit time, and the outward axis of the face
  int64_t tn, td;
  int32_t nudge[3] = {0, 0, 0};
  switch (face) {
    case kTop: tn = O[2] - ((int64_t)h << 16); td = -(int64_t)D[2]; nudge[2] = 1; break;
    case kUnder: tn = ((int64_t)B << 16) - O[2]; td = D[2]; nudge[2] = -1; break;
    case kWmx: tn = ((int64_t)x << 16) - O[0]; td = D[0]; nudge[0] = -1; break;
    case kWpx: tn = O[0] - ((int64_t)(x + 1) << 16); td = -(int64_t)D[0]; nudge[0] = 1; break;
    case kWmy: tn = ((int64_t)y << 16) - O[1]; td = D[1]; nudge[1] = -1; break;
    case kWpy: tn = O[1] - ((int64_t)(y + 1) << 16); td = -(int64_t)D[1]; nudge[1] = 1; break;
    default: tn = 0; td = 1; break;
  }
  if (td <= 0) {   // a face the ray cannot have crossed: not an exact hit
    rgba[idx] = sh.sky_rgba;
    return;
  }
  const float fdx = (float)D[0], fdy = (float)D[1], fdz = (float)D[2];
  const float len = sqrtf((fdx * fdx + fdy * fdy) + fdz * fdz);
  const float q = (float)((double)tn / (double)td);
  const float dist = q * len * (1.0f / 65536.0f);
  float n0, n1, n2;
  if (face == kTop) {
    reads += 4;        // the four neighbouring columns
    const float gx = (float)(surf(sm, x + 1, y, layer, T) - surf(sm, x - 1, y, layer, T)) * 0.5f;
    const float gy = (float)(surf(sm, x, y + 1, layer, T) - surf(sm, x, y - 1, layer, T)) * 0.5f;
    const float nl = sqrtf((gx * gx + gy * gy) + 1.0f);
    n0 = -gx / nl;
    n1 = -gy / nl;
    n2 = 1.0f / nl;
  } else if (face == kUnder) {
    n0 = 0.0f;
    n1 = 0.0f;
    n2 = -1.0f;
  } else if (face >= kWmx && face <= kWpy) {
    n0 = (float)nudge[0];
    n1 = (float)nudge[1];
    n2 = 0.0f;
  } else {
    n0 = 0.0f;
    n1 = 0.0f;
    n2 = 1.0f;
  }
  const float Lx = (float)sh.light[0], Ly = (float)sh.light[1], Lz = (float)sh.light[2];
  const float ll = sqrtf((Lx * Lx + Ly * Ly) + Lz * Lz);
  const float lx = Lx / ll, ly = Ly / ll, lz = Lz / ll;
  const float lambert = (n0 * lx + n1 * ly) + n2 * lz;
  bool lit = false;
  if (face != kInside && lambert > 0.0f) {
    int64_t P[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      P[cc] = O[cc] + floordiv(tn * (int64_t)D[cc], td) + nudge[cc];
    const int32_t top = m.top;
    lit = !occluded<kDir, kCount>(m, lv, P, sh.light, clamp_level(o.start_level, top),
                    clamp_level(o.max_level, top), reads);
  }
  const float amb = (layer == 0 && B > 0) ? sh.cave_ambient : sh.ambient;
  const float I = fminf(amb + (lit ? lambert : 0.0f), 1.0f);
  const uint32_t albedo = sh.palette[layer * 256 + h];
  const float f = fminf(dist / sh.fog_far, 1.0f);
  uint32_t out = 0xFF000000u;
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    const float a = (float)((albedo >> (8 * cc)) & 0xFF);
    const float fogc = (float)((sh.fog_rgba >> (8 * cc)) & 0xFF);
    float val = a * I;
    val = val + (fogc - val) * f;
    out |= (uint32_t)(val + 0.5f) << (8 * cc);
  }
  rgba[idx] = out;
  if (kCount) atomicAdd(o.count, (unsigned long long)reads);
}

}  // namespace

hipError_t tci_launch_shade(const tci_map& m, const tci_view* views, int32_t nviews,
                            const int64_t* pkt_prefix, int64_t npkt, const void* hits,
                            uint32_t* rgba, const tci_shade& sh, const tci_render_opts& o,
                            hipStream_t s) {
  int64_t blocks = (npkt + kPackets - 1) / kPackets;
  if (blocks < 1) return hipSuccess;
  const bool c = o.count != nullptr;
  auto kern = sh.light[2] < 0 ? (c ? shade_kernel<1, true> : shade_kernel<1, false>)
                              : (c ? shade_kernel<2, true> : shade_kernel<2, false>);
  hipLaunchKernelGGL(kern, dim3((uint32_t)blocks), dim3(64 * kPackets), 0, s, m, views, nviews, pkt_prefix,
                     npkt, (const uint2*)hits, rgba, sh, o);
  return hipGetLastError();
}
