// Sampled height-field march: the paper's RAYMARCH (Section 3.1) as a
// render mode beside the exact walk, on the same tiled columns.
//
// Per pixel: the segment from the eye runs to the far limit (a distance
// along the ray) or to the plane z = 0, whichever comes first; `steps`
// interior points spaced uniformly over it are tested in order with the
// SOLID predicate (z <= F, or B <= z <= T on a column with an upper slab);
// the first solid sample and the sample before it (or the eye) bracket the
// crossing, and `bisect` halvings keep the solid end.  The segment's end
// point is never tested: a ray that meets no solid sample is a miss.
//
// Every quantity is an IEEE single computed one operation at a time (this
// file is compiled without floating-point contraction; division and square
// root are correctly rounded):
//   o = (float)O * 2^-16, d = (float)D, len = sqrt((dx*dx + dy*dy) + dz*dz)
//   t_end = far / len, and min(t_end, -oz / dz) when dz < 0
//   dt = t_end / (steps + 1), sample i at t = (float)i * dt
//   point(t) = o + t * d per component, midpoint (ta + tb) * 0.5
//   depth = tb * len
// so the solid/empty decision of every sample, and with it the hit word and
// depth, is reproducible bit for bit by any IEEE single implementation.
//
// MI355X mapping: one thread per pixel in 8x8 packets, as the exact walk.
// Sample positions do not depend on earlier loads, so each lane issues the
// column loads of kGroup samples before testing any of them (the test runs
// in order, so the first solid sample wins exactly as in a one-by-one
// march); the tiled layout keeps a packet's samples in few 256-byte tiles.
// Two exits skip samples that cannot be solid: a point left of, right of,
// before or behind the map while the ray moves away from it, and a point
// above height 255 while the ray does not descend -- rounding is monotone,
// so every later sample stays there.
#include "tc_internal.h"
#include "tc_packet.h"

namespace {

// 8x8 pixel packets (waves) per block: two (the same march time as four, as the render kernels use)
constexpr int32_t kPackets = 2;

constexpr uint32_t kMiss = 0xFFFFFFFFu;
constexpr int32_t kGroup = 8;

// SOLID on a packed column word (F | B << 8 | T << 16): 0 empty, 1 floor,
// 2 slab.
__device__ __forceinline__ int32_t solid(uint32_t col, float z) {
  const uint32_t F = col & 0xFFu, B = (col >> 8) & 0xFFu, T = (col >> 16) & 0xFFu;
  if (z <= (float)F) return 1;
  if (B > 0 && z >= (float)B && z <= (float)T) return 2;
  return 0;
}

struct fray {
  float ox, oy, oz, dx, dy, dz;
};

__device__ __forceinline__ void at(const fray& r, float t, float& x, float& y, float& z) {
  x = r.ox + t * r.dx;
  y = r.oy + t * r.dy;
  z = r.oz + t * r.dz;
}

__global__ __launch_bounds__(64 * kPackets) void march_kernel(
    tci_map m, const tci_view* __restrict__ views, int32_t nviews,
    const int64_t* __restrict__ pkt_prefix, int64_t npkt, void* out,
    tci_render_opts o) {
  const int64_t b = tcp::xcd_block(blockIdx.x, gridDim.x, o.xcd_remap);
  const int32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = b * kPackets + wave;
  if (p >= npkt) return;
  const int32_t vi = __builtin_amdgcn_readfirstlane(tcp::find_view(pkt_prefix, nviews, p));
  const tci_view& v = views[vi];
  int32_t px, py;
  tcp::packet_pixel(v, p - v.pkt_base, lane, o.tile_order, o.rows, px, py);
  if (px >= v.w || py >= v.h) return;

  const int64_t ka = 2 * (int64_t)px + 1, kb = 2 * (int64_t)py + 1;
  int32_t O[3], D[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    O[c] = (int32_t)((int64_t)v.o0[c] + ka * v.opx[c] + kb * v.opy[c]);
    D[c] = (int32_t)((int64_t)v.d0[c] + ka * v.dpx[c] + kb * v.dpy[c]);
  }
  uint32_t word = kMiss;
  float depth = __builtin_inff();
  int32_t reads = 0;
  const int32_t steps = o.march_steps;
  if (D[0] != 0 || D[1] != 0 || D[2] != 0) {
    fray r;
    r.ox = (float)O[0] * 0x1p-16f;
    r.oy = (float)O[1] * 0x1p-16f;
    r.oz = (float)O[2] * 0x1p-16f;
    r.dx = (float)D[0];
    r.dy = (float)D[1];
    r.dz = (float)D[2];
    const float len = sqrtf((r.dx * r.dx + r.dy * r.dy) + r.dz * r.dz);
    float t_end = o.march_far / len;
    if (r.dz < 0.0f) {
      const float t0 = -r.oz / r.dz;
      if (t0 < t_end) t_end = t0;
    }
    if (t_end > 0.0f) {
      const float dt = t_end / (float)(steps + 1);
      const float Wf = (float)m.W, Hf = (float)m.H;
      const float Wm1 = (float)(m.W - 1), Hm1 = (float)(m.H - 1);
      const tci_level l0 = m.lv[0];
      int32_t hit_i = 0;
      for (int32_t i0 = 1; i0 <= steps; i0 += kGroup) {
        uint32_t col[kGroup];
        float zs[kGroup];
        bool in[kGroup];
        float x = 0.0f, y = 0.0f, z = 0.0f;
#pragma unroll
        for (int32_t u = 0; u < kGroup; ++u) {
          const float t = (float)(i0 + u) * dt;
          at(r, t, x, y, z);
          zs[u] = z;
          in[u] = i0 + u <= steps && x >= 0.0f && x < Wf && y >= 0.0f && y < Hf;
          // clamped into the map so every lane loads without a branch;
          // the clamp leaves floor(x) unchanged for points over the map
          col[u] = m.base[tci_tile_index(l0, (int32_t)fminf(fmaxf(x, 0.0f), Wm1),
                                         (int32_t)fminf(fmaxf(y, 0.0f), Hm1))];
        }
        int32_t found = 0, tested = 0;
#pragma unroll
        for (int32_t u = 0; u < kGroup; ++u) {
          if (!found) {
            tested += in[u];
            if (in[u] && solid(col[u], zs[u])) found = i0 + u;
          }
        }
        reads += tested;
        if (found) {
          hit_i = found;
          break;
        }
        // (x, y, z) is the group's last sample
        if ((x < 0.0f && r.dx <= 0.0f) || (x >= Wf && r.dx >= 0.0f) ||
            (y < 0.0f && r.dy <= 0.0f) || (y >= Hf && r.dy >= 0.0f) ||
            (z > 255.0f && r.dz >= 0.0f))
          break;
      }
      if (hit_i) {
        float ta = (float)(hit_i - 1) * dt, tb = (float)hit_i * dt;
        float x, y, z;
        at(r, tb, x, y, z);
        int32_t cx = (int32_t)x, cy = (int32_t)y;
        int32_t layer = solid(m.base[tci_tile_index(l0, cx, cy)], z);
        for (int32_t k = 0; k < o.march_bisect; ++k) {
          const float tm = (ta + tb) * 0.5f;
          at(r, tm, x, y, z);
          const bool inm = x >= 0.0f && x < Wf && y >= 0.0f && y < Hf;
          reads += inm;
          const uint32_t c = m.base[tci_tile_index(l0, (int32_t)fminf(fmaxf(x, 0.0f), Wm1),
                                                   (int32_t)fminf(fmaxf(y, 0.0f), Hm1))];
          const int32_t s = inm ? solid(c, z) : 0;
          if (s) {
            tb = tm;
            cx = (int32_t)x;
            cy = (int32_t)y;
            layer = s;
          } else {
            ta = tm;
          }
        }
        word = (uint32_t)(cy * m.W + cx) | ((uint32_t)(layer == 2) << 30);
        depth = tb * len;
      }
    }
  }
  if (o.count) atomicAdd(o.count, (unsigned long long)reads);
  tcp::store_hit(out, v.out_base + (int64_t)py * v.w + px, word, depth);
}

}  // namespace

hipError_t tci_launch_march(const tci_map& m, const tci_view* views,
                            int32_t nviews, const int64_t* pkt_prefix,
                            int64_t npkt, void* out, const tci_render_opts& o,
                            hipStream_t s) {
  int64_t blocks = (npkt + kPackets - 1) / kPackets;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(march_kernel, dim3((uint32_t)blocks), dim3(64 * kPackets), 0, s, m,
                     views, nviews, pkt_prefix, npkt, out, o);
  return hipGetLastError();
}
