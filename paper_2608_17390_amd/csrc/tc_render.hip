// Ray casting kernels.
//
// Each pixel's ray walks the exact cell sequence of a 2D digital
// differential analyser over the map (the exact limit of the paper's
// per-pixel march, Section 3.1, with the cell-boundary convention fixed:
// start in floor(O / S), closed per-cell parameter intervals, x before y on
// simultaneous crossings).  A cell is hit when the ray's height range over
// its interval meets the column's solid set (z <= F, or B <= z <= T when
// B > 0: the SOLID predicate of Section 3.1).
//
// Acceleration: the walk runs at pyramid level L (a node = 2^L x 2^L
// cells).  The same interval test against a node's (fmax, smin, smax)
// decides whether the ray may meet solid inside the node before leaving
// it; if not, the ray jumps to the node exit in one step -- the skip of the
// paper's hierarchical voxel march (Section 3.2), on a 2D per-layer min/max
// pyramid instead of a 3D occupancy grid.  The jump reproduces the flat
// walk exactly: it advances the x and y crossing counters by the number of
// crossings the flat walk would take, so the state after a skip equals the
// flat walk's state on entering the same cell.
//
// Arithmetic.  With |Dx|, |Dy| = ax, ay and nx, ny the distances (in S
// units) to the next x and y boundaries:
//   crossing keys  Kx = nx * ay,  Ky = ny * ax   (time * ax * ay); the next
//                  crossing is x iff Kx <= Ky;
//   heights        Zx = Oz * ax + nx * Dz  is z (S units) at the next x
//                  crossing scaled by ax, likewise Zy; z <= h*S at that
//                  crossing iff Zx <= h * S * ax.
// All quantities fit in int64 for |O| < 2^31 and |D| < 2^23; products of a
// height (8 bits) or a crossing count (< 2^24) with a direction component
// (< 2^23) are 24-bit multiplies.  Depth is computed once per ray in double
// and rounded to float.
#include "tc_internal.h"

namespace {

constexpr uint32_t kMiss = 0xFFFFFFFFu;
constexpr uint32_t kStuck = 0xFFFFFFFEu;   // iteration cap reached (never
                                           // expected; guards against hangs)
// Key of a crossing that never happens (axis with zero direction).  Real
// keys stay below 2^58 and a node adds at most 2^54, so no sum overflows.
constexpr int64_t kNever = (int64_t)1 << 62;
constexpr int32_t kIterCap = 1 << 22;

enum : int32_t { kTop = 1, kUnder = 2, kWmx = 3, kWpx = 4, kWmy = 5,
                 kWpy = 6, kInside = 7 };
enum : int32_t { kWalking = 0, kHitCell = 1, kMissed = 2, kCapped = 3 };

struct lvl_t {
  uint32_t off;
  int32_t w, h, tiles_x;
};

// a * b for a < 2^24, b < 2^24 as a 48-bit product: two full-rate 24-bit
// multiplies instead of a quarter-rate 64-bit one.
__device__ __forceinline__ uint64_t mul48(uint32_t a, uint32_t b) {
  uint32_t lo, hi;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(lo) : "v"(a), "v"(b));
  asm("v_mul_hi_u32_u24 %0, %1, %2" : "=v"(hi) : "v"(a), "v"(b));
  return ((uint64_t)hi << 32) | lo;
}
// a * b for 0 <= a < 2^23 and |b| < 2^23, signed 48-bit product.
__device__ __forceinline__ int64_t smul48(int32_t a, int32_t b) {
  int32_t lo, hi;
  asm("v_mul_i32_i24 %0, %1, %2" : "=v"(lo) : "v"(a), "v"(b));
  asm("v_mul_hi_i32_i24 %0, %1, %2" : "=v"(hi) : "v"(a), "v"(b));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// h * S * d for a height h <= 255 and d < 2^23
__device__ __forceinline__ int64_t hS(uint32_t h, uint32_t d) {
  return (int64_t)((uint64_t)__umul24(h, d) << 16);
}

struct ray_t {
  int64_t Ox, Oy, Oz;
  int32_t Dx, Dy, Dz;
  uint32_t ax, ay;
};

struct walk_t {
  int32_t cx, cy;
  int64_t Kx, Ky;     // keys of the next x / y crossing
  int64_t Zx, Zy;     // scaled z at the next x / y crossing
  int64_t Zin;        // scaled z at entry of the current cell
  uint32_t Din;       // scale of Zin (1 at the origin, else ax or ay)
  int32_t entry;      // face crossed on entry (kInside for the first cell)
  int32_t L;          // current pyramid level
  int32_t iters;
  int32_t reads;      // nodes and cells read from memory
};

__device__ __forceinline__ void pixel_ray(const tci_view& v, int32_t px,
                                          int32_t py, ray_t& r) {
  int64_t a = 2 * (int64_t)px + 1, b = 2 * (int64_t)py + 1;
  r.Ox = (int64_t)v.o0[0] + a * v.opx[0] + b * v.opy[0];
  r.Oy = (int64_t)v.o0[1] + a * v.opx[1] + b * v.opy[1];
  r.Oz = (int64_t)v.o0[2] + a * v.opx[2] + b * v.opy[2];
  r.Dx = (int32_t)((int64_t)v.d0[0] + a * v.dpx[0] + b * v.dpy[0]);
  r.Dy = (int32_t)((int64_t)v.d0[1] + a * v.dpx[1] + b * v.dpy[1]);
  r.Dz = (int32_t)((int64_t)v.d0[2] + a * v.dpx[2] + b * v.dpy[2]);
  r.ax = (uint32_t)(r.Dx < 0 ? -r.Dx : r.Dx);
  r.ay = (uint32_t)(r.Dy < 0 ? -r.Dy : r.Dy);
}

__device__ __forceinline__ void walk_init(const ray_t& r, int32_t L0,
                                          walk_t& s) {
  s.cx = (int32_t)(r.Ox >> 16);
  s.cy = (int32_t)(r.Oy >> 16);
  int64_t nx = r.Dx > 0 ? ((int64_t)(s.cx + 1) << 16) - r.Ox
                        : r.Ox - ((int64_t)s.cx << 16);
  int64_t ny = r.Dy > 0 ? ((int64_t)(s.cy + 1) << 16) - r.Oy
                        : r.Oy - ((int64_t)s.cy << 16);
  s.Kx = r.Dx != 0 ? nx * (int64_t)r.ay : kNever;
  s.Ky = r.Dy != 0 ? ny * (int64_t)r.ax : kNever;
  s.Zx = r.Oz * (int64_t)r.ax + nx * (int64_t)r.Dz;
  s.Zy = r.Oz * (int64_t)r.ay + ny * (int64_t)r.Dz;
  s.Zin = r.Oz;
  s.Din = 1;
  s.entry = kInside;
  s.L = L0;
  s.iters = 0;
  s.reads = 0;
}

__device__ __forceinline__ void set_hit(const ray_t& r, int32_t W, int32_t x,
                                        int32_t y, int32_t face,
                                        int32_t layer, int64_t tn,
                                        int64_t td, uint32_t& word,
                                        float& depth) {
  word = (uint32_t)(y * W + x) | ((uint32_t)face << 27) |
         ((uint32_t)layer << 30);
  double len = sqrt((double)r.Dx * r.Dx + (double)r.Dy * r.Dy +
                    (double)r.Dz * r.Dz);
  depth = tn == 0 ? 0.0f
                  : (float)(((double)tn / (double)td) * len / 65536.0);
}

// First hit inside the current cell (packed column v), given that the ray's
// height range over the cell meets solid.
__device__ __forceinline__ void resolve_hit(const ray_t& r, const walk_t& s,
                                            int32_t W, uint32_t v,
                                            uint32_t& word, float& depth) {
  uint32_t F = v & 0xFF, B = (v >> 8) & 0xFF, T = (v >> 16) & 0xFF;
  bool in_floor = s.Zin <= hS(F, s.Din);
  bool in_slab = B != 0 && s.Zin >= hS(B, s.Din) && s.Zin <= hS(T, s.Din);
  int32_t face, layer;
  int64_t tn, td;
  if (in_floor || in_slab) {
    face = s.entry;
    layer = in_floor ? 0 : 1;
    switch (face) {
      case kWmx: tn = ((int64_t)s.cx << 16) - r.Ox; td = r.ax; break;
      case kWpx: tn = r.Ox - ((int64_t)(s.cx + 1) << 16); td = r.ax; break;
      case kWmy: tn = ((int64_t)s.cy << 16) - r.Oy; td = r.ay; break;
      case kWpy: tn = r.Oy - ((int64_t)(s.cy + 1) << 16); td = r.ay; break;
      default: tn = 0; td = 1; break;
    }
  } else if (r.Dz < 0) {
    bool above = B != 0 && s.Zin > hS(T, s.Din);
    uint32_t tgt = above ? T : F;
    face = kTop;
    layer = above ? 1 : 0;
    tn = r.Oz - ((int64_t)tgt << 16);
    td = -(int64_t)r.Dz;
  } else {
    face = kUnder;
    layer = 1;
    tn = ((int64_t)B << 16) - r.Oz;
    td = r.Dz;
  }
  set_hit(r, W, s.cx, s.cy, face, layer, tn, td, word, depth);
}

// Hit record of a finished walk.
__device__ __forceinline__ void finish(const ray_t& r, const walk_t& s,
                                       int32_t W, int32_t state, uint32_t v,
                                       uint32_t& word, float& depth) {
  if (state == kHitCell) {
    resolve_hit(r, s, W, v, word, depth);
  } else if (state == kCapped) {
    word = kStuck;
    depth = __builtin_nanf("");
  } else {
    word = kMiss;
    depth = __builtin_inff();
  }
}

// Vertical ray (Dx = Dy = 0): only the start column can be met.
__device__ __forceinline__ void trace_vertical(const tci_map& m,
                                               const lvl_t* lv,
                                               const ray_t& r, uint32_t& word,
                                               float& depth) {
  word = kMiss;
  depth = __builtin_inff();
  if (r.Dz == 0) return;
  int32_t cx = (int32_t)(r.Ox >> 16), cy = (int32_t)(r.Oy >> 16);
  if ((uint32_t)cx >= (uint32_t)m.W || (uint32_t)cy >= (uint32_t)m.H) return;
  const lvl_t l = lv[0];
  uint32_t v = m.base[l.off + ((uint32_t)((cy >> 3) * l.tiles_x + (cx >> 3)) << 6) +
                      ((cy & 7) << 3) + (cx & 7)];
  uint32_t B = (v >> 8) & 0xFF, F = v & 0xFF, T = (v >> 16) & 0xFF;
  walk_t s;
  s.cx = cx; s.cy = cy; s.Zin = r.Oz; s.Din = 1; s.entry = kInside;
  bool in_floor = r.Oz <= ((int64_t)F << 16);
  bool in_slab = B != 0 && r.Oz >= ((int64_t)B << 16) && r.Oz <= ((int64_t)T << 16);
  if (in_floor || in_slab || r.Dz < 0 || (B != 0 && r.Oz < ((int64_t)B << 16)))
    resolve_hit(r, s, m.W, v, word, depth);
}

// Number of terms K + j*(a<<16), j >= 0, strictly below E (E, K < 2^62;
// the count is < 2^15 when E is a node exit).  Float estimate of the
// quotient, then one exact correction.
__device__ __forceinline__ int32_t count_below(int64_t E, int64_t K,
                                               uint32_t a) {
  if (E <= K) return 0;
  const int64_t n = E - K - 1;             // count = floor(n / step) + 1
  const int64_t step = (int64_t)a << 16;
  const float nf = (float)(uint32_t)(n >> 32) * 4294967296.0f +
                   (float)(uint32_t)n;
  int32_t q = (int32_t)(nf * __builtin_amdgcn_rcpf((float)a * 65536.0f));
  q = q < 0 ? 0 : q;
  const int64_t p = (int64_t)(mul48((uint32_t)q, a) << 16);
  q += (p > n) ? -1 : ((n - p >= step) ? 1 : 0);
  return q + 1;
}

// Advance the walk by up to `budget` iterations.  Returns kWalking if the
// budget ran out, else the final state; on kHitCell, `col` holds the
// column of the current cell.
template <bool kFlat>
__device__ __forceinline__ int32_t walk_steps(const tci_map& m,
                                              const lvl_t* lv, const ray_t& r,
                                              walk_t& s, int32_t max_level,
                                              int32_t budget, uint32_t& col) {
  const bool desc = r.Dz < 0;
  const int64_t SZ = (int64_t)r.Dz << 16;
  for (int32_t it = 0; it < budget; ++it) {
    if (++s.iters > kIterCap) return kCapped;
    const int32_t L = kFlat ? 0 : s.L;
    const lvl_t l = lv[L];
    const int32_t ni = s.cx >> L, nj = s.cy >> L;
    const bool inmap = (uint32_t)ni < (uint32_t)l.w && (uint32_t)nj < (uint32_t)l.h;
    uint32_t v = 0;
    s.reads += inmap ? 1 : 0;
    if (inmap)
      v = m.base[l.off + ((__umul24((uint32_t)nj >> 3, (uint32_t)l.tiles_x) +
                           ((uint32_t)ni >> 3)) << 6) +
                 ((nj & 7) << 3) + (ni & 7)];
    // crossings before the node's far face on each axis
    int32_t kxm1 = 0, kym1 = 0;
    int64_t Kxe = s.Kx, Kye = s.Ky;
    if (!kFlat) {
      kxm1 = r.Dx > 0 ? ((ni + 1) << L) - 1 - s.cx : s.cx - (ni << L);
      kym1 = r.Dy > 0 ? ((nj + 1) << L) - 1 - s.cy : s.cy - (nj << L);
      Kxe += (int64_t)(mul48((uint32_t)kxm1, r.ay) << 16);
      Kye += (int64_t)(mul48((uint32_t)kym1, r.ax) << 16);
    }
    const bool ex = Kxe <= Kye;               // leave through an x face
    const int32_t km1 = ex ? kxm1 : kym1;
    int64_t Ze = ex ? s.Zx : s.Zy;
    if (!kFlat) Ze += smul48(km1, r.Dz) << 16;
    const uint32_t De = ex ? r.ax : r.ay;
    bool occ = false;
    if (inmap) {
      const int64_t Zlo = desc ? Ze : s.Zin;
      const uint32_t Dlo = desc ? De : s.Din;
      const int64_t Zhi = desc ? s.Zin : Ze;
      const uint32_t Dhi = desc ? s.Din : De;
      const uint32_t a = v & 0xFF, b = (v >> 8) & 0xFF, c = (v >> 16) & 0xFF;
      occ = (Zlo <= hS(a, Dlo)) || ((Zlo <= hS(c, Dlo)) && (Zhi >= hS(b, Dhi)));
    }
    if (occ) {
      if (L == 0) {
        col = v;
        return kHitCell;
      }
      s.L = L - 1;
      continue;
    }
    // jump to the node exit: km1 + 1 crossings on the exit axis and, on
    // the other axis, those strictly before it (x first on ties)
    int32_t ko = 0;
    if (!kFlat && L > 0)
      ko = ex ? count_below(Kxe, s.Ky, r.ax) : count_below(Kye + 1, s.Kx, r.ay);
    const int32_t kx = ex ? km1 + 1 : ko;
    const int32_t ky = ex ? ko : km1 + 1;
    // exit axis: one step past its exit crossing; other axis: ko steps
    if (ex) {
      s.Kx = Kxe + ((int64_t)r.ay << 16);
      s.Zx = Ze + SZ;
      if (!kFlat && ko) {
        s.Ky += (int64_t)(mul48((uint32_t)ko, r.ax) << 16);
        s.Zy += smul48(ko, r.Dz) << 16;
      }
    } else {
      s.Ky = Kye + ((int64_t)r.ax << 16);
      s.Zy = Ze + SZ;
      if (!kFlat && ko) {
        s.Kx += (int64_t)(mul48((uint32_t)ko, r.ay) << 16);
        s.Zx += smul48(ko, r.Dz) << 16;
      }
    }
    const int32_t pcx = s.cx, pcy = s.cy;
    s.cx += r.Dx > 0 ? kx : -kx;
    s.cy += r.Dy > 0 ? ky : -ky;
    s.Zin = Ze;
    s.Din = De;
    s.entry = ex ? (r.Dx > 0 ? kWmx : kWpx) : (r.Dy > 0 ? kWmy : kWpy);
    // the ray cannot come back into the map, or is above all solid
    const bool away = (s.cx < 0 && r.Dx <= 0) || (s.cx >= m.W && r.Dx >= 0) ||
                      (s.cy < 0 && r.Dy <= 0) || (s.cy >= m.H && r.Dy >= 0);
    const bool above = r.Dz >= 0 && s.Zin > hS(255, s.Din);
    if (away || above) return kMissed;
    // go up one level when the jump left the parent node
    if (!kFlat && L < max_level && (((pcx ^ s.cx) | (pcy ^ s.cy)) >> (L + 1)) != 0)
      s.L = L + 1;
  }
  return kWalking;
}

__device__ __forceinline__ void load_levels(const tci_map& m, lvl_t* lv) {
  if (threadIdx.x < TCI_MAX_LEVELS) {
    const tci_level& l = m.lv[threadIdx.x];
    lv[threadIdx.x] = lvl_t{l.off, l.w, l.h, l.tiles_x};
  }
  __syncthreads();
}

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

// Pixel of ray `k` (0..63, row-major in an 8x8 block) of packet `t` of a
// view; packets run row-major (order 0) or column-major (order 1).
__device__ __forceinline__ void packet_pixel(const tci_view& v, int64_t t,
                                             int32_t k, int32_t order,
                                             int32_t& px, int32_t& py) {
  int32_t tx, ty;
  if (order) {
    const int32_t tiles_y = (v.h + 7) >> 3;
    tx = (int32_t)(t / tiles_y);
    ty = (int32_t)(t % tiles_y);
  } else {
    tx = (int32_t)(t % v.tiles_x);
    ty = (int32_t)(t / v.tiles_x);
  }
  px = tx * 8 + (k & 7);
  py = ty * 8 + (k >> 3);
}

__device__ __forceinline__ void store_hit(void* out, int64_t idx,
                                          uint32_t word, float depth) {
  uint2 h;
  h.x = word;
  h.y = __float_as_uint(depth);
  reinterpret_cast<uint2*>(out)[idx] = h;
}

__device__ __forceinline__ int32_t clamp_level(int32_t v, int32_t top) {
  return v < 0 ? 0 : (v > top ? top : v);
}

// One thread per pixel; a wave casts one 8x8 pixel packet.
template <bool kFlat>
__global__ __launch_bounds__(256) void render_kernel(
    tci_map m, const tci_view* __restrict__ views, int32_t nviews,
    const int64_t* __restrict__ pkt_prefix, int64_t npkt, void* out,
    tci_render_opts o) {
  __shared__ lvl_t lv[TCI_MAX_LEVELS];
  load_levels(m, lv);
  // XCD-aware order: consecutive hardware blocks go to different XCDs, so
  // hand each XCD a contiguous range of packets to share its L2.
  int64_t nb = gridDim.x, b = blockIdx.x;
  if (o.xcd_remap > 0) {
    // hardware block r of a group of 8G runs on XCD r % 8; give each XCD
    // G consecutive logical blocks of the group
    const int64_t G = o.xcd_remap, group = 8 * G;
    if (b < (nb / group) * group) {
      const int64_t g = b / group, r = b - g * group;
      b = g * group + (r & 7) * G + (r >> 3);
    }
  }
  const int32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = b * 4 + wave;
  if (p >= npkt) return;
  const int32_t vi = __builtin_amdgcn_readfirstlane(find_view(pkt_prefix, nviews, p));
  const tci_view& v = views[vi];
  int32_t px, py;
  packet_pixel(v, p - v.pkt_base, lane, o.tile_order, px, py);
  if (px >= v.w || py >= v.h) return;
  ray_t r;
  pixel_ray(v, px, py, r);
  uint32_t word;
  float depth;
  if (r.Dx == 0 && r.Dy == 0) {
    trace_vertical(m, lv, r, word, depth);
  } else {
    walk_t s;
    const int32_t top = kFlat ? 0 : m.top;
    walk_init(r, kFlat ? 0 : clamp_level(o.start_level, top), s);
    uint32_t col = 0;
    const int32_t st = walk_steps<kFlat>(m, lv, r, s,
                                         kFlat ? 0 : clamp_level(o.max_level, top),
                                         kIterCap + 1, col);
    finish(r, s, m.W, st, col, word, depth);
    if (o.count) atomicAdd(o.count, (unsigned long long)s.reads);
  }
  store_hit(out, v.out_base + (int64_t)py * v.w + px, word, depth);
}

// Persistent waves.  Each wave keeps 64 rays in flight; when at least
// refill_min lanes are idle it hands them the next rays of its current
// 8x8 packet and, when that runs out, pops a new packet from the global
// queue counter.  Every wave leaves the loop once the queue is drained and
// all its lanes are idle.
__global__ __launch_bounds__(256) void render_persistent_kernel(
    tci_map m, const tci_view* __restrict__ views, int32_t nviews,
    const int64_t* __restrict__ pkt_prefix, int64_t npkt, void* out,
    uint64_t* __restrict__ counter, tci_render_opts o) {
  __shared__ lvl_t lv[TCI_MAX_LEVELS];
  load_levels(m, lv);
  const int32_t lane = threadIdx.x & 63;
  const int32_t top = m.top;
  const int32_t L0 = clamp_level(o.start_level, top);
  const int32_t Lmax = clamp_level(o.max_level, top);
  const int32_t refill_min = o.refill_min < 1 ? 1 : (o.refill_min > 64 ? 64 : o.refill_min);
  const int32_t iters = o.refill_iters < 1 ? 1 : o.refill_iters;

  int64_t pkt = -1;      // current packet (wave-uniform)
  int32_t taken = 64;    // rays of the current packet already handed out
  bool drained = false;  // queue exhausted (wave-uniform)
  bool active = false;
  ray_t r;
  walk_t s;
  int64_t out_idx = 0;
  for (;;) {
    const uint64_t idle = __ballot(!active);
    const int32_t nidle = __popcll(idle);
    if (!drained && (nidle >= refill_min)) {
      const int32_t rank = __builtin_amdgcn_mbcnt_hi(
          (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0));
      const int32_t remaining = 64 - taken;
      int64_t next = -1;
      if (nidle > remaining) {
        uint64_t q = 0;
        if (lane == 0) q = atomicAdd((unsigned long long*)counter, 1ull);
        next = (int64_t)__shfl(q, 0);
        if (next >= npkt) drained = true;
      }
      if (!active) {
        int64_t mypkt;
        int32_t myray;
        if (rank < remaining) { mypkt = pkt; myray = taken + rank; }
        else { mypkt = next; myray = rank - remaining; }
        if (mypkt >= 0 && mypkt < npkt && myray < 64) {
          const int32_t vi = find_view(pkt_prefix, nviews, mypkt);
          const tci_view& v = views[vi];
          int32_t px, py;
          packet_pixel(v, mypkt - v.pkt_base, myray, o.tile_order, px, py);
          if (px < v.w && py < v.h) {
            pixel_ray(v, px, py, r);
            out_idx = v.out_base + (int64_t)py * v.w + px;
            if (r.Dx == 0 && r.Dy == 0) {
              uint32_t word;
              float depth;
              trace_vertical(m, lv, r, word, depth);
              store_hit(out, out_idx, word, depth);
            } else {
              walk_init(r, L0, s);
              active = true;
            }
          }
        }
      }
      if (nidle > remaining) {
        if (next >= 0 && next < npkt) { pkt = next; taken = nidle - remaining; }
        else { taken = 64; }
      } else {
        taken += nidle;
      }
    }
    if (drained && __ballot(active) == 0) break;
    int32_t st = kWalking;
    uint32_t col = 0;
    if (active) st = walk_steps<false>(m, lv, r, s, Lmax, iters, col);
    if (st != kWalking) {
      uint32_t word;
      float depth;
      finish(r, s, m.W, st, col, word, depth);
      store_hit(out, out_idx, word, depth);
      if (o.count) atomicAdd(o.count, (unsigned long long)s.reads);
      active = false;
    }
  }
}

}  // namespace

hipError_t tci_launch_render(const tci_map& m, const tci_view* views,
                             int32_t nviews, const int64_t* pkt_prefix,
                             int64_t npkt, void* out, int32_t flat,
                             const tci_render_opts& o, hipStream_t s) {
  int64_t blocks = (npkt + 3) / 4;
  if (blocks < 1) return hipSuccess;
  if (flat)
    hipLaunchKernelGGL(render_kernel<true>, dim3((uint32_t)blocks), dim3(256),
                       0, s, m, views, nviews, pkt_prefix, npkt, out, o);
  else
    hipLaunchKernelGGL(render_kernel<false>, dim3((uint32_t)blocks),
                       dim3(256), 0, s, m, views, nviews, pkt_prefix, npkt,
                       out, o);
  return hipGetLastError();
}

hipError_t tci_launch_render_persistent(const tci_map& m,
                                        const tci_view* views, int32_t nviews,
                                        const int64_t* pkt_prefix,
                                        int64_t npkt, void* out,
                                        uint64_t* counter, int32_t nblocks,
                                        const tci_render_opts& o,
                                        hipStream_t s) {
  if (npkt < 1) return hipSuccess;
  hipLaunchKernelGGL(render_persistent_kernel, dim3(nblocks), dim3(256), 0, s,
                     m, views, nviews, pkt_prefix, npkt, out, counter, o);
  return hipGetLastError();
}
