// The exact cell walk, shared by the render kernels and the shading pass.
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
#pragma once

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
enum : int32_t { kWalking = 0, kHitCell = 1, kMissed = 2, kCapped = 3, kSegEnd = 4 };
constexpr int32_t kAnchored = 8;

// (16-byte aligned: the walk reads a level's record with one LDS load)
struct __align__(16) lvl_t {
  uint32_t off;
  int32_t w1, h1, tiles_x;   // the level's width - 1 and height - 1, its tiles per row
};

// min(max(x, 0), hi) for hi >= 0 in one instruction (the compiler does not
// form a median-of-three from a clamp whose upper bound is a variable)
__device__ __forceinline__ int32_t clamp0(int32_t x, int32_t hi) {
  int32_t r;
  asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "v"(hi));
  return r;
}

// a * b for a < 2^24, b < 2^24 as a 48-bit product: two full-rate 24-bit
// multiplies instead of a quarter-rate 64-bit one.
__device__ __forceinline__ uint64_t mul48(uint32_t a, uint32_t b) {
  uint32_t lo, hi;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(lo) : "v"(a), "v"(b));
  asm("v_mul_hi_u32_u24 %0, %1, %2" : "=v"(hi) : "v"(a), "v"(b));
  return ((uint64_t)hi << 32) | lo;
}
// Low 32 bits of a * b for a, b < 2^24: one full-rate 24-bit multiply
// (the compiler otherwise may pick the quarter-rate 32-bit one inside the
// walk loop).
__device__ __forceinline__ uint32_t umul24(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// a * b for 0 <= a < 2^23 and |b| < 2^23, signed 48-bit product.
__device__ __forceinline__ int64_t smul48(int32_t a, int32_t b) {
  int32_t lo, hi;
  asm("v_mul_i32_i24 %0, %1, %2" : "=v"(lo) : "v"(a), "v"(b));
  asm("v_mul_hi_i32_i24 %0, %1, %2" : "=v"(hi) : "v"(a), "v"(b));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// K + a * b for a < 2^24, b < 2^24 and K + a * b + (a product's high half)
// for |a|, |b| < 2^23 signed: the two halves of the 48-bit product are
// added as a carry pair (two 32-bit adds) instead of as a 64-bit value.
__device__ __forceinline__ int64_t add_pair(int64_t K, uint32_t lo, uint32_t hi) {
  uint32_t c;
  const uint32_t rl = __builtin_addc((uint32_t)K, lo, 0u, &c);
  const uint32_t rh = __builtin_addc((uint32_t)((uint64_t)K >> 32), hi, c, &c);
  return (int64_t)(((uint64_t)rh << 32) | rl);
}
__device__ __forceinline__ int64_t add_mul48(int64_t K, uint32_t a, uint32_t b) {
  uint32_t lo, hi;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(lo) : "v"(a), "v"(b));
  asm("v_mul_hi_u32_u24 %0, %1, %2" : "=v"(hi) : "v"(a), "v"(b));
  return add_pair(K, lo, hi);
}
__device__ __forceinline__ int64_t add_smul48(int64_t K, int32_t a, int32_t b) {
  uint32_t lo, hi;
  asm("v_mul_i32_i24 %0, %1, %2" : "=v"(lo) : "v"(a), "v"(b));
  asm("v_mul_hi_i32_i24 %0, %1, %2" : "=v"(hi) : "v"(a), "v"(b));
  return add_pair(K, lo, hi);
}
struct ray_t {
  int64_t Ox, Oy, Oz;
  int32_t Dx, Dy, Dz;
  uint32_t ax, ay;
  int32_t cx0, cy0;   // anchor cell: the start cell, or a segment's first cell
  uint32_t rx, ry;    // residual flags of the x / y crossing heights
};

// Exact state of the cell walk, divided by S.  Every crossing moves its
// key and height by a multiple of S, so the remainders modulo S are fixed
// per axis: they fold into a tie offset of the x keys and a 0/1 flag of
// the heights, and no comparison needs the low 16 bits.
//   keys    the i-th x crossing (i = 0 the first) has key KX0 + i*ay with
//           KX0 = floor(nx*ay / S) + c, c = 1 iff (nx*ay mod S) > (ny*ax mod S),
//           and the j-th y crossing KY0 + j*ax, KY0 = floor(ny*ax / S); an x
//           crossing comes first iff its key is <= the y key (x first on
//           ties), exactly as the times nx/ax and ny/ay compare.
//   heights with Z = Oz*ax + nx*Dz (z * S * ax at the first x crossing),
//           ZX0 = floor(Z / S) and rx = (Z mod S != 0), the i-th x crossing
//           has height ZX0 + i*Dz and there
//           z <= h  iff  height + rx <= h*ax,   z >= h  iff  height >= h*ax.
//           Likewise for y.
// The walk runs on the node grid of its current pyramid level L.  For the
// current node it needs the keys and heights of the crossings through the
// far x and y faces.  The crossing through the far x face of node (ni, L)
// is x crossing number
//   ix = ((ni + 1) << L) - 1 - cx  (Dx > 0),   cx - (ni << L)  (Dx <= 0)
// counted from the origin cell cx (never negative: the far face lies ahead
// of the origin), so its key is KX0 + ix * ay and its height ZX0 + ix * Dz;
// likewise for y.  The walk therefore carries the node, the level and the
// entry crossing only: a step, a climb or a descent changes 32-bit node
// coordinates, and the far faces follow from them.  The child holding the
// ray is the one on the near side of each middle crossing that happens
// after the entry crossing, so the walk enters exactly the cells the flat
// walk enters, at the same keys.
struct walk_idx_t {
  int64_t KX0, KY0;   // keys of crossing number 0 of each axis
  int64_t ZX0, ZY0;   // heights at those crossings
  int32_t offx, offy; // ix = sx ((ni + f) << L) + offx (f = 1 iff Dx > 0), likewise for y
};

struct walk_t {
  int32_t ni, nj;     // node indices at level L
  int32_t L;          // current pyramid level
  int64_t Kin;        // key of the entry crossing (unused while kInside)
  int64_t Zin;        // height at entry of the current node
  uint32_t Din;       // its scale: 1 at the origin, else ax or ay
  uint32_t rin;       // its residual flag
  int32_t entry;      // face crossed on entry (kInside before any crossing),
                      // plus kAnchored until the first step: the walk then
                      // sits in the anchor cell (r.cx0, r.cy0) and picks
                      // children by it
  int32_t iters;
  int32_t reads;      // nodes and cells read from memory
};

// h * d for a height h < 2^8 and a scale d < 2^23 as a 64-bit value: the
// product is below 2^31, so its high word is zero
__device__ __forceinline__ int64_t hmul(uint32_t h, uint32_t d) {
  return (int64_t)(uint32_t)__umul24(h, d);
}
// z <= h and z >= h for a height with floor part zq, flag r and scale d
__device__ __forceinline__ bool z_le(int64_t zq, uint32_t r, uint32_t h, uint32_t d) {
  return zq + (int64_t)r <= hmul(h, d);
}
__device__ __forceinline__ bool z_ge(int64_t zq, uint32_t h, uint32_t d) {
  return zq >= hmul(h, d);
}
// A wave-uniform 64-bit value moved to scalar registers.
__device__ __forceinline__ int64_t rfl64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
// Word `idx` of the map allocation.  The allocation (columns, pyramid and
// masks of at most 2^27 cells, tiles padded) holds about 2^28 words, far
// below the 2^30 whose byte offsets fit in 32 bits, so the byte offset is a
// 32-bit value added to the scalar base: the load's base-plus-offset form,
// with no 64-bit address arithmetic per lane.
__device__ __forceinline__ uint32_t map_word(const uint32_t* base, uint32_t idx) {
  return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(base) + (idx << 2));
}
// a << L for an unsigned 32-bit a as a 64-bit value
__device__ __forceinline__ int64_t ushl(uint32_t a, int32_t L) {
  return (int64_t)((uint64_t)a << L);
}

// Ray of pixel (px, py).  Every pixel's origin and direction fit in 32 bits
// (tc_render_views checks the view's corner rays, and the rays are affine
// in the pixel), so 32-bit wrapping arithmetic gives them exactly.
__device__ __forceinline__ void pixel_ray(const tci_view& v, int32_t px,
                                          int32_t py, ray_t& r) {
  const uint32_t a = 2 * (uint32_t)px + 1, b = 2 * (uint32_t)py + 1;
  auto at = [&](int32_t c0, int32_t ca, int32_t cb) {
    return (int32_t)((uint32_t)c0 + a * (uint32_t)ca + b * (uint32_t)cb);
  };
  r.Ox = at(v.o0[0], v.opx[0], v.opy[0]);
  r.Oy = at(v.o0[1], v.opx[1], v.opy[1]);
  r.Oz = at(v.o0[2], v.opx[2], v.opy[2]);
  r.Dx = at(v.d0[0], v.dpx[0], v.dpy[0]);
  r.Dy = at(v.d0[1], v.dpx[1], v.dpy[1]);
  r.Dz = at(v.d0[2], v.dpx[2], v.dpy[2]);
  r.ax = (uint32_t)(r.Dx < 0 ? -r.Dx : r.Dx);
  r.ay = (uint32_t)(r.Dy < 0 ? -r.Dy : r.Dy);
}

// The same ray for the pixel of lane `lane` in the packet of tile (tx, ty)
// (2^pw x 2^(6 - pw) pixels, pw = v.pw_log2), all of whose lanes call it
// together (tx, ty wave-uniform): the ray of the packet's first pixel is
// wave-uniform (scalar arithmetic), and a lane adds its column
// (lane & (2^pw - 1)) and row (lane >> pw) in the packet times twice the
// view's per-pixel steps, one 24-bit multiply-add each when the view's
// steps are small (the usual case; v.small_steps).  kDir false: the origin
// only.
template <bool kDir = true>
__device__ __forceinline__ void packet_ray(const tci_view& v, int32_t tx, int32_t ty,
                                           int32_t lane, ray_t& r) {
  const int32_t pw = v.pw_log2;
  const uint32_t a0 = ((uint32_t)tx << (pw + 1)) + 1, b0 = ((uint32_t)ty << (7 - pw)) + 1;
  const int32_t lx = lane & ((1 << pw) - 1), ly = lane >> pw;
  int32_t o[6];
  auto base = [&](int32_t c0, int32_t ca, int32_t cb) {
    return (int32_t)((uint32_t)c0 + a0 * (uint32_t)ca + b0 * (uint32_t)cb);
  };
  auto step = [&](int32_t c) {
    return c < 3 ? v.opx[c] : v.dpx[c - 3];
  };
  auto stepy = [&](int32_t c) {
    return c < 3 ? v.opy[c] : v.dpy[c - 3];
  };
  constexpr int kN = kDir ? 6 : 3;
  if (v.small_steps) {
#pragma unroll
    for (int c = 0; c < kN; ++c) {
      const int32_t b = base(c < 3 ? v.o0[c] : v.d0[c - 3], step(c), stepy(c));
      o[c] = __mul24(ly, 2 * stepy(c)) + (__mul24(lx, 2 * step(c)) + b);
    }
  } else {
#pragma unroll
    for (int c = 0; c < kN; ++c) {
      const int32_t b = base(c < 3 ? v.o0[c] : v.d0[c - 3], step(c), stepy(c));
      o[c] = (int32_t)((uint32_t)b + (uint32_t)lx * (2u * (uint32_t)step(c)) +
                       (uint32_t)ly * (2u * (uint32_t)stepy(c)));
    }
  }
  r.Ox = o[0];
  r.Oy = o[1];
  r.Oz = o[2];
  if constexpr (kDir) {
    r.Dx = o[3];
    r.Dy = o[4];
    r.Dz = o[5];
    r.ax = (uint32_t)(r.Dx < 0 ? -r.Dx : r.Dx);
    r.ay = (uint32_t)(r.Dy < 0 ? -r.Dy : r.Dy);
  }
}

// Index-form constants of ray r (crossing numbers counted from its origin
// cell) and its residual flags; the anchor (r.cx0, r.cy0) becomes the
// origin cell.
__device__ __forceinline__ void walk_origin(ray_t& r, walk_idx_t& k) {
  const int32_t cx = (int32_t)(r.Ox >> 16), cy = (int32_t)(r.Oy >> 16);
  r.cx0 = cx;
  r.cy0 = cy;
  // distances to the first boundaries, 0..2^16 (S units)
  const uint32_t fx = (uint32_t)r.Ox & 0xFFFF, fy = (uint32_t)r.Oy & 0xFFFF;
  const uint32_t nx = r.Dx > 0 ? 65536u - fx : fx;
  const uint32_t ny = r.Dy > 0 ? 65536u - fy : fy;
  const int64_t kx = (int64_t)mul48(nx, r.ay), ky = (int64_t)mul48(ny, r.ax);
  const int64_t tie = ((uint32_t)kx & 0xFFFF) <= ((uint32_t)ky & 0xFFFF) ? 0 : 1;
  // Z = Oz * a + n * Dz with Oz = zh * S + zl (|Oz| < 2^31, so |zh| < 2^15):
  // floor(Z / S) = zh * a + floor(w / S) and Z mod S = w mod S for
  // w = zl * a + n * Dz
  const int32_t zh = (int32_t)(r.Oz >> 16);
  const uint32_t zl = (uint32_t)r.Oz & 0xFFFF;
  const int64_t wx = (int64_t)mul48(zl, r.ax) + smul48((int32_t)nx, r.Dz);
  const int64_t wy = (int64_t)mul48(zl, r.ay) + smul48((int32_t)ny, r.Dz);
  r.rx = ((uint32_t)wx & 0xFFFF) != 0;
  r.ry = ((uint32_t)wy & 0xFFFF) != 0;
  k.KX0 = r.Dx == 0 ? kNever : (kx >> 16) + (r.Dy != 0 ? tie : 0);
  k.KY0 = r.Dy == 0 ? kNever : (ky >> 16);
  k.ZX0 = smul48((int32_t)r.ax, zh) + (wx >> 16);
  k.ZY0 = smul48((int32_t)r.ay, zh) + (wy >> 16);
  k.offx = r.Dx > 0 ? -1 - cx : cx;
  k.offy = r.Dy > 0 ? -1 - cy : cy;
}

// Walk state at the origin, on the level-L0 node holding the origin cell
// (after walk_origin).
__device__ __forceinline__ void walk_at_origin(const ray_t& r, int32_t L0, walk_t& s) {
  s.L = L0;
  s.ni = r.cx0 >> L0;
  s.nj = r.cy0 >> L0;
  s.Kin = 0;
  s.Zin = r.Oz >> 16;
  s.rin = (r.Oz & 0xFFFF) != 0;
  s.Din = 1;
  s.entry = kInside | kAnchored;
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

// First hit inside cell (x, y) (packed column v), entered with height zin
// (scale din, flag rin) through face `entry`, given that the ray's height
// range over the cell meets solid.
__device__ __forceinline__ void resolve_hit(const ray_t& r, int32_t x, int32_t y,
                                            int32_t entry, int64_t zin,
                                            uint32_t din, uint32_t rin,
                                            int32_t W, uint32_t v,
                                            uint32_t& word, float& depth) {
  uint32_t F = v & 0xFF, B = (v >> 8) & 0xFF, T = (v >> 16) & 0xFF;
  bool in_floor = z_le(zin, rin, F, din);
  bool in_slab = B != 0 && z_ge(zin, B, din) && z_le(zin, rin, T, din);
  int32_t face, layer;
  int64_t tn, td;
  if (in_floor || in_slab) {
    face = entry;
    layer = in_floor ? 0 : 1;
    switch (face) {
      case kWmx: tn = ((int64_t)x << 16) - r.Ox; td = r.ax; break;
      case kWpx: tn = r.Ox - ((int64_t)(x + 1) << 16); td = r.ax; break;
      case kWmy: tn = ((int64_t)y << 16) - r.Oy; td = r.ay; break;
      case kWpy: tn = r.Oy - ((int64_t)(y + 1) << 16); td = r.ay; break;
      default: tn = 0; td = 1; break;
    }
  } else if (r.Dz < 0) {
    bool above = B != 0 && !z_le(zin, rin, T, din);
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
  set_hit(r, W, x, y, face, layer, tn, td, word, depth);
}

// Hit record of a finished walk.
__device__ __forceinline__ void finish(const ray_t& r, const walk_t& s,
                                       int32_t W, int32_t state, uint32_t v,
                                       uint32_t& word, float& depth) {
  if (state == kHitCell) {
    resolve_hit(r, s.ni, s.nj, s.entry & 7, s.Zin, s.Din, s.rin, W, v, word, depth);
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
  bool in_floor = r.Oz <= ((int64_t)F << 16);
  bool in_slab = B != 0 && r.Oz >= ((int64_t)B << 16) && r.Oz <= ((int64_t)T << 16);
  if (in_floor || in_slab || r.Dz < 0 || (B != 0 && r.Oz < ((int64_t)B << 16)))
    resolve_hit(r, cx, cy, kInside, r.Oz >> 16, 1, (r.Oz & 0xFFFF) != 0, m.W, v,
                word, depth);
}

// Number of terms K + j*a, j >= 0, strictly below E, for counts below 2^24
// and E - K < 2^47: a float estimate of the quotient, then one exact
// correction.
__device__ __forceinline__ int32_t count_below(int64_t E, int64_t K, uint32_t a) {
  if (E <= K) return 0;
  const int64_t n = E - K - 1;             // count = floor(n / a) + 1
  const float nf = (float)(uint32_t)(n >> 32) * 4294967296.0f + (float)(uint32_t)n;
  int32_t q = (int32_t)(nf * __builtin_amdgcn_rcpf((float)a));
  q = q < 0 ? 0 : q;
  const int64_t p = (int64_t)mul48((uint32_t)q, a);
  q += (p > n) ? -1 : ((n - p >= (int64_t)a) ? 1 : 0);
  return q + 1;
}

// Walk state (at level 0) on entering cell line `line` of axis `axis` (a
// column if 0, a row if 1) through the crossing the flat walk takes into
// it (after walk_origin): the crossing's key and height come from its
// index, the cell on the other axis from the number of that axis's
// crossings that come first (x first on ties).  The anchor becomes that
// cell.  False, and nothing changed, if `line` is not ahead of the origin
// cell's.
__device__ __forceinline__ bool walk_at_line(ray_t& r, const walk_idx_t& k, walk_t& s,
                                             int32_t axis, int32_t line) {
  const int32_t cx = r.cx0, cy = r.cy0;
  if (axis == 0) {
    const int32_t i = r.Dx > 0 ? line - cx - 1 : cx - line - 1;
    if (i < 0) return false;
    const int64_t K = k.KX0 + (int64_t)mul48((uint32_t)i, r.ay);
    const int32_t c = count_below(K, k.KY0, r.ax);
    s.Kin = K;
    s.Zin = k.ZX0 + smul48(i, r.Dz);
    s.Din = r.ax;
    s.rin = r.rx;
    s.ni = line;
    s.nj = cy + (r.Dy > 0 ? c : -c);
    s.entry = (r.Dx > 0 ? kWmx : kWpx) | kAnchored;
  } else {
    const int32_t j = r.Dy > 0 ? line - cy - 1 : cy - line - 1;
    if (j < 0) return false;
    const int64_t K = k.KY0 + (int64_t)mul48((uint32_t)j, r.ax);
    const int32_t c = count_below(K + 1, k.KX0, r.ay);
    s.Kin = K;
    s.Zin = k.ZY0 + smul48(j, r.Dz);
    s.Din = r.ay;
    s.rin = r.ry;
    s.nj = line;
    s.ni = cx + (r.Dx > 0 ? c : -c);
    s.entry = (r.Dy > 0 ? kWmy : kWpy) | kAnchored;
  }
  s.L = 0;
  s.iters = 0;
  s.reads = 0;
  r.cx0 = s.ni;
  r.cy0 = s.nj;
  return true;
}

// (n + f) << L with f = 1 when the axis runs forward, times s = +-1, plus
// off: |(n + f) << L| stays below 2^23 (cell coordinates are within
// +-2^16), so one 24-bit multiply-add.
__device__ __forceinline__ int32_t far_index(int32_t n, int32_t L, int32_t f, int32_t s,
                                             int32_t off) {
  return __mul24(s, (n + f) << L) + off;
}

// Does voxel column (X, Y) of level k of the voxel occupancy pyramid hold a
// set bit over heights [zl, zh]?  The heights are float estimates of the
// ray's exact range over the column, already widened to cover their
// rounding; both ends are clipped into the pyramid's heights, so a range
// partly or wholly below height 0 tests the first voxel, which every
// in-map column's floor (unbounded below) sets, and a range wholly above
// the top (z > 256) holds nothing.
// Per 8-voxel tile in z, the column's eight bits sit in four words (two
// 64-bit loads): in-tile Morton index x0 y0 z0 x1 y1 | z1 x2 y2 z2 puts
// z0 in the bit and z1, z2 in the word.  `reads` counts the loads.
__device__ __forceinline__ bool voxel_range(const tci_voxels& vx, int32_t k, int32_t X,
                                            int32_t Y, float zl, float zh, int32_t& reads) {
  const tci_vlevel& l = vx.lv[k];
  const float inv = __builtin_amdgcn_ldexpf(1.0f, -(vx.vz_log2 + k));
  const int32_t z0 = max((int32_t)floorf(fmaxf(zl, -1.0f) * inv), 0);
  const int32_t z1 = min(max((int32_t)floorf(fmaxf(fminf(zh, 1.0e6f), -1.0f) * inv), 0),
                         l.nz - 1);
  if (z0 > z1) return false;
  const uint32_t x = (uint32_t)X & 7, y = (uint32_t)Y & 7;
  const uint32_t wb = ((x >> 2) << 1) | ((y >> 2) << 2);
  const uint32_t sh = (x & 1) | ((y & 1) << 1) | (((x >> 1) & 1) << 3) | (((y >> 1) & 1) << 4);
  const uint32_t* col = vx.base + l.off +
                        (uint32_t)(((Y >> 3) * l.tiles_x + (X >> 3)) << 4) + wb;
  const uint32_t zstride = (uint32_t)(l.tiles_y * l.tiles_x) << 4;
  for (int32_t tz = z0 >> 3; tz <= (z1 >> 3); ++tz) {
    const uint32_t* t = col + (uint32_t)tz * zstride;
    const uint2 a = *reinterpret_cast<const uint2*>(t);
    const uint2 b = *reinterpret_cast<const uint2*>(t + 8);
    reads += 2;
    const uint32_t bits = ((a.x >> sh) & 1u) | (((a.x >> (sh + 4)) & 1u) << 1) |
                          (((a.y >> sh) & 1u) << 2) | (((a.y >> (sh + 4)) & 1u) << 3) |
                          (((b.x >> sh) & 1u) << 4) | (((b.x >> (sh + 4)) & 1u) << 5) |
                          (((b.y >> sh) & 1u) << 6) | (((b.y >> (sh + 4)) & 1u) << 7);
    const int32_t lo = max(z0 - tz * 8, 0), hi = min(z1 - tz * 8, 7);
    const uint32_t want = ((2u << hi) - 1u) & ~((1u << lo) - 1u);
    if (bits & want) return true;
  }
  return false;
}

// Advance the walk by up to `budget` iterations.  Returns kWalking if the
// budget ran out, else the final state; on kHitCell, `col` holds the
// column of the current cell (s.ni, s.nj at level 0).  k holds the ray's
// index-form constants (walk_origin).
// With boost > 0 (wave-uniform loop only), a wave raises its instruction
// issue priority after boost, 2*boost and 4*boost iterations: the few long
// walks of a launch, which otherwise trail it, then win issue slots over
// the many short ones sharing their SIMD.
// With kSeg the walk also stops (kSegEnd) once its node lies wholly
// outside the cell lines [seg_lo, seg_hi] of axis seg_axis (0 x, 1 y).
// With kCap every call counts the walk's iterations in s.iters and stops
// (kCapped) past kIterCap, a guard for callers that resume a walk without
// bound; a caller whose budget already bounds the walk passes false.  With
// count false, s.reads is left alone.
// With kOcc, a node that only the slab test keeps is also tested against
// its occupancy mask (moff: the mask levels' word offsets, in LDS): the
// ray's height range over the node, widened by two units to cover the
// rounding of its float estimate, must meet an occupied band, or the ray
// passes between the node's slabs and the node is skipped.
// kDir fixes the sign of the ray's vertical direction for callers that know
// it for every lane of the wave (1: Dz < 0, 2: Dz >= 0; 0: read it per ray),
// so the loop carries no per-lane selects on it.
// With kVox (the voxel-accelerated march, Section 3.2), nodes above the
// cells are tested against the voxel occupancy pyramid *vx instead of the
// min/max pyramid: a node of level L >= the voxels' footprint level Lv is
// voxel column (ni, nj) of voxel level L - Lv, empty over the ray's height
// range over the node (widened by two units to cover the rounding of its
// float estimate) or not; nodes below Lv are always descended (the leaf
// voxel's cells are then tested exactly, one by one).
template <bool kSeg = false, bool kOcc = false, bool kCap = true, int kDir = 0,
          bool kVox = false>
__device__ __forceinline__ int32_t walk_steps(const tci_map& m, const lvl_t* lv,
                                              const ray_t& r, const walk_idx_t& k, walk_t& s,
                                              int32_t max_level, int32_t budget,
                                              uint32_t& col, int32_t boost = 0,
                                              int32_t seg_axis = 0,
                                              int32_t seg_lo = 0, int32_t seg_hi = 0,
                                              const uint32_t* moff = nullptr,
                                              bool count = true,
                                              const tci_voxels* vx = nullptr) {
  const bool desc = kDir == 1 ? true : (kDir == 2 ? false : r.Dz < 0);
  const bool fx = r.Dx > 0, fy = r.Dy > 0;
  const int32_t sx = fx ? 1 : -1, sy = fy ? 1 : -1;
  const int32_t nx1 = fx ? 1 : 0, ny1 = fy ? 1 : 0;
  const int32_t nearx = 1 - nx1, neary = 1 - ny1;
  for (int32_t it = 0; it < budget; ++it) {
    if (boost > 0) {
      if (it == boost) __builtin_amdgcn_s_setprio(1);
      else if (it == 2 * boost) __builtin_amdgcn_s_setprio(2);
      else if (it == 4 * boost) __builtin_amdgcn_s_setprio(3);
    }
    if constexpr (kCap) {
      if (++s.iters > kIterCap) return kCapped;
    }
    const int32_t L = s.L;
    if (kSeg) {
      const int32_t n = seg_axis == 0 ? s.ni : s.nj;
      if ((n << L) > seg_hi || ((n + 1) << L) - 1 < seg_lo) return kSegEnd;
    }
    // the level's record in one 16-byte LDS read, then every lane loads its
    // node clamped into the level, with no branch around the load: the
    // step's chain holds one LDS round trip and no exec-mask branch before
    // the node load (levels up to max_level are never empty, so the clamp
    // stays in the level)
    const uint4 lq = *reinterpret_cast<const uint4*>(&lv[L]);
    lvl_t l;
    l.off = lq.x;
    l.w1 = (int32_t)lq.y;
    l.h1 = (int32_t)lq.z;
    l.tiles_x = (int32_t)lq.w;
    const bool inmap = ((uint32_t)s.ni <= (uint32_t)l.w1) & ((uint32_t)s.nj <= (uint32_t)l.h1);
    if (count) s.reads += (inmap & (!kVox | (L == 0))) ? 1 : 0;
    const uint32_t ci = (uint32_t)clamp0(s.ni, l.w1);
    const uint32_t cj = (uint32_t)clamp0(s.nj, l.h1);
    const uint32_t vraw = map_word(m.base, l.off + ((umul24(cj >> 3, (uint32_t)l.tiles_x) +
                                                     (ci >> 3)) << 6) +
                                               ((cj & 7) << 3) + (ci & 7));
    const uint32_t v = (inmap & (!kVox | (L == 0))) ? vraw : 0u;
    // keys and heights of the crossings through the node's far faces
    const int32_t ix = far_index(s.ni, L, nx1, sx, k.offx);
    const int32_t iy = far_index(s.nj, L, ny1, sy, k.offy);
    const int64_t KXe = add_mul48(k.KX0, (uint32_t)ix, r.ay);
    const int64_t KYe = add_mul48(k.KY0, (uint32_t)iy, r.ax);
    const bool ex = KXe <= KYe;               // leave through an x face
    const int64_t Ze = add_smul48(ex ? k.ZX0 : k.ZY0, ex ? ix : iy, r.Dz);
    const uint32_t De = ex ? r.ax : r.ay;
    const uint32_t re = ex ? r.rx : r.ry;
    bool occ = false;
    if (inmap) {
      const int64_t lo = (desc ? Ze : s.Zin) + (int64_t)(desc ? re : s.rin);
      const uint32_t Dlo = desc ? De : s.Din;
      const int64_t hi = desc ? s.Zin : Ze;
      const uint32_t Dhi = desc ? s.Din : De;
      const uint32_t a = v & 0xFF, b = (v >> 8) & 0xFF, c = (v >> 16) & 0xFF;
      // the three compares combined without short-circuit branches
      occ = (lo <= hmul(a, Dlo)) | ((lo <= hmul(c, Dlo)) & (hi >= hmul(b, Dhi)));
      if constexpr (kOcc) {
        if (occ && L > 0 && !(lo <= hmul(a, Dlo))) {
          const uint32_t mi = moff[L] +
                              ((__umul24((uint32_t)s.nj >> 3, (uint32_t)l.tiles_x) +
                                ((uint32_t)s.ni >> 3)) << 7) +
                              ((((uint32_t)(s.nj & 7) << 3) + (uint32_t)(s.ni & 7)) << 1);
          const uint2 mw = *reinterpret_cast<const uint2*>(m.base + mi);
          const uint64_t mask = (uint64_t)mw.x | ((uint64_t)mw.y << 32);
          if (count) s.reads += 2;
          const float zl = (float)lo / (float)Dlo - 2.0f;
          const float zh = (float)hi / (float)Dhi + 2.0f;
          const int32_t kl = min(max((int32_t)floorf(zl * 0.25f), 0), 63);
          const int32_t kh = min(max((int32_t)floorf(zh * 0.25f), 0), 63);
          const uint64_t range = (~0ull >> (63 - kh)) & (~0ull << kl);
          occ = (mask & range) != 0;
        }
      }
      if constexpr (kVox) {
        if (L > 0) {
          const int32_t Lv = vx->v_log2;
          occ = true;
          if (L >= Lv) {
            const float zl = (float)lo / (float)Dlo - 2.0f;
            const float zh = (float)hi / (float)Dhi + 2.0f;
            int32_t vr = 0;
            occ = voxel_range(*vx, L - Lv, s.ni, s.nj, zl, zh, vr);
            if (count) s.reads += vr;
          }
        }
      }
    }
    if (occ && L == 0) {
      col = v;
      return kHitCell;
    }
    // one latch for both moves: a descent or a step (and maybe a climb)
    // writes the node and level once, at the end
    int32_t ni = s.ni, nj = s.nj, nL;
    if (occ) {
      // descend into the child holding the ray after the entry crossing
      const int32_t Lc = L - 1;
      int32_t bx, by;
      const bool anchored = (s.entry & kAnchored) != 0;
      if (r.Dx == 0 || anchored) bx = (r.cx0 >> Lc) & 1;
      else if (s.entry == kWmx || s.entry == kWpx) bx = nearx;
      else bx = (KXe - ushl(r.ay, Lc) <= s.Kin) ? 1 - nearx : nearx;
      if (r.Dy == 0 || anchored) by = (r.cy0 >> Lc) & 1;
      else if (s.entry == kWmy || s.entry == kWpy) by = neary;
      else by = (KYe - ushl(r.ax, Lc) < s.Kin) ? 1 - neary : neary;
      ni = 2 * ni + bx;
      nj = 2 * nj + by;
      nL = Lc;
    } else {
      // step to the next node of this level through the exit face
      s.Kin = ex ? KXe : KYe;
      if (ex) {
        ni += sx;
        s.entry = fx ? kWmx : kWpx;
      } else {
        nj += sy;
        s.entry = fy ? kWmy : kWpy;
      }
      s.Zin = Ze;
      s.Din = De;
      s.rin = re;
      // the ray cannot come back into the map, or is above all solid
      // (compares combined bitwise, without short-circuit branches)
      const bool away = ((ni < 0) & (r.Dx <= 0)) | ((ni > l.w1) & (r.Dx >= 0)) |
                        ((nj < 0) & (r.Dy <= 0)) | ((nj > l.h1) & (r.Dy >= 0));
      const bool above = !desc & !z_le(s.Zin, s.rin, 255, s.Din);
      if (away | above) return kMissed;
      // go up one level when the step entered a new parent node
      nL = L;
      int32_t up = 1;
      if constexpr (kVox) {
        // below the voxels' footprint level every node counts as occupied,
        // so a climb stops there only to descend again: inside a leaf
        // voxel the walk stays on the cells, and the step that leaves it
        // climbs straight to the footprint level (the new leaf voxel is
        // entered at this very crossing)
        const int32_t Lv = min(vx->v_log2, max_level);
        if (L < Lv) up = Lv - L;
      }
      if ((L < max_level) & ((((s.ni ^ ni) | (s.nj ^ nj)) >> up) != 0)) {
        ni >>= up;
        nj >>= up;
        nL = L + up;
      }
    }
    s.ni = ni;
    s.nj = nj;
    s.L = nL;
  }
  return kWalking;
}

// The walk kept on the cells (level 0) for up to K cells, for a caller
// whose walk spans a few cell lines: the cells it enters follow from the
// keys alone, so the K columns ahead are loaded together first (indices
// clamped into the map, so every load is valid) and then tested in order
// from registers, and the walk waits on one round of loads instead of one
// per cell.  Results and state as walk_steps<kSeg = true, kOcc = false,
// kCap = true, kDir> with max_level 0: l0 is the cells' level record.
template <int kDir, int K>
__device__ __forceinline__ int32_t walk_flat(const tci_map& m, const lvl_t l0, const ray_t& r,
                                             const walk_idx_t& k, walk_t& s, uint32_t& col,
                                             int32_t seg_axis, int32_t seg_lo, int32_t seg_hi,
                                             bool count) {
  const bool desc = kDir == 1;
  const bool fx = r.Dx > 0, fy = r.Dy > 0;
  const int32_t sx = fx ? 1 : -1, sy = fy ? 1 : -1;
  const int32_t nx1 = fx ? 1 : 0, ny1 = fy ? 1 : 0;
  auto word_at = [&](int32_t ni, int32_t nj) {
    const uint32_t ci = (uint32_t)clamp0(ni, l0.w1), cj = (uint32_t)clamp0(nj, l0.h1);
    return map_word(m.base, l0.off + ((umul24(cj >> 3, (uint32_t)l0.tiles_x) + (ci >> 3)) << 6) +
                                ((cj & 7) << 3) + (ci & 7));
  };
  // the cells ahead: a step leaves through the x face iff the far x
  // crossing's key is not above the far y crossing's
  uint32_t w[K];
  {
    int32_t ni = s.ni, nj = s.nj;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      w[t] = word_at(ni, nj);
      if (t + 1 < K) {
        const int32_t ix = far_index(ni, 0, nx1, sx, k.offx);
        const int32_t iy = far_index(nj, 0, ny1, sy, k.offy);
        const bool ex = add_mul48(k.KX0, (uint32_t)ix, r.ay) <= add_mul48(k.KY0, (uint32_t)iy, r.ax);
        ni += ex ? sx : 0;
        nj += ex ? 0 : sy;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < K; ++t) {
    if (++s.iters > kIterCap) return kCapped;
    const int32_t n = seg_axis == 0 ? s.ni : s.nj;
    if ((n > seg_hi) | (n < seg_lo)) return kSegEnd;
    const bool inmap = ((uint32_t)s.ni <= (uint32_t)l0.w1) & ((uint32_t)s.nj <= (uint32_t)l0.h1);
    if (count) s.reads += inmap ? 1 : 0;
    const uint32_t v = inmap ? w[t] : 0u;
    const int32_t ix = far_index(s.ni, 0, nx1, sx, k.offx);
    const int32_t iy = far_index(s.nj, 0, ny1, sy, k.offy);
    const int64_t KXe = add_mul48(k.KX0, (uint32_t)ix, r.ay);
    const int64_t KYe = add_mul48(k.KY0, (uint32_t)iy, r.ax);
    const bool ex = KXe <= KYe;
    const int64_t Ze = add_smul48(ex ? k.ZX0 : k.ZY0, ex ? ix : iy, r.Dz);
    const uint32_t De = ex ? r.ax : r.ay;
    const uint32_t re = ex ? r.rx : r.ry;
    if (inmap) {
      const int64_t lo = (desc ? Ze : s.Zin) + (int64_t)(desc ? re : s.rin);
      const uint32_t Dlo = desc ? De : s.Din;
      const int64_t hi = desc ? s.Zin : Ze;
      const uint32_t Dhi = desc ? s.Din : De;
      const uint32_t a = v & 0xFF, b = (v >> 8) & 0xFF, c = (v >> 16) & 0xFF;
      if ((lo <= hmul(a, Dlo)) | ((lo <= hmul(c, Dlo)) & (hi >= hmul(b, Dhi)))) {
        col = v;
        return kHitCell;
      }
    }
    s.Kin = ex ? KXe : KYe;
    s.ni += ex ? sx : 0;
    s.nj += ex ? 0 : sy;
    s.entry = ex ? (fx ? kWmx : kWpx) : (fy ? kWmy : kWpy);
    s.Zin = Ze;
    s.Din = De;
    s.rin = re;
    const bool away = ((s.ni < 0) & (r.Dx <= 0)) | ((s.ni > l0.w1) & (r.Dx >= 0)) |
                      ((s.nj < 0) & (r.Dy <= 0)) | ((s.nj > l0.h1) & (r.Dy >= 0));
    const bool above = !desc & !z_le(s.Zin, s.rin, 255, s.Din);
    if (away | above) return kMissed;
  }
  return kWalking;
}

__device__ __forceinline__ void load_levels(const tci_map& m, lvl_t* lv) {
  if (threadIdx.x < TCI_MAX_LEVELS) {
    const tci_level& l = m.lv[threadIdx.x];
    lv[threadIdx.x] = lvl_t{l.off, l.w - 1, l.h - 1, l.tiles_x};
  }
  __syncthreads();
}

// Level table plus the window levels' word offsets (woff) and, if moff is
// given, the occupancy mask levels' word offsets.
__device__ __forceinline__ void load_levels_beam(const tci_map& m, lvl_t* lv, uint32_t* woff,
                                                 uint32_t* moff) {
  if (threadIdx.x < TCI_MAX_LEVELS) {
    const tci_level& l = m.lv[threadIdx.x];
    lv[threadIdx.x] = lvl_t{l.off, l.w - 1, l.h - 1, l.tiles_x};
    woff[threadIdx.x] = m.wl[threadIdx.x].off;
    if (moff) moff[threadIdx.x] = m.mk[threadIdx.x].off;
  }
  __syncthreads();
}

__device__ __forceinline__ int32_t clamp_level(int32_t v, int32_t top) {
  return v < 0 ? 0 : (v > top ? top : v);
}

}  // namespace
