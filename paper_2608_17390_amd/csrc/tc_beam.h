// Packet beam: a conservative common start for the rays of one 8 x 8 pixel
// packet (one wave), so that each ray's exact walk begins where solid can
// first be near instead of at the eye.
//
// A packet's rays are P(a, b, t) = O(a, b) + t D(a, b) with O and D affine in
// the pixel coordinates a = 2 px + 1, b = 2 py + 1.  At a fixed t each
// coordinate is therefore affine in (a, b): over the packet's pixel
// rectangle it lies within
//   centre(t) +- (ha |dO/da + t dD/da| + hb |dO/db + t dD/db|)
// (ha, hb the half-spans of a and b), and for t >= 0 the extent is at most
// e0 + t e1 with e0 = ha |dO/da| + hb |dO/db|, e1 = ha |dD/da| + hb |dD/db|.
// Both bounds are then linear in t, so over a parameter interval [t0, t1]
// their extremes are at its ends.  The box they give, widened by a margin
// that covers the single-precision rounding, is tested against the
// min/max pyramid: at the level whose nodes are wider than the box it
// overlaps at most 2 x 2 nodes, whose combine is one entry of that level's
// window level, and if its height range lies above the entry's fmax and
// outside its [smin, smax], no ray of the packet meets solid during
// [t0, t1] (the node test of the walk, applied to a bundle of rays;
// Section 3.2's skip of empty space).
//
// The 64 lanes test 64 consecutive intervals at once, of geometrically
// growing length, starting at the current start; the start moves to the
// first interval that could not be cleared and the search repeats from
// there with short intervals, at most `passes` times.  Each ray then begins
// its walk on the last cell line of its dominant axis that it enters no
// later than that start, in the exact state the full walk would enter it
// with (seg_init), so every hit record is unchanged.
#pragma once

#include "tc_walk.h"

namespace {

constexpr float kBeamFirst = 0.5f;           // first interval: cells along the centre ray
constexpr float kBeamGrowth = 0.125f;        // each interval 1/8 longer than the last
constexpr float kBeamLog2Growth = 0.169925f; // log2(1 + kBeamGrowth)

// Could solid lie in the box [lox, hix] x [loy, hiy] x [loz, hiz] (cells,
// height units)?  With 2^L the smallest power of two above the box's
// width and depth, the box overlaps at most two level-L nodes per axis,
// all inside the window of the first (tci_map.wl), so one window entry
// bounds its solid: one load, counted in `reads`.  Every test is evaluated
// and the answer combined without branches (lanes test different boxes, so
// early returns would diverge): the load uses an index clamped into the
// level, and the answer is the first of these that applies: no claim for a
// box with a NaN bound (never formed from valid views); clear above every
// height; no claim for a huge box or one wider than the top level's nodes;
// clear beside the map; else the window's test.  A box that starts before
// the map's first node uses that node's window, a superset of what the box
// overlaps.
__device__ __forceinline__ bool beam_box_solid(const tci_map& m, const lvl_t* lv,
                                               const uint32_t* woff, float lox, float hix,
                                               float loy, float hiy, float loz, float hiz,
                                               int32_t& reads) {
  const bool bad = !((lox <= hix) & (loy <= hiy) & (loz <= hiz));
  const bool above = loz > 255.0f;
  const float ext = fmaxf(hix - lox, hiy - loy);
  const bool huge = !(ext < 65536.0f);
  // ext < 2^e (frexp's exponent), and 2^0 = 1 > ext below one cell
  const int32_t e = ext < 1.0f ? 0 : __builtin_amdgcn_frexp_expf(ext);
  const bool wide = e > m.top;
  const int32_t L = min(e, m.top);
  // the first node of each axis, clamped far outside the map
  auto node = [&](float c) {
    return (int32_t)floorf(__builtin_amdgcn_fmed3f(c, -1048576.0f, 1048576.0f)) >> L;
  };
  const int32_t x0 = node(lox), y0 = node(loy);
  const lvl_t l = lv[L];
  const bool beside = (hix < 0.0f) | (hiy < 0.0f) | (x0 > l.w1) | (y0 > l.h1);
  // index clamped into the level, so every lane's load is valid; tiled
  // index (tci_tile_index) with a 24-bit multiply: tile rows and tiles per
  // row are below 2^11
  const uint32_t i = (uint32_t)clamp0(x0, l.w1), j = (uint32_t)clamp0(y0, l.h1);
  const uint32_t w = map_word(m.base, woff[L] + ((umul24(j >> 3, (uint32_t)l.tiles_x) + (i >> 3)) << 6) +
                                          ((j & 7) << 3) + (i & 7));
  const bool test = !bad & !above & !huge & !wide & !beside;
  reads += test ? 1 : 0;
  // a window without a slab has smin = 255 > smax = 0, which fails the
  // slab test
  const bool solid = (loz <= (float)(w & 0xFF)) |
                     ((loz <= (float)((w >> 16) & 0xFF)) & (hiz >= (float)((w >> 8) & 0xFF)));
  return bad | (!above & (huge | wide | (!beside & solid)));
}

// Parameter t >= 0 such that no ray of the packet whose tile is (tx, ty)
// meets solid during [0, t].  Called by all 64 lanes of the wave together
// (it uses ballots); `reads` gains the nodes this lane read.
__device__ __forceinline__ float beam_start(const tci_map& m, const lvl_t* lv,
                                            const uint32_t* woff, const tci_view& v,
                                            int32_t tx, int32_t ty, int32_t passes,
                                            int32_t lane, int32_t& reads) {
  const int32_t pw = v.pw_log2, ph = 6 - pw;
  const int32_t px0 = tx << pw, py0 = ty << ph;
  const int32_t px1 = min(px0 + (1 << pw) - 1, v.w - 1), py1 = min(py0 + (1 << ph) - 1, v.h - 1);
  // centre and half-spans of a and b over the packet's pixels
  const uint32_t ac = px0 + px1 + 1, bc = py0 + py1 + 1;
  const float inv = 1.0f / 65536.0f;
  const float ha = (float)(px1 - px0) * inv, hb = (float)(py1 - py0) * inv;
  // per coordinate, the bundle lies within lo(t) = A + t B, hi(t) = A' + t B'
  // for t >= 0: the centre ray oc + t dc plus or minus the extent bound
  // ha |opx + t dpx| + hb |opy + t dpy| <= e0 + t e1 (all over S).  Over
  // [t0, t1] their extremes are A + t0 B + (t1 - t0) min(B, 0) and
  // A' + t0 B' + (t1 - t0) max(B', 0).  The margin covers the rounding of
  // the view's values, of these coefficients and of the bounds (a few
  // units in the last place of values below 2^16) plus an absolute
  // sixteenth of a cell: 1/16 + 2^-18 (|lo| + |hi|) is at most
  // P + t1 Q with P = 1/16 + 2^-18 (|A| + |A'|), Q = 2^-18 (|B| + |B'|),
  // which folds into the coefficients:
  //   lo = (A - P) + t0 (B - Q) + (t1 - t0) (min(B, 0) - Q)
  //   hi = (A' + P) + t0 (B' + Q) + (t1 - t0) (max(B', 0) + Q)
  float L0[3], L1[3], L2[3], H0[3], H1[3], H2[3], len2 = 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    // the centre ray lies between the view's corner rays, which fit in 32
    // bits: wrapping 32-bit arithmetic gives it exactly
    const float oc =
        (float)(int32_t)((uint32_t)v.o0[c] + ac * (uint32_t)v.opx[c] + bc * (uint32_t)v.opy[c]) *
        inv;
    const float dc =
        (float)(int32_t)((uint32_t)v.d0[c] + ac * (uint32_t)v.dpx[c] + bc * (uint32_t)v.dpy[c]) *
        inv;
    const float e0 = fmaf(ha, fabsf((float)v.opx[c]), hb * fabsf((float)v.opy[c]));
    const float e1 = fmaf(ha, fabsf((float)v.dpx[c]), hb * fabsf((float)v.dpy[c]));
    const float A = oc - e0, Ah = oc + e0, B = dc - e1, Bh = dc + e1;
    const float P = fmaf(fabsf(A) + fabsf(Ah), 0x1p-18f, 0.0625f);
    const float Q = (fabsf(B) + fabsf(Bh)) * 0x1p-18f;
    L0[c] = A - P;
    L1[c] = B - Q;
    L2[c] = fminf(B, 0.0f) - Q;
    H0[c] = Ah + P;
    H1[c] = Bh + Q;
    H2[c] = fmaxf(Bh, 0.0f) + Q;
    len2 = fmaf(dc, dc, len2);
  }
  if (!(len2 > 0.0f)) return 0.0f;
  // the interval lengths need no accuracy: the hardware's reciprocal square
  // root and power of two
  const float u = kBeamFirst * __builtin_amdgcn_rsqf(len2);
  // lane k covers [ta + u g(k), ta + u g(k + 1)], g(k) = ((1 + r)^k - 1) / r;
  // lane k's end and lane k + 1's start are the same float (same inputs,
  // same operations), so the intervals leave no gap
  const float g0 = (__builtin_amdgcn_exp2f((float)lane * kBeamLog2Growth) - 1.0f) *
                   (1.0f / kBeamGrowth);
  const float g1 = (__builtin_amdgcn_exp2f((float)(lane + 1) * kBeamLog2Growth) - 1.0f) *
                   (1.0f / kBeamGrowth);
  float ta = 0.0f;
  for (int32_t pass = 0; pass < passes; ++pass) {
    const float t0 = fmaf(u, g0, ta), t1 = fmaf(u, g1, ta), dt = t1 - t0;
    float lo[3], hi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmaf(dt, L2[c], fmaf(t0, L1[c], L0[c]));
      hi[c] = fmaf(dt, H2[c], fmaf(t0, H1[c], H0[c]));
    }
    const bool solid =
        beam_box_solid(m, lv, woff, lo[0], hi[0], lo[1], hi[1], lo[2], hi[2], reads);
    const uint64_t bad = __ballot(solid);
    if (bad & 1ull) break;                         // no progress
    const int32_t k = bad ? __ffsll((unsigned long long)bad) - 1 : 63;
    const float next = bad ? t0 : t1;
    ta = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(next), k));
  }
  return ta;
}

// Index-form constants of ray r, and its walk state at the last cell line
// of its dominant axis that it enters no later than parameter t
// (beam_start: no solid lies on the ray up to t, nor within the boxes'
// margin beyond it), at level 0: such a ray is close to solid, where coarse
// nodes would only be descended again; at the origin and level L0 if that
// line is the start cell's.  The line comes from O + t D in
// double precision: t, D and O are exact there and the one rounding of the
// fma moves the entry by less than 2^-20 S units, far inside the margin.
__device__ __forceinline__ void start_walk(ray_t& r, walk_idx_t& k, walk_t& s, float t,
                                           int32_t L0, int32_t W, int32_t H) {
  walk_origin(r, k);
  if (t > 0.0f) {
    const bool ax_x = r.ax >= r.ay;
    const int64_t O = ax_x ? r.Ox : r.Oy;
    const int32_t D = ax_x ? r.Dx : r.Dy;
    const int32_t n = ax_x ? W : H;
    const double q = fma((double)t, (double)D, (double)O) * (1.0 / 65536.0);
    // (walk_at_line declines a line that is not ahead of the origin's)
    const int32_t c = D > 0
        ? (int32_t)floor(fmax(fmin(q, (double)n), -1048576.0))      // line c entered at x = c
        : (int32_t)ceil(fmin(fmax(q, 0.0), 1048576.0)) - 1;        // entered at x = c + 1
    if (walk_at_line(r, k, s, ax_x ? 0 : 1, c)) return;
  }
  walk_at_origin(r, L0, s);
}

}  // namespace
