// Ray casting kernels: one thread per pixel over 8x8 pixel packets, the
// split pass for the longest walks, and persistent packet-queue waves.  The
// walk itself (tc_walk.h) is the exact cell sequence of a 2D digital
// differential analyser over the map, accelerated by the per-layer min/max
// pyramid (Section 3.1 SOLID and RAYMARCH, Section 3.2 skip-to-exit).
#include <hip/hip_ext.h>

#include "tc_beam.h"
#include "tc_packet.h"

namespace {

// 8x8 pixel packets (waves) per block of the one-thread-per-pixel kernels.
// Measured on the headline view: two give 1.8 % faster frames than four,
// one 0.4 %.
constexpr int32_t kPackets = 2;

// This lane's index in its wave, from the hardware (two VALU instructions)
// rather than from a register kept live.
__device__ __forceinline__ int32_t lane_now() {
  return (int32_t)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// One thread per pixel; a wave casts one packet of 64 pixels.
// kOcc: node tests also consult the occupancy masks (render mode 4).
// kVox: nodes above the cells are tested against the voxel occupancy
// pyramid *vx instead (render mode 5, the voxel-accelerated march).
// kCount: the launch counts the nodes and cells its rays read (o.count);
// the production instance keeps no counter through the walk.
template <bool kFlat, bool kOcc, bool kCount, bool kVox = false>
__device__ __forceinline__ void render_body(
    const tci_map& m, const tci_view* __restrict__ views, int32_t nviews,
    const int64_t* __restrict__ pkt_prefix, const int32_t* __restrict__ rows, int64_t npkt,
    void* out, const tci_render_opts& o, const tci_voxels* vx = nullptr) {
  __shared__ lvl_t lv[TCI_MAX_LEVELS];
  __shared__ uint32_t woff[TCI_MAX_LEVELS];
  __shared__ uint32_t moff[kOcc ? TCI_MAX_LEVELS : 1];
  load_levels_beam(m, lv, woff, kOcc ? moff : nullptr);
  // clear the queue counter the next render of this ring slot will use
  // (its last user finished before this launch)
  if (o.qzero && blockIdx.x == 0 && threadIdx.x == 0) *o.qzero = 0u;
  // XCD-aware order: hand each XCD a contiguous range of packets to share
  // its L2
  const int64_t b = tcp::xcd_block(blockIdx.x, gridDim.x, o.xcd_remap);
  // the packet is the wave's: keep its index, view and tile in scalar
  // registers
  const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t p = b * kPackets + wave;
  if (p >= npkt) return;
  const int32_t vi = __builtin_amdgcn_readfirstlane(tcp::find_view(pkt_prefix, nviews, p));
  const tci_view& v = views[vi];
  int32_t tx, ty;
  tcp::packet_tile(v, p - v.pkt_base, o.tile_order, rows, tx, ty);
  tx = __builtin_amdgcn_readfirstlane(tx);
  ty = __builtin_amdgcn_readfirstlane(ty);
  const int32_t pw = v.pw_log2;
  const int32_t px = (tx << pw) + (lane & ((1 << pw) - 1)), py = (ty << (6 - pw)) + (lane >> pw);
  // the packet's common start (all 64 lanes take part)
  float t_start = 0.0f;
  int32_t beam_reads = 0;
  if (!kFlat && o.beam_passes > 0)
    t_start = beam_start(m, lv, woff, v, tx, ty, o.beam_passes, lane, beam_reads);
  if (px >= v.w || py >= v.h) {
    if (kCount && beam_reads) atomicAdd(o.count, (unsigned long long)beam_reads);
    return;
  }
  ray_t r;
  packet_ray(v, tx, ty, lane, r);
  uint32_t word;
  float depth;
  if (r.Dx == 0 && r.Dy == 0) {
    trace_vertical(m, lv, r, word, depth);
    if (kCount && beam_reads) atomicAdd(o.count, (unsigned long long)beam_reads);
  } else {
    walk_t s;
    walk_idx_t k;
    const int32_t top = kFlat ? 0 : m.top;
    start_walk(r, k, s, t_start, kFlat ? 0 : clamp_level(o.start_level, top), m.W, m.H);
    s.reads = beam_reads;
    uint32_t col = 0;
    const int32_t Lmax = kFlat ? 0 : clamp_level(o.max_level, top);
    const int32_t boost = __builtin_amdgcn_readfirstlane(o.boost);
    bool split = !kFlat && o.split_budget > 0 && o.qcap > 0;
    // the walk runs a loop specialised to the sign of the ray's vertical
    // direction (a packet's rays mostly share it; a wave holding both signs
    // runs the two loops one after the other)
    const bool down = r.Dz < 0;
    int32_t st;
    for (;;) {
      // the budget bounds the walk: at most the split budget, then (or
      // without a split pass) kIterCap + 1 iterations
      const int32_t budget = split ? o.split_budget : kIterCap + 1;
      if (down)
        st = walk_steps<false, kOcc, false, 1, kVox>(m, lv, r, k, s, Lmax, budget, col, boost,
                                                     0, 0, 0, moff, kCount, vx);
      else
        st = walk_steps<false, kOcc, false, 2, kVox>(m, lv, r, k, s, Lmax, budget, col, boost,
                                                     0, 0, 0, moff, kCount, vx);
      if (!split) break;
      split = false;
      // long walks go to the split pass, as many as the queue holds
      const uint64_t want = __ballot(st == kWalking);
      if (!want) break;
      const uint64_t act = __ballot(1);
      const int32_t leader = __ffsll((unsigned long long)act) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(o.qcount, (uint32_t)__popcll(want));
      base = __shfl(base, leader);
      if (st != kWalking) break;
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
          (uint32_t)(want >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)want, 0));
      if (base + rank < o.qcap) {
        // the walk has reached the current node: the second pass need only
        // split the path from the node's near line on the dominant axis
        const bool ax_x = r.ax >= r.ay;
        // the start cell's line, selected here: selected before the walk it
        // would hold one more register through it
        int32_t cx = r.cx0, cy = r.cy0;
        asm volatile("" : "+v"(cx), "+v"(cy));
        const int32_t n = ax_x ? s.ni : s.nj, c0 = ax_x ? cx : cy;
        const bool fwd = (ax_x ? r.Dx : r.Dy) > 0;
        const int32_t near = fwd ? (n << s.L) : ((n + 1) << s.L) - 1;
        const int32_t from = fwd ? max(near, c0) : min(near, c0);
        o.queue[base + rank] = make_uint4((uint32_t)vi, (uint32_t)(py * v.w + px),
                                          (uint32_t)from, 0u);
        if (kCount) atomicAdd(o.count, (unsigned long long)s.reads);
        return;
      }
    }
    if (st == kWalking) st = kCapped;   // the whole budget ran out (never expected)
    // the origin is needed again only here: recompute it from the view
    // rather than keep it in registers through the walk (the lane index is
    // read again from the hardware, so no register holds it either)
    packet_ray<false>(v, tx, ty, lane_now(), r);
    finish(r, s, m.W, st, col, word, depth);
    if (kCount) atomicAdd(o.count, (unsigned long long)s.reads);
  }
  const int32_t ql = lane_now(), qw = v.pw_log2;
  tcp::store_hit(out, v.out_base + (int64_t)((ty << (6 - qw)) + (ql >> qw)) * v.w + (tx << qw) +
                          (ql & ((1 << qw) - 1)),
                 word, depth);
}

// The three one-thread-per-pixel kernels, each with and without read
// counting.  The hierarchical one is asked for at least 7 waves per SIMD
// (at most 72 VGPRs): each walk step waits on its node load and the
// arithmetic after it, so more waves hide more of that latency.  The
// production instance (no counting) fits 64 VGPRs, enough for 8 waves.
template <bool kCount>
__global__ __launch_bounds__(64 * kPackets) __attribute__((amdgpu_waves_per_eu(7, 8)))
void render_hier_kernel(tci_map m, const tci_view* __restrict__ views, int32_t nviews,
                        const int64_t* __restrict__ pkt_prefix, int64_t npkt, void* out,
                        tci_render_opts o) {
  render_body<false, false, kCount>(m, views, nviews, pkt_prefix, o.rows, npkt, out, o);
}

// The same, with the call's view records, packet prefix and tile-row table
// passed in the kernel's arguments instead of a device table (a small call
// then needs no upload before its render).
__global__ __launch_bounds__(64 * kPackets) __attribute__((amdgpu_waves_per_eu(7, 8)))
void render_hier_inline_kernel(tci_map m, int32_t nviews, int64_t npkt, void* out,
                               tci_render_opts o, tci_inline t) {
  const char* b = (const char*)t.words;
  render_body<false, false, false>(m, (const tci_view*)b, nviews,
                                   (const int64_t*)(b + t.off_prefix),
                                   (const int32_t*)(b + t.off_rows), npkt, out, o);
}

template <bool kCount>
__global__ __launch_bounds__(64 * kPackets)
void render_flat_kernel(tci_map m, const tci_view* __restrict__ views, int32_t nviews,
                        const int64_t* __restrict__ pkt_prefix, int64_t npkt, void* out,
                        tci_render_opts o) {
  render_body<true, false, kCount>(m, views, nviews, pkt_prefix, o.rows, npkt, out, o);
}

template <bool kCount>
__global__ __launch_bounds__(64 * kPackets)
void render_occ_kernel(tci_map m, const tci_view* __restrict__ views, int32_t nviews,
                       const int64_t* __restrict__ pkt_prefix, int64_t npkt, void* out,
                       tci_render_opts o) {
  render_body<false, true, kCount>(m, views, nviews, pkt_prefix, o.rows, npkt, out, o);
}

template <bool kCount>
__global__ __launch_bounds__(64 * kPackets)
void render_vox_kernel(tci_map m, const tci_view* __restrict__ views, int32_t nviews,
                       const int64_t* __restrict__ pkt_prefix, int64_t npkt, void* out,
                       tci_render_opts o, tci_voxels vx) {
  render_body<false, false, kCount, true>(m, views, nviews, pkt_prefix, o.rows, npkt, out, o,
                                          &vx);
}

// Dominant-axis cell line where the ray leaves the map's columns, or rises
// above every height, estimated in double precision (only the sizes of the
// split segments depend on it).
__device__ __forceinline__ int32_t exit_line(const ray_t& r, const tci_map& m,
                                             int32_t axis) {
  const double S = 65536.0;
  double t = 1e300;
  if (r.Dx > 0) t = fmin(t, ((double)m.W * S - (double)r.Ox) / r.Dx);
  if (r.Dx < 0) t = fmin(t, (double)r.Ox / -(double)r.Dx);
  if (r.Dy > 0) t = fmin(t, ((double)m.H * S - (double)r.Oy) / r.Dy);
  if (r.Dy < 0) t = fmin(t, (double)r.Oy / -(double)r.Dy);
  if (r.Dz > 0) t = fmin(t, (256.0 * S - (double)r.Oz) / r.Dz);
  t = fmax(t, 0.0);
  const double c = axis == 0 ? ((double)r.Ox + t * r.Dx) / S : ((double)r.Oy + t * r.Dy) / S;
  const double lim = axis == 0 ? (double)m.W : (double)m.H;
  return (int32_t)floor(fmin(fmax(c, -1.0), lim));
}

// Split pass: G = split_waves (1, 2 or 4) waves of one block per queued
// ray, 4 / G rays per block.  The ray's remaining dominant-axis cell lines
// are cut into 64 G runs (the last one open-ended); lane k of the ray's
// wave g walks run 64 g + k from the exact state in which the flat walk
// enters it.  The earliest run with a hit holds the ray's first hit: inside
// a wave the first lane with a hit wins and the lanes after it stop; across
// the ray's waves, each wave with a hit lowers the ray's best run index in
// LDS and leaves its record there, a wave stops once an earlier wave has a
// hit, and after a barrier the ray's first wave writes the winner (or a
// miss).  Blocks stride over the queue; every wave of a block runs the
// same number of rounds, so the barriers are reached by all of them.
__device__ __forceinline__ void split_body(const tci_map& m,
                                           const tci_view* __restrict__ views, void* out,
                                           const tci_render_opts& o) {
  __shared__ lvl_t lv[TCI_MAX_LEVELS];
  __shared__ uint32_t best[4];      // per ray of the block: lowest run with a hit
  __shared__ uint2 cand[4];         // per wave: its first hit's record
  load_levels(m, lv);
  // every lane of a wave walks the same queued ray: the ray, its exit line
  // and its index-form constants are wave-uniform and stay in scalar
  // registers; only the runs' walk states are per lane
  const int32_t lane = threadIdx.x & 63;
  const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t G = (uint32_t)o.split_waves, per = 4 / G;
  const uint32_t grp = (uint32_t)wave / G, g = (uint32_t)wave - grp * G;
  const int32_t lgR = 6 + (G == 4 ? 2 : (G == 2 ? 1 : 0));   // 64 G runs per ray
  const uint32_t n = min(*o.qcount, o.qcap);
  const lvl_t l0 = lv[0];
  for (uint32_t e0 = blockIdx.x * per; e0 < n; e0 += gridDim.x * per) {
    const uint32_t e = e0 + grp;
    if (threadIdx.x < 4) best[threadIdx.x] = 0xFFFFFFFFu;
    __syncthreads();
    uint32_t qv = 0, qp = 0;
    if (e < n) {
      const uint4 q = o.queue[e];
      qv = __builtin_amdgcn_readfirstlane(q.x);
      qp = __builtin_amdgcn_readfirstlane(q.y);
      const tci_view& v = views[qv];
      const int32_t px = (int32_t)(qp % (uint32_t)v.w), py = (int32_t)(qp / (uint32_t)v.w);
      ray_t r;
      pixel_ray(v, px, py, r);
      const int32_t axis = r.ax >= r.ay ? 0 : 1;
      const int32_t c0 = (int32_t)__builtin_amdgcn_readfirstlane(q.z);  // first line still to walk
      const int32_t dir = (axis == 0 ? r.Dx : r.Dy) > 0 ? 1 : -1;
      const int32_t last = __builtin_amdgcn_readfirstlane(exit_line(r, m, axis));
      // lines still to walk (below 2^17), cut into 2^lgR runs
      const int32_t N = max(1, (last - c0) * dir + 1);
      const int32_t j = 64 * (int32_t)g + lane;          // this lane's run
      const int32_t b0 = c0 + dir * ((j * N) >> lgR);
      const int32_t b1 = c0 + dir * (((j + 1) * N) >> lgR);
      const bool open = j == (1 << lgR) - 1;
      int32_t lo = INT32_MIN, hi = INT32_MAX;
      if (!open) {
        if (dir > 0) hi = b1 - 1; else lo = b1 + 1;
      }
      walk_idx_t k;
      walk_origin(r, k);
      k.KX0 = rfl64(k.KX0);
      k.KY0 = rfl64(k.KY0);
      k.ZX0 = rfl64(k.ZX0);
      k.ZY0 = rfl64(k.ZY0);
      k.offx = __builtin_amdgcn_readfirstlane(k.offx);
      k.offy = __builtin_amdgcn_readfirstlane(k.offy);
      r.rx = __builtin_amdgcn_readfirstlane(r.rx);
      r.ry = __builtin_amdgcn_readfirstlane(r.ry);
      walk_t s;
      uint32_t col = 0;
      int32_t st = kSegEnd;
      if (open || b0 != b1) {
        // a run spans a few cell lines close to the terrain, where coarse
        // nodes would only be descended again: it walks the cells
        if (!walk_at_line(r, k, s, axis, b0)) walk_at_origin(r, 0, s);
        st = kWalking;
      }
      // walk in chunks of 10 cells, each chunk's columns loaded together
      // before it is tested; once some run holds a hit, the runs after it
      // cannot matter and stop.  The ray's vertical direction is the
      // wave's, so the loop is specialised to its sign.
      const bool down = r.Dz < 0;
      for (;;) {
        const uint64_t hit_now = __ballot(st == kHitCell || st == kCapped);
        const int32_t first = hit_now ? __ffsll((unsigned long long)hit_now) - 1 : 64;
        if (st == kWalking && (lane > first || *(volatile uint32_t*)&best[grp] < 64 * g))
          st = kSegEnd;
        if (!__ballot(st == kWalking)) break;
        if (st == kWalking) {
          if (down)
            st = walk_flat<1, 10>(m, l0, r, k, s, col, axis, lo, hi, o.count != nullptr);
          else
            st = walk_flat<2, 10>(m, l0, r, k, s, col, axis, lo, hi, o.count != nullptr);
        }
      }
      if (o.count && (open || b0 != b1)) atomicAdd(o.count, (unsigned long long)s.reads);
      const uint64_t hits = __ballot(st == kHitCell || st == kCapped);
      if (hits && lane == __ffsll((unsigned long long)hits) - 1) {
        uint32_t word;
        float depth;
        finish(r, s, m.W, st, col, word, depth);
        cand[wave] = make_uint2(word, __float_as_uint(depth));
        atomicMin(&best[grp], 64 * g + (uint32_t)lane);
      }
    }
    __syncthreads();
    if (e < n && g == 0 && lane == 0) {
      const uint32_t b = best[grp];
      const int64_t idx = views[qv].out_base + qp;
      if (b == 0xFFFFFFFFu) {
        tcp::store_hit(out, idx, kMiss, __builtin_inff());
      } else {
        const uint2 c = cand[grp * G + (b >> 6)];
        tcp::store_hit(out, idx, c.x, __uint_as_float(c.y));
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void split_kernel(tci_map m,
                                                    const tci_view* __restrict__ views,
                                                    void* out, tci_render_opts o) {
  split_body(m, views, out, o);
}

// The split pass of a render whose tables came in the kernel's arguments.
__global__ __launch_bounds__(256) void split_inline_kernel(tci_map m, void* out,
                                                           tci_render_opts o, tci_inline t) {
  split_body(m, (const tci_view*)(const char*)t.words, out, o);
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
  walk_idx_t k;
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
          const int32_t vi = tcp::find_view(pkt_prefix, nviews, mypkt);
          const tci_view& v = views[vi];
          int32_t px, py;
          tcp::packet_pixel(v, mypkt - v.pkt_base, myray, o.tile_order, o.rows, px, py);
          if (px < v.w && py < v.h) {
            pixel_ray(v, px, py, r);
            out_idx = v.out_base + (int64_t)py * v.w + px;
            if (r.Dx == 0 && r.Dy == 0) {
              uint32_t word;
              float depth;
              trace_vertical(m, lv, r, word, depth);
              tcp::store_hit(out, out_idx, word, depth);
            } else {
              walk_origin(r, k);
              walk_at_origin(r, L0, s);
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
    if (active) st = walk_steps(m, lv, r, k, s, Lmax, iters, col);
    if (st != kWalking) {
      uint32_t word;
      float depth;
      finish(r, s, m.W, st, col, word, depth);
      tcp::store_hit(out, out_idx, word, depth);
      if (o.count) atomicAdd(o.count, (unsigned long long)s.reads);
      active = false;
    }
  }
}

}  // namespace

hipError_t tci_launch_render(const tci_map& m, const tci_view* views,
                             int32_t nviews, const int64_t* pkt_prefix,
                             int64_t npkt, void* out, int32_t flat,
                             const tci_render_opts& o, hipStream_t s,
                             const tci_voxels* vx) {
  int64_t blocks = (npkt + kPackets - 1) / kPackets;
  if (blocks < 1) return hipSuccess;
  const bool c = o.count != nullptr;
  if (flat == 3) {
    if (!vx) return hipErrorInvalidValue;
    hipLaunchKernelGGL(c ? render_vox_kernel<true> : render_vox_kernel<false>,
                       dim3((uint32_t)blocks), dim3(64 * kPackets), 0, s, m, views, nviews,
                       pkt_prefix, npkt, out, o, *vx);
    return hipGetLastError();
  }
  auto kern = flat == 1 ? (c ? render_flat_kernel<true> : render_flat_kernel<false>)
            : flat == 2 ? (c ? render_occ_kernel<true> : render_occ_kernel<false>)
                        : (c ? render_hier_kernel<true> : render_hier_kernel<false>);
  hipLaunchKernelGGL(kern, dim3((uint32_t)blocks), dim3(64 * kPackets), 0, s, m, views, nviews,
                     pkt_prefix, npkt, out, o);
  return hipGetLastError();
}

hipError_t tci_launch_split(const tci_map& m, const tci_view* views,
                            const tci_render_opts& o, void* out, int32_t nblocks,
                            hipStream_t s, const tci_inline* t, hipEvent_t ev_start,
                            hipEvent_t ev_stop) {
  if (t && (ev_start || ev_stop))
    hipExtLaunchKernelGGL(split_inline_kernel, dim3(nblocks), dim3(256), 0, s, ev_start, ev_stop,
                          0, m, out, o, *t);
  else if (t)
    hipLaunchKernelGGL(split_inline_kernel, dim3(nblocks), dim3(256), 0, s, m, out, o, *t);
  else
    hipLaunchKernelGGL(split_kernel, dim3(nblocks), dim3(256), 0, s, m, views, out, o);
  return hipGetLastError();
}

hipError_t tci_launch_render_inline(const tci_map& m, int32_t nviews, int64_t npkt, void* out,
                                    const tci_render_opts& o, const tci_inline& t,
                                    hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
  const int64_t blocks = (npkt + kPackets - 1) / kPackets;
  if (blocks < 1) return hipSuccess;
  if (ev_start || ev_stop)
    hipExtLaunchKernelGGL(render_hier_inline_kernel, dim3((uint32_t)blocks), dim3(64 * kPackets),
                          0, s, ev_start, ev_stop, 0, m, nviews, npkt, out, o, t);
  else
    hipLaunchKernelGGL(render_hier_inline_kernel, dim3((uint32_t)blocks), dim3(64 * kPackets), 0,
                       s, m, nviews, npkt, out, o, t);
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
