// Host-side planning of the library's calls (see tc_plan.h).  Plain C++,
// no HIP: the sanitizer test builds this file with g++.
#include "tc_plan.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

namespace tci {

namespace {

// TC_INVALID_ARG with a formatted reason in *err.
tc_status fail(std::string* err, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (err) *err = buf;
  return TC_INVALID_ARG;
}

}  // namespace

bool columns_valid(const uint8_t* F, const uint8_t* B, const uint8_t* T,
                   int32_t w, int32_t h, size_t stride, int32_t* bad_x,
                   int32_t* bad_y) {
  for (int32_t y = 0; y < h; ++y) {
    const uint8_t* f = F + (size_t)y * stride;
    const uint8_t* b = B + (size_t)y * stride;
    const uint8_t* t = T + (size_t)y * stride;
    for (int32_t x = 0; x < w; ++x) {
      bool ok = b[x] == 0 ? t[x] == 0 : (b[x] > f[x] && t[x] >= b[x]);
      if (!ok) {
        *bad_x = x;
        *bad_y = y;
        return false;
      }
    }
  }
  return true;
}

int32_t top_level(int32_t W, int32_t H) {
  int32_t m = std::max(W, H), L = 0;
  while ((1 << L) < m) ++L;
  return L;
}

tci_map layout_map(int32_t W, int32_t H, size_t* words_out) {
  tci_map d{};
  d.W = W;
  d.H = H;
  d.top = top_level(W, H);
  size_t words = 0;
  for (int32_t L = 0; L < TCI_MAX_LEVELS; ++L) {
    tci_level& l = d.lv[L];
    if (L > d.top) {
      l = tci_level{0, 0, 0, 0};
      continue;
    }
    l.w = (int32_t)(((int64_t)W + (1 << L) - 1) >> L);
    l.h = (int32_t)(((int64_t)H + (1 << L) - 1) >> L);
    l.tiles_x = (l.w + 7) >> 3;
    l.off = (uint32_t)words;
    words += (size_t)l.tiles_x * ((l.h + 7) >> 3) * 64;
  }
  // occupancy masks of levels 1..top after the pyramid, 2 words a node
  for (int32_t L = 0; L < TCI_MAX_LEVELS; ++L) {
    tci_level& k = d.mk[L];
    k = tci_level{0, 0, 0, 0};
    if (L < 1 || L > d.top) continue;
    k = d.lv[L];
    k.off = (uint32_t)words;
    words += (size_t)k.tiles_x * ((k.h + 7) >> 3) * 128;
  }
  // window levels 0..top after the masks, one word an entry, tiled like
  // the level they summarise
  for (int32_t L = 0; L < TCI_MAX_LEVELS; ++L) {
    tci_level& k = d.wl[L];
    k = tci_level{0, 0, 0, 0};
    if (L > d.top) continue;
    k = d.lv[L];
    k.off = (uint32_t)words;
    words += (size_t)k.tiles_x * ((k.h + 7) >> 3) * 64;
  }
  *words_out = words;
  return d;
}

tci_voxels layout_voxels(int32_t W, int32_t H, int32_t v_log2, int32_t vz_log2,
                         size_t* words_out) {
  tci_voxels x{};
  x.v_log2 = v_log2;
  x.vz_log2 = vz_log2;
  int32_t nx = (int32_t)(((int64_t)W + (1 << v_log2) - 1) >> v_log2);
  int32_t ny = (int32_t)(((int64_t)H + (1 << v_log2) - 1) >> v_log2);
  int32_t nz = 256 >> vz_log2;
  size_t words = 0;
  int32_t k = 0;
  for (;; ++k) {
    tci_vlevel& l = x.lv[k];
    l.nx = nx;
    l.ny = ny;
    l.nz = nz;
    l.tiles_x = (nx + 7) >> 3;
    l.tiles_y = (ny + 7) >> 3;
    l.tiles_z = (nz + 7) >> 3;
    l.off = (uint32_t)words;
    words += (size_t)l.tiles_x * l.tiles_y * l.tiles_z * 16;
    if ((nx == 1 && ny == 1 && nz == 1) || k == TCI_MAX_LEVELS - 1) break;
    nx = (nx + 1) >> 1;
    ny = (ny + 1) >> 1;
    nz = (nz + 1) >> 1;
  }
  x.levels = k + 1;
  *words_out = words;
  return x;
}

tc_status check_edits(const tc_edit* edits, int32_t n, size_t* patch_bytes,
                      std::string* err) {
  if (n < 0 || n > 65536) return fail(err, "edits: bad n %d", n);
  if (n > 0 && !edits) return fail(err, "edits: list is NULL");
  size_t pb = 0;
  for (int32_t i = 0; i < n; ++i) {
    const tc_edit& e = edits[i];
    if (e.kind == TC_EDIT_SET) {
      if (e.w < 1 || e.h < 1 || e.w > TC_MAX_DIM || e.h > TC_MAX_DIM)
        return fail(err, "edits: edit %d bad size", i);
      if (!e.floor_top || !e.slab_bottom || !e.slab_top)
        return fail(err, "edits: edit %d null patch", i);
      int32_t bx, by;
      if (!columns_valid(e.floor_top, e.slab_bottom, e.slab_top, e.w, e.h, e.w, &bx, &by))
        return fail(err,
                    "edits: edit %d patch cell (%d,%d) violates the column "
                    "invariants", i, bx, by);
      pb += (size_t)3 * e.w * e.h;
    } else if (e.kind == TC_EDIT_CRATER) {
      if (e.w < 1 || e.w > 4096 || e.h != e.w)
        return fail(err, "edits: edit %d bad crater size", i);
      if (e.depth < 0 || e.depth > 255)
        return fail(err, "edits: edit %d bad crater depth", i);
    } else {
      return fail(err, "edits: edit %d bad kind %d", i, e.kind);
    }
    if ((int64_t)e.x0 + e.w > INT32_MAX || (int64_t)e.y0 + e.h > INT32_MAX ||
        e.x0 < -(1 << 28) || e.y0 < -(1 << 28))
      return fail(err, "edits: edit %d rectangle overflows", i);
  }
  *patch_bytes = pb;
  return TC_OK;
}

namespace {

// For every edit, the other edits whose clipped rectangles ([x0, x1) x
// [y0, y1), empty for an edit wholly outside the map) meet its own, in
// ascending order: start[n + 1], then the lists.  Candidates come from a
// grid of 128 x 128-cell buckets (every pair for short lists); false if
// they would be too many to list (a bucket with more than 512 edits, or
// more than 8 n + 2^20 entries), and the edits kernel then tests every
// edit against every other.
bool edit_overlaps(const std::vector<int32_t>& cr, int32_t n, std::vector<int32_t>& out) {
  auto live = [&](int32_t i) { return cr[4 * i] < cr[4 * i + 2] && cr[4 * i + 1] < cr[4 * i + 3]; };
  auto meet = [&](int32_t i, int32_t j) {
    return cr[4 * i] < cr[4 * j + 2] && cr[4 * j] < cr[4 * i + 2] &&
           cr[4 * i + 1] < cr[4 * j + 3] && cr[4 * j + 1] < cr[4 * i + 3];
  };
  const size_t cap = 8 * (size_t)n + ((size_t)1 << 20);
  std::vector<std::vector<int32_t>> lists(n);
  size_t total = 0;
  if (n <= 64) {
    for (int32_t i = 0; i < n; ++i)
      for (int32_t j = 0; j < n; ++j)
        if (j != i && live(i) && live(j) && meet(i, j)) lists[i].push_back(j);
  } else {
    constexpr int32_t kB = 7;   // 128-cell buckets
    std::vector<std::pair<int64_t, int32_t>> keys;
    for (int32_t i = 0; i < n; ++i) {
      if (!live(i)) continue;
      const int64_t bx0 = cr[4 * i] >> kB, by0 = cr[4 * i + 1] >> kB;
      const int64_t bx1 = (cr[4 * i + 2] - 1) >> kB, by1 = (cr[4 * i + 3] - 1) >> kB;
      if ((size_t)((bx1 - bx0 + 1) * (by1 - by0 + 1)) + keys.size() > cap) return false;
      for (int64_t by = by0; by <= by1; ++by)
        for (int64_t bx = bx0; bx <= bx1; ++bx) keys.emplace_back((by << 20) | bx, i);
    }
    std::sort(keys.begin(), keys.end());
    for (size_t a = 0; a < keys.size();) {
      size_t b = a;
      while (b < keys.size() && keys[b].first == keys[a].first) ++b;
      if (b - a > 512) return false;
      for (size_t u = a; u < b; ++u)
        for (size_t v = a; v < b; ++v)
          if (u != v && meet(keys[u].second, keys[v].second))
            lists[keys[u].second].push_back(keys[v].second);
      if ((total += (b - a) * (b - a)) > 64 * cap) return false;
      a = b;
    }
  }
  out.assign(n + 1, 0);
  total = 0;
  for (int32_t i = 0; i < n; ++i) {
    std::vector<int32_t>& l = lists[i];
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
    out[i] = (int32_t)total;
    total += l.size();
    if (total > cap) return false;
  }
  out[n] = (int32_t)total;
  for (int32_t i = 0; i < n; ++i) out.insert(out.end(), lists[i].begin(), lists[i].end());
  return true;
}

}  // namespace

void plan_edits(const tci_map& d, const tc_edit* edits, int32_t n,
                size_t patch_bytes, char* host, EditPlan& p) {
  const int32_t top = d.top;
  p.n = n;
  p.top = top;
  p.off_edits = 0;
  p.off_rects = (sizeof(tci_edit) * (size_t)n + 15) & ~(size_t)15;
  p.off_olap = p.off_rects + sizeof(int32_t) * 4 * (size_t)n * (size_t)(top + 1);
  std::vector<int32_t> cr(4 * (size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    const tc_edit& e = edits[i];
    cr[4 * i] = std::max(e.x0, 0);
    cr[4 * i + 1] = std::max(e.y0, 0);
    cr[4 * i + 2] = std::min(e.x0 + e.w, d.W);
    cr[4 * i + 3] = std::min(e.y0 + e.h, d.H);
  }
  p.olap_all = !edit_overlaps(cr, n, p.olap);
  if (p.olap_all) p.olap.assign(n + 1, 0);
  p.off_patch = (p.off_olap + sizeof(int32_t) * p.olap.size() + 15) & ~(size_t)15;
  p.total = p.off_patch + patch_bytes;
  if (host) memcpy(host + p.off_olap, p.olap.data(), sizeof(int32_t) * p.olap.size());
  p.nrect.assign(top + 1, 0);
  p.rmw.assign(top + 1, 1);
  p.rmh.assign(top + 1, 1);
  p.max_w = p.max_h = 1;
  tci_edit* he = host ? (tci_edit*)(host + p.off_edits) : nullptr;
  int32_t* hr = host ? (int32_t*)(host + p.off_rects) : nullptr;
  uint8_t* hp = host ? (uint8_t*)(host + p.off_patch) : nullptr;
  size_t po = 0;
  for (int32_t i = 0; i < n; ++i) {
    const tc_edit& e = edits[i];
    if (he) {
      tci_edit& o = he[i];
      o.kind = e.kind;
      o.x0 = e.x0;
      o.y0 = e.y0;
      o.w = e.w;
      o.h = e.h;
      o.depth = e.depth;
      o.data_off = (int64_t)po;
    }
    if (e.kind == TC_EDIT_SET) {
      size_t m = (size_t)e.w * e.h;
      if (hp) {
        memcpy(hp + po, e.floor_top, m);
        memcpy(hp + po + m, e.slab_bottom, m);
        memcpy(hp + po + 2 * m, e.slab_top, m);
      }
      po += 3 * m;
    }
    int32_t x0 = std::max(e.x0, 0), y0 = std::max(e.y0, 0);
    int32_t x1 = std::min(e.x0 + e.w, d.W), y1 = std::min(e.y0 + e.h, d.H);
    if (x0 >= x1 || y0 >= y1) continue;
    p.max_w = std::max(p.max_w, x1 - x0);
    p.max_h = std::max(p.max_h, y1 - y0);
    // the rectangle on every level, cells (level 0) included: the dirty
    // update of the pyramid reads levels 1..top, that of the window levels
    // all of them
    for (int32_t L = 0; L <= top; ++L) {
      int32_t r[4] = {x0 >> L, y0 >> L, (x1 - 1) >> L, (y1 - 1) >> L};
      if (hr) memcpy(hr + 4 * ((size_t)L * n + p.nrect[L]), r, sizeof(r));
      p.rmw[L] = std::max(p.rmw[L], r[2] - r[0] + 1);
      p.rmh[L] = std::max(p.rmh[L], r[3] - r[1] + 1);
      p.nrect[L]++;
    }
  }
}

tc_status make_view_plan(const PlanOpts& opt, const tc_view* views, int32_t n, ViewPlan& p,
                         bool allow_split, std::string* err) {
  if (n < 1 || !views) return fail(err, "render: no views");
  p.n = n;
  p.views.resize(n);
  p.prefix.resize((size_t)n + 1);
  int64_t out = 0, pk = 0;
  for (int32_t i = 0; i < n; ++i) {
    const tc_view& v = views[i];
    if (v.width < 1 || v.height < 1 || v.width > 16384 || v.height > 16384)
      return fail(err, "render: view %d bad size %dx%d", i, v.width, v.height);
    if (v.flags != 0) return fail(err, "render: view %d flags != 0", i);
    for (int cx = 0; cx < 2; ++cx)
      for (int cy = 0; cy < 2; ++cy) {
        int64_t a = cx ? 2 * (int64_t)v.width - 1 : 1;
        int64_t b = cy ? 2 * (int64_t)v.height - 1 : 1;
        for (int c = 0; c < 3; ++c) {
          int64_t O = (int64_t)v.o0[c] + a * v.o_px[c] + b * v.o_py[c];
          int64_t D = (int64_t)v.d0[c] + a * v.d_px[c] + b * v.d_py[c];
          if (O < INT32_MIN || O > INT32_MAX)
            return fail(err, "render: view %d origin overflows int32", i);
          if (D < -TC_MAX_DIR || D > TC_MAX_DIR)
            return fail(err, "render: view %d |direction| > 2^23-1", i);
        }
      }
    tci_view& o = p.views[i];
    o.w = v.width;
    o.h = v.height;
    for (int c = 0; c < 3; ++c) {
      o.o0[c] = v.o0[c]; o.opx[c] = v.o_px[c]; o.opy[c] = v.o_py[c];
      o.d0[c] = v.d0[c]; o.dpx[c] = v.d_px[c]; o.dpy[c] = v.d_py[c];
    }
    const int32_t pw = opt.packet_width == 4 ? 2 : opt.packet_width == 16 ? 4
                     : opt.packet_width == 32 ? 5 : 3;
    const int32_t ph = 6 - pw;
    o.pw_log2 = pw;
    o.tiles_x = (int32_t)(((int64_t)v.width + (1 << pw) - 1) >> pw);
    o.small_steps = 1;
    for (int c = 0; c < 3; ++c)
      for (int32_t st : {v.o_px[c], v.o_py[c], v.d_px[c], v.d_py[c]})
        if (st <= -(1 << 22) || st >= (1 << 22)) o.small_steps = 0;
    o.out_base = out;
    o.pkt_base = pk;
    o.rows_off = (int64_t)p.rows.size();
    // tile rows ordered by how level the ray through the row's centre is:
    // near-horizontal rays take the longest walks, so their packets start
    // first and do not trail the launch
    {
      const int32_t ty_n = (int32_t)(((int64_t)v.height + (1 << ph) - 1) >> ph);
      std::vector<std::pair<double, int32_t>> key((size_t)ty_n);
      const int64_t a = v.width;  // 2 * (width / 2) + 1, rounded
      for (int32_t ty = 0; ty < ty_n; ++ty) {
        const int64_t b =
            2 * (int64_t)std::min((ty << ph) + (1 << (ph - 1)), v.height - 1) + 1;
        const double dx = (double)v.d0[0] + (double)a * v.d_px[0] + (double)b * v.d_py[0];
        const double dy = (double)v.d0[1] + (double)a * v.d_px[1] + (double)b * v.d_py[1];
        const double dz = (double)v.d0[2] + (double)a * v.d_px[2] + (double)b * v.d_py[2];
        const double hz = std::sqrt(dx * dx + dy * dy);
        key[ty] = {hz > 0 ? std::fabs(dz) / hz : 1e30, ty};
      }
      std::stable_sort(key.begin(), key.end(),
                       [](const std::pair<double, int32_t>& x,
                          const std::pair<double, int32_t>& y) { return x.first < y.first; });
      for (auto& k : key) p.rows.push_back(k.second);
    }
    p.prefix[i] = pk;
    out += (int64_t)v.width * v.height;
    pk += (int64_t)o.tiles_x * (((int64_t)v.height + (1 << ph) - 1) >> ph);
  }
  p.prefix[n] = pk;
  if (out > ((int64_t)1 << 31))
    return fail(err, "render: more than 2^31 rays");
  p.rays = out;
  p.npkt = pk;
  p.off_views = 0;
  p.off_prefix = (sizeof(tci_view) * (size_t)n + 15) & ~(size_t)15;
  p.off_rows = (p.off_prefix + sizeof(int64_t) * ((size_t)n + 1) + 15) & ~(size_t)15;
  p.off_counter = (p.off_rows + sizeof(int32_t) * p.rows.size() + 15) & ~(size_t)15;
  // the split queue follows the counters (device only, never uploaded)
  p.qcap = (allow_split && opt.render_mode == 0 && opt.split_budget > 0)
               ? (uint32_t)std::min<int64_t>(out, opt.split_queue) : 0;
  p.off_queue = p.off_counter + 64;
  p.qwaves = opt.split_waves;
  p.total = p.off_queue + kQueueEntry * (size_t)p.qcap;
  return TC_OK;
}

void write_views(const ViewPlan& p, char* host) {
  memcpy(host + p.off_views, p.views.data(), sizeof(tci_view) * (size_t)p.n);
  memcpy(host + p.off_prefix, p.prefix.data(), sizeof(int64_t) * ((size_t)p.n + 1));
  memcpy(host + p.off_rows, p.rows.data(), sizeof(int32_t) * p.rows.size());
  memset(host + p.off_counter, 0, 64);
}

}  // namespace tci
