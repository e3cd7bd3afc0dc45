// Exercises the library's HIP-free planning layer (tc_plan.cpp: column
// validation, map layout, edit and view validation, and the layout of the
// tables a call uploads) on random and adversarial inputs, built with
// AddressSanitizer and UBSan (tests/test_sanitizers.py).  Every table is
// written into a buffer of exactly the planned size, so an offset past the
// end aborts the run.  It also checks the plans' invariants: aligned,
// ordered, non-overlapping regions; packet prefixes; one tile-row
// permutation per view; dirty rectangles inside their levels; the map
// levels inside the allocation.
//
// Usage: plan_sanitize [iterations] [seed]
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "tc_plan.h"

namespace {

uint64_t g_state;

uint64_t rnd() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int32_t rint_in(int32_t lo, int32_t hi) {  // [lo, hi]
  return lo + (int32_t)(rnd() % (uint64_t)((int64_t)hi - lo + 1));
}

int g_fails = 0;

#define CHECK(cond, ...)                \
  do {                                  \
    if (!(cond)) {                      \
      std::fprintf(stderr, __VA_ARGS__); \
      std::fputc('\n', stderr);         \
      ++g_fails;                        \
    }                                   \
  } while (0)

tc_view random_view(bool valid) {
  tc_view v;
  std::memset(&v, 0, sizeof(v));
  v.width = rint_in(1, rint_in(0, 9) == 0 ? 16384 : 300);
  v.height = rint_in(1, rint_in(0, 9) == 0 ? 4000 : 300);
  for (int c = 0; c < 3; ++c) {
    v.o0[c] = rint_in(-(1 << 24), 1 << 24);
    v.d0[c] = rint_in(-(1 << 20), 1 << 20);
    v.d_px[c] = rint_in(-64, 64);
    v.d_py[c] = rint_in(-64, 64);
  }
  if (!valid) {
    switch (rint_in(0, 5)) {
      case 0: v.width = rint_in(-5, 0); break;
      case 1: v.height = 16385 + rint_in(0, 100); break;
      case 2: v.flags = 1 + (uint32_t)rint_in(0, 7); break;
      case 3: {
        const int c = rint_in(0, 2);
        v.d0[c] = (1 << 23) + rint_in(0, 1000);
        v.d_px[c] = v.d_py[c] = 0;
        break;
      }
      case 4: v.o0[0] = 2147483647 - rint_in(0, 10); v.o_px[0] = 1 << 20; break;
      // pixel (0, 0)'s direction has y component 2^22 + 2^22 = 2^23, beyond
      // the limit whatever the view's size
      default: v.d_px[1] = (1 << 22); v.d0[1] = 1 << 22; v.d_py[1] = 0; break;
    }
  }
  return v;
}

struct Patch {
  std::vector<uint8_t> F, B, T;
};

tc_edit random_edit(int32_t W, int32_t H, std::vector<Patch>& keep, bool valid) {
  tc_edit e;
  std::memset(&e, 0, sizeof(e));
  e.x0 = rint_in(-70, W + 10);
  e.y0 = rint_in(-70, H + 10);
  if (rint_in(0, 1)) {
    e.kind = TC_EDIT_CRATER;
    e.w = e.h = rint_in(1, 64);
    e.depth = rint_in(0, 255);
  } else {
    e.kind = TC_EDIT_SET;
    e.w = rint_in(1, 40);
    e.h = rint_in(1, 40);
    keep.emplace_back();
    Patch& p = keep.back();
    const size_t m = (size_t)e.w * e.h;
    p.F.resize(m);
    p.B.resize(m);
    p.T.resize(m);
    for (size_t i = 0; i < m; ++i) {
      p.F[i] = (uint8_t)rint_in(0, 200);
      if (rint_in(0, 2) == 0) {
        p.B[i] = (uint8_t)rint_in(p.F[i] + 1, 254);
        p.T[i] = (uint8_t)rint_in(p.B[i], 255);
      }
    }
    e.floor_top = p.F.data();
    e.slab_bottom = p.B.data();
    e.slab_top = p.T.data();
  }
  if (!valid) {
    switch (rint_in(0, 4)) {
      case 0: e.kind = 7; break;
      case 1: e.kind = TC_EDIT_CRATER; e.w = 8; e.h = 9; break;
      case 2: e.kind = TC_EDIT_CRATER; e.w = e.h = 4; e.depth = 256; break;
      case 3: e.kind = TC_EDIT_SET; e.floor_top = nullptr; break;
      default:
        if (e.kind == TC_EDIT_SET) {
          keep.back().B[0] = 5;
          keep.back().F[0] = 9;   // B <= F with B > 0
        } else {
          e.w = e.h = 0;
        }
        break;
    }
  }
  return e;
}

void check_map_layout(int32_t W, int32_t H) {
  size_t words = 0;
  const tci_map d = tci::layout_map(W, H, &words);
  CHECK((1 << d.top) >= std::max(W, H) && (d.top == 0 || (1 << (d.top - 1)) < std::max(W, H)),
        "layout %dx%d: top %d", W, H, d.top);
  size_t end = 0;
  for (int32_t L = 0; L <= d.top; ++L) {
    const tci_level& l = d.lv[L];
    CHECK(l.w == (int32_t)(((int64_t)W + (1 << L) - 1) >> L), "layout level %d width", L);
    CHECK(l.off == end, "layout level %d offset %u, expected %zu", L, l.off, end);
    end = l.off + (size_t)l.tiles_x * ((l.h + 7) >> 3) * 64;
  }
  for (int32_t L = 1; L <= d.top; ++L) {
    const tci_level& k = d.mk[L];
    CHECK(k.off == end, "layout mask level %d offset", L);
    end = k.off + (size_t)k.tiles_x * ((k.h + 7) >> 3) * 128;
  }
  for (int32_t L = 0; L <= d.top; ++L) {
    const tci_level& k = d.wl[L];
    CHECK(k.off == end && k.w == d.lv[L].w && k.h == d.lv[L].h, "layout window level %d", L);
    end = k.off + (size_t)k.tiles_x * ((k.h + 7) >> 3) * 64;
  }
  CHECK(end == words, "layout %dx%d: %zu words planned, %zu used", W, H, words, end);
  CHECK(words < ((size_t)1 << 30), "layout %dx%d: byte offsets beyond 32 bits", W, H);
}

}  // namespace

int main(int argc, char** argv) {
  const int iters = argc > 1 ? std::atoi(argv[1]) : 500;
  g_state = argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 777;
  check_map_layout(16384, 8192);
  check_map_layout(1, 1);
  check_map_layout(2048, 16384);
  for (int it = 0; it < iters; ++it) {
    const int32_t W = rint_in(1, 3000), H = rint_in(1, 3000);
    check_map_layout(W, H);
    size_t words = 0;
    const tci_map d = tci::layout_map(W, H, &words);
    // columns
    {
      const int32_t w = rint_in(1, 30), h = rint_in(1, 30);
      const size_t stride = (size_t)w + rint_in(0, 5);
      std::vector<uint8_t> F(stride * h), B(stride * h), T(stride * h);
      for (size_t i = 0; i < F.size(); ++i) F[i] = (uint8_t)rint_in(0, 250);
      const bool bad = rint_in(0, 1);
      const int32_t bx = rint_in(0, w - 1), by = rint_in(0, h - 1);
      if (bad) T[by * stride + bx] = 1;   // B == 0 but T != 0
      int32_t gx = -1, gy = -1;
      const bool ok = tci::columns_valid(F.data(), B.data(), T.data(), w, h, stride, &gx, &gy);
      CHECK(ok == !bad && (!bad || (gx == bx && gy == by)), "columns_valid");
    }
    // views
    {
      const bool valid = rint_in(0, 3) != 0;
      const int32_t n = rint_in(1, 40);
      std::vector<tc_view> v;
      for (int32_t i = 0; i < n; ++i) v.push_back(random_view(valid || i != n / 2));
      tci::PlanOpts o;
      o.render_mode = rint_in(0, 4);
      o.split_budget = rint_in(0, 1) * 128;
      o.split_queue = rint_in(1, 1 << 17);
      o.split_waves = 1 << rint_in(0, 2);
      tci::ViewPlan p;
      std::string err;
      const tc_status st = tci::make_view_plan(o, v.data(), n, p, rint_in(0, 1), &err);
      if (!valid) {
        CHECK(st == TC_INVALID_ARG && !err.empty(), "invalid view list accepted");
      } else if (st == TC_OK) {
        CHECK(p.off_views == 0 && p.off_prefix % 16 == 0 && p.off_rows % 16 == 0 &&
                  p.off_counter % 16 == 0 && p.off_queue == p.off_counter + 64,
              "view plan alignment");
        CHECK(p.off_prefix >= sizeof(tci_view) * (size_t)n &&
                  p.off_rows >= p.off_prefix + 8 * ((size_t)n + 1) &&
                  p.off_counter >= p.off_rows + 4 * p.rows.size(),
              "view plan regions overlap");
        CHECK(p.total == p.off_queue + tci::kQueueEntry * p.qcap, "view plan total");
        int64_t rays = 0, pk = 0;
        size_t roff = 0;
        for (int32_t i = 0; i < n; ++i) {
          const tci_view& t = p.views[i];
          CHECK(t.out_base == rays && t.pkt_base == pk && p.prefix[i] == pk &&
                    t.rows_off == (int64_t)roff,
                "view %d bases", i);
          const int32_t ty_n = (v[i].height + 7) / 8;
          std::vector<int> seen(ty_n, 0);
          for (int32_t r = 0; r < ty_n; ++r) {
            const int32_t row = p.rows[roff + r];
            if (row >= 0 && row < ty_n) seen[row]++;
          }
          for (int32_t r = 0; r < ty_n; ++r) CHECK(seen[r] == 1, "view %d row table", i);
          roff += ty_n;
          rays += (int64_t)v[i].width * v[i].height;
          pk += (int64_t)((v[i].width + 7) / 8) * ty_n;
        }
        CHECK(p.rays == rays && p.npkt == pk && p.prefix[n] == pk, "view plan totals");
        CHECK(p.qcap <= (uint32_t)o.split_queue, "split queue beyond its option");
        std::vector<char> host(p.off_queue);
        tci::write_views(p, host.data());
      }
    }
    // edits
    {
      const bool valid = rint_in(0, 3) != 0;
      // (now and then a list long enough for the overlap lists' bucket grid)
      const int32_t n = rint_in(0, 7) == 0 ? rint_in(65, 400) : rint_in(0, 30);
      std::vector<Patch> keep;
      keep.reserve(512);
      std::vector<tc_edit> e;
      for (int32_t i = 0; i < n; ++i)
        e.push_back(random_edit(W, H, keep, valid || i != n / 2));
      size_t pb = 0;
      std::string err;
      const tc_status st = tci::check_edits(n ? e.data() : nullptr, n, &pb, &err);
      if (!valid && n > 0) {
        CHECK(st == TC_INVALID_ARG && !err.empty(), "invalid edit list accepted");
      } else {
        CHECK(st == TC_OK, "valid edit list rejected: %s", err.c_str());
        tci::EditPlan sized, p;
        tci::plan_edits(d, e.data(), n, pb, nullptr, sized);
        std::vector<char> host(sized.total);
        tci::plan_edits(d, e.data(), n, pb, host.data(), p);
        CHECK(p.total == sized.total && p.off_patch + pb == p.total, "edit plan sizes");
        CHECK(p.off_olap >= p.off_rects + 16 * (size_t)n * (size_t)(d.top + 1) &&
                  p.off_patch >= p.off_olap + 4 * p.olap.size() &&
                  p.olap.size() >= (size_t)n + 1,
              "edit plan regions overlap");
        // overlap lists: written, and for every edit exactly the other edits
        // whose clipped rectangles meet its own, ascending
        const int32_t* ol = reinterpret_cast<const int32_t*>(host.data() + p.off_olap);
        CHECK(std::equal(p.olap.begin(), p.olap.end(), ol), "overlap lists not written");
        if (!p.olap_all) {
          auto clip = [&](const tc_edit& x, int32_t c[4]) {
            c[0] = std::max(x.x0, 0);
            c[1] = std::max(x.y0, 0);
            c[2] = std::min(x.x0 + x.w, W);
            c[3] = std::min(x.y0 + x.h, H);
          };
          for (int32_t i = 0; i < n; ++i) {
            int32_t a[4];
            clip(e[i], a);
            std::vector<int32_t> want;
            for (int32_t j = 0; j < n && a[0] < a[2] && a[1] < a[3]; ++j) {
              int32_t c[4];
              clip(e[j], c);
              if (j != i && c[0] < c[2] && c[1] < c[3] && a[0] < c[2] && c[0] < a[2] &&
                  a[1] < c[3] && c[1] < a[3])
                want.push_back(j);
            }
            CHECK(ol[i + 1] - ol[i] == (int32_t)want.size() &&
                      std::equal(want.begin(), want.end(), ol + n + 1 + ol[i]),
                  "overlap list of edit %d", i);
          }
        }
        const int32_t* r = reinterpret_cast<const int32_t*>(host.data() + p.off_rects);
        for (int32_t L = 0; L <= d.top; ++L) {
          for (int32_t k = 0; k < p.nrect[L]; ++k) {
            const int32_t* q = r + 4 * ((size_t)L * n + k);
            CHECK(q[0] >= 0 && q[1] >= 0 && q[0] <= q[2] && q[1] <= q[3] &&
                      q[2] < d.lv[L].w && q[3] < d.lv[L].h,
                  "edit rectangle outside level %d", L);
            CHECK(q[2] - q[0] + 1 <= p.rmw[L] && q[3] - q[1] + 1 <= p.rmh[L],
                  "edit rectangle larger than the level's maximum");
          }
        }
      }
    }
    if (g_fails > 20) break;
  }
  std::printf("plan_sanitize: %d iterations, %d failures\n", iters, g_fails);
  return g_fails ? 1 : 0;
}
