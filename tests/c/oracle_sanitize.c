/*
 * Exercises every entry point of the C oracle (oracle.c, march.c, shade.c)
 * on small random maps and random rays, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Any out-of-bounds
 * access, use after free, signed overflow or other undefined behaviour
 * aborts the run.  It also checks that the entry points agree with each
 * other: whole-view renders (several threads) against per-pixel casts,
 * the exact-time variant against the plain one, and the same for the
 * sampled march and the shading pass.
 *
 * Usage: oracle_sanitize [iterations] [seed]
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t w, h;
    int32_t o0[3], opx[3], opy[3];
    int32_t d0[3], dpx[3], dpy[3];
    uint32_t flags;
} view_t;

typedef struct {
    int32_t light[3];
    float ambient, cave_ambient, fog_far;
    uint32_t sky_rgba, fog_rgba;
} shade_t;

int64_t or_render_rows(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                       const uint8_t *T, const view_t *views, int nviews,
                       int32_t row0, int32_t row1, int32_t row_step,
                       uint32_t *word, double *depth, int nthreads);
void or_cast_list(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                  const uint8_t *T, const int64_t *O, const int64_t *D,
                  int64_t n, uint32_t *word, double *depth);
void or_cast_list_exact(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                        const uint8_t *T, const int64_t *O, const int64_t *D,
                        int64_t n, uint32_t *word, double *depth, int64_t *tn,
                        int64_t *td);
void or_cast_pixels(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                    const uint8_t *T, const view_t *views, const int32_t *vi,
                    const int32_t *px, const int32_t *py, int64_t n,
                    uint32_t *word, double *depth);
int64_t om_march_rows(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                      const uint8_t *T, const view_t *views, int nviews,
                      int32_t row0, int32_t row1, int32_t row_step, float far,
                      int steps, int bisect, uint32_t *word, float *depth,
                      int nthreads, int64_t *reads);
void om_march_list(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                   const uint8_t *T, const int64_t *O, const int64_t *D,
                   int64_t n, float far, int steps, int bisect, uint32_t *word,
                   float *depth);
void om_march_pixels(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                     const uint8_t *T, const view_t *views, const int32_t *vi,
                     const int32_t *px, const int32_t *py, int64_t n, float far,
                     int steps, int bisect, uint32_t *word, float *depth);
int64_t os_shade_views(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                       const uint8_t *T, const view_t *views, int nviews,
                       const shade_t *p, const uint32_t *palette, uint32_t *rgba);
int64_t os_shade_pixels(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                        const uint8_t *T, const view_t *views, const int32_t *vi,
                        const int32_t *px, const int32_t *py, int64_t n,
                        const shade_t *p, const uint32_t *palette, uint32_t *rgba);

static uint64_t rng_state;

/* splitmix64 */
static uint64_t rnd(void)
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int32_t rint_in(int32_t lo, int32_t hi) /* [lo, hi] */
{
    return lo + (int32_t)(rnd() % (uint64_t)(hi - lo + 1));
}

static int fails;

#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            fprintf(stderr, __VA_ARGS__);                 \
            fputc('\n', stderr);                          \
            fails++;                                      \
        }                                                 \
    } while (0)

/* A random map obeying the column invariants: B == 0 => T == 0, else
 * B > F and T >= B. */
static void random_map(int W, int H, uint8_t *F, uint8_t *B, uint8_t *T)
{
    const int top = rint_in(0, 3) == 0 ? 8 : 255;
    for (int i = 0; i < W * H; ++i) {
        F[i] = (uint8_t)rint_in(0, top < 250 ? top : 200);
        B[i] = T[i] = 0;
        if (rint_in(0, 2) == 0 && F[i] < 254) {
            B[i] = (uint8_t)rint_in(F[i] + 1, 254);
            T[i] = (uint8_t)rint_in(B[i], 255);
        }
    }
}

/* Random direction component: zero, tiny, or up to the largest the
 * library accepts (2^23 - 1). */
static int32_t rdir(void)
{
    switch (rint_in(0, 4)) {
    case 0: return 0;
    case 1: return rint_in(-3, 3);
    case 2: return rint_in(-(1 << 16), 1 << 16);
    default: return rint_in(-(1 << 23) + 1, (1 << 23) - 1);
    }
}

static void random_view(int W, int H, view_t *v)
{
    memset(v, 0, sizeof(*v));
    v->w = rint_in(1, 9);
    v->h = rint_in(1, 7);
    /* origins around and inside the map, heights -20..300, on the lattice
     * now and then (boundary origins) */
    const int lattice = rint_in(0, 3) == 0;
    int32_t o[3] = {rint_in(-8, W + 8) * 65536, rint_in(-8, H + 8) * 65536,
                    rint_in(-20, 300) * 65536};
    for (int c = 0; c < 3 && !lattice; ++c) o[c] += rint_in(0, 65535);
    int32_t d[3] = {rdir(), rdir(), rdir()};
    const int ortho = rint_in(0, 2) == 0;
    for (int c = 0; c < 3; ++c) {
        v->o0[c] = o[c];
        v->d0[c] = d[c];
        if (ortho) {
            v->opx[c] = c == 0 ? rint_in(0, 1 << 15) : 0;
            v->opy[c] = c == 1 ? rint_in(0, 1 << 15) : 0;
        } else {
            /* keep every corner's direction within 2^23 - 1 */
            int32_t lim = ((1 << 23) - 1 - abs(d[c])) / 24;
            v->dpx[c] = lim > 0 ? rint_in(-lim, lim) : 0;
            v->dpy[c] = lim > 0 ? rint_in(-lim, lim) : 0;
        }
    }
}

static void pixel_ray(const view_t *v, int px, int py, int64_t O[3], int64_t D[3])
{
    for (int c = 0; c < 3; ++c) {
        O[c] = (int64_t)v->o0[c] + (2 * (int64_t)px + 1) * v->opx[c] + (2 * (int64_t)py + 1) * v->opy[c];
        D[c] = (int64_t)v->d0[c] + (2 * (int64_t)px + 1) * v->dpx[c] + (2 * (int64_t)py + 1) * v->dpy[c];
    }
}

int main(int argc, char **argv)
{
    const int iters = argc > 1 ? atoi(argv[1]) : 200;
    rng_state = argc > 2 ? strtoull(argv[2], NULL, 10) : 12345;
    uint32_t palette[512];
    for (int i = 0; i < 512; ++i) palette[i] = (uint32_t)rnd() | 0xFF000000u;
    int64_t total = 0;
    for (int it = 0; it < iters; ++it) {
        const int W = rint_in(1, 40), H = rint_in(1, 33);
        uint8_t *F = malloc((size_t)W * H), *B = malloc((size_t)W * H), *T = malloc((size_t)W * H);
        random_map(W, H, F, B, T);
        const int nv = rint_in(1, 6);
        view_t views[6];
        int64_t n = 0;
        for (int i = 0; i < nv; ++i) {
            random_view(W, H, &views[i]);
            n += (int64_t)views[i].w * views[i].h;
        }
        uint32_t *word = malloc(sizeof(uint32_t) * n), *w2 = malloc(sizeof(uint32_t) * n);
        uint32_t *w3 = malloc(sizeof(uint32_t) * n);
        double *depth = malloc(sizeof(double) * n), *d2 = malloc(sizeof(double) * n);
        double *d3 = malloc(sizeof(double) * n);
        float *fd = malloc(sizeof(float) * n), *fd2 = malloc(sizeof(float) * n);
        int64_t *O = malloc(sizeof(int64_t) * 3 * n), *D = malloc(sizeof(int64_t) * 3 * n);
        int64_t *tn = malloc(sizeof(int64_t) * n), *td = malloc(sizeof(int64_t) * n);
        int32_t *vi = malloc(sizeof(int32_t) * n), *px = malloc(sizeof(int32_t) * n);
        int32_t *py = malloc(sizeof(int32_t) * n);
        uint32_t *rgba = malloc(sizeof(uint32_t) * n), *rgba2 = malloc(sizeof(uint32_t) * n);
        int64_t k = 0;
        for (int i = 0; i < nv; ++i)
            for (int y = 0; y < views[i].h; ++y)
                for (int x = 0; x < views[i].w; ++x, ++k) {
                    vi[k] = i;
                    px[k] = x;
                    py[k] = y;
                    pixel_ray(&views[i], x, y, O + 3 * k, D + 3 * k);
                }
        /* exact cast: views (3 threads) == pixels == ray list == exact list */
        int64_t got = or_render_rows(W, H, F, B, T, views, nv, 0, 1 << 30, 1, word, depth, 3);
        CHECK(got == n, "render_rows returned %lld of %lld", (long long)got, (long long)n);
        or_cast_pixels(W, H, F, B, T, views, vi, px, py, n, w2, d2);
        or_cast_list_exact(W, H, F, B, T, O, D, n, w3, d3, tn, td);
        for (int64_t j = 0; j < n; ++j) {
            CHECK(word[j] == w2[j] && depth[j] == d2[j], "iter %d ray %lld: views vs pixels", it,
                  (long long)j);
            CHECK(word[j] == w3[j] && depth[j] == d3[j], "iter %d ray %lld: views vs exact list",
                  it, (long long)j);
            CHECK((word[j] == 0xFFFFFFFFu) == (tn[j] < 0), "iter %d ray %lld: miss flag vs time",
                  it, (long long)j);
        }
        or_cast_list(W, H, F, B, T, O, D, n, w2, d2);
        for (int64_t j = 0; j < n; ++j)
            CHECK(word[j] == w2[j], "iter %d ray %lld: ray list", it, (long long)j);
        /* every other row only */
        got = or_render_rows(W, H, F, B, T, views, nv, 1, 1 << 30, 2, w2, d2, 2);
        CHECK(got >= 0 && got <= n, "render_rows (odd rows) returned %lld", (long long)got);
        /* sampled march: views (2 threads) == pixels == ray list */
        const float far = (float)rint_in(1, 2000);
        const int steps = rint_in(1, 200), bisect = rint_in(0, 6);
        int64_t reads = 0;
        got = om_march_rows(W, H, F, B, T, views, nv, 0, 1 << 30, 1, far, steps, bisect, word,
                            fd, 2, &reads);
        CHECK(got == n && reads >= 0, "march_rows returned %lld", (long long)got);
        om_march_pixels(W, H, F, B, T, views, vi, px, py, n, far, steps, bisect, w2, fd2);
        for (int64_t j = 0; j < n; ++j)
            CHECK(word[j] == w2[j] && memcmp(&fd[j], &fd2[j], 4) == 0,
                  "iter %d ray %lld: march views vs pixels", it, (long long)j);
        om_march_list(W, H, F, B, T, O, D, n, far, steps, bisect, w2, fd2);
        for (int64_t j = 0; j < n; ++j)
            CHECK(word[j] == w2[j], "iter %d ray %lld: march ray list", it, (long long)j);
        /* shading: views == pixels, and no face time disagrees */
        shade_t sp = {{rdir(), rdir(), rint_in(1, 1 << 20)}, 0.25f, 0.1f,
                      (float)rint_in(1, 900), 0xFF102030u, 0xFF405060u};
        if (!sp.light[0] && !sp.light[1] && !sp.light[2]) sp.light[2] = 1;
        int64_t e1 = os_shade_views(W, H, F, B, T, views, nv, &sp, palette, rgba);
        int64_t e2 = os_shade_pixels(W, H, F, B, T, views, vi, px, py, n, &sp, palette, rgba2);
        CHECK(e1 == 0 && e2 == 0, "iter %d: shading face times disagree (%lld, %lld)", it,
              (long long)e1, (long long)e2);
        for (int64_t j = 0; j < n; ++j)
            CHECK(rgba[j] == rgba2[j], "iter %d ray %lld: shade views vs pixels", it,
                  (long long)j);
        total += n;
        free(F); free(B); free(T); free(word); free(w2); free(w3); free(depth); free(d2);
        free(d3); free(fd); free(fd2); free(O); free(D); free(tn); free(td); free(vi);
        free(px); free(py); free(rgba); free(rgba2);
        if (fails > 20) break;
    }
    printf("oracle_sanitize: %d maps, %lld rays, %d failures\n", iters, (long long)total, fails);
    return fails ? 1 : 0;
}
