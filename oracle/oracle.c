/*
 * CPU oracle: exact first intersection of a ray with a two-layer
 * height-column map.
 *
 * TEST INFRASTRUCTURE.  This file is the reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it; the library never does, and it shares no
 * code, header or table with the library.
 *
 * What it computes (the paper's reference, Section 4.1, taken to its exact
 * limit):
 *  - The paper's solidity predicate (Section 3.1, SOLID): a point at height z
 *    over column (x, y) is solid iff z <= low, or mid <= z <= high.  With the
 *    encoding F = low, B = mid, T = high and B == 0 meaning "no upper
 *    interval" (Section 2: a single-level texel carries one interval), the
 *    solid set of a column is (-inf, F] united with [B, T] when B > 0.  Both
 *    intervals are closed, and the floor interval is unbounded below so a
 *    height-0 floor is hittable (the z >= 0 pitfall of Section 4.1).
 *  - The reference ray cast marches a ray and brackets the first crossing
 *    into solid (Section 3.1 listing, Section 4.1).  Here the march is the
 *    exact cell sequence of a 2D digital differential analyser instead of
 *    uniform samples, so the first solid point is found exactly: column
 *    (x, y) covers the closed square [x, x+1] x [y, y+1]; the walk starts in
 *    floor(O / S); a cell is tested over the closed parameter interval
 *    during which the ray is inside it; when the x and y boundaries are
 *    crossed at the same instant the x step is taken first (a zero-length
 *    visit of the x neighbour), which fixes the cell-boundary convention that
 *    Section 6.1 leaves implicit.
 *  - No solid exists outside the map or above z = 255; a ray that leaves
 *    the map and cannot come back is a miss (misses keep the cleared far
 *    depth, Section 3.1).
 *
 * Fixed point: origins are Q16 (S = 65536 per cell), directions are plain
 * integers.  P(t) = O + t * D with t >= 0 rational.  Every comparison is an
 * exact cross-multiplication, done in 128-bit integers so no bound analysis
 * is needed to trust it.  Depth is the Euclidean distance from the origin in
 * world units, t * |D| / S, in double precision.
 *
 * Hit record: word bits 0-26 cell index y*W + x, bits 27-29 face, bit 30
 * layer (0 floor, 1 slab); a miss is 0xFFFFFFFF with depth +inf.  Faces:
 * 1 top (+Z), 2 slab underside (-Z), 3 wall facing -X (ray moving +x),
 * 4 wall facing +X, 5 wall facing -Y, 6 wall facing +Y, 7 origin inside
 * solid (depth 0).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

typedef __int128 i128;

#define OR_S 65536
#define OR_MISS 0xFFFFFFFFu

enum { F_TOP = 1, F_UNDER = 2, F_WMX = 3, F_WPX = 4, F_WMY = 5, F_WPY = 6,
       F_INSIDE = 7 };

/* 84-byte view record, same field order as the input generator writes. */
typedef struct {
    int32_t w, h;
    int32_t o0[3], opx[3], opy[3];
    int32_t d0[3], dpx[3], dpy[3];
    uint32_t flags;
} or_view;

typedef struct {
    int32_t W, H;
    const uint8_t *F, *B, *T; /* row-major [y * W + x] */
} or_map;

static int64_t floordiv(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

/* z(t) compared with h (in cells), t = tn / td, td > 0.
 * Returns sign of z(t) - h*S: -1, 0, +1. */
static int zcmp(int64_t Oz, int64_t Dz, int64_t tn, int64_t td, int h)
{
    i128 lhs = (i128)Oz * td + (i128)tn * Dz;
    i128 rhs = (i128)h * OR_S * td;
    return (lhs > rhs) - (lhs < rhs);
}

/* a/b <= c/d for b, d > 0 */
static int rat_le(int64_t a, int64_t b, int64_t c, int64_t d)
{
    return (i128)a * d <= (i128)c * b;
}

static void set_hit(uint32_t *word, double *depth, int64_t *hit_tn,
                    int64_t *hit_td, int32_t W, int x, int y, int face,
                    int layer, int64_t tn, int64_t td, const int64_t D[3])
{
    *hit_tn = tn;
    *hit_td = td;
    double len = sqrt((double)D[0] * D[0] + (double)D[1] * D[1] +
                      (double)D[2] * D[2]);
    *word = (uint32_t)((int64_t)y * W + x) | ((uint32_t)face << 27) |
            ((uint32_t)layer << 30);
    *depth = (tn == 0) ? 0.0 : ((double)tn / (double)td) * len / OR_S;
}

/* Cast one ray; writes the hit record and the exact hit time tn / td.
 * Returns 1 on hit, 0 on miss. */
static int cast_exact(const or_map *m, const int64_t O[3], const int64_t D[3],
                      uint32_t *word, double *depth, int64_t *hit_tn,
                      int64_t *hit_td)
{
    *word = OR_MISS;
    *depth = INFINITY;
    *hit_tn = -1;
    *hit_td = 1;
    if (D[0] == 0 && D[1] == 0 && D[2] == 0) return 0;

    const int64_t S = OR_S;
    int64_t cx = floordiv(O[0], S), cy = floordiv(O[1], S);
    const int64_t ax = D[0] < 0 ? -D[0] : D[0];
    const int64_t ay = D[1] < 0 ? -D[1] : D[1];
    const int64_t Dz = D[2], Oz = O[2];
    /* distance (in S units along the axis) to the next boundary */
    int64_t nx = D[0] > 0 ? (cx + 1) * S - O[0] : O[0] - cx * S;
    int64_t ny = D[1] > 0 ? (cy + 1) * S - O[1] : O[1] - cy * S;

    int64_t tin_n = 0, tin_d = 1; /* entry time of the current cell */
    int entry_face = F_INSIDE;    /* face crossed to enter the current cell */

    for (;;) {
        /* exit time of the current cell; x first on ties */
        int exit_axis; /* 0 x, 1 y, -1 never (vertical ray) */
        int64_t tout_n = 0, tout_d = 1;
        if (ax == 0 && ay == 0) exit_axis = -1;
        else if (ay == 0) exit_axis = 0;
        else if (ax == 0) exit_axis = 1;
        else exit_axis = rat_le(nx, ax, ny, ay) ? 0 : 1;
        if (exit_axis == 0) { tout_n = nx; tout_d = ax; }
        if (exit_axis == 1) { tout_n = ny; tout_d = ay; }

        int inside = cx >= 0 && cx < m->W && cy >= 0 && cy < m->H;
        if (inside) {
            size_t idx = (size_t)cy * m->W + cx;
            int F = m->F[idx], B = m->B[idx], T = m->T[idx];
            int zf = zcmp(Oz, Dz, tin_n, tin_d, F);
            int in_floor = zf <= 0;
            int in_slab = B > 0 && zcmp(Oz, Dz, tin_n, tin_d, B) >= 0 &&
                          zcmp(Oz, Dz, tin_n, tin_d, T) <= 0;
            if (in_floor || in_slab) {
                set_hit(word, depth, hit_tn, hit_td, m->W, (int)cx, (int)cy, entry_face,
                        in_floor ? 0 : 1, tin_n, tin_d, D);
                return 1;
            }
            if (Dz < 0) {
                /* descending: the next solid below is the slab top if the
                 * ray is above the slab, else the floor top */
                int above_slab = B > 0 && zcmp(Oz, Dz, tin_n, tin_d, T) > 0;
                int target = above_slab ? T : F;
                int64_t th_n = Oz - (int64_t)target * S, th_d = -Dz;
                if (exit_axis < 0 || rat_le(th_n, th_d, tout_n, tout_d)) {
                    set_hit(word, depth, hit_tn, hit_td, m->W, (int)cx, (int)cy, F_TOP,
                            above_slab ? 1 : 0, th_n, th_d, D);
                    return 1;
                }
            } else if (Dz > 0 && B > 0 &&
                       zcmp(Oz, Dz, tin_n, tin_d, B) < 0) {
                /* ascending below the slab: the underside is next */
                int64_t th_n = (int64_t)B * S - Oz, th_d = Dz;
                if (exit_axis < 0 || rat_le(th_n, th_d, tout_n, tout_d)) {
                    set_hit(word, depth, hit_tn, hit_td, m->W, (int)cx, (int)cy, F_UNDER, 1,
                            th_n, th_d, D);
                    return 1;
                }
            }
        } else {
            /* outside the map: give up once the ray cannot come back */
            if ((cx < 0 && D[0] <= 0) || (cx >= m->W && D[0] >= 0) ||
                (cy < 0 && D[1] <= 0) || (cy >= m->H && D[1] >= 0))
                return 0;
        }
        /* nothing is solid above 255 */
        if (Dz >= 0 && zcmp(Oz, Dz, tin_n, tin_d, 255) > 0) return 0;
        if (exit_axis < 0) return 0;

        /* advance to the neighbour across the exit boundary */
        tin_n = tout_n;
        tin_d = tout_d;
        if (exit_axis == 0) {
            if (D[0] > 0) { cx += 1; entry_face = F_WMX; }
            else          { cx -= 1; entry_face = F_WPX; }
            nx += S;
        } else {
            if (D[1] > 0) { cy += 1; entry_face = F_WMY; }
            else          { cy -= 1; entry_face = F_WPY; }
            ny += S;
        }
    }
}

int or_cast(const or_map *m, const int64_t O[3], const int64_t D[3],
            uint32_t *word, double *depth)
{
    int64_t tn, td;
    return cast_exact(m, O, D, word, depth, &tn, &td);
}

/* Ray of pixel (px, py) of a view: O = o0 + (2px+1) o_px + (2py+1) o_py,
 * D likewise. */
static void pixel_ray(const or_view *v, int px, int py, int64_t O[3],
                      int64_t D[3])
{
    int64_t a = 2 * (int64_t)px + 1, b = 2 * (int64_t)py + 1;
    for (int c = 0; c < 3; ++c) {
        O[c] = (int64_t)v->o0[c] + a * v->opx[c] + b * v->opy[c];
        D[c] = (int64_t)v->d0[c] + a * v->dpx[c] + b * v->dpy[c];
    }
}

typedef struct {
    const or_map *m;
    const or_view *views;
    int nviews;
    const int64_t *row_base; /* output offset of each (view,row) job */
    const int32_t *job_view, *job_row;
    int64_t njobs;
    uint32_t *word;
    double *depth;
    int64_t next; /* shared job counter */
    pthread_mutex_t lock;
} or_job;

static void *worker(void *arg)
{
    or_job *j = (or_job *)arg;
    for (;;) {
        pthread_mutex_lock(&j->lock);
        int64_t k = j->next++;
        pthread_mutex_unlock(&j->lock);
        if (k >= j->njobs) break;
        const or_view *v = &j->views[j->job_view[k]];
        int py = j->job_row[k];
        int64_t base = j->row_base[k];
        for (int px = 0; px < v->w; ++px) {
            int64_t O[3], D[3];
            pixel_ray(v, px, py, O, D);
            or_cast(j->m, O, D, &j->word[base + px], &j->depth[base + px]);
        }
    }
    return NULL;
}

/* Render rows [row0, row1) of every view (row indices are per view and
 * clipped to its height); outputs are packed view by view, row by row, for
 * the selected rows only.  Returns the number of rays cast, or -1. */
int64_t or_render_rows(int32_t W, int32_t H, const uint8_t *F,
                       const uint8_t *B, const uint8_t *T,
                       const or_view *views, int nviews, int32_t row0,
                       int32_t row1, int32_t row_step, uint32_t *word,
                       double *depth, int nthreads)
{
    or_map m = {W, H, F, B, T};
    int64_t njobs = 0;
    for (int i = 0; i < nviews; ++i)
        for (int32_t r = row0; r < row1 && r < views[i].h; r += row_step)
            njobs++;
    int64_t *row_base = malloc(sizeof(int64_t) * (njobs + 1));
    int32_t *jv = malloc(sizeof(int32_t) * (njobs + 1));
    int32_t *jr = malloc(sizeof(int32_t) * (njobs + 1));
    if (!row_base || !jv || !jr) {
        free(row_base); free(jv); free(jr);
        return -1;
    }
    int64_t k = 0, off = 0;
    for (int i = 0; i < nviews; ++i)
        for (int32_t r = row0; r < row1 && r < views[i].h; r += row_step) {
            row_base[k] = off;
            jv[k] = i;
            jr[k] = r;
            off += views[i].w;
            k++;
        }
    or_job j = {&m, views, nviews, row_base, jv, jr, njobs, word, depth, 0,
                PTHREAD_MUTEX_INITIALIZER};
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    int started = 0;
    for (int t = 1; t < nthreads && th; ++t)
        if (pthread_create(&th[t], NULL, worker, &j) == 0) started = t;
    worker(&j);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    free(th);
    free(row_base); free(jv); free(jr);
    return off;
}

/* Cast an explicit list of rays (origins and directions, 3 int64 each). */
void or_cast_list(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                  const uint8_t *T, const int64_t *O, const int64_t *D,
                  int64_t n, uint32_t *word, double *depth)
{
    or_map m = {W, H, F, B, T};
    for (int64_t i = 0; i < n; ++i)
        or_cast(&m, O + 3 * i, D + 3 * i, &word[i], &depth[i]);
}

/* Cast an explicit list of rays and also return the exact hit times
 * tn / td (tn = -1 on a miss). */
void or_cast_list_exact(int32_t W, int32_t H, const uint8_t *F,
                        const uint8_t *B, const uint8_t *T, const int64_t *O,
                        const int64_t *D, int64_t n, uint32_t *word,
                        double *depth, int64_t *tn, int64_t *td)
{
    or_map m = {W, H, F, B, T};
    for (int64_t i = 0; i < n; ++i)
        cast_exact(&m, O + 3 * i, D + 3 * i, &word[i], &depth[i], &tn[i],
                   &td[i]);
}

/* Cast selected pixels: for each k, view vi[k], pixel (px[k], py[k]). */
void or_cast_pixels(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                    const uint8_t *T, const or_view *views, const int32_t *vi,
                    const int32_t *px, const int32_t *py, int64_t n,
                    uint32_t *word, double *depth)
{
    or_map m = {W, H, F, B, T};
    for (int64_t k = 0; k < n; ++k) {
        int64_t O[3], D[3];
        pixel_ray(&views[vi[k]], px[k], py[k], O, D);
        or_cast(&m, O, D, &word[k], &depth[k]);
    }
}
