/*
 * CPU oracle of the sampled height-field march (paper Section 3.1, the
 * RAYMARCH procedure), in single precision.
 *
 * TEST INFRASTRUCTURE.  The GPU library's sampled render mode is checked
 * against this file.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the library never does, and
 * it shares no code, header or table with the library.
 *
 * What it computes, in the paper's order:
 *  1. The segment.  The march runs from the eye o along d and stops at the
 *     far limit or where the ray reaches the plane z = 0, whichever comes
 *     first (the clip of Section 3.1).  Reading: the far limit is a
 *     distance along each ray (`far` world units).
 *  2. Uniform samples.  The segment is cut into steps + 1 equal parts and
 *     the steps interior points are tested in order, nearest first; the
 *     first sample inside the solid set ends the forward march.  (The
 *     printed listing advances `a` inside the loop while dividing by
 *     steps + 1, which would shrink the step each time; the text says the
 *     segment is sampled uniformly, so sample i sits at i / (steps + 1) of
 *     the segment.)  The segment's end point itself is never tested, so a
 *     ray that meets no solid before it is a miss (Section 3.1: misses keep
 *     the cleared far depth rather than a made-up hit on the ground plane).
 *  3. Bisection.  Between the last empty sample (or the eye) and the first
 *     solid one, `bisect` halvings keep the solid end (four in the paper).
 *  4. The hit is the solid end of the bracket.
 *
 * SOLID (Section 3.1): a point at height z over column (x, y) is solid iff
 * z <= F, or B <= z <= T when the column has an upper slab (B > 0).  There
 * is no solid outside the map.
 *
 * Precision.  The paper's shaders work in 32-bit floats, and here every
 * quantity of the march is an IEEE single computed one operation at a time
 * (this file is compiled without floating-point contraction):
 *   o_c = (float)O_c * 2^-16, d_c = (float)D_c     (O Q16, D integer)
 *   len = sqrt((d_x*d_x + d_y*d_y) + d_z*d_z)
 *   t_end = far / len;  if d_z < 0: t_end = min(t_end, -o_z / d_z)
 *   dt = t_end / (steps + 1);  sample i at t_i = (float)i * dt
 *   point(t)_c = o_c + t * d_c (product rounded, then the sum)
 *   bisection midpoint (t_a + t_b) * 0.5
 *   depth = t_b * len
 * A sample decides solidity from its rounded point; the same arithmetic on
 * another IEEE machine gives the same decisions, so hit words and depths are
 * reproducible bit for bit.
 *
 * Hit record: word bits 0-26 cell index y*W + x of the column that made the
 * final point solid, bits 27-29 face 0 (a sampled hit carries no face),
 * bit 30 layer (0 floor, 1 slab); a miss is 0xFFFFFFFF with depth +inf.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

#define OM_MISS 0xFFFFFFFFu

/* 84-byte view record, same field order as the input generator writes. */
typedef struct {
    int32_t w, h;
    int32_t o0[3], opx[3], opy[3];
    int32_t d0[3], dpx[3], dpy[3];
    uint32_t flags;
} om_view;

typedef struct {
    int32_t W, H;
    const uint8_t *F, *B, *T; /* row-major [y * W + x] */
} om_map;

typedef struct {
    float far;
    int steps, bisect;
} om_params;

static int in_map(const om_map *m, const float p[3])
{
    return p[0] >= 0.0f && p[0] < (float)m->W && p[1] >= 0.0f &&
           p[1] < (float)m->H;
}

/* SOLID at point p: 0 empty, 1 floor, 2 slab; *cell gets the column. */
static int solid(const om_map *m, const float p[3], int64_t *cell)
{
    if (!in_map(m, p)) return 0;
    const int x = (int)floorf(p[0]), y = (int)floorf(p[1]);
    const int64_t k = (int64_t)y * m->W + x;
    *cell = k;
    if (p[2] <= (float)m->F[k]) return 1;
    if (m->B[k] > 0 && p[2] >= (float)m->B[k] && p[2] <= (float)m->T[k])
        return 2;
    return 0;
}

static void point(const float o[3], const float d[3], float t, float p[3])
{
    for (int c = 0; c < 3; ++c) {
        const float s = t * d[c];
        p[c] = o[c] + s;
    }
}

/* March one ray; returns the number of in-map samples tested (the column
 * reads of the march). */
static int64_t march(const om_map *m, const int64_t O[3], const int64_t D[3],
                     const om_params *q, uint32_t *word, float *depth)
{
    *word = OM_MISS;
    *depth = INFINITY;
    if (D[0] == 0 && D[1] == 0 && D[2] == 0) return 0;
    float o[3], d[3];
    for (int c = 0; c < 3; ++c) {
        o[c] = (float)O[c] * 0x1p-16f;
        d[c] = (float)D[c];
    }
    const float len = sqrtf((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    float t_end = q->far / len;
    if (d[2] < 0.0f) {
        const float t0 = -o[2] / d[2];
        if (t0 < t_end) t_end = t0;
    }
    if (!(t_end > 0.0f)) return 0;
    const float dt = t_end / (float)(q->steps + 1);
    float ta = 0.0f, tb = 0.0f, p[3];
    int64_t cell = 0, reads = 0;
    int layer = 0;
    for (int i = 1; i <= q->steps; ++i) {
        const float t = (float)i * dt;
        point(o, d, t, p);
        int64_t c;
        const int s = solid(m, p, &c);
        reads += in_map(m, p);
        if (s) {
            tb = t;
            cell = c;
            layer = s;
            break;
        }
        ta = t;
    }
    if (!layer) return reads;
    for (int k = 0; k < q->bisect; ++k) {
        const float tm = (ta + tb) * 0.5f;
        point(o, d, tm, p);
        int64_t c;
        const int s = solid(m, p, &c);
        reads += in_map(m, p);
        if (s) {
            tb = tm;
            cell = c;
            layer = s;
        } else {
            ta = tm;
        }
    }
    *word = (uint32_t)cell | ((uint32_t)(layer == 2) << 30);
    *depth = tb * len;
    return reads;
}

static void pixel_ray(const om_view *v, int px, int py, int64_t O[3],
                      int64_t D[3])
{
    int64_t a = 2 * (int64_t)px + 1, b = 2 * (int64_t)py + 1;
    for (int c = 0; c < 3; ++c) {
        O[c] = (int64_t)v->o0[c] + a * v->opx[c] + b * v->opy[c];
        D[c] = (int64_t)v->d0[c] + a * v->dpx[c] + b * v->dpy[c];
    }
}

typedef struct {
    const om_map *m;
    const om_params *q;
    const om_view *views;
    const int64_t *row_base;
    const int32_t *job_view, *job_row;
    int64_t njobs;
    uint32_t *word;
    float *depth;
    int64_t next, reads;
    pthread_mutex_t lock;
} om_job;

static void *worker(void *arg)
{
    om_job *j = (om_job *)arg;
    int64_t reads = 0;
    for (;;) {
        pthread_mutex_lock(&j->lock);
        int64_t k = j->next++;
        pthread_mutex_unlock(&j->lock);
        if (k >= j->njobs) break;
        const om_view *v = &j->views[j->job_view[k]];
        int py = j->job_row[k];
        int64_t base = j->row_base[k];
        for (int px = 0; px < v->w; ++px) {
            int64_t O[3], D[3];
            pixel_ray(v, px, py, O, D);
            reads += march(j->m, O, D, j->q, &j->word[base + px],
                           &j->depth[base + px]);
        }
    }
    pthread_mutex_lock(&j->lock);
    j->reads += reads;
    pthread_mutex_unlock(&j->lock);
    return NULL;
}

/* March rows [row0, row1) (step row_step) of every view; outputs packed
 * view by view, row by row.  Returns the number of rays, or -1; *reads
 * gets the number of in-map samples tested. */
int64_t om_march_rows(int32_t W, int32_t H, const uint8_t *F,
                      const uint8_t *B, const uint8_t *T,
                      const om_view *views, int nviews, int32_t row0,
                      int32_t row1, int32_t row_step, float far, int steps,
                      int bisect, uint32_t *word, float *depth,
                      int nthreads, int64_t *reads)
{
    om_map m = {W, H, F, B, T};
    om_params q = {far, steps, bisect};
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
    om_job j = {&m, &q, views, row_base, jv, jr, njobs, word, depth, 0, 0,
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
    if (reads) *reads = j.reads;
    return off;
}

/* March an explicit list of rays (origins and directions, 3 int64 each). */
void om_march_list(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                   const uint8_t *T, const int64_t *O, const int64_t *D,
                   int64_t n, float far, int steps, int bisect,
                   uint32_t *word, float *depth)
{
    om_map m = {W, H, F, B, T};
    om_params q = {far, steps, bisect};
    for (int64_t i = 0; i < n; ++i)
        march(&m, O + 3 * i, D + 3 * i, &q, &word[i], &depth[i]);
}

/* March selected pixels: for each k, view vi[k], pixel (px[k], py[k]). */
void om_march_pixels(int32_t W, int32_t H, const uint8_t *F,
                     const uint8_t *B, const uint8_t *T, const om_view *views,
                     const int32_t *vi, const int32_t *px, const int32_t *py,
                     int64_t n, float far, int steps, int bisect,
                     uint32_t *word, float *depth)
{
    om_map m = {W, H, F, B, T};
    om_params q = {far, steps, bisect};
    for (int64_t k = 0; k < n; ++k) {
        int64_t O[3], D[3];
        pixel_ray(&views[vi[k]], px[k], py[k], O, D);
        march(&m, O, D, &q, &word[k], &depth[k]);
    }
}
