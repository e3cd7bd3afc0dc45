/*
 * CPU oracle of the shading pass: the colour of every pixel from its exact
 * hit, a shadow ray toward the light, a palette, a diffuse term with a
 * height-field gradient normal, cave ambient and fog.
 *
 * TEST INFRASTRUCTURE.  The GPU library's shading pass is checked against
 * this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it; the library never does, and it shares no
 * code, header or table with the library.  It calls the exact caster of
 * oracle.c for the primary and the shadow rays.
 *
 * The paper's methods share one palette, fog, diffuse lighting function and
 * shadow term, and all but the mesh estimate a height-field gradient for
 * the normal (Section 3); its resolve adds cave ambient (Section 3.5).  It
 * gives no formulas, so every step below is this build's reading, stated
 * once here and once in the library's header:
 *
 *  miss              sky colour
 *  hit               cell (x, y), face f, layer; column (F, B, T);
 *                    h = T on the slab layer, else F
 *  exact time        t = tn / td by face: top: (Oz - h S) / -Dz;
 *                    underside: (B S - Oz) / Dz; walls facing -X / +X:
 *                    (x S - Ox) / Dx, (Ox - (x+1) S) / -Dx; facing -Y / +Y
 *                    likewise in y; inside: 0 / 1
 *  distance          d = q * len * 2^-16 with q = (float)((double)tn / (double)td)
 *                    and len = sqrtf(((float)Dx*Dx + (float)Dy*Dy) + (float)Dz*Dz)
 *  normal            top face: the gradient of the hit layer's surface
 *                    s(x', y') (floor: F; slab: T where the neighbour has a
 *                    slab, else the hit column's T), neighbours clamped to
 *                    the map: gx = (float)(s(x+1,y) - s(x-1,y)) * 0.5,
 *                    gy likewise, n = (-gx, -gy, 1) / sqrtf((gx*gx + gy*gy) + 1);
 *                    underside (0, 0, -1); walls their outward axis;
 *                    inside (0, 0, 1)
 *  light             l = L / sqrtf(((float)Lx*Lx + (float)Ly*Ly) + (float)Lz*Lz)
 *  lambert           (nx*lx + ny*ly) + nz*lz
 *  shadow            for lambert > 0 and not inside: a ray from
 *                    P = O + floor(tn * D / td) (Q16, per component), moved
 *                    one Q16 unit out through the hit face, along L, cast
 *                    exactly; lit iff it meets nothing
 *  ambient           cave_ambient for a floor hit under a slab (B > 0),
 *                    else ambient
 *  intensity         I = fminf(ambient + (lit ? lambert : 0), 1)
 *  colour            c = (float)albedo * I, albedo = palette[layer*256 + h];
 *                    fog f = fminf(d / fog_far, 1), c = c + ((float)fog - c) * f;
 *                    byte = (uint8)(c + 0.5); alpha 255
 * All single-precision steps are one IEEE operation each, in this order
 * (the file is built without contraction), so the result is reproducible
 * bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define OS_S 65536
#define OS_MISS 0xFFFFFFFFu

/* exported by oracle.c */
void or_cast_list_exact(int32_t W, int32_t H, const uint8_t *F,
                        const uint8_t *B, const uint8_t *T, const int64_t *O,
                        const int64_t *D, int64_t n, uint32_t *word,
                        double *depth, int64_t *tn, int64_t *td);

typedef struct {
    int32_t w, h;
    int32_t o0[3], opx[3], opy[3];
    int32_t d0[3], dpx[3], dpy[3];
    uint32_t flags;
} os_view;

typedef struct {
    int32_t light[3];
    float ambient, cave_ambient, fog_far;
    uint32_t sky_rgba, fog_rgba;
} os_params;

typedef struct {
    int32_t W, H;
    const uint8_t *F, *B, *T;
} os_map;

static int64_t floordiv(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q--;
    return q;
}

/* surface height of the hit layer at (x, y), clamped to the map */
static int surf(const os_map *m, int x, int y, int layer, int hT)
{
    if (x < 0) x = 0;
    if (x >= m->W) x = m->W - 1;
    if (y < 0) y = 0;
    if (y >= m->H) y = m->H - 1;
    const int64_t k = (int64_t)y * m->W + x;
    if (layer == 0) return m->F[k];
    return m->B[k] > 0 ? m->T[k] : hT;
}

static uint32_t shade_ray(const os_map *m, const int64_t O[3],
                          const int64_t D[3], const os_params *p,
                          const uint32_t *palette, int64_t *errors)
{
    uint32_t word;
    double depth;
    int64_t tn0, td0;
    or_cast_list_exact(m->W, m->H, m->F, m->B, m->T, O, D, 1, &word, &depth,
                       &tn0, &td0);
    if (word == OS_MISS) return p->sky_rgba;
    const int64_t k = word & 0x07FFFFFF;
    const int x = (int)(k % m->W), y = (int)(k / m->W);
    const int face = (int)((word >> 27) & 7), layer = (int)((word >> 30) & 1);
    const int F = m->F[k], B = m->B[k], T = m->T[k];
    const int h = layer ? T : F;
    int64_t tn, td;
    float n[3];
    int64_t nudge[3] = {0, 0, 0};
    switch (face) {
    case 1: tn = O[2] - (int64_t)h * OS_S; td = -D[2]; nudge[2] = 1; break;
    case 2: tn = (int64_t)B * OS_S - O[2]; td = D[2]; nudge[2] = -1; break;
    case 3: tn = (int64_t)x * OS_S - O[0]; td = D[0]; nudge[0] = -1; break;
    case 4: tn = O[0] - (int64_t)(x + 1) * OS_S; td = -D[0]; nudge[0] = 1; break;
    case 5: tn = (int64_t)y * OS_S - O[1]; td = D[1]; nudge[1] = -1; break;
    case 6: tn = O[1] - (int64_t)(y + 1) * OS_S; td = -D[1]; nudge[1] = 1; break;
    default: tn = 0; td = 1; break;
    }
    /* the face formula must give the exact caster's time */
    if ((__int128)tn * td0 != (__int128)tn0 * td) (*errors)++;
    /* distance */
    const float len = sqrtf(((float)D[0] * (float)D[0] + (float)D[1] * (float)D[1]) +
                            (float)D[2] * (float)D[2]);
    const float q = (float)((double)tn / (double)td);
    const float dist = q * len * (1.0f / 65536.0f);
    /* normal */
    if (face == 1) {
        const float gx = (float)(surf(m, x + 1, y, layer, T) - surf(m, x - 1, y, layer, T)) * 0.5f;
        const float gy = (float)(surf(m, x, y + 1, layer, T) - surf(m, x, y - 1, layer, T)) * 0.5f;
        const float nl = sqrtf((gx * gx + gy * gy) + 1.0f);
        n[0] = -gx / nl;
        n[1] = -gy / nl;
        n[2] = 1.0f / nl;
    } else if (face == 2) {
        n[0] = 0.0f; n[1] = 0.0f; n[2] = -1.0f;
    } else if (face >= 3 && face <= 6) {
        n[0] = (float)nudge[0]; n[1] = (float)nudge[1]; n[2] = 0.0f;
    } else {
        n[0] = 0.0f; n[1] = 0.0f; n[2] = 1.0f;
    }
    /* light */
    const float Lx = (float)p->light[0], Ly = (float)p->light[1], Lz = (float)p->light[2];
    const float ll = sqrtf((Lx * Lx + Ly * Ly) + Lz * Lz);
    const float lx = Lx / ll, ly = Ly / ll, lz = Lz / ll;
    const float lambert = (n[0] * lx + n[1] * ly) + n[2] * lz;
    int lit = 0;
    if (face != 7 && lambert > 0.0f) {
        int64_t P[3], L[3];
        for (int c = 0; c < 3; ++c) {
            P[c] = O[c] + floordiv(tn * D[c], td) + nudge[c];
            L[c] = p->light[c];
        }
        uint32_t sw;
        double sd;
        int64_t stn, std_;
        or_cast_list_exact(m->W, m->H, m->F, m->B, m->T, P, L, 1, &sw, &sd, &stn, &std_);
        lit = sw == OS_MISS;
    }
    const float amb = (layer == 0 && B > 0) ? p->cave_ambient : p->ambient;
    const float I = fminf(amb + (lit ? lambert : 0.0f), 1.0f);
    const uint32_t albedo = palette[layer * 256 + h];
    float f = dist / p->fog_far;
    f = fminf(f, 1.0f);
    uint32_t out = 0xFF000000u;
    for (int c = 0; c < 3; ++c) {
        const float a = (float)((albedo >> (8 * c)) & 0xFF);
        const float fogc = (float)((p->fog_rgba >> (8 * c)) & 0xFF);
        float v = a * I;
        v = v + (fogc - v) * f;
        out |= (uint32_t)(v + 0.5f) << (8 * c);
    }
    return out;
}

static void pixel_ray(const os_view *v, int px, int py, int64_t O[3],
                      int64_t D[3])
{
    int64_t a = 2 * (int64_t)px + 1, b = 2 * (int64_t)py + 1;
    for (int c = 0; c < 3; ++c) {
        O[c] = (int64_t)v->o0[c] + a * v->opx[c] + b * v->opy[c];
        D[c] = (int64_t)v->d0[c] + a * v->dpx[c] + b * v->dpy[c];
    }
}

/* Shade every pixel of every view (views concatenated, rows top-down);
 * returns the number of hits whose face formula disagreed with the exact
 * caster's time (0 unless the oracle is broken). */
int64_t os_shade_views(int32_t W, int32_t H, const uint8_t *F, const uint8_t *B,
                       const uint8_t *T, const os_view *views, int nviews,
                       const os_params *p, const uint32_t *palette,
                       uint32_t *rgba)
{
    os_map m = {W, H, F, B, T};
    int64_t errors = 0, o = 0;
    for (int i = 0; i < nviews; ++i)
        for (int py = 0; py < views[i].h; ++py)
            for (int px = 0; px < views[i].w; ++px) {
                int64_t O[3], D[3];
                pixel_ray(&views[i], px, py, O, D);
                rgba[o++] = shade_ray(&m, O, D, p, palette, &errors);
            }
    return errors;
}

/* Shade selected pixels: for each k, view vi[k], pixel (px[k], py[k]). */
int64_t os_shade_pixels(int32_t W, int32_t H, const uint8_t *F,
                        const uint8_t *B, const uint8_t *T,
                        const os_view *views, const int32_t *vi,
                        const int32_t *px, const int32_t *py, int64_t n,
                        const os_params *p, const uint32_t *palette,
                        uint32_t *rgba)
{
    os_map m = {W, H, F, B, T};
    int64_t errors = 0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t O[3], D[3];
        pixel_ray(&views[vi[k]], px[k], py[k], O, D);
        rgba[k] = shade_ray(&m, O, D, p, palette, &errors);
    }
    return errors;
}
