/* A plain C99 consumer of the library's C ABI (test program).
 *
 * Builds a small map from a fixed integer formula, loads it, applies one
 * crater edit, renders one perspective view and one straight-down
 * orthographic view into device memory allocated with the HIP runtime's C
 * API, and writes the map planes, the views and the hit records to a file
 * for the test to check against the oracle.
 *
 * usage: consumer <out-file>
 * file:  int32 W, H, nviews; W*H bytes F, B, T (before the edit); int32
 *        crater x0, y0, size, depth; nviews x 84-byte tc_view; (total rays)
 *        x tc_hit.  Exit status 0 on success. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tc.h"

#define CHECK(x)                                                          \
    do {                                                                  \
        tc_status st_ = (x);                                              \
        if (st_ != TC_OK) {                                               \
            fprintf(stderr, "%s failed: %d (%s)\n", #x, st_,             \
                    tc_last_error(ctx));                                  \
            return 1;                                                     \
        }                                                                 \
    } while (0)

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    enum { W = 96, H = 80 };
    static uint8_t F[W * H], B[W * H], T[W * H];
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int k = y * W + x;
            F[k] = (uint8_t)(20 + (x * 7 + y * 13) % 41 + ((x / 16 + y / 16) % 2) * 30);
            if (x >= 30 && x < 60 && y >= 20 && y < 50) {
                B[k] = (uint8_t)(F[k] + 10 + (x + y) % 7);
                T[k] = (uint8_t)(B[k] + 5 + (x * y) % 9);
            }
        }
    tc_context *ctx = NULL;
    tc_status st = tc_create(0, &ctx);
    if (st != TC_OK) {
        fprintf(stderr, "tc_create: %d (%s)\n", st, tc_last_error(NULL));
        return 1;
    }
    CHECK(tc_load_columns(ctx, W, H, F, B, T, W, NULL));
    tc_edit ed;
    memset(&ed, 0, sizeof(ed));
    ed.kind = TC_EDIT_CRATER;
    ed.x0 = 40;
    ed.y0 = 30;
    ed.w = ed.h = 16;
    ed.depth = 25;
    CHECK(tc_apply_edit(ctx, &ed, 1, NULL));

    tc_view v[2];
    memset(v, 0, sizeof(v));
    /* perspective: eye (5.5, 5.5, 90), 64 x 48 pixels, looking along +x+y and down */
    v[0].width = 64;
    v[0].height = 48;
    v[0].o0[0] = 5 * TC_S + TC_S / 2;
    v[0].o0[1] = 5 * TC_S + TC_S / 2;
    v[0].o0[2] = 90 * TC_S;
    v[0].d0[0] = 1 << 21;
    v[0].d0[1] = (1 << 21) - 64 * 9000;
    v[0].d0[2] = -(1 << 20) + 48 * 9000;
    v[0].d_px[1] = 9000;
    v[0].d_py[2] = -9000;
    /* orthographic, straight down over every cell centre of a 40 x 30 window */
    v[1].width = 40;
    v[1].height = 30;
    v[1].o0[0] = 20 * TC_S;
    v[1].o0[1] = 25 * TC_S;
    v[1].o0[2] = 250 * TC_S;
    v[1].o_px[0] = TC_S / 2;
    v[1].o_py[1] = TC_S / 2;
    v[1].d0[2] = -(1 << 22);
    const int nviews = 2;
    const size_t rays = (size_t)64 * 48 + (size_t)40 * 30;
    tc_hit *dev = NULL;
    if (hipMalloc((void **)&dev, rays * sizeof(tc_hit)) != hipSuccess) return 1;
    for (int mode = 0; mode <= 4; ++mode) {
        if (mode == 3) continue;   /* the sampled march is not an exact cast */
        CHECK(tc_set_option(ctx, TC_OPT_RENDER_MODE, mode));
        CHECK(tc_render_views(ctx, v, nviews, dev, NULL));
    }
    tc_hit *host = malloc(rays * sizeof(tc_hit));
    if (!host) return 1;
    if (hipMemcpy(host, dev, rays * sizeof(tc_hit), hipMemcpyDeviceToHost) != hipSuccess) return 1;
    FILE *f = fopen(argv[1], "wb");
    if (!f) return 1;
    int32_t hdr[3] = {W, H, nviews};
    fwrite(hdr, sizeof(hdr), 1, f);
    fwrite(F, 1, sizeof(F), f);
    fwrite(B, 1, sizeof(B), f);
    fwrite(T, 1, sizeof(T), f);
    int32_t crater[4] = {ed.x0, ed.y0, ed.w, ed.depth};
    fwrite(crater, sizeof(crater), 1, f);
    fwrite(v, sizeof(tc_view), (size_t)nviews, f);
    fwrite(host, sizeof(tc_hit), rays, f);
    fclose(f);
    free(host);
    (void)hipFree(dev);
    tc_destroy(ctx);
    return 0;
}
