/* Runs the oracle's C entry points on small inputs and their edge cases
 * (eye inside the brick, orthographic view, pixel subsets, early
 * termination, no ghost layer, double voxels, empty and over-long composite
 * lists) under AddressSanitizer / UndefinedBehaviorSanitizer; the oracle
 * source is compiled into this file.  Exits non-zero on a failed check. */
#include "../../oracle/dpvr_oracle.c"

#include <stdio.h>

static int g_fail = 0;
#define CHECK(c) do { if (!(c)) { printf("FAILED line %d: %s\n", __LINE__, #c); ++g_fail; } } while (0)

static double urand(unsigned* s) { *s = *s * 1664525u + 1013904223u; return (*s >> 8) / 16777216.0; }

int main(void) {
    unsigned seed = 7;
    enum { W = 24, H = 16, NX = 6, NY = 5, NZ = 4 };
    float vox[(NZ + 2) * (NY + 2) * (NX + 2)];
    double voxd[(NZ + 2) * (NY + 2) * (NX + 2)];
    for (int i = 0; i < (NZ + 2) * (NY + 2) * (NX + 2); ++i) { vox[i] = (float)urand(&seed); voxd[i] = vox[i]; }
    double table[256 * 4];
    for (int i = 0; i < 256 * 4; ++i) table[i] = urand(&seed);
    oc_tf tf = {table, 256, 0, 0.0, 1.0, 2.0};
    oc_brick b = {{NX, NY, NZ}, 1, {0, 0, 0}, {1, 1, 1}, vox, 0, 0};
    oc_camera persp = {0, W, H, 0, {3, 2.5, -12}, {3, 2.5, 2}, {0, 0, 0}, {0, 1, 0}, 40.0, 0.0};
    oc_camera inside = {0, W, H, 0, {3, 2.5, 2}, {9, 2.5, 2}, {0, 0, 0}, {0, 1, 0}, 60.0, 0.0};
    oc_camera ortho = {1, W, H, 0, {3, 2.5, -5}, {0, 0, 0}, {0.1, 0.05, 1}, {0, 1, 0}, 0.0, 8.0};
    const oc_camera* cams[3] = {&persp, &inside, &ortho};
    static double rgba[W * H * 4], depth[W * H];
    for (int c = 0; c < 3; ++c) {
        int64_t cnt[2] = {0, 0};
        oc_render_brick(cams[c], &b, &tf, 0.5, 0.0, NULL, 0, rgba, depth, cnt);
        CHECK(cnt[0] > 0 && cnt[1] == cnt[0]);
        for (int q = 0; q < W * H; ++q) CHECK(rgba[4 * q + 3] >= 0.0 && rgba[4 * q + 3] <= 1.0);
        int64_t cnt2[2] = {0, 0};
        oc_render_brick(cams[c], &b, &tf, 0.5, 0.01, NULL, 0, rgba, depth, cnt2);
        CHECK(cnt2[1] <= cnt2[0]);
    }
    /* pixel subset, double voxels, no ghost layer */
    int32_t pix[6] = {0, 0, W - 1, H - 1, 11, 7};
    double r3[12], d3[3];
    oc_brick bd = b;
    bd.vox = voxd;
    bd.vox_f64 = 1;
    oc_render_brick(&persp, &bd, &tf, 0.25, 0.0, pix, 3, r3, d3, NULL);
    oc_brick b0 = {{NX + 2, NY + 2, NZ + 2}, 0, {-1, -1, -1}, {1, 1, 1}, vox, 0, 0};
    oc_render_brick(&persp, &b0, &tf, 0.5, 0.0, pix, 3, r3, d3, NULL);

    /* composite: none, three, too many */
    static double ra[3][W * H * 4], da[3][W * H];
    const double* rp[3] = {ra[0], ra[1], ra[2]};
    const double* dpp[3] = {da[0], da[1], da[2]};
    for (int k = 0; k < 3; ++k) {
        oc_render_brick(cams[k], &b, &tf, 0.5, 0.0, NULL, 0, ra[k], da[k], NULL);
    }
    const double bg[4] = {0.1, 0.2, 0.3, 1.0};
    static double out[W * H * 4];
    CHECK(oc_composite(0, rp, dpp, W * H, bg, out) == 0);
    CHECK(oc_composite(3, rp, dpp, W * H, bg, out) == 0);
    CHECK(oc_composite(100000, rp, dpp, W * H, bg, out) != 0);
    static double ga[3][W * H * 4];
    double* gp[3] = {ga[0], ga[1], ga[2]};
    CHECK(oc_composite_grad(3, rp, dpp, W * H, bg, out, gp) == 0);

    /* adjoint */
    static double g[W * H * 4];
    for (int i = 0; i < W * H * 4; ++i) g[i] = urand(&seed) - 0.5;
    double gtf[256 * 4] = {0};
    static double gvox[(NZ + 2) * (NY + 2) * (NX + 2)];
    for (int c = 0; c < 3; ++c) CHECK(oc_render_brick_grad(cams[c], &b, &tf, 0.5, g, gtf, gvox) == 0);
    double o[3], d[3];
    oc_ray(&ortho, 3, 4, o, d);
    CHECK(fabs(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - 1.0) < 1e-12);
    CHECK(oc_threads() >= 1);
    printf("%s: %d failed checks\n", g_fail ? "FAIL" : "OK", g_fail);
    return g_fail ? 1 : 0;
}
