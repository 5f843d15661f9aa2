// Drives the library's host code (linked with the host-memory HIP stand-in)
// through valid calls and every kind of rejected argument, under
// AddressSanitizer / UndefinedBehaviorSanitizer.  Prints one line per
// failed expectation and exits non-zero if there was any.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "dpvr.h"

// inspection hooks of the fake runtime (fake_hip.cpp)
extern "C" void fake_reset_launches();
extern "C" size_t fake_queue_parts(const void** out, size_t cap);
extern "C" size_t fake_composite_frames(const void** out, size_t cap);

static int g_fail = 0;
#define EXPECT(cond)                                                             \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::printf("FAILED line %d: %s\n", __LINE__, #cond);               \
            ++g_fail;                                                            \
        }                                                                        \
    } while (0)

static void* aligned_buf(size_t bytes) {
    void* p = nullptr;
    if (posix_memalign(&p, 256, bytes ? bytes : 256) != 0) std::abort();
    std::memset(p, 0, bytes ? bytes : 256);
    return p;
}

int main() {
    EXPECT(vr_abi_version() == DPVR_ABI_VERSION);
    for (int s = -8; s <= 1; ++s) EXPECT(vr_status_string((vr_status)s) != nullptr);

    // workspace sizes: valid, degenerate, overflowing
    size_t bytes = 0;
    const int32_t d_ok[3] = {30, 20, 10}, d_zero[3] = {0, 4, 4}, d_huge[3] = {2048, 2048, 2048};
    EXPECT(vr_brick_workspace_size(d_ok, 1, VR_F32, &bytes) == VR_OK && bytes > 0);
    EXPECT(vr_brick_workspace_size(d_zero, 1, VR_F32, &bytes) == VR_ERR_INVALID_ARG);
    EXPECT(vr_brick_workspace_size(d_ok, 2, VR_F32, &bytes) != VR_OK);
    EXPECT(vr_brick_workspace_size(d_huge, 1, VR_F16, &bytes) == VR_ERR_UNSUPPORTED);
    EXPECT(vr_brick_workspace_size(nullptr, 1, VR_F32, &bytes) != VR_OK);
    EXPECT(vr_frame_workspace_size(-1, &bytes) == VR_ERR_INVALID_ARG);
    EXPECT(vr_frame_workspace_size(64, &bytes) == VR_OK && bytes > 0);
    EXPECT(vr_batch_workspace_size(-1, 1, &bytes) != VR_OK);

    // context
    vr_context ctx = nullptr;
    EXPECT(vr_context_create(5, nullptr, &ctx) == VR_ERR_INVALID_ARG);
    EXPECT(vr_context_create(0, nullptr, &ctx) == VR_OK && ctx);
    EXPECT(vr_last_error(ctx) != nullptr);
    EXPECT(vr_set_render_params(ctx, -1.0, 0.0f) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_render_params(ctx, NAN, 0.0f) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_render_params(ctx, 0.5, 1.5f) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_render_params(ctx, 0.5, 0.0f) == VR_OK);
    EXPECT(vr_set_march_path(ctx, (vr_path)7) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_march_config(ctx, VR_F32, VR_STAGING_SLAB, 32, 4) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_march_config(ctx, VR_F32, VR_STAGING_RING, 24, 4) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_march_config(ctx, (vr_dtype)3, VR_STAGING_RING, 32, 4) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_march_config(ctx, VR_F16, VR_STAGING_RING, 16, 8) == VR_OK);

    // transfer function
    std::vector<float> tf(256 * 4, 0.5f);
    EXPECT(vr_set_transfer_function(ctx, tf.data(), 255, 0.f, 1.f, 1.f) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_transfer_function(ctx, tf.data(), 256, 1.f, 0.f, 1.f) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_transfer_function(ctx, tf.data(), 256, 0.f, 1.f, -1.f) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_transfer_function(ctx, tf.data(), 256, 0.f, 1.f, 1.f) == VR_OK);

    // bricks: two float32, one float16
    const int32_t dims[3][3] = {{30, 20, 10}, {17, 20, 10}, {8, 8, 33}};
    const double origins[3][3] = {{0, 0, 0}, {30, 0, 0}, {0, 20, 0}};
    const double spacing[3] = {1, 1, 1};
    vr_brick bricks[3];
    void* ws[3];
    for (int i = 0; i < 3; ++i) {
        const vr_dtype st = i == 2 ? VR_F16 : VR_F32;
        EXPECT(vr_brick_workspace_size(dims[i], 1, st, &bytes) == VR_OK);
        ws[i] = aligned_buf(bytes);
        vr_brick b = nullptr;
        EXPECT(vr_brick_create(ctx, dims[i], 1, origins[i], spacing, st, ws[i], bytes - 1, &b) ==
               VR_ERR_WORKSPACE);
        EXPECT(vr_brick_create(ctx, dims[i], 1, origins[i], spacing, st,
                               static_cast<char*>(ws[i]) + 4, bytes, &b) == VR_ERR_WORKSPACE);
        const double bad_sp[3] = {1, 0, 1};
        EXPECT(vr_brick_create(ctx, dims[i], 1, origins[i], bad_sp, st, ws[i], bytes, &b) ==
               VR_ERR_INVALID_ARG);
        EXPECT(vr_brick_create(ctx, dims[i], 1, origins[i], spacing, st, ws[i], bytes, &bricks[i]) == VR_OK);
        std::vector<float> vox((size_t)(dims[i][0] + 2) * (dims[i][1] + 2) * (dims[i][2] + 2), 0.25f);
        EXPECT(vr_brick_set_data(bricks[i], vox.data()) == VR_OK);
    }
    const int32_t vol[3] = {47, 40, 33}, lo_ok[3] = {0, 0, 0}, lo_bad[3] = {40, 0, 0};
    std::vector<float> volume((size_t)vol[0] * vol[1] * vol[2], 0.5f);
    EXPECT(vr_brick_set_data_global(bricks[0], volume.data(), vol, lo_ok) == VR_OK);
    EXPECT(vr_brick_set_data_global(bricks[0], volume.data(), vol, lo_bad) == VR_ERR_INVALID_ARG);

    // no camera yet
    int32_t roi[4];
    EXPECT(vr_partial_roi(ctx, bricks[0], roi) == VR_ERR_STATE);
    const double eye[3] = {23, 20, -80}, tgt[3] = {23, 20, 16}, up[3] = {0, 1, 0}, up_bad[3] = {0, 0, 1};
    EXPECT(vr_set_camera_perspective(ctx, eye, eye, up, 45, 64, 48) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_camera_perspective(ctx, eye, tgt, up_bad, 45, 64, 48) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_camera_perspective(ctx, eye, tgt, up, 180, 64, 48) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_camera_perspective(ctx, eye, tgt, up, 45, 0, 48) == VR_ERR_INVALID_ARG);
    EXPECT(vr_set_camera_perspective(ctx, eye, tgt, up, 45, 64, 48) == VR_OK);

    // partials of the frame
    vr_partial parts[3];
    std::vector<void*> bufs;
    for (int i = 0; i < 3; ++i) {
        EXPECT(vr_partial_roi(ctx, bricks[i], roi) == VR_OK);
        EXPECT(roi[0] >= 0 && roi[1] >= 0 && roi[0] + roi[2] <= 64 && roi[1] + roi[3] <= 48);
        const size_t px = (size_t)(roi[2] > 0 ? roi[2] : 1) * (roi[3] > 0 ? roi[3] : 1);
        float* rgba = static_cast<float*>(aligned_buf(px * 16));
        float* depth = static_cast<float*>(aligned_buf(px * 4));
        bufs.push_back(rgba);
        bufs.push_back(depth);
        parts[i] = vr_partial{roi[0], roi[1], roi[2], roi[3], rgba, depth, nullptr};
        EXPECT(vr_render_partial(ctx, bricks[i], &parts[i]) == VR_OK);
    }
    vr_partial bad = parts[0];
    bad.x0 = 60;
    bad.w = 10;                                     // past the frame's right edge
    EXPECT(vr_render_partial(ctx, bricks[0], &bad) == VR_ERR_INVALID_ARG);
    bad = parts[0];
    bad.rgba = reinterpret_cast<float*>(reinterpret_cast<char*>(bad.rgba) + 4);   // misaligned
    EXPECT(vr_render_partial(ctx, bricks[0], &bad) == VR_ERR_INVALID_ARG);

    // the frame queue with a workspace, then without
    EXPECT(vr_frame_workspace_size(3, &bytes) == VR_OK);
    void* fws = aligned_buf(bytes);
    EXPECT(vr_render_partials(ctx, 3, bricks, parts, fws, bytes - 1) == VR_ERR_WORKSPACE);
    EXPECT(vr_render_partials(ctx, 3, bricks, parts, fws, bytes) == VR_OK);
    EXPECT(vr_render_partials(ctx, 3, bricks, parts, fws, bytes) == VR_OK);   // both pinned slots
    EXPECT(vr_render_partials(ctx, 0, nullptr, nullptr, nullptr, 0) == VR_OK);
    EXPECT(vr_render_partials_static(ctx, 3, bricks, parts) == VR_OK);
    EXPECT(vr_render_partials_static(ctx, 65, bricks, parts) == VR_ERR_INVALID_ARG);
    // a frame of more partials than the pinned slots hold at first (they grow)
    {
        const int n = 200;
        std::vector<vr_brick> bb(n, bricks[1]);
        std::vector<vr_partial> pp(n, parts[1]);
        EXPECT(vr_frame_workspace_size(n, &bytes) == VR_OK);
        void* big = aligned_buf(bytes);
        EXPECT(vr_render_partials(ctx, n, bb.data(), pp.data(), big, bytes) == VR_OK);
        EXPECT(vr_synchronize(ctx) == VR_OK);
        std::free(big);
    }

    // composite and its backward
    float* out = static_cast<float*>(aligned_buf(64 * 48 * 16));
    const float bg[4] = {0.1f, 0.2f, 0.3f, 1.f}, bg_bad[4] = {NAN, 0, 0, 0};
    EXPECT(vr_composite(ctx, parts, 3, bg, out) == VR_OK);
    EXPECT(vr_composite(ctx, parts, 3, bg_bad, out) == VR_ERR_INVALID_ARG);
    EXPECT(vr_composite(ctx, parts, DPVR_MAX_PARTIALS + 1, bg, out) == VR_ERR_INVALID_ARG);
    EXPECT(vr_composite(ctx, parts, 0, bg, out) == VR_OK);
    float* d_parts[3];
    for (int i = 0; i < 3; ++i) {
        d_parts[i] = static_cast<float*>(aligned_buf((size_t)parts[i].w * parts[i].h * 16 + 16));
        bufs.push_back(d_parts[i]);
    }
    EXPECT(vr_composite_backward(ctx, parts, 3, bg, out, d_parts) == VR_OK);

    // ray-queue cycling: sizes, plan, renders with and without shadows
    {
        size_t rb = 0;
        EXPECT(vr_rqc_workspace_size(ctx, 0, bricks, &rb) == VR_ERR_INVALID_ARG);
        vr_brick twice[2] = {bricks[0], bricks[0]};
        EXPECT(vr_rqc_workspace_size(ctx, 2, twice, &rb) == VR_ERR_INVALID_ARG);
        EXPECT(vr_rqc_workspace_size(ctx, 3, bricks, &rb) == VR_OK && rb > 0);
        void* rws = aligned_buf(rb);
        int64_t total = -1;
        vr_light light = {{1.0, 0.5, -0.25}, 0.3f, 0};
        float* frame = static_cast<float*>(aligned_buf(64 * 48 * 16));
        EXPECT(vr_render_rqc(ctx, 3, bricks, &light, bg, rws, rb, nullptr, 0, frame, nullptr) == VR_ERR_STATE);  // no plan
        EXPECT(vr_rqc_plan(ctx, 3, bricks, rws, rb - 1, &total) == VR_ERR_WORKSPACE);
        EXPECT(vr_rqc_plan(ctx, 3, bricks, rws, rb, &total) == VR_OK && total >= 0);
        float* shade = static_cast<float*>(aligned_buf((size_t)(total > 0 ? total : 1) * 4));
        EXPECT(vr_render_rqc(ctx, 3, bricks, &light, bg, rws, rb, shade, 0, frame, nullptr) ==
               (total > 0 ? VR_ERR_WORKSPACE : VR_OK));
        EXPECT(vr_render_rqc(ctx, 3, bricks, &light, bg, rws, rb, shade, (size_t)total * 4, frame, nullptr) == VR_OK);
        vr_light off = {{0.0, 0.0, 0.0}, 1.0f, 0};
        EXPECT(vr_render_rqc(ctx, 3, bricks, &off, bg, rws, rb, nullptr, 0, frame, nullptr) == VR_ERR_INVALID_ARG);
        off.direction[1] = 1.0;
        EXPECT(vr_render_rqc(ctx, 3, bricks, &off, bg, rws, rb, nullptr, 0, frame, nullptr) == VR_OK);
        light.ambient = 1.5f;
        EXPECT(vr_render_rqc(ctx, 3, bricks, &light, bg, rws, rb, shade, (size_t)total * 4, frame, nullptr) ==
               VR_ERR_INVALID_ARG);
        EXPECT(vr_render_rqc(ctx, 2, bricks, &off, bg, rws, rb, nullptr, 0, frame, nullptr) == VR_ERR_STATE);  // other bricks
        std::free(shade);
        std::free(frame);
        std::free(rws);
    }

    // tetrahedral parts: a cube of 2 x 2 x 2 lattice cells, 6 tetrahedra
    // each, split into two parts, plus an empty part
    {
        std::vector<double> tv;
        for (int i = 0; i <= 2; ++i)
            for (int j = 0; j <= 2; ++j)
                for (int k = 0; k <= 2; ++k) {
                    tv.push_back(i);
                    tv.push_back(j);
                    tv.push_back(k);
                }
        auto vid = [](int i, int j, int k) { return (i * 3 + j) * 3 + k; };
        const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        std::vector<int32_t> tt;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 2; ++k)
                    for (const auto& pm : perms) {
                        int c[3] = {i, j, k};
                        tt.push_back(vid(c[0], c[1], c[2]));
                        for (int a = 0; a < 3; ++a) {
                            ++c[pm[a]];
                            tt.push_back(vid(c[0], c[1], c[2]));
                        }
                    }
        const int nt = (int)tt.size() / 4, nv = (int)tv.size() / 3;
        vr_tetpart tp[3] = {nullptr, nullptr, nullptr};
        EXPECT(vr_tetpart_create(ctx, tv.data(), nv, tt.data(), 20, &tp[0]) == VR_OK);
        EXPECT(vr_tetpart_create(ctx, tv.data(), nv, tt.data() + 80, nt - 20, &tp[1]) == VR_OK);
        EXPECT(vr_tetpart_create(ctx, tv.data(), 0, tt.data(), 0, &tp[2]) == VR_OK);
        vr_tetpart bad = nullptr;
        std::vector<int32_t> tbad(tt.begin(), tt.begin() + 4);
        tbad[3] = nv;
        EXPECT(vr_tetpart_create(ctx, tv.data(), nv, tbad.data(), 1, &bad) == VR_ERR_INVALID_ARG && !bad);
        tbad[3] = tbad[0];
        EXPECT(vr_tetpart_create(ctx, tv.data(), nv, tbad.data(), 1, &bad) == VR_ERR_INVALID_ARG);
        EXPECT(vr_tetpart_create(ctx, nullptr, nv, tt.data(), 1, &bad) == VR_ERR_INVALID_ARG);
        std::vector<double> tnan(tv);
        tnan[5] = NAN;
        EXPECT(vr_tetpart_create(ctx, tnan.data(), nv, tt.data(), nt, &bad) == VR_ERR_INVALID_ARG);
        double lo[3], hi[3];
        int32_t grid[3];
        int64_t entries = 0;
        size_t need[3] = {0, 0, 0};
        int32_t ntets = 0;
        for (int q = 0; q < 3; ++q) EXPECT(vr_tetpart_info(tp[q], lo, hi, grid, &entries, &need[q], nullptr) == VR_OK);
        EXPECT(vr_tetpart_info(tp[1], lo, hi, grid, &entries, nullptr, &ntets) == VR_OK && entries >= nt - 20 &&
               ntets == nt - 20);
        EXPECT(hi[0] == 2.0 && lo[0] == 0.0 && grid[0] >= 1);
        // mixed cells: one hexahedron, two wedges and a pyramid on the unit cubes of the lattice
        {
            auto h8 = [&](int i, int j, int k, int32_t out8[8]) {
                const int c[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
                for (int a = 0; a < 8; ++a) out8[a] = vid(i + c[a][0], j + c[a][1], k + c[a][2]);
            };
            int32_t h[8], w[8];
            h8(0, 0, 0, h);
            h8(1, 0, 0, w);
            std::vector<uint8_t> sizes = {8, 6, 6, 5};
            std::vector<int32_t> cells(h, h + 8);
            for (int a : {0, 1, 2, 4, 5, 6, 0, 2, 3, 4, 6, 7}) cells.push_back(w[a]);
            int32_t pz[8];
            h8(0, 1, 0, pz);
            for (int a : {0, 1, 2, 3}) cells.push_back(pz[a]);
            cells.push_back(pz[6]);   // apex on the opposite corner (a valid, if skewed, pyramid)
            std::vector<int64_t> ids(nv);
            for (int v = 0; v < nv; ++v) ids[v] = 1000 + v;
            vr_tetpart mp = nullptr;
            EXPECT(vr_tetpart_create_cells(ctx, tv.data(), nv, ids.data(), sizes.data(), cells.data(), 4, &mp) == VR_OK);
            size_t mneed = 0;
            EXPECT(vr_tetpart_info(mp, lo, hi, grid, &entries, &mneed, &ntets) == VR_OK && ntets == 12 + 8 + 8 + 2);
            std::vector<uint8_t> bad = {8, 7};
            vr_tetpart bp = nullptr;
            EXPECT(vr_tetpart_create_cells(ctx, tv.data(), nv, nullptr, bad.data(), cells.data(), 2, &bp) ==
                   VR_ERR_INVALID_ARG && !bp);
            cells[3] = nv + 5;
            EXPECT(vr_tetpart_create_cells(ctx, tv.data(), nv, nullptr, sizes.data(), cells.data(), 4, &bp) ==
                   VR_ERR_INVALID_ARG);
            void* mws = aligned_buf(mneed);
            EXPECT(vr_tetpart_attach(mp, mws, mneed) == VR_OK);
            float* mv = static_cast<float*>(aligned_buf(nv * 4));
            for (int v = 0; v < nv; ++v) mv[v] = 0.5f;
            EXPECT(vr_tetpart_set_values(mp, mv) == VR_OK);
            EXPECT(vr_tetpart_release(mp) == VR_OK);
            std::free(mws);
            std::free(mv);
        }
        float* vals = static_cast<float*>(aligned_buf(nv * 4));
        for (int v = 0; v < nv; ++v) vals[v] = 0.1f * v;
        void* tws[3];
        for (int q = 0; q < 3; ++q) {
            tws[q] = aligned_buf(need[q]);
            EXPECT(vr_tetpart_set_values(tp[q], vals) == VR_ERR_STATE);   // no workspace yet
            EXPECT(vr_tetpart_attach(tp[q], tws[q], need[q] - 1) == VR_ERR_WORKSPACE);
            EXPECT(vr_tetpart_attach(tp[q], tws[q], need[q]) == VR_OK);
        }
        size_t fb = 0;
        EXPECT(vr_tetparts_workspace_size(ctx, 3, tp, 0, &fb) == VR_ERR_INVALID_ARG);
        EXPECT(vr_tetparts_workspace_size(ctx, 3, tp, DPVR_MAX_TET_RUNS + 1, &fb) == VR_ERR_INVALID_ARG);
        vr_tetpart twice[2] = {tp[0], tp[0]};
        EXPECT(vr_tetparts_workspace_size(ctx, 2, twice, 4, &fb) == VR_ERR_INVALID_ARG);
        EXPECT(vr_tetparts_workspace_size(ctx, 3, tp, 4, &fb) == VR_OK && fb > 0);
        void* fw = aligned_buf(fb);
        float* frame = static_cast<float*>(aligned_buf(64 * 48 * 16));
        EXPECT(vr_render_tetparts(ctx, 3, tp, 4, bg, fw, fb, frame, nullptr) == VR_ERR_STATE);   // no values
        for (int q = 0; q < 3; ++q) EXPECT(vr_tetpart_set_values(tp[q], vals) == VR_OK);
        EXPECT(vr_render_tetparts(ctx, 3, tp, 4, bg, fw, fb - 1, frame, nullptr) == VR_ERR_WORKSPACE);
        EXPECT(vr_render_tetparts(ctx, 3, tp, 4, bg_bad, fw, fb, frame, nullptr) == VR_ERR_INVALID_ARG);
        EXPECT(vr_render_tetparts(ctx, 3, tp, 4, bg, fw, fb, frame + 1, nullptr) == VR_ERR_INVALID_ARG);
        EXPECT(vr_render_tetparts(ctx, 3, tp, 4, bg, fw, fb, frame, nullptr) == VR_OK);
        EXPECT(vr_set_tet_locator(ctx, (vr_tet_locator)7) == VR_ERR_INVALID_ARG);
        EXPECT(vr_set_tet_locator(ctx, VR_TET_BVH) == VR_OK);
        EXPECT(vr_render_tetparts(ctx, 2, tp + 1, 1, bg, fw, fb, frame, nullptr) == VR_OK);
        EXPECT(vr_set_tet_locator(ctx, VR_TET_GRID) == VR_OK);
        EXPECT(vr_resolve_tetparts(ctx, 3, tp, 4, bg, fw, fb, frame) == VR_ERR_STATE);   // last march: other parts
        EXPECT(vr_march_tetparts(ctx, 3, tp, 4, fw, fb, nullptr) == VR_OK);
        EXPECT(vr_resolve_tetparts(ctx, 3, tp, 2, bg, fw, fb, frame) == VR_ERR_STATE);   // other max_runs
        EXPECT(vr_resolve_tetparts(ctx, 3, tp, 4, bg, fw, fb, frame) == VR_OK);
        // shadow rays: plan, slots, render
        size_t pb = 0, sb = 0;
        int64_t total = -1;
        EXPECT(vr_tetparts_shadow_plan_size(ctx, 3, tp, &pb) == VR_OK && pb > 0);
        void* plan = aligned_buf(pb);
        vr_light tl = {{0.2, 1.0, -0.3}, 0.25f, 0};
        EXPECT(vr_render_tetparts_shadowed(ctx, 3, tp, 4, &tl, bg, fw, fb, plan, pb, nullptr, 0, frame, nullptr) ==
               VR_ERR_STATE);   // no plan yet
        EXPECT(vr_tetparts_shadow_plan(ctx, 3, tp, 4, fw, fb, plan, pb - 1, &total) == VR_ERR_WORKSPACE);
        EXPECT(vr_tetparts_shadow_plan(ctx, 3, tp, 4, fw, fb, plan, pb, nullptr) == VR_ERR_INVALID_ARG);
        EXPECT(vr_tetparts_shadow_plan(ctx, 3, tp, 4, fw, fb, plan, pb, &total) == VR_OK && total >= 0);
        EXPECT(vr_tetparts_slot_bytes(total, &sb) == VR_OK);
        EXPECT(vr_tetparts_slot_bytes(-1, &sb) == VR_ERR_INVALID_ARG);
        EXPECT(vr_tetparts_slot_bytes(total, &sb) == VR_OK);
        void* slots = aligned_buf(sb > 0 ? sb : 1);
        if (total > 0)
            EXPECT(vr_render_tetparts_shadowed(ctx, 3, tp, 4, &tl, bg, fw, fb, plan, pb, slots, sb - 1, frame,
                                               nullptr) == VR_ERR_WORKSPACE);
        EXPECT(vr_render_tetparts_shadowed(ctx, 3, tp, 4, &tl, bg, fw, fb, plan, pb, slots, sb, frame, nullptr) ==
               VR_OK);
        vr_light zero = {{0.0, 0.0, 0.0}, 0.5f, 0};
        EXPECT(vr_render_tetparts_shadowed(ctx, 3, tp, 4, &zero, bg, fw, fb, plan, pb, slots, sb, frame, nullptr) ==
               VR_ERR_INVALID_ARG);
        EXPECT(vr_render_tetparts_shadowed(ctx, 2, tp, 4, &tl, bg, fw, fb, plan, pb, slots, sb, frame, nullptr) ==
               VR_ERR_STATE);   // other parts than planned
        EXPECT(vr_resolve_tetparts(ctx, 3, tp, 4, bg, fw, fb, frame) == VR_OK);   // the shaded march counts
        std::free(plan);
        std::free(slots);
        EXPECT(frame[0] == bg[0] && frame[3] == bg[3]);
        EXPECT(vr_context_release(ctx) == VR_ERR_STATE);     // parts still live
        for (int q = 0; q < 3; ++q) EXPECT(vr_tetpart_release(tp[q]) == VR_OK);
        EXPECT(vr_tetpart_release(tp[0]) == VR_ERR_INVALID_HANDLE);
        EXPECT(vr_render_tetparts(ctx, 1, tp, 4, bg, fw, fb, frame, nullptr) == VR_ERR_INVALID_HANDLE);
        for (int q = 0; q < 3; ++q) std::free(tws[q]);
        std::free(fw);
        std::free(frame);
        std::free(vals);
    }

    // time-step streaming: three steps of the three bricks, two resident
    {
        vr_brick_desc desc[3];
        for (int i = 0; i < 3; ++i) {
            std::memcpy(desc[i].dims, dims[i], sizeof desc[i].dims);
            desc[i].ghost = 1;
            std::memcpy(desc[i].origin, origins[i], sizeof desc[i].origin);
            std::memcpy(desc[i].spacing, spacing, sizeof desc[i].spacing);
            desc[i].storage = i == 2 ? VR_F16 : VR_F32;
            desc[i].pad_ = 0;
        }
        size_t tb = 0;
        EXPECT(vr_timeseries_workspace_size(3, desc, 0, &tb) == VR_ERR_INVALID_ARG);
        EXPECT(vr_timeseries_workspace_size(3, desc, 2, &tb) == VR_OK && tb > 0);
        std::vector<std::vector<float>> host;
        std::vector<const float*> ptrs;
        for (int t = 0; t < 3; ++t)
            for (int i = 0; i < 3; ++i)
                host.emplace_back((size_t)(dims[i][0] + 2) * (dims[i][1] + 2) * (dims[i][2] + 2), 0.1f * t);
        for (auto& h : host) ptrs.push_back(h.data());
        void* tws = aligned_buf(tb);
        vr_timeseries ts = nullptr;
        EXPECT(vr_timeseries_create(ctx, 3, desc, 3, ptrs.data(), 2, tws, tb - 1, &ts) == VR_ERR_WORKSPACE);
        EXPECT(vr_timeseries_create(ctx, 3, desc, 3, ptrs.data(), 2, tws, tb, &ts) == VR_OK);
        vr_brick got[3];
        EXPECT(vr_timeseries_acquire(ts, 3, got) == VR_ERR_INVALID_ARG);
        EXPECT(vr_timeseries_acquire(ts, 0, got) == VR_OK);
        EXPECT(vr_brick_release(got[0]) == VR_ERR_STATE);
        EXPECT(vr_render_partials_static(ctx, 3, got, parts) == VR_OK);
        EXPECT(vr_timeseries_prefetch(ts, 1) == VR_OK);
        EXPECT(vr_timeseries_acquire(ts, 2, got) == VR_OK);     // evicts step 0 (least recently used)
        int64_t loads = 0;
        int32_t res[2] = {-2, -2};
        EXPECT(vr_timeseries_stats(ts, &loads, res) == VR_OK);
        EXPECT(loads == 3 && ((res[0] == 2 && res[1] == 1) || (res[0] == 1 && res[1] == 2)));
        EXPECT(vr_timeseries_acquire(ts, 1, got) == VR_OK);     // resident: no load
        EXPECT(vr_timeseries_stats(ts, &loads, nullptr) == VR_OK && loads == 3);
        EXPECT(vr_context_release(ctx) == VR_ERR_STATE);
        EXPECT(vr_timeseries_release(ts) == VR_OK);
        EXPECT(vr_timeseries_release(ts) == VR_ERR_INVALID_HANDLE);
        std::free(tws);
    }

    // checkpointed forward and adjoint of one partial
    size_t ck = 0;
    EXPECT(vr_checkpoint_size(ctx, bricks[0], &parts[0], 0, &ck) == VR_ERR_INVALID_ARG);
    EXPECT(vr_checkpoint_size(ctx, bricks[0], &parts[0], 65, &ck) == VR_ERR_INVALID_ARG);
    EXPECT(vr_checkpoint_size(ctx, bricks[0], &parts[0], 16, &ck) == VR_OK && ck > 0);
    float* ckpt = static_cast<float*>(aligned_buf(ck));
    EXPECT(vr_render_partial_checkpointed(ctx, bricks[0], &parts[0], 16, ckpt, ck - 4) == VR_ERR_WORKSPACE);
    EXPECT(vr_render_partial_checkpointed(ctx, bricks[0], &parts[0], 16, ckpt, ck) == VR_OK);
    float* gtf = static_cast<float*>(aligned_buf(256 * 16));
    float* gvol = static_cast<float*>(aligned_buf(volume.size() * 4));
    EXPECT(vr_render_partial_backward(ctx, bricks[0], &parts[0], 16, ckpt, ck, d_parts[0], gtf, gvol, vol,
                                      lo_ok) == VR_OK);
    EXPECT(vr_render_partial_backward(ctx, bricks[0], &parts[0], 16, ckpt, ck, d_parts[0], gtf, gvol, vol,
                                      lo_bad) == VR_ERR_INVALID_ARG);
    {
        size_t cb = 0;
        EXPECT(vr_checkpointed_workspace_size(2, &cb) == VR_OK && cb > 0);
        void* cws = aligned_buf(cb);
        float* cks2[2] = {ckpt, ckpt};
        const size_t ckb2[2] = {ck, ck - 4};
        vr_brick two2[2] = {bricks[0], bricks[0]};
        vr_partial pp2[2] = {parts[0], parts[0]};
        EXPECT(vr_render_partials_checkpointed(ctx, 2, two2, pp2, 16, cks2, ckb2, cws, cb) == VR_ERR_WORKSPACE);
        const size_t ckb3[2] = {ck, ck};
        EXPECT(vr_render_partials_checkpointed(ctx, 2, two2, pp2, 16, cks2, ckb3, cws, cb) == VR_OK);
        std::free(cws);
    }
    {
        size_t bb = 0;
        EXPECT(vr_backward_workspace_size(2, &bb) == VR_OK && bb > 0);
        void* bws_ = aligned_buf(bb);
        const float* cks[2] = {ckpt, ckpt};
        const size_t ckb[2] = {ck, ck};
        const float* dps[2] = {d_parts[0], d_parts[0]};
        const int32_t los[6] = {0, 0, 0, 0, 0, 0};
        vr_brick two[2] = {bricks[0], bricks[0]};
        vr_partial pp[2] = {parts[0], parts[0]};
        EXPECT(vr_render_partials_backward(ctx, 2, two, pp, 16, cks, ckb, dps, gtf, gvol, vol, los, bws_, bb - 1) ==
               VR_ERR_WORKSPACE);
        EXPECT(vr_render_partials_backward(ctx, 2, two, pp, 16, cks, ckb, dps, gtf, gvol, vol, los, bws_, bb) == VR_OK);
        const int32_t los_bad[6] = {0, 0, 0, 40, 0, 0};
        EXPECT(vr_render_partials_backward(ctx, 2, two, pp, 16, cks, ckb, dps, gtf, gvol, vol, los_bad, bws_, bb) ==
               VR_ERR_INVALID_ARG);
        std::free(bws_);
    }

    // a batch of two frames (two cameras), its launch, tuning and release
    vr_camera_desc cams[2] = {};
    for (int c = 0; c < 2; ++c) {
        cams[c].kind = c;
        cams[c].width = 40 + 8 * c;
        cams[c].height = 32;
        std::memcpy(cams[c].eye, c == 0 ? eye : tgt, sizeof eye);
        const double dir[3] = {0, 0, 1};
        std::memcpy(cams[c].target, c == 0 ? tgt : dir, sizeof tgt);
        std::memcpy(cams[c].up, up, sizeof up);
        cams[c].fovy_deg = c == 0 ? 40.0 : 50.0;
    }
    vr_tf_desc tfs[1] = {{tf.data(), 0.f, 1.f, 1.f, 0}};
    std::vector<vr_batch_job> jobs;
    std::vector<vr_batch_frame> frames;
    for (int c = 0; c < 2; ++c) {
        vr_batch_frame f{};
        f.camera = c;
        f.first_job = (int32_t)jobs.size();
        f.n_jobs = 3;
        f.out = static_cast<float*>(aligned_buf((size_t)cams[c].width * cams[c].height * 16));
        bufs.push_back(f.out);
        for (int i = 0; i < 3; ++i) {
            int32_t r[4];
            EXPECT(vr_camera_roi(ctx, bricks[i], &cams[c], r) == VR_OK);
            const size_t px = (size_t)(r[2] > 0 ? r[2] : 1) * (r[3] > 0 ? r[3] : 1);
            float* rgba = static_cast<float*>(aligned_buf(px * 16));
            float* depth = static_cast<float*>(aligned_buf(px * 4));
            bufs.push_back(rgba);
            bufs.push_back(depth);
            jobs.push_back(vr_batch_job{bricks[i], c, 0, vr_partial{r[0], r[1], r[2], r[3], rgba, depth, nullptr}});
        }
        frames.push_back(f);
    }
    {   // a job no frame uses (it runs with the last release group)
        int32_t r[4];
        EXPECT(vr_camera_roi(ctx, bricks[0], &cams[0], r) == VR_OK);
        const size_t px = (size_t)(r[2] > 0 ? r[2] : 1) * (r[3] > 0 ? r[3] : 1);
        float* rgba = static_cast<float*>(aligned_buf(px * 16));
        float* depth = static_cast<float*>(aligned_buf(px * 4));
        bufs.push_back(rgba);
        bufs.push_back(depth);
        jobs.push_back(vr_batch_job{bricks[0], 0, 0, vr_partial{r[0], r[1], r[2], r[3], rgba, depth, nullptr}});
    }
    EXPECT(vr_batch_workspace_size((int32_t)jobs.size(), (int32_t)frames.size(), &bytes) == VR_OK);
    void* bws = aligned_buf(bytes);
    vr_batch batch = nullptr;
    std::vector<vr_batch_job> bad_jobs = jobs;
    bad_jobs[1].camera = 7;
    EXPECT(vr_batch_create(ctx, 2, cams, 1, tfs, (int32_t)bad_jobs.size(), bad_jobs.data(), 2, frames.data(), bws,
                           bytes, &batch) == VR_ERR_INVALID_ARG);
    EXPECT(vr_batch_create(ctx, 2, cams, 1, tfs, (int32_t)jobs.size(), jobs.data(), 2, frames.data(), bws,
                           bytes - 1, &batch) == VR_ERR_WORKSPACE);
    EXPECT(vr_batch_create(ctx, 2, cams, 1, tfs, (int32_t)jobs.size(), jobs.data(), 2, frames.data(), bws,
                           bytes, &batch) == VR_OK);
    EXPECT(vr_batch_launch(batch) == VR_OK);
    double best = 0;
    EXPECT(vr_batch_autotune(batch, 0, &best) == VR_ERR_INVALID_ARG);
    EXPECT(vr_batch_autotune(batch, 1, &best) == VR_OK);
    int32_t wg, order, staging, tile, chunk;
    EXPECT(vr_batch_config(batch, &wg, &order, &staging, &tile, &chunk) == VR_OK);
    EXPECT(wg >= 1 && (order == 0 || order == 1) && (tile == 16 || tile == 32) && (chunk == 4 || chunk == 8));
    // release groups: every job rendered once, frames composited in order,
    // a group's composites after its own queues
    EXPECT(vr_batch_set_groups(batch, 0) == VR_ERR_INVALID_ARG);
    EXPECT(vr_batch_set_groups(batch, 3) == VR_ERR_INVALID_ARG);
    for (int G = 1; G <= 2; ++G) {
        fake_reset_launches();
        EXPECT(vr_batch_set_groups(batch, G) == VR_OK);
        const void* seen[64];
        const size_t np = fake_queue_parts(seen, 64);
        EXPECT(np == jobs.size());
        for (const auto& j : jobs) {
            int hits = 0;
            for (size_t i = 0; i < np && i < 64; ++i) hits += seen[i] == j.part.rgba;
            EXPECT(hits == 1);
        }
        const void* fr[8];
        EXPECT(fake_composite_frames(fr, 8) == 2 && fr[0] == frames[0].out && fr[1] == frames[1].out);
        int32_t f0 = -1, nf = -1;
        for (int g = 0; g < G; ++g) {
            EXPECT(vr_batch_group(batch, g, &f0, &nf) == VR_OK);
            EXPECT(f0 == (G == 1 ? 0 : g) && nf == (G == 1 ? 2 : 1));
        }
        EXPECT(vr_batch_group(batch, G, &f0, &nf) == VR_ERR_INVALID_ARG);
        EXPECT(vr_batch_launch(batch) == VR_OK);
        int32_t done = -1;
        EXPECT(vr_batch_wait_group(batch, G - 1, nullptr) == VR_OK);
        EXPECT(vr_batch_group_done(batch, G - 1, &done) == VR_OK && done == 1);
        EXPECT(vr_batch_group_done(batch, G, &done) == VR_ERR_INVALID_ARG);
        EXPECT(vr_batch_group_done(batch, 0, nullptr) == VR_ERR_INVALID_ARG);
        EXPECT(vr_batch_wait_group(batch, -1, nullptr) == VR_ERR_INVALID_ARG);
    }
    EXPECT(vr_batch_autotune(batch, 1, &best) == VR_OK);   // tunes the grouped batch
    EXPECT(vr_context_release(ctx) == VR_ERR_STATE);     // bricks and the batch still live
    EXPECT(vr_batch_release(batch) == VR_OK);
    EXPECT(vr_batch_release(batch) == VR_ERR_INVALID_HANDLE);

    // release, then use of released handles
    for (int i = 0; i < 3; ++i) EXPECT(vr_brick_release(bricks[i]) == VR_OK);
    EXPECT(vr_brick_release(bricks[0]) == VR_ERR_INVALID_HANDLE);
    EXPECT(vr_synchronize(ctx) == VR_OK);
    EXPECT(vr_context_release(ctx) == VR_OK);
    EXPECT(vr_context_release(ctx) == VR_ERR_INVALID_HANDLE);
    EXPECT(vr_set_render_params(ctx, 0.5, 0.0f) == VR_ERR_INVALID_HANDLE);

    for (void* p : bufs) std::free(p);
    for (void* p : ws) std::free(p);
    std::free(fws);
    std::free(out);
    std::free(ckpt);
    std::free(gtf);
    std::free(gvol);
    std::free(bws);
    std::printf("%s: %d failed expectations\n", g_fail ? "FAIL" : "OK", g_fail);
    return g_fail ? 1 : 0;
}
