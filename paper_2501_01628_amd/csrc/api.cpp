// Host side of the C-ABI declared in include/dpvr.h: handle bookkeeping,
// argument validation (always before anything is enqueued), the float64
// camera frame, region-of-interest projection and kernel launches.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>

#include "../../include/dpvr.h"
#include "dpvr_kernels.h"

using namespace dpvr;

struct vr_context_s {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    bool has_camera = false, has_tf = false;
    CameraK cam{};
    TFK tf{};
    double dt = 0.5;
    float ert_eps = 0x1p-20f;
    int32_t live_bricks = 0;
    std::string err;
};

struct vr_brick_s {
    vr_context ctx = nullptr;
    int32_t dims[3] = {0, 0, 0};
    int32_t ghost = 1;
    double origin[3] = {0, 0, 0}, spacing[3] = {1, 1, 1};
    vr_dtype storage = VR_F32;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool has_data = false;
};

namespace {

std::mutex g_mu;
std::unordered_set<const void*> g_live;   // live context and brick handles
thread_local std::string t_err;

bool live(const void* h) {
    std::lock_guard<std::mutex> lk(g_mu);
    return h && g_live.count(h);
}

vr_status fail(vr_context ctx, vr_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx && live(ctx))
        ctx->err = buf;
    else
        t_err = buf;
    return st;
}

vr_status ok(vr_context ctx) {
    if (ctx) ctx->err.clear();
    return VR_OK;
}

// Switch to the context's device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool finite3(const double v[3]) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

int64_t stored_count(const int32_t dims[3], int32_t ghost) {
    return (int64_t)(dims[0] + 2 * ghost) * (dims[1] + 2 * ghost) * (dims[2] + 2 * ghost);
}

// float64 vector helpers; the operation order matches the documented camera
// formula (no contraction: this file is compiled with -ffp-contract=off).
void sub3(const double a[3], const double b[3], double r[3]) {
    r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
void cross3(const double a[3], const double b[3], double r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
double norm3(const double v[3]) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }
void scale3(double v[3], double n) { v[0] = v[0] / n; v[1] = v[1] / n; v[2] = v[2] / n; }
double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

vr_status make_frame(vr_context ctx, const double fwd[3], const double up[3], CameraK& cam) {
    double f[3] = {fwd[0], fwd[1], fwd[2]};
    double nf = norm3(f);
    if (!(nf > 0) || !std::isfinite(nf)) return fail(ctx, VR_ERR_INVALID_ARG, "camera: zero view direction");
    scale3(f, nf);
    double r[3];
    cross3(f, up, r);
    double nr = norm3(r);
    if (!(nr > 1e-12 * norm3(up)) || !std::isfinite(nr))
        return fail(ctx, VR_ERR_INVALID_ARG, "camera: up vector parallel to the view direction");
    scale3(r, nr);
    double u[3];
    cross3(r, f, u);
    for (int c = 0; c < 3; ++c) { cam.f[c] = f[c]; cam.r[c] = r[c]; cam.u[c] = u[c]; }
    return VR_OK;
}

}  // namespace

extern "C" {

int32_t vr_abi_version(void) { return DPVR_ABI_VERSION; }

const char* vr_status_string(vr_status s) {
    switch (s) {
        case VR_OK: return "VR_OK";
        case VR_ERR_INVALID_ARG: return "VR_ERR_INVALID_ARG";
        case VR_ERR_INVALID_HANDLE: return "VR_ERR_INVALID_HANDLE";
        case VR_ERR_WORKSPACE: return "VR_ERR_WORKSPACE";
        case VR_ERR_UNSUPPORTED: return "VR_ERR_UNSUPPORTED";
        case VR_ERR_DEVICE: return "VR_ERR_DEVICE";
        case VR_ERR_STATE: return "VR_ERR_STATE";
    }
    return "VR_ERR_UNKNOWN";
}

const char* vr_last_error(vr_context ctx) {
    if (ctx && live(ctx)) return ctx->err.c_str();
    return t_err.c_str();
}

vr_status vr_context_create(int32_t device, void* stream, vr_context* out) {
    if (!out) return fail(nullptr, VR_ERR_INVALID_ARG, "vr_context_create: out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(nullptr, VR_ERR_DEVICE, "vr_context_create: no HIP device available");
    if (device < 0 || device >= count)
        return fail(nullptr, VR_ERR_INVALID_ARG, "vr_context_create: device %d out of range [0, %d)",
                    device, count);
    vr_context c = new (std::nothrow) vr_context_s;
    if (!c) return fail(nullptr, VR_ERR_INVALID_ARG, "vr_context_create: out of host memory");
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(c);
    }
    *out = c;
    return VR_OK;
}

vr_status vr_context_release(vr_context ctx) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_context_release: invalid context");
    if (ctx->live_bricks > 0)
        return fail(ctx, VR_ERR_STATE, "vr_context_release: %d bricks still alive", ctx->live_bricks);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.erase(ctx);
    }
    delete ctx;
    return VR_OK;
}

vr_status vr_context_set_stream(vr_context ctx, void* stream) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_context_set_stream: invalid context");
    ctx->stream = reinterpret_cast<hipStream_t>(stream);
    return ok(ctx);
}

vr_status vr_synchronize(vr_context ctx) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_synchronize: invalid context");
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_synchronize: %s", hipGetErrorString(e));
    e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_synchronize: %s", hipGetErrorString(e));
    return ok(ctx);
}

vr_status vr_brick_workspace_size(const int32_t dims[3], int32_t ghost, vr_dtype storage,
                                  size_t* bytes) {
    if (!dims || !bytes) return fail(nullptr, VR_ERR_INVALID_ARG, "vr_brick_workspace_size: NULL argument");
    if (ghost != 1) return fail(nullptr, VR_ERR_INVALID_ARG, "vr_brick_workspace_size: ghost must be 1 (got %d)", ghost);
    if (storage != VR_F32 && storage != VR_F16)
        return fail(nullptr, VR_ERR_INVALID_ARG, "vr_brick_workspace_size: unknown storage %d", (int)storage);
    for (int c = 0; c < 3; ++c)
        if (dims[c] < 1 || dims[c] > (1 << 20))
            return fail(nullptr, VR_ERR_INVALID_ARG, "vr_brick_workspace_size: dims[%d] = %d out of range", c, dims[c]);
    const int64_t n = stored_count(dims, ghost);
    const size_t elt = storage == VR_F16 ? 2 : 4;
    *bytes = ((size_t)n * elt + 255) & ~(size_t)255;
    return VR_OK;
}

vr_status vr_brick_create(vr_context ctx, const int32_t dims[3], int32_t ghost,
                          const double origin[3], const double spacing[3], vr_dtype storage,
                          void* workspace, size_t workspace_bytes, vr_brick* out) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_brick_create: invalid context");
    if (!out || !origin || !spacing) return fail(ctx, VR_ERR_INVALID_ARG, "vr_brick_create: NULL argument");
    *out = nullptr;
    size_t need = 0;
    vr_status st = vr_brick_workspace_size(dims, ghost, storage, &need);
    if (st != VR_OK) return fail(ctx, st, "vr_brick_create: %s", t_err.c_str());
    if (!finite3(origin)) return fail(ctx, VR_ERR_INVALID_ARG, "vr_brick_create: origin not finite");
    for (int c = 0; c < 3; ++c)
        if (!(spacing[c] > 0) || !std::isfinite(spacing[c]))
            return fail(ctx, VR_ERR_INVALID_ARG, "vr_brick_create: spacing[%d] must be finite and > 0", c);
    if (!workspace) return fail(ctx, VR_ERR_WORKSPACE, "vr_brick_create: workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(ctx, VR_ERR_WORKSPACE, "vr_brick_create: workspace must be 256-byte aligned");
    if (workspace_bytes < need)
        return fail(ctx, VR_ERR_WORKSPACE, "vr_brick_create: workspace holds %zu bytes, need %zu",
                    workspace_bytes, need);
    vr_brick b = new (std::nothrow) vr_brick_s;
    if (!b) return fail(ctx, VR_ERR_INVALID_ARG, "vr_brick_create: out of host memory");
    b->ctx = ctx;
    for (int c = 0; c < 3; ++c) {
        b->dims[c] = dims[c];
        b->origin[c] = origin[c];
        b->spacing[c] = spacing[c];
    }
    b->ghost = ghost;
    b->storage = storage;
    b->ws = workspace;
    b->ws_bytes = workspace_bytes;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(b);
    }
    ctx->live_bricks++;
    *out = b;
    return ok(ctx);
}

vr_status vr_brick_set_data(vr_brick b, const float* voxels) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_brick_set_data: invalid brick");
    vr_context ctx = b->ctx;
    if (!voxels) return fail(ctx, VR_ERR_INVALID_ARG, "vr_brick_set_data: voxels is NULL");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_brick_set_data: cannot select device %d", ctx->device);
    hipError_t e = launch_ingest(voxels, b->ws, stored_count(b->dims, b->ghost),
                                 b->storage == VR_F16 ? kF16 : kF32, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_brick_set_data: %s", hipGetErrorString(e));
    b->has_data = true;
    return ok(ctx);
}

vr_status vr_brick_release(vr_brick b) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_brick_release: invalid brick");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.erase(b);
    }
    if (live(b->ctx)) b->ctx->live_bricks--;
    delete b;
    return VR_OK;
}

vr_status vr_set_transfer_function(vr_context ctx, const float* rgba, int32_t n, float vmin,
                                   float vmax, float opacity_scale) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_set_transfer_function: invalid context");
    if (!rgba) return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_transfer_function: table is NULL");
    if ((reinterpret_cast<uintptr_t>(rgba) & 15) != 0)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_transfer_function: table must be 16-byte aligned");
    if (n != DPVR_TF_ENTRIES)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_transfer_function: n must be %d (got %d)", DPVR_TF_ENTRIES, n);
    if (!std::isfinite(vmin) || !std::isfinite(vmax) || !(vmin < vmax))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_transfer_function: need finite vmin < vmax");
    if (!(opacity_scale >= 0) || !std::isfinite(opacity_scale))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_transfer_function: opacity_scale must be finite and >= 0");
    ctx->tf.rgba = rgba;
    ctx->tf.n = n;
    ctx->tf.vmin = vmin;
    ctx->tf.vmax = vmax;
    ctx->tf.opacity_scale = opacity_scale;
    ctx->has_tf = true;
    return ok(ctx);
}

vr_status vr_set_camera_perspective(vr_context ctx, const double eye[3], const double target[3],
                                    const double up[3], double fovy_deg, int32_t width,
                                    int32_t height) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_set_camera_perspective: invalid context");
    if (!eye || !target || !up) return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_camera_perspective: NULL argument");
    if (!finite3(eye) || !finite3(target) || !finite3(up))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_camera_perspective: non-finite vector");
    if (!(fovy_deg > 0 && fovy_deg < 180))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_camera_perspective: fovy must be in (0, 180)");
    if (width < 1 || height < 1 || width > 32768 || height > 32768)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_camera_perspective: bad image size %dx%d", width, height);
    CameraK cam{};
    double fwd[3];
    sub3(target, eye, fwd);
    vr_status st = make_frame(ctx, fwd, up, cam);
    if (st != VR_OK) return st;
    const double W = (double)width, H = (double)height;
    const double th = std::tan(0.5 * fovy_deg * (M_PI / 180.0));
    cam.ax = (th * W) / H;
    cam.ay = th;
    for (int c = 0; c < 3; ++c) cam.eye[c] = eye[c];
    cam.kind = 0;
    cam.width = width;
    cam.height = height;
    ctx->cam = cam;
    ctx->has_camera = true;
    return ok(ctx);
}

vr_status vr_set_camera_orthographic(vr_context ctx, const double pos[3], const double dir[3],
                                     const double up[3], double view_height, int32_t width,
                                     int32_t height) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_set_camera_orthographic: invalid context");
    if (!pos || !dir || !up) return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_camera_orthographic: NULL argument");
    if (!finite3(pos) || !finite3(dir) || !finite3(up))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_camera_orthographic: non-finite vector");
    if (!(view_height > 0) || !std::isfinite(view_height))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_camera_orthographic: view_height must be > 0");
    if (width < 1 || height < 1 || width > 32768 || height > 32768)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_camera_orthographic: bad image size %dx%d", width, height);
    CameraK cam{};
    vr_status st = make_frame(ctx, dir, up, cam);
    if (st != VR_OK) return st;
    const double W = (double)width, H = (double)height;
    const double hh = 0.5 * view_height;
    cam.ax = (hh * W) / H;
    cam.ay = hh;
    for (int c = 0; c < 3; ++c) cam.eye[c] = pos[c];
    cam.kind = 1;
    cam.width = width;
    cam.height = height;
    ctx->cam = cam;
    ctx->has_camera = true;
    return ok(ctx);
}

vr_status vr_set_render_params(vr_context ctx, double dt, float ert_epsilon) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_set_render_params: invalid context");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_render_params: dt must be finite and > 0");
    if (!(ert_epsilon >= 0) || !(ert_epsilon < 1))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_render_params: ert_epsilon must be in [0, 1)");
    ctx->dt = dt;
    ctx->ert_eps = ert_epsilon;
    return ok(ctx);
}

vr_status vr_partial_roi(vr_context ctx, vr_brick b, int32_t roi[4]) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_partial_roi: invalid context");
    if (!live(b) || b->ctx != ctx) return fail(ctx, VR_ERR_INVALID_HANDLE, "vr_partial_roi: invalid brick");
    if (!roi) return fail(ctx, VR_ERR_INVALID_ARG, "vr_partial_roi: roi is NULL");
    if (!ctx->has_camera) return fail(ctx, VR_ERR_STATE, "vr_partial_roi: no camera set");
    const CameraK& cam = ctx->cam;
    const int W = cam.width, H = cam.height;
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = b->origin[c];
        hi[c] = b->origin[c] + (double)b->dims[c] * b->spacing[c];
    }
    double imin = INFINITY, imax = -INFINITY, jmin = INFINITY, jmax = -INFINITY;
    bool full = false;
    for (int k = 0; k < 8 && !full; ++k) {
        double p[3] = {(k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]};
        double v[3];
        sub3(p, cam.eye, v);
        double x, y;
        if (cam.kind == 0) {
            double z = dot3(v, cam.f);
            // corner at or behind the eye plane: the projection is unbounded
            if (!(z > 1e-9 * (1.0 + norm3(v)))) { full = true; break; }
            x = dot3(v, cam.r) / z;
            y = dot3(v, cam.u) / z;
        } else {
            x = dot3(v, cam.r);
            y = dot3(v, cam.u);
        }
        // invert x = (2 (i + 1/2) / W - 1) ax, y = (1 - 2 (j + 1/2) / H) ay
        double i = (x / cam.ax + 1.0) * 0.5 * W - 0.5;
        double j = (1.0 - y / cam.ay) * 0.5 * H - 0.5;
        imin = std::fmin(imin, i); imax = std::fmax(imax, i);
        jmin = std::fmin(jmin, j); jmax = std::fmax(jmax, j);
    }
    if (full) {
        roi[0] = 0; roi[1] = 0; roi[2] = W; roi[3] = H;
        return ok(ctx);
    }
    double x0 = std::floor(imin) - 1, x1 = std::ceil(imax) + 1;
    double y0 = std::floor(jmin) - 1, y1 = std::ceil(jmax) + 1;
    x0 = std::fmax(x0, 0.0); y0 = std::fmax(y0, 0.0);
    x1 = std::fmin(x1, (double)W - 1); y1 = std::fmin(y1, (double)H - 1);
    if (x1 < x0 || y1 < y0) {
        roi[0] = 0; roi[1] = 0; roi[2] = 0; roi[3] = 0;
        return ok(ctx);
    }
    roi[0] = (int32_t)x0;
    roi[1] = (int32_t)y0;
    roi[2] = (int32_t)(x1 - x0) + 1;
    roi[3] = (int32_t)(y1 - y0) + 1;
    return ok(ctx);
}

static vr_status check_partial(vr_context ctx, const vr_partial* part, const char* who, bool need_buffers) {
    const int W = ctx->cam.width, H = ctx->cam.height;
    if (part->w < 0 || part->h < 0 || part->x0 < 0 || part->y0 < 0 ||
        (int64_t)part->x0 + part->w > W || (int64_t)part->y0 + part->h > H)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: ROI (%d, %d, %d, %d) outside the %dx%d frame", who,
                    part->x0, part->y0, part->w, part->h, W, H);
    if (need_buffers && part->w > 0 && part->h > 0) {
        if (!part->rgba || !part->depth) return fail(ctx, VR_ERR_INVALID_ARG, "%s: NULL image buffer", who);
        if ((reinterpret_cast<uintptr_t>(part->rgba) & 15) != 0 ||
            (reinterpret_cast<uintptr_t>(part->depth) & 3) != 0 ||
            (reinterpret_cast<uintptr_t>(part->samples) & 7) != 0)
            return fail(ctx, VR_ERR_INVALID_ARG,
                        "%s: rgba must be 16-, depth 4- and samples 8-byte aligned", who);
    }
    return VR_OK;
}

static vr_status prepare_march(vr_context ctx, vr_brick b, const vr_partial* part, const char* who,
                               MarchParams& p) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (!live(b) || b->ctx != ctx) return fail(ctx, VR_ERR_INVALID_HANDLE, "%s: invalid brick", who);
    if (!part) return fail(ctx, VR_ERR_INVALID_ARG, "%s: part is NULL", who);
    if (!ctx->has_camera) return fail(ctx, VR_ERR_STATE, "%s: no camera set", who);
    if (!ctx->has_tf) return fail(ctx, VR_ERR_STATE, "%s: no transfer function set", who);
    if (!b->has_data) return fail(ctx, VR_ERR_STATE, "%s: brick has no voxel data", who);
    vr_status st = check_partial(ctx, part, who, true);
    if (st != VR_OK) return st;
    p = MarchParams{};
    p.cam = ctx->cam;
    p.brick.data = b->ws;
    for (int c = 0; c < 3; ++c) {
        p.brick.sdim[c] = b->dims[c] + 2 * b->ghost;
        p.brick.lo[c] = b->origin[c];
        p.brick.hi[c] = b->origin[c] + (double)b->dims[c] * b->spacing[c];
        p.brick.origin[c] = b->origin[c];
        p.brick.spacing[c] = b->spacing[c];
    }
    p.brick.ghost = b->ghost;
    p.tf = ctx->tf;
    p.dt = ctx->dt;
    p.ert_eps = ctx->ert_eps;
    p.roi_x0 = part->x0;
    p.roi_y0 = part->y0;
    p.roi_w = part->w;
    p.roi_h = part->h;
    p.tiles_x = (part->w + 7) / 8;
    p.tiles_y = (part->h + 7) / 8;
    p.out_rgba = part->rgba;
    p.out_depth = part->depth;
    p.samples = part->samples;
    return VR_OK;
}

vr_status vr_render_partial(vr_context ctx, vr_brick b, const vr_partial* part) {
    MarchParams p;
    vr_status st = prepare_march(ctx, b, part, "vr_render_partial", p);
    if (st != VR_OK) return st;
    if (part->w == 0 || part->h == 0) return ok(ctx);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_render_partial: cannot select device %d", ctx->device);
    hipError_t e = launch_march(p, b->storage == VR_F16 ? kF16 : kF32, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_render_partial: %s", hipGetErrorString(e));
    return ok(ctx);
}

static vr_status prepare_composite(vr_context ctx, const vr_partial* parts, int32_t n,
                                   const float bg[4], const char* who, CompositeParams& p) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (n < 0 || n > DPVR_MAX_PARTIALS)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: n = %d outside [0, %d]", who, n, DPVR_MAX_PARTIALS);
    if ((n > 0 && !parts) || !bg) return fail(ctx, VR_ERR_INVALID_ARG, "%s: NULL argument", who);
    if (!ctx->has_camera) return fail(ctx, VR_ERR_STATE, "%s: no camera set", who);
    for (int c = 0; c < 4; ++c)
        if (!std::isfinite(bg[c])) return fail(ctx, VR_ERR_INVALID_ARG, "%s: background not finite", who);
    p = CompositeParams{};
    for (int i = 0; i < n; ++i) {
        vr_status st = check_partial(ctx, &parts[i], who, true);
        if (st != VR_OK) return st;
        p.parts[i].x0 = parts[i].x0;
        p.parts[i].y0 = parts[i].y0;
        p.parts[i].w = parts[i].w;
        p.parts[i].h = parts[i].h;
        p.parts[i].rgba = parts[i].rgba;
        p.parts[i].depth = parts[i].depth;
    }
    p.n = n;
    p.width = ctx->cam.width;
    p.height = ctx->cam.height;
    p.tiles_x = (p.width + 7) / 8;
    for (int c = 0; c < 4; ++c) p.bg[c] = bg[c];
    return VR_OK;
}

vr_status vr_composite(vr_context ctx, const vr_partial* parts, int32_t n, const float bg[4],
                       float* out) {
    CompositeParams p;
    vr_status st = prepare_composite(ctx, parts, n, bg, "vr_composite", p);
    if (st != VR_OK) return st;
    if (!out) return fail(ctx, VR_ERR_INVALID_ARG, "vr_composite: out is NULL");
    if ((reinterpret_cast<uintptr_t>(out) & 15) != 0)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_composite: out must be 16-byte aligned");
    p.out = out;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_composite: cannot select device %d", ctx->device);
    hipError_t e = launch_composite(p, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_composite: %s", hipGetErrorString(e));
    return ok(ctx);
}

vr_status vr_brick_set_data_global(vr_brick b, const float* volume, const int32_t vol_dims[3],
                                   const int32_t lo[3]) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_brick_set_data_global: invalid brick");
    vr_context ctx = b->ctx;
    if (!volume || !vol_dims || !lo) return fail(ctx, VR_ERR_INVALID_ARG, "vr_brick_set_data_global: NULL argument");
    for (int c = 0; c < 3; ++c)
        if (vol_dims[c] < 1 || lo[c] < 0 || (int64_t)lo[c] + b->dims[c] > vol_dims[c])
            return fail(ctx, VR_ERR_INVALID_ARG,
                        "vr_brick_set_data_global: owned box [%d, %d) on axis %d outside the %d-voxel grid",
                        lo[c], lo[c] + b->dims[c], c, vol_dims[c]);
    GatherParams gp{};
    gp.volume = volume;
    for (int c = 0; c < 3; ++c) {
        gp.vol_dims[c] = vol_dims[c];
        gp.lo[c] = lo[c];
        gp.sdim[c] = b->dims[c] + 2 * b->ghost;
    }
    gp.ghost = b->ghost;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_brick_set_data_global: cannot select device %d", ctx->device);
    hipError_t e = launch_gather(gp, b->ws, b->storage == VR_F16 ? kF16 : kF32, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_brick_set_data_global: %s", hipGetErrorString(e));
    b->has_data = true;
    return ok(ctx);
}

// Upper bound of the owned samples of any ray in the brick: a chord is at
// most the box diagonal long and holds at most floor(len / dt) + 1 lattice
// points; two more absorb rounding of the diagonal.
static int64_t ckpt_segments(vr_brick b, double dt, int32_t interval) {
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double e = (double)b->dims[c] * b->spacing[c];
        d2 += e * e;
    }
    int64_t max_samples = (int64_t)std::floor(std::sqrt(d2) / dt) + 3;
    return (max_samples + interval - 1) / interval;
}

vr_status vr_checkpoint_size(vr_context ctx, vr_brick b, const vr_partial* part, int32_t interval,
                             size_t* bytes) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_checkpoint_size: invalid context");
    if (!live(b) || b->ctx != ctx) return fail(ctx, VR_ERR_INVALID_HANDLE, "vr_checkpoint_size: invalid brick");
    if (!part || !bytes) return fail(ctx, VR_ERR_INVALID_ARG, "vr_checkpoint_size: NULL argument");
    if (interval < 1 || interval > DPVR_MAX_CKPT_INTERVAL)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_checkpoint_size: interval %d outside [1, %d]", interval,
                    DPVR_MAX_CKPT_INTERVAL);
    if (part->w < 0 || part->h < 0) return fail(ctx, VR_ERR_INVALID_ARG, "vr_checkpoint_size: negative ROI");
    *bytes = (size_t)part->w * part->h * (size_t)ckpt_segments(b, ctx->dt, interval) * sizeof(float);
    return ok(ctx);
}

vr_status vr_render_partial_checkpointed(vr_context ctx, vr_brick b, const vr_partial* part,
                                         int32_t interval, float* ckpt, size_t ckpt_bytes) {
    MarchParams p;
    vr_status st = prepare_march(ctx, b, part, "vr_render_partial_checkpointed", p);
    if (st != VR_OK) return st;
    size_t need = 0;
    st = vr_checkpoint_size(ctx, b, part, interval, &need);
    if (st != VR_OK) return st;
    if (!ckpt || ckpt_bytes < need || (reinterpret_cast<uintptr_t>(ckpt) & 3) != 0)
        return fail(ctx, VR_ERR_WORKSPACE, "vr_render_partial_checkpointed: checkpoint buffer of %zu bytes, need %zu",
                    ckpt_bytes, need);
    if (part->w == 0 || part->h == 0) return ok(ctx);
    p.ert_eps = 0.0f;
    p.ckpt = ckpt;
    p.ckpt_interval = interval;
    p.ckpt_nseg = (int32_t)ckpt_segments(b, ctx->dt, interval);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_render_partial_checkpointed: cannot select device %d", ctx->device);
    hipError_t e = launch_march(p, b->storage == VR_F16 ? kF16 : kF32, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_render_partial_checkpointed: %s", hipGetErrorString(e));
    return ok(ctx);
}

vr_status vr_composite_backward(vr_context ctx, const vr_partial* parts, int32_t n,
                                const float bg[4], const float* d_out, float* const* d_parts) {
    CompositeParams p;
    vr_status st = prepare_composite(ctx, parts, n, bg, "vr_composite_backward", p);
    if (st != VR_OK) return st;
    if (!d_out || (n > 0 && !d_parts)) return fail(ctx, VR_ERR_INVALID_ARG, "vr_composite_backward: NULL argument");
    if ((reinterpret_cast<uintptr_t>(d_out) & 15) != 0)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_composite_backward: d_out must be 16-byte aligned");
    CompositeBackParams bp{};
    bp.d_out = d_out;
    for (int i = 0; i < n; ++i) {
        if (parts[i].w > 0 && parts[i].h > 0 &&
            (!d_parts[i] || (reinterpret_cast<uintptr_t>(d_parts[i]) & 15) != 0))
            return fail(ctx, VR_ERR_INVALID_ARG, "vr_composite_backward: d_parts[%d] NULL or not 16-byte aligned", i);
        bp.d_parts[i] = d_parts[i];
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_composite_backward: cannot select device %d", ctx->device);
    hipError_t e = launch_composite_backward(p, bp, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_composite_backward: %s", hipGetErrorString(e));
    return ok(ctx);
}

vr_status vr_render_partial_backward(vr_context ctx, vr_brick b, const vr_partial* part,
                                     int32_t interval, const float* ckpt, size_t ckpt_bytes,
                                     const float* d_part, float* grad_tf, float* grad_volume,
                                     const int32_t vol_dims[3], const int32_t lo[3]) {
    MarchParams p;
    vr_status st = prepare_march(ctx, b, part, "vr_render_partial_backward", p);
    if (st != VR_OK) return st;
    size_t need = 0;
    st = vr_checkpoint_size(ctx, b, part, interval, &need);
    if (st != VR_OK) return st;
    if (!ckpt || ckpt_bytes < need)
        return fail(ctx, VR_ERR_WORKSPACE, "vr_render_partial_backward: checkpoint buffer of %zu bytes, need %zu",
                    ckpt_bytes, need);
    if (!d_part || !grad_tf || !grad_volume || !vol_dims || !lo)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_render_partial_backward: NULL argument");
    if ((reinterpret_cast<uintptr_t>(d_part) & 15) != 0 || (reinterpret_cast<uintptr_t>(grad_tf) & 3) != 0 ||
        (reinterpret_cast<uintptr_t>(grad_volume) & 3) != 0)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_render_partial_backward: misaligned buffer");
    BackwardParams bp{};
    for (int c = 0; c < 3; ++c) {
        if (vol_dims[c] < 1 || lo[c] < 0 || (int64_t)lo[c] + b->dims[c] > vol_dims[c])
            return fail(ctx, VR_ERR_INVALID_ARG,
                        "vr_render_partial_backward: owned box [%d, %d) on axis %d outside the %d-voxel grid",
                        lo[c], lo[c] + b->dims[c], c, vol_dims[c]);
        bp.vol_dims[c] = vol_dims[c];
        bp.lo[c] = lo[c];
    }
    bp.d_part = d_part;
    bp.grad_tf = grad_tf;
    bp.grad_vox = grad_volume;
    if (part->w == 0 || part->h == 0) return ok(ctx);
    p.ert_eps = 0.0f;
    p.ckpt = const_cast<float*>(ckpt);
    p.ckpt_interval = interval;
    p.ckpt_nseg = (int32_t)ckpt_segments(b, ctx->dt, interval);
    p.samples = nullptr;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_render_partial_backward: cannot select device %d", ctx->device);
    hipError_t e = launch_march_backward(p, bp, b->storage == VR_F16 ? kF16 : kF32, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_render_partial_backward: %s", hipGetErrorString(e));
    return ok(ctx);
}

}  // extern "C"
