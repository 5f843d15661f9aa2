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
#include <algorithm>
#include <cstdlib>
#include <memory>
#include <vector>

#include "../../include/dpvr.h"
#include "dpvr_kernels.h"
#include "tet_kernels.h"
#include "tet_build.h"

using namespace dpvr;

static_assert(DPVR_MAX_TET_PARTS == kMaxTetParts && DPVR_MAX_TET_RUNS == kMaxTetRuns,
              "tetrahedral-part limits of the header and the kernels differ");

// Staged-march launch shape (see vr_set_march_config).
struct MarchCfg {
    int32_t staging, tile_w, chunk;
};

struct vr_context_s {
    int32_t device = 0;
    int32_t cus = 0;               // compute units of the device
    // persistent march workgroups per CU [F32/F16][direct, slab, ring tile 16/32 x chunk 4/8];
    // 0 = not yet queried
    int32_t queue_wg[2][6] = {{0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}};
    // staged march configuration per storage precision [F32, F16]: the
    // fastest measured on the 1920x1080 frame of 16 bricks -- float32: ring,
    // 32-pixel tiles, 4-slice chunks; float16: slab
    MarchCfg cfg[2] = {{kStagingRing, 32, 4}, {kStagingSlab, 16, 4}};
    hipStream_t stream = nullptr;
    bool has_camera = false, has_tf = false;
    CameraK cam{};
    TFK tf{};
    double dt = 0.5;
    float ert_eps = 0x1p-20f;
    int32_t path = kPathStaged;
    int32_t live_bricks = 0;
    int32_t live_tetparts = 0;
    int32_t tet_locator = kTetGrid;   // structure searched after the walk (vr_set_tet_locator)
    std::string err;
    // vr_render_partials_static: this device's library-owned scratch array
    // (address from hipGetSymbolAddress at context creation) and two pinned
    // host staging slots for its job table, each guarded by an event that
    // completes when the copy out of it has run
    void* scratch = nullptr;
    void* pinned[2] = {nullptr, nullptr};
    size_t pinned_bytes[2] = {0, 0};
    hipEvent_t pinned_done[2] = {nullptr, nullptr};
    int32_t pinned_next = 0;
    // host copies of the current frame's job table and tile prefix (capacity
    // for kStaticMaxPartials reserved at creation, so that a frame of at most
    // that many partials allocates nothing)
    std::vector<MarchParams> fjobs;
    std::vector<int32_t> fprefix;
    // the last vr_rqc_plan: its workspace, bricks, camera and spacing, plan
    // entries and owned primary samples (vr_render_rqc must match it)
    struct {
        const void* ws = nullptr;
        std::vector<const void*> bricks;
        CameraK cam{};
        double dt = 0.0;
        long long entries = 0, total = -1;
    } rqc;
    // the last vr_tetparts_shadow_plan: its plan buffer, parts, camera,
    // spacing, entries and slots (vr_render_tetparts_shadowed must match it)
    struct {
        const void* plan = nullptr;
        std::vector<const void*> parts;
        CameraK cam{};
        double dt = 0.0;
        long long entries = 0, total = -1;
    } tetplan;
    // the last vr_march_tetparts / vr_render_tetparts: workspace, parts,
    // max_runs and camera (vr_resolve_tetparts must match them)
    struct {
        const void* ws = nullptr;
        std::vector<const void*> parts;
        int32_t max_runs = 0;
        CameraK cam{};
    } tetmarch;
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
    const void* owner = nullptr;   // the time series whose slot holds this brick (NULL: the caller's)
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

// Stored elements of a brick: rows of (nx + 2g) voxels padded to a pitch of a
// multiple of 8 elements, (ny + 2g) * (nz + 2g) rows.
int64_t stored_count(const int32_t dims[3], int32_t ghost) {
    const int64_t pitch = ((int64_t)dims[0] + 2 * ghost + 7) & ~(int64_t)7;
    return pitch * (dims[1] + 2 * ghost) * (dims[2] + 2 * ghost);
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

// Pinned staging of vr_render_partials_static (waits for copies still
// reading it).
void release_static_staging(vr_context c) {
    for (int i = 0; i < 2; ++i) {
        if (c->pinned_done[i]) {
            (void)hipEventSynchronize(c->pinned_done[i]);
            (void)hipEventDestroy(c->pinned_done[i]);
            c->pinned_done[i] = nullptr;
        }
        if (c->pinned[i]) {
            (void)hipHostFree(c->pinned[i]);
            c->pinned[i] = nullptr;
        }
    }
}

// Device error word of a context's device: kernels OR error bits into it
// (the word lives in the library's static scratch array of that device).
int32_t* err_word(vr_context c) {
    return reinterpret_cast<int32_t*>(reinterpret_cast<char*>(c->scratch) + kErrWordOffset);
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
        case VR_ERR_OUT_OF_MEMORY: return "VR_ERR_OUT_OF_MEMORY";
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
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        return fail(nullptr, VR_ERR_DEVICE, "vr_context_create: cannot query device %d", device);
    vr_context c = new (std::nothrow) vr_context_s;
    if (!c) return fail(nullptr, VR_ERR_OUT_OF_MEMORY, "vr_context_create: out of host memory");
    c->device = device;
    c->cus = cus;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    {
        // set-up of vr_render_partials_static, with the context's device current
        DeviceGuard g(device);
        hipError_t e = g.ok ? hipSuccess : hipErrorInvalidDevice;
        if (e == hipSuccess) e = static_scratch_address(&c->scratch);
        for (int i = 0; i < 2 && e == hipSuccess; ++i) {
            e = hipHostMalloc(&c->pinned[i], kStaticScratchBytes, hipHostMallocDefault);
            if (e == hipSuccess) c->pinned_bytes[i] = kStaticScratchBytes;
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->pinned_done[i], hipEventDisableTiming);
        }
        if (e == hipSuccess) {
            try {
                c->fjobs.reserve(kStaticMaxPartials);
                c->fprefix.reserve(kStaticMaxPartials + 2);
            } catch (const std::bad_alloc&) {
                e = hipErrorOutOfMemory;
            }
        }
        if (e == hipSuccess && !c->scratch) e = hipErrorInvalidSymbol;
        if (e != hipSuccess) {
            release_static_staging(c);
            delete c;
            return fail(nullptr, VR_ERR_DEVICE, "vr_context_create: static scratch set-up on device %d: %s",
                        device, hipGetErrorString(e));
        }
    }
    try {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(c);
    } catch (const std::bad_alloc&) {
        release_static_staging(c);
        delete c;
        return fail(nullptr, VR_ERR_OUT_OF_MEMORY, "vr_context_create: out of host memory");
    }
    *out = c;
    return VR_OK;
}

vr_status vr_context_release(vr_context ctx) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_context_release: invalid context");
    if (ctx->live_bricks > 0)
        return fail(ctx, VR_ERR_STATE, "vr_context_release: %d bricks still alive", ctx->live_bricks);
    if (ctx->live_tetparts > 0)
        return fail(ctx, VR_ERR_STATE, "vr_context_release: %d tetrahedral parts still alive", ctx->live_tetparts);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.erase(ctx);
    }
    {
        DeviceGuard g(ctx->device);
        release_static_staging(ctx);
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
    // kernel guards (bounded waits) report through the device error word
    int32_t word = 0;
    e = hipMemcpy(&word, err_word(ctx), sizeof word, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_synchronize: %s", hipGetErrorString(e));
    if (word != 0) {
        const int32_t zero = 0;
        (void)hipMemcpy(err_word(ctx), &zero, sizeof zero, hipMemcpyHostToDevice);
        const char* what = (word & kErrSpin)   ? "a march kernel gave up a bounded wait"
                           : (word & kErrRuns) ? "a ray crossed a tetrahedral part in more runs than max_runs"
                                               : "a sample index exceeded 2^31 - 1, or a shadow plan's counts "
                                                 "did not match its frame";
        return fail(ctx, VR_ERR_DEVICE,
                    "vr_synchronize: %s (device error bits 0x%x); images rendered since the last "
                    "synchronisation are unreliable", what, (unsigned)word);
    }
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
    if (n >= ((int64_t)1 << 31))   // the kernels index a brick with 32-bit element offsets
        return fail(nullptr, VR_ERR_UNSUPPORTED, "vr_brick_workspace_size: %lld stored voxels (limit 2^31 - 1)",
                    (long long)n);
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
    if (!b) return fail(ctx, VR_ERR_OUT_OF_MEMORY, "vr_brick_create: out of host memory");
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
    try {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(b);
    } catch (const std::bad_alloc&) {
        delete b;
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "vr_brick_create: out of host memory");
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
    int32_t sdim[3];
    for (int c = 0; c < 3; ++c) sdim[c] = b->dims[c] + 2 * b->ghost;
    hipError_t e = launch_ingest(voxels, b->ws, sdim, b->storage == VR_F16 ? kF16 : kF32, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_brick_set_data: %s", hipGetErrorString(e));
    b->has_data = true;
    return ok(ctx);
}

vr_status vr_brick_release(vr_brick b) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_brick_release: invalid brick");
    if (b->owner) return fail(b->ctx, VR_ERR_STATE, "vr_brick_release: the brick belongs to a time series");
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

// Camera frame from its description (kind 0: eye, look-at point, fovy in
// degrees; kind 1: image centre, view direction, view height), validated.
static vr_status build_camera(vr_context ctx, int kind, const double eye[3], const double tgt[3],
                              const double up[3], double fov_or_h, int32_t width, int32_t height,
                              const char* who, CameraK& cam) {
    if (!eye || !tgt || !up) return fail(ctx, VR_ERR_INVALID_ARG, "%s: NULL argument", who);
    if (kind != 0 && kind != 1) return fail(ctx, VR_ERR_INVALID_ARG, "%s: unknown camera kind %d", who, kind);
    if (!finite3(eye) || !finite3(tgt) || !finite3(up))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: non-finite vector", who);
    if (kind == 0 && !(fov_or_h > 0 && fov_or_h < 180))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: fovy must be in (0, 180)", who);
    if (kind == 1 && (!(fov_or_h > 0) || !std::isfinite(fov_or_h)))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: view_height must be > 0", who);
    if (width < 1 || height < 1 || width > 32768 || height > 32768)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: bad image size %dx%d", who, width, height);
    cam = CameraK{};
    double fwd[3];
    if (kind == 0)
        sub3(tgt, eye, fwd);
    else
        for (int c = 0; c < 3; ++c) fwd[c] = tgt[c];
    vr_status st = make_frame(ctx, fwd, up, cam);
    if (st != VR_OK) return st;
    const double W = (double)width, H = (double)height;
    if (kind == 0) {
        const double th = std::tan(0.5 * fov_or_h * (M_PI / 180.0));
        cam.ax = (th * W) / H;
        cam.ay = th;
    } else {
        const double hh = 0.5 * fov_or_h;
        cam.ax = (hh * W) / H;
        cam.ay = hh;
    }
    for (int c = 0; c < 3; ++c) cam.eye[c] = eye[c];
    cam.kind = kind;
    cam.width = width;
    cam.height = height;
    return VR_OK;
}

vr_status vr_set_camera_perspective(vr_context ctx, const double eye[3], const double target[3],
                                    const double up[3], double fovy_deg, int32_t width,
                                    int32_t height) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_set_camera_perspective: invalid context");
    CameraK cam;
    vr_status st = build_camera(ctx, 0, eye, target, up, fovy_deg, width, height,
                                "vr_set_camera_perspective", cam);
    if (st != VR_OK) return st;
    ctx->cam = cam;
    ctx->has_camera = true;
    return ok(ctx);
}

vr_status vr_set_camera_orthographic(vr_context ctx, const double pos[3], const double dir[3],
                                     const double up[3], double view_height, int32_t width,
                                     int32_t height) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_set_camera_orthographic: invalid context");
    CameraK cam;
    vr_status st = build_camera(ctx, 1, pos, dir, up, view_height, width, height,
                                "vr_set_camera_orthographic", cam);
    if (st != VR_OK) return st;
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

vr_status vr_set_march_path(vr_context ctx, vr_path path) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_set_march_path: invalid context");
    if (path != VR_PATH_STAGED && path != VR_PATH_DIRECT)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_march_path: unknown path %d", (int)path);
    ctx->path = path == VR_PATH_DIRECT ? kPathDirect : kPathStaged;
    return ok(ctx);
}

vr_status vr_set_march_config(vr_context ctx, vr_dtype storage, vr_staging staging, int32_t tile_width,
                              int32_t chunk_slices) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_set_march_config: invalid context");
    if (storage != VR_F32 && storage != VR_F16)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_march_config: unknown storage %d", (int)storage);
    const int st = staging == VR_STAGING_SLAB ? kStagingSlab : kStagingRing;
    if ((staging != VR_STAGING_SLAB && staging != VR_STAGING_RING) ||
        !valid_march_config(st, tile_width, st == kStagingSlab ? 4 : chunk_slices))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_march_config: slab staging takes 16-pixel tiles, ring staging "
                    "16 or 32 with chunks of 4 or 8 slices (got %d, %d, %d)", (int)staging, tile_width, chunk_slices);
    ctx->cfg[storage == VR_F16 ? 1 : 0] = MarchCfg{st, tile_width, st == kStagingSlab ? 4 : chunk_slices};
    return ok(ctx);
}

// Pixel rectangle of the frame of `cam` whose rays can meet the box [lo, hi]
// (a brick's owned box, a part's bounding box): the box corners projected to
// the image plus one pixel of margin, the whole frame when a corner lies at
// or behind the eye plane.
static void roi_for_box(const CameraK& cam, const double lo[3], const double hi[3], int32_t roi[4]) {
    const int W = cam.width, H = cam.height;
    double imin = INFINITY, imax = -INFINITY, jmin = INFINITY, jmax = -INFINITY;
    for (int k = 0; k < 8; ++k) {
        double p[3] = {(k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]};
        double v[3];
        sub3(p, cam.eye, v);
        double x, y;
        if (cam.kind == 0) {
            double z = dot3(v, cam.f);
            if (!(z > 1e-9 * (1.0 + norm3(v)))) {   // unbounded projection
                roi[0] = 0; roi[1] = 0; roi[2] = W; roi[3] = H;
                return;
            }
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
    double x0 = std::floor(imin) - 1, x1 = std::ceil(imax) + 1;
    double y0 = std::floor(jmin) - 1, y1 = std::ceil(jmax) + 1;
    x0 = std::fmax(x0, 0.0); y0 = std::fmax(y0, 0.0);
    x1 = std::fmin(x1, (double)W - 1); y1 = std::fmin(y1, (double)H - 1);
    if (x1 < x0 || y1 < y0) {
        roi[0] = 0; roi[1] = 0; roi[2] = 0; roi[3] = 0;
        return;
    }
    roi[0] = (int32_t)x0;
    roi[1] = (int32_t)y0;
    roi[2] = (int32_t)(x1 - x0) + 1;
    roi[3] = (int32_t)(y1 - y0) + 1;
}

static void roi_for(const CameraK& cam, vr_brick b, int32_t roi[4]) {
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = b->origin[c];
        hi[c] = b->origin[c] + (double)b->dims[c] * b->spacing[c];
    }
    roi_for_box(cam, lo, hi, roi);
}

vr_status vr_partial_roi(vr_context ctx, vr_brick b, int32_t roi[4]) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_partial_roi: invalid context");
    if (!live(b) || b->ctx != ctx) return fail(ctx, VR_ERR_INVALID_HANDLE, "vr_partial_roi: invalid brick");
    if (!roi) return fail(ctx, VR_ERR_INVALID_ARG, "vr_partial_roi: roi is NULL");
    if (!ctx->has_camera) return fail(ctx, VR_ERR_STATE, "vr_partial_roi: no camera set");
    roi_for(ctx->cam, b, roi);
    return ok(ctx);
}

static vr_status camera_from_desc(vr_context ctx, const vr_camera_desc* d, const char* who, CameraK& cam) {
    if (!d) return fail(ctx, VR_ERR_INVALID_ARG, "%s: NULL camera", who);
    return build_camera(ctx, d->kind, d->eye, d->target, d->up, d->fovy_deg, d->width, d->height, who, cam);
}

vr_status vr_camera_roi(vr_context ctx, vr_brick b, const vr_camera_desc* cam, int32_t roi[4]) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_camera_roi: invalid context");
    if (!live(b) || b->ctx != ctx) return fail(ctx, VR_ERR_INVALID_HANDLE, "vr_camera_roi: invalid brick");
    if (!roi) return fail(ctx, VR_ERR_INVALID_ARG, "vr_camera_roi: roi is NULL");
    CameraK c;
    vr_status st = camera_from_desc(ctx, cam, "vr_camera_roi", c);
    if (st != VR_OK) return st;
    roi_for(c, b, roi);
    return ok(ctx);
}

static vr_status check_partial(vr_context ctx, const CameraK& cam, const vr_partial* part, const char* who,
                               bool need_buffers) {
    const int W = cam.width, H = cam.height;
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

// Kernel parameters of one partial for camera `cam` and transfer function `tf`.
static vr_status prepare_march_with(vr_context ctx, vr_brick b, const vr_partial* part, const CameraK& cam,
                                    const TFK& tf, const char* who, MarchParams& p) {
    if (!live(b) || b->ctx != ctx) return fail(ctx, VR_ERR_INVALID_HANDLE, "%s: invalid brick", who);
    if (!part) return fail(ctx, VR_ERR_INVALID_ARG, "%s: part is NULL", who);
    if (!b->has_data) return fail(ctx, VR_ERR_STATE, "%s: brick has no voxel data", who);
    vr_status st = check_partial(ctx, cam, part, who, true);
    if (st != VR_OK) return st;
    p = MarchParams{};
    p.cam = cam;
    p.brick.data = b->ws;
    for (int c = 0; c < 3; ++c) {
        p.brick.sdim[c] = b->dims[c] + 2 * b->ghost;
        p.brick.lo[c] = b->origin[c];
        p.brick.hi[c] = b->origin[c] + (double)b->dims[c] * b->spacing[c];
        p.brick.origin[c] = b->origin[c];
        p.brick.spacing[c] = b->spacing[c];
        p.brick.inv_spacing[c] = 1.0 / b->spacing[c];
    }
    p.brick.ghost = b->ghost;
    p.tf = tf;
    p.dt = ctx->dt;
    p.inv_dt = 1.0 / ctx->dt;
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
    p.path = ctx->path;
    const MarchCfg& mc = ctx->cfg[b->storage == VR_F16 ? 1 : 0];
    p.staging = mc.staging;
    p.tile_w = mc.tile_w;
    p.chunk = mc.chunk;
    p.err = err_word(ctx);
    return VR_OK;
}

// ... with the context's camera and transfer function.
static vr_status prepare_march(vr_context ctx, vr_brick b, const vr_partial* part, const char* who,
                               MarchParams& p) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (!ctx->has_camera) return fail(ctx, VR_ERR_STATE, "%s: no camera set", who);
    if (!ctx->has_tf) return fail(ctx, VR_ERR_STATE, "%s: no transfer function set", who);
    return prepare_march_with(ctx, b, part, ctx->cam, ctx->tf, who, p);
}

// Layout of a frame workspace: [2 x kQueueParts queue counters | 256 B] [tile_start[n + 2] | 256-aligned]
// [MarchParams jobs[n] | 256-aligned].
static size_t frame_ws_bytes(int32_t n, size_t* off_tiles, size_t* off_jobs) {
    const size_t a = 256;
    size_t t = a;
    size_t j = t + (((size_t)(n + 2) * sizeof(int32_t) + a - 1) / a) * a;
    size_t end = j + (((size_t)n * sizeof(MarchParams) + a - 1) / a) * a;
    if (off_tiles) *off_tiles = t;
    if (off_jobs) *off_jobs = j;
    return end;
}

vr_status vr_frame_workspace_size(int32_t n, size_t* bytes) {
    if (n < 0 || !bytes) return fail(nullptr, VR_ERR_INVALID_ARG, "vr_frame_workspace_size: bad argument");
    *bytes = frame_ws_bytes(n, nullptr, nullptr);
    return VR_OK;
}

static int queue_workgroups(vr_context ctx, StorageK st, bool staged, int staging, int tile_w, int chunk) {
    const int cfg = !staged ? 0 : staging == kStagingSlab ? 1 : 2 + (tile_w == 32 ? 2 : 0) + (chunk == 8 ? 1 : 0);
    int& n = ctx->queue_wg[st == kF16 ? 1 : 0][cfg];
    if (n == 0) n = march_queue_workgroups_per_cu(st, staged, staging, tile_w, chunk) * ctx->cus;
    return n;
}

// Tile width of the frame queue of storage group g (0 float32, 1 float16)
// with the context's current path.
static int frame_tile_w(vr_context ctx, int g) {
    return ctx->path == kPathDirect || ctx->cfg[g].staging == kStagingSlab ? 16 : ctx->cfg[g].tile_w;
}

// Job table and tile prefix of a frame of n partials, grouped by storage
// precision (float32 jobs first): each group is one queue with its own
// exclusive tile prefix (prefix[0 .. n32] and prefix[n32 + 1 .. n + 1]).
static vr_status frame_tables(vr_context ctx, int32_t n, const vr_brick* bricks, const vr_partial* parts,
                              const char* who, int* n32_out) {
    std::vector<MarchParams>& jobs = ctx->fjobs;
    std::vector<int32_t>& prefix = ctx->fprefix;
    jobs.clear();
    try {
        jobs.reserve(n);
        prefix.assign(n + 2, 0);
    } catch (const std::bad_alloc&) {
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory for the tables of %d partials", who, n);
    }
    int n32 = 0;
    for (int pass = 0; pass < 2; ++pass) {
        int32_t acc = 0;
        const int base = pass == 0 ? 0 : n32 + 1;   // prefix offset of this group
        int cnt = 0;
        for (int i = 0; i < n; ++i) {
            if (!live(bricks[i]) || bricks[i]->ctx != ctx)
                return fail(ctx, VR_ERR_INVALID_HANDLE, "%s: invalid brick %d", who, i);
            if ((bricks[i]->storage == VR_F16) != (pass == 1)) continue;
            MarchParams p;
            vr_status st = prepare_march(ctx, bricks[i], &parts[i], who, p);
            if (st != VR_OK) return st;
            prefix[base + cnt] = acc;
            acc += queue_tiles(parts[i].w, parts[i].h, frame_tile_w(ctx, pass));
            jobs.push_back(p);
            ++cnt;
        }
        prefix[base + cnt] = acc;
        if (pass == 0) n32 = cnt;
    }
    *n32_out = n32;
    return VR_OK;
}

// Stream-ordered copy of the frame tables (ctx->fprefix at off_t, ctx->fjobs
// at off_j; `need` bytes of frame workspace layout) to device memory at ws,
// through the next of the context's two pinned host slots (once the copy
// that last read that slot has run).  A slot smaller than `need` is
// reallocated, which never happens for kStaticMaxPartials or fewer partials.
static hipError_t stage_frame_tables(vr_context ctx, char* ws, size_t off_t, size_t off_j, size_t need) {
    const int slot = ctx->pinned_next;
    ctx->pinned_next ^= 1;
    hipError_t e = hipEventSynchronize(ctx->pinned_done[slot]);
    if (e != hipSuccess) return e;
    if (ctx->pinned_bytes[slot] < need) {
        (void)hipHostFree(ctx->pinned[slot]);
        ctx->pinned[slot] = nullptr;
        ctx->pinned_bytes[slot] = 0;
        e = hipHostMalloc(&ctx->pinned[slot], need, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        ctx->pinned_bytes[slot] = need;
    }
    char* host = reinterpret_cast<char*>(ctx->pinned[slot]);
    std::memcpy(host + off_t, ctx->fprefix.data(), ctx->fprefix.size() * sizeof(int32_t));
    std::memcpy(host + off_j, ctx->fjobs.data(), ctx->fjobs.size() * sizeof(MarchParams));
    e = hipMemcpyAsync(ws + off_t, host + off_t, need - off_t, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->pinned_done[slot], ctx->stream);
    return e;
}

// The frame's queue launches over tables already in (or enqueued into)
// device memory at ws (frame workspace layout).
static hipError_t launch_frame(vr_context ctx, char* ws, size_t off_t, size_t off_j, int32_t n, int n32,
                               const std::vector<int32_t>& prefix) {
    const MarchParams* djobs = reinterpret_cast<const MarchParams*>(ws + off_j);
    const int32_t* dtiles = reinterpret_cast<const int32_t*>(ws + off_t);
    int32_t* heads = reinterpret_cast<int32_t*>(ws);
    const int staged = ctx->path == kPathDirect ? 0 : 1;
    hipError_t e = hipSuccess;
    if (n32 > 0) {
        const int tw = frame_tile_w(ctx, 0), ch = ctx->cfg[0].chunk, sk = ctx->cfg[0].staging;
        QueueParams q{djobs, dtiles, n32, prefix[n32], heads, staged, sk, tw, ch, err_word(ctx)};
        e = launch_march_queue(q, kF32, queue_workgroups(ctx, kF32, staged, sk, tw, ch), ctx->stream);
    }
    if (e == hipSuccess && n - n32 > 0) {
        const int tw = frame_tile_w(ctx, 1), ch = ctx->cfg[1].chunk, sk = ctx->cfg[1].staging;
        QueueParams q{djobs + n32, dtiles + n32 + 1, n - n32, prefix[n + 1], heads + kQueueParts, staged, sk, tw,
                      ch, err_word(ctx)};
        e = launch_march_queue(q, kF16, queue_workgroups(ctx, kF16, staged, sk, tw, ch), ctx->stream);
    }
    return e;
}

vr_status vr_render_partials(vr_context ctx, int32_t n, const vr_brick* bricks,
                             const vr_partial* parts, void* workspace, size_t workspace_bytes) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_render_partials: invalid context");
    if (n < 0 || (n > 0 && (!bricks || !parts)))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_render_partials: bad n or NULL arrays");
    if (n == 0) return ok(ctx);
    size_t off_t = 0, off_j = 0;
    const size_t need = frame_ws_bytes(n, &off_t, &off_j);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(ctx, VR_ERR_WORKSPACE, "vr_render_partials: workspace of %zu bytes (256-aligned), need %zu",
                    workspace_bytes, need);
    int n32 = 0;
    vr_status st = frame_tables(ctx, n, bricks, parts, "vr_render_partials", &n32);
    if (st != VR_OK) return st;
    char* ws = reinterpret_cast<char*>(workspace);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_render_partials: cannot select device %d", ctx->device);
    hipError_t e = stage_frame_tables(ctx, ws, off_t, off_j, need);
    if (e == hipErrorOutOfMemory)
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "vr_render_partials: pinned staging of %zu bytes", need);
    if (e == hipSuccess) e = launch_frame(ctx, ws, off_t, off_j, n, n32, ctx->fprefix);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_render_partials: %s", hipGetErrorString(e));
    return ok(ctx);
}

vr_status vr_render_partials_static(vr_context ctx, int32_t n, const vr_brick* bricks,
                                    const vr_partial* parts) {
    static const char* who = "vr_render_partials_static";
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (n < 0 || (n > 0 && (!bricks || !parts)))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: bad n or NULL arrays", who);
    if (n > kStaticMaxPartials)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: %d partials exceed the static scratch limit of %d "
                    "(use vr_render_partials with a workspace)", who, n, kStaticMaxPartials);
    if (n == 0) return ok(ctx);
    size_t off_t = 0, off_j = 0;
    const size_t need = frame_ws_bytes(n, &off_t, &off_j);
    if (need > kStaticScratchBytes)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: tables of %zu bytes exceed the %zu-byte scratch", who, need,
                    kStaticScratchBytes);
    int n32 = 0;
    vr_status st = frame_tables(ctx, n, bricks, parts, who, &n32);
    if (st != VR_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
    // the pinned slots hold kStaticScratchBytes from creation: nothing is allocated
    char* scratch = reinterpret_cast<char*>(ctx->scratch);
    hipError_t e = stage_frame_tables(ctx, scratch, off_t, off_j, need);
    if (e == hipSuccess) e = launch_frame(ctx, scratch, off_t, off_j, n, n32, ctx->fprefix);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    return ok(ctx);
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

// Kernel parameters of one frame composite for camera `cam`'s frame.
static vr_status prepare_composite_with(vr_context ctx, const CameraK& cam, const vr_partial* parts,
                                        int32_t n, const float bg[4], const char* who, CompositeParams& p) {
    if (n < 0 || n > DPVR_MAX_PARTIALS)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: n = %d outside [0, %d]", who, n, DPVR_MAX_PARTIALS);
    if ((n > 0 && !parts) || !bg) return fail(ctx, VR_ERR_INVALID_ARG, "%s: NULL argument", who);
    for (int c = 0; c < 4; ++c)
        if (!std::isfinite(bg[c])) return fail(ctx, VR_ERR_INVALID_ARG, "%s: background not finite", who);
    p = CompositeParams{};
    for (int i = 0; i < n; ++i) {
        vr_status st = check_partial(ctx, cam, &parts[i], who, true);
        if (st != VR_OK) return st;
        p.parts[i].x0 = parts[i].x0;
        p.parts[i].y0 = parts[i].y0;
        p.parts[i].w = parts[i].w;
        p.parts[i].h = parts[i].h;
        p.parts[i].rgba = parts[i].rgba;
        p.parts[i].depth = parts[i].depth;
    }
    p.n = n;
    p.width = cam.width;
    p.height = cam.height;
    p.tiles_x = (p.width + 7) / 8;
    for (int c = 0; c < 4; ++c) p.bg[c] = bg[c];
    return VR_OK;
}

static vr_status prepare_composite(vr_context ctx, const vr_partial* parts, int32_t n,
                                   const float bg[4], const char* who, CompositeParams& p) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (!ctx->has_camera) return fail(ctx, VR_ERR_STATE, "%s: no camera set", who);
    return prepare_composite_with(ctx, ctx->cam, parts, n, bg, who, p);
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

// Workspace of vr_render_partials_checkpointed: [MarchParams x n | 256][tile prefix int32 x (n + 2) | 256].
static size_t ckpt_ws_bytes(int32_t n, size_t* off_prefix) {
    const size_t jobs = (((size_t)n * sizeof(MarchParams)) + 255) / 256 * 256;
    if (off_prefix) *off_prefix = jobs;
    return jobs + (((size_t)(n + 2) * sizeof(int32_t)) + 255) / 256 * 256;
}

vr_status vr_checkpointed_workspace_size(int32_t n, size_t* bytes) {
    if (n < 0 || !bytes) return fail(nullptr, VR_ERR_INVALID_ARG, "vr_checkpointed_workspace_size: bad argument");
    *bytes = ckpt_ws_bytes(n, nullptr);
    return VR_OK;
}

vr_status vr_render_partials_checkpointed(vr_context ctx, int32_t n, const vr_brick* bricks, const vr_partial* parts,
                                          int32_t interval, float* const* ckpts, const size_t* ckpt_bytes,
                                          void* workspace, size_t workspace_bytes) {
    static const char* who = "vr_render_partials_checkpointed";
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (n < 0 || (n > 0 && (!bricks || !parts || !ckpts || !ckpt_bytes)))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: bad n or NULL arrays", who);
    if (n == 0) return ok(ctx);
    size_t off_prefix = 0;
    const size_t need = ckpt_ws_bytes(n, &off_prefix);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(ctx, VR_ERR_WORKSPACE, "%s: workspace of %zu bytes (256-aligned), need %zu", who,
                    workspace_bytes, need);
    try {
        std::vector<MarchParams> jobs;
        std::vector<int32_t> prefix(n + 2, 0);
        int n32 = 0;
        for (int pass = 0; pass < 2; ++pass) {
            int32_t acc = 0;
            const int base = pass == 0 ? 0 : n32 + 1;
            int cnt = 0;
            for (int i = 0; i < n; ++i) {
                if (!live(bricks[i]) || bricks[i]->ctx != ctx)
                    return fail(ctx, VR_ERR_INVALID_HANDLE, "%s: invalid brick %d", who, i);
                if ((bricks[i]->storage == VR_F16) != (pass == 1)) continue;
                MarchParams p;
                vr_status st = prepare_march(ctx, bricks[i], &parts[i], who, p);
                if (st != VR_OK) return st;
                size_t nb = 0;
                st = vr_checkpoint_size(ctx, bricks[i], &parts[i], interval, &nb);
                if (st != VR_OK) return st;
                if (!ckpts[i] || ckpt_bytes[i] < nb || (reinterpret_cast<uintptr_t>(ckpts[i]) & 3) != 0)
                    return fail(ctx, VR_ERR_WORKSPACE, "%s: checkpoint buffer %d of %zu bytes, need %zu", who, i,
                                ckpt_bytes[i], nb);
                p.ert_eps = 0.0f;
                p.ckpt = ckpts[i];
                p.ckpt_interval = interval;
                p.ckpt_nseg = (int32_t)ckpt_segments(bricks[i], ctx->dt, interval);
                prefix[base + cnt] = acc;
                acc += p.tiles_x * p.tiles_y;
                jobs.push_back(p);
                ++cnt;
            }
            prefix[base + cnt] = acc;
            if (pass == 0) n32 = cnt;
        }
        char* ws = reinterpret_cast<char*>(workspace);
        DeviceGuard g(ctx->device);
        if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
        hipError_t e = hipMemcpyAsync(ws, jobs.data(), jobs.size() * sizeof(MarchParams), hipMemcpyHostToDevice,
                                      ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws + off_prefix, prefix.data(), prefix.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               ctx->stream);
        const MarchParams* dj = reinterpret_cast<const MarchParams*>(ws);
        const int32_t* dp = reinterpret_cast<const int32_t*>(ws + off_prefix);
        // a group of one partial takes the by-value kernel
        if (e == hipSuccess && n32 == 1)
            e = launch_march(jobs[0], kF32, ctx->stream);
        else if (e == hipSuccess && n32 > 1)
            e = launch_march_checkpointed_many(dj, dp, n32, prefix[n32], kF32, ctx->stream);
        if (e == hipSuccess && n - n32 == 1)
            e = launch_march(jobs[n32], kF16, ctx->stream);
        else if (e == hipSuccess && n - n32 > 1)
            e = launch_march_checkpointed_many(dj + n32, dp + n32 + 1, n - n32, prefix[n + 1], kF16, ctx->stream);
        if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    } catch (const std::bad_alloc&) {
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    }
    return ok(ctx);
}

// Kernel parameters of the adjoint of one partial (validated).
static vr_status prepare_backward(vr_context ctx, vr_brick b, const vr_partial* part, int32_t interval,
                                  const float* ckpt, size_t ckpt_bytes, const float* d_part, float* grad_tf,
                                  float* grad_volume, const int32_t vol_dims[3], const int32_t lo[3], const char* who,
                                  MarchParams& p, BackwardParams& bp) {
    vr_status st = prepare_march(ctx, b, part, who, p);
    if (st != VR_OK) return st;
    size_t need = 0;
    st = vr_checkpoint_size(ctx, b, part, interval, &need);
    if (st != VR_OK) return st;
    if (!ckpt || ckpt_bytes < need)
        return fail(ctx, VR_ERR_WORKSPACE, "%s: checkpoint buffer of %zu bytes, need %zu", who, ckpt_bytes, need);
    if (!d_part || !grad_tf || !grad_volume || !vol_dims || !lo)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: NULL argument", who);
    if ((reinterpret_cast<uintptr_t>(d_part) & 15) != 0 || (reinterpret_cast<uintptr_t>(grad_tf) & 3) != 0 ||
        (reinterpret_cast<uintptr_t>(grad_volume) & 3) != 0)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: misaligned buffer", who);
    bp = BackwardParams{};
    for (int c = 0; c < 3; ++c) {
        if (vol_dims[c] < 1 || lo[c] < 0 || (int64_t)lo[c] + b->dims[c] > vol_dims[c])
            return fail(ctx, VR_ERR_INVALID_ARG, "%s: owned box [%d, %d) on axis %d outside the %d-voxel grid", who,
                        lo[c], lo[c] + b->dims[c], c, vol_dims[c]);
        bp.vol_dims[c] = vol_dims[c];
        bp.lo[c] = lo[c];
    }
    bp.d_part = d_part;
    bp.grad_tf = grad_tf;
    bp.grad_vox = grad_volume;
    p.ert_eps = 0.0f;
    p.ckpt = const_cast<float*>(ckpt);
    p.ckpt_interval = interval;
    p.ckpt_nseg = (int32_t)ckpt_segments(b, ctx->dt, interval);
    p.samples = nullptr;
    return VR_OK;
}

vr_status vr_render_partial_backward(vr_context ctx, vr_brick b, const vr_partial* part,
                                     int32_t interval, const float* ckpt, size_t ckpt_bytes,
                                     const float* d_part, float* grad_tf, float* grad_volume,
                                     const int32_t vol_dims[3], const int32_t lo[3]) {
    static const char* who = "vr_render_partial_backward";
    MarchParams p;
    BackwardParams bp;
    vr_status st = prepare_backward(ctx, b, part, interval, ckpt, ckpt_bytes, d_part, grad_tf, grad_volume, vol_dims,
                                    lo, who, p, bp);
    if (st != VR_OK) return st;
    if (part->w == 0 || part->h == 0) return ok(ctx);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
    hipError_t e = launch_march_backward(p, bp, b->storage == VR_F16 ? kF16 : kF32, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    return ok(ctx);
}

// Workspace of vr_render_partials_backward: [BackwardJob x n | 256][block prefix int32 x (n + 2) | 256].
static size_t backward_ws_bytes(int32_t n, size_t* off_prefix) {
    const size_t jobs = (((size_t)n * sizeof(BackwardJob)) + 255) / 256 * 256;
    if (off_prefix) *off_prefix = jobs;
    return jobs + (((size_t)(n + 2) * sizeof(int32_t)) + 255) / 256 * 256;
}

vr_status vr_backward_workspace_size(int32_t n, size_t* bytes) {
    if (n < 0 || !bytes) return fail(nullptr, VR_ERR_INVALID_ARG, "vr_backward_workspace_size: bad argument");
    *bytes = backward_ws_bytes(n, nullptr);
    return VR_OK;
}

vr_status vr_render_partials_backward(vr_context ctx, int32_t n, const vr_brick* bricks, const vr_partial* parts,
                                      int32_t interval, const float* const* ckpts, const size_t* ckpt_bytes,
                                      const float* const* d_parts, float* grad_tf, float* grad_volume,
                                      const int32_t vol_dims[3], const int32_t* los, void* workspace,
                                      size_t workspace_bytes) {
    static const char* who = "vr_render_partials_backward";
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (n < 0 || (n > 0 && (!bricks || !parts || !ckpts || !ckpt_bytes || !d_parts || !los)))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: bad n or NULL arrays", who);
    if (n == 0) return ok(ctx);
    size_t off_prefix = 0;
    const size_t need = backward_ws_bytes(n, &off_prefix);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(ctx, VR_ERR_WORKSPACE, "%s: workspace of %zu bytes (256-aligned), need %zu", who,
                    workspace_bytes, need);
    try {
        // jobs grouped by storage precision (float32 first); each group is one launch
        std::vector<BackwardJob> jobs;
        std::vector<int32_t> prefix(n + 2, 0);
        const int W = backward_many_waves();
        int n32 = 0;
        for (int pass = 0; pass < 2; ++pass) {
            int32_t acc = 0;
            const int base = pass == 0 ? 0 : n32 + 1;
            int cnt = 0;
            for (int i = 0; i < n; ++i) {
                if (!live(bricks[i]) || bricks[i]->ctx != ctx)
                    return fail(ctx, VR_ERR_INVALID_HANDLE, "%s: invalid brick %d", who, i);
                if ((bricks[i]->storage == VR_F16) != (pass == 1)) continue;
                BackwardJob j;
                vr_status st = prepare_backward(ctx, bricks[i], &parts[i], interval, ckpts[i], ckpt_bytes[i],
                                                d_parts[i], grad_tf, grad_volume, vol_dims, los + 3 * i, who, j.p,
                                                j.bp);
                if (st != VR_OK) return st;
                prefix[base + cnt] = acc;
                acc += (j.p.tiles_x * j.p.tiles_y + W - 1) / W;
                jobs.push_back(j);
                ++cnt;
            }
            prefix[base + cnt] = acc;
            if (pass == 0) n32 = cnt;
        }
        char* ws = reinterpret_cast<char*>(workspace);
        DeviceGuard g(ctx->device);
        if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
        hipError_t e = hipMemcpyAsync(ws, jobs.data(), jobs.size() * sizeof(BackwardJob), hipMemcpyHostToDevice,
                                      ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws + off_prefix, prefix.data(), prefix.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               ctx->stream);
        const BackwardJob* dj = reinterpret_cast<const BackwardJob*>(ws);
        const int32_t* dp = reinterpret_cast<const int32_t*>(ws + off_prefix);
        // a group of one partial takes the by-value kernel (its parameters in
        // kernel arguments rather than in the table)
        if (e == hipSuccess && n32 == 1)
            e = launch_march_backward(jobs[0].p, jobs[0].bp, kF32, ctx->stream);
        else if (e == hipSuccess && n32 > 1)
            e = launch_march_backward_many(dj, dp, n32, prefix[n32], kF32, ctx->stream);
        if (e == hipSuccess && n - n32 == 1)
            e = launch_march_backward(jobs[n32].p, jobs[n32].bp, kF16, ctx->stream);
        else if (e == hipSuccess && n - n32 > 1)
            e = launch_march_backward_many(dj + n32, dp + n32 + 1, n - n32, prefix[n + 1], kF16, ctx->stream);
        if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    } catch (const std::bad_alloc&) {
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    }
    return ok(ctx);
}

// ---------------------------------------------------- time-step streaming
struct vr_timeseries_s {
    vr_context ctx = nullptr;
    int32_t n_bricks = 0, n_steps = 0, slots = 0;
    std::vector<vr_brick_desc> desc;
    std::vector<const float*> host;       // n_steps x n_bricks host pointers (borrowed)
    std::vector<vr_brick> slot_bricks;    // slots x n_bricks
    std::vector<int32_t> slot_step;       // step a slot holds (-1: none)
    std::vector<uint64_t> slot_used;      // last acquire/prefetch (LRU clock)
    std::vector<hipEvent_t> slot_ready;   // copy stream: the slot's last ingest done
    std::vector<int32_t> step_slot;       // slot of a step (-1: not resident)
    hipEvent_t render_mark = nullptr;     // render stream: work enqueued before an eviction
    hipStream_t copy = nullptr;
    float* staging = nullptr;             // device, largest float32 ghost-padded brick
    uint64_t clock = 0;
    int64_t loads = 0;
};

namespace {

size_t ts_brick_bytes(const vr_brick_desc& d) {
    size_t b = 0;
    (void)vr_brick_workspace_size(d.dims, d.ghost, d.storage, &b);
    return b;
}

// Bytes of a step's host array of one brick: the ghost-padded voxels as
// float32, rows unpadded (the ingest kernel's source layout).
size_t ts_source_bytes(const vr_brick_desc& d) {
    return (size_t)(d.dims[0] + 2 * d.ghost) * (size_t)(d.dims[1] + 2 * d.ghost) *
           (size_t)(d.dims[2] + 2 * d.ghost) * sizeof(float);
}

size_t ts_staging_bytes(const std::vector<vr_brick_desc>& desc) {
    size_t m = 0;
    for (const vr_brick_desc& d : desc) m = std::max(m, ts_source_bytes(d));
    return (m + 255) & ~(size_t)255;
}

size_t ts_workspace_bytes(const std::vector<vr_brick_desc>& desc, int32_t slots) {
    size_t per = 0;
    for (const vr_brick_desc& d : desc) per += ts_brick_bytes(d);
    return (size_t)slots * per + ts_staging_bytes(desc);
}

vr_status ts_check(vr_context ctx, int32_t n_bricks, const vr_brick_desc* bricks, int32_t slots, const char* who) {
    if (n_bricks < 1 || n_bricks > DPVR_MAX_PARTIALS || !bricks)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: n_bricks = %d outside [1, %d] or NULL", who, n_bricks,
                    DPVR_MAX_PARTIALS);
    if (slots < 1) return fail(ctx, VR_ERR_INVALID_ARG, "%s: slots must be >= 1", who);
    for (int i = 0; i < n_bricks; ++i) {
        const vr_brick_desc& d = bricks[i];
        size_t b = 0;
        if (vr_brick_workspace_size(d.dims, d.ghost, d.storage, &b) != VR_OK)
            return fail(ctx, VR_ERR_INVALID_ARG, "%s: brick %d: %s", who, i, t_err.c_str());
        if (!finite3(d.origin)) return fail(ctx, VR_ERR_INVALID_ARG, "%s: brick %d: origin not finite", who, i);
        for (int c = 0; c < 3; ++c)
            if (!(d.spacing[c] > 0) || !std::isfinite(d.spacing[c]))
                return fail(ctx, VR_ERR_INVALID_ARG, "%s: brick %d: spacing must be finite and > 0", who, i);
    }
    return VR_OK;
}

void ts_destroy(vr_timeseries ts) {
    if (ts->copy) (void)hipStreamSynchronize(ts->copy);
    for (vr_brick b : ts->slot_bricks) {
        if (!b) continue;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            g_live.erase(b);
        }
        if (live(b->ctx)) b->ctx->live_bricks--;
        delete b;
    }
    for (hipEvent_t e : ts->slot_ready)
        if (e) (void)hipEventDestroy(e);
    if (ts->render_mark) (void)hipEventDestroy(ts->render_mark);
    if (ts->copy) (void)hipStreamDestroy(ts->copy);
    delete ts;
}

// Make `step` resident (no-op if it is): take the least recently used slot,
// let the copy stream wait for the render work enqueued so far (which is
// all the work that can read the evicted step), then upload and ingest the
// step's bricks on the copy stream and record the slot's ready event.
vr_status ts_load(vr_timeseries ts, int32_t step, const char* who) {
    vr_context ctx = ts->ctx;
    ++ts->clock;
    if (ts->step_slot[step] >= 0) {
        ts->slot_used[ts->step_slot[step]] = ts->clock;
        return VR_OK;
    }
    int s = -1;                           // an empty slot, else the least recently used one
    for (int i = 0; i < ts->slots && s < 0; ++i)
        if (ts->slot_step[i] < 0) s = i;
    if (s < 0) {
        s = 0;
        for (int i = 1; i < ts->slots; ++i)
            if (ts->slot_used[i] < ts->slot_used[s]) s = i;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
    hipError_t e = hipSuccess;
    if (ts->slot_step[s] >= 0) {
        ts->step_slot[ts->slot_step[s]] = -1;
        e = hipEventRecord(ts->render_mark, ctx->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(ts->copy, ts->render_mark, 0);
    }
    for (int b = 0; b < ts->n_bricks && e == hipSuccess; ++b) {
        const vr_brick_desc& d = ts->desc[b];
        int32_t sdim[3];
        for (int c = 0; c < 3; ++c) sdim[c] = d.dims[c] + 2 * d.ghost;
        e = hipMemcpyAsync(ts->staging, ts->host[(size_t)step * ts->n_bricks + b], ts_source_bytes(d),
                           hipMemcpyHostToDevice, ts->copy);
        if (e == hipSuccess)
            e = launch_ingest(ts->staging, ts->slot_bricks[(size_t)s * ts->n_bricks + b]->ws, sdim,
                              d.storage == VR_F16 ? kF16 : kF32, ts->copy);
    }
    if (e == hipSuccess) e = hipEventRecord(ts->slot_ready[s], ts->copy);
    if (e != hipSuccess) {
        ts->slot_step[s] = -1;
        return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    }
    for (int b = 0; b < ts->n_bricks; ++b) ts->slot_bricks[(size_t)s * ts->n_bricks + b]->has_data = true;
    ts->slot_step[s] = step;
    ts->step_slot[step] = s;
    ts->slot_used[s] = ts->clock;
    ++ts->loads;
    return VR_OK;
}

}  // namespace

vr_status vr_timeseries_workspace_size(int32_t n_bricks, const vr_brick_desc* bricks, int32_t slots, size_t* bytes) {
    static const char* who = "vr_timeseries_workspace_size";
    if (!bytes) return fail(nullptr, VR_ERR_INVALID_ARG, "%s: bytes is NULL", who);
    vr_status st = ts_check(nullptr, n_bricks, bricks, slots, who);
    if (st != VR_OK) return st;
    try {
        *bytes = ts_workspace_bytes(std::vector<vr_brick_desc>(bricks, bricks + n_bricks), slots);
    } catch (const std::bad_alloc&) {
        return fail(nullptr, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    }
    return VR_OK;
}

vr_status vr_timeseries_create(vr_context ctx, int32_t n_bricks, const vr_brick_desc* bricks, int32_t n_steps,
                               const float* const* host_voxels, int32_t slots, void* workspace,
                               size_t workspace_bytes, vr_timeseries* out) {
    static const char* who = "vr_timeseries_create";
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (!out) return fail(ctx, VR_ERR_INVALID_ARG, "%s: out is NULL", who);
    *out = nullptr;
    vr_status st = ts_check(ctx, n_bricks, bricks, slots, who);
    if (st != VR_OK) return st;
    if (n_steps < 1 || !host_voxels) return fail(ctx, VR_ERR_INVALID_ARG, "%s: n_steps < 1 or NULL host array", who);
    for (int64_t i = 0; i < (int64_t)n_steps * n_bricks; ++i)
        if (!host_voxels[i]) return fail(ctx, VR_ERR_INVALID_ARG, "%s: host voxel pointer %lld is NULL", who, (long long)i);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(ctx, VR_ERR_WORKSPACE, "%s: workspace NULL or not 256-byte aligned", who);
    vr_timeseries ts = new (std::nothrow) vr_timeseries_s;
    if (!ts) return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    try {
        ts->ctx = ctx;
        ts->n_bricks = n_bricks;
        ts->n_steps = n_steps;
        ts->slots = slots;
        ts->desc.assign(bricks, bricks + n_bricks);
        const size_t need = ts_workspace_bytes(ts->desc, slots);
        if (workspace_bytes < need) {
            delete ts;
            return fail(ctx, VR_ERR_WORKSPACE, "%s: workspace of %zu bytes, need %zu", who, workspace_bytes, need);
        }
        ts->host.assign(host_voxels, host_voxels + (size_t)n_steps * n_bricks);
        ts->slot_step.assign(slots, -1);
        ts->slot_used.assign(slots, 0);
        ts->slot_ready.assign(slots, nullptr);
        ts->step_slot.assign(n_steps, -1);
        ts->slot_bricks.assign((size_t)slots * n_bricks, nullptr);
        char* w = reinterpret_cast<char*>(workspace);
        for (int s = 0; s < slots; ++s)
            for (int b = 0; b < n_bricks; ++b) {
                const vr_brick_desc& d = ts->desc[b];
                vr_brick br = new vr_brick_s;
                br->ctx = ctx;
                for (int c = 0; c < 3; ++c) {
                    br->dims[c] = d.dims[c];
                    br->origin[c] = d.origin[c];
                    br->spacing[c] = d.spacing[c];
                }
                br->ghost = d.ghost;
                br->storage = d.storage;
                br->ws = w;
                br->ws_bytes = ts_brick_bytes(d);
                br->owner = ts;
                w += br->ws_bytes;
                {
                    std::lock_guard<std::mutex> lk(g_mu);
                    g_live.insert(br);
                }
                ctx->live_bricks++;
                ts->slot_bricks[(size_t)s * n_bricks + b] = br;
            }
        ts->staging = reinterpret_cast<float*>(w);
        DeviceGuard g(ctx->device);
        hipError_t e = g.ok ? hipSuccess : hipErrorInvalidDevice;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&ts->copy, hipStreamNonBlocking);
        for (int s = 0; s < slots && e == hipSuccess; ++s)
            e = hipEventCreateWithFlags(&ts->slot_ready[s], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ts->render_mark, hipEventDisableTiming);
        if (e != hipSuccess) {
            ts_destroy(ts);
            return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
        }
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(ts);
    } catch (const std::bad_alloc&) {
        ts_destroy(ts);
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    }
    ctx->live_bricks++;   // the series pins the context like a brick does
    *out = ts;
    return ok(ctx);
}

vr_status vr_timeseries_prefetch(vr_timeseries ts, int32_t step) {
    static const char* who = "vr_timeseries_prefetch";
    if (!live(ts)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid time series", who);
    if (step < 0 || step >= ts->n_steps)
        return fail(ts->ctx, VR_ERR_INVALID_ARG, "%s: step %d outside [0, %d)", who, step, ts->n_steps);
    vr_status st = ts_load(ts, step, who);
    return st == VR_OK ? ok(ts->ctx) : st;
}

vr_status vr_timeseries_acquire(vr_timeseries ts, int32_t step, vr_brick* bricks) {
    static const char* who = "vr_timeseries_acquire";
    if (!live(ts)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid time series", who);
    vr_context ctx = ts->ctx;
    if (step < 0 || step >= ts->n_steps || !bricks)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: step %d outside [0, %d) or NULL output", who, step, ts->n_steps);
    vr_status st = ts_load(ts, step, who);
    if (st != VR_OK) return st;
    const int s = ts->step_slot[step];
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
    const hipError_t e = hipStreamWaitEvent(ctx->stream, ts->slot_ready[s], 0);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    for (int b = 0; b < ts->n_bricks; ++b) bricks[b] = ts->slot_bricks[(size_t)s * ts->n_bricks + b];
    return ok(ctx);
}

vr_status vr_timeseries_stats(vr_timeseries ts, int64_t* loads, int32_t* resident_steps) {
    if (!live(ts)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_timeseries_stats: invalid time series");
    if (loads) *loads = ts->loads;
    if (resident_steps)
        for (int s = 0; s < ts->slots; ++s) resident_steps[s] = ts->slot_step[s];
    return ok(ts->ctx);
}

vr_status vr_timeseries_release(vr_timeseries ts) {
    if (!live(ts)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_timeseries_release: invalid time series");
    vr_context ctx = ts->ctx;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.erase(ts);
    }
    if (live(ctx)) {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);   // renders that read the slots
        ctx->live_bricks--;
    }
    ts_destroy(ts);
    return VR_OK;
}

// ------------------------------------------------------- ray-queue cycling
// Workspace of vr_rqc_plan / vr_render_rqc: [RqcBrick x n][kf int32 x E]
// [offsets int64 x (E + 1)][scan block sums int64][segments float x W H n 5],
// each part 256-byte aligned.
static size_t rqc_layout(int32_t n, long long E, int W, int H, size_t off[5]) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    size_t o = 0;
    off[0] = o; o += up((size_t)n * sizeof(RqcBrick));
    off[1] = o; o += up((size_t)E * sizeof(int32_t));
    off[2] = o; o += up((size_t)(E + 1) * sizeof(long long));
    off[3] = o; o += up((size_t)(rqc_scan_blocks(E) + 1) * sizeof(long long));
    off[4] = o; o += up((size_t)W * H * (size_t)n * 5 * sizeof(float));
    return o;
}

// The bricks' ROIs and RqcBrick table for the context camera; E = ROI pixels.
static vr_status rqc_bricks(vr_context ctx, int32_t n, const vr_brick* bricks, const char* who, bool need_data,
                            std::vector<RqcBrick>& tab, long long* E) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (n < 1 || n > DPVR_MAX_PARTIALS || !bricks)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: n = %d outside [1, %d] or NULL bricks", who, n, DPVR_MAX_PARTIALS);
    if (!ctx->has_camera) return fail(ctx, VR_ERR_STATE, "%s: no camera set", who);
    tab.assign(n, RqcBrick{});
    long long e = 0;
    for (int i = 0; i < n; ++i) {
        vr_brick b = bricks[i];
        if (!live(b) || b->ctx != ctx) return fail(ctx, VR_ERR_INVALID_HANDLE, "%s: invalid brick %d", who, i);
        if (need_data && !b->has_data) return fail(ctx, VR_ERR_STATE, "%s: brick %d has no voxel data", who, i);
        for (int j = 0; j < i; ++j)
            if (bricks[j] == b) return fail(ctx, VR_ERR_INVALID_ARG, "%s: brick %d repeats brick %d", who, i, j);
        RqcBrick& r = tab[i];
        r.brick.data = b->ws;
        for (int c = 0; c < 3; ++c) {
            r.brick.sdim[c] = b->dims[c] + 2 * b->ghost;
            r.brick.lo[c] = b->origin[c];
            r.brick.hi[c] = b->origin[c] + (double)b->dims[c] * b->spacing[c];
            r.brick.origin[c] = b->origin[c];
            r.brick.spacing[c] = b->spacing[c];
            r.brick.inv_spacing[c] = 1.0 / b->spacing[c];
        }
        r.brick.ghost = b->ghost;
        int32_t roi[4];
        roi_for(ctx->cam, b, roi);
        r.roi_x0 = roi[0];
        r.roi_y0 = roi[1];
        r.roi_w = roi[2];
        r.roi_h = roi[3];
        r.entry0 = e;
        r.storage = b->storage == VR_F16 ? kF16 : kF32;
        e += (long long)roi[2] * roi[3];
    }
    *E = e;
    return VR_OK;
}

vr_status vr_rqc_workspace_size(vr_context ctx, int32_t n, const vr_brick* bricks, size_t* bytes) {
    static const char* who = "vr_rqc_workspace_size";
    if (!bytes) return fail(live(ctx) ? ctx : nullptr, VR_ERR_INVALID_ARG, "%s: bytes is NULL", who);
    std::vector<RqcBrick> tab;
    long long E = 0;
    try {
        vr_status st = rqc_bricks(ctx, n, bricks, who, false, tab, &E);
        if (st != VR_OK) return st;
    } catch (const std::bad_alloc&) {
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    }
    size_t off[5];
    *bytes = rqc_layout(n, E, ctx->cam.width, ctx->cam.height, off);
    return ok(ctx);
}

vr_status vr_rqc_plan(vr_context ctx, int32_t n, const vr_brick* bricks, void* workspace, size_t workspace_bytes,
                      int64_t* total_samples) {
    static const char* who = "vr_rqc_plan";
    std::vector<RqcBrick> tab;
    long long E = 0;
    try {
        vr_status st = rqc_bricks(ctx, n, bricks, who, false, tab, &E);
        if (st != VR_OK) return st;
        if (!total_samples) return fail(ctx, VR_ERR_INVALID_ARG, "%s: total_samples is NULL", who);
        size_t off[5];
        const size_t need = rqc_layout(n, E, ctx->cam.width, ctx->cam.height, off);
        if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
            return fail(ctx, VR_ERR_WORKSPACE, "%s: workspace of %zu bytes (256-aligned), need %zu", who,
                        workspace_bytes, need);
        DeviceGuard g(ctx->device);
        if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
        char* ws = reinterpret_cast<char*>(workspace);
        RqcParams p{};
        p.cam = ctx->cam;
        p.dt = ctx->dt;
        p.inv_dt = 1.0 / ctx->dt;
        p.n = n;
        p.width = ctx->cam.width;
        p.height = ctx->cam.height;
        p.bricks = reinterpret_cast<const RqcBrick*>(ws + off[0]);
        p.n_entries = E;
        p.kf = reinterpret_cast<int32_t*>(ws + off[1]);
        p.offsets = reinterpret_cast<long long*>(ws + off[2]);
        p.err = err_word(ctx);
        long long total = 0;
        hipError_t e = hipMemcpyAsync(ws + off[0], tab.data(), tab.size() * sizeof(RqcBrick), hipMemcpyHostToDevice,
                                      ctx->stream);
        if (e == hipSuccess)
            e = launch_rqc_plan(p, reinterpret_cast<long long*>(ws + off[3]), p.offsets + E, ctx->stream);
        if (e == hipSuccess && E > 0)
            e = hipMemcpyAsync(&total, p.offsets + E, sizeof(long long), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
        ctx->rqc.ws = workspace;
        ctx->rqc.bricks.assign(bricks, bricks + n);
        ctx->rqc.cam = ctx->cam;
        ctx->rqc.dt = ctx->dt;
        ctx->rqc.entries = E;
        ctx->rqc.total = total;
        *total_samples = total;
    } catch (const std::bad_alloc&) {
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    }
    return ok(ctx);
}

vr_status vr_render_rqc(vr_context ctx, int32_t n, const vr_brick* bricks, const vr_light* light, const float bg[4],
                        void* workspace, size_t workspace_bytes, float* shade, size_t shade_bytes, float* out,
                        unsigned long long* samples) {
    static const char* who = "vr_render_rqc";
    std::vector<RqcBrick> tab;
    long long E = 0;
    try {
        vr_status st = rqc_bricks(ctx, n, bricks, who, true, tab, &E);
        if (st != VR_OK) return st;
    } catch (const std::bad_alloc&) {
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    }
    if (!ctx->has_tf) return fail(ctx, VR_ERR_STATE, "%s: no transfer function set", who);
    const auto& pl = ctx->rqc;
    if (pl.ws != workspace || pl.total < 0 || (int32_t)pl.bricks.size() != n ||
        !std::equal(pl.bricks.begin(), pl.bricks.end(), bricks) || std::memcmp(&pl.cam, &ctx->cam, sizeof(CameraK)) != 0 ||
        pl.dt != ctx->dt || pl.entries != E)
        return fail(ctx, VR_ERR_STATE, "%s: no vr_rqc_plan of this workspace for these bricks, camera and spacing",
                    who);
    if (!light || !bg || !out) return fail(ctx, VR_ERR_INVALID_ARG, "%s: NULL argument", who);
    const double ln = std::sqrt(light->direction[0] * light->direction[0] + light->direction[1] * light->direction[1] +
                                light->direction[2] * light->direction[2]);
    if (!finite3(light->direction) || !(ln > 0.0) || !(light->ambient >= 0.0f && light->ambient <= 1.0f))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: light direction must be finite and non-zero, ambient in [0, 1]",
                    who);
    for (int c = 0; c < 4; ++c)
        if (!std::isfinite(bg[c])) return fail(ctx, VR_ERR_INVALID_ARG, "%s: background not finite", who);
    if ((reinterpret_cast<uintptr_t>(out) & 15) != 0 || (reinterpret_cast<uintptr_t>(samples) & 7) != 0)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: out must be 16-, samples 8-byte aligned", who);
    const bool shadows = light->ambient < 1.0f;
    if (shadows && (size_t)pl.total * sizeof(float) > shade_bytes)
        return fail(ctx, VR_ERR_WORKSPACE, "%s: shade buffer of %zu bytes, need %lld", who, shade_bytes,
                    pl.total * (long long)sizeof(float));
    if (shadows && pl.total > 0 && (!shade || (reinterpret_cast<uintptr_t>(shade) & 3) != 0))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: shade buffer NULL or misaligned", who);
    size_t off[5];
    const size_t need = rqc_layout(n, E, ctx->cam.width, ctx->cam.height, off);
    if (workspace_bytes < need) return fail(ctx, VR_ERR_WORKSPACE, "%s: workspace of %zu bytes, need %zu", who,
                                            workspace_bytes, need);
    char* ws = reinterpret_cast<char*>(workspace);
    RqcParams p{};
    p.cam = ctx->cam;
    p.tf = ctx->tf;
    p.dt = ctx->dt;
    p.inv_dt = 1.0 / ctx->dt;
    for (int c = 0; c < 3; ++c) p.light[c] = light->direction[c] / ln;
    p.ert_eps = ctx->ert_eps;
    p.ambient = light->ambient;
    p.shadows = shadows ? 1 : 0;
    p.n = n;
    p.width = ctx->cam.width;
    p.height = ctx->cam.height;
    p.bricks = reinterpret_cast<const RqcBrick*>(ws + off[0]);
    p.n_entries = E;
    p.kf = reinterpret_cast<int32_t*>(ws + off[1]);
    p.offsets = reinterpret_cast<long long*>(ws + off[2]);
    p.total = pl.total;
    p.shade = shade;
    p.segs = reinterpret_cast<float*>(ws + off[4]);
    p.out = out;
    for (int c = 0; c < 4; ++c) p.bg[c] = bg[c];
    p.samples = samples;
    p.err = err_word(ctx);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
    const hipError_t e = launch_rqc_frame(p, ctx->cus, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    return ok(ctx);
}

// ------------------------------------------------------ tetrahedral parts
struct vr_tetpart_s {
    vr_context ctx = nullptr;
    TetTables tab;
    int32_t n_input_vertices = 0;        // vertices whose values the caller gives
    std::vector<int32_t> centre_nodes;   // cell centres: 8 node indices each (-1 padded)
    // device workspace: [planes][vals][owned][tets][cell_start][cell_tets][nbr][centre_nodes]
    // [bvh_nodes][bvh_tets], each 256-aligned
    size_t off[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    size_t need = 0;
    char* ws = nullptr;
    bool has_values = false;
};

namespace {

size_t tetpart_layout(const TetTables& t, const std::vector<int32_t>& centre_nodes, size_t off[10]) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t nt = (size_t)t.n_tets;
    size_t o = 0;
    off[0] = o; o += up(nt * 16 * sizeof(double));
    off[1] = o; o += up(nt * 4 * sizeof(float));
    off[2] = o; o += up(nt * sizeof(uint32_t));
    off[3] = o; o += up(nt * 4 * sizeof(int32_t));
    off[4] = o; o += up(t.cell_start.size() * sizeof(int32_t));
    off[5] = o; o += up(t.cell_tets.size() * sizeof(int32_t));
    off[6] = o; o += up(t.nbr.size() * sizeof(int32_t));
    off[7] = o; o += up(centre_nodes.size() * sizeof(int32_t));
    off[8] = o; o += up(t.bvh_nodes.size() * sizeof(int32_t));
    off[9] = o; o += up(t.bvh_tets.size() * sizeof(int32_t));
    return o;
}

// Frame workspace of n parts: [TetPartK x n][tile prefix n + 1], then per
// part [run counts][run keys x max_runs][run colours x max_runs] over its ROI,
// each 256-aligned; ROIs from the context camera.
size_t tetframe_layout(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs,
                       std::vector<TetPartK>* jobs, std::vector<int32_t>* prefix, long long* entries = nullptr) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    size_t o = up((size_t)n * sizeof(TetPartK)) + up((size_t)(n + 1) * sizeof(int32_t));
    int32_t tiles = 0;
    long long E = 0;
    for (int i = 0; i < n; ++i) {
        const TetTables& t = parts[i]->tab;
        int32_t roi[4] = {0, 0, 0, 0};
        if (t.n_tets > 0) roi_for_box(ctx->cam, t.lo, t.hi, roi);
        const size_t np = (size_t)roi[2] * roi[3];
        if (jobs) {
            TetPartK k{};
            const vr_tetpart q = parts[i];
            k.planes = reinterpret_cast<const double*>(q->ws + q->off[0]);
            k.vals = reinterpret_cast<const float*>(q->ws + q->off[1]);
            k.owned = reinterpret_cast<const uint32_t*>(q->ws + q->off[2]);
            k.cell_start = reinterpret_cast<const int32_t*>(q->ws + q->off[4]);
            k.cell_tets = reinterpret_cast<const int32_t*>(q->ws + q->off[5]);
            k.nbr = reinterpret_cast<const int32_t*>(q->ws + q->off[6]);
            k.bvh_nodes = reinterpret_cast<const int32_t*>(q->ws + q->off[8]);
            k.bvh_tets = reinterpret_cast<const int32_t*>(q->ws + q->off[9]);
            for (int c = 0; c < 3; ++c) {
                k.lo[c] = t.lo[c];
                k.hi[c] = t.hi[c];
                k.glo[c] = t.glo[c];
                k.ginv[c] = t.ginv[c];
                k.gdim[c] = t.gdim[c];
            }
            k.n_tets = t.n_tets;
            k.roi_x0 = roi[0];
            k.roi_y0 = roi[1];
            k.roi_w = roi[2];
            k.roi_h = roi[3];
            k.entry0 = E;
            // run buffers: offsets now, device addresses once the workspace is known
            k.rcount = reinterpret_cast<int32_t*>(o);
            k.rkey = reinterpret_cast<int32_t*>(o + up(np * sizeof(int32_t)));
            k.rcol = reinterpret_cast<float*>(o + up(np * sizeof(int32_t)) + up(np * max_runs * sizeof(int32_t)));
            jobs->push_back(k);
            prefix->push_back(tiles);
        }
        tiles += tet_tiles(roi[2], roi[3]);
        E += (long long)np;
        o += up(np * sizeof(int32_t)) + up(np * max_runs * sizeof(int32_t)) + up(np * max_runs * 4 * sizeof(float));
    }
    if (prefix) prefix->push_back(tiles);
    if (entries) *entries = E;
    return o;
}

// Shadow plan of a tetrahedral frame: [offsets int64 x (E + 1)][scan block
// sums int64], each 256-aligned; E = the parts' ROI pixels.
size_t tetplan_layout(long long E, size_t* off_sums) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t a = up((size_t)(E + 1) * sizeof(long long));
    if (off_sums) *off_sums = a;
    return a + up((size_t)(scan_blocks(E) + 1) * sizeof(long long));
}

// Slots of a shadowed tetrahedral frame: [sample index int32 x total][shadow
// transmittance float x total], the second 256-aligned.
size_t tetslot_bytes(long long total, size_t* off_shade) {
    const size_t a = ((size_t)total * sizeof(int32_t) + 255) / 256 * 256;
    if (off_shade) *off_shade = a;
    return a + (size_t)total * sizeof(float);
}

vr_status tetparts_check(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs, const char* who,
                         bool need_values, bool need_tables = false) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (n < 1 || n > kMaxTetParts || !parts)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: n = %d outside [1, %d] or NULL parts", who, n, kMaxTetParts);
    if (max_runs < 1 || max_runs > kMaxTetRuns)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: max_runs = %d outside [1, %d]", who, max_runs, kMaxTetRuns);
    if (!ctx->has_camera) return fail(ctx, VR_ERR_STATE, "%s: no camera set", who);
    for (int i = 0; i < n; ++i) {
        vr_tetpart q = parts[i];
        if (!live(q) || q->ctx != ctx) return fail(ctx, VR_ERR_INVALID_HANDLE, "%s: invalid part %d", who, i);
        if (need_values && (!q->ws || !q->has_values))
            return fail(ctx, VR_ERR_STATE, "%s: part %d has no workspace or no vertex values", who, i);
        if (need_tables && !q->ws) return fail(ctx, VR_ERR_STATE, "%s: part %d has no workspace", who, i);
        for (int j = 0; j < i; ++j)
            if (parts[j] == q) return fail(ctx, VR_ERR_INVALID_ARG, "%s: part %d repeats part %d", who, i, j);
    }
    return VR_OK;
}

// Copy `bytes` from host memory to device memory at dst, in stream order,
// through the next of the context's two pinned host slots (once the copy that
// last read that slot has run; a slot smaller than `bytes` is reallocated).
hipError_t stage_copy(vr_context ctx, void* dst, const void* src, size_t bytes) {
    const int slot = ctx->pinned_next;
    ctx->pinned_next ^= 1;
    hipError_t e = hipEventSynchronize(ctx->pinned_done[slot]);
    if (e != hipSuccess) return e;
    if (ctx->pinned_bytes[slot] < bytes) {
        (void)hipHostFree(ctx->pinned[slot]);
        ctx->pinned[slot] = nullptr;
        ctx->pinned_bytes[slot] = 0;
        e = hipHostMalloc(&ctx->pinned[slot], bytes, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        ctx->pinned_bytes[slot] = bytes;
    }
    std::memcpy(ctx->pinned[slot], src, bytes);
    e = hipMemcpyAsync(dst, ctx->pinned[slot], bytes, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->pinned_done[slot], ctx->stream);
    return e;
}

}  // namespace

// A part from tetrahedra (cells == NULL) or from mixed cells.
static vr_status tetpart_create(vr_context ctx, const double* vertices, int32_t n_vertices, const int64_t* ids,
                                const int32_t* tets, int32_t n_tets, const uint8_t* sizes, const int32_t* cells,
                                int32_t n_cells, vr_tetpart* out, const char* who) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (!out) return fail(ctx, VR_ERR_INVALID_ARG, "%s: out is NULL", who);
    *out = nullptr;
    if (n_vertices < 0 || n_tets < 0 || n_cells < 0 || (n_vertices > 0 && !vertices) || (n_tets > 0 && !tets) ||
        (n_cells > 0 && (!sizes || !cells)))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: negative count or NULL array", who);
    std::unique_ptr<vr_tetpart_s> q(new (std::nothrow) vr_tetpart_s);
    if (!q) return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    try {
        std::string msg;
        q->n_input_vertices = n_vertices;
        bool okb;
        if (sizes) {
            std::vector<double> v;
            std::vector<int32_t> t;
            if (!decompose_cells(vertices, n_vertices, ids, sizes, cells, n_cells, v, t, q->centre_nodes, msg))
                return fail(ctx, VR_ERR_INVALID_ARG, "%s: %s", who, msg.c_str());
            okb = build_tet_tables(v.data(), (int32_t)(v.size() / 3), t.data(), (int32_t)(t.size() / 4), q->tab, msg);
        } else {
            okb = build_tet_tables(vertices, n_vertices, tets, n_tets, q->tab, msg);
        }
        if (!okb) return fail(ctx, VR_ERR_INVALID_ARG, "%s: %s", who, msg.c_str());
        q->need = tetpart_layout(q->tab, q->centre_nodes, q->off);
        q->ctx = ctx;
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(q.get());
    } catch (const std::bad_alloc&) {
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory for the location tables", who);
    }
    ctx->live_tetparts++;
    *out = q.release();
    return ok(ctx);
}

vr_status vr_set_tet_locator(vr_context ctx, vr_tet_locator locator) {
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_set_tet_locator: invalid context");
    if (locator != VR_TET_GRID && locator != VR_TET_BVH)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_set_tet_locator: unknown locator %d", (int)locator);
    ctx->tet_locator = locator == VR_TET_BVH ? kTetBvh : kTetGrid;
    return ok(ctx);
}

vr_status vr_tetpart_create(vr_context ctx, const double* vertices, int32_t n_vertices, const int32_t* tets,
                            int32_t n_tets, vr_tetpart* out) {
    return tetpart_create(ctx, vertices, n_vertices, nullptr, tets, n_tets, nullptr, nullptr, 0, out,
                          "vr_tetpart_create");
}

vr_status vr_tetpart_create_cells(vr_context ctx, const double* vertices, int32_t n_vertices, const int64_t* vertex_ids,
                                  const uint8_t* cell_sizes, const int32_t* cell_vertices, int32_t n_cells,
                                  vr_tetpart* out) {
    return tetpart_create(ctx, vertices, n_vertices, vertex_ids, nullptr, 0, cell_sizes, cell_vertices, n_cells, out,
                          "vr_tetpart_create_cells");
}

vr_status vr_tetpart_info(vr_tetpart q, double lo[3], double hi[3], int32_t grid[3], int64_t* grid_entries,
                          size_t* workspace_bytes, int32_t* n_tets) {
    if (!live(q)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_tetpart_info: invalid part");
    if (n_tets) *n_tets = q->tab.n_tets;
    for (int c = 0; c < 3; ++c) {
        if (lo) lo[c] = q->tab.lo[c];
        if (hi) hi[c] = q->tab.hi[c];
        if (grid) grid[c] = q->tab.gdim[c];
    }
    if (grid_entries) *grid_entries = (int64_t)q->tab.cell_tets.size();
    if (workspace_bytes) *workspace_bytes = q->need;
    return ok(q->ctx);
}

vr_status vr_tetpart_attach(vr_tetpart q, void* workspace, size_t workspace_bytes) {
    static const char* who = "vr_tetpart_attach";
    if (!live(q)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid part", who);
    vr_context ctx = q->ctx;
    if (!workspace || workspace_bytes < q->need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(ctx, VR_ERR_WORKSPACE, "%s: workspace of %zu bytes (256-aligned), need %zu", who,
                    workspace_bytes, q->need);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
    char* ws = reinterpret_cast<char*>(workspace);
    const TetTables& t = q->tab;
    // the tables stay in the part's host memory until it is released, which
    // waits for the context stream
    struct {
        size_t off;
        const void* src;
        size_t bytes;
    } copies[9] = {{q->off[0], t.planes.data(), t.planes.size() * sizeof(double)},
                   {q->off[2], t.owned.data(), t.owned.size() * sizeof(uint32_t)},
                   {q->off[3], t.tets.data(), t.tets.size() * sizeof(int32_t)},
                   {q->off[4], t.cell_start.data(), t.cell_start.size() * sizeof(int32_t)},
                   {q->off[5], t.cell_tets.data(), t.cell_tets.size() * sizeof(int32_t)},
                   {q->off[6], t.nbr.data(), t.nbr.size() * sizeof(int32_t)},
                   {q->off[7], q->centre_nodes.data(), q->centre_nodes.size() * sizeof(int32_t)},
                   {q->off[8], t.bvh_nodes.data(), t.bvh_nodes.size() * sizeof(int32_t)},
                   {q->off[9], t.bvh_tets.data(), t.bvh_tets.size() * sizeof(int32_t)}};
    hipError_t e = hipSuccess;
    for (const auto& c : copies)
        if (e == hipSuccess && c.bytes > 0)
            e = hipMemcpyAsync(ws + c.off, c.src, c.bytes, hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    q->ws = ws;
    q->has_values = false;
    return ok(ctx);
}

vr_status vr_tetpart_set_values(vr_tetpart q, const float* values) {
    static const char* who = "vr_tetpart_set_values";
    if (!live(q)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid part", who);
    vr_context ctx = q->ctx;
    if (!q->ws) return fail(ctx, VR_ERR_STATE, "%s: no workspace attached", who);
    if (!values && q->n_input_vertices > 0) return fail(ctx, VR_ERR_INVALID_ARG, "%s: values is NULL", who);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
    hipError_t e = launch_tet_values(values, q->n_input_vertices, reinterpret_cast<const int32_t*>(q->ws + q->off[7]),
                                     reinterpret_cast<const int32_t*>(q->ws + q->off[3]), q->tab.n_tets,
                                     reinterpret_cast<float*>(q->ws + q->off[1]), ctx->stream);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    q->has_values = true;
    return ok(ctx);
}

vr_status vr_tetpart_release(vr_tetpart q) {
    if (!live(q)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_tetpart_release: invalid part");
    vr_context ctx = q->ctx;
    if (q->ws) {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);   // copies out of the host tables may still run
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.erase(q);
    }
    if (live(ctx)) ctx->live_tetparts--;
    delete q;
    return VR_OK;
}

vr_status vr_tetparts_workspace_size(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs,
                                     size_t* bytes) {
    static const char* who = "vr_tetparts_workspace_size";
    vr_status st = tetparts_check(ctx, n, parts, max_runs, who, false);
    if (st != VR_OK) return st;
    if (!bytes) return fail(ctx, VR_ERR_INVALID_ARG, "%s: bytes is NULL", who);
    *bytes = tetframe_layout(ctx, n, parts, max_runs, nullptr, nullptr);
    return ok(ctx);
}

// Shadow inputs of a tetrahedral frame: the plan call fills the plan and
// reports the slot count; the shadowed render reads the plan and uses the
// slots.
struct TetShadowArgs {
    void* plan = nullptr;
    size_t plan_bytes = 0;
    void* slots = nullptr;
    size_t slot_bytes = 0;
    const vr_light* light = nullptr;
    int64_t* total_out = nullptr;
};

// The frame of n parts, `stages` a mask of the kTet* stages (march into the
// workspace's run buffers, resolve into out; with `sh`: count + scan into
// the plan, or record + shadow steps + shaded march).
static vr_status tet_frame(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs, const float bg[4],
                           void* workspace, size_t workspace_bytes, float* out, unsigned long long* samples,
                           int stages, const char* who, const TetShadowArgs* sh = nullptr) {
    const bool shading = stages & (kTetMarch | kTetShadow | kTetShaded);
    vr_status st = tetparts_check(ctx, n, parts, max_runs, who, shading, true);
    if (st != VR_OK) return st;
    if (shading && !ctx->has_tf) return fail(ctx, VR_ERR_STATE, "%s: no transfer function set", who);
    if ((stages & kTetResolve) && (!bg || !out)) return fail(ctx, VR_ERR_INVALID_ARG, "%s: NULL argument", who);
    if (stages & kTetResolve)
        for (int c = 0; c < 4; ++c)
            if (!std::isfinite(bg[c])) return fail(ctx, VR_ERR_INVALID_ARG, "%s: background not finite", who);
    if ((reinterpret_cast<uintptr_t>(out) & 15) != 0 || (reinterpret_cast<uintptr_t>(samples) & 7) != 0)
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: out must be 16-, samples 8-byte aligned", who);
    if (stages == kTetResolve) {
        const auto& lm = ctx->tetmarch;
        if (lm.ws != workspace || lm.max_runs != max_runs || (int32_t)lm.parts.size() != n ||
            !std::equal(lm.parts.begin(), lm.parts.end(), parts) || std::memcmp(&lm.cam, &ctx->cam, sizeof(CameraK)))
            return fail(ctx, VR_ERR_STATE, "%s: no vr_march_tetparts of these parts, max_runs and camera into "
                        "this workspace", who);
    }
    std::vector<TetPartK> jobs;
    std::vector<int32_t> prefix;
    size_t need = 0;
    long long E = 0;
    try {
        jobs.reserve(n);
        prefix.reserve(n + 1);
        need = tetframe_layout(ctx, n, parts, max_runs, &jobs, &prefix, &E);
    } catch (const std::bad_alloc&) {
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    }
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(ctx, VR_ERR_WORKSPACE, "%s: workspace of %zu bytes (256-aligned), need %zu", who,
                    workspace_bytes, need);
    TetFrameParams f{};
    if (sh) {
        size_t off_sums = 0;
        const size_t pneed = tetplan_layout(E, &off_sums);
        if (!sh->plan || sh->plan_bytes < pneed || (reinterpret_cast<uintptr_t>(sh->plan) & 255) != 0)
            return fail(ctx, VR_ERR_WORKSPACE, "%s: plan of %zu bytes (256-aligned), need %zu", who, sh->plan_bytes,
                        pneed);
        f.offsets = reinterpret_cast<long long*>(sh->plan);
        f.n_entries = E;
        if (stages & kTetRecord) {
            const auto& pl = ctx->tetplan;
            if (pl.plan != sh->plan || pl.total < 0 || (int32_t)pl.parts.size() != n ||
                !std::equal(pl.parts.begin(), pl.parts.end(), parts) ||
                std::memcmp(&pl.cam, &ctx->cam, sizeof(CameraK)) != 0 || pl.dt != ctx->dt || pl.entries != E)
                return fail(ctx, VR_ERR_STATE, "%s: no vr_tetparts_shadow_plan of this plan for these parts, camera "
                            "and spacing", who);
            if (!sh->light) return fail(ctx, VR_ERR_INVALID_ARG, "%s: light is NULL", who);
            const double* L = sh->light->direction;
            const double ln = std::sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
            if (!finite3(L) || !(ln > 0.0) || !(sh->light->ambient >= 0.0f && sh->light->ambient <= 1.0f))
                return fail(ctx, VR_ERR_INVALID_ARG, "%s: light direction must be finite and non-zero, ambient in "
                            "[0, 1]", who);
            size_t off_shade = 0;
            const size_t sneed = tetslot_bytes(pl.total, &off_shade);
            if (pl.total > 0 && (!sh->slots || sh->slot_bytes < sneed || (reinterpret_cast<uintptr_t>(sh->slots) & 255)))
                return fail(ctx, VR_ERR_WORKSPACE, "%s: slots of %zu bytes (256-aligned), need %zu", who,
                            sh->slot_bytes, sneed);
            f.total = pl.total;
            f.slot_k = reinterpret_cast<int32_t*>(sh->slots);
            f.shade = sh->slots ? reinterpret_cast<float*>(reinterpret_cast<char*>(sh->slots) + off_shade) : nullptr;
            for (int c = 0; c < 3; ++c) f.light[c] = L[c] / ln;
            f.ambient = sh->light->ambient;
        }
    }
    char* ws = reinterpret_cast<char*>(workspace);
    for (auto& k : jobs) {
        k.rcount = reinterpret_cast<int32_t*>(ws + reinterpret_cast<uintptr_t>(k.rcount));
        k.rkey = reinterpret_cast<int32_t*>(ws + reinterpret_cast<uintptr_t>(k.rkey));
        k.rcol = reinterpret_cast<float*>(ws + reinterpret_cast<uintptr_t>(k.rcol));
    }
    const size_t jb = ((size_t)n * sizeof(TetPartK) + 255) / 256 * 256;
    std::vector<char> tables;
    try {
        tables.assign(jb + (size_t)(n + 1) * sizeof(int32_t), 0);
    } catch (const std::bad_alloc&) {
        return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    }
    std::memcpy(tables.data(), jobs.data(), (size_t)n * sizeof(TetPartK));
    std::memcpy(tables.data() + jb, prefix.data(), (size_t)(n + 1) * sizeof(int32_t));
    f.cam = ctx->cam;
    f.tf = ctx->tf;
    f.dt = ctx->dt;
    f.parts = reinterpret_cast<const TetPartK*>(ws);
    f.tile_start = reinterpret_cast<const int32_t*>(ws + jb);
    f.n = n;
    f.total_tiles = prefix[n];
    f.max_runs = max_runs;
    f.width = ctx->cam.width;
    f.height = ctx->cam.height;
    for (int c = 0; c < 4; ++c) f.bg[c] = bg ? bg[c] : 0.0f;
    f.out = out;
    f.samples = samples;
    f.err = err_word(ctx);
    f.locator = ctx->tet_locator;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
    hipError_t e = hipSuccess;
    if (stages != kTetResolve) {
        e = stage_copy(ctx, ws, tables.data(), tables.size());
        if (e == hipErrorOutOfMemory) return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: pinned staging", who);
    }
    if (e == hipSuccess) e = launch_tet_frame(f, stages, ctx->stream);
    if (stages & kTetCount) {
        // the plan: scan the counts into slots, then read the total back
        size_t off_sums = 0;
        (void)tetplan_layout(E, &off_sums);
        long long total = 0;
        if (e == hipSuccess && E > 0)
            e = launch_exclusive_scan(f.offsets, E, reinterpret_cast<long long*>(reinterpret_cast<char*>(sh->plan) +
                                                                                   off_sums), ctx->stream);
        if (e == hipSuccess && E > 0)
            e = hipMemcpyAsync(&total, f.offsets + E, sizeof(long long), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
        try {
            ctx->tetplan.parts.assign(parts, parts + n);
        } catch (const std::bad_alloc&) {
            ctx->tetplan.plan = nullptr;
            return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
        }
        ctx->tetplan.plan = sh->plan;
        ctx->tetplan.cam = ctx->cam;
        ctx->tetplan.dt = ctx->dt;
        ctx->tetplan.entries = E;
        ctx->tetplan.total = total;
        *sh->total_out = total;
    }
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    if (stages & (kTetMarch | kTetShaded)) {
        try {
            ctx->tetmarch.parts.assign(parts, parts + n);
        } catch (const std::bad_alloc&) {
            ctx->tetmarch.ws = nullptr;
            return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
        }
        ctx->tetmarch.ws = workspace;
        ctx->tetmarch.max_runs = max_runs;
        ctx->tetmarch.cam = ctx->cam;
    }
    return ok(ctx);
}

vr_status vr_render_tetparts(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs, const float bg[4],
                             void* workspace, size_t workspace_bytes, float* out, unsigned long long* samples) {
    return tet_frame(ctx, n, parts, max_runs, bg, workspace, workspace_bytes, out, samples, kTetMarch | kTetResolve,
                     "vr_render_tetparts");
}

vr_status vr_march_tetparts(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs, void* workspace,
                            size_t workspace_bytes, unsigned long long* samples) {
    return tet_frame(ctx, n, parts, max_runs, nullptr, workspace, workspace_bytes, nullptr, samples, kTetMarch,
                     "vr_march_tetparts");
}

vr_status vr_resolve_tetparts(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs, const float bg[4],
                              void* workspace, size_t workspace_bytes, float* out) {
    return tet_frame(ctx, n, parts, max_runs, bg, workspace, workspace_bytes, out, nullptr, kTetResolve,
                     "vr_resolve_tetparts");
}

vr_status vr_tetparts_shadow_plan_size(vr_context ctx, int32_t n, const vr_tetpart* parts, size_t* bytes) {
    static const char* who = "vr_tetparts_shadow_plan_size";
    vr_status st = tetparts_check(ctx, n, parts, 1, who, false);
    if (st != VR_OK) return st;
    if (!bytes) return fail(ctx, VR_ERR_INVALID_ARG, "%s: bytes is NULL", who);
    long long E = 0;
    (void)tetframe_layout(ctx, n, parts, 1, nullptr, nullptr, &E);
    *bytes = tetplan_layout(E, nullptr);
    return ok(ctx);
}

vr_status vr_tetparts_shadow_plan(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs,
                                  void* workspace, size_t workspace_bytes, void* plan, size_t plan_bytes,
                                  int64_t* total_samples) {
    static const char* who = "vr_tetparts_shadow_plan";
    if (!total_samples) return fail(live(ctx) ? ctx : nullptr, VR_ERR_INVALID_ARG, "%s: total_samples is NULL", who);
    TetShadowArgs sh;
    sh.plan = plan;
    sh.plan_bytes = plan_bytes;
    sh.total_out = total_samples;
    return tet_frame(ctx, n, parts, max_runs, nullptr, workspace, workspace_bytes, nullptr, nullptr, kTetCount, who,
                     &sh);
}

vr_status vr_render_tetparts_shadowed(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs,
                                      const vr_light* light, const float bg[4], void* workspace,
                                      size_t workspace_bytes, void* plan, size_t plan_bytes, void* slots,
                                      size_t slot_bytes, float* out, unsigned long long* samples) {
    TetShadowArgs sh;
    sh.plan = plan;
    sh.plan_bytes = plan_bytes;
    sh.slots = slots;
    sh.slot_bytes = slot_bytes;
    sh.light = light;
    return tet_frame(ctx, n, parts, max_runs, bg, workspace, workspace_bytes, out, samples,
                     kTetRecord | kTetShadow | kTetShaded | kTetResolve, "vr_render_tetparts_shadowed", &sh);
}

vr_status vr_tetparts_slot_bytes(int64_t total_samples, size_t* bytes) {
    if (total_samples < 0 || !bytes) return fail(nullptr, VR_ERR_INVALID_ARG, "vr_tetparts_slot_bytes: bad argument");
    *bytes = tetslot_bytes(total_samples, nullptr);
    return VR_OK;
}

// ---------------------------------------------------------------- batches
// A release group: the frames [f0, f1) of a batch, the jobs that their
// partials come from (a job belongs to the group of the first frame that
// uses it; jobs no frame uses, to the last group), and its own graph: the
// group's march queues, then its composites.  vr_batch_launch replays the
// groups' graphs in order and records `done` after each.
struct BatchGroup {
    int32_t f0 = 0, f1 = 0;
    int32_t job0 = 0, n32 = 0, n16 = 0;      // table rows [job0, job0 + n32) float32, then n16 float16
    int32_t total32 = 0, total16 = 0;        // tiles of each queue
    int32_t pre32 = 0, pre16 = 0;            // first entries of the queues' tile prefixes
    int32_t cpre = 0, ctotal = 0;            // first entry of the frames' block prefix, blocks
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
};

struct vr_batch_s {
    vr_context ctx = nullptr;
    std::vector<MarchParams> jobs;        // as given
    std::vector<int32_t> f16;             // storage of each job (0 / 1)
    std::vector<const void*> brick_of;    // brick identity of each job (grouping key)
    std::vector<CompositeParams> frames;
    std::vector<int32_t> fjob0, fnjobs;   // each frame's jobs [fjob0, fjob0 + fnjobs)
    std::vector<int32_t> fblocks;         // each frame's composite blocks
    char* ws = nullptr;
    size_t off_mprefix = 0, off_mjobs = 0, off_cprefix = 0, off_cframes = 0;
    int32_t n_groups = 1;
    std::vector<BatchGroup> groups;
    int32_t wg_per_cu = 0, order = 0;
    int32_t staging = kStagingRing, tile_w = 32, chunk = 4;   // staged configuration of the tables
    uint64_t shape_key = 0;
    hipStream_t cap = nullptr;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace layout: [2 x kQueueParts counters | 256] [march prefixes (n_jobs + 2 G)] [march jobs]
// [composite prefixes (n_frames + G)] [composite frames], for up to G = max(n_frames, 1) release groups.
size_t batch_layout(int32_t n_jobs, int32_t n_frames, size_t* mp, size_t* mj, size_t* cp, size_t* cf) {
    const size_t G = (size_t)std::max(n_frames, 1);
    size_t o = 256;
    *mp = o; o = align256(o + ((size_t)n_jobs + 2 * G) * sizeof(int32_t));
    *mj = o; o = align256(o + (size_t)n_jobs * sizeof(MarchParams));
    *cp = o; o = align256(o + ((size_t)n_frames + G) * sizeof(int32_t));
    *cf = o; o = align256(o + (size_t)n_frames * sizeof(CompositeParams));
    return o;
}

void fnv(uint64_t& h, const void* p, size_t n) {
    const unsigned char* c = reinterpret_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
}

// Upload the job tables: per release group (in group order) its float32
// jobs, then its float16 jobs, each run in the given order or grouped by
// brick, with tickets of tile_w x 16 pixels; a tile prefix per queue and a
// composite-block prefix per group.  Work already enqueued on the context
// stream (an earlier launch of this batch reads the tables) finishes first.
vr_status batch_upload_tables(vr_batch b, int order, int staging, int tile_w, int chunk) {
    const int n = (int)b->jobs.size();
    const int nf = (int)b->frames.size();
    const int G = b->n_groups;
    hipError_t se = hipStreamSynchronize(b->ctx->stream);
    if (se != hipSuccess) return fail(b->ctx, VR_ERR_DEVICE, "batch upload: %s", hipGetErrorString(se));
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    if (order == 1) {   // group the jobs of each brick, bricks in order of first appearance
        std::vector<int> first(n);
        for (int i = 0; i < n; ++i) {
            first[i] = i;
            for (int j = 0; j < i; ++j)
                if (b->brick_of[j] == b->brick_of[i]) { first[i] = first[j]; break; }
        }
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return first[x] < first[y]; });
    }
    // frames of group g: [g nf / G, (g + 1) nf / G); a job's group: that of
    // the first frame using it (the last group if none does)
    std::vector<BatchGroup> gr(G);
    std::vector<int> job_group(n, G - 1);
    std::vector<char> seen(n, 0);
    for (int g = 0; g < G; ++g) {
        gr[g].f0 = (int)((long long)nf * g / G);
        gr[g].f1 = (int)((long long)nf * (g + 1) / G);
        for (int f = gr[g].f0; f < gr[g].f1; ++f)
            for (int k = 0; k < b->fnjobs[f]; ++k) {
                const int j = b->fjob0[f] + k;
                if (!seen[j]) {
                    seen[j] = 1;
                    job_group[j] = g;
                }
            }
    }
    std::vector<MarchParams> table;
    table.reserve(n);
    std::vector<int32_t> prefix;
    prefix.reserve((size_t)n + 2 * G);
    std::vector<int32_t> cprefix;
    cprefix.reserve((size_t)nf + G);
    for (int g = 0; g < G; ++g) {
        BatchGroup& q = gr[g];
        q.job0 = (int32_t)table.size();
        for (int pass = 0; pass < 2; ++pass) {
            (pass == 0 ? q.pre32 : q.pre16) = (int32_t)prefix.size();
            int cnt = 0;
            int32_t acc = 0;
            for (int k = 0; k < n; ++k) {
                const int i = idx[k];
                if (b->f16[i] != pass || job_group[i] != g) continue;
                prefix.push_back(acc);
                acc += queue_tiles(b->jobs[i].roi_w, b->jobs[i].roi_h, tile_w);
                table.push_back(b->jobs[i]);
                ++cnt;
            }
            prefix.push_back(acc);
            if (pass == 0) { q.n32 = cnt; q.total32 = acc; } else { q.n16 = cnt; q.total16 = acc; }
        }
        q.cpre = (int32_t)cprefix.size();
        int32_t acc = 0;
        for (int f = q.f0; f < q.f1; ++f) {
            cprefix.push_back(acc);
            acc += b->fblocks[f];
        }
        cprefix.push_back(acc);
        q.ctotal = acc;
    }
    hipError_t e = hipMemcpy(b->ws + b->off_mprefix, prefix.data(), prefix.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(b->ws + b->off_mjobs, table.data(), (size_t)n * sizeof(MarchParams), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->ws + b->off_cprefix, cprefix.data(), cprefix.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(b->ctx, VR_ERR_DEVICE, "batch upload: %s", hipGetErrorString(e));
    // keep the groups' events; their graphs are captured again by batch_capture
    for (int g = 0; g < G && g < (int)b->groups.size(); ++g) std::swap(gr[g].done, b->groups[g].done);
    for (auto& old : b->groups) {
        if (old.exec) (void)hipGraphExecDestroy(old.exec);
        if (old.graph) (void)hipGraphDestroy(old.graph);
        if (old.done) (void)hipEventDestroy(old.done);
    }
    b->groups = std::move(gr);
    for (auto& q : b->groups)
        if (!q.done && hipEventCreateWithFlags(&q.done, hipEventDisableTiming) != hipSuccess) {
            q.done = nullptr;
            return fail(b->ctx, VR_ERR_DEVICE, "batch upload: cannot create an event");
        }
    b->order = order;
    b->staging = staging;
    b->tile_w = tile_w;
    b->chunk = chunk;
    for (MarchParams& jp : b->jobs) {      // (single-partial fields; the queue passes its own)
        jp.staging = staging;
        jp.tile_w = tile_w;
        jp.chunk = chunk;
    }
    return VR_OK;
}

vr_status batch_upload(vr_batch b, int order, int staging, int tile_w, int chunk) {
    try {
        return batch_upload_tables(b, order, staging, tile_w, chunk);
    } catch (const std::bad_alloc&) {
        return fail(b->ctx, VR_ERR_OUT_OF_MEMORY, "batch upload: out of host memory");
    }
}

void batch_drop_graph(vr_batch b) {
    for (auto& q : b->groups) {
        if (q.exec) (void)hipGraphExecDestroy(q.exec);
        if (q.graph) (void)hipGraphDestroy(q.graph);
        q.exec = nullptr;
        q.graph = nullptr;
    }
}

// Capture each group's launches (queue counters are reset by a kernel, so a
// graph holds kernel nodes only) with `wg_per_cu` persistent workgroups per CU.
vr_status batch_capture(vr_batch b, int wg_per_cu) {
    vr_context ctx = b->ctx;
    batch_drop_graph(b);
    const MarchParams* djobs = reinterpret_cast<const MarchParams*>(b->ws + b->off_mjobs);
    const int32_t* dprefix = reinterpret_cast<const int32_t*>(b->ws + b->off_mprefix);
    const CompositeParams* dframes = reinterpret_cast<const CompositeParams*>(b->ws + b->off_cframes);
    const int32_t* dcprefix = reinterpret_cast<const int32_t*>(b->ws + b->off_cprefix);
    int32_t* heads = reinterpret_cast<int32_t*>(b->ws);
    for (auto& q : b->groups) {
        hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            batch_drop_graph(b);
            return fail(ctx, VR_ERR_DEVICE, "batch capture: %s", hipGetErrorString(e));
        }
        hipError_t le = hipSuccess;
        if (q.n32 > 0) {
            QueueParams qp{djobs + q.job0, dprefix + q.pre32, q.n32, q.total32, heads, 1,
                           b->staging, b->tile_w, b->chunk, err_word(ctx)};
            le = launch_march_queue(qp, kF32, wg_per_cu * ctx->cus, b->cap);
        }
        if (le == hipSuccess && q.n16 > 0) {
            QueueParams qp{djobs + q.job0 + q.n32, dprefix + q.pre16, q.n16, q.total16, heads + kQueueParts, 1,
                           b->staging, b->tile_w, b->chunk, err_word(ctx)};
            le = launch_march_queue(qp, kF16, wg_per_cu * ctx->cus, b->cap);
        }
        if (le == hipSuccess && q.f1 > q.f0)
            le = launch_composite_many(dframes + q.f0, dcprefix + q.cpre, q.f1 - q.f0, q.ctotal, b->cap);
        e = hipStreamEndCapture(b->cap, &q.graph);
        if (le != hipSuccess || e != hipSuccess) {
            batch_drop_graph(b);
            return fail(ctx, VR_ERR_DEVICE, "batch capture: %s", hipGetErrorString(le != hipSuccess ? le : e));
        }
        e = hipGraphInstantiate(&q.exec, q.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            batch_drop_graph(b);
            return fail(ctx, VR_ERR_DEVICE, "batch graph instantiate: %s", hipGetErrorString(e));
        }
    }
    b->wg_per_cu = wg_per_cu;
    return VR_OK;
}

// Graphs, events and the capture stream of a batch.
void batch_destroy(vr_batch b) {
    batch_drop_graph(b);
    for (auto& q : b->groups)
        if (q.done) (void)hipEventDestroy(q.done);
    b->groups.clear();
    if (b->cap) (void)hipStreamDestroy(b->cap);
    b->cap = nullptr;
}

// Replay the groups' graphs in order on `stream`, recording each group's
// event after its graph when `events` is set.
hipError_t batch_replay(vr_batch b, hipStream_t stream, bool events) {
    hipError_t e = hipSuccess;
    for (auto& q : b->groups) {
        if (e == hipSuccess) e = hipGraphLaunch(q.exec, stream);
        if (e == hipSuccess && events) e = hipEventRecord(q.done, stream);
    }
    return e;
}

int max_wg_per_cu(const vr_batch b, int staging, int tile_w, int chunk) {
    int m = 0;
    const long long n16 = std::count(b->f16.begin(), b->f16.end(), 1);
    if ((long long)b->f16.size() > n16)
        m = std::max(m, march_queue_workgroups_per_cu(kF32, true, staging, tile_w, chunk));
    if (n16 > 0) m = std::max(m, march_queue_workgroups_per_cu(kF16, true, staging, tile_w, chunk));
    return std::max(m, 1);
}

}  // namespace

vr_status vr_batch_workspace_size(int32_t n_jobs, int32_t n_frames, size_t* bytes) {
    if (n_jobs < 0 || n_frames < 0 || !bytes)
        return fail(nullptr, VR_ERR_INVALID_ARG, "vr_batch_workspace_size: bad argument");
    size_t a, b2, c, d;
    *bytes = batch_layout(n_jobs, n_frames, &a, &b2, &c, &d);
    return VR_OK;
}

static vr_status batch_create(vr_context ctx, int32_t n_cameras, const vr_camera_desc* cameras,
                              int32_t n_tfs, const vr_tf_desc* tfs, int32_t n_jobs,
                              const vr_batch_job* jobs, int32_t n_frames, const vr_batch_frame* frames,
                              void* workspace, size_t workspace_bytes, vr_batch* out) {
    static const char* who = "vr_batch_create";
    if (!live(ctx)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "%s: invalid context", who);
    if (!out) return fail(ctx, VR_ERR_INVALID_ARG, "%s: out is NULL", who);
    *out = nullptr;
    if (n_cameras < 1 || !cameras || n_tfs < 1 || !tfs || n_jobs < 0 || (n_jobs > 0 && !jobs) ||
        n_frames < 0 || (n_frames > 0 && !frames))
        return fail(ctx, VR_ERR_INVALID_ARG, "%s: bad counts or NULL arrays", who);
    size_t mp, mj, cp, cf;
    const size_t need = batch_layout(n_jobs, n_frames, &mp, &mj, &cp, &cf);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(ctx, VR_ERR_WORKSPACE, "%s: workspace of %zu bytes (256-aligned), need %zu", who,
                    workspace_bytes, need);
    std::vector<CameraK> cams(n_cameras);
    for (int i = 0; i < n_cameras; ++i) {
        vr_status st = camera_from_desc(ctx, &cameras[i], who, cams[i]);
        if (st != VR_OK) return st;
    }
    std::vector<TFK> tfk(n_tfs);
    for (int i = 0; i < n_tfs; ++i) {
        const vr_tf_desc& t = tfs[i];
        if (!t.rgba || (reinterpret_cast<uintptr_t>(t.rgba) & 15) != 0 || !std::isfinite(t.vmin) ||
            !std::isfinite(t.vmax) || !(t.vmin < t.vmax) || !(t.opacity_scale >= 0) ||
            !std::isfinite(t.opacity_scale))
            return fail(ctx, VR_ERR_INVALID_ARG, "%s: transfer function %d invalid", who, i);
        tfk[i] = TFK{t.rgba, t.vmin, t.vmax, t.opacity_scale, DPVR_TF_ENTRIES};
    }
    std::unique_ptr<vr_batch_s> b(new (std::nothrow) vr_batch_s);
    if (!b) return fail(ctx, VR_ERR_OUT_OF_MEMORY, "%s: out of host memory", who);
    b->ctx = ctx;
    uint64_t key = 1469598103934665603ull;
    for (int i = 0; i < n_jobs; ++i) {
        const vr_batch_job& j = jobs[i];
        if (j.camera < 0 || j.camera >= n_cameras || j.tf < 0 || j.tf >= n_tfs)
            return fail(ctx, VR_ERR_INVALID_ARG, "%s: job %d: camera or tf index out of range", who, i);
        if (!live(j.brick) || j.brick->ctx != ctx)
            return fail(ctx, VR_ERR_INVALID_HANDLE, "%s: job %d: invalid brick", who, i);
        if (!j.brick->has_data) return fail(ctx, VR_ERR_STATE, "%s: job %d: brick has no data", who, i);
        MarchParams p;
        vr_status st = prepare_march_with(ctx, j.brick, &j.part, cams[j.camera], tfk[j.tf], who, p);
        if (st != VR_OK) return st;
        p.tiles_x = (j.part.w + 15) / 16;
        p.tiles_y = (j.part.h + 15) / 16;
        b->jobs.push_back(p);
        b->f16.push_back(j.brick->storage == VR_F16 ? 1 : 0);
        b->brick_of.push_back(j.brick);
        const int32_t sig[8] = {j.brick->dims[0], j.brick->dims[1], j.brick->dims[2], j.part.w, j.part.h,
                                cams[j.camera].width, cams[j.camera].height, (int32_t)j.brick->storage};
        fnv(key, sig, sizeof sig);
    }
    for (int f = 0; f < n_frames; ++f) {
        const vr_batch_frame& fr = frames[f];
        if (fr.camera < 0 || fr.camera >= n_cameras || fr.first_job < 0 || fr.n_jobs < 0 ||
            fr.n_jobs > DPVR_MAX_PARTIALS || fr.first_job + fr.n_jobs > n_jobs || !fr.out ||
            (reinterpret_cast<uintptr_t>(fr.out) & 15) != 0)
            return fail(ctx, VR_ERR_INVALID_ARG, "%s: frame %d invalid", who, f);
        std::vector<vr_partial> parts(fr.n_jobs);
        for (int k = 0; k < fr.n_jobs; ++k) {
            const vr_batch_job& j = jobs[fr.first_job + k];
            if (j.camera != fr.camera)
                return fail(ctx, VR_ERR_INVALID_ARG, "%s: frame %d: job %d uses another camera", who, f,
                            fr.first_job + k);
            parts[k] = j.part;
        }
        CompositeParams cpar;
        vr_status st = prepare_composite_with(ctx, cams[fr.camera], parts.data(), fr.n_jobs, fr.bg, who, cpar);
        if (st != VR_OK) return st;
        cpar.out = fr.out;
        b->frames.push_back(cpar);
        b->fjob0.push_back(fr.first_job);
        b->fnjobs.push_back(fr.n_jobs);
        b->fblocks.push_back(composite_blocks(cams[fr.camera].width, cams[fr.camera].height));
        fnv(key, &cams[fr.camera].width, 2 * sizeof(int32_t));
    }
    int dev_id[2] = {ctx->device, ctx->cus};
    fnv(key, dev_id, sizeof dev_id);
    b->shape_key = key;
    b->ws = reinterpret_cast<char*>(workspace);
    b->off_mprefix = mp;
    b->off_mjobs = mj;
    b->off_cprefix = cp;
    b->off_cframes = cf;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "%s: cannot select device %d", who, ctx->device);
    hipError_t e = hipSuccess;
    if (n_frames > 0)
        e = hipMemcpy(b->ws + cf, b->frames.data(), b->frames.size() * sizeof(CompositeParams),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
    // until tuned, the context's configuration of the storage with more jobs
    const long long n16 = std::count(b->f16.begin(), b->f16.end(), 1);
    const MarchCfg& mc = ctx->cfg[n16 > (long long)b->f16.size() - n16 ? 1 : 0];
    vr_status st = batch_upload(b.get(), 0, mc.staging, mc.tile_w, mc.chunk);
    if (st == VR_OK) st = batch_capture(b.get(), max_wg_per_cu(b.get(), mc.staging, mc.tile_w, mc.chunk));
    if (st != VR_OK) {
        batch_destroy(b.get());
        return st;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(b.get());
    }
    ctx->live_bricks++;   // a batch pins the context like a brick does
    *out = b.release();
    return ok(ctx);
}

vr_status vr_batch_create(vr_context ctx, int32_t n_cameras, const vr_camera_desc* cameras,
                          int32_t n_tfs, const vr_tf_desc* tfs, int32_t n_jobs,
                          const vr_batch_job* jobs, int32_t n_frames, const vr_batch_frame* frames,
                          void* workspace, size_t workspace_bytes, vr_batch* out) {
    try {
        return batch_create(ctx, n_cameras, cameras, n_tfs, tfs, n_jobs, jobs, n_frames, frames, workspace,
                            workspace_bytes, out);
    } catch (const std::bad_alloc&) {
        return fail(live(ctx) ? ctx : nullptr, VR_ERR_OUT_OF_MEMORY, "vr_batch_create: out of host memory");
    }
}

vr_status vr_batch_launch(vr_batch b) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_batch_launch: invalid batch");
    vr_context ctx = b->ctx;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_batch_launch: cannot select device %d", ctx->device);
    hipError_t e = batch_replay(b, ctx->stream, true);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_batch_launch: %s", hipGetErrorString(e));
    return ok(ctx);
}

vr_status vr_batch_set_groups(vr_batch b, int32_t n_groups) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_batch_set_groups: invalid batch");
    vr_context ctx = b->ctx;
    if (n_groups < 1 || n_groups > std::max((int32_t)b->frames.size(), 1))
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_batch_set_groups: n_groups must be in [1, %d]",
                    std::max((int32_t)b->frames.size(), 1));
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_batch_set_groups: cannot select device %d", ctx->device);
    b->n_groups = n_groups;
    vr_status st = batch_upload(b, b->order, b->staging, b->tile_w, b->chunk);
    if (st == VR_OK) st = batch_capture(b, b->wg_per_cu);
    return st == VR_OK ? ok(ctx) : st;
}

vr_status vr_batch_group(vr_batch b, int32_t group, int32_t* first_frame, int32_t* n_frames) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_batch_group: invalid batch");
    if (group < 0 || group >= (int32_t)b->groups.size())
        return fail(b->ctx, VR_ERR_INVALID_ARG, "vr_batch_group: group %d out of range", group);
    if (first_frame) *first_frame = b->groups[group].f0;
    if (n_frames) *n_frames = b->groups[group].f1 - b->groups[group].f0;
    return ok(b->ctx);
}

vr_status vr_batch_wait_group(vr_batch b, int32_t group, void* stream) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_batch_wait_group: invalid batch");
    vr_context ctx = b->ctx;
    if (group < 0 || group >= (int32_t)b->groups.size())
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_batch_wait_group: group %d out of range", group);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_batch_wait_group: cannot select device %d", ctx->device);
    const hipError_t e = stream ? hipStreamWaitEvent(reinterpret_cast<hipStream_t>(stream), b->groups[group].done, 0)
                                : hipEventSynchronize(b->groups[group].done);
    if (e != hipSuccess) return fail(ctx, VR_ERR_DEVICE, "vr_batch_wait_group: %s", hipGetErrorString(e));
    return ok(ctx);
}

vr_status vr_batch_group_done(vr_batch b, int32_t group, int32_t* done) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_batch_group_done: invalid batch");
    vr_context ctx = b->ctx;
    if (group < 0 || group >= (int32_t)b->groups.size() || !done)
        return fail(ctx, VR_ERR_INVALID_ARG, "vr_batch_group_done: group %d out of range or done is NULL", group);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_batch_group_done: cannot select device %d", ctx->device);
    const hipError_t e = hipEventQuery(b->groups[group].done);
    if (e != hipSuccess && e != hipErrorNotReady)
        return fail(ctx, VR_ERR_DEVICE, "vr_batch_group_done: %s", hipGetErrorString(e));
    *done = e == hipSuccess ? 1 : 0;
    return ok(ctx);
}

vr_status vr_batch_config(vr_batch b, int32_t* wg_per_cu, int32_t* order, int32_t* staging,
                          int32_t* tile_width, int32_t* chunk_slices) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_batch_config: invalid batch");
    if (wg_per_cu) *wg_per_cu = b->wg_per_cu;
    if (order) *order = b->order;
    if (staging) *staging = b->staging == kStagingSlab ? VR_STAGING_SLAB : VR_STAGING_RING;
    if (tile_width) *tile_width = b->tile_w;
    if (chunk_slices) *chunk_slices = b->chunk;
    return ok(b->ctx);
}

namespace {

struct TuneChoice {
    int wg, order, staging, tile_w, chunk;
};

// Staged configurations the autotuner times: slab, and ring with 16- or
// 32-pixel tiles and 4- or 8-slice chunks.
constexpr int kTuneConfigs[5][3] = {
    {kStagingSlab, 16, 4}, {kStagingRing, 16, 4}, {kStagingRing, 16, 8}, {kStagingRing, 32, 4}, {kStagingRing, 32, 8}};

// Autotuner cache: one line per tuned batch shape,
// "key wg order staging tile chunk ms".
bool cache_lookup(const char* path, uint64_t key, TuneChoice* c) {
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        unsigned long long k;
        TuneChoice t;
        double ms;
        if (std::sscanf(line, "%llx %d %d %d %d %d %lf", &k, &t.wg, &t.order, &t.staging, &t.tile_w, &t.chunk,
                        &ms) == 7 &&
            k == key) {
            *c = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, uint64_t key, const TuneChoice& c, double ms) {
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%llx %d %d %d %d %d %.6f\n", (unsigned long long)key, c.wg, c.order, c.staging, c.tile_w,
                 c.chunk, ms);
    std::fclose(f);
}

bool choice_valid(const vr_batch b, const TuneChoice& c) {
    return valid_march_config(c.staging, c.tile_w, c.chunk) && (c.order == 0 || c.order == 1) && c.wg >= 1 &&
           c.wg <= max_wg_per_cu(b, c.staging, c.tile_w, c.chunk);
}

vr_status apply_choice(vr_batch b, const TuneChoice& c) {
    vr_status st = batch_upload(b, c.order, c.staging, c.tile_w, c.chunk);
    if (st == VR_OK) st = batch_capture(b, c.wg);
    return st;
}

}  // namespace

vr_status vr_batch_autotune(vr_batch b, int32_t reps, double* best_ms) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_batch_autotune: invalid batch");
    vr_context ctx = b->ctx;
    if (reps < 1) return fail(ctx, VR_ERR_INVALID_ARG, "vr_batch_autotune: reps must be >= 1");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, VR_ERR_DEVICE, "vr_batch_autotune: cannot select device %d", ctx->device);
    const char* path = std::getenv("DPVR_AUTOTUNE_CACHE");
    TuneChoice cached{};
    if (cache_lookup(path, b->shape_key, &cached) && choice_valid(b, cached)) {
        vr_status st = apply_choice(b, cached);
        if (best_ms) *best_ms = -1.0;   // taken from the cache, not timed
        return st == VR_OK ? ok(ctx) : st;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ctx, VR_ERR_DEVICE, "vr_batch_autotune: cannot create events");
    double best = 1e300;
    TuneChoice bc{b->wg_per_cu, b->order, b->staging, b->tile_w, b->chunk};
    vr_status st = VR_OK;
    // candidates: staged configuration x job order x persistent workgroups per CU
    for (const auto& cfg : kTuneConfigs) {
        for (int order = 0; order < 2 && st == VR_OK; ++order) {
            st = batch_upload(b, order, cfg[0], cfg[1], cfg[2]);
            const int maxwg = max_wg_per_cu(b, cfg[0], cfg[1], cfg[2]);
            for (int wg = 1; wg <= maxwg && st == VR_OK; ++wg) {
                st = batch_capture(b, wg);
                if (st != VR_OK) break;
                hipError_t e = batch_replay(b, ctx->stream, false);   // warm-up
                if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
                for (int r = 0; r < reps && e == hipSuccess; ++r) e = batch_replay(b, ctx->stream, false);
                if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    st = fail(ctx, VR_ERR_DEVICE, "vr_batch_autotune: %s", hipGetErrorString(e));
                    break;
                }
                const double per = ms / reps;
                if (per < best) {
                    best = per;
                    bc = TuneChoice{wg, order, cfg[0], cfg[1], cfg[2]};
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != VR_OK) return st;
    st = apply_choice(b, bc);
    if (st != VR_OK) return st;
    cache_store(path, b->shape_key, bc, best);
    if (best_ms) *best_ms = best;
    return ok(ctx);
}

vr_status vr_batch_release(vr_batch b) {
    if (!live(b)) return fail(nullptr, VR_ERR_INVALID_HANDLE, "vr_batch_release: invalid batch");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.erase(b);
    }
    batch_destroy(b);
    if (live(b->ctx)) b->ctx->live_bricks--;
    delete b;
    return VR_OK;
}

}  // extern "C"
