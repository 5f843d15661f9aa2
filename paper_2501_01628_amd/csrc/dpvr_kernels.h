// Internal interface between the host-side C-ABI (api.cpp) and the HIP
// kernels (*.hip).  Plain structs passed to kernels by value.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace dpvr {

// Camera frame, float64 (computed once per frame on the host).  Pixel (i, j)
// maps to sx = 2 (i + 1/2) / W - 1, sy = 1 - 2 (j + 1/2) / H and
//   perspective:  o = eye, d = normalize(f + (sx ax) r + (sy ay) u)
//   orthographic: o = eye + (sx ax) r + (sy ay) u, d = f
struct CameraK {
    double eye[3], f[3], r[3], u[3];
    double ax, ay;
    int32_t kind;          // 0 perspective, 1 orthographic
    int32_t width, height;
    int32_t pad_;
};

// A brick as the kernels see it.
struct BrickK {
    const void* data;      // stored voxels (with ghost layer), x fastest
    int32_t sdim[3];       // stored extents (owned + 2 ghost) in x, y, z
    int32_t ghost;
    double lo[3], hi[3];   // owned world box [lo, hi)
    double origin[3];      // == lo
    double spacing[3];
    double inv_spacing[3]; // 1 / spacing
};

struct TFK {
    const float* rgba;     // 256 x 4, device
    float vmin, vmax, opacity_scale;
    int32_t n;
};

struct MarchParams {
    CameraK cam;
    BrickK brick;
    TFK tf;
    double dt;
    double inv_dt;         // 1 / dt
    float ert_eps;
    int32_t roi_x0, roi_y0, roi_w, roi_h;
    int32_t tiles_x, tiles_y;
    float* out_rgba;       // roi_h x roi_w x 4
    float* out_depth;      // roi_h x roi_w
    unsigned long long* samples;  // optional evaluated-sample counter
    // checkpoints of the transmittance (adjoint support): when ckpt != NULL
    // the forward writes, and the backward reads, T in front of every
    // ckpt_interval-th owned sample, ckpt_nseg slots per ROI pixel
    float* ckpt;
    int32_t ckpt_interval;
    int32_t ckpt_nseg;
    int32_t path;          // kPathStaged or kPathDirect (bit-identical results)
    int32_t staging;       // staged path: kStagingSlab or kStagingRing
    int32_t tile_w;        // staged path: tile width in pixels (slab: 16; ring: 16 or 32; 16 rows)
    int32_t chunk;         // staged ring: slices per chunk of the walk (4 or 8)
    int32_t* err;          // device error word: a kernel guard that trips ORs a bit in (may be NULL)
};

enum : int32_t { kPathStaged = 0, kPathDirect = 1 };
// Staged-march families: slab (all waves stage a slab, then all march it)
// and ring (a producer wave streams slices ahead of the marching waves).
enum : int32_t { kStagingSlab = 0, kStagingRing = 1 };

// A device work queue of march jobs (partial images): tickets
// tile_start[j] .. tile_start[j + 1] - 1 are the tiles of job j (tile_w x 16
// pixels when staged, 16 x 16 when direct).
struct QueueParams {
    const MarchParams* jobs;   // device, n_jobs entries
    const int32_t* tile_start; // device, n_jobs + 1 entries (exclusive prefix of tiles)
    int32_t n_jobs;
    int32_t total_tiles;
    int32_t* head;             // device, kQueueParts ticket counters (reset by the launcher)
    int32_t staged;            // 1: LDS-staged tiles, 0: every lane marches from HBM
    int32_t staging;           // kStagingSlab or kStagingRing
    int32_t tile_w;            // staged tile width (16, or 32 for the ring)
    int32_t chunk;             // staged chunk length in slices (4 or 8)
    int32_t* err;              // device error word (see MarchParams::err)
};

// Error bits of the device error word, which sits at byte kErrWordOffset of
// the library's static scratch array of each device (zero at load).
enum : int32_t { kErrSpin = 1, kErrRange = 2 };   // kErrRuns = 4: tet_kernels.h
constexpr size_t kErrWordOffset = 128;

// Launch-configuration knobs of the staged march.
constexpr int kTileWidths[2] = {16, 32};
constexpr int kChunks[2] = {4, 8};

// The tickets are split into kQueueParts contiguous parts, one per XCD
// (workgroup i runs on XCD i mod 8): a workgroup drains its own XCD's part
// first, so neighbouring tiles (which share voxels) meet in one L2, and then
// helps with the other parts in turn.
constexpr int kQueueParts = 8;

// Tickets of a w x h ROI with tiles tile_w pixels wide and 16 rows high.
inline int32_t queue_tiles(int32_t w, int32_t h, int32_t tile_w) {
    return ((w + tile_w - 1) / tile_w) * ((h + 15) / 16);
}

constexpr int kMaxCkptInterval = 64;

struct BackwardParams {
    const float* d_part;   // roi_h x roi_w x 4: dL/dC_rgb, dL/dA
    float* grad_tf;        // 256 x 4, accumulated (table units: raw alpha)
    float* grad_vox;       // global voxel array, accumulated
    int32_t vol_dims[3];   // global voxel grid (nx, ny, nz)
    int32_t lo[3];         // global index of the brick's owned min corner
};

constexpr int kMaxPartials = 64;

struct PartialK {
    int32_t x0, y0, w, h;
    const float* rgba;
    const float* depth;
};

struct CompositeParams {
    PartialK parts[kMaxPartials];
    int32_t n;
    int32_t width, height;
    int32_t tiles_x;
    float bg[4];
    float* out;
};

// Backward of the composite: upstream dL/d(frame) and one ROI-sized output
// buffer (h x w x 4) per partial.
struct CompositeBackParams {
    const float* d_out;
    float* d_parts[kMaxPartials];
};

// Ingest from a global voxel array: gather the brick's ghost-padded box
// (clamped to the grid) into its workspace.
struct GatherParams {
    const float* volume;
    int32_t vol_dims[3];
    int32_t lo[3];         // owned min corner, global index
    int32_t sdim[3];       // stored extents (owned + 2 ghost)
    int32_t ghost;
};

enum StorageK : int32_t { kF32 = 0, kF16 = 1 };

// Library-owned scratch of vr_render_partials_static (static_scratch.hip):
// the frame workspace layout of vr_render_partials for up to
// kStaticMaxPartials partials -- queue counters (256 B), tile prefix
// (n + 2 int32, 256-aligned), job table (n MarchParams, 256-aligned).
constexpr int kStaticMaxPartials = 64;
constexpr size_t kStaticScratchBytes =
    256 + (((size_t)(kStaticMaxPartials + 2) * sizeof(int32_t) + 255) / 256) * 256 +
    (((size_t)kStaticMaxPartials * sizeof(MarchParams) + 255) / 256) * 256;
// Device address of this GPU's scratch array (call with the device current).
hipError_t static_scratch_address(void** out);

// Launchers (return the hipError_t of the launch).
hipError_t launch_ingest(const float* src, void* dst, const int32_t sdim[3], StorageK storage,
                         hipStream_t stream);
hipError_t launch_march(const MarchParams& p, StorageK storage, hipStream_t stream);
hipError_t launch_march_queue(const QueueParams& q, StorageK storage, int workgroups,
                              hipStream_t stream);
// Resident workgroups per CU of the persistent march for this configuration.
int march_queue_workgroups_per_cu(StorageK storage, bool staged, int staging, int tile_w, int chunk);
// A valid staged configuration: slab with 16-pixel tiles, or ring with 16- or
// 32-pixel tiles and chunks of 4 or 8 slices.
inline bool valid_march_config(int staging, int tile_w, int chunk) {
    if (staging == kStagingSlab) return tile_w == 16;
    return staging == kStagingRing && (tile_w == 16 || tile_w == 32) && (chunk == 4 || chunk == 8);
}
hipError_t launch_composite(const CompositeParams& p, hipStream_t stream);
hipError_t launch_composite_many(const CompositeParams* frames, const int32_t* block_start,
                                 int32_t n_frames, int32_t total_blocks, hipStream_t stream);
// Workgroups of the forward composite of a w x h frame (64 x 4 pixel blocks).
inline int32_t composite_blocks(int32_t w, int32_t h) { return ((w + 63) / 64) * ((h + 3) / 4); }
hipError_t launch_march_backward(const MarchParams& p, const BackwardParams& bp, StorageK storage,
                                 hipStream_t stream);
// The adjoint of many partials in one launch (one storage precision): job j's
// tiles are taken backward_many_waves() per workgroup, workgroups
// block_start[j] .. block_start[j + 1] - 1.
struct BackwardJob {
    MarchParams p;
    BackwardParams bp;
};
int backward_many_waves();
// The checkpointed forward of many partials in one launch (one storage
// precision): job j's 8x8 tiles are workgroups tile_start[j] .. tile_start[j + 1] - 1.
hipError_t launch_march_checkpointed_many(const MarchParams* jobs, const int32_t* tile_start, int32_t n_jobs,
                                          int32_t total_tiles, StorageK storage, hipStream_t stream);
hipError_t launch_march_backward_many(const BackwardJob* jobs, const int32_t* block_start, int32_t n_jobs,
                                      int32_t total_blocks, StorageK storage, hipStream_t stream);
hipError_t launch_composite_backward(const CompositeParams& p, const CompositeBackParams& bp,
                                     hipStream_t stream);
hipError_t launch_gather(const GatherParams& g, void* dst, StorageK storage, hipStream_t stream);

// Ray-queue cycling (rqc.hip): bricks as ranks, one directional light.
struct RqcBrick {
    BrickK brick;
    int32_t roi_x0, roi_y0, roi_w, roi_h;   // pixels whose rays can own samples of the brick
    long long entry0;                       // first plan entry of the brick (its ROI pixels, row-major)
    int32_t storage;                        // kF32 / kF16
    int32_t pad_;
};

struct RqcParams {
    CameraK cam;
    TFK tf;
    double dt, inv_dt;
    double light[3];            // unit direction toward the light
    float ert_eps;
    float ambient;              // a0: emission scaled by a0 + (1 - a0) S
    int32_t shadows;            // 0: a0 = 1, no shadow rays traced
    int32_t n;                  // bricks (ranks)
    int32_t step;               // cycle step of a step launch
    int32_t width, height;
    const RqcBrick* bricks;     // device, n
    long long n_entries;        // sum of ROI pixels over the bricks
    int32_t* kf;                // per entry: first owned sample index (-1: none)
    long long* offsets;         // per entry: first sample slot; offsets[n_entries] = total
    long long total;            // owned primary samples (shadow rays)
    float* shade;               // per slot: shadow transmittance
    float* segs;                // per pixel: n x (key, C_r, C_g, C_b, alpha)
    float* out;                 // height x width x 4
    float bg[4];
    unsigned long long* samples;  // optional: += primary and shadow samples evaluated
    int32_t* err;               // device error word
};

hipError_t launch_rqc_plan(const RqcParams& p, long long* scan_sums, long long* total, hipStream_t stream);
long long rqc_scan_blocks(long long n_entries);
hipError_t launch_rqc_frame(RqcParams p, int cus, hipStream_t stream);

// Exclusive scan of v[0 .. n) in place, v[n] = total (sums: scan_blocks(n) + 1 entries).
hipError_t launch_exclusive_scan(long long* v, long long n, long long* sums, hipStream_t stream);
long long scan_blocks(long long n);

}  // namespace dpvr
