/*
 * dpvr.h -- C-ABI of the MI355X data-parallel volume renderer.
 *
 * The library renders a volume that is split into bricks (the "ranks" of a
 * data-parallel decomposition, several of which can live on one GPU): each
 * brick is ray cast on its own into a partial image (premultiplied RGBA plus
 * a depth key), and the partial images are then combined by sort-last,
 * visibility-ordered compositing.  The call set follows the paper's
 * ANARI-style problem statement (Zellmann, "Data Parallel Visualization and
 * Rendering on the RAMSES Supercomputer with ANARI", Sec. 3): the
 * application describes the scene (bricks = the locally owned part of the
 * world, a transfer function, a camera), calls render, and finds the image
 * in memory it owns; rendering a partial image is the per-rank local step,
 * compositing is the step that runs as a collective across ranks and leaves
 * the framebuffer with the main rank (Sec. 3, DP-ANARI conventions).
 *
 * Conventions for every call
 *   - Device memory is always owned by the caller.  The library allocates no
 *     device memory: bricks live in caller-provided workspaces, partial and
 *     final images in caller-provided buffers.  Pointers are borrowed for the
 *     duration of the work the call enqueues.  (One exception:
 *     vr_render_partials_static keeps its tables in a small static device
 *     array of the library.)
 *   - Work is enqueued asynchronously on the context's HIP stream; nothing
 *     returns to the host until the caller synchronises (vr_synchronize or
 *     its own stream/device synchronisation).
 *   - Every call returns a vr_status.  Arguments are validated on the host
 *     before anything is enqueued; an invalid call enqueues nothing.
 *     Asynchronous device faults surface as VR_ERR_DEVICE at the next call
 *     that checks the HIP runtime (vr_synchronize always does).
 *     vr_last_error() returns a message for the last failing call.
 *   - A context is not thread-safe; separate contexts are independent.
 *
 * Optical model (cited per call below; all readings of the paper, which
 * gives no rendering mathematics):
 *   grid     voxel (i, j, k) of a brick is a cell centred at
 *            origin + spacing * (i + 1/2, j + 1/2, k + 1/2); a brick owns the
 *            half-open box [origin, origin + dims * spacing) per axis and
 *            stores one ghost layer (copies of the neighbours' voxels, or of
 *            its own edge voxels at the domain boundary) on every face.
 *   lattice  along each camera ray (origin o, unit direction d) samples sit
 *            at t_k = (k + 1/2) dt, k = 0, 1, ...; sample k is evaluated by
 *            the brick whose owned box contains o + t_k d, so the sample set
 *            does not depend on how the volume is split.
 *   sample   trilinear interpolation of the stored voxels.
 *   classify 256-entry RGBA table over [vmin, vmax], endpoint aligned,
 *            piecewise linear; extinction sigma = opacity_scale * alpha.
 *   shade    emission-absorption front to back: a = 1 - exp(-sigma dt),
 *            C += T a rgb, T *= 1 - a (premultiplied colour, alpha 1 - T).
 *   depth    the partial's depth key is t of the first sample the brick
 *            owns on that ray (+inf if it owns none).
 *   over     partials are combined per pixel in ascending key order,
 *            C += (1 - A) C_i, A += (1 - A) A_i, then put over a background.
 */
#ifndef DPVR_H
#define DPVR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPVR_ABI_VERSION 2
#define DPVR_TF_ENTRIES 256          /* transfer-function table size */
#define DPVR_MAX_PARTIALS 64         /* partials per vr_composite call */

typedef struct vr_context_s* vr_context;
typedef struct vr_brick_s* vr_brick;

typedef enum {
    VR_OK = 0,
    VR_ERR_INVALID_ARG = -1,     /* argument out of range or inconsistent */
    VR_ERR_INVALID_HANDLE = -2,  /* NULL or released handle */
    VR_ERR_WORKSPACE = -3,       /* caller workspace too small or misaligned */
    VR_ERR_UNSUPPORTED = -4,     /* valid request the library does not implement */
    VR_ERR_DEVICE = -5,          /* HIP runtime error (launch or asynchronous fault) */
    VR_ERR_STATE = -6,           /* required state (camera, transfer function) not set */
    VR_ERR_OUT_OF_MEMORY = -7    /* a host (or pinned host) allocation of the library failed */
} vr_status;

/* Storage precision of a brick's internal copy.  VR_F16 stores IEEE
 * binary16 (round to nearest even) and reconstructs in FP32; accumulation is
 * FP32 either way. */
typedef enum { VR_F32 = 0, VR_F16 = 1 } vr_dtype;

/* A partial image: a region of interest (ROI) of the frame, in pixels, and
 * caller-owned device buffers for it.  rgba holds h * w * 4 floats
 * (premultiplied r, g, b, alpha), row-major with row 0 at the top; depth
 * holds h * w floats (the depth key, +inf where the brick owns no sample).
 * Pixels of the frame outside the ROI count as (0, 0, 0, 0) at depth +inf.
 * samples is optional (NULL = off): a device counter to which a render call
 * adds the number of samples it evaluated (owned samples up to and including
 * the one at which early termination stopped the ray); the caller zeroes it. */
typedef struct {
    int32_t x0, y0, w, h;
    float* rgba;
    float* depth;
    unsigned long long* samples;
} vr_partial;

/* ------------------------------------------------------------------ misc */
/* Returns DPVR_ABI_VERSION of the loaded library. */
int32_t vr_abi_version(void);

/* Static English name of a status code (never NULL). */
const char* vr_status_string(vr_status status);

/* Message of the last failing call on ctx; with ctx == NULL, of the last
 * failing call on this thread that had no usable context (e.g. a failed
 * vr_context_create).  Valid until the next call on the same context /
 * thread.  Never NULL (empty string when there was no error). */
const char* vr_last_error(vr_context ctx);

/* --------------------------------------------------------------- context */
/* Create a context bound to HIP device `device` and HIP stream `stream`
 * (a hipStream_t; NULL = the device's default stream).  The stream is
 * borrowed: the caller keeps it alive for the context's lifetime.
 * Errors: VR_ERR_INVALID_ARG (out == NULL, bad device), VR_ERR_DEVICE. */
vr_status vr_context_create(int32_t device, void* stream, vr_context* out);

/* Release a context.  Bricks created on it must be released first
 * (VR_ERR_STATE otherwise).  Does not synchronise the stream. */
vr_status vr_context_release(vr_context ctx);

/* Re-bind the context to another stream of the same device. */
vr_status vr_context_set_stream(vr_context ctx, void* stream);

/* Block until all work enqueued on the context's stream has finished and
 * report any asynchronous device error (VR_ERR_DEVICE).  This includes the
 * device's error word: the staged march bounds every wait between the
 * wavefronts of a workgroup, and a wait that times out (which only a logic
 * error could cause) ends the launch early and sets the word instead of
 * hanging the GPU; the word is per device, so the next vr_synchronize of any
 * context on that device reports it (and clears it). */
vr_status vr_synchronize(vr_context ctx);

/* ---------------------------------------------------------------- bricks */
/* Bytes of device workspace a brick of `dims` owned voxels (nx, ny, nz, each
 * >= 1) with `ghost` ghost layers (must be 1) needs at precision `storage`:
 * the ghost-padded voxels with rows padded to a multiple of 8 elements.
 * Host-only; needs no context.  Errors: VR_ERR_INVALID_ARG; VR_ERR_UNSUPPORTED
 * when the padded brick holds 2^31 or more voxels (kernels use 32-bit
 * element offsets within a brick). */
vr_status vr_brick_workspace_size(const int32_t dims[3], int32_t ghost, vr_dtype storage,
                                  size_t* bytes);

/* Create a brick: the part of the world one rank owns (paper Sec. 2.2:
 * the data is spatially distributed, each rank owning a share; Sec. 3:
 * world updates are local).  dims = owned voxels (nx, ny, nz); ghost = 1;
 * origin = world position of the owned box's min corner; spacing = world
 * size of a voxel (> 0, finite); storage = internal precision.  workspace is
 * a caller-owned device buffer of at least vr_brick_workspace_size() bytes,
 * 256-byte aligned, that must outlive the brick.  The brick has no voxel
 * data until vr_brick_set_data() is called.
 * Errors: VR_ERR_INVALID_HANDLE, VR_ERR_INVALID_ARG, VR_ERR_WORKSPACE. */
vr_status vr_brick_create(vr_context ctx, const int32_t dims[3], int32_t ghost,
                          const double origin[3], const double spacing[3], vr_dtype storage,
                          void* workspace, size_t workspace_bytes, vr_brick* out);

/* Ingest voxel values (a new time step or field): voxels is a device array of
 * (nz + 2g) * (ny + 2g) * (nx + 2g) floats, x fastest, including the ghost
 * layer.  The values are converted into the brick's workspace by a kernel
 * enqueued on the context stream; `voxels` is borrowed until that kernel has
 * run (the next synchronisation of the stream).  FP16 storage rounds to
 * nearest even; values beyond the binary16 range become +-inf. */
vr_status vr_brick_set_data(vr_brick brick, const float* voxels);

/* Ingest the brick's data straight out of a global voxel array: volume is a
 * device array of vol_dims = (NX, NY, NZ) floats, x fastest; lo = global
 * index of the brick's owned min corner.  The brick's box plus its ghost
 * layer is gathered, with indices clamped to the grid (so ghosts at the
 * domain boundary replicate the edge voxel), into the workspace at the
 * brick's storage precision.  `volume` is borrowed until the enqueued kernel
 * has run.  Errors: VR_ERR_INVALID_ARG (box outside the grid). */
vr_status vr_brick_set_data_global(vr_brick brick, const float* volume, const int32_t vol_dims[3],
                                   const int32_t lo[3]);

/* Release a brick (host state only; the caller frees the workspace). */
vr_status vr_brick_release(vr_brick brick);

/* ----------------------------------------------------------------- state */
/* Transfer function (classification): rgba is a device array of n = 256
 * entries (r, g, b, alpha) as floats, colour non-premultiplied, alpha >= 0.
 * Entry i sits at value vmin + i (vmax - vmin) / 255; values in between are
 * linearly interpolated, values outside [vmin, vmax] clamp to the end
 * entries.  Extinction per world unit is opacity_scale * alpha.  The table is
 * read by render calls enqueued after this call: it is borrowed until they
 * have run.  Errors: VR_ERR_INVALID_ARG (n != 256, vmin >= vmax, non-finite
 * values, opacity_scale < 0). */
vr_status vr_set_transfer_function(vr_context ctx, const float* rgba, int32_t n, float vmin,
                                   float vmax, float opacity_scale);

/* Pinhole camera: forward f = normalize(target - eye), right r =
 * normalize(f x up), true up u = r x f; pixel (i, j) (row 0 at the top)
 * casts o = eye, d = normalize(f + x r + y u) with
 * x = (2 (i + 1/2) / width - 1) tan(fovy / 2) width / height,
 * y = (1 - 2 (j + 1/2) / height) tan(fovy / 2).  fovy in (0, 180) degrees.
 * Errors: VR_ERR_INVALID_ARG (degenerate frame: eye == target, up parallel
 * to the view direction, non-finite values, size < 1). */
vr_status vr_set_camera_perspective(vr_context ctx, const double eye[3], const double target[3],
                                    const double up[3], double fovy_deg, int32_t width,
                                    int32_t height);

/* Orthographic camera: d = normalize(dir); pixel (i, j) casts from
 * o = pos + x r + y u with x, y as above but scaled so that the image is
 * view_height world units tall (pos is the image centre). */
vr_status vr_set_camera_orthographic(vr_context ctx, const double pos[3], const double dir[3],
                                     const double up[3], double view_height, int32_t width,
                                     int32_t height);

/* Sample spacing dt along each ray in world units (> 0; the samples sit at
 * (k + 1/2) dt from the ray origin), and the early-termination threshold: a
 * ray stops once its transmittance drops below ert_epsilon (0 disables; the
 * neglected remainder is at most ert_epsilon per channel; the test is made
 * after every second sample of the ray, so a ray may take one sample past the
 * threshold).  Defaults: dt = 0.5, ert_epsilon = 2^-20. */
vr_status vr_set_render_params(vr_context ctx, double dt, float ert_epsilon);

/* Launch path of the forward march; every path computes bit-identical
 * images (the sample positions and values do not depend on it):
 *   VR_PATH_STAGED  a workgroup per 16x16 pixel tile stages each slab of
 *                   brick slices its rays cross through LDS (default);
 *   VR_PATH_DIRECT  every lane reads its voxels from HBM (vr_render_partials:
 *                   the same persistent work queue; vr_render_partial: one
 *                   wavefront per 8x8 tile). */
typedef enum { VR_PATH_STAGED = 0, VR_PATH_DIRECT = 1 } vr_path;
vr_status vr_set_march_path(vr_context ctx, vr_path path);

/* Launch shape of the staged path for bricks of one storage precision
 * (results are bit-identical for every choice).  Two families stage brick
 * data in LDS:
 *   VR_STAGING_SLAB  a 16x16-pixel tile per 256-thread workgroup; per slab of
 *                    16 brick slices every wavefront first stages its share of
 *                    the slab, then marches (two workgroups per CU overlap);
 *                    tile_width must be 16, chunk_slices is ignored;
 *   VR_STAGING_RING  a tile_width x 16 tile (16 or 32) per workgroup with one
 *                    marching wavefront per 8x8 quarter and one wavefront that
 *                    streams brick slices into an LDS ring ahead of them
 *                    (direct LDS loads); chunk_slices = 4 or 8 slices marched
 *                    between two synchronisations of a wavefront with the
 *                    streaming wavefront (about 2.9 samples per slice at step
 *                    0.5 along the slab axis).
 * Defaults: VR_F32 bricks ring, 32, 4; VR_F16 bricks slab (the fastest
 * measured for each on a 1920x1080 frame of 16 bricks).  A batch takes the
 * configuration of the storage most of its jobs use until it is tuned.
 * Errors: VR_ERR_INVALID_ARG. */
typedef enum { VR_STAGING_SLAB = 0, VR_STAGING_RING = 1 } vr_staging;
vr_status vr_set_march_config(vr_context ctx, vr_dtype storage, vr_staging staging, int32_t tile_width,
                              int32_t chunk_slices);

/* --------------------------------------------------------------- render */
/* Host-only: the smallest pixel rectangle of the current camera's frame that
 * holds every pixel whose ray can own a sample of `brick` (its owned box
 * projected to the image, plus one pixel of margin), clipped to the frame;
 * the whole frame when the eye is inside or behind the box's projection
 * plane.  roi = (x0, y0, w, h); w or h may be 0 when the box is off-screen.
 * Errors: VR_ERR_STATE (no camera). */
vr_status vr_partial_roi(vr_context ctx, vr_brick brick, int32_t roi[4]);

/* Render the partial image of one brick (paper Sec. 2.2: each rank traces
 * the rays through the data it owns) into part->rgba / part->depth for the
 * pixels of part's ROI.  The ROI must lie within the frame; rays of pixels
 * outside it are not cast.  Enqueued on the context stream.
 * Errors: VR_ERR_INVALID_HANDLE, VR_ERR_INVALID_ARG (ROI, NULL buffers),
 * VR_ERR_STATE (no camera, no transfer function, brick has no data),
 * VR_ERR_DEVICE. */
vr_status vr_render_partial(vr_context ctx, vr_brick brick, const vr_partial* part);

/* Device workspace vr_render_partials needs for n partials (a job table and
 * a work-queue counter).  Host-only.  Errors: VR_ERR_INVALID_ARG (n < 0). */
vr_status vr_frame_workspace_size(int32_t n, size_t* bytes);

/* Render the partial images of n bricks in one persistent launch (per
 * storage precision): the tiles (16 rows by 16 or 32 pixels) of all n ROIs form one device work
 * queue, so bricks that are small on screen still fill the GPU.  Results are
 * bit-identical to n calls of vr_render_partial.  bricks and parts are host
 * arrays of n entries; workspace is caller device memory of at least
 * vr_frame_workspace_size(n) bytes, 256-byte aligned, written by this call
 * and borrowed until the enqueued work has run.  The job table is built on
 * the host and copied in stream order from one of two pinned host slots the
 * context owns (the call waits until the copy that used that slot two calls
 * earlier has run; a slot grows, once, for frames of more than 64 partials),
 * so the call is not meant for stream capture; the batch API below keeps its
 * tables resident and is.  Errors: as vr_render_partial, VR_ERR_WORKSPACE,
 * VR_ERR_OUT_OF_MEMORY. */
vr_status vr_render_partials(vr_context ctx, int32_t n, const vr_brick* bricks,
                             const vr_partial* parts, void* workspace, size_t workspace_bytes);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc -- and so
 * cannot provide vr_render_partials' workspace: the same call (same results,
 * bit for bit) with the job table, tile prefix and work-queue counters kept
 * in a fixed device array the library owns (about 26 KB, one copy per GPU,
 * held until the process ends; its address is taken once per context at
 * vr_context_create, which also allocates two pinned host staging buffers of
 * the same size).  This call allocates nothing: the tables are staged through the
 * context's pinned buffers and copied into the array on the context stream.
 * n <= DPVR_STATIC_MAX_PARTIALS (VR_ERR_INVALID_ARG otherwise).  Every call on
 * one GPU, from any context, uses the same array: calls whose work overlaps
 * on one GPU (different streams, or several contexts) race and give wrong
 * images; calls ordered on one stream are safe.  The host may block until
 * the table copy of the call before the previous one has run.
 * Errors: as vr_render_partials (except VR_ERR_WORKSPACE). */
#define DPVR_STATIC_MAX_PARTIALS 64
vr_status vr_render_partials_static(vr_context ctx, int32_t n, const vr_brick* bricks,
                                    const vr_partial* parts);

/* Sort-last composite (paper Sec. 3: the framebuffer ends up on the main
 * rank): for every pixel of the frame, the n partials (0 <= n <=
 * DPVR_MAX_PARTIALS) are ordered by ascending depth key (ties: lower index
 * first) and combined front to back with "over", then over the background
 * bg (host array, 4 floats, premultiplied).  out is a device array of
 * height * width * 4 floats, row 0 at the top.  parts is a host array; its
 * buffers are borrowed until the enqueued kernel has run.
 * Errors: VR_ERR_INVALID_ARG, VR_ERR_STATE (no camera), VR_ERR_DEVICE. */
vr_status vr_composite(vr_context ctx, const vr_partial* parts, int32_t n, const float bg[4],
                       float* out);

/* -------------------------------------------------------------- batches */
/* Many partial images -- bricks x time steps x fields x cameras -- and the
 * frames composited from them, as one unit of work: one persistent march
 * launch per storage precision over a device work queue of (job, tile)
 * tickets, then one launch compositing every frame, captured once into a
 * HIP graph and replayed by vr_batch_launch (one such graph per release
 * group when the frames are split, see vr_batch_set_groups).  The paper's data-parallel
 * renderers queue and batch work to amortise latency (Sec. 2.2); here the
 * unit is a 16x16 tile of a partial image. */
typedef struct vr_batch_s* vr_batch;

typedef struct {
    int32_t kind;          /* 0 perspective (pinhole), 1 orthographic */
    int32_t width, height;
    int32_t pad_;
    double eye[3];         /* perspective eye / orthographic image centre */
    double target[3];      /* perspective look-at point / orthographic view direction */
    double up[3];
    double fovy_deg;       /* perspective vertical field of view / orthographic view height */
} vr_camera_desc;

typedef struct {
    const float* rgba;     /* device, 256 x 4, as for vr_set_transfer_function */
    float vmin, vmax, opacity_scale;
    int32_t pad_;
} vr_tf_desc;

typedef struct {
    vr_brick brick;        /* the brick, with the data this job renders */
    int32_t camera;        /* index into the batch's cameras */
    int32_t tf;            /* index into the batch's transfer functions */
    vr_partial part;       /* ROI (see vr_camera_roi) and output buffers */
} vr_batch_job;

typedef struct {
    int32_t camera;        /* the frame's camera (all its jobs use it) */
    int32_t first_job;     /* its partials are jobs [first_job, first_job + n_jobs) */
    int32_t n_jobs;        /* 0 .. DPVR_MAX_PARTIALS */
    int32_t pad_;
    float bg[4];
    float* out;            /* device, height * width * 4 floats */
} vr_batch_frame;

/* Host-only: the ROI of `brick` in the frame of camera `cam` (as
 * vr_partial_roi does for the context camera). */
vr_status vr_camera_roi(vr_context ctx, vr_brick brick, const vr_camera_desc* cam,
                        int32_t roi[4]);

/* Device workspace a batch of n_jobs jobs and n_frames frames needs. */
vr_status vr_batch_workspace_size(int32_t n_jobs, int32_t n_frames, size_t* bytes);

/* Build a batch: validates every job and frame, writes the job tables into
 * workspace (caller device memory, >= vr_batch_workspace_size, 256-byte
 * aligned, borrowed for the batch's lifetime; a synchronous copy), and
 * captures the launches into a HIP graph.  dt and ert_epsilon come from the
 * context at creation.  Bricks' data must not change while the batch may
 * run; output and TF buffers are borrowed for its lifetime.
 * Errors: VR_ERR_INVALID_HANDLE, VR_ERR_INVALID_ARG, VR_ERR_WORKSPACE,
 * VR_ERR_STATE (a brick without data), VR_ERR_DEVICE. */
vr_status vr_batch_create(vr_context ctx, int32_t n_cameras, const vr_camera_desc* cameras,
                          int32_t n_tfs, const vr_tf_desc* tfs, int32_t n_jobs,
                          const vr_batch_job* jobs, int32_t n_frames, const vr_batch_frame* frames,
                          void* workspace, size_t workspace_bytes, vr_batch* out);

/* Enqueue the whole batch on the context stream (one graph launch per
 * release group, see vr_batch_set_groups).  Every
 * partial and frame equals what vr_render_partial / vr_composite would
 * produce, bit for bit, whatever launch configuration the batch uses. */
vr_status vr_batch_launch(vr_batch batch);

/* Launch-configuration search: time each candidate configuration -- staged
 * family and tile shape (slab 16x16; ring 16 or 32 pixels wide) x chunk
 * length (ring: 4 or 8 slices, i.e. the samples a marching wavefront takes
 * between synchronisations) x job order (as given, or grouped by brick so
 * that the cameras of one brick run together and share L2) x persistent
 * workgroups per CU -- over `reps` replays, keep the
 * fastest and report its average time per launch in *best_ms.  When the
 * environment variable DPVR_AUTOTUNE_CACHE names a file, a configuration
 * found earlier for the same batch shape and device is reused from it (and
 * new results are appended).  Synchronises the context stream. */
vr_status vr_batch_autotune(vr_batch batch, int32_t reps, double* best_ms);

/* The batch's current configuration: workgroups per CU, job order
 * (0 = as given, 1 = grouped by brick), staged family (vr_staging), tile
 * width and chunk length.  Any pointer may be NULL.  A new batch starts with
 * the context's march configuration and the most workgroups per CU that fit. */
vr_status vr_batch_config(vr_batch batch, int32_t* wg_per_cu, int32_t* order, int32_t* staging,
                          int32_t* tile_width, int32_t* chunk_slices);

/* Release groups, so that a caller can use the first images of a batch
 * while the rest still render: split the batch's frames into n_groups
 * consecutive runs of (nearly) equal length, group g holding frames
 * [g F / n_groups, (g + 1) F / n_groups) of the F frames.  Each group is
 * then its own graph -- the march queues of the jobs its frames use first
 * (a job used by frames of several groups runs with the earliest; jobs no
 * frame uses run with the last group), then those frames' composites --
 * and vr_batch_launch replays the groups in order, marking each group done
 * on the context stream as its graph completes.  Every partial and frame
 * stays bit-identical to the one-group batch.  A new batch has one group.
 * n_groups in [1, max(F, 1)], else VR_ERR_INVALID_ARG.  Keeps the current
 * launch configuration (vr_batch_autotune afterwards tunes the grouped
 * batch).  Synchronises the context stream. */
vr_status vr_batch_set_groups(vr_batch batch, int32_t n_groups);

/* The frames of release group `group`: [*first_frame, *first_frame +
 * *n_frames).  Either pointer may be NULL.  VR_ERR_INVALID_ARG for a group
 * out of range. */
vr_status vr_batch_group(vr_batch batch, int32_t group, int32_t* first_frame, int32_t* n_frames);

/* Wait for release group `group` of the most recent vr_batch_launch: with
 * stream NULL the calling thread blocks until the group's frames are
 * written; otherwise `stream` (a hipStream_t of the context's device) waits
 * for them on the device and the call returns at once.  Before any launch it
 * returns at once.  VR_ERR_INVALID_ARG for a group out of range,
 * VR_ERR_DEVICE on a runtime error. */
vr_status vr_batch_wait_group(vr_batch batch, int32_t group, void* stream);

/* *done = 1 once release group `group` of the most recent vr_batch_launch
 * has completed (or before any launch), else 0; does not block. */
vr_status vr_batch_group_done(vr_batch batch, int32_t group, int32_t* done);

vr_status vr_batch_release(vr_batch batch);

/* -------------------------------------------------------------- adjoint */
/* Differentiable rendering: gradients of a scalar loss L of the frame with
 * respect to the transfer-function table and the voxel values, for
 * transfer-function and inverse-volume fitting.  The forward pass stores the
 * transmittance in front of every `interval`-th owned sample of every ray
 * (segment checkpoints, 1 <= interval <= DPVR_MAX_CKPT_INTERVAL); the
 * backward re-marches each segment from its checkpoint, last segment first.
 * Early termination is off in both passes.  Gradients are exact derivatives
 * of the rendered image (readings: emission-absorption as above; the table
 * lookup is differentiated on the segment it uses, min(floor(s), 254), and
 * has zero derivative in v outside [vmin, vmax]). */
#define DPVR_MAX_CKPT_INTERVAL 64

/* Host-only: bytes of checkpoint storage vr_render_partial_checkpointed needs
 * for `part`'s ROI with this interval (ROI pixels x ceil((max owned samples
 * per ray) / interval) floats, the maximum taken over the brick's diagonal). */
vr_status vr_checkpoint_size(vr_context ctx, vr_brick brick, const vr_partial* part,
                             int32_t interval, size_t* bytes);

/* Forward march of one partial without early termination, writing the same
 * partial image as vr_render_partial with ert_epsilon = 0 and the
 * checkpoints into ckpt (device, >= vr_checkpoint_size bytes). */
vr_status vr_render_partial_checkpointed(vr_context ctx, vr_brick brick, const vr_partial* part,
                                         int32_t interval, float* ckpt, size_t ckpt_bytes);

/* Backward of vr_composite: given d_out = dL/d(frame) (device, height * width
 * * 4 floats), writes dL/d(partial p) into d_parts[p] (device, part p's ROI,
 * h * w * 4 floats: dL/dC_r, dL/dC_g, dL/dC_b, dL/dA); pixels where partial
 * p's key is +inf get zeros.  parts must hold the forward's partial images. */
vr_status vr_composite_backward(vr_context ctx, const vr_partial* parts, int32_t n,
                                const float bg[4], const float* d_out, float* const* d_parts);

/* Backward of one partial: d_part (device, ROI h * w * 4) = dL/d(partial);
 * ckpt = the checkpoints of vr_render_partial_checkpointed with the same
 * interval, camera, transfer function and brick data.  Accumulates (adds
 * to) dL/d(table) into grad_tf (device, 256 x 4, same layout as the table)
 * and dL/d(voxel) into grad_volume (device, vol_dims floats, x fastest): a
 * stored voxel (ghosts included) is a copy of the global voxel
 * clamp(lo + s - 1), so its gradient lands there.  Uses float atomics, so
 * the summation order (last bits) varies from run to run. */
vr_status vr_render_partial_backward(vr_context ctx, vr_brick brick, const vr_partial* part,
                                     int32_t interval, const float* ckpt, size_t ckpt_bytes,
                                     const float* d_part, float* grad_tf, float* grad_volume,
                                     const int32_t vol_dims[3], const int32_t lo[3]);

/* Host-only: device workspace bytes of vr_render_partials_checkpointed for
 * n partials.  Errors: VR_ERR_INVALID_ARG. */
vr_status vr_checkpointed_workspace_size(int32_t n, size_t* bytes);

/* n calls of vr_render_partial_checkpointed in one launch per storage
 * precision over all partials' 8x8 tiles (arrays of n entries; ckpts[i] of
 * ckpt_bytes[i] bytes).  workspace: device, 256-byte aligned,
 * vr_checkpointed_workspace_size bytes, written by this call and borrowed
 * until the enqueued work has run.  Errors: as
 * vr_render_partial_checkpointed, VR_ERR_WORKSPACE. */
vr_status vr_render_partials_checkpointed(vr_context ctx, int32_t n, const vr_brick* bricks, const vr_partial* parts,
                                          int32_t interval, float* const* ckpts, const size_t* ckpt_bytes,
                                          void* workspace, size_t workspace_bytes);

/* Host-only: device workspace bytes of vr_render_partials_backward for n
 * partials (their job table and workgroup prefix).  Errors:
 * VR_ERR_INVALID_ARG. */
vr_status vr_backward_workspace_size(int32_t n, size_t* bytes);

/* The backward of n partials at once (same arguments as n calls of
 * vr_render_partial_backward, arrays of n entries; los = n x 3 owned min
 * corners): one launch per storage precision over all partials' tiles, so
 * that partials of few tiles still fill the GPU.  workspace: device,
 * 256-byte aligned, vr_backward_workspace_size bytes, written by this call
 * (the table is copied from host memory) and borrowed until the enqueued
 * work has run.  Errors: as vr_render_partial_backward, VR_ERR_WORKSPACE. */
vr_status vr_render_partials_backward(vr_context ctx, int32_t n, const vr_brick* bricks, const vr_partial* parts,
                                      int32_t interval, const float* const* ckpts, const size_t* ckpt_bytes,
                                      const float* const* d_parts, float* grad_tf, float* grad_volume,
                                      const int32_t vol_dims[3], const int32_t* los, void* workspace,
                                      size_t workspace_bytes);

/* ------------------------------------------------- time-step streaming */
/* Time-varying data with only some time steps resident (paper Sec. 4: the
 * time steps of the data set are loaded selectively and evicted later, so
 * that the GPUs never hold the whole series).  A series owns `slots` sets of
 * bricks (one brick per vr_brick_desc in every set) in a caller-provided
 * device workspace; step t of brick b comes from host_voxels[t * n_bricks +
 * b], a ghost-padded float32 host array (pinned memory lets the copy run
 * asynchronously; borrowed for the series' lifetime).  Loading a step takes
 * the least recently used slot, waits (on the GPU) for all render work
 * enqueued on the context stream so far, then copies the step's arrays to a
 * device staging buffer and ingests them into the slot's bricks, all on the
 * series' own copy stream, so uploads overlap rendering. */
typedef struct vr_timeseries_s* vr_timeseries;

typedef struct {
    int32_t dims[3];       /* owned voxels (nx, ny, nz) */
    int32_t ghost;         /* must be 1 */
    double origin[3];      /* as for vr_brick_create */
    double spacing[3];
    vr_dtype storage;
    int32_t pad_;
} vr_brick_desc;

/* Host-only: device workspace bytes of a series of these bricks with
 * `slots` resident steps (slots x the bricks' workspaces + one staging
 * buffer of the largest float32 brick).  Errors: VR_ERR_INVALID_ARG. */
vr_status vr_timeseries_workspace_size(int32_t n_bricks, const vr_brick_desc* bricks, int32_t slots, size_t* bytes);

/* Create a series of n_steps steps of n_bricks bricks (1 <= n_bricks <=
 * DPVR_MAX_PARTIALS) with `slots` >= 1 resident steps.  workspace: device,
 * 256-byte aligned, vr_timeseries_workspace_size bytes, owned by the caller
 * and kept until vr_timeseries_release.  Errors: VR_ERR_INVALID_HANDLE,
 * VR_ERR_INVALID_ARG, VR_ERR_WORKSPACE, VR_ERR_OUT_OF_MEMORY, VR_ERR_DEVICE. */
vr_status vr_timeseries_create(vr_context ctx, int32_t n_bricks, const vr_brick_desc* bricks, int32_t n_steps,
                               const float* const* host_voxels, int32_t slots, void* workspace,
                               size_t workspace_bytes, vr_timeseries* out);

/* Start loading `step` if it is not resident (returns at once; the load
 * runs on the copy stream).  Errors: VR_ERR_INVALID_HANDLE,
 * VR_ERR_INVALID_ARG, VR_ERR_DEVICE. */
vr_status vr_timeseries_prefetch(vr_timeseries ts, int32_t step);

/* The bricks of `step` (loading it first if needed) into bricks[0 ..
 * n_bricks): the context stream waits (on the GPU) until the step's load has
 * run, so render calls enqueued after this one see its data.  The handles
 * belong to the series (vr_brick_release refuses them) and hold this step
 * until a later prefetch or acquire evicts their slot: enqueue the renders
 * that read a step before a call that may evict it (an eviction waits for
 * the work already enqueued on the context stream, not for later work).
 * Errors: as vr_timeseries_prefetch. */
vr_status vr_timeseries_acquire(vr_timeseries ts, int32_t step, vr_brick* bricks);

/* Steps loaded so far, and the step each slot holds (-1: none; `slots`
 * entries).  Either pointer may be NULL. */
vr_status vr_timeseries_stats(vr_timeseries ts, int64_t* loads, int32_t* resident_steps);

/* Release the series (waits for its copies and the context stream). */
vr_status vr_timeseries_release(vr_timeseries ts);

/* ---------------------------------------------------- ray-queue cycling */
/* Data-parallel ray tracing by ray-queue cycling (paper Sec. 2.2 and Fig. 2:
 * rays are queued and batched, every ray is cycled through every rank's
 * data, and a shadow ray must visit the rank that holds its occluder; Sec. 3:
 * the DP-ANARI conventions assume this, so the data need not be
 * redistributed).  Here the n bricks play the ranks on one GPU.  One
 * directional light: every owned primary sample's emitted colour is scaled
 * by ambient + (1 - ambient) S, S the transmittance toward the light of a
 * shadow ray from the sample (samples at p + (j + 1/2) dt l, j >= 0, each
 * evaluated in the brick that owns it; alpha, depth keys and the primary
 * transmittance are unchanged).  ambient = 1: no shadow rays; the image then
 * equals the sort-last image of the same bricks (vr_render_partials +
 * vr_composite) exactly. */
typedef struct {
    double direction[3];   /* toward the light, world units, non-zero (normalised here) */
    float ambient;         /* in [0, 1] */
    int32_t pad_;
} vr_light;

/* Host-only: bytes of the workspace vr_rqc_plan and vr_render_rqc use for
 * these n bricks (1 <= n <= DPVR_MAX_PARTIALS, no brick twice) and the
 * context camera: the brick table, one plan entry per (brick, ROI pixel), the
 * per-pixel segment slots of every brick.  Errors: VR_ERR_INVALID_HANDLE,
 * VR_ERR_INVALID_ARG, VR_ERR_STATE (no camera). */
vr_status vr_rqc_workspace_size(vr_context ctx, int32_t n, const vr_brick* bricks, size_t* bytes);

/* Plan a frame: counts every (brick, ROI pixel)'s owned primary samples and
 * gives each a slot (device scan), then synchronises the context stream and
 * returns the number of slots, which sizes the shade buffer of
 * vr_render_rqc (total_samples * 4 bytes).  workspace: device memory of
 * vr_rqc_workspace_size bytes, 256-byte aligned, kept by the caller for the
 * renders of this plan.  Depends on the bricks' geometry, the camera and dt
 * only.  Errors: as vr_rqc_workspace_size, VR_ERR_WORKSPACE, VR_ERR_DEVICE. */
vr_status vr_rqc_plan(vr_context ctx, int32_t n, const vr_brick* bricks, void* workspace, size_t workspace_bytes,
                      int64_t* total_samples);

/* Render the frame of the last vr_rqc_plan (same workspace, bricks, camera
 * and dt, or VR_ERR_STATE) with the current transfer function and data:
 * n cycle steps of the shadow-ray queues (skipped when ambient = 1), n cycle
 * steps of the primary-ray queues, then per pixel the bricks' segments in
 * depth order over bg.  shade: device, total_samples floats (ignored when
 * ambient = 1); out: device, height x width x 4 floats, 16-byte aligned;
 * samples: optional device counter (8-byte aligned) to which the primary and
 * shadow samples evaluated are added.  Enqueued on the context stream.
 * Errors: VR_ERR_INVALID_HANDLE, VR_ERR_INVALID_ARG, VR_ERR_STATE,
 * VR_ERR_WORKSPACE, VR_ERR_DEVICE. */
vr_status vr_render_rqc(vr_context ctx, int32_t n, const vr_brick* bricks, const vr_light* light, const float bg[4],
                        void* workspace, size_t workspace_bytes, float* shade, size_t shade_bytes, float* out,
                        unsigned long long* samples);

/* ---------------------------------------------------- tetrahedral parts */
/* Unstructured data: a volume given as a tetrahedral mesh split into parts,
 * each the share of one rank (paper Sec. 2.2 and Fig. 2: finite elements are
 * distributed so that every rank holds a share; Sec. 4: the lander's
 * mixed-element data keeps the simulation's partition, which is uneven in
 * space).  A part need not be convex; together the parts of one frame must
 * form one conforming mesh (neighbouring tetrahedra share whole faces, no
 * two overlap).
 *   locate   a lattice sample p belongs to the tetrahedron whose four signed
 *            sub-volumes (p against each face, float64) are positive; a
 *            sub-volume of exactly zero counts as inside when the fixed
 *            direction g = (1, 2^-10, 2^-20) enters the tetrahedron across
 *            that face.  Faces are evaluated from their vertices in
 *            lexicographic order, so in a conforming mesh every sample has
 *            at most one owner and the owners do not depend on the split.
 *   value    barycentric interpolation of the four vertex values (the
 *            sub-volumes over their sum), then the context's transfer
 *            function, extinction and front-to-back accumulation as for
 *            bricks; no early termination.
 *   runs     a ray's samples held by one part fall into runs of consecutive
 *            lattice indices (a non-convex part can hold several); each run
 *            is accumulated on its own and the frame is the runs of all
 *            parts in index order, "over" one another, over a background --
 *            the same image as accumulating the ray through the whole mesh.
 * The paper locates elements with a bounding volume hierarchy (Sec. 2.1);
 * here a sample is first sought by a walk from the previous sample's
 * tetrahedron across face neighbours, then in a uniform grid over the part's
 * bounding box whose cells list the tetrahedra that can hold a point of the
 * cell (or, by vr_set_tet_locator, in a BVH). */
typedef struct vr_tetpart_s* vr_tetpart;

#define DPVR_MAX_TET_PARTS 64        /* parts per vr_render_tetparts call */
#define DPVR_MAX_TET_RUNS 32         /* runs per ray and part */

/* Create a part from host arrays: vertices (n_vertices x 3 doubles, x, y, z),
 * tets (n_tets x 4 vertex indices, either orientation).  Builds the part's
 * location tables in host memory (face planes, tie bits, face neighbours,
 * the grid, the BVH); the arrays are not kept.  At most 2^28 - 1
 * tetrahedra per part.  n_tets may be 0 (a part that owns nothing).
 * Errors: VR_ERR_INVALID_HANDLE, VR_ERR_INVALID_ARG (index out of range,
 * non-finite coordinate, zero-volume tetrahedron, a face shared by more than
 * two tetrahedra, more than 2^31 - 1 grid entries), VR_ERR_OUT_OF_MEMORY. */
vr_status vr_tetpart_create(vr_context ctx, const double* vertices, int32_t n_vertices, const int32_t* tets,
                            int32_t n_tets, vr_tetpart* out);

/* Mixed finite elements (the paper's lander data mixes element types,
 * Sec. 4), read as tetrahedra: cell c has cell_sizes[c] = 4, 5, 6 or 8 nodes
 * (tetrahedron v0..v3; pyramid: base v0..v3 in cyclic order, apex v4; wedge:
 * bottom triangle v0 v1 v2, top v3 v4 v5 with v3 above v0; hexahedron:
 * bottom v0..v3 cyclic, top v4..v7 with v4 above v0), cell_vertices their
 * node indices one cell after another.  Every quadrilateral face is cut
 * along the diagonal through its node of smallest vertex_ids value (a
 * global id per vertex, so that parts sharing the face cut it alike; NULL
 * = the vertex index); a pyramid becomes its two base triangles joined to
 * the apex; a wedge or a hexahedron gets a centre vertex (position: the
 * sum of its node positions in node order over the node count; value: the
 * mean of its node values, recomputed at every vr_tetpart_set_values) joined
 * to every triangle of its faces.  The field is then piecewise linear on
 * these tetrahedra, not the elements' own interpolation.  vertices and the
 * values of vr_tetpart_set_values are the n_vertices input vertices.
 * Errors: as vr_tetpart_create, VR_ERR_INVALID_ARG also for a cell size
 * other than 4, 5, 6, 8. */
vr_status vr_tetpart_create_cells(vr_context ctx, const double* vertices, int32_t n_vertices, const int64_t* vertex_ids,
                                  const uint8_t* cell_sizes, const int32_t* cell_vertices, int32_t n_cells,
                                  vr_tetpart* out);

/* Where a sample is searched when the walk from the previous sample's
 * tetrahedron does not find it (every choice locates the same owner, so
 * images are bit-identical): VR_TET_GRID, the part's uniform grid of
 * candidate lists (default); VR_TET_BVH, a bounding volume hierarchy over
 * the part's tetrahedra (the paper's element-location structure, Sec. 2.1:
 * boxes tested top down, tetrahedra at the leaves), traversed without a
 * stack through skip links. */
typedef enum { VR_TET_GRID = 0, VR_TET_BVH = 1 } vr_tet_locator;
vr_status vr_set_tet_locator(vr_context ctx, vr_tet_locator locator);

/* The part's closed bounding box, grid cells per axis, grid entries, the
 * bytes of device workspace it needs and its tetrahedra (any pointer may be
 * NULL). */
vr_status vr_tetpart_info(vr_tetpart part, double lo[3], double hi[3], int32_t grid[3], int64_t* grid_entries,
                          size_t* workspace_bytes, int32_t* n_tets);

/* Give the part its device workspace (caller-owned, 256-byte aligned, at
 * least the bytes vr_tetpart_info reports, kept until the part is released)
 * and enqueue the upload of its tables on the context stream.  Vertex values
 * must be set (again) afterwards. */
vr_status vr_tetpart_attach(vr_tetpart part, void* workspace, size_t workspace_bytes);

/* Vertex values (a new time step or field): values is a device array of
 * n_vertices floats (the vertices the part was created with), borrowed until
 * the enqueued gather has run.
 * Errors: VR_ERR_STATE (no workspace attached). */
vr_status vr_tetpart_set_values(vr_tetpart part, const float* values);

/* Release a part (waits for the context stream first, since uploads may
 * still read its host tables; the caller frees the workspace). */
vr_status vr_tetpart_release(vr_tetpart part);

/* Bytes of the frame workspace of vr_render_tetparts for these parts
 * (1 <= n <= DPVR_MAX_TET_PARTS, no part twice), max_runs (1 ..
 * DPVR_MAX_TET_RUNS) and the context camera: the part table and, per part,
 * run buffers over the pixels its bounding box covers.
 * Errors: VR_ERR_INVALID_HANDLE, VR_ERR_INVALID_ARG, VR_ERR_STATE (no camera). */
vr_status vr_tetparts_workspace_size(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs,
                                     size_t* bytes);

/* Render the parts into out (device, height x width x 4 floats,
 * premultiplied, 16-byte aligned) over bg, with the context camera, transfer
 * function and dt.  workspace: device, 256-byte aligned, at least
 * vr_tetparts_workspace_size bytes.  samples: optional device counter
 * (8-byte aligned) to which the samples held by a tetrahedron are added.  A
 * ray that crosses a part in more than max_runs runs sets the device error
 * word (reported as VR_ERR_DEVICE by vr_synchronize; that image is wrong).
 * Enqueued on the context stream.  Errors: VR_ERR_INVALID_HANDLE,
 * VR_ERR_INVALID_ARG, VR_ERR_STATE (no camera, transfer function or values),
 * VR_ERR_WORKSPACE, VR_ERR_OUT_OF_MEMORY, VR_ERR_DEVICE. */
vr_status vr_render_tetparts(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs, const float bg[4],
                             void* workspace, size_t workspace_bytes, float* out, unsigned long long* samples);

/* The two stages of vr_render_tetparts on their own (same arguments): the
 * march leaves every part's runs in the workspace -- the per-rank step of a
 * data-parallel renderer, whose runs would travel to the compositing rank --
 * and the resolve merges them into out.  vr_resolve_tetparts requires that
 * the last vr_march_tetparts (or vr_render_tetparts) of the context used
 * the same workspace, parts, max_runs and camera (VR_ERR_STATE otherwise);
 * it needs no transfer function or vertex values. */
vr_status vr_march_tetparts(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs, void* workspace,
                            size_t workspace_bytes, unsigned long long* samples);
vr_status vr_resolve_tetparts(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs, const float bg[4],
                              void* workspace, size_t workspace_bytes, float* out);

/* Shadow rays through tetrahedral parts (paper Fig. 2: the hit lies in one
 * rank's elements, its occluder in another's, so the shadow ray must visit
 * every rank; Sec. 2.2).  One directional light as for vr_render_rqc: every
 * held primary sample's emitted colour is scaled by ambient + (1 - ambient)
 * S, S the transmittance of its shadow ray (samples p + (j + 1/2) dt l,
 * j >= 0, each located in the parts as a primary sample); alpha and T are
 * unchanged.  The shadow rays are queued per part and cycled: in step s the
 * queue of part h is traced through part (h + s) mod n.
 *
 * vr_tetparts_shadow_plan_size: bytes of the plan buffer for these parts and
 * the context camera (one slot offset per ROI pixel of every part).
 * vr_tetparts_shadow_plan: counts every ray's held samples per part (one
 * march without shading into the plan; workspace as for vr_render_tetparts)
 * and gives each a slot (device scan), then synchronises the context stream
 * and returns the slot count; depends on geometry, camera and dt only.
 * vr_tetparts_slot_bytes: bytes of the slot buffer for that count (a sample
 * index and a transmittance per slot).
 * vr_render_tetparts_shadowed: the frame of the last plan (same plan buffer,
 * parts, camera and dt, else VR_ERR_STATE): records the slots' sample
 * indices, runs n shadow cycle steps, marches the shaded runs and resolves
 * them into out over bg.  plan, slots: device, 256-byte aligned, kept by the
 * caller; samples (optional) counts primary and shadow samples held.
 * Errors: as vr_render_tetparts, VR_ERR_WORKSPACE for a short plan or slot
 * buffer, VR_ERR_INVALID_ARG for a zero or non-finite light direction or an
 * ambient outside [0, 1]. */
vr_status vr_tetparts_shadow_plan_size(vr_context ctx, int32_t n, const vr_tetpart* parts, size_t* bytes);
vr_status vr_tetparts_shadow_plan(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs,
                                  void* workspace, size_t workspace_bytes, void* plan, size_t plan_bytes,
                                  int64_t* total_samples);
vr_status vr_tetparts_slot_bytes(int64_t total_samples, size_t* bytes);
vr_status vr_render_tetparts_shadowed(vr_context ctx, int32_t n, const vr_tetpart* parts, int32_t max_runs,
                                      const vr_light* light, const float bg[4], void* workspace,
                                      size_t workspace_bytes, void* plan, size_t plan_bytes, void* slots,
                                      size_t slot_bytes, float* out, unsigned long long* samples);

#ifdef __cplusplus
}
#endif

#endif /* DPVR_H */
