// Adjoint of the per-brick ray march for gfx950: gradients of a loss with
// respect to the transfer-function table and the global voxel array, given
// the loss gradient of the brick's partial image (dL/dC_rgb, dL/dA per ROI
// pixel) and the transmittance checkpoints written by the checkpointing
// forward march.
//
// One wavefront per 8x8 tile, one lane per ray, four tiles per workgroup
// (sharing the table and its gradient in LDS) when the partial has many
// tiles, one otherwise.  A ray's
// owned samples are cut into segments of ckpt_interval (<= 64) samples.
// Segments are processed last to first: the segment is re-marched forward
// from its checkpoint, storing the transmittance T_k in front of each sample
// in LDS (no division by T anywhere), then walked backwards with
//   R_k = a_k rgb_k + (1 - a_k) R_{k+1},  Q_k = (1 - a_k) Q_{k+1}
// (R = colour, Q = transmittance of what lies behind sample k in the brick),
//   dC/drgb_k = T_k a_k,  dC/da_k = T_k (rgb_k - R_{k+1}),  dA/da_k = T_k Q_{k+1}.
// The opacity a_k = 1 - exp2(-a'_k) with a' the pre-scaled table opacity;
// table gradients are summed per lane while consecutive samples use one
// table segment, accumulated per workgroup in LDS (ds_add_f32) and flushed
// with one global atomic per touched entry; voxel gradients are
// scattered with the 8 trilinear weights to the global voxels that the stored
// (ghost-padded) voxels copy, so ghost contributions fold back to their source
// (summed per lane per corner while the walk stays in one cell; moving to a
// neighbouring cell keeps the sums of the shared corners, so a corner is
// added with one atomic when the walk leaves it).
#include "march_common.h"

namespace dpvr {
namespace {

constexpr int kTile = 8;
// Wavefronts per workgroup, one 8x8 tile each: four share the table and its
// gradient in LDS, so that the per-wave transmittance buffers set occupancy;
// a partial of few tiles takes one per workgroup, so that its tiles still
// spread over the compute units.
constexpr int kWavesWide = 4;
constexpr int kWideMinTiles = 2048;
constexpr float kLn2 = 0.6931471805599453f;

// One workgroup's work: tiles first_tile .. first_tile + kWaves - 1 of the
// partial (p, bp), one per wavefront.
template <typename TS, int kWaves>
__device__ inline void backward_tiles(const MarchParams& p, const BackwardParams& bp, int first_tile) {
    __shared__ TFTable tft;
    __shared__ float gtf[256 * 4];
    __shared__ float tbuf_all[kWaves][kMaxCkptInterval * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float* tbuf = tbuf_all[wave];
    load_tf(tft, p.tf, p.dt, threadIdx.x, kWaves * 64);
    for (int e = threadIdx.x; e < 1024; e += kWaves * 64) gtf[e] = 0.0f;
    __syncthreads();

    const int tile = first_tile + wave;
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int lx = tx * kTile + (lane & 7), ly = ty * kTile + (lane >> 3);
    const bool valid = tile < p.tiles_x * p.tiles_y && lx < p.roi_w && ly < p.roi_h;
    const int px = p.roi_x0 + lx, py = p.roi_y0 + ly;
    const long long pix = (long long)ly * p.roi_w + lx;

    const BrickK& b = p.brick;
    const TS* __restrict__ vox = reinterpret_cast<const TS*>(b.data);
    const int snx = b.sdim[0], sny = b.sdim[1], snz = b.sdim[2];
    const int pitch = row_pitch(snx);
    const long long sxy = (long long)pitch * sny;
    const float tf_k = 255.0f / (p.tf.vmax - p.tf.vmin);
    const float tf_o = -p.tf.vmin * tf_k;
    // d a' / d alpha_table: converts pre-scaled opacity gradients to table units
    const float a_scale = p.tf.opacity_scale * (float)p.dt * kLog2e;
    const int I = p.ckpt_interval;
    const long long gnx = bp.vol_dims[0], gny = bp.vol_dims[1], gnz = bp.vol_dims[2];

    RaySetup rs;
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    bool has = valid && setup_ray(p.cam, b, p.dt, px, py, rs);
    if (has) {
        g = reinterpret_cast<const float4*>(bp.d_part)[pix];
        has = g.x != 0.f || g.y != 0.f || g.z != 0.f || g.w != 0.f;
    }
    if (has) {
        const Step st = make_step(rs, b, p.dt);
        const Blocks bl = make_blocks(rs, b);
        const long long N = rs.kl - rs.kf + 1;
        const int nseg = (int)min((N + I - 1) / I, (long long)p.ckpt_nseg);
        float R0 = 0.f, R1 = 0.f, R2 = 0.f, Q = 1.f;
        // anchor cursor: block n holds samples [kA, kNext) anchored at kA
        long long bn = 0, kA = 0, kNext = 0;
        Anchor an{};
        auto seek = [&](long long k) {
            bn = block_of(bl, p.dt, p.inv_dt, k);
            kA = max(rs.kf, block_start(bl, p.inv_dt, bn));
            kNext = block_start(bl, p.inv_dt, bn + 1);
            an = make_anchor(rs, b, p.dt, kA);
        };
        auto sample = [&](long long k) {
            if (k < kA || k >= kNext) seek(k);
            const Cell c = locate(an, st, (float)(k - kA), snx, sny, snz);
            return c;
        };
        // voxel-gradient contributions of the current cell's 8 corners, not
        // yet added (acc[cx + 2 cy + 4 cz] for corner (ix + cx, iy + cy,
        // iz + cz) of the stored grid)
        int pend_key = -1, pend_ix = 0, pend_iy = 0, pend_iz = 0;
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float* G = bp.grad_vox;
        const long long glo0 = (long long)bp.lo[0] - b.ghost, glo1 = (long long)bp.lo[1] - b.ghost,
                        glo2 = (long long)bp.lo[2] - b.ghost;
        // stored index s -> global index clamp(lo + s - ghost)
        auto add_voxel = [&](int sx, int sy, int sz, float v) {
            if (v == 0.0f) return;
            const long long gx = min(max(glo0 + sx, 0LL), gnx - 1);
            const long long gy = min(max(glo1 + sy, 0LL), gny - 1);
            const long long gz = min(max(glo2 + sz, 0LL), gnz - 1);
            atomicAdd(G + (gz * gny + gy) * gnx + gx, v);
        };
        auto flush = [&]() {
            if (pend_key < 0) return;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                add_voxel(pend_ix + (i & 1), pend_iy + ((i >> 1) & 1), pend_iz + (i >> 2), acc[i]);
                acc[i] = 0.f;
            }
        };
        // the walk moves to cell (nx, ny, nz): a corner the two cells share
        // keeps its sum (moving by one cell along an axis keeps the 4 corners
        // of the face crossed); the corners left behind are added now, one
        // axis at a time; a jump of more than one cell adds all 8
        auto move_to = [&](int nx, int ny, int nz, int key) {
            const int dx = nx - pend_ix, dy = ny - pend_iy, dz = nz - pend_iz;
            if (pend_key < 0 || dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) {
                flush();
            } else {
                if (dx != 0) {
#pragma unroll
                    for (int yz = 0; yz < 4; ++yz) {   // corner pairs along x: acc[2 yz], acc[2 yz + 1]
                        const int cy = yz & 1, cz = yz >> 1;
                        const float a0 = acc[2 * yz], a1 = acc[2 * yz + 1];
                        add_voxel(pend_ix + (dx > 0 ? 0 : 1), pend_iy + cy, pend_iz + cz, dx > 0 ? a0 : a1);
                        acc[2 * yz] = dx > 0 ? a1 : 0.f;
                        acc[2 * yz + 1] = dx > 0 ? 0.f : a0;
                    }
                }
                if (dy != 0) {
#pragma unroll
                    for (int xz = 0; xz < 4; ++xz) {   // pairs along y: acc[i], acc[i + 2], i = cx + 4 cz
                        const int cx = xz & 1, cz = xz >> 1, i = cx + 4 * cz;
                        const float a0 = acc[i], a1 = acc[i + 2];
                        add_voxel(nx + cx, pend_iy + (dy > 0 ? 0 : 1), pend_iz + cz, dy > 0 ? a0 : a1);
                        acc[i] = dy > 0 ? a1 : 0.f;
                        acc[i + 2] = dy > 0 ? 0.f : a0;
                    }
                }
                if (dz != 0) {
#pragma unroll
                    for (int xy = 0; xy < 4; ++xy) {   // pairs along z: acc[i], acc[i + 4], i = cx + 2 cy
                        const float a0 = acc[xy], a1 = acc[xy + 4];
                        add_voxel(nx + (xy & 1), ny + (xy >> 1), pend_iz + (dz > 0 ? 0 : 1), dz > 0 ? a0 : a1);
                        acc[xy] = dz > 0 ? a1 : 0.f;
                        acc[xy + 4] = dz > 0 ? 0.f : a0;
                    }
                }
            }
            pend_key = key;
            pend_ix = nx;
            pend_iy = ny;
            pend_iz = nz;
        };
        // table-gradient contributions of the current segment index, not
        // yet added (entries seg and seg + 1): consecutive samples mostly
        // use one segment, so LDS atomics happen once per change
        int tseg = -1;
        float tacc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        auto tflush = [&]() {
            if (tseg < 0) return;
            float* g0 = &gtf[4 * tseg];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (tacc[i] != 0.0f) atomicAdd(g0 + i, tacc[i]);
                tacc[i] = 0.f;
            }
        };
        for (int s = nseg - 1; s >= 0; --s) {
            const long long k0 = rs.kf + (long long)s * I;
            const int n = (int)min((long long)I, rs.kl - k0 + 1);
            // forward over the segment from its checkpoint
            float T = p.ckpt[pix * p.ckpt_nseg + s];
            for (int j = 0; j < n; ++j) {
                tbuf[j * 64 + lane] = T;
                const Cell c = sample(k0 + j);
                const Classified e = classify(tft, trilinear(vox, c, pitch, sxy), tf_k, tf_o);
                T = T * trans_exp2(-e.a);
            }
            // reverse over the segment
            for (int j = n - 1; j >= 0; --j) {
                const Cell c = sample(k0 + j);
                const Classified e = classify(tft, trilinear(vox, c, pitch, sxy), tf_k, tf_o);
                const float Tk = tbuf[j * 64 + lane];
                const float om = trans_exp2(-e.a);          // 1 - alpha
                const float al = 1.0f - om;
                const float ta = Tk * al;
                const float d_r = g.x * ta, d_g = g.y * ta, d_b = g.z * ta;
                const float d_al = Tk * (g.x * (e.r - R0) + g.y * (e.g - R1) + g.z * (e.b - R2) +
                                         g.w * Q);
                const float d_ap = d_al * kLn2 * om;   // dL/da'
                const float w1 = e.phi, w0 = 1.0f - e.phi;
                if (e.seg != tseg) {
                    tflush();
                    tseg = e.seg;
                }
                tacc[0] += w0 * d_r;
                tacc[1] += w0 * d_g;
                tacc[2] += w0 * d_b;
                tacc[3] += w0 * d_ap * a_scale;
                tacc[4] += w1 * d_r;
                tacc[5] += w1 * d_g;
                tacc[6] += w1 * d_b;
                tacc[7] += w1 * d_ap * a_scale;
                if (e.inside) {
                    const float4 D = tft.diff[e.seg];
                    const float dv = tf_k * (d_r * D.x + d_g * D.y + d_b * D.z + d_ap * D.w);
                    if (dv != 0.0f) {
                        // consecutive samples mostly share a cell: sum their
                        // corner weights here, one set of atomics per cell
                        const int key = (c.iz * sny + c.iy) * snx + c.ix;
                        if (key != pend_key) move_to(c.ix, c.iy, c.iz, key);
                        const float ux = 1.0f - c.fx, uy = 1.0f - c.fy, uz = 1.0f - c.fz;
                        acc[0] += dv * ux * uy * uz;
                        acc[1] += dv * c.fx * uy * uz;
                        acc[2] += dv * ux * c.fy * uz;
                        acc[3] += dv * c.fx * c.fy * uz;
                        acc[4] += dv * ux * uy * c.fz;
                        acc[5] += dv * c.fx * uy * c.fz;
                        acc[6] += dv * ux * c.fy * c.fz;
                        acc[7] += dv * c.fx * c.fy * c.fz;
                    }
                }
                R0 = fmaf(al, e.r, om * R0);
                R1 = fmaf(al, e.g, om * R1);
                R2 = fmaf(al, e.b, om * R2);
                Q = om * Q;
            }
        }
        flush();
        tflush();
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += kWaves * 64) {
        const float v = gtf[e];
        if (v != 0.0f) atomicAdd(bp.grad_tf + e, v);
    }
}

template <typename TS, int kWaves>
__global__ __launch_bounds__(kWaves * 64) void march_backward(MarchParams p, BackwardParams bp) {
    backward_tiles<TS, kWaves>(p, bp, blockIdx.x * kWaves);
}

// Many partials in one launch: workgroup b takes kWaves tiles of job j, the
// last j with block_start[j] <= b (so that partials of few tiles still fill
// the GPU together).
template <typename TS, int kWaves>
__global__ __launch_bounds__(kWaves * 64) void march_backward_many(const BackwardJob* __restrict__ jobs,
                                                                   const int32_t* __restrict__ block_start,
                                                                   int32_t n_jobs) {
    const int b = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block_start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);      // uniform: the job's fields load as scalars
    const BackwardJob& J = jobs[lo];
    backward_tiles<TS, kWaves>(J.p, J.bp, (b - __builtin_amdgcn_readfirstlane(block_start[lo])) * kWaves);
}

}  // namespace

int backward_many_waves() { return kWavesWide; }

hipError_t launch_march_backward_many(const BackwardJob* jobs, const int32_t* block_start, int32_t n_jobs,
                                      int32_t total_blocks, StorageK storage, hipStream_t stream) {
    if (n_jobs <= 0 || total_blocks <= 0) return hipSuccess;
    if (storage == kF16)
        hipLaunchKernelGGL((march_backward_many<__half, kWavesWide>), dim3(total_blocks), dim3(kWavesWide * 64), 0,
                           stream, jobs, block_start, n_jobs);
    else
        hipLaunchKernelGGL((march_backward_many<float, kWavesWide>), dim3(total_blocks), dim3(kWavesWide * 64), 0,
                           stream, jobs, block_start, n_jobs);
    return hipGetLastError();
}

hipError_t launch_march_backward(const MarchParams& p, const BackwardParams& bp, StorageK storage,
                                 hipStream_t stream) {
    const int tiles = p.tiles_x * p.tiles_y;
    if (tiles == 0) return hipSuccess;
    if (tiles >= kWideMinTiles) {
        const int blocks = (tiles + kWavesWide - 1) / kWavesWide;
        if (storage == kF16)
            hipLaunchKernelGGL((march_backward<__half, kWavesWide>), dim3(blocks), dim3(kWavesWide * 64), 0,
                               stream, p, bp);
        else
            hipLaunchKernelGGL((march_backward<float, kWavesWide>), dim3(blocks), dim3(kWavesWide * 64), 0,
                               stream, p, bp);
    } else if (storage == kF16) {
        hipLaunchKernelGGL((march_backward<__half, 1>), dim3(tiles), dim3(64), 0, stream, p, bp);
    } else {
        hipLaunchKernelGGL((march_backward<float, 1>), dim3(tiles), dim3(64), 0, stream, p, bp);
    }
    return hipGetLastError();
}

}  // namespace dpvr
