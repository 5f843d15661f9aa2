// Per-brick volume ray casting into a partial image (RGBA premultiplied +
// depth key) for gfx950.
//
// One wavefront per 8x8 pixel tile of the brick's region of interest, one
// lane per ray.  Per ray, in float64 and without FMA contraction (so that
// ownership decisions are bit-identical however the volume is split):
// camera ray, slab test against the brick's owned box, first/last owned
// sample of the global lattice t_k = (k + 1/2) dt.  Per sample, in float32,
// in the brick's stored-index coordinates re-anchored to a float64 position
// every kAnchor samples (keeps the float32 coordinates small, so position
// error stays ~1e-6 voxel even far from the brick origin): trilinear
// reconstruction, transfer-function lookup from an LDS table, emission-
// absorption update, early termination once T < eps.
//
// The checkpointing variant (used by the adjoint) runs without early
// termination and stores the transmittance in front of every
// ckpt_interval-th owned sample of each ray.
#include "march_common.h"

namespace dpvr {
namespace {

constexpr int kTile = 8;          // 8x8 pixels per wavefront

template <typename TS, bool kCkpt>
__global__ __launch_bounds__(64) void march_direct(MarchParams p) {
    __shared__ TFTable tft;
    const int lane = threadIdx.x;
    load_tf(tft, p.tf, p.dt, lane, 64);
    __syncthreads();

    const int tile = blockIdx.x;
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int lx = tx * kTile + (lane & 7), ly = ty * kTile + (lane >> 3);
    const bool valid = lx < p.roi_w && ly < p.roi_h;
    const int px = p.roi_x0 + lx, py = p.roi_y0 + ly;
    const long long pix = (long long)ly * p.roi_w + lx;

    const BrickK& b = p.brick;
    const TS* __restrict__ vox = reinterpret_cast<const TS*>(b.data);
    const int snx = b.sdim[0], sny = b.sdim[1], snz = b.sdim[2];
    const long long sxy = (long long)snx * sny;
    const float tf_k = 255.0f / (p.tf.vmax - p.tf.vmin);
    const float tf_o = -p.tf.vmin * tf_k;
    const float eps = kCkpt ? 0.0f : p.ert_eps;

    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
    float depth = INFINITY;
    long long evaluated = 0;
    RaySetup rs;
    if (valid && setup_ray(p.cam, b, p.dt, px, py, rs)) {
        depth = (float)(((double)rs.kf + 0.5) * p.dt);
        const Step st = make_step(rs, b, p.dt);
        for (long long kb = rs.kf; kb <= rs.kl; kb += kAnchor) {
            const Anchor an = make_anchor(rs, b, p.dt, kb);
            const int n = (int)min((long long)kAnchor, rs.kl - kb + 1);
            evaluated += n;
            for (int j = 0; j < n; ++j) {
                if (kCkpt) {
                    const long long q = kb + j - rs.kf;
                    if (q % p.ckpt_interval == 0 && q / p.ckpt_interval < p.ckpt_nseg)
                        p.ckpt[pix * p.ckpt_nseg + q / p.ckpt_interval] = T;
                }
                const Cell c = locate(an, st, j, snx, sny, snz);
                const float v = trilinear(vox, c, snx, sxy);
                const Classified e = classify(tft, v, tf_k, tf_o);
                // emission-absorption: T_next = T exp2(-a'), weight = T - T_next
                const float Tn = T * exp2f(-e.a);
                const float w = T - Tn;
                C0 = fmaf(w, e.r, C0);
                C1 = fmaf(w, e.g, C1);
                C2 = fmaf(w, e.b, C2);
                T = Tn;
                if (T < eps) {
                    evaluated -= n - 1 - j;   // samples of this block not taken
                    goto done;
                }
            }
        }
    }
done:
    if (valid) {
        reinterpret_cast<float4*>(p.out_rgba)[pix] = make_float4(C0, C1, C2, 1.0f - T);
        p.out_depth[pix] = depth;
    }
    if (p.samples) {
        // wave-wide sum, one atomic per wave
        unsigned long long cnt = (unsigned long long)evaluated;
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        if (lane == 0 && cnt) atomicAdd(p.samples, cnt);
    }
}

template <bool kCkpt>
hipError_t launch(const MarchParams& p, StorageK storage, hipStream_t stream) {
    const int blocks = p.tiles_x * p.tiles_y;
    if (blocks == 0) return hipSuccess;
    if (storage == kF16)
        hipLaunchKernelGGL((march_direct<__half, kCkpt>), dim3(blocks), dim3(64), 0, stream, p);
    else
        hipLaunchKernelGGL((march_direct<float, kCkpt>), dim3(blocks), dim3(64), 0, stream, p);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_march(const MarchParams& p, StorageK storage, hipStream_t stream) {
    return p.ckpt ? launch<true>(p, storage, stream) : launch<false>(p, storage, stream);
}

}  // namespace dpvr
