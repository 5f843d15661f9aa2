// Sort-last compositing of partial images for gfx950.
//
// One wavefront per 8x8 pixel tile, one lane per pixel.  The wave first
// tests every partial's region of interest against the tile (wave-uniform
// scalar work) and skips partials whose ROI misses it; a ballot then skips
// partials that are empty (depth +inf) on every lane of the tile.  Each lane
// inserts the finite depth keys of its pixel into a sorted list held in LDS
// (stable: equal keys keep the lower partial index first), then composites
// front to back with "over" and finally over the background.
#include <hip/hip_runtime.h>
#include <math.h>

#include "dpvr_kernels.h"

namespace dpvr {
namespace {

// Sorted list of the finite depth keys of this lane's pixel, in LDS
// (column `lane` of key_s / idx_s); returns its length.  Every lane of the
// wave must call it (it votes with __ballot).
__device__ int sort_keys(const CompositeParams& p, int t0x, int t0y, int px, int py, bool valid,
                         int lane, float* key_s, unsigned char* idx_s) {
    int m = 0;   // number of finite keys of this pixel
    for (int c = 0; c < p.n; ++c) {
        const PartialK& q = p.parts[c];
        // wave-uniform: does the ROI overlap this tile at all?
        if (q.w <= 0 || q.h <= 0 || q.x0 >= t0x + 8 || q.x0 + q.w <= t0x || q.y0 >= t0y + 8 ||
            q.y0 + q.h <= t0y)
            continue;
        float z = INFINITY;
        const int lx = px - q.x0, ly = py - q.y0;
        if (valid && lx >= 0 && ly >= 0 && lx < q.w && ly < q.h) z = q.depth[(long long)ly * q.w + lx];
        const bool finite = z < INFINITY;
        if (__ballot(finite) == 0) continue;
        if (finite) {
            int pos = m;
            while (pos > 0 && key_s[(pos - 1) * 64 + lane] > z) {
                key_s[pos * 64 + lane] = key_s[(pos - 1) * 64 + lane];
                idx_s[pos * 64 + lane] = idx_s[(pos - 1) * 64 + lane];
                --pos;
            }
            key_s[pos * 64 + lane] = z;
            idx_s[pos * 64 + lane] = (unsigned char)c;
            ++m;
        }
    }
    return m;
}

// One 8x8 tile of one frame (one wavefront).
__device__ inline void composite_tile(const CompositeParams& p, int tile, float* key_s,
                                      unsigned char* idx_s) {
    const int lane = threadIdx.x;
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int t0x = tx * 8, t0y = ty * 8;
    const int px = t0x + (lane & 7), py = t0y + (lane >> 3);
    const bool valid = px < p.width && py < p.height;
    const int m = sort_keys(p, t0x, t0y, px, py, valid, lane, key_s, idx_s);
    if (!valid) return;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
    for (int k = 0; k < m; ++k) {
        const PartialK& q = p.parts[idx_s[k * 64 + lane]];
        const long long o = (long long)(py - q.y0) * q.w + (px - q.x0);
        const float4 s = reinterpret_cast<const float4*>(q.rgba)[o];
        const float w = 1.0f - A;
        C0 = fmaf(w, s.x, C0);
        C1 = fmaf(w, s.y, C1);
        C2 = fmaf(w, s.z, C2);
        A = fmaf(w, s.w, A);
    }
    const float w = 1.0f - A;
    reinterpret_cast<float4*>(p.out)[(long long)py * p.width + px] =
        make_float4(fmaf(w, p.bg[0], C0), fmaf(w, p.bg[1], C1), fmaf(w, p.bg[2], C2),
                    fmaf(w, p.bg[3], A));
}

__global__ __launch_bounds__(64) void composite_kernel(CompositeParams p) {
    __shared__ float key_s[kMaxPartials * 64];
    __shared__ unsigned char idx_s[kMaxPartials * 64];
    composite_tile(p, blockIdx.x, key_s, idx_s);
}

// Many frames in one launch: workgroup b composites tile b - tile_start[i]
// of frame i (the last i with tile_start[i] <= b); frame descriptors in
// device memory.
__global__ __launch_bounds__(64) void composite_many_kernel(const CompositeParams* __restrict__ frames,
                                                            const int32_t* __restrict__ tile_start,
                                                            int32_t n_frames) {
    __shared__ float key_s[kMaxPartials * 64];
    __shared__ unsigned char idx_s[kMaxPartials * 64];
    const int b = blockIdx.x;
    int lo = 0, hi = n_frames - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    composite_tile(frames[lo], b - tile_start[lo], key_s, idx_s);
}

// Backward of the composite.  With the partials of a pixel in visibility
// order, P_k = prod_{j<k} (1 - A_j) and S_k = what lies behind partial k
// composited over the background (S_{m-1} = bg, S_{k-1} = X_k + (1 - A_k) S_k):
//   dL/dC_k = g_rgb P_k,
//   dL/dA_k = P_k (g_a (1 - S_k,a) - g_rgb . S_k,rgb).
// Partials whose key is +inf at a pixel of their ROI get a zero gradient.
__global__ __launch_bounds__(64) void composite_backward_kernel(CompositeParams p,
                                                                CompositeBackParams bp) {
    __shared__ float key_s[kMaxPartials * 64];
    __shared__ unsigned char idx_s[kMaxPartials * 64];
    const int lane = threadIdx.x;
    const int tile = blockIdx.x;
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int t0x = tx * 8, t0y = ty * 8;
    const int px = t0x + (lane & 7), py = t0y + (lane >> 3);
    const bool valid = px < p.width && py < p.height;
    const int m = sort_keys(p, t0x, t0y, px, py, valid, lane, key_s, idx_s);
    if (!valid) return;
    // zero every covering partial's gradient at this pixel first
    for (int c = 0; c < p.n; ++c) {
        const PartialK& q = p.parts[c];
        const int lx = px - q.x0, ly = py - q.y0;
        if (lx >= 0 && ly >= 0 && lx < q.w && ly < q.h)
            reinterpret_cast<float4*>(bp.d_parts[c])[(long long)ly * q.w + lx] =
                make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // prefix transmittance P_k, kept in key_s (the keys are no longer needed)
    float P = 1.0f;
    for (int k = 0; k < m; ++k) {
        const PartialK& q = p.parts[idx_s[k * 64 + lane]];
        const float4 s = reinterpret_cast<const float4*>(q.rgba)[(long long)(py - q.y0) * q.w + (px - q.x0)];
        key_s[k * 64 + lane] = P;
        P = P * (1.0f - s.w);
    }
    const float4 g = reinterpret_cast<const float4*>(bp.d_out)[(long long)py * p.width + px];
    float S0 = p.bg[0], S1 = p.bg[1], S2 = p.bg[2], S3 = p.bg[3];
    for (int k = m - 1; k >= 0; --k) {
        const int c = idx_s[k * 64 + lane];
        const PartialK& q = p.parts[c];
        const long long o = (long long)(py - q.y0) * q.w + (px - q.x0);
        const float4 s = reinterpret_cast<const float4*>(q.rgba)[o];
        const float Pk = key_s[k * 64 + lane];
        const float dA = Pk * (g.w * (1.0f - S3) - g.x * S0 - g.y * S1 - g.z * S2);
        reinterpret_cast<float4*>(bp.d_parts[c])[o] = make_float4(g.x * Pk, g.y * Pk, g.z * Pk, dA);
        const float om = 1.0f - s.w;
        S0 = fmaf(om, S0, s.x);
        S1 = fmaf(om, S1, s.y);
        S2 = fmaf(om, S2, s.z);
        S3 = fmaf(om, S3, s.w);
    }
}

}  // namespace

hipError_t launch_composite_backward(const CompositeParams& p, const CompositeBackParams& bp,
                                     hipStream_t stream) {
    const int tiles_y = (p.height + 7) / 8;
    const int blocks = p.tiles_x * tiles_y;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(composite_backward_kernel, dim3(blocks), dim3(64), 0, stream, p, bp);
    return hipGetLastError();
}

hipError_t launch_composite_many(const CompositeParams* frames, const int32_t* tile_start,
                                 int32_t n_frames, int32_t total_tiles, hipStream_t stream) {
    if (total_tiles <= 0 || n_frames <= 0) return hipSuccess;
    hipLaunchKernelGGL(composite_many_kernel, dim3(total_tiles), dim3(64), 0, stream, frames,
                       tile_start, n_frames);
    return hipGetLastError();
}

hipError_t launch_composite(const CompositeParams& p, hipStream_t stream) {
    const int tiles_y = (p.height + 7) / 8;
    const int blocks = p.tiles_x * tiles_y;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(composite_kernel, dim3(blocks), dim3(64), 0, stream, p);
    return hipGetLastError();
}

}  // namespace dpvr
