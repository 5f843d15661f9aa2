// Brick ingest for gfx950: copy the caller's ghost-padded float32 voxels into
// the brick's workspace at the brick's storage precision (float32, or IEEE
// binary16 rounded to nearest even), re-pitching rows to a multiple of 8
// elements (16-byte aligned rows for the staged march).  Pure streaming, one
// pass over HBM.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "dpvr_kernels.h"

namespace dpvr {
namespace {

// Re-pitch the caller's x-fastest voxels (row length snx) into the workspace
// (row pitch P = snx rounded up to 8, pad columns zeroed).  One thread per
// workspace element of a row block; reads and writes are both row-contiguous.
template <typename TD>
__global__ __launch_bounds__(256) void ingest_kernel(const float* __restrict__ src,
                                                     TD* __restrict__ dst, int snx, int pitch,
                                                     long long rows) {
    const long long total = rows * pitch;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long row = i / pitch;
        const int x = (int)(i - row * pitch);
        const float v = x < snx ? src[row * snx + x] : 0.0f;
        if constexpr (sizeof(TD) == 2)
            dst[i] = __float2half_rn(v);
        else
            dst[i] = v;
    }
}

// Gather a brick's ghost-padded box out of a global voxel array (indices
// clamped to the grid, i.e. edge replication at the domain boundary).  One
// thread per stored voxel, x fastest: reads of a stored row are one
// contiguous global row.
template <typename TD>
__global__ __launch_bounds__(256) void gather_kernel(GatherParams g, TD* __restrict__ dst) {
    const long long nx = g.sdim[0], ny = g.sdim[1], nz = g.sdim[2];
    const long long pitch = (nx + 7) & ~7LL;
    const long long total = pitch * ny * nz;
    const long long gnx = g.vol_dims[0], gny = g.vol_dims[1], gnz = g.vol_dims[2];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long sx = i % pitch, sy = (i / pitch) % ny, sz = i / (pitch * ny);
        const long long x = min(max((long long)g.lo[0] + sx - g.ghost, 0LL), gnx - 1);
        const long long y = min(max((long long)g.lo[1] + sy - g.ghost, 0LL), gny - 1);
        const long long z = min(max((long long)g.lo[2] + sz - g.ghost, 0LL), gnz - 1);
        const float v = sx < nx ? g.volume[(z * gny + y) * gnx + x] : 0.0f;
        if constexpr (sizeof(TD) == 2)
            dst[i] = __float2half_rn(v);
        else
            dst[i] = v;
    }
}

}  // namespace

hipError_t launch_gather(const GatherParams& g, void* dst, StorageK storage, hipStream_t stream) {
    const long long total = (long long)((g.sdim[0] + 7) & ~7) * g.sdim[1] * g.sdim[2];
    const long long want = (total + 255) / 256;
    const int blocks = (int)(want < 16384 ? want : 16384);
    if (blocks == 0) return hipSuccess;
    if (storage == kF16)
        hipLaunchKernelGGL(gather_kernel<__half>, dim3(blocks), dim3(256), 0, stream, g,
                           reinterpret_cast<__half*>(dst));
    else
        hipLaunchKernelGGL(gather_kernel<float>, dim3(blocks), dim3(256), 0, stream, g,
                           reinterpret_cast<float*>(dst));
    return hipGetLastError();
}

hipError_t launch_ingest(const float* src, void* dst, const int32_t sdim[3], StorageK storage,
                         hipStream_t stream) {
    const int snx = sdim[0];
    const int pitch = (snx + 7) & ~7;
    const long long rows = (long long)sdim[1] * sdim[2];
    const long long want = (rows * pitch + 255) / 256;
    const int blocks = (int)(want < 16384 ? want : 16384);
    if (blocks == 0) return hipSuccess;
    if (storage == kF16)
        hipLaunchKernelGGL(ingest_kernel<__half>, dim3(blocks), dim3(256), 0, stream, src,
                           reinterpret_cast<__half*>(dst), snx, pitch, rows);
    else
        hipLaunchKernelGGL(ingest_kernel<float>, dim3(blocks), dim3(256), 0, stream, src,
                           reinterpret_cast<float*>(dst), snx, pitch, rows);
    return hipGetLastError();
}

}  // namespace dpvr
