// Brick ingest for gfx950: copy the caller's ghost-padded float32 voxels into
// the brick's workspace at the brick's storage precision (float32, or IEEE
// binary16 rounded to nearest even).  Pure streaming: 16-byte loads, grid
// stride, one pass over HBM.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "dpvr_kernels.h"

namespace dpvr {
namespace {

__global__ __launch_bounds__(256) void ingest_f32(const float4* __restrict__ src,
                                                  float4* __restrict__ dst, long long n4) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void ingest_f16(const float4* __restrict__ src,
                                                  uint2* __restrict__ dst, long long n4) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (long long)gridDim.x * blockDim.x) {
        const float4 v = src[i];
        const __half h0 = __float2half_rn(v.x), h1 = __float2half_rn(v.y);
        const __half h2 = __float2half_rn(v.z), h3 = __float2half_rn(v.w);
        uint2 o;
        o.x = (uint32_t)__half_as_ushort(h0) | ((uint32_t)__half_as_ushort(h1) << 16);
        o.y = (uint32_t)__half_as_ushort(h2) | ((uint32_t)__half_as_ushort(h3) << 16);
        dst[i] = o;
    }
}

__global__ void ingest_tail(const float* __restrict__ src, void* __restrict__ dst, long long from,
                            long long count, int storage) {
    const long long i = from + (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    if (storage == kF16)
        reinterpret_cast<__half*>(dst)[i] = __float2half_rn(src[i]);
    else
        reinterpret_cast<float*>(dst)[i] = src[i];
}

// Gather a brick's ghost-padded box out of a global voxel array (indices
// clamped to the grid, i.e. edge replication at the domain boundary).  One
// thread per stored voxel, x fastest: reads of a stored row are one
// contiguous global row.
template <typename TD>
__global__ __launch_bounds__(256) void gather_kernel(GatherParams g, TD* __restrict__ dst) {
    const long long nx = g.sdim[0], ny = g.sdim[1], nz = g.sdim[2];
    const long long total = nx * ny * nz;
    const long long gnx = g.vol_dims[0], gny = g.vol_dims[1], gnz = g.vol_dims[2];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long sx = i % nx, sy = (i / nx) % ny, sz = i / (nx * ny);
        const long long x = min(max((long long)g.lo[0] + sx - g.ghost, 0LL), gnx - 1);
        const long long y = min(max((long long)g.lo[1] + sy - g.ghost, 0LL), gny - 1);
        const long long z = min(max((long long)g.lo[2] + sz - g.ghost, 0LL), gnz - 1);
        const float v = g.volume[(z * gny + y) * gnx + x];
        if constexpr (sizeof(TD) == 2)
            dst[i] = __float2half_rn(v);
        else
            dst[i] = v;
    }
}

}  // namespace

hipError_t launch_gather(const GatherParams& g, void* dst, StorageK storage, hipStream_t stream) {
    const long long total = (long long)g.sdim[0] * g.sdim[1] * g.sdim[2];
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

hipError_t launch_ingest(const float* src, void* dst, int64_t count, StorageK storage,
                         hipStream_t stream) {
    // vector body needs 16-byte aligned source; the workspace is 256-byte aligned
    const bool aligned = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
    const long long n4 = aligned ? count / 4 : 0;
    if (n4 > 0) {
        const long long want = (n4 + 255) / 256;
        const int blocks = (int)(want < 8192 ? want : 8192);
        if (storage == kF16)
            hipLaunchKernelGGL(ingest_f16, dim3(blocks), dim3(256), 0, stream,
                               reinterpret_cast<const float4*>(src), reinterpret_cast<uint2*>(dst),
                               n4);
        else
            hipLaunchKernelGGL(ingest_f32, dim3(blocks), dim3(256), 0, stream,
                               reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst),
                               n4);
    }
    const long long from = n4 * 4;
    if (from < count) {
        const long long rest = count - from;
        hipLaunchKernelGGL(ingest_tail, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, stream,
                           src, dst, from, (long long)count, (int)storage);
    }
    return hipGetLastError();
}

}  // namespace dpvr
