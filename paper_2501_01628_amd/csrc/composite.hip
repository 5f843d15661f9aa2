// Sort-last compositing of partial images for gfx950.
//
// Forward: a 256-thread workgroup composites a 64 x 4 pixel block, one
// wavefront per 64 consecutive pixels of a row, so that every partial's row
// segment is one contiguous run (256 B of depth keys, 1 KB of colour).
// Partials whose ROI misses the wave's row segment are skipped by a
// wave-uniform test.  A pass reads the depth key and the colour of every
// covering partial together (kBatch partials' loads in flight at once) and
// keeps, in registers, the kList smallest entries in (key, partial index)
// order that come after the last entry already composited; those are
// composited front to back with "over".  A pixel with more than kList finite
// keys takes further passes; the frame pixel is finally "over" the
// background.  Ties between equal keys go to the lower partial index first.
//
// Backward: one wavefront per 8x8 tile with the key lists in LDS.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>

#include "dpvr_kernels.h"

namespace dpvr {
namespace {

constexpr int kList = 4;
constexpr int kBatch = 2;

// Word 3 of a raw (untyped, unswizzled) buffer resource on gfx9-family
// chips: 32-bit data format; with stride 0 an access at or past the
// resource's byte size returns zero and reads nothing.
constexpr int kRawBuffer = 0x00020000;

static_assert(kMaxPartials <= 64, "one lane per partial in the overlap vote");
static_assert(offsetof(PartialK, x0) == 0 && offsetof(PartialK, h) == 12, "ROI read as one int4: x0, y0, w, h");

// One 64-pixel row segment (this wave's) of one frame.
__device__ inline void composite_row(const CompositeParams& p, int bx, int by) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sx0 = bx * 64;
    const int px = sx0 + lane, py = by * 4 + wave;
    if (py >= p.height) return;                 // (wave-uniform)
    const bool valid = px < p.width;
    // lane c reads partial c's ROI (one 16-byte load per lane) and votes for
    // it when the ROI holds part of this row segment; a pass then reads the
    // descriptors of the partials it visits with scalar loads
    int4 roi = make_int4(0, 0, 0, 0);
    if (lane < p.n) roi = *reinterpret_cast<const int4*>(&p.parts[lane]);
    const bool hit = (roi.z > 0) & (roi.w > 0) & (py >= roi.y) & (py < roi.y + roi.w) & (roi.x < sx0 + 64) &
                     (roi.x + roi.z > sx0);
    const unsigned long long covering = __ballot(hit);
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
    float lk = -INFINITY;                       // (key, index) of the last composited entry
    int li = -1;
    bool active = valid;
    while (__ballot(active) != 0) {
        float key[kList];
        int idx[kList];
        float4 val[kList];
#pragma unroll
        for (int s = 0; s < kList; ++s) {
            key[s] = INFINITY;
            idx[s] = 0;
            val[s] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        int cnt = 0;   // entries after (lk, li) at this pixel
        unsigned long long rest = covering;
        while (rest != 0) {
            // the next kBatch covering partials in index order; slots past
            // the last repeat the first and are masked (use[u] false), so
            // that every load of the batch is issued without a branch
            int cs[kBatch];
            bool use[kBatch];
            const int first = __builtin_ctzll(rest);
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                use[u] = rest != 0;
                cs[u] = use[u] ? __builtin_ctzll(rest) : first;
                rest &= rest - 1;
            }
            float z[kBatch];
            float4 v[kBatch];
            unsigned zraw[kBatch];
            bool inside[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int c = cs[u];
                const PartialK q = p.parts[c];
                const int qx0 = q.x0;
                const int qw = q.w;
                const float4* rgba = reinterpret_cast<const float4*>(q.rgba);
                const float* depth = q.depth;
                const int lx = px - qx0;
                const bool in = use[u] & active & (lx >= 0) & (lx < qw);
                // the row lies inside the ROI (the partial covers this row
                // segment): buffer loads over that one row, addressed by the
                // lane's column; lanes off the ROI (and inactive lanes) ask
                // for column -1, which the buffer's range check turns into
                // zeros without a read
                const long long row = (long long)(py - q.y0) * qw;
                const int col = in ? lx : -1;
                const __amdgpu_buffer_rsrc_t rd =
                    __builtin_amdgcn_make_buffer_rsrc((void*)(depth + row), 0, qw * 4, kRawBuffer);
                const __amdgpu_buffer_rsrc_t rc =
                    __builtin_amdgcn_make_buffer_rsrc((void*)(rgba + row), 0, qw * 16, kRawBuffer);
                zraw[u] = __builtin_amdgcn_raw_buffer_load_b32(rd, col * 4, 0, 0);
                const auto vv = __builtin_amdgcn_raw_buffer_load_b128(rc, col * 16, 0, 0);
                v[u] = make_float4(__uint_as_float(vv[0]), __uint_as_float(vv[1]), __uint_as_float(vv[2]),
                                   __uint_as_float(vv[3]));
                inside[u] = in;
            }
            // off the ROI the load returned 0, which or-ing turns into the
            // bits of +inf (an unconditional use of every load, so that none
            // is deferred behind a branch)
#pragma unroll
            for (int u = 0; u < kBatch; ++u) z[u] = __uint_as_float(zraw[u] | (inside[u] ? 0u : 0x7f800000u));
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int c = cs[u];
                const bool take = z[u] < INFINITY && (z[u] > lk || (z[u] == lk && c > li));
                if (__ballot(take) == 0) continue;     // no lane takes it (wave-uniform)
                cnt += take;
                // insert (branch-free; an entry not taken enters as +inf and
                // moves nothing): entries compare by (key, index), so that an
                // entry displaced from its slot lands before equal keys of
                // higher index; the largest drops out
                float nk = take ? z[u] : INFINITY;
                int ni = c;
                float4 nv = v[u];
#pragma unroll
                for (int s = 0; s < kList; ++s) {
                    const bool before = nk < key[s] || (nk == key[s] && ni < idx[s]);
                    const float tk = key[s];
                    const int ti = idx[s];
                    const float4 tv = val[s];
                    key[s] = before ? nk : tk;
                    idx[s] = before ? ni : ti;
                    val[s].x = before ? nv.x : tv.x;
                    val[s].y = before ? nv.y : tv.y;
                    val[s].z = before ? nv.z : tv.z;
                    val[s].w = before ? nv.w : tv.w;
                    nk = before ? tk : nk;
                    ni = before ? ti : ni;
                    nv.x = before ? tv.x : nv.x;
                    nv.y = before ? tv.y : nv.y;
                    nv.z = before ? tv.z : nv.z;
                    nv.w = before ? tv.w : nv.w;
                }
            }
        }
#pragma unroll
        for (int s = 0; s < kList; ++s) {
            if (s < cnt) {
                const float w = 1.0f - A;
                C0 = fmaf(w, val[s].x, C0);
                C1 = fmaf(w, val[s].y, C1);
                C2 = fmaf(w, val[s].z, C2);
                A = fmaf(w, val[s].w, A);
            }
        }
        if (cnt > kList) {
            lk = key[kList - 1];
            li = idx[kList - 1];
        } else {
            active = false;
        }
    }
    if (!valid) return;
    const float w = 1.0f - A;
    reinterpret_cast<float4*>(p.out)[(long long)py * p.width + px] =
        make_float4(fmaf(w, p.bg[0], C0), fmaf(w, p.bg[1], C1), fmaf(w, p.bg[2], C2), fmaf(w, p.bg[3], A));
}

__global__ __launch_bounds__(256) void composite_kernel(CompositeParams p) {
    const int bxs = (p.width + 63) / 64;
    composite_row(p, blockIdx.x % bxs, blockIdx.x / bxs);
}

// Many frames in one launch: workgroup b composites block b - block_start[i]
// of frame i (the last i with block_start[i] <= b); frame descriptors in
// device memory.
__global__ __launch_bounds__(256) void composite_many_kernel(const CompositeParams* __restrict__ frames,
                                                            const int32_t* __restrict__ block_start,
                                                            int32_t n_frames) {
    const int b = blockIdx.x;
    int lo = 0, hi = n_frames - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block_start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const CompositeParams& p = frames[lo];
    const int local = b - block_start[lo];
    const int bxs = (p.width + 63) / 64;
    composite_row(p, local % bxs, local / bxs);
}

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

hipError_t launch_composite_many(const CompositeParams* frames, const int32_t* block_start,
                                 int32_t n_frames, int32_t total_blocks, hipStream_t stream) {
    if (total_blocks <= 0 || n_frames <= 0) return hipSuccess;
    hipLaunchKernelGGL(composite_many_kernel, dim3(total_blocks), dim3(256), 0, stream, frames,
                       block_start, n_frames);
    return hipGetLastError();
}

hipError_t launch_composite(const CompositeParams& p, hipStream_t stream) {
    const int blocks = composite_blocks(p.width, p.height);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(composite_kernel, dim3(blocks), dim3(256), 0, stream, p);
    return hipGetLastError();
}

}  // namespace dpvr
