// Ray-queue cycling (RQC) on one GPU, with shadow rays.
//
// The bricks play the ranks of a data-parallel renderer: every ray is
// traced through every brick's data by cycling ray queues from brick to
// brick, so the data never moves and its decomposition can be arbitrary.
// One directional light: each primary sample's emitted colour is scaled by
// a0 + (1 - a0) S, S the transmittance of its shadow ray toward the light,
// which has to visit the bricks that hold the occluders.
//
// A frame, for n bricks (ranks) and the context camera:
//   plan      one entry per (brick b, ROI pixel of b): the first owned sample
//             index of the pixel's ray in b and the number of owned samples;
//             an exclusive scan gives every owned primary sample a slot.
//   shadow    n cycle steps.  The shadow rays spawned by the samples that
//             brick b owns form b's queue; in step s that queue is traced
//             through brick (b + s) mod n, multiplying each ray's
//             transmittance in its slot (products commute, so the cycle order
//             does not matter to the value).
//   primary   n cycle steps.  The primary ray of pixel (x, y) starts at brick
//             h = (x / 8 + y / 8) mod n; in step s it is traced through
//             brick (h + s) mod n, giving the segment (premultiplied colour,
//             alpha, depth key) of the samples that brick owns, with the
//             shaded emission; segments go to the pixel's slot of that brick.
//   resolve   per pixel, the n segments in (key, brick index) order with
//             "over", then the background.
// For emission-absorption on disjoint bricks this equals sort-last
// compositing of per-brick partials: with shadows off (a0 = 1) every segment
// is bit-identical to the brick's partial pixel and the resolve repeats the
// composite's arithmetic, so the image equals the sort-last image exactly.
#include "march_common.h"

namespace dpvr {
namespace {

constexpr int kScanBlock = 1024;     // elements per workgroup of the scan (256 threads x 4)

// Brick of an entry: the largest b with entry0[b] <= e.
__device__ inline int brick_of_entry(const RqcParams& p, long long e) {
    int lo = 0, hi = p.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.bricks[mid].entry0 <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Entry of a sample slot: the largest e with offsets[e] <= q.
__device__ inline long long entry_of_slot(const RqcParams& p, long long q) {
    long long lo = 0, hi = p.n_entries - 1;
    while (lo < hi) {
        const long long mid = (lo + hi + 1) >> 1;
        if (p.offsets[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// entry_of_slot for the active lanes of a wavefront whose slots are
// consecutive (lane i holds the lowest active slot + i or fewer): two
// wavefront-uniform searches bound the entries of the wavefront's slots, and
// each lane searches only between them.
__device__ inline long long entry_of_slot_wave(const RqcParams& p, long long q) {
    const unsigned lo32 = __builtin_amdgcn_readfirstlane((unsigned)q);
    const unsigned hi32 = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)q >> 32));
    const long long q0 = (long long)(((unsigned long long)hi32 << 32) | lo32);   // the first active lane's slot
    long long lo = entry_of_slot(p, q0);
    long long hi = entry_of_slot(p, q0 + 63);
    while (lo < hi) {
        const long long mid = (lo + hi + 1) >> 1;
        if (p.offsets[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Adds every lane's n to *counter (one atomic per wavefront); all lanes of
// the wavefront must call it.
__device__ inline void count_samples(unsigned long long* counter, unsigned long long n) {
    if (!counter) return;
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(counter, n);
}

// ----------------------------------------------------------------- plan
__global__ __launch_bounds__(256) void rqc_count(RqcParams p) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p.n_entries) return;
    const int b = brick_of_entry(p, e);
    const RqcBrick& rb = p.bricks[b];
    const long long r = e - rb.entry0;
    const int px = rb.roi_x0 + (int)(r % rb.roi_w), py = rb.roi_y0 + (int)(r / rb.roi_w);
    RaySetup rs;
    long long cnt = 0;
    int kf = -1;
    if (setup_ray(p.cam, rb.brick, p.dt, px, py, rs)) {
        if (rs.kl > 0x7fffffffLL) {
            if (p.err) atomicOr(p.err, kErrRange);
        } else {
            cnt = rs.kl - rs.kf + 1;
            kf = (int)rs.kf;
        }
    }
    p.kf[e] = kf;
    p.offsets[e] = cnt;
}

// Exclusive scan of offsets[0 .. n) in place (offsets[n] = total), in three
// launches: per-block scans with block totals, a scan of the totals, and the
// block carries added back.
__global__ __launch_bounds__(256) void scan_blocks(long long* v, long long n, long long* sums) {
    __shared__ long long s[256];
    const long long base = (long long)blockIdx.x * kScanBlock + threadIdx.x * 4;
    long long x[4], run = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[i] = base + i < n ? v[base + i] : 0;
        run += x[i];
    }
    s[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {      // inclusive scan of the thread totals
        const long long add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    long long acc = s[threadIdx.x] - run;          // exclusive prefix of this thread
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) v[base + i] = acc;
        acc += x[i];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = s[255];
}

__global__ __launch_bounds__(256) void scan_sums(long long* sums, long long nb, long long* total) {
    __shared__ long long s[256];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (long long b0 = 0; b0 < nb; b0 += 256) {
        const long long i = b0 + threadIdx.x;
        const long long x = i < nb ? sums[i] : 0;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const long long add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + s[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 255) carry += s[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void scan_add(long long* v, long long n, const long long* sums) {
    const long long i = (long long)blockIdx.x * kScanBlock + threadIdx.x;
    const long long c = sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (i + k * 256 < n) v[i + k * 256] += c;
}

// ------------------------------------------------------ one brick's samples
// The 8 corner values of cell c, in lerp3's order.
template <typename TS>
__device__ inline void corners(const TS* __restrict__ vox, const Cell& c, int pitch, long long sxy, float (&v)[8]) {
    const long long base = (long long)c.iz * sxy + (long long)c.iy * pitch + c.ix;
    v[0] = ld(vox, base);
    v[1] = ld(vox, base + 1);
    v[2] = ld(vox, base + pitch);
    v[3] = ld(vox, base + pitch + 1);
    v[4] = ld(vox, base + sxy);
    v[5] = ld(vox, base + sxy + 1);
    v[6] = ld(vox, base + sxy + pitch);
    v[7] = ld(vox, base + sxy + pitch + 1);
}

// The samples kf .. kl of ray rs in brick b, block by block as the partial
// march takes them (same anchors, same float32 positions, same trilinear
// arithmetic), each passed to fn(k, value); the next sample's corner loads
// are issued before fn runs on the current one, so their latency overlaps
// its work.  Returns false if fn stops the walk.
template <typename TS, typename Fn>
__device__ inline bool walk(const BrickK& b, double dt, double inv_dt, const RaySetup& rs, Fn fn) {
    const TS* __restrict__ vox = reinterpret_cast<const TS*>(b.data);
    const int snx = b.sdim[0], sny = b.sdim[1], snz = b.sdim[2];
    const int pitch = row_pitch(snx);
    const long long sxy = (long long)pitch * sny;
    const Step st = make_step(rs, b, dt);
    const Blocks bl = make_blocks(rs, b);
    long long n = block_of(bl, dt, inv_dt, rs.kf);
    long long k = rs.kf;
    while (k <= rs.kl) {
        const long long knext = block_start(bl, inv_dt, n + 1);
        const long long kend = min(knext - 1, rs.kl);
        if (kend >= k) {
            const Anchor an = make_anchor(rs, b, dt, k);
            float fj = 0.0f;
            Cell c = locate(an, st, fj, snx, sny, snz);
            float v[8];
            corners(vox, c, pitch, sxy, v);
            for (long long kk = k; kk <= kend; ++kk) {
                const Cell cur = c;
                const float w[8] = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
                if (kk < kend) {
                    fj += 1.0f;
                    c = locate(an, st, fj, snx, sny, snz);
                    corners(vox, c, pitch, sxy, v);
                }
                if (!fn(kk, lerp3(cur, w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7]))) return false;
            }
            k = kend + 1;
        }
        ++n;
    }
    return true;
}

// --------------------------------------------------------------- shadows
// Step s: every owned primary sample's shadow ray through brick
// (home + s) mod n; slot q holds its transmittance.
__global__ __launch_bounds__(256) void rqc_shadow_step(RqcParams p) {
    __shared__ TFTable tft;
    load_tf(tft, p.tf, p.dt, threadIdx.x, blockDim.x);
    __syncthreads();
    const float tf_k = 255.0f / (p.tf.vmax - p.tf.vmin);
    const float tf_o = -p.tf.vmin * tf_k;
    unsigned long long evaluated = 0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < p.total;
         q += (long long)gridDim.x * blockDim.x) {
        const long long e = entry_of_slot_wave(p, q);
        const int h = brick_of_entry(p, e);
        const RqcBrick& home = p.bricks[h];
        const RqcBrick& at = p.bricks[(h + p.step) % p.n];
        const long long r = e - home.entry0;
        const int px = home.roi_x0 + (int)(r % home.roi_w), py = home.roi_y0 + (int)(r / home.roi_w);
        const long long k = (long long)p.kf[e] + (q - p.offsets[e]);
        const CamRay cr = camera_ray(p.cam, px, py);
        double x0, x1, x2;
        {
#pragma clang fp contract(off)
            const double t = ((double)k + 0.5) * p.dt;
            x0 = cr.o[0] + t * cr.d[0];
            x1 = cr.o[1] + t * cr.d[1];
            x2 = cr.o[2] + t * cr.d[2];
        }
        float T = 1.0f;
        RaySetup rs;
        if (setup_ray_from(x0, x1, x2, p.light[0], p.light[1], p.light[2], at.brick, p.dt, rs)) {
            auto absorb = [&](long long, float v) {
                T = T * trans_exp2(-classify(tft, v, tf_k, tf_o).a);
                ++evaluated;
                return true;
            };
            if (at.storage == kF16)
                walk<__half>(at.brick, p.dt, p.inv_dt, rs, absorb);
            else
                walk<float>(at.brick, p.dt, p.inv_dt, rs, absorb);
        }
        p.shade[q] = p.step == 0 ? T : p.shade[q] * T;
    }
    count_samples(p.samples, evaluated);
}

// --------------------------------------------------------------- primary
// Step s: the primary ray of every frame pixel through brick (home + s) mod
// n, home = (x / 8 + y / 8) mod n; its segment (key, C, alpha) goes to the
// pixel's slot of that brick.  The accumulation is the partial march's
// (emission-absorption, the same early-termination rule), the emitted colour
// scaled by a0 + (1 - a0) S.
__global__ __launch_bounds__(256) void rqc_primary_step(RqcParams p) {
    __shared__ TFTable tft;
    load_tf(tft, p.tf, p.dt, threadIdx.x, blockDim.x);
    __syncthreads();
    const long long npx = (long long)p.width * p.height;
    const long long pix = min((long long)blockIdx.x * blockDim.x + threadIdx.x, npx - 1);
    const bool live = (long long)blockIdx.x * blockDim.x + threadIdx.x < npx;   // the rest mirror the last pixel
    const int px = (int)(pix % p.width), py = (int)(pix / p.width);
    const int c = ((px / 8 + py / 8) % p.n + p.step) % p.n;
    const RqcBrick& rb = p.bricks[c];
    const float tf_k = 255.0f / (p.tf.vmax - p.tf.vmin);
    const float tf_o = -p.tf.vmin * tf_k;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f, key = INFINITY;
    unsigned long long evaluated = 0;
    const int lx = px - rb.roi_x0, ly = py - rb.roi_y0;
    RaySetup rs;
    if (live && lx >= 0 && ly >= 0 && lx < rb.roi_w && ly < rb.roi_h &&
        setup_ray(p.cam, rb.brick, p.dt, px, py, rs)) {
        key = (float)(((double)rs.kf + 0.5) * p.dt);
        const long long q0 = p.offsets[rb.entry0 + (long long)ly * rb.roi_w + lx];
        const float a0 = p.ambient, a1 = 1.0f - p.ambient;
        auto accumulate = [&](long long k, float v) {
#pragma clang fp contract(off)
            const Classified e = classify(tft, v, tf_k, tf_o);
            float f = 1.0f;
            if (p.shadows) f = a0 + a1 * p.shade[q0 + (k - rs.kf)];
            const float Tn = T * trans_exp2(-e.a);
            const float w = T - Tn;
            C0 = fmaf(w, e.r * f, C0);
            C1 = fmaf(w, e.g * f, C1);
            C2 = fmaf(w, e.b * f, C2);
            T = Tn;
            ++evaluated;
            // the partial march tests termination after odd offsets
            return !(((k - rs.kf) & 1) && T < p.ert_eps);
        };
        if (rb.storage == kF16)
            walk<__half>(rb.brick, p.dt, p.inv_dt, rs, accumulate);
        else
            walk<float>(rb.brick, p.dt, p.inv_dt, rs, accumulate);
    }
    count_samples(p.samples, evaluated);
    if (!live) return;
    float* sg = p.segs + (pix * p.n + c) * 5;
    sg[0] = key;
    sg[1] = C0;
    sg[2] = C1;
    sg[3] = C2;
    sg[4] = 1.0f - T;
}

// --------------------------------------------------------------- resolve
// The pixel's n segments with finite keys in (key, brick index) order, each
// "over" the result so far, then over the background (the composite's
// arithmetic).
__global__ __launch_bounds__(256) void rqc_resolve(RqcParams p) {
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= (long long)p.width * p.height) return;
    const float* sg = p.segs + pix * p.n * 5;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
    float lk = -INFINITY;
    int li = -1;
    for (int m = 0; m < p.n; ++m) {
        float bk = INFINITY;
        int bi = -1;
        for (int c = 0; c < p.n; ++c) {
            const float z = sg[c * 5];
            const bool after = z > lk || (z == lk && c > li);
            if (z < INFINITY && after && (z < bk || (z == bk && c < bi))) {
                bk = z;
                bi = c;
            }
        }
        if (bi < 0) break;
        const float w = 1.0f - A;
        C0 = fmaf(w, sg[bi * 5 + 1], C0);
        C1 = fmaf(w, sg[bi * 5 + 2], C1);
        C2 = fmaf(w, sg[bi * 5 + 3], C2);
        A = fmaf(w, sg[bi * 5 + 4], A);
        lk = bk;
        li = bi;
    }
    const float w = 1.0f - A;
    reinterpret_cast<float4*>(p.out)[pix] =
        make_float4(fmaf(w, p.bg[0], C0), fmaf(w, p.bg[1], C1), fmaf(w, p.bg[2], C2), fmaf(w, p.bg[3], A));
}

inline int grid_for(long long n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_exclusive_scan(long long* v, long long n, long long* sums, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const long long nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(scan_blocks, dim3((unsigned)nb), dim3(256), 0, stream, v, n, sums);
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(256), 0, stream, sums, nb, v + n);
    hipLaunchKernelGGL(scan_add, dim3((unsigned)nb), dim3(256), 0, stream, v, n, sums);
    return hipGetLastError();
}

long long scan_blocks(long long n) { return (n + kScanBlock - 1) / kScanBlock; }

hipError_t launch_rqc_plan(const RqcParams& p, long long* scan_sums_buf, long long* total, hipStream_t stream) {
    if (p.n_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(rqc_count, dim3(grid_for(p.n_entries, 256)), dim3(256), 0, stream, p);
    (void)total;   // the scan leaves the total in p.offsets[n_entries]
    return launch_exclusive_scan(p.offsets, p.n_entries, scan_sums_buf, stream);
}

long long rqc_scan_blocks(long long n_entries) { return scan_blocks(n_entries); }

hipError_t launch_rqc_frame(RqcParams p, int cus, hipStream_t stream) {
    const long long npx = (long long)p.width * p.height;
    if (p.shadows && p.total > 0) {
        const int grid = (int)min((long long)cus * 8, (p.total + 255) / 256);
        for (int s = 0; s < p.n; ++s) {
            p.step = s;
            hipLaunchKernelGGL(rqc_shadow_step, dim3(grid), dim3(256), 0, stream, p);
        }
    }
    for (int s = 0; s < p.n; ++s) {
        p.step = s;
        hipLaunchKernelGGL(rqc_primary_step, dim3(grid_for(npx, 256)), dim3(256), 0, stream, p);
    }
    hipLaunchKernelGGL(rqc_resolve, dim3(grid_for(npx, 256)), dim3(256), 0, stream, p);
    return hipGetLastError();
}

}  // namespace dpvr
