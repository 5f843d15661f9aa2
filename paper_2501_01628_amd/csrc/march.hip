// Per-brick volume ray casting into a partial image (RGBA premultiplied +
// depth key) for gfx950.
//
// Per ray, in float64 and without FMA contraction (so that ownership
// decisions are bit-identical however the volume is split): camera ray, slab
// test against the brick's owned box, first/last owned sample of the global
// lattice t_k = (k + 1/2) dt.  Per sample, in float32, in the brick's
// stored-index coordinates re-anchored from float64 at the start of every
// anchor block (slab of kSlab slices, see march_common.h), so the float32
// coordinates stay small: trilinear reconstruction, transfer-function lookup
// from an LDS table, emission-absorption update, early termination once
// T < eps.
//
// Two kernels compute bit-identical images:
//  * march_staged (default): a 256-thread workgroup owns a 16x16 pixel tile,
//    one wavefront per 8x8 quarter.  The workgroup walks the slabs of the
//    tile's common slab axis w (y or z; rows along x stay contiguous in HBM)
//    in ray order; for each slab it stages, per slice, the sheared rectangle
//    the tile's rays cross (16-byte loads, converted to float32) into LDS,
//    then every lane marches its samples of that slab out of LDS.  Tiles
//    whose rays do not share a slab axis and direction, or whose slab does
//    not fit in LDS, march from HBM directly.
//  * march_direct: one wavefront per 8x8 tile, corner values straight from
//    HBM; also writes transmittance checkpoints for the adjoint.
#include "march_common.h"

namespace dpvr {
namespace {

constexpr int kSlices = kSlab + 3;       // staged slices per slab: [wlo - 1, whi + 1]
// Build-time sizes of the staged kernels: LDS floats of the slab stage and
// rows of the row table.  (64 KB measured best on C2: a 40 KB stage with
// 3 workgroups per CU ran within 3 %, a 24 KB stage with 4 per CU 20 %
// slower, from register spills and more sub-slabs.)
#ifndef DPVR_STAGE_FLOATS
#define DPVR_STAGE_FLOATS 16384          // 64 KB: 2 workgroups per CU
#endif
#ifndef DPVR_STAGE_ROWS
#define DPVR_STAGE_ROWS 1024
#endif
constexpr int kStageFloats = DPVR_STAGE_FLOATS;
constexpr int kMaxRows = DPVR_STAGE_ROWS;
constexpr float kMinStageDw = 0.25f;     // |d_w| below this: march from HBM

struct LaneState {
    float C0, C1, C2, T;
    long long evaluated;
    bool stopped;
};

// March samples kb + j0 .. kb + j1 - 1 of the anchor block anchored (float64)
// at sample kb; sample(fj) returns the interpolated value of sample kb + j
// (fj = j as float).  Returns false once early termination stops the ray.
// Two samples are fetched and classified before either is accumulated, so
// the memory round trips of consecutive samples overlap; accumulation stays
// in sample order.  Termination is tested after every sample whose offset
// from the ray's first owned sample is odd (the end of each pair of the ray),
// wherever the runs of a ray are cut, so every path stops a ray at the same
// sample; a ray may take one sample past T < eps, which changes its colour by
// less than eps.
template <bool kCkpt, typename Sample>
__device__ inline bool march_run(const MarchParams& p, const TFTable& tft, const RaySetup& rs,
                                 long long kb, int j0, int j1, long long pix, float tf_k,
                                 float tf_o, float eps, LaneState& s, Sample sample) {
    auto accumulate = [&](const Classified& e, int j) {
        // no contraction (T - T x must not become an FMA in some
        // instantiations only: every path rounds alike)
#pragma clang fp contract(off)
        if (kCkpt) {
            const long long q = kb + j - rs.kf;
            if (q % p.ckpt_interval == 0 && q / p.ckpt_interval < p.ckpt_nseg)
                p.ckpt[pix * p.ckpt_nseg + q / p.ckpt_interval] = s.T;
        }
        // emission-absorption: T_next = T exp2(-a'), weight = T - T_next
        const float Tn = s.T * trans_exp2(-e.a);
        const float w = s.T - Tn;
        s.C0 = fmaf(w, e.r, s.C0);
        s.C1 = fmaf(w, e.g, s.C1);
        s.C2 = fmaf(w, e.b, s.C2);
        s.T = Tn;
    };
    int j = j0;
    float fj = (float)j0;
    if (((kb + j0 - rs.kf) & 1) && j < j1) {   // second sample of a pair begun in the previous run
        accumulate(classify(tft, sample(fj), tf_k, tf_o), j);
        ++j;
        fj += 1.0f;
        if (s.T < eps) {
            s.evaluated += 1;
            s.stopped = true;
            return false;
        }
    }
    for (; j + 1 < j1; j += 2, fj += 2.0f) {
        const float v0 = sample(fj);
        const float v1 = sample(fj + 1.0f);
        const Classified e0 = classify(tft, v0, tf_k, tf_o);
        const Classified e1 = classify(tft, v1, tf_k, tf_o);
        accumulate(e0, j);
        accumulate(e1, j + 1);
        if (s.T < eps) {
            s.evaluated += j - j0 + 2;
            s.stopped = true;
            return false;
        }
    }
    // first sample of a pair: its test comes after the next sample (next run)
    if (j < j1) accumulate(classify(tft, sample(fj), tf_k, tf_o), j);
    s.evaluated += j1 - j0;
    return true;
}

// Whole ray from HBM, block by block.
template <typename TS, bool kCkpt>
__device__ inline void march_ray_direct(const MarchParams& p, const TFTable& tft,
                                        const RaySetup& rs, long long pix, float tf_k, float tf_o,
                                        float eps, LaneState& s) {
    const BrickK& b = p.brick;
    const TS* __restrict__ vox = reinterpret_cast<const TS*>(b.data);
    const int snx = b.sdim[0], sny = b.sdim[1], snz = b.sdim[2];
    const int pitch = row_pitch(snx);
    const long long sxy = (long long)pitch * sny;
    const Step st = make_step(rs, b, p.dt);
    const Blocks bl = make_blocks(rs, b);
    long long n = block_of(bl, p.dt, p.inv_dt, rs.kf);
    long long k = rs.kf;
    while (k <= rs.kl) {
        const long long knext = block_start(bl, p.inv_dt, n + 1);
        const long long kend = min(knext - 1, rs.kl);
        if (kend >= k) {
            const Anchor an = make_anchor(rs, b, p.dt, k);
            auto sample = [&](float fj) {
                return trilinear(vox, locate(an, st, fj, snx, sny, snz), pitch, sxy);
            };
            if (!march_run<kCkpt>(p, tft, rs, k, 0, (int)(kend - k + 1), pix, tf_k, tf_o, eps, s,
                                  sample))
                return;
            k = kend + 1;
        }
        ++n;
    }
}

__device__ inline void finish(const MarchParams& p, bool valid, long long pix, float depth,
                              const LaneState& s, int lane) {
    if (valid) {
        reinterpret_cast<float4*>(p.out_rgba)[pix] = make_float4(s.C0, s.C1, s.C2, 1.0f - s.T);
        p.out_depth[pix] = depth;
    }
    if (p.samples) {
        unsigned long long cnt = (unsigned long long)s.evaluated;
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        if (lane == 0 && cnt) atomicAdd(p.samples, cnt);
    }
}

// ------------------------------------------------------------ direct kernel
template <typename TS, bool kCkpt>
__global__ __launch_bounds__(64) void march_direct(MarchParams p) {
    __shared__ TFTable tft;
    const int lane = threadIdx.x;
    load_tf(tft, p.tf, p.dt, lane, 64);
    __syncthreads();

    const int tile = blockIdx.x;
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int lx = tx * 8 + (lane & 7), ly = ty * 8 + (lane >> 3);
    const bool valid = lx < p.roi_w && ly < p.roi_h;
    const long long pix = (long long)ly * p.roi_w + lx;
    const float tf_k = 255.0f / (p.tf.vmax - p.tf.vmin);
    const float tf_o = -p.tf.vmin * tf_k;
    const float eps = kCkpt ? 0.0f : p.ert_eps;

    LaneState s{0.f, 0.f, 0.f, 1.f, 0, false};
    float depth = INFINITY;
    RaySetup rs;
    if (valid && setup_ray(p.cam, p.brick, p.dt, p.roi_x0 + lx, p.roi_y0 + ly, rs)) {
        depth = (float)(((double)rs.kf + 0.5) * p.dt);
        march_ray_direct<TS, kCkpt>(p, tft, rs, pix, tf_k, tf_o, eps, s);
    }
    finish(p, valid, pix, depth, s, lane);
}

// ------------------------------------------------------------ staged kernel
// Workgroup-wide reduction of kRed values: wave reduction by shuffles, one
// LDS round trip (double-buffered by `buf`, so one barrier per call).
constexpr int kRed = 12;

template <int N>
__device__ inline void wg_reduce(float (&v)[N], const bool (&is_max)[N], float (*red)[4][kRed],
                                 int buf, int lane, int wave) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        float x = v[i];
        for (int off = 32; off > 0; off >>= 1) {
            const float y = __shfl_xor(x, off);
            x = is_max[i] ? fmaxf(x, y) : fminf(x, y);
        }
        v[i] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) red[buf][wave][i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        float x = red[buf][0][i];
        for (int w = 1; w < 4; ++w) x = is_max[i] ? fmaxf(x, red[buf][w][i]) : fminf(x, red[buf][w][i]);
        v[i] = x;
    }
}

// 16-byte staging vectors: load() from the brick in HBM (global address
// space: the loads count only against vmcnt), store() into the float32 stage
// (float16 decoded here).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 gu32x4;

template <typename TS>
struct StageVec;
template <>
struct StageVec<float> {
    static constexpr int V = 4;
    __device__ static u32x4 load(const float* src) { return *(gu32x4*)src; }
    __device__ static void store(const u32x4& raw, float* dst) {
        *reinterpret_cast<u32x4*>(dst) = raw;
    }
};
template <>
struct StageVec<__half> {
    static constexpr int V = 8;
    __device__ static u32x4 load(const __half* src) { return *(gu32x4*)src; }
    __device__ static void store(const u32x4& raw, float* dst) {
        const __half2* h = reinterpret_cast<const __half2*>(&raw);
        const float2 a = __half22float2(h[0]), b = __half22float2(h[1]);
        const float2 c = __half22float2(h[2]), d = __half22float2(h[3]);
        reinterpret_cast<float4*>(dst)[0] = make_float4(a.x, a.y, b.x, b.y);
        reinterpret_cast<float4*>(dst)[1] = make_float4(c.x, c.y, d.x, d.y);
    }
};

// LDS of a staged-march workgroup.
struct StagedShared {
    TFTable tft;
    __align__(16) float stage[kStageFloats];
    unsigned row_src[kMaxRows];          // element offset in the brick of each staged row
    int tab_off[kSlices];
    float red[2][4][kRed];
};

__device__ inline float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ inline int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Walk of one eligible tile through the slabs of its common slab axis W
// (2: z, rows along y; 1: y, rows along z) in ray order.  Per slab, a
// workgroup reduction gives the extent of the tile's rays in the slab; the
// slab (or each of its sub-slabs, when it does not fit) is staged into LDS
// slice by slice as sheared rectangles, then every lane marches its samples
// of it from LDS.
template <typename TS, int W>
__device__ void staged_walk(const MarchParams& p, StagedShared& sh, int& buf, const RaySetup& rs,
                            const Blocks& bl, bool has, int sg, long long pix, float tf_k,
                            float tf_o, float eps, LaneState& s) {
    constexpr int B = 3 - W;                 // the other of y (1) and z (2)
    constexpr int V = StageVec<TS>::V;
    const TFTable& tft = sh.tft;
    float* stage = sh.stage;
    int* tab_off = sh.tab_off;
    unsigned* row_src = sh.row_src;
    float (*red)[4][kRed] = sh.red;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const BrickK& b = p.brick;
    const TS* __restrict__ vox = reinterpret_cast<const TS*>(b.data);
    const int snx = b.sdim[0], sny = b.sdim[1], snz = b.sdim[2];
    const int pitch = row_pitch(snx);
    const long long sxy = (long long)pitch * sny;
    const int snw = b.sdim[W], snb = b.sdim[B];
    // slopes of x and b per unit of stored w along each ray
    float kx = 0.f, kb = 0.f;
    if (has) {
        const double dwu = rs.d[W] * b.inv_spacing[W];
        kx = (float)((rs.d[0] * b.inv_spacing[0]) / dwu);
        kb = (float)((rs.d[B] * b.inv_spacing[B]) / dwu);
    }
    const Step st = has ? make_step(rs, b, p.dt) : Step{0.f, 0.f, 0.f};
    long long n_cur = 0, k_cur = 0, k_next = 0;
    bool alive = has;
    if (has) {
        n_cur = block_of(bl, p.dt, p.inv_dt, rs.kf);
        k_cur = rs.kf;
        k_next = block_start(bl, p.inv_dt, n_cur + 1);
    }
    // first slab: the smallest block index of the tile
    long long n_chunk;
    {
        float v[1] = {has ? (float)n_cur : 3e38f};
        const bool mx[1] = {false};
        wg_reduce(v, mx, red, buf, lane, wave);
        buf ^= 1;
        n_chunk = (long long)uniform_f(v[0]);
    }
    const double gh = (double)b.ghost - 0.5;
    // slopes of all rays of the tile (constant along each ray)
    float kxmin, kxmax, kbmin, kbmax;
    {
        float v[4] = {has ? kx : 3e38f, has ? kx : -3e38f, has ? kb : 3e38f, has ? kb : -3e38f};
        const bool mx[4] = {false, true, false, true};
        wg_reduce(v, mx, red, buf, lane, wave);
        buf ^= 1;
        kxmin = uniform_f(v[0]); kxmax = uniform_f(v[1]);
        kbmin = uniform_f(v[2]); kbmax = uniform_f(v[3]);
    }
    const float Kx = fmaxf(fabsf(kxmin), fabsf(kxmax)), Kb = fmaxf(fabsf(kbmin), fabsf(kbmax));
    // at most snw / kSlab + 3 slabs intersect the brick; the bound only guards
    // against a logic error turning into a hang
    const int max_iter = 2 * (snw / kSlab + 4);
    for (int iter = 0; iter < max_iter; ++iter) {
        const bool part = alive && n_cur == n_chunk;
        // slab [wlo, wlo + kSlab] of stored w; crossing of plane wlo per ray
        const long long wlo = sg > 0 ? (long long)kSlab * n_chunk : -(long long)kSlab * (n_chunk + 1);
        float xr = 0.f, br = 0.f;
        if (part) {
#pragma clang fp contract(off)
            const double t = bl.c0 + (double)(sg > 0 ? n_chunk : n_chunk + 1) * bl.c1;
            xr = (float)((rs.o[0] + t * rs.d[0] - b.origin[0]) * b.inv_spacing[0] + gh);
            br = (float)((rs.o[B] + t * rs.d[B] - b.origin[B]) * b.inv_spacing[B] + gh);
        }
        // extent of the participating rays at the slab's entry plane, and the
        // next slab a ray that skips this one needs (none participates: the
        // max of x stays at -3e38)
        float v[5] = {part ? xr : 3e38f, part ? xr : -3e38f, part ? br : 3e38f, part ? br : -3e38f,
                      (alive && !part) ? (float)n_cur : 3e38f};
        const bool mx[5] = {false, true, false, true, false};
        wg_reduce(v, mx, red, buf, lane, wave);
        buf ^= 1;
        const float xmin0 = uniform_f(v[0]), xmax0 = uniform_f(v[1]);
        const float bmin0 = uniform_f(v[2]), bmax0 = uniform_f(v[3]);
        if (xmax0 < -1e38f) {                      // no ray of the tile in this slab
            const float nn = uniform_f(v[4]);
            if (nn > 1e38f) break;                 // every ray of the tile is done
            n_chunk = (long long)nn;               // gap: jump to the next slab someone needs
            continue;
        }
        // a per-slice rectangle of RW x RH bounds every slice's footprint:
        // width <= ceil(span + 2 eps) + 1 (corner column) + 1, plus up to V - 1
        // columns of 16-byte alignment (spans clamped so that they cannot
        // overflow an int)
        constexpr float kEps = 0.01f;
        const float span_x = fminf((xmax0 - xmin0) + 2.0f * Kx + (float)kSlices * (kxmax - kxmin), 65536.0f);
        const float span_b = fminf((bmax0 - bmin0) + 2.0f * Kb + (float)kSlices * (kbmax - kbmin), 65536.0f);
        int RW = (int)ceilf(span_x + 2.0f * kEps) + 2 + V - 1;
        RW = (RW + V - 1) / V * V;
        if (RW > pitch) RW = pitch;
        int RH = (int)ceilf(span_b + 2.0f * kEps) + 2;
        if (RH > snb) RH = snb;
        RW = uniform_i(RW);
        RH = uniform_i(RH);
        // split the slab into S sub-slabs of L slices until L + 3 slices fit
        int S = 1;
        auto fits = [&](int sl) {
            return (long long)sl * RW * RH <= kStageFloats && sl * RH <= kMaxRows;
        };
        while (S < kSlab && !fits(kSlab / S + 3)) S *= 2;
        const int L = kSlab / S, nsl = L + 3;
        const bool use_lds = fits(nsl) && RW > 0 && RH > 0;
        if (!use_lds) S = 1;
        const long long kend_blk = part ? min(k_next, rs.kl + 1) : 0;   // exclusive
        Anchor an{};
        if (part && kend_blk > k_cur) an = make_anchor(rs, b, p.dt, k_cur);
        long long kpos = k_cur;
        bool cont = true;
        for (int q = 0; q < S; ++q) {
            // lower stored-w plane of sub-slab q (sub-slabs in ray order)
            const int w_a = (int)wlo + (sg > 0 ? q * L : kSlab - (q + 1) * L);
            if (use_lds) {
                // slice w = w_a - 1 + i is touched by samples with s_w in
                // [w - 1, w + 1), i.e. s_w - wlo in [d0 + i - 2, d0 + i]; its
                // rectangle starts at (x0, b0)
                auto slice_origin = [&](int i, int& x0, int& b0) {
                    const float da = (float)(w_a - (int)wlo + i - 2), db = da + 2.0f;
                    const float xl = xmin0 + fminf(fminf(da * kxmin, da * kxmax), fminf(db * kxmin, db * kxmax));
                    const float bl0 = bmin0 + fminf(fminf(da * kbmin, da * kbmax), fminf(db * kbmin, db * kbmax));
                    x0 = max((int)floorf(xl - kEps), 0) / V * V;
                    if (x0 + RW > pitch) x0 = pitch - RW;
                    b0 = max((int)floorf(bl0 - kEps), 0);
                };
                const int nrows = nsl * RH;
                const float inv_rh = 1.0f / (float)RH;
                if (tid < nsl) {
                    int x0, b0;
                    slice_origin(tid, x0, b0);
                    tab_off[tid] = (tid * RH * RW - b0 * RW - x0) * 4;   // bytes
                }
                // source of every staged row (slices w_a - 1 .. w_a + L + 1)
                for (int qr = tid; qr < nrows; qr += 256) {
                    const int i = (int)(((float)qr + 0.5f) * inv_rh);
                    const int r = qr - i * RH;
                    int x0, b0;
                    slice_origin(i, x0, b0);
                    const int wabs = min(max(w_a - 1 + i, 0), snw - 1);
                    const int babs = min(b0 + r, snb - 1);
                    const int yz = W == 2 ? wabs * sny + babs : babs * sny + wabs;
                    row_src[qr] = (unsigned)yz * (unsigned)pitch + (unsigned)x0;
                }
                __syncthreads();
                // copy: a fixed 16-byte column per thread, rows strided; the
                // loads of kBatch rows are all issued before the first store,
                // so their HBM latencies overlap
                constexpr int kBatch = 2;
                const int cols = RW / V;
                const int tpr = min(cols, 256), rpi = 256 / tpr;
                const int c0 = tid % tpr, r0 = tid / tpr;
                if (r0 < rpi) {
                    if (cols <= 256) {
                        for (int qb = r0; qb < nrows; qb += kBatch * rpi) {
                            u32x4 v[kBatch];
#pragma unroll
                            for (int m = 0; m < kBatch; ++m) {
                                const int qr = qb + m * rpi;
                                if (qr < nrows) v[m] = StageVec<TS>::load(vox + row_src[qr] + c0 * V);
                            }
#pragma unroll
                            for (int m = 0; m < kBatch; ++m) {
                                const int qr = qb + m * rpi;
                                if (qr < nrows) StageVec<TS>::store(v[m], stage + qr * RW + c0 * V);
                            }
                        }
                    } else {
                        for (int qr = r0; qr < nrows; qr += rpi)
                            for (int c = c0; c < cols; c += tpr)
                                StageVec<TS>::store(StageVec<TS>::load(vox + row_src[qr] + c * V),
                                                    stage + qr * RW + c * V);
                    }
                }
                __syncthreads();
            }
            if (part && cont && kpos < kend_blk) {
                // samples of this ray before the crossing of the next sub-plane
                long long ke = kend_blk;
                if (q + 1 < S) {
#pragma clang fp contract(off)
                    const double t = bl.c0 + ((double)n_chunk + (double)(q + 1) / (double)S) * bl.c1;
                    ke = min(ke, (long long)ceil(t * p.inv_dt - 0.5));
                }
                if (ke > kpos) {
                    const int j0 = (int)(kpos - k_cur), j1 = (int)(ke - k_cur);
                    if (use_lds) {
                        // byte offsets: lane constants of this anchor block and
                        // sub-slab, then 3 FMA + 3 fract + 3 floor per sample
                        const int RW4 = RW * 4;
                        const int lim4 = (kStageFloats - RW - 2) * 4;
                        const int ia_b = W == 2 ? an.ia1 : an.ia2, ia_w = W == 2 ? an.ia2 : an.ia1;
                        const int base4 = ia_b * RW4 + an.ia0 * 4;
                        const int sio = ia_w - (w_a - 1);
                        const char* S8 = reinterpret_cast<const char*>(stage);
                        auto sample_lds = [&](float fj) {
                            const float x = fmaf(fj, st.s0, an.uf0);
                            const float y = fmaf(fj, st.s1, an.uf1);
                            const float z = fmaf(fj, st.s2, an.uf2);
                            Cell c;
                            c.fx = fract(x); c.fy = fract(y); c.fz = fract(z);
                            const int fx_i = floor_int(x);
                            const int fb = floor_int(W == 2 ? y : z), fw = floor_int(W == 2 ? z : y);
                            // (unsigned clamps keep every read inside the stage;
                            // the slab bounds make them inactive)
                            const unsigned si = min((unsigned)(fw + sio), (unsigned)(nsl - 2));
                            const int row4 = __mul24(fb, RW4) + fx_i * 4 + base4;
                            const unsigned a0 = min((unsigned)(tab_off[si] + row4), (unsigned)lim4);
                            const unsigned a1 = min((unsigned)(tab_off[si + 1] + row4), (unsigned)lim4);
                            const float p00 = *reinterpret_cast<const float*>(S8 + a0);
                            const float p01 = *reinterpret_cast<const float*>(S8 + a0 + 4);
                            const float p10 = *reinterpret_cast<const float*>(S8 + a0 + RW4);
                            const float p11 = *reinterpret_cast<const float*>(S8 + a0 + RW4 + 4);
                            const float q00 = *reinterpret_cast<const float*>(S8 + a1);
                            const float q01 = *reinterpret_cast<const float*>(S8 + a1 + 4);
                            const float q10 = *reinterpret_cast<const float*>(S8 + a1 + RW4);
                            const float q11 = *reinterpret_cast<const float*>(S8 + a1 + RW4 + 4);
                            // (p: slice w, q: slice w+1; second index: row b+1)
                            return W == 2 ? lerp3(c, p00, p01, p10, p11, q00, q01, q10, q11)
                                          : lerp3(c, p00, p01, q00, q01, p10, p11, q10, q11);
                        };
                        cont = march_run<false>(p, tft, rs, k_cur, j0, j1, pix, tf_k, tf_o, eps, s,
                                                sample_lds);
                    } else {
                        auto sample_hbm = [&](float fj) {
                            return trilinear(vox, locate(an, st, fj, snx, sny, snz), pitch, sxy);
                        };
                        cont = march_run<false>(p, tft, rs, k_cur, j0, j1, pix, tf_k, tf_o, eps, s,
                                                sample_hbm);
                    }
                    kpos = ke;
                }
            }
            if (use_lds && q + 1 < S) __syncthreads();   // sub-slab done before the next is staged
        }
        if (part) {
            k_cur = max(k_cur, kend_blk);
            ++n_cur;
            k_next = block_start(bl, p.inv_dt, n_cur + 1);
            alive = cont && k_cur <= rs.kl;
        }
        ++n_chunk;
    }
}

// One 16x16 tile of one partial image, by the whole 256-thread workgroup.
// The classification table must already be in sh.tft; `buf` selects the
// reduction buffer and is carried between calls.  Every thread of the
// workgroup must call it with the same arguments.
template <typename TS>
__device__ void staged_tile(const MarchParams& p, int tile, StagedShared& sh, int& buf) {
    const TFTable& tft = sh.tft;
    float (*red)[4][kRed] = sh.red;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x16 = (p.roi_w + 15) / 16;
    const int tx = tile % tiles_x16, ty = tile / tiles_x16;
    const int lx = tx * 16 + (wave & 1) * 8 + (lane & 7);
    const int ly = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
    const bool valid = tile < p.tiles_x * p.tiles_y && lx < p.roi_w && ly < p.roi_h;
    const long long pix = (long long)ly * p.roi_w + lx;
    const BrickK& b = p.brick;
    const float tf_k = 255.0f / (p.tf.vmax - p.tf.vmin);
    const float tf_o = -p.tf.vmin * tf_k;
    const float eps = p.ert_eps;

    LaneState s{0.f, 0.f, 0.f, 1.f, 0, false};
    float depth = INFINITY;
    RaySetup rs;
    const bool has = valid && setup_ray(p.cam, b, p.dt, p.roi_x0 + lx, p.roi_y0 + ly, rs);
    Blocks bl{0.0, 1.0, 0, 1};
    float dw_abs = 1.0f;
    if (has) {
        depth = (float)(((double)rs.kf + 0.5) * p.dt);
        bl = make_blocks(rs, b);
        dw_abs = (float)fabs(pick3(rs.d, bl.axis));
    }
    // eligibility: every ray of the tile shares slab axis (y or z) and direction
    float v[4] = {has ? (float)(bl.axis * 2 + (bl.sg > 0 ? 1 : 0)) : 1e9f,
                  has ? (float)(bl.axis * 2 + (bl.sg > 0 ? 1 : 0)) : -1e9f,
                  has ? dw_abs : 1e9f, has ? 1.0f : 0.0f};
    const bool mx[4] = {false, true, false, true};
    wg_reduce(v, mx, red, buf, lane, wave);
    buf ^= 1;
    const float kmin = uniform_f(v[0]), kmax = uniform_f(v[1]);
    if (uniform_f(v[3]) == 0.0f) {                // no ray of this tile hits the brick
        finish(p, valid, pix, depth, s, lane);
        return;
    }
    if (!(kmin == kmax && kmin >= 2.0f && uniform_f(v[2]) >= kMinStageDw)) {
        if (has) march_ray_direct<TS, false>(p, tft, rs, pix, tf_k, tf_o, eps, s);
        finish(p, valid, pix, depth, s, lane);
        return;
    }
    // the tile's common slab axis and direction: key = 2 axis + (sg > 0)
    const int key = (int)kmin;
    const int sg = (key & 1) ? 1 : -1;
    if ((key >> 1) == 2)
        staged_walk<TS, 2>(p, sh, buf, rs, bl, has, sg, pix, tf_k, tf_o, eps, s);
    else
        staged_walk<TS, 1>(p, sh, buf, rs, bl, has, sg, pix, tf_k, tf_o, eps, s);
    finish(p, valid, pix, depth, s, lane);
}

template <typename TS>
__global__ __launch_bounds__(256) void march_staged(MarchParams p) {
    __shared__ StagedShared sh;
    load_tf(sh.tft, p.tf, p.dt, threadIdx.x, 256);
    // XCD-aware order: workgroup i runs on XCD i mod 8, so give each XCD a
    // contiguous run of tiles (neighbouring tiles share L2 lines); the map is
    // a bijection on [0, gridDim.x)
    const int nb = gridDim.x, bid = blockIdx.x;
    const int per = nb / 8, rem = nb % 8, xcd = bid % 8;
    const int tile = xcd * per + min(xcd, rem) + bid / 8;
    int buf = 0;
    staged_tile<TS>(p, tile, sh, buf);
}

// Persistent work-queue march: each workgroup repeatedly takes the next
// ticket (one 16x16 tile of one job = one partial image) until the tickets
// run out, so many small partials (bricks x time steps x fields x cameras)
// fill the GPU together.  Tickets come from kQueueParts parts, the own XCD's
// part first.  The table is reloaded only when a job's transfer function (or
// dt) differs from the previous ticket's.
template <typename TS, bool kStaged>
__device__ void direct_tile(const MarchParams& p, int tile, const TFTable& tft);

// LDS of a queue workgroup: the staging buffers only where tiles are staged.
template <bool kStaged>
struct QueueShared {
    StagedShared st;
    __device__ TFTable& tf() { return st.tft; }
};
template <>
struct QueueShared<false> {
    TFTable t;
    __device__ TFTable& tf() { return t; }
};

template <typename TS, bool kStaged>
__global__ __launch_bounds__(256) void march_queue(QueueParams q) {
    __shared__ QueueShared<kStaged> sh;
    __shared__ int ticket;
    const int tid = threadIdx.x;
    const float* tf_loaded = nullptr;
    float scale_loaded = -1.0f;
    double dt_loaded = -1.0;
    int buf = 0;
    (void)buf;
    const int home = blockIdx.x % kQueueParts;
    for (int c = 0; c < kQueueParts; ++c) {
        const int part = (home + c) % kQueueParts;
        const int lo_t = (int)((long long)q.total_tiles * part / kQueueParts);
        const int hi_t = (int)((long long)q.total_tiles * (part + 1) / kQueueParts);
        for (;;) {
            // the counter only grows, so every workgroup leaves each part
            // after at most one ticket past its end
            if (tid == 0) ticket = lo_t + atomicAdd(q.head + part, 1);
            __syncthreads();
            const int t = ticket;
            __syncthreads();
            if (t >= hi_t) break;
            // job of ticket t: the last j with tile_start[j] <= t
            int lo = 0, hi = q.n_jobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (q.tile_start[mid] <= t) lo = mid; else hi = mid - 1;
            }
            const MarchParams& p = q.jobs[lo];
            if (p.tf.rgba != tf_loaded || p.tf.opacity_scale != scale_loaded || p.dt != dt_loaded) {
                load_tf(sh.tf(), p.tf, p.dt, tid, 256);
                tf_loaded = p.tf.rgba;
                scale_loaded = p.tf.opacity_scale;
                dt_loaded = p.dt;
                if (!kStaged) __syncthreads();
                // (staged_tile's first reduction barrier orders these writes before use)
            }
            if constexpr (kStaged)
                staged_tile<TS>(p, t - q.tile_start[lo], sh.st, buf);
            else
                direct_tile<TS, false>(p, t - q.tile_start[lo], sh.tf());
            __syncthreads();
        }
    }
}

// One 16x16 tile, every lane marching its own ray from HBM (no staging, no
// workgroup-wide steps).
template <typename TS, bool kStaged>
__device__ void direct_tile(const MarchParams& p, int tile, const TFTable& tft) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x16 = (p.roi_w + 15) / 16;
    const int tx = tile % tiles_x16, ty = tile / tiles_x16;
    const int lx = tx * 16 + (wave & 1) * 8 + (lane & 7);
    const int ly = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
    const bool valid = lx < p.roi_w && ly < p.roi_h;
    const long long pix = (long long)ly * p.roi_w + lx;
    const float tf_k = 255.0f / (p.tf.vmax - p.tf.vmin);
    const float tf_o = -p.tf.vmin * tf_k;
    LaneState s{0.f, 0.f, 0.f, 1.f, 0, false};
    float depth = INFINITY;
    RaySetup rs;
    if (valid && setup_ray(p.cam, p.brick, p.dt, p.roi_x0 + lx, p.roi_y0 + ly, rs)) {
        depth = (float)(((double)rs.kf + 0.5) * p.dt);
        march_ray_direct<TS, false>(p, tft, rs, pix, tf_k, tf_o, p.ert_eps, s);
    }
    finish(p, valid, pix, depth, s, lane);
}

__global__ void queue_reset(int* head) {
    if (threadIdx.x < kQueueParts) head[threadIdx.x] = 0;
}

template <bool kCkpt>
hipError_t launch_direct(const MarchParams& p, StorageK storage, hipStream_t stream) {
    const int blocks = p.tiles_x * p.tiles_y;
    if (blocks == 0) return hipSuccess;
    if (storage == kF16)
        hipLaunchKernelGGL((march_direct<__half, kCkpt>), dim3(blocks), dim3(64), 0, stream, p);
    else
        hipLaunchKernelGGL((march_direct<float, kCkpt>), dim3(blocks), dim3(64), 0, stream, p);
    return hipGetLastError();
}

}  // namespace

template <typename TS, bool kStaged>
hipError_t launch_queue_t(const QueueParams& q, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((march_queue<TS, kStaged>), dim3(grid), dim3(256), 0, stream, q);
    return hipGetLastError();
}

template <typename TS, bool kStaged>
int queue_occupancy() {
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, march_queue<TS, kStaged>, 256, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_march_queue(const QueueParams& q, StorageK storage, int workgroups,
                              hipStream_t stream) {
    if (q.total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(queue_reset, dim3(1), dim3(64), 0, stream, q.head);
    const int grid = min(workgroups, q.total_tiles);
    if (storage == kF16)
        return q.staged ? launch_queue_t<__half, true>(q, grid, stream)
                        : launch_queue_t<__half, false>(q, grid, stream);
    return q.staged ? launch_queue_t<float, true>(q, grid, stream)
                    : launch_queue_t<float, false>(q, grid, stream);
}

int march_queue_workgroups_per_cu(StorageK storage, bool staged) {
    if (storage == kF16) return staged ? queue_occupancy<__half, true>() : queue_occupancy<__half, false>();
    return staged ? queue_occupancy<float, true>() : queue_occupancy<float, false>();
}

hipError_t launch_march(const MarchParams& p, StorageK storage, hipStream_t stream) {
    if (p.ckpt) return launch_direct<true>(p, storage, stream);
    if (p.path == kPathDirect) return launch_direct<false>(p, storage, stream);
    // staged: one workgroup per 16x16 tile; tiles_x/tiles_y count 16x16 tiles
    MarchParams q = p;
    q.tiles_x = (p.roi_w + 15) / 16;
    q.tiles_y = (p.roi_h + 15) / 16;
    const int blocks = q.tiles_x * q.tiles_y;
    if (blocks == 0) return hipSuccess;
    if (storage == kF16)
        hipLaunchKernelGGL(march_staged<__half>, dim3(blocks), dim3(256), 0, stream, q);
    else
        hipLaunchKernelGGL(march_staged<float>, dim3(blocks), dim3(256), 0, stream, q);
    return hipGetLastError();
}

}  // namespace dpvr
