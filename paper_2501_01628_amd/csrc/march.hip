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
// Two families of kernels compute bit-identical images:
//  * staged (default): a workgroup owns a TW x 16 pixel tile (TW = 16 or 32),
//    one consumer wavefront per 8x8 quarter plus one producer wavefront that
//    streams, with the LDS DMA, the slices of brick data the tile's rays
//    cross into a ring of LDS slots ahead of the consumers, which march
//    their rays chunk by chunk out of LDS.  Tiles whose rays do not share a
//    slab axis and direction, or whose slice footprint does not fit the
//    ring, march from HBM directly.
//  * direct: every lane reads its voxels straight from HBM (one wavefront per
//    8x8 tile, or a 16x16 tile per workgroup in the work queue); the
//    checkpointing forward of the adjoint uses it.
#include "march_common.h"

namespace dpvr {
namespace {

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

// march_run for a sampler in three stages -- pre(fj) locates sample j and
// issues its first dependent reads, gather(P) issues its voxel reads,
// value(G) interpolates -- with the two samples of a pair interleaved stage
// by stage (scheduling barriers keep both samples' reads of a stage in
// flight together): three memory round trips per pair instead of six.  The
// loop walks the ray's pairs (aligned to its first owned sample) that
// overlap [j0, j1), so a run that starts or ends inside a pair takes that
// pair too, with the sample outside the run located and read (from clamped
// addresses) but not accumulated: no separate single-sample steps, which a
// wavefront would otherwise take whenever any of its rays needs one.  The
// arithmetic of every sample, the order of accumulation and the termination
// tests are those of march_run, so results are bit-identical.
template <typename Pre, typename Gather, typename Value>
__device__ inline bool march_run_pipe(const TFTable& tft, const RaySetup& rs, long long kb, int j0,
                                      int j1, float tf_k, float tf_o, float eps, LaneState& s,
                                      Pre pre, Gather gather, Value value) {
    auto accumulate = [&](const Classified& e) {
#pragma clang fp contract(off)
        const float Tn = s.T * trans_exp2(-e.a);
        const float w = s.T - Tn;
        s.C0 = fmaf(w, e.r, s.C0);
        s.C1 = fmaf(w, e.g, s.C1);
        s.C2 = fmaf(w, e.b, s.C2);
        s.T = Tn;
    };
    if (j0 >= j1) return true;
    // first sample of the pair that holds sample j0
    for (int j = j0 - (int)((kb + j0 - rs.kf) & 1); j < j1; j += 2) {
        const float fj = (float)j;
        const auto pa = pre(fj);
        const auto pb = pre(fj + 1.0f);
        __builtin_amdgcn_sched_barrier(0);
        const auto ga = gather(pa);
        const auto gb = gather(pb);
        __builtin_amdgcn_sched_barrier(0);
        const float v0 = value(ga), v1 = value(gb);
        // classification in two stages (table index, then both table reads)
        const float sr0 = fmaf(v0, tf_k, tf_o), sr1 = fmaf(v1, tf_k, tf_o);
        const float s0 = fminf(fmaxf(sr0, 0.0f), 255.0f), s1 = fminf(fmaxf(sr1, 0.0f), 255.0f);
        const int g0 = min((int)s0, 254), g1 = min((int)s1, 254);
        const float4 b0 = tft.base[g0], d0 = tft.diff[g0], b1 = tft.base[g1], d1 = tft.diff[g1];
        __builtin_amdgcn_sched_barrier(0);
        const float ph0 = s0 - (float)g0, ph1 = s1 - (float)g1;
        Classified e0, e1;
        e0.r = fmaf(ph0, d0.x, b0.x); e0.g = fmaf(ph0, d0.y, b0.y);
        e0.b = fmaf(ph0, d0.z, b0.z); e0.a = fmaf(ph0, d0.w, b0.w);
        e1.r = fmaf(ph1, d1.x, b1.x); e1.g = fmaf(ph1, d1.y, b1.y);
        e1.b = fmaf(ph1, d1.z, b1.z); e1.a = fmaf(ph1, d1.w, b1.w);
        if (j >= j0) accumulate(e0);
        // the pair's second sample closes it: the termination test follows
        // it (a run ending after the first sample leaves both to the next run)
        if (j + 1 < j1) {
            accumulate(e1);
            if (s.T < eps) {
                s.evaluated += j + 2 - j0;
                s.stopped = true;
                return false;
            }
        }
    }
    s.evaluated += j1 - j0;
    return true;
}

// march_run_pipe with the pairs software-pipelined four deep: iteration i
// issues the first reads of pair i + 3, the voxel reads of pair i + 2 and the
// table reads of pair i + 1, then accumulates pair i, so every read has a
// whole iteration to arrive.  Pairs past the run's end are located and read
// (from clamped addresses) but never accumulated.  Same arithmetic and
// accumulation order as march_run_pipe: bit-identical results.
template <typename Pre, typename Gather, typename Value>
__device__ inline bool march_run_deep(const TFTable& tft, const RaySetup& rs, long long kb, int j0,
                                      int j1, float tf_k, float tf_o, float eps, LaneState& s,
                                      Pre pre, Gather gather, Value value) {
    auto accumulate = [&](const Classified& e) {
#pragma clang fp contract(off)
        const float Tn = s.T * trans_exp2(-e.a);
        const float w = s.T - Tn;
        s.C0 = fmaf(w, e.r, s.C0);
        s.C1 = fmaf(w, e.g, s.C1);
        s.C2 = fmaf(w, e.b, s.C2);
        s.T = Tn;
    };
    auto one = [&](float fj) { return classify(tft, value(gather(pre(fj))), tf_k, tf_o); };
    using P = decltype(pre(0.0f));
    using G = decltype(gather(pre(0.0f)));
    struct P2 { P a, b; };
    struct G2 { G a, b; };
    struct T2 { float ph0, ph1; float4 b0, d0, b1, d1; };
    auto pre2 = [&](float f) { return P2{pre(f), pre(f + 1.0f)}; };
    auto gather2 = [&](const P2& x) { return G2{gather(x.a), gather(x.b)}; };
    auto table2 = [&](const G2& x) {
        const float v0 = value(x.a), v1 = value(x.b);
        const float s0 = fminf(fmaxf(fmaf(v0, tf_k, tf_o), 0.0f), 255.0f);
        const float s1 = fminf(fmaxf(fmaf(v1, tf_k, tf_o), 0.0f), 255.0f);
        const int g0 = min((int)s0, 254), g1 = min((int)s1, 254);
        return T2{s0 - (float)g0, s1 - (float)g1, tft.base[g0], tft.diff[g0], tft.base[g1], tft.diff[g1]};
    };
    auto finish2 = [&](const T2& t) {
        Classified e0, e1;
        e0.r = fmaf(t.ph0, t.d0.x, t.b0.x); e0.g = fmaf(t.ph0, t.d0.y, t.b0.y);
        e0.b = fmaf(t.ph0, t.d0.z, t.b0.z); e0.a = fmaf(t.ph0, t.d0.w, t.b0.w);
        e1.r = fmaf(t.ph1, t.d1.x, t.b1.x); e1.g = fmaf(t.ph1, t.d1.y, t.b1.y);
        e1.b = fmaf(t.ph1, t.d1.z, t.b1.z); e1.a = fmaf(t.ph1, t.d1.w, t.b1.w);
        accumulate(e0);
        accumulate(e1);
    };
    int j = j0;
    float fj = (float)j0;
    if (((kb + j0 - rs.kf) & 1) && j < j1) {   // second sample of a pair begun in the previous run
        accumulate(one(fj));
        ++j;
        fj += 1.0f;
        if (s.T < eps) {
            s.evaluated += 1;
            s.stopped = true;
            return false;
        }
    }
    const int npairs = (j1 - j) >> 1;
    if (npairs > 0) {
        P2 p2 = pre2(fj + 4.0f);
        const P2 p1 = pre2(fj + 2.0f);
        const P2 p0 = pre2(fj);
        __builtin_amdgcn_sched_barrier(0);
        G2 g1 = gather2(p1);
        const G2 g0 = gather2(p0);
        __builtin_amdgcn_sched_barrier(0);
        T2 t0 = table2(g0);
        __builtin_amdgcn_sched_barrier(0);
        for (int i = 0; i < npairs; ++i) {
            const P2 p3 = pre2(fj + (float)(2 * i + 6));
            const G2 g2 = gather2(p2);
            const T2 t1 = table2(g1);
            __builtin_amdgcn_sched_barrier(0);
            finish2(t0);
            if (s.T < eps) {
                s.evaluated += j - j0 + 2 * i + 2;
                s.stopped = true;
                return false;
            }
            t0 = t1;
            g1 = g2;
            p2 = p3;
        }
        j += 2 * npairs;
        fj += (float)(2 * npairs);
    }
    // first sample of a pair: its test comes after the next sample (next run)
    if (j < j1) accumulate(one(fj));
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
// One 8x8 tile of partial p per 64-thread workgroup, every lane marching
// from HBM.
template <typename TS, bool kCkpt>
__device__ inline void march_tile_hbm(const MarchParams& p, int tile) {
    __shared__ TFTable tft;
    const int lane = threadIdx.x;
    load_tf(tft, p.tf, p.dt, lane, 64);
    __syncthreads();

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

template <typename TS, bool kCkpt>
__global__ __launch_bounds__(64) void march_direct(MarchParams p) {
    march_tile_hbm<TS, kCkpt>(p, blockIdx.x);
}

// The checkpointed forward of many partials in one launch: workgroup b takes
// tile b - tile_start[j] of job j, the last j with tile_start[j] <= b.
template <typename TS>
__global__ __launch_bounds__(64) void march_checkpointed_many(const MarchParams* __restrict__ jobs,
                                                              const int32_t* __restrict__ tile_start,
                                                              int32_t n_jobs) {
    const int b = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    march_tile_hbm<TS, true>(jobs[lo], b - __builtin_amdgcn_readfirstlane(tile_start[lo]));
}

// ------------------------------------------------- shared by the staged kernels
constexpr int kRed = 8;                  // values per workgroup reduction (at most)
constexpr float kMinStageDw = 0.25f;     // |d_w| below this: march from HBM

// Workgroup-wide reduction of N values over NW waves: shuffles within each
// wave, one LDS round trip (double-buffered by `buf`: one barrier per call).
template <int N, int NW>
__device__ inline void wg_reduce(float (&v)[N], const bool (&is_max)[N], float (*red)[NW][kRed],
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
        for (int w = 1; w < NW; ++w) x = is_max[i] ? fmaxf(x, red[buf][w][i]) : fminf(x, red[buf][w][i]);
        v[i] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
    }
}

__device__ inline int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------- staged kernel (slabs)
// A 256-thread workgroup owns a 16x16 pixel tile (one wavefront per 8x8
// quarter) and walks the slabs of the tile's common slab axis w (y or z;
// rows along x stay contiguous in HBM) in ray order, all four waves in step:
// per slab (one 16-slice anchor block), a workgroup reduction gives the
// extent of the tile's rays in the slab; the slab (or each of its sub-slabs,
// when it does not fit) is staged into LDS slice by slice as sheared
// rectangles, then every lane marches its samples of it from LDS.  Two
// workgroups share a CU, so one stages while the other marches.
constexpr int kSlices = kSlab + 3;       // staged slices per slab: [wlo - 1, whi + 1]
constexpr int kStageFloats = 16384;      // 64 KB stage: 2 workgroups per CU
constexpr int kMaxRows = 1024;

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

// LDS of a slab-march workgroup.
struct StagedShared {
    TFTable tft;
    __align__(16) float stage[kStageFloats];
    unsigned row_src[kMaxRows];          // element offset in the brick of each staged row
    int tab_off[kSlices];
    float red[2][4][kRed];
    int ticket;
};

__device__ inline float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Walk of one eligible tile through the slabs of its common slab axis W
// (2: z, rows along y; 1: y, rows along z) in ray order.  Per slab, a
// workgroup reduction gives the extent of the tile's rays in the slab; the
// slab (or each of its sub-slabs, when it does not fit) is staged into LDS
// slice by slice as sheared rectangles, then every lane marches its samples
// of it from LDS.
template <typename TS, int W>
__device__ void slab_walk(const MarchParams& p, StagedShared& sh, int& buf, const RaySetup& rs,
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
        wg_reduce<sizeof(v) / sizeof(v[0]), 4>(v, mx, red, buf, lane, wave);
        buf ^= 1;
        n_chunk = (long long)uniform_f(v[0]);
    }
    const double gh = (double)b.ghost - 0.5;
    // slopes of all rays of the tile (constant along each ray)
    float kxmin, kxmax, kbmin, kbmax;
    {
        float v[4] = {has ? kx : 3e38f, has ? kx : -3e38f, has ? kb : 3e38f, has ? kb : -3e38f};
        const bool mx[4] = {false, true, false, true};
        wg_reduce<sizeof(v) / sizeof(v[0]), 4>(v, mx, red, buf, lane, wave);
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
        wg_reduce<sizeof(v) / sizeof(v[0]), 4>(v, mx, red, buf, lane, wave);
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
                        struct SlabPre {
                            Cell c;
                            int row4, t0, t1;
                        };
                        struct SlabGather {
                            Cell c;
                            float v[8];
                        };
                        auto pre = [&](float fj) {
                            const float x = fmaf(fj, st.s0, an.uf0);
                            const float y = fmaf(fj, st.s1, an.uf1);
                            const float z = fmaf(fj, st.s2, an.uf2);
                            SlabPre r;
                            r.c.fx = fract(x); r.c.fy = fract(y); r.c.fz = fract(z);
                            const int fx_i = floor_int(x);
                            const int fb = floor_int(W == 2 ? y : z), fw = floor_int(W == 2 ? z : y);
                            // (unsigned clamps keep every read inside the stage;
                            // the slab bounds make them inactive)
                            const unsigned si = min((unsigned)(fw + sio), (unsigned)(nsl - 2));
                            r.row4 = __mul24(fb, RW4) + fx_i * 4 + base4;
                            r.t0 = tab_off[si];
                            r.t1 = tab_off[si + 1];
                            return r;
                        };
                        auto gather = [&](const SlabPre& r) {
                            const unsigned a0 = min((unsigned)(r.t0 + r.row4), (unsigned)lim4);
                            const unsigned a1 = min((unsigned)(r.t1 + r.row4), (unsigned)lim4);
                            SlabGather g;
                            g.c = r.c;
                            g.v[0] = *reinterpret_cast<const float*>(S8 + a0);
                            g.v[1] = *reinterpret_cast<const float*>(S8 + a0 + 4);
                            g.v[2] = *reinterpret_cast<const float*>(S8 + a0 + RW4);
                            g.v[3] = *reinterpret_cast<const float*>(S8 + a0 + RW4 + 4);
                            g.v[4] = *reinterpret_cast<const float*>(S8 + a1);
                            g.v[5] = *reinterpret_cast<const float*>(S8 + a1 + 4);
                            g.v[6] = *reinterpret_cast<const float*>(S8 + a1 + RW4);
                            g.v[7] = *reinterpret_cast<const float*>(S8 + a1 + RW4 + 4);
                            return g;
                        };
                        // (v[0..3]: slice w, v[4..7]: slice w + 1; odd: x + 1;
                        // 2, 3, 6, 7: row b + 1)
                        auto value = [&](const SlabGather& g) {
                            return W == 2 ? lerp3(g.c, g.v[0], g.v[1], g.v[2], g.v[3], g.v[4], g.v[5], g.v[6], g.v[7])
                                          : lerp3(g.c, g.v[0], g.v[1], g.v[4], g.v[5], g.v[2], g.v[3], g.v[6], g.v[7]);
                        };
                        // (the plain two-sample loop: measured faster here than the
                        // staged loop, whose scheduling barriers the slab's lock-step
                        // waves cannot hide)
                        auto sample_lds = [&](float fj) { return value(gather(pre(fj))); };
                        cont = march_run<false>(p, tft, rs, k_cur, j0, j1, pix, tf_k, tf_o, eps, s, sample_lds);
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
__device__ void slab_tile(const MarchParams& p, int tile, StagedShared& sh, int& buf) {
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
    wg_reduce<sizeof(v) / sizeof(v[0]), 4>(v, mx, red, buf, lane, wave);
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
        slab_walk<TS, 2>(p, sh, buf, rs, bl, has, sg, pix, tf_k, tf_o, eps, s);
    else
        slab_walk<TS, 1>(p, sh, buf, rs, bl, has, sg, pix, tf_k, tf_o, eps, s);
    finish(p, valid, pix, depth, s, lane);
}

template <typename TS>
__global__ __launch_bounds__(256) void march_slab_single(MarchParams p) {
    __shared__ StagedShared sh;
    load_tf(sh.tft, p.tf, p.dt, threadIdx.x, 256);
    // XCD-aware order (see march_staged)
    const int nb = gridDim.x, bid = blockIdx.x;
    const int per = nb / 8, rem = nb % 8, xcd = bid % 8;
    const int tile = xcd * per + min(xcd, rem) + bid / 8;
    int buf = 0;
    slab_tile<TS>(p, tile, sh, buf);
}

// ------------------------------------------------------- staged kernel (slice ring)
// A workgroup owns a TW x 16 pixel tile: NCW = TW / 4 consumer wavefronts
// march the 8 x 8 quarters, one producer wavefront streams the brick slices
// the tile's rays cross into a ring of LDS slots with the gfx950 LDS DMA
// (global_load_lds_dwordx4: no registers, up to 63 KB in flight per wave).
// The tile walks the slices of its common slab axis w in ray order, in
// chunks of CH slices (CH divides the 16-slice anchor block); a chunk's
// samples touch the CH + 3 slices [CH k, CH k + CH + 2] of the walk (one
// slice of margin each side for float32 rounding across a chunk plane).
// Producer and consumers synchronise through LDS words only: `ready` (walk
// slices published so far) and one `done` word per consumer wave (the lowest
// walk slice it may still read); a slot is refilled once every consumer wave
// has moved past its slice.  No workgroup barrier is taken during the walk.
// Every wait is bounded: a wait that times out sets `abort` (all later waits
// of the workgroup return at once) and the kErrSpin bit of the device error
// word, so a logic error ends the launch with an error instead of a hang.
constexpr int kTabSize = 512;            // walk slices per tile (a deeper walk marches from HBM)
constexpr int kTabMask = kTabSize - 1;
constexpr int kMaxSlots = 64;
constexpr int kAllDone = 1 << 30;
constexpr int kSpinLimit = 1 << 22;      // polls of ~64 cycles: ~0.1 s per wait at most
constexpr double kMargin = 0.01;         // voxels of slack around a slice's footprint
constexpr long long kNoBlock = -(1LL << 62);

template <int NCW>
constexpr int ring_bytes() { return 144 * 1024; }

template <int NCW>
struct RingShared {
    // the table first, at LDS address 0: its reads then need no base address
    TFTable tft;
    __align__(1024) unsigned char ring[ring_bytes<NCW>()];
    // walk slice q: tab[2 q] = LDS byte address of its slot minus its
    // rectangle's origin, tab[2 q + 1] = the same for walk slice q + sg (the
    // next slice along +w), so a sample reads both of its slices' entries at once
    __align__(8) int tab[2 * kTabSize];
    __align__(16) int src[kTabSize];   // walk slice q: element offset of its rectangle's origin in the brick
    int ready;           // walk slices published by the producer
    __align__(16) int done[NCW];   // per consumer wave: walk slices below this are no longer read
    int abort;
    int ticket;
    float red[2][NCW + 1][kRed];
};

// LDS words accessed as volatile through LDS-qualified pointers (a volatile
// access through a generic pointer becomes a FLAT access, which counts
// against the vector-memory counter and so waits behind the LDS DMA).
typedef __attribute__((address_space(3))) volatile int lds_vint;
__device__ inline int ld_volatile(const int& w) { return uniform_i(*(lds_vint*)&w); }
// The same read, written as inline asm that waits for its own result: the
// producer wave uses it while its LDS DMA is in flight, where the compiler
// would otherwise wait for every outstanding DMA (vmcnt(0)) before any LDS
// read, since it cannot tell that the read does not touch the ring.
__device__ inline int ld_lds_nowait_dma(const int& w) {
    typedef __attribute__((address_space(3))) const int lds_int;
    const unsigned a = (unsigned)(uintptr_t)((lds_int*)&w);
    int v;
    __asm__ volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(a) : "memory");
    return uniform_i(v);
}
__device__ inline void st_volatile(int& w, int v) { *(lds_vint*)&w = v; }
__device__ inline void compiler_fence() { __asm__ volatile("" ::: "memory"); }

// s_waitcnt with only the vector-memory counter (gfx9 encoding: vmcnt in
// bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 at their no-wait maxima).
template <int N>
__device__ inline void wait_vmcnt() {
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
// Wait until at most n vector-memory operations of this wave are pending
// (rounded down to a listed count: waiting for more is always safe).
__device__ inline void wait_vmcnt_le(int n) {
    if (n >= 48) wait_vmcnt<48>();
    else if (n >= 32) wait_vmcnt<32>();
    else if (n >= 24) wait_vmcnt<24>();
    else if (n >= 16) wait_vmcnt<16>();
    else if (n >= 12) wait_vmcnt<12>();
    else if (n >= 8) wait_vmcnt<8>();
    else if (n >= 4) wait_vmcnt<4>();
    else wait_vmcnt<0>();
}

// Minimum of the NCW done words (16-byte aligned), read with one or two
// 16-byte LDS reads in an asm block that waits for its own results (see
// ld_lds_nowait_dma).
template <int NCW>
__device__ inline int min_done(const int (&done)[NCW]) {
    typedef __attribute__((address_space(3))) const int lds_int;
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    const unsigned a = (unsigned)(uintptr_t)((lds_int*)&done[0]);
    i32x4 v0, v1;
    if constexpr (NCW == 4) {
        __asm__ volatile("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v0) : "v"(a) : "memory");
        v1 = v0;
    } else {
        static_assert(NCW == 8, "4 or 8 consumer waves");
        __asm__ volatile("ds_read_b128 %0, %2\n\tds_read_b128 %1, %2 offset:16\n\ts_waitcnt lgkmcnt(0)"
                         : "=&v"(v0), "=&v"(v1) : "v"(a) : "memory");
    }
    const int m = min(min(min(v0.x, v0.y), min(v0.z, v0.w)), min(min(v1.x, v1.y), min(v1.z, v1.w)));
    return uniform_i(m);
}

template <int NCW>
__device__ inline void trip(RingShared<NCW>& sh, int* err) {
    st_volatile(sh.abort, 1);
    if (err && (threadIdx.x & 63) == 0) atomicOr(err, kErrSpin);
}

// Bounded wait until word >= target; false on abort or time-out.
template <int NCW>
__device__ inline bool wait_ge(RingShared<NCW>& sh, const int& word, int target, int* err) {
    for (int it = 0; it < kSpinLimit; ++it) {
        if (ld_volatile(word) >= target) {
            compiler_fence();
            return true;
        }
        if (ld_volatile(sh.abort)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    trip(sh, err);
    return false;
}

// Uniform geometry of a tile's walk.  The rays of the tile cross the plane
// s_w = s (stored-index coordinate of the slab axis) at x = xa + xb s,
// b = ba + bb s; on a plane, x and b are ratios of affine functions of the
// pixel coordinates (pinhole) or affine (orthographic), monotone along rows
// and columns, so over the tile's pixel rectangle they are bounded by the
// four corner rays.  A slice w is read by samples with s_w in [w - 1, w + 1).
struct Lines {
    double xa[4], xb[4], ba[4], bb[4];
};

template <int W>
__device__ inline void corner_lines(const MarchParams& p, int px0, int px1, int py0, int py1, Lines& L) {
#pragma clang fp contract(off)
    constexpr int B = 3 - W;
    const BrickK& b = p.brick;
    const double g = (double)b.ghost - 0.5;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const CamRay r = camera_ray(p.cam, (c & 1) ? px1 : px0, (c & 2) ? py1 : py0);
        const double t0 = ((0.5 - (double)b.ghost) * b.spacing[W] + b.origin[W] - r.o[W]) / r.d[W];
        const double dt_ds = b.spacing[W] / r.d[W];    // dt per unit of s_w
        L.xa[c] = (r.o[0] + t0 * r.d[0] - b.origin[0]) * b.inv_spacing[0] + g;
        L.xb[c] = r.d[0] * dt_ds * b.inv_spacing[0];
        L.ba[c] = (r.o[B] + t0 * r.d[B] - b.origin[B]) * b.inv_spacing[B] + g;
        L.bb[c] = r.d[B] * dt_ds * b.inv_spacing[B];
    }
}

// Footprint of slice w: x in [xlo, xhi], b in [blo, bhi] (before margins).
__device__ inline void slice_bounds(const Lines& L, double w, double& xlo, double& xhi, double& blo,
                                    double& bhi) {
    xlo = blo = INFINITY;
    xhi = bhi = -INFINITY;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double xm = L.xa[c] + L.xb[c] * w, xr = fabs(L.xb[c]);
        const double bm = L.ba[c] + L.bb[c] * w, br = fabs(L.bb[c]);
        xlo = fmin(xlo, xm - xr); xhi = fmax(xhi, xm + xr);
        blo = fmin(blo, bm - br); bhi = fmax(bhi, bm + br);
    }
}

// First sample of chunk kap of a ray: chunks cut the anchor blocks into
// 16 / CH parts, at the planes n = kap CH / 16 of the block numbering (a
// chunk plane with kap CH a multiple of 16 is a block plane, computed with
// the same expression as block_start).
__device__ inline long long chunk_start(const Blocks& bl, double inv_dt, long long kap, int ch) {
#pragma clang fp contract(off)
    const double n = (double)(kap * ch) * 0.0625;
    const double t = bl.c0 + n * bl.c1;
    return (long long)ceil(t * inv_dt - 0.5);
}

__device__ inline long long chunk_of(const Blocks& bl, double dt, double inv_dt, long long k, int ch) {
#pragma clang fp contract(off)
    const double t = ((double)k + 0.5) * dt;
    long long kap = (long long)floor(((t - bl.c0) / bl.c1) * (16.0 / (double)ch));
    while (chunk_start(bl, inv_dt, kap, ch) > k) --kap;
    while (chunk_start(bl, inv_dt, kap + 1, ch) <= k) ++kap;
    return kap;
}

struct RingGeom {
    int ok;
    int RW, RH;     // slot rectangle (elements x rows)
    int SB;         // slot stride in bytes (multiple of 1 KB)
    int R;          // slots in the ring
    int NI;         // DMA instructions per slice (SB / 1 KB)
    int D;          // slices the producer keeps in flight before publishing
    int Q;          // walk slices
    int K;          // chunks
    int w_start;    // stored slice of walk slice 0
    long long klo;  // first chunk
};

template <typename TS, int NCW, int CH, int W>
__device__ inline RingGeom ring_geometry(const MarchParams& p, const Lines& L, int sg, long long klo,
                                         long long khi) {
    constexpr int ESZ = sizeof(TS);
    constexpr int V = 16 / ESZ;                  // elements per 16-byte vector
    constexpr int B = 3 - W;
    const BrickK& b = p.brick;
    const int pitch = row_pitch(b.sdim[0]);
    const int snb = b.sdim[B];
    RingGeom G{};
    G.klo = klo;
    G.K = (int)(khi - klo + 1);
    G.Q = CH * G.K + 3;
    G.w_start = sg > 0 ? (int)(CH * klo - 1) : (int)(-CH * klo + 1);
    // the footprint width is convex in w: its maximum is at an end of the walk
    double sx = 0.0, sb = 0.0;
    for (int e = 0; e < 2; ++e) {
        const double w = (double)(G.w_start + (e ? sg * (G.Q - 1) : 0));
        double xlo, xhi, blo, bhi;
        slice_bounds(L, w, xlo, xhi, blo, bhi);
        sx = fmax(sx, xhi - xlo);
        sb = fmax(sb, bhi - blo);
    }
    const double cap = 65536.0;
    int RW = (int)ceil(fmin(sx, cap) + 2.0 * kMargin) + 2 + V - 1;
    RW = (RW + V - 1) / V * V;
    if (RW > pitch) RW = pitch;
    int RH = (int)ceil(fmin(sb, cap) + 2.0 * kMargin) + 2;
    if (RH > snb) RH = snb;
    G.RW = RW;
    G.RH = RH;
    // slots hold float32 (float16 slices are copied raw into a slot's upper
    // half and decoded in place, see ring_produce)
    const long long bytes = (long long)RW * RH * 4;
    const long long align = ESZ == 2 ? 2048 : 1024;
    G.SB = (int)(((bytes + align - 1) / align) * align);
    G.R = bytes > 0 ? (int)min((long long)kMaxSlots, (long long)ring_bytes<NCW>() / G.SB) : 0;
    G.NI = (int)(((long long)RW * RH * ESZ + 1023) / 1024);
    // the producer addresses a slice's rows with 32-bit byte offsets
    const long long b_stride = W == 2 ? (long long)pitch : (long long)b.sdim[1] * pitch;
    const bool offsets32 = ((long long)(RH - 1) * b_stride + RW) * ESZ < (1LL << 32);
    G.ok = G.R >= CH + 4 && G.K >= 1 && G.Q <= kTabSize && offsets32;
    int D = G.R - (CH + 3);
    D = min(D, 8);
    if (G.NI * (D - 1) > 48) D = 48 / G.NI + 1;
    G.D = max(D, 1);
    return G;
}

// The walk's slice tables, filled by every thread of the workgroup at tile
// set-up: walk slice q (stored slice w = w_start + sg q) is staged in slot
// q mod R as the RW x RH rectangle at (x0, b0) that bounds the footprint of
// the tile's rays on it; consumers address a voxel (b, x) of the slice at
// byte tab[q] + 4 (b RW + x) (float32 in LDS), the producer copies from element src[q] of
// the brick.
template <typename TS, int NCW, int CH, int W>
__device__ void ring_tables(const MarchParams& p, RingShared<NCW>& sh, const Lines& L, const RingGeom& G,
                            int sg) {
    constexpr int ESZ = sizeof(TS);
    constexpr int V = 16 / ESZ;
    constexpr int B = 3 - W;
    const BrickK& b = p.brick;
    const int snx = b.sdim[0], sny = b.sdim[1];
    const int snw = b.sdim[W], snb = b.sdim[B];
    const int pitch = row_pitch(snx);
    const int w_stride = W == 2 ? sny * pitch : pitch;   // elements (a brick holds < 2^31)
    const int b_stride = W == 2 ? pitch : sny * pitch;
    const int RW = G.RW, RH = G.RH, RWB = RW * 4;   // LDS rows hold float32
    const int ring_off = (int)offsetof(RingShared<NCW>, ring);
    // rectangle origin (x0, b0) of walk slice q
    auto origin = [&](int q, int& x0, int& b0) {
        const int w = G.w_start + sg * q;
        double xlo, xhi, blo, bhi;
        slice_bounds(L, (double)w, xlo, xhi, blo, bhi);
        const double xf = fmin(fmax(floor(xlo - kMargin), 0.0), 65536.0);
        const double bf = fmin(fmax(floor(blo - kMargin), 0.0), 65536.0);
        x0 = ((int)xf) / V * V;
        if (x0 + RW > pitch) x0 = pitch - RW;
        b0 = (int)bf;
        if (b0 + RH > snb) b0 = snb - RH;
    };
    for (int q = threadIdx.x; q < G.Q; q += (NCW + 1) * 64) {
        int x0, b0, x1, b1;
        origin(q, x0, b0);
        origin(q + sg, x1, b1);   // walk slice q + sg: past either end of the walk it is never sampled
        const int w = G.w_start + sg * q;
        const int wl = min(max(w, 0), snw - 1);         // slices outside the brick: never sampled
        sh.tab[2 * q] = ring_off + (q % G.R) * G.SB - b0 * RWB - x0 * 4;
        sh.tab[2 * q + 1] = ring_off + ((q + sg) % G.R) * G.SB - b1 * RWB - x1 * 4;
        sh.src[q] = wl * w_stride + b0 * b_stride + x0;
    }
}

// DMA instructions per slice the producer can issue (a slot of at most
// ring_bytes / 8: the ring holds at least CH + 4 >= 8 slots).
template <int NCW>
constexpr int max_ni() { return ring_bytes<NCW>() / (8 * 1024); }

// Producer wavefront: stream the walk's slices into the ring.  It runs at a
// raised wave priority, so that the issue of its few instructions per slice
// is not held back by the marching wavefronts on its SIMD.  float16 slices
// land raw in the upper half of their slot and are decoded to float32 in
// place (front to back in 512-element chunks: chunk c writes bytes
// [2048 c, 2048 c + 2048), which lie below every byte of the halves still to
// be read) before the slice is published.
template <typename TS, int NCW, int CH, int W>
__device__ void ring_produce(const MarchParams& p, RingShared<NCW>& sh, const RingGeom& G, int* err) {
    constexpr int ESZ = sizeof(TS);
    constexpr int V = 16 / ESZ;
    constexpr int B = 3 - W;
    constexpr int EPI = 1024 / ESZ;              // elements per DMA instruction (64 lanes x 16 B)
    constexpr int MNI = max_ni<NCW>();
    typedef __attribute__((address_space(1))) void gvoid_t;
    typedef __attribute__((address_space(3))) void lvoid_t;
    __builtin_amdgcn_s_setprio(2);
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) const int lds_int;
    const int lane = threadIdx.x & 63;
    const BrickK& b = p.brick;
    const unsigned char* vox = reinterpret_cast<const unsigned char*>(b.data);
    const int sny = b.sdim[1];
    const int pitch = row_pitch(b.sdim[0]);
    const long long b_stride = W == 2 ? (long long)pitch : (long long)sny * pitch;
    const int RW = uniform_i(G.RW), RH = uniform_i(G.RH);
    const int NI = uniform_i(G.NI), SB = uniform_i(G.SB), R = uniform_i(G.R), D = uniform_i(G.D);
    const int Q = uniform_i(G.Q);
    const unsigned bstr = (unsigned)(b_stride * ESZ);
    const unsigned src_addr = (unsigned)(uintptr_t)((lds_int*)&sh.src[0]);
    const unsigned ring_addr = (unsigned)(uintptr_t)((lds_int*)(const void*)sh.ring);
    const int dma_base = ESZ == 2 ? SB / 2 : 0;         // float16: raw halves in the slot's upper half
    i32x4 src4 = {0, 0, 0, 0};
    // the LDS reads and writes of the decoding are inline asm for the reason
    // given at ld_lds_nowait_dma (other slices' DMA is still in flight)
    auto decode = [&](int sl) {
        if constexpr (ESZ == 2) {
            const unsigned base = ring_addr + (unsigned)(sl * SB);
            const int nch = (RW * RH + 511) >> 9;
            auto convert_store = [&](const i32x4& raw, int c) {
                const __half2* h = reinterpret_cast<const __half2*>(&raw);
                const float2 f0 = __half22float2(h[0]), f1 = __half22float2(h[1]);
                const float2 f2 = __half22float2(h[2]), f3 = __half22float2(h[3]);
                const i32x4 lo = {__float_as_int(f0.x), __float_as_int(f0.y), __float_as_int(f1.x),
                                  __float_as_int(f1.y)};
                const i32x4 hi = {__float_as_int(f2.x), __float_as_int(f2.y), __float_as_int(f3.x),
                                  __float_as_int(f3.y)};
                __asm__ volatile("ds_write_b128 %0, %1\n\tds_write_b128 %0, %2 offset:16"
                                 :: "v"(base + (unsigned)(2048 * c + 32 * lane)), "v"(lo), "v"(hi) : "memory");
            };
            // eight chunks per round trip: all read before any is written;
            // reads past the slice's last chunk stay inside the workgroup's LDS
            // (the slot's neighbour, or the tables after the ring) and their
            // results are dropped
            for (int c = 0; c < nch; c += 8) {
                i32x4 r0, r1, r2, r3, r4, r5, r6, r7;
                __asm__ volatile("ds_read_b128 %0, %8\n\tds_read_b128 %1, %8 offset:1024\n\t"
                                 "ds_read_b128 %2, %8 offset:2048\n\tds_read_b128 %3, %8 offset:3072\n\t"
                                 "ds_read_b128 %4, %8 offset:4096\n\tds_read_b128 %5, %8 offset:5120\n\t"
                                 "ds_read_b128 %6, %8 offset:6144\n\tds_read_b128 %7, %8 offset:7168\n\t"
                                 "s_waitcnt lgkmcnt(0)"
                                 : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6),
                                   "=&v"(r7)
                                 : "v"(base + (unsigned)(dma_base + 1024 * c + 16 * lane)) : "memory");
                convert_store(r0, c);
                if (c + 1 < nch) convert_store(r1, c + 1);
                if (c + 2 < nch) convert_store(r2, c + 2);
                if (c + 3 < nch) convert_store(r3, c + 3);
                if (c + 4 < nch) convert_store(r4, c + 4);
                if (c + 5 < nch) convert_store(r5, c + 5);
                if (c + 6 < nch) convert_store(r6, c + 6);
                if (c + 7 < nch) convert_store(r7, c + 7);
            }
            __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        }
        (void)sl;
    };
    int pub = 0, pslot = 0;                              // slices published; slot of slice `pub`
    auto publish = [&](int n) {                          // slices < n have landed: decode, publish
        for (; pub < n; ++pub) {
            decode(pslot);
            pslot = pslot + 1 == R ? 0 : pslot + 1;
        }
        compiler_fence();
        st_volatile(sh.ready, n);
    };
    // byte offset, within a slice's rectangle, of this lane's 16 bytes of each
    // DMA instruction (the same for every slice of the tile; lanes past the
    // rectangle's last row fetch its first bytes into the slot's padding)
    unsigned off[MNI];
#pragma unroll
    for (int i = 0; i < MNI; ++i) {
        const int e = i * EPI + lane * V;
        const int r = e / RW, c = e - r * RW;
        off[i] = r < RH ? (unsigned)r * bstr + (unsigned)(c * ESZ) : 0u;
    }
    int slot = 0, inflight = 0;
    int q = 0;
    int md = 0;                                          // last seen minimum of the done words
    for (; q < Q; ++q) {
        // wait for the slot of walk slice q: every consumer past slice q - R
        bool go = q < md + R;
        for (int it = 0; !go && it < kSpinLimit; ++it) {
            md = min_done<NCW>(sh.done);
            if (md >= kAllDone) break;                   // every consumer has finished
            if (q < md + R) {
                go = true;
                break;
            }
            if (inflight) {                               // publish before blocking
                wait_vmcnt<0>();
                publish(q);
                inflight = 0;
            }
            if (ld_lds_nowait_dma(sh.abort)) break;
            __builtin_amdgcn_s_sleep(1);
            if (it == kSpinLimit - 1) trip(sh, err);
        }
        compiler_fence();
        if (!go) break;
        // source offsets of four slices at a time (one 16-byte LDS read that
        // waits for itself; see ld_lds_nowait_dma)
        if ((q & 3) == 0) {
            __asm__ volatile("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(src4)
                             : "v"(src_addr + (unsigned)q * 4u) : "memory");
        }
        const int qi = q & 3;
        const int el = uniform_i(qi == 0 ? src4.x : qi == 1 ? src4.y : qi == 2 ? src4.z : src4.w);
        const unsigned char* sbase = vox + (long long)el * ESZ;
        unsigned char* dst = sh.ring + slot * SB;
#pragma unroll
        for (int i = 0; i < MNI; ++i)
            if (i < NI)
                __builtin_amdgcn_global_load_lds((gvoid_t*)(sbase + off[i]),
                                                 (lvoid_t*)(dst + dma_base + i * 1024), 16, 0, 0);
        slot = slot + 1 == R ? 0 : slot + 1;
        if (++inflight == D) {
            wait_vmcnt_le(NI * (D - 1));                 // slice q - D + 1 has landed
            publish(q - D + 2);
            --inflight;
        }
    }
    wait_vmcnt<0>();
    publish(q);
    __builtin_amdgcn_s_setprio(0);
}

template <typename TS>
__device__ inline float ring_ld(const unsigned char* p);
template <>
__device__ inline float ring_ld<float>(const unsigned char* p) {
    return *reinterpret_cast<const float*>(p);
}

// Consumer wavefront: march every lane's ray chunk by chunk from the ring.
template <typename TS, int NCW, int CH, int W>
__device__ void ring_consume(const MarchParams& p, RingShared<NCW>& sh, const RingGeom& G, int sg,
                             const RaySetup& rs, const Blocks& bl, bool has, long long pix, float tf_k,
                             float tf_o, float eps, LaneState& s, int* err) {
    constexpr int ESZ = 4;                       // the ring holds float32 for both storages
    constexpr int B = 3 - W;
    const int wave = threadIdx.x >> 6;
    const BrickK& b = p.brick;
    const TFTable& tft = sh.tft;
    const int RWB = G.RW * ESZ;
    // ring reads address the LDS from the start of sh (address 0), the slot
    // bases in tab include the ring's offset
    const unsigned lim = (unsigned)(offsetof(RingShared<NCW>, ring) + ring_bytes<NCW>() - RWB - 2 * ESZ);
    const unsigned char* R8 = reinterpret_cast<const unsigned char*>(&sh);
    const Step st = has ? make_step(rs, b, p.dt) : Step{0.f, 0.f, 0.f};
    long long k_cur = has ? rs.kf : 0;
    bool alive = has;
    long long an_blk = kNoBlock, k_anchor = 0;
    Anchor an{};
    int qoff = 0, rbase = 0;
    const int sgm = sg < 0 ? -1 : 0;                     // sg fw = (fw ^ sgm) - sgm for sg = +-1
    int seen = 0;                                        // last seen value of the ready word
    for (int kk = 0; kk < G.K; ++kk) {
        const long long kap = G.klo + kk;
        long long ke = 0;
        if (alive) ke = min(chunk_start(bl, p.inv_dt, kap + 1, CH), rs.kl + 1);
        const bool work = alive && k_cur < ke;
        if (__ballot(work)) {
            const int need = CH * kk + CH + 3;
            if (seen < need) {
                if (!wait_ge(sh, sh.ready, need, err)) break;
                seen = ld_volatile(sh.ready);
                compiler_fence();
            }
            if (work) {
                const long long blk = (kap * CH) >> 4;   // floor(kap CH / 16)
                if (blk != an_blk) {
                    an = make_anchor(rs, b, p.dt, k_cur);
                    an_blk = blk;
                    k_anchor = k_cur;
                    const int ia_w = W == 2 ? an.ia2 : an.ia1, ia_b = W == 2 ? an.ia1 : an.ia2;
                    qoff = sg * (ia_w - G.w_start) - sgm;
                    rbase = ia_b * RWB + an.ia0 * ESZ;
                }
                // stage 1: position, cell, and the two slices' table entries
                struct RingPre {
                    Cell c;
                    int row, t0, t1;
                };
                struct RingGather {
                    Cell c;
                    float v[8];
                };
                auto pre = [&](float fj) {
                    const float x = fmaf(fj, st.s0, an.uf0);
                    const float y = fmaf(fj, st.s1, an.uf1);
                    const float z = fmaf(fj, st.s2, an.uf2);
                    RingPre r;
                    r.c.fx = fract(x); r.c.fy = fract(y); r.c.fz = fract(z);
                    const int fx_i = floor_int(x);
                    const int fb = floor_int(W == 2 ? y : z), fw = floor_int(W == 2 ? z : y);
                    const int q = (fw ^ sgm) + qoff;   // sg fw + qoff (a single xor-add)
                    r.row = __mul24(fb, RWB) + fx_i * ESZ + rbase;
                    const int2 tp = reinterpret_cast<const int2*>(sh.tab)[q & kTabMask];
                    r.t0 = tp.x;
                    r.t1 = tp.y;
                    return r;
                };
                // stage 2: the 8 corner reads (unsigned clamps keep every read
                // inside the ring; for owned samples they never act)
                auto gather = [&](const RingPre& r) {
                    const unsigned a0 = min((unsigned)(r.t0 + r.row), lim);
                    const unsigned a1 = min((unsigned)(r.t1 + r.row), lim);
                    RingGather g;
                    g.c = r.c;
                    g.v[0] = ring_ld<float>(R8 + a0);       g.v[1] = ring_ld<float>(R8 + a0 + ESZ);
                    g.v[2] = ring_ld<float>(R8 + a0 + RWB); g.v[3] = ring_ld<float>(R8 + a0 + RWB + ESZ);
                    g.v[4] = ring_ld<float>(R8 + a1);       g.v[5] = ring_ld<float>(R8 + a1 + ESZ);
                    g.v[6] = ring_ld<float>(R8 + a1 + RWB); g.v[7] = ring_ld<float>(R8 + a1 + RWB + ESZ);
                    return g;
                };
                // stage 3: trilinear (v[0..3]: slice w, v[4..7]: slice w + 1;
                // odd index: x + 1; 2, 3, 6, 7: row b + 1)
                auto value = [&](const RingGather& g) {
                    return W == 2 ? lerp3(g.c, g.v[0], g.v[1], g.v[2], g.v[3], g.v[4], g.v[5], g.v[6], g.v[7])
                                  : lerp3(g.c, g.v[0], g.v[1], g.v[4], g.v[5], g.v[2], g.v[3], g.v[6], g.v[7]);
                };
                // 16-wide tiles (five waves, two per SIMD: 256 registers)
                // take the four-deep pipeline; 32-wide tiles (nine waves,
                // three per SIMD: 168 registers) the two-sample one
                bool cont;
                if constexpr (NCW == 4)
                    cont = march_run_deep(tft, rs, k_anchor, (int)(k_cur - k_anchor), (int)(ke - k_anchor),
                                          tf_k, tf_o, eps, s, pre, gather, value);
                else
                    cont = march_run_pipe(tft, rs, k_anchor, (int)(k_cur - k_anchor), (int)(ke - k_anchor),
                                          tf_k, tf_o, eps, s, pre, gather, value);
                k_cur = ke;
                alive = cont && k_cur <= rs.kl;
            }
        }
        compiler_fence();
        if ((threadIdx.x & 63) == 0) st_volatile(sh.done[wave], CH * (kk + 1));
        if (!__ballot(alive)) break;
    }
    compiler_fence();
    if ((threadIdx.x & 63) == 0) st_volatile(sh.done[wave], kAllDone);
}

// One TW x 16 tile of one partial image, by the whole workgroup (NCW + 1
// waves).  The classification table must already be in sh.tft (ordered by
// the first reduction's barrier); every thread must call it.
template <typename TS, int NCW, int CH>
__device__ void ring_tile(const MarchParams& p, int tile, RingShared<NCW>& sh, int& buf, int* err) {
    constexpr int NW = NCW + 1, TW = NCW * 4;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool producer = wave == NCW;
    const int tiles_x = (p.roi_w + TW - 1) / TW;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int wx = wave % (TW / 8), wy = wave / (TW / 8);
    const int lx = tx * TW + wx * 8 + (lane & 7), ly = ty * 16 + wy * 8 + (lane >> 3);
    const bool valid = !producer && lx < p.roi_w && ly < p.roi_h;
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
    long long kf_chunk = 0, kl_chunk = 0;
    if (has) {
        depth = (float)(((double)rs.kf + 0.5) * p.dt);
        bl = make_blocks(rs, b);
        dw_abs = (float)fabs(pick3(rs.d, bl.axis));
        kf_chunk = chunk_of(bl, p.dt, p.inv_dt, rs.kf, CH);
        kl_chunk = chunk_of(bl, p.dt, p.inv_dt, rs.kl, CH);
    }
    // the previous tile ended with a barrier: nobody reads the words now
    if (tid == 0) st_volatile(sh.ready, 0);
    if (lane == 0 && !producer) st_volatile(sh.done[wave], 0);
    // eligibility: every ray shares slab axis (y or z) and direction; the walk's chunk range
    const float key = (float)(bl.axis * 2 + (bl.sg > 0 ? 1 : 0));
    float v[6] = {has ? key : 1e9f, has ? key : -1e9f, has ? dw_abs : 1e9f, has ? 1.0f : 0.0f,
                  has ? (float)kf_chunk : 3e38f, has ? (float)kl_chunk : -3e38f};
    const bool mx[6] = {false, true, false, true, false, true};
    wg_reduce<6, NW>(v, mx, sh.red, buf, lane, wave);
    buf ^= 1;
    if (v[3] == 0.0f) {                      // no ray of this tile hits the brick
        finish(p, valid, pix, depth, s, lane);
        return;
    }
    bool ok = v[0] == v[1] && v[0] >= 2.0f && v[2] >= kMinStageDw;
    const int ukey = (int)v[0];
    const int W = ukey >> 1, sg = (ukey & 1) ? 1 : -1;
    const long long klo = (long long)v[4], khi = (long long)v[5];
    RingGeom G{};
    Lines L;
    if (ok) {
        const int px0 = p.roi_x0 + tx * TW, px1 = p.roi_x0 + min(tx * TW + TW - 1, p.roi_w - 1);
        const int py0 = p.roi_y0 + ty * 16, py1 = p.roi_y0 + min(ty * 16 + 15, p.roi_h - 1);
        if (W == 2) {
            corner_lines<2>(p, px0, px1, py0, py1, L);
            G = ring_geometry<TS, NCW, CH, 2>(p, L, sg, klo, khi);
        } else {
            corner_lines<1>(p, px0, px1, py0, py1, L);
            G = ring_geometry<TS, NCW, CH, 1>(p, L, sg, klo, khi);
        }
        ok = G.ok;
    }
    if (!ok) {                               // march this tile from HBM
        if (has) march_ray_direct<TS, false>(p, sh.tft, rs, pix, tf_k, tf_o, eps, s);
        finish(p, valid, pix, depth, s, lane);
        return;
    }
    if (W == 2) ring_tables<TS, NCW, CH, 2>(p, sh, L, G, sg);
    else ring_tables<TS, NCW, CH, 1>(p, sh, L, G, sg);
    __syncthreads();
    if (producer) {
        if (W == 2) ring_produce<TS, NCW, CH, 2>(p, sh, G, err);
        else ring_produce<TS, NCW, CH, 1>(p, sh, G, err);
    } else {
        if (W == 2) ring_consume<TS, NCW, CH, 2>(p, sh, G, sg, rs, bl, has, pix, tf_k, tf_o, eps, s, err);
        else ring_consume<TS, NCW, CH, 1>(p, sh, G, sg, rs, bl, has, pix, tf_k, tf_o, eps, s, err);
    }
    finish(p, valid, pix, depth, s, lane);
}

// One partial, one workgroup per tile (tiles in an XCD-aware order:
// workgroup i runs on XCD i mod 8, each XCD takes a contiguous run of tiles,
// a bijection on [0, gridDim.x)).
template <typename TS, int NCW, int CH>
__global__ __launch_bounds__((NCW + 1) * 64, 2) void march_staged(MarchParams p) {
    __shared__ RingShared<NCW> sh;
    load_tf(sh.tft, p.tf, p.dt, threadIdx.x, (NCW + 1) * 64);
    if (threadIdx.x == 0) sh.abort = 0;
    const int nb = gridDim.x, bid = blockIdx.x;
    const int per = nb / 8, rem = nb % 8, xcd = bid % 8;
    const int tile = xcd * per + min(xcd, rem) + bid / 8;
    int buf = 0;
    ring_tile<TS, NCW, CH>(p, tile, sh, buf, p.err);
}

// One 16x16 tile, every lane marching its own ray from HBM (no staging, no
// workgroup-wide steps).
template <typename TS>
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

// Persistent work-queue march: each workgroup repeatedly takes the next
// ticket (one tile of one job = one partial image) until the tickets run
// out, so many small partials (bricks x time steps x fields x cameras) fill
// the GPU together.  Tickets come from kQueueParts parts, the own XCD's part
// first.  The table is reloaded only when a job's transfer function (or dt)
// differs from the previous ticket's.
template <typename TS, typename Shared, typename TileFn>
__device__ inline void queue_loop(const QueueParams& q, Shared& sh, TFTable& tft, int& ticket, bool sync_tf,
                                  TileFn tile_fn) {
    const int tid = threadIdx.x;
    const float* tf_loaded = nullptr;
    float scale_loaded = -1.0f;
    double dt_loaded = -1.0;
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
                load_tf(tft, p.tf, p.dt, tid, blockDim.x);
                tf_loaded = p.tf.rgba;
                scale_loaded = p.tf.opacity_scale;
                dt_loaded = p.dt;
                if (sync_tf) __syncthreads();
            }
            tile_fn(p, t - q.tile_start[lo]);
            __syncthreads();
        }
    }
}

template <typename TS, int NCW, int CH>
__global__ __launch_bounds__((NCW + 1) * 64, 2) void march_queue_ring(QueueParams q) {
    __shared__ RingShared<NCW> sh;
    if (threadIdx.x == 0) sh.abort = 0;
    int buf = 0;
    // (ring_tile's first reduction barrier orders table writes before use)
    queue_loop<TS>(q, sh, sh.tft, sh.ticket, false, [&](const MarchParams& p, int tile) {
        ring_tile<TS, NCW, CH>(p, tile, sh, buf, q.err);
    });
}

template <typename TS>
__global__ __launch_bounds__(256) void march_queue_slab(QueueParams q) {
    __shared__ StagedShared sh;
    int buf = 0;
    // (slab_tile's first reduction barrier orders table writes before use)
    queue_loop<TS>(q, sh, sh.tft, sh.ticket, false,
                   [&](const MarchParams& p, int tile) { slab_tile<TS>(p, tile, sh, buf); });
}

struct DirectShared {
    TFTable tft;
    int ticket;
};

template <typename TS>
__global__ __launch_bounds__(256) void march_queue_direct(QueueParams q) {
    __shared__ DirectShared sh;
    queue_loop<TS>(q, sh, sh.tft, sh.ticket, true,
                   [&](const MarchParams& p, int tile) { direct_tile<TS>(p, tile, sh.tft); });
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

// Dispatch over the compiled staged configurations (tile width 16 or 32,
// chunk 4 or 8 slices) and storage precisions.
template <template <typename, int, int> class Fn, typename... A>
auto staged_dispatch(StorageK storage, int tile_w, int chunk, A&&... a) {
    const bool wide = tile_w == 32, long_chunk = chunk == 8;
    if (storage == kF16) {
        if (wide) return long_chunk ? Fn<__half, 8, 8>::run(a...) : Fn<__half, 8, 4>::run(a...);
        return long_chunk ? Fn<__half, 4, 8>::run(a...) : Fn<__half, 4, 4>::run(a...);
    }
    if (wide) return long_chunk ? Fn<float, 8, 8>::run(a...) : Fn<float, 8, 4>::run(a...);
    return long_chunk ? Fn<float, 4, 8>::run(a...) : Fn<float, 4, 4>::run(a...);
}

template <typename TS, int NCW, int CH>
struct LaunchQueueRing {
    static hipError_t run(const QueueParams& q, int grid, hipStream_t stream) {
        hipLaunchKernelGGL((march_queue_ring<TS, NCW, CH>), dim3(grid), dim3((NCW + 1) * 64), 0, stream, q);
        return hipGetLastError();
    }
};

template <typename TS, int NCW, int CH>
struct OccupancyRing {
    static int run() {
        int n = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, march_queue_ring<TS, NCW, CH>,
                                                                    (NCW + 1) * 64, 0);
        return (e == hipSuccess && n > 0) ? n : 1;
    }
};

template <typename TS, int NCW, int CH>
struct LaunchStaged {
    static hipError_t run(const MarchParams& p, int blocks, hipStream_t stream) {
        hipLaunchKernelGGL((march_staged<TS, NCW, CH>), dim3(blocks), dim3((NCW + 1) * 64), 0, stream, p);
        return hipGetLastError();
    }
};

template <typename TS>
int occupancy_direct() {
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, march_queue_direct<TS>, 256, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

template <typename TS>
int occupancy_slab() {
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, march_queue_slab<TS>, 256, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

hipError_t launch_march_queue(const QueueParams& q, StorageK storage, int workgroups,
                              hipStream_t stream) {
    if (q.total_tiles <= 0) return hipSuccess;
    if (q.staged && !valid_march_config(q.staging, q.tile_w, q.chunk)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(queue_reset, dim3(1), dim3(64), 0, stream, q.head);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = min(workgroups, q.total_tiles);
    if (!q.staged) {
        if (storage == kF16)
            hipLaunchKernelGGL(march_queue_direct<__half>, dim3(grid), dim3(256), 0, stream, q);
        else
            hipLaunchKernelGGL(march_queue_direct<float>, dim3(grid), dim3(256), 0, stream, q);
        return hipGetLastError();
    }
    if (q.staging == kStagingSlab) {
        if (storage == kF16)
            hipLaunchKernelGGL(march_queue_slab<__half>, dim3(grid), dim3(256), 0, stream, q);
        else
            hipLaunchKernelGGL(march_queue_slab<float>, dim3(grid), dim3(256), 0, stream, q);
        return hipGetLastError();
    }
    return staged_dispatch<LaunchQueueRing>(storage, q.tile_w, q.chunk, q, grid, stream);
}

int march_queue_workgroups_per_cu(StorageK storage, bool staged, int staging, int tile_w, int chunk) {
    if (!staged) return storage == kF16 ? occupancy_direct<__half>() : occupancy_direct<float>();
    if (!valid_march_config(staging, tile_w, chunk)) return 1;
    if (staging == kStagingSlab) return storage == kF16 ? occupancy_slab<__half>() : occupancy_slab<float>();
    return staged_dispatch<OccupancyRing>(storage, tile_w, chunk);
}

hipError_t launch_march_checkpointed_many(const MarchParams* jobs, const int32_t* tile_start, int32_t n_jobs,
                                          int32_t total_tiles, StorageK storage, hipStream_t stream) {
    if (n_jobs <= 0 || total_tiles <= 0) return hipSuccess;
    if (storage == kF16)
        hipLaunchKernelGGL(march_checkpointed_many<__half>, dim3(total_tiles), dim3(64), 0, stream, jobs, tile_start,
                           n_jobs);
    else
        hipLaunchKernelGGL(march_checkpointed_many<float>, dim3(total_tiles), dim3(64), 0, stream, jobs, tile_start,
                           n_jobs);
    return hipGetLastError();
}

hipError_t launch_march(const MarchParams& p, StorageK storage, hipStream_t stream) {
    if (p.ckpt) return launch_direct<true>(p, storage, stream);
    if (p.path == kPathDirect) return launch_direct<false>(p, storage, stream);
    if (!valid_march_config(p.staging, p.tile_w, p.chunk)) return hipErrorInvalidValue;
    // staged: one workgroup per tile_w x 16 tile
    const int blocks = queue_tiles(p.roi_w, p.roi_h, p.tile_w);
    if (blocks == 0) return hipSuccess;
    if (p.staging == kStagingSlab) {
        MarchParams q = p;
        q.tiles_x = (p.roi_w + 15) / 16;
        q.tiles_y = (p.roi_h + 15) / 16;
        if (storage == kF16)
            hipLaunchKernelGGL(march_slab_single<__half>, dim3(blocks), dim3(256), 0, stream, q);
        else
            hipLaunchKernelGGL(march_slab_single<float>, dim3(blocks), dim3(256), 0, stream, q);
        return hipGetLastError();
    }
    return staged_dispatch<LaunchStaged>(storage, p.tile_w, p.chunk, p, blocks, stream);
}

}  // namespace dpvr
