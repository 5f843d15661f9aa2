// Device-side pieces shared by every kernel that marches rays through a
// brick (forward, checkpointed forward, adjoint, batched): the float64 ray
// setup and ownership scan, the float64 re-anchoring of float32 stored-index
// coordinates, the trilinear sample and the classification table.  Sharing
// them keeps the sample positions and values of all paths bit-identical.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <math.h>

#include "dpvr_kernels.h"

namespace dpvr {

constexpr int kSlab = 16;         // anchor block = slab of kSlab slices along the ray's w axis
constexpr float kLog2e = 1.4426950408889634f;

struct RaySetup {
    double o[3], d[3];
    long long kf, kl;             // first / last owned sample index
};

__device__ inline bool owned(const double o[3], const double d[3], double t, const double lo[3],
                             const double hi[3]) {
#pragma clang fp contract(off)
    double p0 = o[0] + t * d[0], p1 = o[1] + t * d[1], p2 = o[2] + t * d[2];
    return p0 >= lo[0] && p0 < hi[0] && p1 >= lo[1] && p1 < hi[1] && p2 >= lo[2] && p2 < hi[2];
}

// Camera ray (origin o, unit direction d) through the centre of pixel
// (px, py).  float64, no contraction, in the operation order of the
// documented formulas (the same expressions as setup_ray).
struct CamRay {
    double o[3], d[3];
};

__device__ inline CamRay camera_ray(const CameraK& cam, int px, int py) {
#pragma clang fp contract(off)
    const double W = (double)cam.width, H = (double)cam.height;
    const double sx = (2.0 * ((double)px + 0.5)) / W - 1.0;
    const double sy = 1.0 - (2.0 * ((double)py + 0.5)) / H;
    const double x = sx * cam.ax, y = sy * cam.ay;
    CamRay r;
    if (cam.kind == 0) {
        double d0 = (cam.f[0] + x * cam.r[0]) + y * cam.u[0];
        double d1 = (cam.f[1] + x * cam.r[1]) + y * cam.u[1];
        double d2 = (cam.f[2] + x * cam.r[2]) + y * cam.u[2];
        double n = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        r.d[0] = d0 / n; r.d[1] = d1 / n; r.d[2] = d2 / n;
        r.o[0] = cam.eye[0]; r.o[1] = cam.eye[1]; r.o[2] = cam.eye[2];
    } else {
        r.o[0] = (cam.eye[0] + x * cam.r[0]) + y * cam.u[0];
        r.o[1] = (cam.eye[1] + x * cam.r[1]) + y * cam.u[1];
        r.o[2] = (cam.eye[2] + x * cam.r[2]) + y * cam.u[2];
        r.d[0] = cam.f[0]; r.d[1] = cam.f[1]; r.d[2] = cam.f[2];
    }
    return r;
}

// Camera ray through pixel (px, py) and the brick's owned run [kf, kl] of the
// global lattice t_k = (k + 1/2) dt.  float64, no contraction; the same
// expressions as camera_ray (written out: storing through array pointers
// there would keep the ray in scratch memory).
__device__ inline bool setup_ray(const CameraK& cam, const BrickK& b, double dt, int px, int py,
                                 RaySetup& rs) {
#pragma clang fp contract(off)
    const double W = (double)cam.width, H = (double)cam.height;
    const double sx = (2.0 * ((double)px + 0.5)) / W - 1.0;
    const double sy = 1.0 - (2.0 * ((double)py + 0.5)) / H;
    const double x = sx * cam.ax, y = sy * cam.ay;
    if (cam.kind == 0) {
        double d0 = (cam.f[0] + x * cam.r[0]) + y * cam.u[0];
        double d1 = (cam.f[1] + x * cam.r[1]) + y * cam.u[1];
        double d2 = (cam.f[2] + x * cam.r[2]) + y * cam.u[2];
        double n = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        rs.d[0] = d0 / n; rs.d[1] = d1 / n; rs.d[2] = d2 / n;
        rs.o[0] = cam.eye[0]; rs.o[1] = cam.eye[1]; rs.o[2] = cam.eye[2];
    } else {
        rs.o[0] = (cam.eye[0] + x * cam.r[0]) + y * cam.u[0];
        rs.o[1] = (cam.eye[1] + x * cam.r[1]) + y * cam.u[1];
        rs.o[2] = (cam.eye[2] + x * cam.r[2]) + y * cam.u[2];
        rs.d[0] = cam.f[0]; rs.d[1] = cam.f[1]; rs.d[2] = cam.f[2];
    }
    double tin = 0.0, tout = INFINITY;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (rs.d[c] == 0.0) {
            if (rs.o[c] < b.lo[c] || rs.o[c] >= b.hi[c]) return false;
            continue;
        }
        double ta = (b.lo[c] - rs.o[c]) / rs.d[c], tb = (b.hi[c] - rs.o[c]) / rs.d[c];
        tin = fmax(tin, fmin(ta, tb));
        tout = fmin(tout, fmax(ta, tb));
    }
    if (!(tout >= tin - 2.0 * dt)) return false;
    long long k0 = (long long)fmax(floor(tin / dt - 0.5) - 2.0, 0.0);
    long long k1 = (long long)(ceil(tout / dt - 0.5) + 2.0);
    if (k1 < k0) return false;
    // The owned samples form one contiguous run (convex box; every rounded
    // coordinate is monotone in k); scan in from both ends of the widened range.
    long long kf = k0;
    while (kf <= k1 && !owned(rs.o, rs.d, ((double)kf + 0.5) * dt, b.lo, b.hi)) ++kf;
    if (kf > k1) return false;
    long long kl = k1;
    while (kl > kf && !owned(rs.o, rs.d, ((double)kl + 0.5) * dt, b.lo, b.hi)) --kl;
    rs.kf = kf;
    rs.kl = kl;
    return true;
}

// Any ray (origin o, unit direction d, float64) and its owned run [kf, kl] of
// the lattice t_k = (k + 1/2) dt in brick b, by the ownership scan of
// setup_ray (shadow rays start at a primary sample and head for the light).
__device__ inline bool setup_ray_from(double o0, double o1, double o2, double d0, double d1, double d2,
                                      const BrickK& b, double dt, RaySetup& rs) {
#pragma clang fp contract(off)
    rs.o[0] = o0; rs.o[1] = o1; rs.o[2] = o2;
    rs.d[0] = d0; rs.d[1] = d1; rs.d[2] = d2;
    double tin = 0.0, tout = INFINITY;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (rs.d[c] == 0.0) {
            if (rs.o[c] < b.lo[c] || rs.o[c] >= b.hi[c]) return false;
            continue;
        }
        double ta = (b.lo[c] - rs.o[c]) / rs.d[c], tb = (b.hi[c] - rs.o[c]) / rs.d[c];
        tin = fmax(tin, fmin(ta, tb));
        tout = fmin(tout, fmax(ta, tb));
    }
    if (!(tout >= tin - 2.0 * dt)) return false;
    long long k0 = (long long)fmax(floor(tin / dt - 0.5) - 2.0, 0.0);
    long long k1 = (long long)(ceil(tout / dt - 0.5) + 2.0);
    if (k1 < k0) return false;
    long long kf = k0;
    while (kf <= k1 && !owned(rs.o, rs.d, ((double)kf + 0.5) * dt, b.lo, b.hi)) ++kf;
    if (kf > k1) return false;
    long long kl = k1;
    while (kl > kf && !owned(rs.o, rs.d, ((double)kl + 0.5) * dt, b.lo, b.hi)) --kl;
    rs.kf = kf;
    rs.kl = kl;
    return true;
}

// Anchor blocks.  Every ray picks a slab axis w (z or y, whichever has the
// larger direction component; x only if both are below 1/16) and cuts its
// owned samples at the planes s_w = kSlab * m of the brick's stored-index
// coordinate (s = (p - origin) / spacing - 1/2 + ghost).  In ray order the
// planes are numbered n (plane s_w = kSlab * sg * n, sg = sign d_w); the ray
// crosses plane n at t_n = c0 + n * c1 (c1 > 0), and block n holds the samples
// k with k_n <= k < k_{n+1}, k_n = ceil(t_n / dt - 1/2).  A block's float32
// positions are anchored (float64) at its first owned sample max(kf, k_n).
// The rule depends on the ray alone, so every kernel and every launch
// configuration evaluates every sample at the same float32 position.
struct Blocks {
    double c0, c1;
    int axis, sg;
};

// v[i] for a run-time i without indexing a register array (which would spill
// the array to scratch memory).
template <typename T>
__device__ inline T pick3(const T (&v)[3], int i) {
    return i == 2 ? v[2] : (i == 1 ? v[1] : v[0]);
}

__device__ inline Blocks make_blocks(const RaySetup& rs, const BrickK& b) {
#pragma clang fp contract(off)
    Blocks bl;
    const double ay = fabs(rs.d[1]), az = fabs(rs.d[2]);
    bl.axis = (az >= ay) ? 2 : 1;
    if (fmax(ay, az) < 0.0625) bl.axis = 0;
    const int w = bl.axis;
    const double dw = pick3(rs.d, w);
    bl.sg = dw > 0.0 ? 1 : -1;
    // s_w(t) = (o_w + t d_w - origin_w) / sp_w - 1/2 + g = kSlab sg n
    const double spw = pick3(b.spacing, w);
    bl.c0 = ((0.5 - (double)b.ghost) * spw + pick3(b.origin, w) - pick3(rs.o, w)) / dw;
    bl.c1 = ((double)(kSlab * bl.sg) * spw) / dw;
    return bl;
}

__device__ inline long long block_start(const Blocks& bl, double inv_dt, long long n) {
#pragma clang fp contract(off)
    const double t = bl.c0 + (double)n * bl.c1;
    return (long long)ceil(t * inv_dt - 0.5);
}

// Block (plane index n) holding sample k: the largest n with k_n <= k.
__device__ inline long long block_of(const Blocks& bl, double dt, double inv_dt, long long k) {
#pragma clang fp contract(off)
    const double t = ((double)k + 0.5) * dt;
    long long n = (long long)floor((t - bl.c0) / bl.c1);
    while (block_start(bl, inv_dt, n) > k) --n;
    while (block_start(bl, inv_dt, n + 1) <= k) ++n;
    return n;
}

// float32 stored-index coordinate of sample k = kb + j is  anchor + j * step,
// with the anchor (integer part ia, fraction uf) computed in float64 at kb.
struct Anchor {
    int ia0, ia1, ia2;
    float uf0, uf1, uf2;
};

__device__ inline Anchor make_anchor(const RaySetup& rs, const BrickK& b, double dt, long long kb) {
#pragma clang fp contract(off)
    const double t = ((double)kb + 0.5) * dt;
    const double g = (double)b.ghost - 0.5;
    Anchor a;
    double s0 = (rs.o[0] + t * rs.d[0] - b.origin[0]) * b.inv_spacing[0] + g;
    double s1 = (rs.o[1] + t * rs.d[1] - b.origin[1]) * b.inv_spacing[1] + g;
    double s2 = (rs.o[2] + t * rs.d[2] - b.origin[2]) * b.inv_spacing[2] + g;
    double f0 = floor(s0), f1 = floor(s1), f2 = floor(s2);
    a.ia0 = (int)f0; a.ia1 = (int)f1; a.ia2 = (int)f2;
    a.uf0 = (float)(s0 - f0); a.uf1 = (float)(s1 - f1); a.uf2 = (float)(s2 - f2);
    return a;
}

struct Step {
    float s0, s1, s2;
};

__device__ inline Step make_step(const RaySetup& rs, const BrickK& b, double dt) {
    Step s;
    s.s0 = (float)(dt * rs.d[0] / b.spacing[0]);
    s.s1 = (float)(dt * rs.d[1] / b.spacing[1]);
    s.s2 = (float)(dt * rs.d[2] / b.spacing[2]);
    return s;
}

// floor(x) as an int, and the fraction x - floor(x) (v_fract_f32, which
// returns the largest float below 1 where that difference would round up
// to 1).
// floor to int in one instruction (v_cvt_flr_i32_f32: floor, then convert;
// the same integer as (int)floorf(x) for every x whose floor fits an int)
__device__ inline int floor_int(float x) {
    int r;
    __asm__("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}
__device__ inline float fract(float x) { return __builtin_amdgcn_fractf(x); }

// Position of sample j (fj = j as float) after the anchor: base stored index
// (clamped so that the +1 neighbours stay inside the stored array) and
// trilinear fractions.  For owned samples the clamp never acts (the ghost
// layer covers every corner), so paths that skip it read the same voxels.
struct Cell {
    int ix, iy, iz;
    float fx, fy, fz;
};

__device__ inline Cell locate(const Anchor& a, const Step& st, float fj, int snx, int sny, int snz) {
    // snx = stored extent in x (not the row pitch)
    const float x = fmaf(fj, st.s0, a.uf0);
    const float y = fmaf(fj, st.s1, a.uf1);
    const float z = fmaf(fj, st.s2, a.uf2);
    Cell c;
    c.fx = fract(x); c.fy = fract(y); c.fz = fract(z);
    c.ix = min(max(a.ia0 + floor_int(x), 0), snx - 2);
    c.iy = min(max(a.ia1 + floor_int(y), 0), sny - 2);
    c.iz = min(max(a.ia2 + floor_int(z), 0), snz - 2);
    return c;
}

// Transmittance factor exp2(-a') with the hardware exp2 (1 ulp).  a' >= 0,
// so the result lies in (0, 1]; results below the smallest normal float
// flush to 0, which only affects transmittances below 2^-126.  Every kernel
// uses this one function, so all paths agree bit for bit.
__device__ inline float trans_exp2(float neg_a) { return __builtin_amdgcn_exp2f(neg_a); }

// Voxel loads through global-address-space pointers (the brick pointer comes
// from a job table in memory, where the compiler cannot infer the address
// space and would emit flat loads).
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) const unsigned short ghalf_bits;

template <typename TS>
__device__ inline float ld(const TS* p, long long i);
template <>
__device__ inline float ld<float>(const float* p, long long i) {
    return ((gfloat*)p)[i];
}
template <>
__device__ inline float ld<__half>(const __half* p, long long i) {
    return __half2float(__ushort_as_half(((ghalf_bits*)p)[i]));
}

// Trilinear interpolation of the 8 corner values, x first, then y, then z
// (the one order every path uses).
__device__ inline float lerp3(const Cell& c, float v000, float v100, float v010, float v110,
                              float v001, float v101, float v011, float v111) {
    const float v00 = fmaf(c.fx, v100 - v000, v000);
    const float v10 = fmaf(c.fx, v110 - v010, v010);
    const float v01 = fmaf(c.fx, v101 - v001, v001);
    const float v11 = fmaf(c.fx, v111 - v011, v011);
    const float v0 = fmaf(c.fy, v10 - v00, v00);
    const float v1 = fmaf(c.fy, v11 - v01, v01);
    return fmaf(c.fz, v1 - v0, v0);
}

// Corner values straight from the brick in HBM: pitch = row pitch (elements),
// sxy = pitch * stored y extent.
template <typename TS>
__device__ inline float trilinear(const TS* __restrict__ vox, const Cell& c, int pitch, long long sxy) {
    const long long base = (long long)c.iz * sxy + (long long)c.iy * pitch + c.ix;
    return lerp3(c, ld(vox, base), ld(vox, base + 1), ld(vox, base + pitch),
                 ld(vox, base + pitch + 1), ld(vox, base + sxy), ld(vox, base + sxy + 1),
                 ld(vox, base + sxy + pitch), ld(vox, base + sxy + pitch + 1));
}

// Row pitch of the stored brick (elements): x extent rounded up to 8, so that
// every row starts 16-byte aligned for both storage precisions.
__host__ __device__ inline int row_pitch(int snx) { return (snx + 7) & ~7; }

// Classification table in LDS: entry i = (r, g, b, a') with a' = alpha *
// opacity_scale * dt * log2(e), and the difference to entry i + 1.
struct TFTable {
    float4 base[256];
    float4 diff[256];
};

__device__ inline void load_tf(TFTable& t, const TFK& tf, double dt, int tid, int nthreads) {
    const float a_scale = tf.opacity_scale * (float)dt * kLog2e;
    for (int e = tid; e < 256; e += nthreads) {
        float4 v0 = reinterpret_cast<const float4*>(tf.rgba)[e];
        float4 v1 = reinterpret_cast<const float4*>(tf.rgba)[e < 255 ? e + 1 : 255];
        v0.w *= a_scale;
        v1.w *= a_scale;
        t.base[e] = v0;
        t.diff[e] = make_float4(v1.x - v0.x, v1.y - v0.y, v1.z - v0.z, v1.w - v0.w);
    }
}

struct Classified {
    float r, g, b, a;   // a = pre-scaled opacity a'
    float phi;
    int seg;
    bool inside;        // v within [vmin, vmax] (the lookup is not clamped)
};

__device__ inline Classified classify(const TFTable& t, float v, float tf_k, float tf_o) {
    Classified c;
    const float sr = fmaf(v, tf_k, tf_o);
    c.inside = sr >= 0.0f && sr <= 255.0f;
    const float s = fminf(fmaxf(sr, 0.0f), 255.0f);
    c.seg = min((int)s, 254);
    c.phi = s - (float)c.seg;
    const float4 eb = t.base[c.seg], ed = t.diff[c.seg];
    c.r = fmaf(c.phi, ed.x, eb.x);
    c.g = fmaf(c.phi, ed.y, eb.y);
    c.b = fmaf(c.phi, ed.z, eb.z);
    c.a = fmaf(c.phi, ed.w, eb.w);
    return c;
}

}  // namespace dpvr
