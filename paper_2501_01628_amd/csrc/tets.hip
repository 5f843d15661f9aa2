// Tetrahedral parts: volume ray casting of unstructured meshes split into
// (possibly non-convex) parts, the parts standing in for the ranks that own
// a share of a finite-element data set.
//
// A frame, for n parts and the context camera:
//   march     one workgroup per tile of a part's ROI (the part's bounding
//             box projected), wavefronts of 8 x 8 rays.
//             Every lattice sample t_k = (k + 1/2) dt of the ray inside the
//             part's bounding box is located in the part: by a short walk
//             from the tetrahedron that held the ray's previous sample (to the
//             neighbour across the first face that rejects the sample), else
//             among the tetrahedra listed in the sample's cell of the part's
//             uniform grid.  A tetrahedron holds p when its four signed sub-volumes
//             are positive, a zero one counting when the tie direction enters
//             across that face, so a sample has one owner in the whole mesh
//             and the first tetrahedron found is that owner.  The value is
//             the barycentric interpolation of the vertex values, classified
//             and accumulated front to back as in the brick march.  A part
//             that is not convex can hold several stretches of a ray: each
//             maximal run of consecutive held samples becomes a run
//             (first sample index, premultiplied colour, alpha).
//   resolve   per pixel, the runs of all parts in sample-index order with
//             "over", then the background.  Runs of different parts never
//             share a sample, so this equals accumulating the whole ray.
// With one directional light, before the march: a count pass (held samples
// per ROI pixel of every part), an exclusive scan (a slot per held sample), a
// record pass (each slot's sample index), then n cycle steps in which every
// slot's shadow ray visits part (home + s) mod n, and the march scales each
// held sample's emission by a0 + (1 - a0) S from its slot.
// Locations use float64 with contraction off (the planes come from the host
// in float64), so the owner of a sample does not depend on the launch.
#include "march_common.h"
#include "tet_kernels.h"

namespace dpvr {
namespace {

typedef __attribute__((address_space(1))) const double gdouble;
typedef __attribute__((address_space(1))) const float gfloat_t;
typedef __attribute__((address_space(1))) const int32_t gint;
typedef __attribute__((address_space(1))) const uint32_t guint;

// Value of vertex v: given, or (a cell centre) the mean of its cell's
// nodes, summed in node order.
__device__ inline float vertex_value(const float* __restrict__ vv, int32_t n_input,
                                     const int32_t* __restrict__ centre_nodes, int32_t v) {
    if (v < n_input) return vv[v];
    const int32_t* c = centre_nodes + 8 * (long long)(v - n_input);
    float s = 0.0f;
    int n = 0;
    for (; n < 8 && c[n] >= 0; ++n) s += vv[c[n]];
    return s / (float)n;
}

__global__ __launch_bounds__(256) void tet_values(const float* __restrict__ vv, int32_t n_input,
                                                  const int32_t* __restrict__ centre_nodes,
                                                  const int4* __restrict__ tets, int32_t n,
                                                  float4* __restrict__ vals) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const int4 t = tets[e];
    vals[e] = make_float4(vertex_value(vv, n_input, centre_nodes, t.x), vertex_value(vv, n_input, centre_nodes, t.y),
                          vertex_value(vv, n_input, centre_nodes, t.z), vertex_value(vv, n_input, centre_nodes, t.w));
}

// Candidate sample indices [k0, k1] of the ray against the closed box
// [lo, hi], widened by two samples on each side (rounding of the slab
// parameters never drops a sample; ownership is decided per sample).
__device__ inline bool box_range(const CamRay& r, const double lo[3], const double hi[3], double dt,
                                 long long& k0, long long& k1) {
#pragma clang fp contract(off)
    double tin = 0.0, tout = INFINITY;
    for (int c = 0; c < 3; ++c) {
        if (r.d[c] == 0.0) {
            if (r.o[c] < lo[c] || r.o[c] > hi[c]) return false;
            continue;
        }
        const double ta = (lo[c] - r.o[c]) / r.d[c], tb = (hi[c] - r.o[c]) / r.d[c];
        tin = fmax(tin, fmin(ta, tb));
        tout = fmin(tout, fmax(ta, tb));
    }
    if (!(tout >= tin - 2.0 * dt)) return false;
    const double a = fmax(floor(tin / dt - 0.5) - 2.0, 0.0), b = ceil(tout / dt - 0.5) + 2.0;
    if (!(b >= a)) return false;
    k0 = (long long)a;
    k1 = (long long)b;
    return true;
}

// Whether tetrahedron e holds p; if so its four sub-volumes in D, if not
// the first face that rejects p in *out.
__device__ inline bool holds(const TetPartK& P, int e, double p0, double p1, double p2, double D[4], int* out) {
#pragma clang fp contract(off)
    gdouble* pl = ((gdouble*)P.planes) + 16 * (long long)e;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        D[i] = ((pl[4 * i] * p0 + pl[4 * i + 1] * p1) + pl[4 * i + 2] * p2) - pl[4 * i + 3];
        if (D[i] < 0.0 || (D[i] == 0.0 && !((((guint*)P.owned)[e] >> i) & 1u))) {
            *out = i;
            return false;
        }
    }
    return true;
}

// Steps of the walk from the previous sample's tetrahedron across rejecting
// faces before the grid is searched.
constexpr int kWalkSteps = 4;

// Adds every lane's n to *counter (one atomic per wavefront); all lanes of
// the wavefront call it.
__device__ inline void count_held(unsigned long long* counter, unsigned long long n) {
    if (!counter) return;
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(counter, n);
}

// The tetrahedron of part P that holds p (-1: none) by the BVH: from the
// root, a node whose box holds p is entered (its first child follows it; a
// leaf's tetrahedra are tested), any other is skipped through its skip link.
__device__ inline int bvh_locate(const TetPartK& P, double p0, double p1, double p2, double D[4]) {
    int node = P.n_tets > 0 ? 0 : -1, face = 0;
    while (node >= 0) {
        gint* nd = ((gint*)P.bvh_nodes) + 8 * (long long)node;
        const int skip = nd[3], leaf = nd[7];
        const bool in = p0 >= (double)__int_as_float(nd[0]) && p1 >= (double)__int_as_float(nd[1]) &&
                        p2 >= (double)__int_as_float(nd[2]) && p0 <= (double)__int_as_float(nd[4]) &&
                        p1 <= (double)__int_as_float(nd[5]) && p2 <= (double)__int_as_float(nd[6]);
        if (!in) {
            node = skip;
        } else if (leaf >= 0) {
            const int first = leaf >> 3, count = leaf & 7;
            for (int i = 0; i < count; ++i) {
                const int e = ((gint*)P.bvh_tets)[first + i];
                if (holds(P, e, p0, p1, p2, D, &face)) return e;
            }
            node = skip;
        } else {
            node = node + 1;
        }
    }
    return -1;
}

// The tetrahedron of part P that holds p (-1: none): one candidate per loop
// trip, so that the lanes of a wavefront stay on the same code -- first the
// walk from tetrahedron `from` (kWalkSteps tests, across the first face that
// rejects p), then the tetrahedra of p's grid cell.  D: its sub-volumes.
template <int kLocator>
__device__ inline int locate(const TetPartK& P, int from, double p0, double p1, double p2, double D[4]) {
#pragma clang fp contract(off)
    int cand = from, face = 0, walk = kWalkSteps, q = 0, qend = 0;
    bool grid = false;
    for (;;) {
        if (cand < 0) {
            if (kLocator == kTetBvh) return bvh_locate(P, p0, p1, p2, D);
            if (!grid) {
                grid = true;
                const double u0 = (p0 - P.glo[0]) * P.ginv[0], u1 = (p1 - P.glo[1]) * P.ginv[1],
                             u2 = (p2 - P.glo[2]) * P.ginv[2];
                if (u0 >= 0.0 && u1 >= 0.0 && u2 >= 0.0 && u0 < (double)P.gdim[0] && u1 < (double)P.gdim[1] &&
                    u2 < (double)P.gdim[2]) {
                    const long long cell = ((long long)(int)u2 * P.gdim[1] + (int)u1) * P.gdim[0] + (int)u0;
                    q = ((gint*)P.cell_start)[cell];
                    qend = ((gint*)P.cell_start)[cell + 1];
                }
            }
            if (q >= qend) return -1;
            cand = ((gint*)P.cell_tets)[q++];
        }
        if (holds(P, cand, p0, p1, p2, D, &face)) return cand;
        cand = !grid && --walk > 0 ? ((gint*)P.nbr)[4 * (long long)cand + face] : -1;
    }
}

// Barycentric value of a point with sub-volumes D in tetrahedron e: the
// weighted sum in float64, one float32 division (the value is classified in
// float32).
__device__ inline float tet_value(const TetPartK& P, int e, const double D[4]) {
#pragma clang fp contract(off)
    gfloat_t* vv = ((gfloat_t*)P.vals) + 4 * (long long)e;
    const double s = ((D[0] + D[1]) + D[2]) + D[3];
    const double num = ((D[0] * (double)vv[0] + D[1] * (double)vv[1]) + D[2] * (double)vv[2]) + D[3] * (double)vv[3];
    return __fdividef((float)num, (float)s);
}

constexpr int kTetThreads = kTetTile * kTetTile;

// The march of every part's ROI rays, in one of four modes: kTetMarch
// (runs), kTetCount (held samples per frame entry into offsets), kTetRecord
// (the sample index of every held sample into its slot) and kTetShaded (runs
// with every held sample's emission scaled by a0 + (1 - a0) S from its slot).
template <int kMode, int kLocator>
__global__ __launch_bounds__(kTetThreads) void tet_march(TetFrameParams f) {
    constexpr bool kRuns = kMode == kTetMarch || kMode == kTetShaded;
    __shared__ TFTable tft;
    if (kRuns) {
        load_tf(tft, f.tf, f.dt, threadIdx.x, kTetThreads);
        __syncthreads();
    }
    const int wg = blockIdx.x;
    int lo = 0, hi = f.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (f.tile_start[mid] <= wg) lo = mid; else hi = mid - 1;
    }
    const int j = __builtin_amdgcn_readfirstlane(lo);
    // a copy in registers: the run stores below cannot alias it, so its
    // fields are loaded once
    const TetPartK P = f.parts[j];
    const int tile = wg - f.tile_start[j];
    const int tiles_x = (P.roi_w + kTetTile - 1) / kTetTile;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lx = (tile % tiles_x) * kTetTile + (wave % (kTetTile / 8)) * 8 + (lane & 7);
    const int ly = (tile / tiles_x) * kTetTile + (wave / (kTetTile / 8)) * 8 + (lane >> 3);
    const bool live = lx < P.roi_w && ly < P.roi_h;
    const long long npix = (long long)P.roi_w * P.roi_h;
    const long long li = (long long)ly * P.roi_w + lx;
    const float tf_k = 255.0f / (f.tf.vmax - f.tf.vmin);
    const float tf_o = -f.tf.vmin * tf_k;
    const float a0 = f.ambient, a1 = 1.0f - f.ambient;
    unsigned long long held = 0;
    int nrun = 0;
    long long k0 = 0, k1 = -1, slot0 = 0, slots = 0;
    CamRay r{};
    if (live) {
        r = camera_ray(f.cam, P.roi_x0 + lx, P.roi_y0 + ly);
        if (box_range(r, P.lo, P.hi, f.dt, k0, k1) && k1 > 0x7fffffffLL) {
            if (f.err) atomicOr(f.err, kErrRange);
            k1 = k0 - 1;
        }
        if (kMode == kTetRecord || kMode == kTetShaded) {
            slot0 = f.offsets[P.entry0 + li];
            slots = f.offsets[P.entry0 + li + 1] - slot0;   // the count pass's held samples of this ray
        }
    }
    bool in_run = false, overflow = false;
    int key = 0, last = -1;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
    auto close_run = [&]() {
        if (nrun < f.max_runs) {
            const long long q = (long long)nrun * npix + li;
            P.rkey[q] = key;
            reinterpret_cast<float4*>(P.rcol)[q] = make_float4(C0, C1, C2, 1.0f - T);
            ++nrun;
        } else {
            overflow = true;
        }
        in_run = false;
    };
    for (long long k = k0; k <= k1; ++k) {
#pragma clang fp contract(off)
        const double t = ((double)k + 0.5) * f.dt;
        const double p0 = r.o[0] + t * r.d[0], p1 = r.o[1] + t * r.d[1], p2 = r.o[2] + t * r.d[2];
        double D[4];
        const int e = locate<kLocator>(P, last, p0, p1, p2, D);
        last = e;
        if (e < 0) {
            if (kRuns && in_run) close_run();
            continue;
        }
        if (kMode == kTetCount) {
            ++held;
            continue;
        }
        if (kMode == kTetRecord) {
            // the passes locate alike, so a ray holds as many samples as
            // counted; a mismatch (which only a logic error could cause) is
            // reported and never writes outside the ray's slots
            if ((long long)held < slots) f.slot_k[slot0 + (long long)held] = (int)k;
            else if (f.err) atomicOr(f.err, kErrRange);
            ++held;
            continue;
        }
        if (!in_run) {
            in_run = true;
            key = (int)k;
            C0 = C1 = C2 = 0.f;
            T = 1.f;
        }
        const Classified c = classify(tft, tet_value(P, e, D), tf_k, tf_o);
        float sh = 1.0f;
        if (kMode == kTetShaded) sh = a0 + a1 * ((long long)held < slots ? f.shade[slot0 + (long long)held] : 1.0f);
        const float Tn = T * trans_exp2(-c.a);
        const float w = T - Tn;
        C0 = fmaf(w, c.r * sh, C0);
        C1 = fmaf(w, c.g * sh, C1);
        C2 = fmaf(w, c.b * sh, C2);
        T = Tn;
        ++held;
    }
    if (kMode == kTetCount) {
        if (live) f.offsets[P.entry0 + li] = (long long)held;
        return;
    }
    if (kMode == kTetRecord) return;
    if (in_run) close_run();
    if (overflow && f.err) atomicOr(f.err, kErrRuns);
    if (live) P.rcount[li] = nrun;
    count_held(f.samples, held);
}

// Cycle step s of the shadow rays: the shadow ray of every held primary
// sample (its slot) through part (home + s) mod n, home the part that holds
// the sample; the slot's transmittance is multiplied by the part's (products
// commute, so the visiting order does not matter to the value).
template <int kLocator>
__global__ __launch_bounds__(256) void tet_shadow_step(TetFrameParams f) {
    __shared__ TFTable tft;
    load_tf(tft, f.tf, f.dt, threadIdx.x, 256);
    __syncthreads();
    const float tf_k = 255.0f / (f.tf.vmax - f.tf.vmin);
    const float tf_o = -f.tf.vmin * tf_k;
    unsigned long long evaluated = 0;
    // the largest e with offsets[e] <= slot (over [lo, hi])
    auto entry_in = [&](long long slot, long long lo, long long hi) {
        while (lo < hi) {
            const long long mid = (lo + hi + 1) >> 1;
            if (f.offsets[mid] <= slot) lo = mid; else hi = mid - 1;
        }
        return lo;
    };
    for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < f.total; q += (long long)gridDim.x * 256) {
        // the slot's entry and home part; the active lanes of a wavefront
        // hold consecutive slots from its first active lane's, so two
        // wavefront-uniform searches bound every lane's entry
        const unsigned q_lo = __builtin_amdgcn_readfirstlane((unsigned)q);
        const unsigned q_hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)q >> 32));
        const long long q0 = (long long)(((unsigned long long)q_hi << 32) | q_lo);
        const long long elo = entry_in(q, entry_in(q0, 0, f.n_entries - 1), entry_in(q0 + 63, 0, f.n_entries - 1));
        int hlo = 0, hhi = f.n - 1;
        while (hlo < hhi) {
            const int mid = (hlo + hhi + 1) >> 1;
            if (f.parts[mid].entry0 <= elo) hlo = mid; else hhi = mid - 1;
        }
        const TetPartK& home = f.parts[hlo];
        const TetPartK& at = f.parts[(hlo + f.step) % f.n];
        const long long r = elo - home.entry0;
        const CamRay cr = camera_ray(f.cam, home.roi_x0 + (int)(r % home.roi_w), home.roi_y0 + (int)(r / home.roi_w));
        CamRay sr;
        {
#pragma clang fp contract(off)
            const double t = ((double)f.slot_k[q] + 0.5) * f.dt;
            for (int a = 0; a < 3; ++a) {
                sr.o[a] = cr.o[a] + t * cr.d[a];
                sr.d[a] = f.light[a];
            }
        }
        float S = 1.0f;
        long long j0, j1;
        if (at.n_tets > 0 && box_range(sr, at.lo, at.hi, f.dt, j0, j1)) {
            int last = -1;
            for (long long jj = j0; jj <= j1; ++jj) {
#pragma clang fp contract(off)
                const double t = ((double)jj + 0.5) * f.dt;
                const double p0 = sr.o[0] + t * sr.d[0], p1 = sr.o[1] + t * sr.d[1], p2 = sr.o[2] + t * sr.d[2];
                double D[4];
                last = locate<kLocator>(at, last, p0, p1, p2, D);
                if (last < 0) continue;
                S = S * trans_exp2(-classify(tft, tet_value(at, last, D), tf_k, tf_o).a);
                ++evaluated;
            }
        }
        f.shade[q] = f.step == 0 ? S : f.shade[q] * S;
    }
    count_held(f.samples, evaluated);
}

// Per pixel: the runs of every part whose ROI holds the pixel, merged by
// first sample index (each part's runs are already in ray order), each
// "over" the result so far, then over the background.
__global__ __launch_bounds__(256) void tet_resolve(TetFrameParams f) {
    __shared__ uint8_t head[kMaxTetParts * 256];
    const int tid = threadIdx.x;
    for (int q = 0; q < f.n; ++q) head[q * 256 + tid] = 0;
    const long long npx = (long long)f.width * f.height;
    const long long pix = (long long)blockIdx.x * 256 + tid;
    if (pix >= npx) return;
    const int px = (int)(pix % f.width), py = (int)(pix / f.width);
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
    for (;;) {
        int best = 0x7fffffff, bq = -1;
        long long bslot = 0;
        for (int q = 0; q < f.n; ++q) {
            const TetPartK& P = f.parts[q];
            const int lx = px - P.roi_x0, ly = py - P.roi_y0;
            if (lx < 0 || ly < 0 || lx >= P.roi_w || ly >= P.roi_h) continue;
            const long long li = (long long)ly * P.roi_w + lx;
            const int h = head[q * 256 + tid];
            if (h >= min(P.rcount[li], f.max_runs)) continue;
            const long long slot = (long long)h * P.roi_w * P.roi_h + li;
            const int k = P.rkey[slot];
            if (k < best) {
                best = k;
                bq = q;
                bslot = slot;
            }
        }
        if (bq < 0) break;
        const float4 c = reinterpret_cast<const float4*>(f.parts[bq].rcol)[bslot];
        const float w = 1.0f - A;
        C0 = fmaf(w, c.x, C0);
        C1 = fmaf(w, c.y, C1);
        C2 = fmaf(w, c.z, C2);
        A = fmaf(w, c.w, A);
        ++head[bq * 256 + tid];
    }
    const float w = 1.0f - A;
    reinterpret_cast<float4*>(f.out)[pix] =
        make_float4(fmaf(w, f.bg[0], C0), fmaf(w, f.bg[1], C1), fmaf(w, f.bg[2], C2), fmaf(w, f.bg[3], A));
}

template <int kLocator>
void launch_tet_stages(TetFrameParams p, int stages, hipStream_t stream) {
    const dim3 tiles(p.total_tiles), threads(kTetThreads);
    if (p.total_tiles <= 0) return;
    if (stages & kTetCount) hipLaunchKernelGGL((tet_march<kTetCount, kLocator>), tiles, threads, 0, stream, p);
    if (stages & kTetRecord) hipLaunchKernelGGL((tet_march<kTetRecord, kLocator>), tiles, threads, 0, stream, p);
    if ((stages & kTetShadow) && p.total > 0) {
        const unsigned grid = (unsigned)min((p.total + 255) / 256, (long long)65536);
        for (int s = 0; s < p.n; ++s) {
            p.step = s;
            hipLaunchKernelGGL(tet_shadow_step<kLocator>, dim3(grid), dim3(256), 0, stream, p);
        }
    }
    if (stages & kTetMarch) hipLaunchKernelGGL((tet_march<kTetMarch, kLocator>), tiles, threads, 0, stream, p);
    if (stages & kTetShaded) hipLaunchKernelGGL((tet_march<kTetShaded, kLocator>), tiles, threads, 0, stream, p);
}

}  // namespace

hipError_t launch_tet_values(const float* vertex_values, int32_t n_input, const int32_t* centre_nodes,
                             const int32_t* tets, int32_t n_tets, float* vals, hipStream_t stream) {
    if (n_tets <= 0) return hipSuccess;
    hipLaunchKernelGGL(tet_values, dim3((n_tets + 255) / 256), dim3(256), 0, stream, vertex_values, n_input,
                       centre_nodes, reinterpret_cast<const int4*>(tets), n_tets, reinterpret_cast<float4*>(vals));
    return hipGetLastError();
}

hipError_t launch_tet_frame(TetFrameParams p, int stages, hipStream_t stream) {
    if (p.locator == kTetBvh)
        launch_tet_stages<kTetBvh>(p, stages, stream);
    else
        launch_tet_stages<kTetGrid>(p, stages, stream);
    const long long npx = (long long)p.width * p.height;
    if (stages & kTetResolve)
        hipLaunchKernelGGL(tet_resolve, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, stream, p);
    return hipGetLastError();
}

}  // namespace dpvr
