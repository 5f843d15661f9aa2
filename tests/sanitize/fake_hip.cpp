// Host-memory stand-in for the HIP runtime calls and kernel launchers that
// the library's host code (api.cpp) makes, so that its argument checks,
// table building, staging and handle bookkeeping can run under
// AddressSanitizer / UndefinedBehaviorSanitizer on a machine without a GPU.
// "Device" memory is host memory here; copies are memcpy; streams, events
// and graphs are small heap objects (so leaks of them are reported); every
// kernel launcher validates nothing and returns success.
#include <hip/hip_runtime_api.h>

#include <cstdlib>
#include <cstring>
#include <vector>

#include "dpvr_kernels.h"
#include "tet_kernels.h"

namespace {
int g_device = 0;
template <typename T>
T fresh() { return reinterpret_cast<T>(std::malloc(16)); }
alignas(256) unsigned char g_scratch[dpvr::kStaticScratchBytes];
}  // namespace

extern "C" {
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake HIP error"; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipGetDeviceCount(int* count) { *count = 1; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = g_device; return hipSuccess; }
hipError_t hipSetDevice(int d) { if (d != 0) return hipErrorInvalidDevice; g_device = d; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
    *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) { std::memmove(dst, src, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
    std::memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
    *p = std::malloc(n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) { *s = fresh<hipStream_t>(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { std::free(s); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = fresh<hipEvent_t>(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = fresh<hipEvent_t>(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { std::free(e); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.0f; return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = fresh<hipGraph_t>(); return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t, hipGraphNode_t*, char*, size_t) {
    *x = fresh<hipGraphExec_t>();
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t x) { std::free(x); return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { std::free(g); return hipSuccess; }
}

namespace dpvr {
hipError_t static_scratch_address(void** out) { *out = g_scratch; return hipSuccess; }
hipError_t launch_ingest(const float*, void*, const int32_t*, StorageK, hipStream_t) { return hipSuccess; }
hipError_t launch_march(const MarchParams&, StorageK, hipStream_t) { return hipSuccess; }
// queue launches check their tables (a prefix of each job's tiles) and
// record the partials they render, for the batch checks of the driver
std::vector<const void*> g_queue_parts;
hipError_t launch_march_queue(const QueueParams& q, StorageK, int, hipStream_t) {
    if (q.n_jobs < 1 || q.tile_start[0] != 0 || q.tile_start[q.n_jobs] != q.total_tiles) std::abort();
    for (int j = 0; j < q.n_jobs; ++j) {
        const int tw = q.staged ? q.tile_w : 16;
        if (q.tile_start[j + 1] - q.tile_start[j] != queue_tiles(q.jobs[j].roi_w, q.jobs[j].roi_h, tw)) std::abort();
        g_queue_parts.push_back(q.jobs[j].out_rgba);
    }
    return hipSuccess;
}
int march_queue_workgroups_per_cu(StorageK, bool, int, int, int) { return 2; }
hipError_t launch_composite(const CompositeParams&, hipStream_t) { return hipSuccess; }
std::vector<const void*> g_composite_frames;
hipError_t launch_composite_many(const CompositeParams* frames, const int32_t* prefix, int32_t n, int32_t total,
                                 hipStream_t) {
    if (n < 1 || prefix[0] != 0 || prefix[n] != total) std::abort();
    for (int f = 0; f < n; ++f) {
        if (prefix[f + 1] < prefix[f]) std::abort();
        g_composite_frames.push_back(frames[f].out);
    }
    return hipSuccess;
}
hipError_t launch_march_backward(const MarchParams&, const BackwardParams&, StorageK, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_composite_backward(const CompositeParams&, const CompositeBackParams&, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_gather(const GatherParams&, void*, StorageK, hipStream_t) { return hipSuccess; }
hipError_t launch_rqc_plan(const RqcParams& p, long long*, long long* total, hipStream_t) {
    // every plan entry one sample, so the total is known on the host side
    for (long long e = 0; e < p.n_entries; ++e) { p.kf[e] = 0; p.offsets[e] = e; }
    *total = p.n_entries;
    return hipSuccess;
}
long long rqc_scan_blocks(long long n_entries) { return (n_entries + 1023) / 1024; }
int backward_many_waves() { return 4; }
hipError_t launch_march_checkpointed_many(const MarchParams*, const int32_t*, int32_t, int32_t, StorageK, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_march_backward_many(const BackwardJob*, const int32_t*, int32_t, int32_t, StorageK, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_rqc_frame(RqcParams, int, hipStream_t) { return hipSuccess; }
// The tetrahedral-part launchers touch every byte their kernels may touch,
// so that a layout the host code sized wrongly shows up under ASan.
hipError_t launch_tet_values(const float* vv, int32_t n_input, const int32_t* centre_nodes, const int32_t* tets,
                             int32_t n, float* vals, hipStream_t) {
    for (int32_t e = 0; e < n; ++e)
        for (int j = 0; j < 4; ++j) {
            const int32_t v = tets[4 * e + j];
            if (v < n_input) {
                vals[4 * e + j] = vv[v];
                continue;
            }
            float s = 0.0f;
            int m = 0;
            for (; m < 8 && centre_nodes[8 * (v - n_input) + m] >= 0; ++m) s += vv[centre_nodes[8 * (v - n_input) + m]];
            vals[4 * e + j] = s / (float)m;
        }
    return hipSuccess;
}
long long scan_blocks(long long n) { return (n + 1023) / 1024; }
hipError_t launch_exclusive_scan(long long* v, long long n, long long* sums, hipStream_t) {
    long long acc = 0;
    for (long long i = 0; i < n; ++i) {
        const long long x = v[i];
        v[i] = acc;
        acc += x;
    }
    v[n] = acc;
    for (long long b = 0; b <= scan_blocks(n); ++b) sums[b] = 0;
    return hipSuccess;
}
hipError_t launch_tet_frame(TetFrameParams f, int stages, hipStream_t) {
    // every ROI pixel of every part one held sample (count), then its slot
    // written (record, shadow)
    if (stages & kTetCount)
        for (long long e = 0; e < f.n_entries; ++e) f.offsets[e] = 1;
    if (stages & kTetRecord)
        for (long long q = 0; q < f.total; ++q) f.slot_k[q] = 0;
    if (stages & kTetShadow)
        for (long long q = 0; q < f.total; ++q) f.shade[q] = 1.0f;
    int32_t tiles = 0;
    for (int32_t q = 0; q < f.n; ++q) {
        const TetPartK& P = f.parts[q];
        if (f.tile_start[q] != tiles) return hipErrorInvalidValue;
        tiles += tet_tiles(P.roi_w, P.roi_h);
        const long long np = (long long)P.roi_w * P.roi_h;
        for (long long i = 0; i < np; ++i) P.rcount[i] = 0;
        for (long long i = 0; i < np * f.max_runs; ++i) P.rkey[i] = 0;
        for (long long i = 0; i < np * f.max_runs * 4; ++i) P.rcol[i] = 0.0f;
        if (P.n_tets > 0) {
            volatile double x = P.planes[16LL * P.n_tets - 1] + P.vals[4LL * P.n_tets - 1] + P.owned[P.n_tets - 1] +
                                P.nbr[4LL * P.n_tets - 1];
            const long long cells = (long long)P.gdim[0] * P.gdim[1] * P.gdim[2];
            const int32_t entries = P.cell_start[cells];
            x = x + P.bvh_nodes[7] + P.bvh_tets[P.n_tets - 1];
            if (entries > 0) x = x + P.cell_tets[entries - 1];
            (void)x;
        }
    }
    if (f.tile_start[f.n] != tiles || f.total_tiles != tiles) return hipErrorInvalidValue;
    if (stages & 2)
        for (long long i = 0; i < 4LL * f.width * f.height; ++i) f.out[i] = f.bg[i & 3];
    return hipSuccess;
}
}  // namespace dpvr

// what the queue and composite launches since the last reset rendered
extern "C" void fake_reset_launches() {
    dpvr::g_queue_parts.clear();
    dpvr::g_composite_frames.clear();
}
extern "C" size_t fake_queue_parts(const void** out, size_t cap) {
    for (size_t i = 0; i < dpvr::g_queue_parts.size() && i < cap; ++i) out[i] = dpvr::g_queue_parts[i];
    return dpvr::g_queue_parts.size();
}
extern "C" size_t fake_composite_frames(const void** out, size_t cap) {
    for (size_t i = 0; i < dpvr::g_composite_frames.size() && i < cap; ++i) out[i] = dpvr::g_composite_frames[i];
    return dpvr::g_composite_frames.size();
}
