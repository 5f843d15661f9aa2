// Library-owned device scratch for vr_render_partials_static: the frame's
// job table, tile prefix and work-queue counters live in one file-scope
// device array instead of a caller workspace, so that entry point calls no
// allocator.  Every GPU the library runs on holds its own copy of the array
// until the process ends; host code must use the address returned by
// static_scratch_address() (queried with the device current), never the
// array's name.
#include <hip/hip_runtime.h>

#include "dpvr_kernels.h"

namespace dpvr {
namespace {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

}  // namespace

hipError_t static_scratch_address(void** out) {
    *out = nullptr;
    return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

}  // namespace dpvr
