// Host-only stand-ins for the HIP runtime calls and kernel launchers that the
// library's C ABI (api.cpp) makes, so that plan creation and destruction run on a
// machine without a GPU, under AddressSanitizer.  "Device" allocations are host
// allocations counted in fake_live(); graph objects are counted the same way.
// Kernels and table generators do nothing (no numerical result is checked here).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "kernels.h"

static long g_live = 0;
static long g_made = 0;

long fake_live() { return g_live; }
long fake_made() { return g_made; }

extern "C" {
hipError_t hipMalloc(void **ptr, size_t size)
{
    *ptr = std::malloc(size ? size : 1);
    if (!*ptr) return hipErrorOutOfMemory;
    ++g_live;
    ++g_made;
    return hipSuccess;
}
hipError_t hipFree(void *ptr)
{
    if (ptr) {
        std::free(ptr);
        --g_live;
    }
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind)
{
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "fake HIP error"; }
hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus *s)
{
    *s = hipStreamCaptureStatusNone;
    return hipSuccess;
}
hipError_t hipLaunchKernel(const void *, dim3, dim3, void **, size_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphCreate(hipGraph_t *g, unsigned int)
{
    *g = reinterpret_cast<hipGraph_t>(new char[1]);
    ++g_live;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g)
{
    delete[] reinterpret_cast<char *>(g);
    --g_live;
    return hipSuccess;
}
hipError_t hipGraphAddKernelNode(hipGraphNode_t *node, hipGraph_t g, const hipGraphNode_t *, size_t,
                                 const hipKernelNodeParams *)
{
    *node = reinterpret_cast<hipGraphNode_t>(g);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ex, hipGraph_t, hipGraphNode_t *, char *, size_t)
{
    *ex = reinterpret_cast<hipGraphExec_t>(new char[1]);
    ++g_live;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex)
{
    delete[] reinterpret_cast<char *>(ex);
    --g_live;
    return hipSuccess;
}
hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t, hipGraphNode_t, const hipKernelNodeParams *)
{
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
} // extern "C"

namespace mifft {
hipError_t prepare_pass(PassArgs &a, bool)
{
    a.grid = a.ntiles;
    return hipSuccess;
}
hipError_t launch_pass(const PassArgs &, bool, const void *, void *, hipStream_t) { return hipSuccess; }
hipError_t launch_line(int, const LineArgs &, bool, const void *, void *, int64_t, int, hipStream_t)
{
    return hipSuccess;
}
const void *ragged_kernel(bool f64) { return f64 ? &g_live : &g_made; }
hipError_t gen_range(double2 *, int64_t, int64_t, int64_t, int64_t, hipStream_t) { return hipSuccess; }
hipError_t gen_inner(double2 *, const StagesArg &, int64_t, hipStream_t) { return hipSuccess; }
hipError_t gen_chirp(double2 *, int64_t, int64_t, hipStream_t) { return hipSuccess; }
hipError_t gen_bwrap(double2 *, const double2 *, int64_t, int64_t, hipStream_t) { return hipSuccess; }
hipError_t convert_d2f(float2 *, const double2 *, int64_t, hipStream_t) { return hipSuccess; }
} // namespace mifft
