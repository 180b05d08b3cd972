// Host-only stand-ins for the HIP runtime calls and kernel launchers that
// plan.cpp references, so the planner links without a GPU runtime for the
// sanitizer build.  Every one reports failure: the driver only takes host
// paths (host-only plans, validation), and a device path reached by mistake
// fails loudly instead of touching memory.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

#include "fft_internal.h"

static hipError_t reached(const char* what)
{
    fprintf(stderr, "host sanitizer driver reached a device path: %s\n", what);
    abort();
}

extern "C" {
hipError_t hipGetDevice(int*) { return reached("hipGetDevice"); }
hipError_t hipDeviceGetAttribute(int*, hipDeviceAttribute_t, int) { return reached("hipDeviceGetAttribute"); }
hipError_t hipMalloc(void**, size_t) { return reached("hipMalloc"); }
hipError_t hipFree(void*) { return reached("hipFree"); }
hipError_t hipMemcpy(void*, const void*, size_t, hipMemcpyKind) { return reached("hipMemcpy"); }
hipError_t hipGraphCreate(hipGraph_t*, unsigned int) { return reached("hipGraphCreate"); }
hipError_t hipGraphDestroy(hipGraph_t) { return reached("hipGraphDestroy"); }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return reached("hipGraphExecDestroy"); }
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t)
{
    return reached("hipGraphInstantiate");
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return reached("hipGraphLaunch"); }
hipError_t hipGraphAddKernelNode(hipGraphNode_t*, hipGraph_t, const hipGraphNode_t*, size_t,
                                 const hipKernelNodeParams*)
{
    return reached("hipGraphAddKernelNode");
}
}

namespace moa {
hipError_t launch_pass(bool, const PassDesc&, const PassArgs&, hipStream_t) { return reached("launch_pass"); }
hipError_t launch_batched(bool, const BatchArgs&, int, int, int, hipStream_t) { return reached("launch_batched"); }
hipError_t prepare_pass_kernel(bool, const PassDesc&) { return reached("prepare_pass_kernel"); }
hipError_t prepare_batched_kernel(bool, int) { return reached("prepare_batched_kernel"); }
const void* pass_kernel_fn(bool, const PassDesc&, bool)
{
    reached("pass_kernel_fn");
    return nullptr;
}
const void* batched_kernel_fn(bool, bool)
{
    reached("batched_kernel_fn");
    return nullptr;
}
}  // namespace moa
