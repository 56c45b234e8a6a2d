// Device fault report maintenance.
#include <hip/hip_runtime.h>

#include "ftg_batched.hpp"

namespace ftg {

// Clears counters and append indices (a kernel, not a memset, so that the
// reset can sit inside a captured graph).
__global__ void report_reset_kernel(DevReport* rep)
{
    const int t = threadIdx.x;
    if (t < 8) rep->cnt[t] = 0ull;
    if (t == 8) rep->n_records = 0u;
    if (t == 9) rep->n_inject = 0u;
}

hipError_t launch_report_reset(DevReport* rep, hipStream_t s)
{
    hipLaunchKernelGGL(report_reset_kernel, dim3(1), dim3(64), 0, s, rep);
    return hipGetLastError();
}

}  // namespace ftg
