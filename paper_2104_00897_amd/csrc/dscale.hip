// C := beta C for the calls without a product (alpha = 0 or k = 0).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ftg_kernels.hpp"

namespace ftg {

// C := beta C (alpha = 0 or k = 0); beta = 0 writes zeros without reading C.
__global__ void dscale_kernel(double* C, int64_t m, int64_t n, int64_t ldc, double beta)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % m, j = e / m;
        double* c = &C[i + j * ldc];
        *c = beta == 0.0 ? 0.0 : beta * *c;
    }
}

hipError_t launch_dscale(double* C, int64_t m, int64_t n, int64_t ldc, double beta, hipStream_t s)
{
    const int64_t total = m * n;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(dscale_kernel, dim3((unsigned)blocks), dim3(256), 0, s, C, m, n, ldc, beta);
    return hipGetLastError();
}

}  // namespace ftg
