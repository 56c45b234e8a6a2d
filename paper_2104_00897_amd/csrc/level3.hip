// Packing kernels of the Level-3 routines that run on the protected GEMM
// (FT-DSYMM, FT-DTRMM; §6.2.3: the same scheme as DGEMM with modified
// packing).  A symmetric or triangular operand, stored in one triangle of a
// column-major matrix, is expanded into a dense copy that the protected GEMM
// then reads like any other operand.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ftg_kernels.hpp"

namespace ftg {

namespace {

constexpr int kPackTile = 64;

// Symmetric expansion: out(i, j) = A(i, j) when (i, j) lies in the stored
// triangle (lower: i >= j), else A(j, i).  One workgroup per 64 x 64 output
// tile; the source tile is staged in LDS so that mirrored tiles are read with
// coalesced loads and written transposed.
__global__ __launch_bounds__(256) void pack_sym_kernel(const double* __restrict__ A, int64_t lda, int64_t n,
                                                       int lower, double* __restrict__ out, int64_t ldo)
{
    __shared__ double t[kPackTile][kPackTile + 1];
    const int64_t I0 = (int64_t)blockIdx.x * kPackTile, J0 = (int64_t)blockIdx.y * kPackTile;
    const bool diag = I0 == J0;
    const bool stored = lower ? I0 > J0 : I0 < J0;
    // source tile rows/cols: (I0, J0) when stored (or diagonal), else (J0, I0)
    const int64_t R0 = (stored || diag) ? I0 : J0, C0 = (stored || diag) ? J0 : I0;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int c = ty; c < kPackTile; c += 4) {
        const int64_t r = R0 + tx, cc = C0 + c;
        t[tx][c] = (r < n && cc < n) ? A[r + cc * lda] : 0.0;
    }
    __syncthreads();
    for (int c = ty; c < kPackTile; c += 4) {
        const int64_t i = I0 + tx, j = J0 + c;
        if (i >= n || j >= n) continue;
        double v;
        if (diag) v = (lower ? i >= j : i <= j) ? t[tx][c] : t[c][tx];
        else v = stored ? t[tx][c] : t[c][tx];
        out[i + j * ldo] = v;
    }
}

// Triangular expansion: out(i, j) = A(i, j) inside the stored triangle, 0
// outside it, and 1 on the diagonal when the diagonal is unit (not read).
__global__ __launch_bounds__(256) void pack_tri_kernel(const double* __restrict__ A, int64_t lda, int64_t n,
                                                       int lower, int unit, double* __restrict__ out, int64_t ldo)
{
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, j = e / n;
        double v;
        if (i == j) v = unit ? 1.0 : A[i + j * lda];
        else if (lower ? i > j : i < j) v = A[i + j * lda];
        else v = 0.0;
        out[i + j * ldo] = v;
    }
}

}  // namespace

hipError_t launch_pack_sym(const double* A, int64_t lda, int64_t n, int lower, double* out, int64_t ldo,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)((n + kPackTile - 1) / kPackTile);
    hipLaunchKernelGGL(pack_sym_kernel, dim3(g, g), dim3(256), 0, s, A, lda, n, lower, out, ldo);
    return hipGetLastError();
}

hipError_t launch_pack_tri(const double* A, int64_t lda, int64_t n, int lower, int unit, double* out, int64_t ldo,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n * n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(pack_tri_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, n, lower, unit, out, ldo);
    return hipGetLastError();
}

}  // namespace ftg
