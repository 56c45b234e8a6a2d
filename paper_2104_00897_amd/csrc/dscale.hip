// FP64 helper kernels: C := beta C for the calls without a product (alpha = 0
// or k = 0) and the encode pass of the operands.
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

// Encode pass (FP64): for every panel of `panel` rows and every step p the sum
// and absolute sum of the panel's column p -- the checksum row e^T A_I (or
// column B_J e) of the encoded operands of §2.1 and the magnitude sum of the
// threshold.  One workgroup per (panel, 16 steps); the panel is staged in LDS
// with loads along the contiguous dimension, then 16 lanes per step sum
// interleaved rows and one lane adds the 16 partial sums in order.
__device__ __attribute__((always_inline)) inline void dencode_block(const DEncOperand& E, int pi, int c)
{
    __shared__ double t[256][kDEncChunk + 1];
    __shared__ double part[16][kDEncChunk][2];
    const int tid = threadIdx.x;
    const int P = E.panel;
    const int64_t r0 = (int64_t)pi * P, p0 = (int64_t)c * kDEncChunk;
    for (int q = tid; q < P * kDEncChunk; q += 256) {
        int r, p;
        if (E.kcontig) { r = q / kDEncChunk; p = q % kDEncChunk; }
        else { r = q % P; p = q / P; }
        const int64_t gr = r0 + r, gp = p0 + p;
        double v = 0.0;
        if (gr < E.rows && gp < E.K) v = E.X[E.kcontig ? gp + gr * E.ld : gr + gp * E.ld];
        t[r][p] = v;
    }
    __syncthreads();
    {
        const int p = tid % kDEncChunk, g = tid / kDEncChunk;
        double s = 0.0, sa = 0.0;
        for (int r = g; r < P; r += 16) {
            s += t[r][p];
            sa += fabs(t[r][p]);
        }
        part[g][p][0] = s;
        part[g][p][1] = sa;
    }
    __syncthreads();
    if (tid < kDEncChunk && p0 + tid < E.K) {
        double s = 0.0, sa = 0.0;
        for (int g = 0; g < 16; ++g) {
            s += part[g][tid][0];
            sa += part[g][tid][1];
        }
        double* o = E.out + ((int64_t)pi * E.K + p0 + tid) * 2;
        o[0] = s;
        o[1] = sa;
    }
}

__global__ __launch_bounds__(256) void dgemm_encode_kernel(DEncArgs args)
{
    const DEncOperand& E = args.op[blockIdx.y];
    const int pi = blockIdx.x / E.chunks, c = blockIdx.x % E.chunks;
    if (pi >= E.panels) return;
    dencode_block(E, pi, c);
}

__global__ __launch_bounds__(256) void dgemm_encode_batched_kernel(const DGemmArgs* __restrict__ desc,
                                                                   const int* __restrict__ efirst, int count)
{
    const int item = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (efirst[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const DGemmArgs& a = desc[lo];
    const int chunks = (a.k + kDEncChunk - 1) / kDEncChunk;
    const int local = item - efirst[lo];
    const int q = local / chunks, c = local % chunks;
    DEncOperand E;
    if (q < a.tiles_m) {
        E = DEncOperand{a.A, a.lda, a.m, a.k, a.ta, a.bm, a.tiles_m, chunks, const_cast<double*>(a.asp)};
        dencode_block(E, q, c);
    } else {
        E = DEncOperand{a.B, a.ldb, a.n, a.k, !a.tb, a.bn, a.tiles_n, chunks, const_cast<double*>(a.bsp)};
        dencode_block(E, q - a.tiles_m, c);
    }
}

hipError_t launch_dencode(const DEncArgs& e, int grid_x, hipStream_t s)
{
    hipLaunchKernelGGL(dgemm_encode_kernel, dim3(grid_x, 2), dim3(256), 0, s, e);
    return hipGetLastError();
}

hipError_t launch_dencode_batched(const DGemmArgs* desc, const int* efirst, int count, int total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(dgemm_encode_batched_kernel, dim3(total), dim3(256), 0, s, desc, efirst, count);
    return hipGetLastError();
}

}  // namespace ftg
