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
// threshold.  One workgroup of four waves per (panel, kDEncChunk steps); each
// wave issues up to kDEncBatch loads before it adds any (a few memory round
// trips per item, also for small problems):
//   steps contiguous (element (r, p) at X[p + r ld]): lane = step, wave w takes
//     a quarter of the panel's rows (each load a coalesced 512-byte run of one
//     row) and sums them in row order; the four partial sums are added in
//     wave order through LDS;
//   rows contiguous (X[r + p ld]): wave w takes a quarter of the steps; per
//     step, lane l loads rows l, l + 64, ... (coalesced runs of one column) and
//     adds them in that order, and a fixed butterfly over the 64 lanes
//     finishes the column.
// Elements outside the matrix read 0 through out-of-range buffer offsets.
constexpr int kDEncBatch = 32;

__device__ __attribute__((always_inline)) inline void dencode_item(const DEncOperand& E, int pi, int c)
{
    __shared__ double part[4][64][2];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t r0 = (int64_t)pi * E.panel, p0 = (int64_t)c * kDEncChunk;
    const int rows = (int)min((int64_t)E.panel, (int64_t)E.rows - r0);
    if (E.kcontig) {
        const int64_t p = p0 + lane;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(E.X + r0 * E.ld + p0);
        const int vo = p < E.K ? lane * 8 : kOOB;
        const int64_t rstep = E.ld * 8;
        const int rq = (E.panel + 3) / 4;  // rows per wave
        const int rb = w * rq, re = min(rows, rb + rq);
        double s = 0.0, sa = 0.0;
        for (int r = rb; r < re; r += kDEncBatch) {
            double x[kDEncBatch];
#pragma unroll
            for (int u = 0; u < kDEncBatch; ++u)
                x[u] = buf_load_f64(rs, (vo == kOOB || r + u >= re) ? kOOB : (int)(vo + (r + u) * rstep), 0);
#pragma unroll
            for (int u = 0; u < kDEncBatch; ++u) {
                s += x[u];
                sa += fabs(x[u]);
            }
        }
        part[w][lane][0] = s;
        part[w][lane][1] = sa;
        __syncthreads();
        if (w == 0 && p < E.K) {
            double t = 0.0, ta = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                t += part[v][lane][0];
                ta += part[v][lane][1];
            }
            double* o = E.out + ((int64_t)pi * E.K + p) * 2;
            o[0] = t;
            o[1] = ta;
        }
    } else {
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(E.X + r0 + p0 * E.ld);
        const int64_t pstep = E.ld * 8;
        const int steps = (int)min((int64_t)kDEncChunk, E.K - p0);
        constexpr int U = 256 / 64;          // rows per lane for panels up to 256
        constexpr int SQ = kDEncChunk / 4;   // steps per wave
        constexpr int SB = kDEncBatch / 2;   // steps per batch (panels up to 128)
        int vo[U];
#pragma unroll
        for (int u = 0; u < U; ++u) vo[u] = lane + 64 * u < rows ? (lane + 64 * u) * 8 : kOOB;
        for (int q0 = w * SQ; q0 < (w + 1) * SQ; q0 += SB) {
            double x[SB][U];
#pragma unroll
            for (int q = 0; q < SB; ++q)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (64 * u < E.panel)
                        x[q][u] = buf_load_f64(rs, (vo[u] == kOOB || q0 + q >= steps) ? kOOB
                                                                                     : (int)(vo[u] + (q0 + q) * pstep), 0);
#pragma unroll
            for (int q = 0; q < SB; ++q) {
                double s = 0.0, sa = 0.0;
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (64 * u < E.panel) {
                        s += x[q][u];
                        sa += fabs(x[q][u]);
                    }
                s = group_sum<64>(s);
                sa = group_sum<64>(sa);
                if (lane == 0 && q0 + q < steps) {
                    double* o = E.out + ((int64_t)pi * E.K + p0 + q0 + q) * 2;
                    o[0] = s;
                    o[1] = sa;
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void dgemm_encode_kernel(DEncArgs args)
{
    const DEncOperand& E = args.op[blockIdx.y];
    if ((int)blockIdx.x >= E.panels * E.chunks) return;
    dencode_item(E, blockIdx.x / E.chunks, blockIdx.x % E.chunks);
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
        dencode_item(E, q, c);
    } else {
        E = DEncOperand{a.B, a.ldb, a.n, a.k, !a.tb, a.bn, a.tiles_n, chunks, const_cast<double*>(a.bsp)};
        dencode_item(E, q - a.tiles_m, c);
    }
}

hipError_t launch_dencode(const DEncArgs& e, int items, hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(dgemm_encode_kernel, dim3(items, 2), dim3(256), 0, s, e);
    return hipGetLastError();
}

hipError_t launch_dencode_batched(const DGemmArgs* desc, const int* efirst, int count, int total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(dgemm_encode_batched_kernel, dim3(total), dim3(256), 0, s, desc, efirst, count);
    return hipGetLastError();
}

}  // namespace ftg
