// FP8 operand x bf16 checksum pieces (the checksum products of the FP8 path,
// fp8 staged as exact bf16), the encode pass, the C := beta C kernel and the
// dispatch of the low-precision launches.
#include "lowp_kernel.hpp"

namespace ftg {

template hipError_t launch_lowp_t<StFP8, StBF16, false, 0>(const LowpArgs&, int, int, hipStream_t);
template hipError_t launch_lowp_t<StBF16, StFP8, false, 0>(const LowpArgs&, int, int, hipStream_t);

// ---------------------------------------------------------------- encode
template <typename ST>
__global__ __launch_bounds__(256, 4) void lowp_encode_kernel(EncArgs args)
{
    const EncOperand& E = args.op[blockIdx.y];
    const int pi = blockIdx.x / E.chunks, c = blockIdx.x % E.chunks;
    if (pi >= E.panels) return;
    __shared__ float t[kLowpTile][kLowpChunk + 1];
    __shared__ float pmax[kLowpChunk];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)pi * kLowpTile, p0 = (int64_t)c * kLowpChunk;
    const typename ST::T* X = (const typename ST::T*)E.X;
    constexpr int V = 16 / ST::bytes;  // elements per 16-byte load
    if (E.vec && r0 + kLowpTile <= E.rows && p0 + kLowpChunk <= E.K) {
        // interior block: 16-byte loads along the contiguous dimension
        if (E.kcontig) {
            for (int q = tid; q < kLowpTile * (kLowpChunk / V); q += 256) {
                const int r = q / (kLowpChunk / V), pv = (q % (kLowpChunk / V)) * V;
                const u32x4_t w = *(const u32x4_t*)(X + (p0 + pv) + (r0 + r) * E.ld);
#pragma unroll
                for (int e = 0; e < V; ++e)
                    t[r][pv + e] = st_to_f32<ST>((w[(e * ST::bytes) / 4] >> (8 * ((e * ST::bytes) % 4))) &
                                                 (ST::bytes == 2 ? 0xFFFFu : 0xFFu));
            }
        } else {
            for (int q = tid; q < kLowpChunk * (kLowpTile / V); q += 256) {
                const int p = q / (kLowpTile / V), rv = (q % (kLowpTile / V)) * V;
                const u32x4_t w = *(const u32x4_t*)(X + (r0 + rv) + (p0 + p) * E.ld);
#pragma unroll
                for (int e = 0; e < V; ++e)
                    t[rv + e][p] = st_to_f32<ST>((w[(e * ST::bytes) / 4] >> (8 * ((e * ST::bytes) % 4))) &
                                                 (ST::bytes == 2 ? 0xFFFFu : 0xFFu));
            }
        }
    } else {
        for (int q = tid; q < kLowpTile * kLowpChunk; q += 256) {
            int r, p;
            if (E.kcontig) { r = q / kLowpChunk; p = q % kLowpChunk; }
            else { r = q % kLowpTile; p = q / kLowpTile; }
            const int64_t gr = r0 + r, gp = p0 + p;
            float v = 0.0f;
            if (gr < E.rows && gp < E.K) v = st_to_f32<ST>(X[E.kcontig ? gp + gr * E.ld : gr + gp * E.ld]);
            t[r][p] = v;
        }
    }
    __syncthreads();
    if (tid < kLowpTile) {
        double s = 0.0;
        for (int p = 0; p < kLowpChunk; ++p) s += fabs((double)t[tid][p]);
        if (r0 + tid < E.rows) E.XRp[(int64_t)c * E.rows + r0 + tid] = f64_to_f32_up(s);
    } else if (tid < kLowpTile + kLowpChunk) {
        const int p = tid - kLowpTile;
        double s = 0.0, sa = 0.0;
        for (int r = 0; r < kLowpTile; ++r) {
            const double v = t[r][p];
            s += v;
            sa += fabs(v);
        }
        pmax[p] = f64_to_f32_up(sa);
        if (p0 + p < E.K) {
            // three bf16 pieces: hi + mid + lo = s to within 2^-24 |s|
            const uint16_t hi = f32_to_bf16_rne((float)s);
            const double r1 = s - (double)bf16_bits_to_f32(hi);
            const uint16_t mid = f32_to_bf16_rne((float)r1);
            const double r2 = r1 - (double)bf16_bits_to_f32(mid);
            const uint16_t lo = f32_to_bf16_rne((float)r2);
            uint16_t* o = E.XS + (int64_t)3 * pi * E.K + p0 + p;
            o[0] = hi;
            o[E.K] = mid;
            o[2 * E.K] = lo;
        }
    }
    __syncthreads();
    if (tid == 0) {
        float mx = 0.0f;
        for (int p = 0; p < kLowpChunk; ++p) mx = fmaxf(mx, pmax[p]);
        E.XMp[(int64_t)pi * E.chunks + c] = mx;
    }
}

// XR[r] = sum over chunks (binary64, rounded up); XM[panel] = max over chunks.
__global__ __launch_bounds__(256) void lowp_encode_finish_kernel(EncArgs args)
{
    const EncOperand& E = args.op[blockIdx.y];
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (x < E.rows) {
        double s = 0.0;
        for (int c = 0; c < E.chunks; ++c) s += (double)E.XRp[(int64_t)c * E.rows + x];
        E.XR[x] = f64_to_f32_up(s);
    }
    if (x < E.panels) {
        float mx = 0.0f;
        for (int c = 0; c < E.chunks; ++c) mx = fmaxf(mx, E.XMp[x * E.chunks + c]);
        E.XM[x] = mx;
    }
}


hipError_t launch_lowp_gemm(const LowpArgs& a, ftg_dtype sta, ftg_dtype stb, int ta, int tb, int mode,
                            hipStream_t s)
{
    if (a.tiles_m <= 0 || a.tiles_n <= 0) return hipSuccess;
    const bool f8a = sta == FTG_F8_E4M3, f8b = stb == FTG_F8_E4M3;
    if (f8a && f8b) {
        return mode ? launch_lowp_t<StFP8, StFP8, true, 1>(a, ta, tb, s)
                    : launch_lowp_t<StFP8, StFP8, true, 0>(a, ta, tb, s);
    }
    if (!f8a && !f8b) {
        return mode ? launch_lowp_t<StBF16, StBF16, false, 1>(a, ta, tb, s)
                    : launch_lowp_t<StBF16, StBF16, false, 0>(a, ta, tb, s);
    }
    if (mode) return hipErrorInvalidValue;
    return f8a ? launch_lowp_t<StFP8, StBF16, false, 0>(a, ta, tb, s)
               : launch_lowp_t<StBF16, StFP8, false, 0>(a, ta, tb, s);
}

hipError_t launch_lowp_encode(const EncArgs& e, ftg_dtype st, int grid_x, int finish_x, hipStream_t s)
{
    if (st == FTG_F8_E4M3)
        hipLaunchKernelGGL(lowp_encode_kernel<StFP8>, dim3(grid_x, 2), dim3(256), 0, s, e);
    else
        hipLaunchKernelGGL(lowp_encode_kernel<StBF16>, dim3(grid_x, 2), dim3(256), 0, s, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(lowp_encode_finish_kernel, dim3(finish_x, 2), dim3(256), 0, s, e);
    return hipGetLastError();
}

__global__ void sscale_kernel(float* C, int64_t m, int64_t n, int64_t ldc, float beta)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    for (int64_t jj = j; jj < n; jj += gridDim.y)
        if (i < m) C[i + jj * ldc] = beta == 0.0f ? 0.0f : beta * C[i + jj * ldc];
}

hipError_t launch_sscale(float* C, int64_t m, int64_t n, int64_t ldc, float beta, hipStream_t s)
{
    const dim3 grid((unsigned)((m + 255) / 256), (unsigned)std::min<int64_t>(n, 65535));
    hipLaunchKernelGGL(sscale_kernel, grid, dim3(256), 0, s, C, m, n, ldc, beta);
    return hipGetLastError();
}

void lowp_tile_shape(ftg_dtype t, int id, int* bm, int* bn, int* bk)
{
    *bm = *bn = *bk = 0;
    if ((t == FTG_BF16 || t == FTG_F8_E4M3) && id == 1) {
        *bm = kLowpTile;
        *bn = kLowpTile;
        *bk = kLowpBK;
    }
}

int lowp_heuristic_tile(ftg_dtype t, int64_t, int64_t, int64_t)
{
    return (t == FTG_BF16 || t == FTG_F8_E4M3) ? 1 : 0;
}

}  // namespace ftg
