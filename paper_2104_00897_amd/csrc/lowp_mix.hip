// FP8 operand x bf16 checksum pieces (the checksum products of the FP8 path,
// fp8 staged as exact bf16), the encode pass, the C := beta C kernel and the
// dispatch of the low-precision launches.
#include "lowp_kernel.hpp"

namespace ftg {

template hipError_t launch_lowp_t<StFP8, StBF16, false, 0>(const LowpArgs&, int, int, hipStream_t);
template hipError_t launch_lowp_t<StBF16, StFP8, false, 0>(const LowpArgs&, int, int, hipStream_t);

// ---------------------------------------------------------------- encode
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// A binary32 value moved between lanes of a 16-lane row by a DPP control.
template <int CTRL>
__device__ inline float dpp_f32(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// e4m3 pieces of a panel sum s = sum_t 2^(7 - 4 t) q_t (+ residual), written
// to o[t stride].  Each step scales the residual by a power of two (exact),
// rounds it to e4m3 and subtracts the rounded value, taken straight from the
// rounding (exact in binary64).
__device__ inline void e4m3_pieces(double s, uint8_t* o, int64_t stride)
{
    double r = s;
#pragma unroll
    for (int t = 0; t < kFp8Pieces; ++t) {
        double v;
        const uint32_t q = f64_to_e4m3_rne(r * ldexp(1.0, 4 * t - 7), &v);
        o[(int64_t)t * stride] = (uint8_t)q;
        r -= ldexp(v, 7 - 4 * t);
    }
}

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
        if (p0 + p < E.K && E.XS) {
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
        if (p0 + p < E.K && E.XS8) {
            // e4m3 pieces s = sum_t 2^(7 - 4 t) q_t (+ residual).  A panel sum of
            // 128 e4m3 values has abs(s) <= 128 * 448; with the residual r_t below
            // 448 * 2^(7 - 4 t) each rounding leaves at most 1/16 of it (3
            // mantissa bits; below 2^-6 the subnormal step), so the next piece
            // stays in range and eight pieces leave abs(r_8) <= 2^-28 abs(s) +
            // 2^-31 (2^-21 times the half subnormal step)
            e4m3_pieces(s, E.XS8 + (int64_t)kFp8Pieces * pi * E.K + p0 + p, E.K);
        }
    }
    __syncthreads();
    if (tid == 0) {
        float mx = 0.0f;
        for (int p = 0; p < kLowpChunk; ++p) mx = fmaxf(mx, pmax[p]);
        E.XMp[(int64_t)pi * E.chunks + c] = mx;
    }
}

// The same encode for an operand whose steps are contiguous (element (r, p)
// at X[p + r ld]; packed operands always are).  Thread t takes steps
// V (t % SG) .. + V - 1 (V = 8) of rows RPT (t / SG) .. + RPT - 1 of the
// block (kLowpTile rows x kLowpChunk steps) with RPT loads issued together.
// Column sums: per thread over its rows, then a fixed xor butterfly over the
// lanes of a wave that share its steps, then the four waves in order through
// LDS.  Row sums of |x|: per thread over its steps, then a fixed butterfly
// over the SG lanes that share its rows.  bf16 sums are binary64; fp8 sums
// are binary32 up to the LDS stage, where they are still exact.
template <typename ST>
__global__ __launch_bounds__(256) void lowp_encode_k_kernel(EncArgs args)
{
    const EncOperand& E = args.op[blockIdx.y];
    const int pi = blockIdx.x / E.chunks, c = blockIdx.x % E.chunks;
    if (pi >= E.panels) return;
    constexpr int LB = ST::bytes == 2 ? 16 : 8;    // bytes per load: 8 steps of either type
    constexpr int V = LB / ST::bytes;              // steps per load
    constexpr int SG = kLowpChunk / V;             // step groups
    constexpr int RG = 256 / SG;                   // row groups
    constexpr int RPT = kLowpTile / RG;            // rows per thread
    static_assert(kLowpTile % RG == 0 && 64 % SG == 0, "encode map");
    __shared__ double cpart[4][4][kLowpChunk][2];  // [wave][16-lane row][step]
    __shared__ float pmax[kLowpChunk];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int sg = tid % SG, rg = tid / SG;
    const int64_t r0 = (int64_t)pi * kLowpTile, p0 = (int64_t)c * kLowpChunk;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc((const unsigned char*)E.X + (r0 * E.ld + p0) * ST::bytes);
    const bool full = E.vec && r0 + kLowpTile <= E.rows && p0 + kLowpChunk <= E.K;
    u32x4_t x[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int r = rg * RPT + u, pv = sg * V;
        if (full) {
            if constexpr (LB == 16) {
                x[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(((int64_t)r * E.ld + pv) * ST::bytes), 0, 0);
            } else {
                const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(((int64_t)r * E.ld + pv) * ST::bytes), 0, 0);
                x[u] = (u32x4_t){v[0], v[1], 0u, 0u};
            }
        } else {
            uint32_t wv[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const bool ok = r0 + r < E.rows && p0 + pv + e < E.K;
                const int off = ok ? (int)(((int64_t)r * E.ld + pv + e) * ST::bytes) : kOOB;
                const uint32_t b = ST::bytes == 2 ? __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0)
                                                  : __builtin_amdgcn_raw_buffer_load_b8(rs, off, 0, 0);
                wv[(e * ST::bytes) / 4] |= b << (8 * ((e * ST::bytes) % 4));
            }
            x[u] = (u32x4_t){wv[0], wv[1], wv[2], wv[3]};
        }
    }
    static_assert(SG == 8, "lane map of the reductions");
    if constexpr (ST::bytes == 1) {
        // e4m3fn values are multiples of 2^-9 of magnitude at most 448, so every
        // sum formed here (64 steps of a row, 8 rows of a step: below 2^24
        // units of 2^-9) is exact in binary32 and equals the binary64 sum
        float xf[RPT][V];
#pragma unroll
        for (int u = 0; u < RPT; ++u)
#pragma unroll
            for (int q = 0; q < V / 4; ++q) {
                const f32x2_t lo = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(x[u][q], 1.0f, false);
                const f32x2_t hi = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(x[u][q], 1.0f, true);
                xf[u][4 * q] = lo[0];
                xf[u][4 * q + 1] = lo[1];
                xf[u][4 * q + 2] = hi[0];
                xf[u][4 * q + 3] = hi[1];
            }
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            float ra = 0.0f;
#pragma unroll
            for (int e = 0; e < V; ++e) ra += fabsf(xf[u][e]);
            ra += dpp_f32<0xB1>(ra);
            ra += dpp_f32<0x4E>(ra);
            ra += dpp_f32<0x141>(ra);
            const int64_t r = r0 + rg * RPT + u;
            if (sg == 0 && r < E.rows) E.XRp[(int64_t)c * E.rows + r] = ra;
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            float cs = 0.0f, ca = 0.0f;
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                cs += xf[u][e];
                ca += fabsf(xf[u][e]);
            }
            cs += dpp_f32<0x128>(cs);
            ca += dpp_f32<0x128>(ca);
            if ((lane & 8) == 0) {
                cpart[w][lane >> 4][sg * V + e][0] = (double)cs;
                cpart[w][lane >> 4][sg * V + e][1] = (double)ca;
            }
        }
    } else {
        uint32_t hv[RPT][V / 2];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
#pragma unroll
            for (int j = 0; j < V / 2; ++j) hv[u][j] = x[u][j];
        }
        auto val = [&](int u, int e) __attribute__((always_inline)) -> double {
            return (double)bf16_bits_to_f32((hv[u][e / 2] >> (16 * (e % 2))) & 0xFFFFu);
        };
        // row sums of |x| over this block's steps: the 8 step groups of a row are
        // 8 neighbouring lanes, summed by data-parallel moves (no LDS traffic)
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            double ra = 0.0;
#pragma unroll
            for (int e = 0; e < V; ++e) ra += fabs(val(u, e));
            ra += dpp_f64<0xB1>(ra);   // quad_perm [1,0,3,2]
            ra += dpp_f64<0x4E>(ra);   // quad_perm [2,3,0,1]
            ra += dpp_f64<0x141>(ra);  // row_half_mirror: the other quad of the 8
            const int64_t r = r0 + rg * RPT + u;
            if (sg == 0 && r < E.rows) E.XRp[(int64_t)c * E.rows + r] = f64_to_f32_up(ra);
        }
        // column sums over this block's rows: the two row groups of a 16-lane row
        // by a rotation of 8 lanes, the 4 x 4 rows of the workgroup through LDS
#pragma unroll
        for (int e = 0; e < V; ++e) {
            double cs = 0.0, ca = 0.0;
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const double v = val(u, e);
                cs += v;
                ca += fabs(v);
            }
            cs += dpp_f64<0x128>(cs);  // row_ror:8
            ca += dpp_f64<0x128>(ca);
            if ((lane & 8) == 0) {
                cpart[w][lane >> 4][sg * V + e][0] = cs;
                cpart[w][lane >> 4][sg * V + e][1] = ca;
            }
        }
    }
    __syncthreads();
    if (tid < kLowpChunk) {
        const int p = tid;
        double s = 0.0, sa = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                s += cpart[v][q][p][0];
                sa += cpart[v][q][p][1];
            }
        pmax[p] = f64_to_f32_up(sa);
        if (p0 + p < E.K && E.XS) {
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
        if (p0 + p < E.K && E.XS8) {
            // e4m3 pieces s = sum_t 2^(7 - 4 t) q_t (+ residual).  A panel sum of
            // 128 e4m3 values has abs(s) <= 128 * 448; with the residual r_t below
            // 448 * 2^(7 - 4 t) each rounding leaves at most 1/16 of it (3
            // mantissa bits; below 2^-6 the subnormal step), so the next piece
            // stays in range and eight pieces leave abs(r_8) <= 2^-28 abs(s) +
            // 2^-31 (2^-21 times the half subnormal step)
            e4m3_pieces(s, E.XS8 + (int64_t)kFp8Pieces * pi * E.K + p0 + p, E.K);
        }
    }
    __syncthreads();
    if (tid < 64) {
        float mx = pmax[tid];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
        if (tid == 0) E.XMp[(int64_t)pi * E.chunks + c] = mx;
    }
}

// XR[r] = sum over chunks (binary64, rounded up); XM[panel] = max over chunks,
// per verification interval (blockIdx.z: chunks z ichunks .. + ichunks - 1).
// A workgroup takes 64 rows; its four waves sum every fourth chunk, then the
// partial sums are added through LDS (the chunks of a row are far apart in
// memory, the rows of a chunk contiguous).  It also takes 64 panels, four
// lanes each.
constexpr int kFinishRows = 64;
__global__ __launch_bounds__(256) void lowp_encode_finish_kernel(EncArgs args)
{
    const EncOperand& E = args.op[blockIdx.y];
    __shared__ double part[4][kFinishRows];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t x = (int64_t)blockIdx.x * kFinishRows + lane;
    const int c0 = blockIdx.z * E.ichunks, c1 = min(E.chunks, c0 + E.ichunks);
    double s = 0.0;
    if (x < E.rows) {
        // eight loads in flight per lane
        int c = c0 + w;
        for (; c + 28 < c1; c += 32) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = E.XRp[(int64_t)(c + 4 * u) * E.rows + x];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += (double)v[u];
        }
        for (; c < c1; c += 4) s += (double)E.XRp[(int64_t)c * E.rows + x];
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && x < E.rows)
        E.XR[(int64_t)blockIdx.z * E.rows + x] =
            f64_to_f32_up(part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]);
    // panel maxima: four lanes per panel, each over every fourth chunk, eight
    // loads in flight, then the four combined by lane exchanges
    const int64_t pnl = (int64_t)blockIdx.x * (kFinishRows) + (threadIdx.x >> 2);
    const int q = threadIdx.x & 3;
    float mx = 0.0f;
    if (pnl < E.panels) {
        const float* xm = E.XMp + pnl * E.chunks;
        int c = c0 + q;
        for (; c + 28 < c1; c += 32) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = xm[c + 4 * u];
#pragma unroll
            for (int u = 0; u < 8; ++u) mx = fmaxf(mx, v[u]);
        }
        for (; c < c1; c += 4) mx = fmaxf(mx, xm[c]);
    }
    mx = fmaxf(mx, __shfl_xor(mx, 1));
    mx = fmaxf(mx, __shfl_xor(mx, 2));
    if (pnl < E.panels && q == 0) E.XM[(int64_t)blockIdx.z * E.panels + pnl] = mx;
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
    if (e.op[0].ichunks <= 0 || e.op[0].ichunks != e.op[1].ichunks || e.op[0].chunks != e.op[1].chunks)
        return hipErrorInvalidValue;
    // operands with contiguous steps (both, once packed) take the k-major encode
    const bool kc = e.op[0].kcontig && e.op[1].kcontig;
    if (st == FTG_F8_E4M3) {
        if (kc) hipLaunchKernelGGL(lowp_encode_k_kernel<StFP8>, dim3(grid_x, 2), dim3(256), 0, s, e);
        else hipLaunchKernelGGL(lowp_encode_kernel<StFP8>, dim3(grid_x, 2), dim3(256), 0, s, e);
    } else {
        if (kc) hipLaunchKernelGGL(lowp_encode_k_kernel<StBF16>, dim3(grid_x, 2), dim3(256), 0, s, e);
        else hipLaunchKernelGGL(lowp_encode_kernel<StBF16>, dim3(grid_x, 2), dim3(256), 0, s, e);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    (void)finish_x;
    const int64_t rows = std::max<int64_t>(std::max(e.op[0].rows, e.op[1].rows),
                                           (int64_t)std::max(e.op[0].panels, e.op[1].panels));
    // one z layer per verification interval (both operands share the split)
    const int n_int = (e.op[0].chunks + e.op[0].ichunks - 1) / e.op[0].ichunks;
    hipLaunchKernelGGL(lowp_encode_finish_kernel,
                       dim3((unsigned)((rows + kFinishRows - 1) / kFinishRows), 2, (unsigned)std::max(1, n_int)),
                       dim3(256), 0, s, e);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pack
// Packs an operand stored with its rows contiguous (element (r, p) at
// X[r + p ld]) into a copy with the steps contiguous (P[p + r ldp]), the
// layout the product kernels stage without register transposes (the packing
// of BLAS-style GEMMs, here with the checksum encode reading the packed copy).
// One workgroup per tile of TR rows x TS steps (TR and TS elements = 128
// bytes each): coalesced 16-byte loads along the rows (a step's 128 bytes per
// 8 lanes), the transpose through LDS, then each row's 128 bytes written by 8
// neighbouring lanes (whole cache lines).  fp8 tile rows take 128 bytes of
// LDS with 16-byte chunk c at chunk c ^ ((row / V) % 8): the 8 lanes that load
// one step write 8 different chunks (different banks), and the row's chunks
// stay whole for the 16-byte reads (measured 36 -> 33 us for an 8192^2
// operand).  bf16 rows keep a padded 144-byte pitch (the swizzle measured
// slower there).
template <int EB>
__global__ __launch_bounds__(256) void lowp_pack_kernel(const unsigned char* __restrict__ X, int64_t ld, int rows,
                                                        int K, unsigned char* __restrict__ P, int64_t ldp, int vec)
{
    constexpr int TR = 128 / EB, TS = 128 / EB, V = 16 / EB;  // rows, steps, elements per 16 bytes
    constexpr bool SWZ = EB == 1;
    constexpr int PITCH = SWZ ? 128 : 128 + 16;  // LDS bytes per tile row
    __shared__ __attribute__((aligned(16))) unsigned char t[TR * PITCH];
    auto at = [](int r, int byte) __attribute__((always_inline)) {
        return SWZ ? r * PITCH + ((((byte >> 4) ^ (r / V)) & 7) << 4) + (byte & 15) : r * PITCH + byte;
    };
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * TR, p0 = (int64_t)blockIdx.y * TS;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(X + (r0 + p0 * ld) * EB);
    const bool full = vec && r0 + TR <= rows && p0 + TS <= K;
    // load: TS steps x (TR / V) chunks of V rows
#pragma unroll
    for (int u = 0; u < TS * (TR / V) / 256; ++u) {
        const int i = tid + 256 * u;
        const int p = i / (TR / V), rc = (i % (TR / V)) * V;
        uint32_t w[4];
        if (full) {
            const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)((rc + p * ld) * EB), 0, 0);
#pragma unroll
            for (int d = 0; d < 4; ++d) w[d] = v[d];
        } else {
#pragma unroll
            for (int d = 0; d < 4; ++d) w[d] = 0u;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const bool ok = r0 + rc + e < rows && p0 + p < K;
                const int off = ok ? (int)((rc + e + p * ld) * EB) : kOOB;
                const uint32_t x = EB == 2 ? __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0)
                                           : __builtin_amdgcn_raw_buffer_load_b8(rs, off, 0, 0);
                w[(e * EB) / 4] |= x << (8 * ((e * EB) % 4));
            }
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const uint32_t x = (w[(e * EB) / 4] >> (8 * ((e * EB) % 4))) & (EB == 2 ? 0xFFFFu : 0xFFu);
            if constexpr (EB == 2) *(uint16_t*)(t + at(rc + e, p * 2)) = (uint16_t)x;
            else t[at(rc + e, p)] = (unsigned char)x;
        }
    }
    __syncthreads();
    // store: row r, 16-byte chunk c (8 chunks = the row's 128 bytes)
#pragma unroll
    for (int u = 0; u < TR * 8 / 256; ++u) {
        const int i = tid + 256 * u;
        const int r = i / 8, c = i % 8;
        if (r0 + r < rows && p0 + c * V < ldp)
            *(u32x4_t*)(P + ((r0 + r) * ldp + p0) * EB + c * 16) = *(const u32x4_t*)(t + at(r, c * 16));
    }
}

hipError_t launch_lowp_pack(const void* X, int64_t ld, int64_t rows, int64_t K, int eb, void* P, int64_t ldp,
                            int vec, hipStream_t s)
{
    const int TS = 128 / eb, TR = 128 / eb;
    const dim3 grid((unsigned)((rows + TR - 1) / TR), (unsigned)((K + TS - 1) / TS));
    if (eb == 2)
        hipLaunchKernelGGL(lowp_pack_kernel<2>, grid, dim3(256), 0, s, (const unsigned char*)X, ld, (int)rows, (int)K,
                           (unsigned char*)P, ldp, vec);
    else
        hipLaunchKernelGGL(lowp_pack_kernel<1>, grid, dim3(256), 0, s, (const unsigned char*)X, ld, (int)rows, (int)K,
                           (unsigned char*)P, ldp, vec);
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
    // id 2 keeps the 128 x 128 checksum tile; its workgroups compute 2 x 2 of them
    if ((t == FTG_BF16 || t == FTG_F8_E4M3) && (id == 1 || id == kLowpWideTile)) {
        *bm = kLowpTile;
        *bn = kLowpTile;
        *bk = kLowpBK;
    }
}

int lowp_heuristic_tile(ftg_dtype t, int64_t m, int64_t n, int64_t)
{
    if (t != FTG_BF16 && t != FTG_F8_E4M3) return 0;
    // the wide tile once its workgroups fill the chip (256 CUs, one workgroup
    // each); the 128 x 128 tile gives smaller problems four times as many
    const int64_t wide_tiles = ((m + 255) / 256) * ((n + 255) / 256);
    return wide_tiles >= 192 ? kLowpWideTile : 1;
}

}  // namespace ftg
