// Device fault report maintenance and the repair kernel.
//
// A protected GEMM kernel only computes flags for a tile's final check; a
// flagged tile is stored as computed and queued.  The repair kernel, launched
// after it on the same stream, classifies each queued slot and corrects a
// located element in global memory: subtract the error magnitude (FT-BLAS
// §6.3) and re-verify the element's row and column against their expected
// checksums; failing that, recompute the element from a fresh dot product and
// re-verify; failing that too, restore it and report the slot uncorrectable.
#include <hip/hip_runtime.h>

#include "ftg_batched.hpp"

namespace ftg {

__global__ void report_reset_kernel(DevReport* rep)
{
    const int t = threadIdx.x;
    if (t < 8) rep->cnt[t] = 0ull;
    if (t == 8) rep->n_records = 0u;
    if (t == 9) rep->n_inject = 0u;
    if (t == 10) rep->rq_lost = 0u;
}

hipError_t launch_report_reset(DevReport* rep, hipStream_t s)
{
    hipLaunchKernelGGL(report_reset_kernel, dim3(1), dim3(64), 0, s, rep);
    return hipGetLastError();
}

// operand element of op(A)(i, p) / op(B)(p, j) as binary64 (exact for bf16/fp8)
__device__ inline double opnd(const RepairProblem& P, bool isA, int64_t r, int64_t c)
{
    const void* base = isA ? P.A : P.B;
    const int t = isA ? P.ta : P.tb;
    const int64_t ld = isA ? P.lda : P.ldb;
    const int64_t idx = t ? (c + r * ld) : (r + c * ld);  // op = T swaps the roles
    if (P.ab_type == FTG_F64) return ((const double*)base)[idx];
    if (P.ab_type == FTG_BF16) {
        const unsigned short b = ((const unsigned short*)base)[idx];
        return (double)__uint_as_float((unsigned int)b << 16);
    }
    // FP8 e4m3fn code
    const unsigned char q = ((const unsigned char*)base)[idx];
    const int s = q >> 7, e = (q >> 3) & 0xF, f = q & 7;
    double v = (e == 0) ? ldexp((double)f / 8.0, -6) : ldexp(1.0 + (double)f / 8.0, e - 7);
    if (e == 0xF && f == 7) v = __longlong_as_double(0x7FF8000000000000ll);
    return s ? -v : v;
}

__device__ inline double c_get(const RepairProblem& P, int64_t i, int64_t j)
{
    // device-scope atomic loads: not served from a stale vector L1 line (this
    // kernel's own corrections are re-read), and unlike volatile accesses they
    // are not serialized, so a wave's loads overlap
    if (P.c_type == FTG_F64)
        return __hip_atomic_load((const double*)P.C + i + j * P.ldc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (double)__hip_atomic_load((const float*)P.C + i + j * P.ldc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void c_set(const RepairProblem& P, int64_t i, int64_t j, double v)
{
    if (P.c_type == FTG_F64) ((volatile double*)P.C)[i + j * P.ldc] = v;
    else ((volatile float*)P.C)[i + j * P.ldc] = (float)v;
    __threadfence();
}

// sum over p = p0, p0 + step, ... < k of op(A)(i, p) op(B)(p, j), accumulated
// in that order; eight steps' operands are loaded before they are used, so a
// lane's strided loads overlap instead of forming one round trip per step
__device__ inline double dot_strided(const RepairProblem& P, int64_t i, int64_t j, int64_t p0, int64_t step)
{
    double s = 0.0;
    int64_t p = p0;
    for (; p + 7 * step < P.k; p += 8 * step) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a[u] = opnd(P, true, i, p + u * step);
            b[u] = opnd(P, false, p + u * step, j);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s = fma(a[u], b[u], s);
    }
    for (; p < P.k; p += step) s = fma(opnd(P, true, i, p), opnd(P, false, p, j), s);
    return s;
}

// One workgroup per queued request: the dot product of a recomputed element is
// split over the 256 threads (thread t takes p = t, t + 256, ...) and the
// partial sums are combined in a fixed order, so a repair costs a few rounds
// of strided loads instead of one wave's long chain.  Every branch below
// depends only on the request and on values all threads read alike, so the
// barriers are reached uniformly.
__global__ __launch_bounds__(256) void repair_kernel(DevReport* rep, RepairProblem single,
                                                     const RepairProblem* table)
{
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const unsigned int n = min(rep->rq_count, rep->rq_capacity);
    auto block_sum = [&](double v) {
        v = group_sum<64>(v);
        if (lane == 0) red[wave] = v;
        __syncthreads();
        const double t = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
        return t;
    };
    for (unsigned int r = blockIdx.x; r < n; r += gridDim.x) {
        const RepairReq q = rep->rq[r];
        const RepairProblem P = table ? table[q.problem] : single;
        if (q.whole) {
            // policy 1, several errors in the final slot of a tile that was left
            // unstored: every element from a fresh dot product and C_in (the
            // kernel has counted and recorded the slot)
            const double scale =
                (double)(P.scale_a ? *P.scale_a : 1.0f) * (double)(P.scale_b ? *P.scale_b : 1.0f);
            for (int e = tid; e < q.R * q.Q; e += 256) {
                const int64_t gi = q.m0 + e % q.R, gj = q.n0 + e / q.R;
                const double s = dot_strided(P, gi, gj, 0, 1);
                double v = P.alpha * s * scale;
                if (P.beta != 0.0) v += P.beta * c_get(P, gi, gj);
                c_set(P, gi, gj, v);
            }
            continue;
        }
        int kind;
        int64_t row = -1, col = -1;
        double d = q.nr ? q.dfi : q.dfj, tau = q.nr ? q.tfi : q.tfj;
        if (q.nr == 1 && q.nc == 1) {
            const int64_t gi = q.m0 + q.fi, gj = q.n0 + q.fj;
            // C's row and column sums over the tile against the expected ones
            auto lines_ok = [&]() {
                double rs = 0.0, cs = 0.0;
                for (int j = tid; j < q.Q; j += 256) rs += c_get(P, gi, q.n0 + j);
                for (int i = tid; i < q.R; i += 256) cs += c_get(P, q.m0 + i, gj);
                rs = block_sum(rs);
                cs = block_sum(cs);
                return !flagged(rs - q.exp_row, q.tfi) && !flagged(cs - q.exp_col, q.tfj);
            };
            const double x = c_get(P, gi, gj);
            __syncthreads();  // every thread holds the stored value before thread 0 changes it
            kind = 0;
            if (P.correct_policy == 0 && isfinite(q.dfi) && isfinite(x) &&
                !absorbed(P.c_type == FTG_F32, x, q.tfi, q.Q)) {
                if (tid == 0) c_set(P, gi, gj, x - q.dfi);
                __syncthreads();
                if (lines_ok()) kind = FTG_KIND_SUBTRACT;
            }
            if (!kind) {
                const double s = block_sum(dot_strided(P, gi, gj, tid, 256));
                const double scale = (double)(P.scale_a ? *P.scale_a : 1.0f) * (double)(P.scale_b ? *P.scale_b : 1.0f);
                double v = P.alpha * s * scale;
                if (P.beta != 0.0) v += P.beta * q.cin;
                if (tid == 0) c_set(P, gi, gj, v);
                __syncthreads();
                kind = lines_ok() ? FTG_KIND_RECOMPUTE : FTG_KIND_UNCORRECTABLE;
                if (kind == FTG_KIND_UNCORRECTABLE && tid == 0) c_set(P, gi, gj, x);
            }
            if (kind != FTG_KIND_UNCORRECTABLE) { row = gi; col = gj; }
            d = q.dfi;
            tau = q.tfi;
        } else if (q.nr + q.nc == 1) {
            kind = FTG_KIND_CHECKSUM_ONLY;
            if (q.nr) row = q.m0 + q.fi; else col = q.n0 + q.fj;
        } else {
            kind = FTG_KIND_UNCORRECTABLE;
        }
        if (tid == 0) {
            atomicAdd(&rep->cnt[kDetected], 1ull);
            if (kind == FTG_KIND_SUBTRACT) atomicAdd(&rep->cnt[kCorrSub], 1ull);
            else if (kind == FTG_KIND_RECOMPUTE) atomicAdd(&rep->cnt[kCorrRecomp], 1ull);
            else if (kind == FTG_KIND_CHECKSUM_ONLY) atomicAdd(&rep->cnt[kChecksumOnly], 1ull);
            else atomicAdd(&rep->cnt[kUncorrectable], 1ull);
            push_record(rep, q.problem, q.tm, q.tn, q.interval, row, col, kind, d, tau);
        }
    }
    // the last workgroup to finish empties the queue for the next call
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&rep->rq_done, 1u) == gridDim.x - 1) {
            rep->rq_count = 0u;
            rep->rq_done = 0u;
            __threadfence();
        }
    }
}

hipError_t launch_repair(DevReport* rep, const RepairProblem& single, const RepairProblem* table,
                         hipStream_t s)
{
    hipLaunchKernelGGL(repair_kernel, dim3(kRepairBlocks), dim3(256), 0, s, rep, single, table);
    return hipGetLastError();
}

}  // namespace ftg
