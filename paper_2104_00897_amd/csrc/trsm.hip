// Diagonal-block solve of FT-DTRSM (§3.3.3: the macro kernel for the blocks on
// the diagonal; the off-diagonal updates run on the protected GEMM).
//
// One launch solves M Y = s R for every right-hand side of a block of RHS,
// where M is an nb x nb triangular block (nb <= 256) of op(A) and R sits in
// B's memory (overwritten by Y).  A workgroup takes kRhs right-hand sides:
// it stages them in LDS and runs the substitution one step at a time (the
// step's unknowns divided by the diagonal, then the rank-1 update of the rows
// still to solve), with the triangle staged in LDS half by half.  The result
// is checked per right-hand side against the checksum relation
// e^T M Y = e^T (s R) -- the column checksum of §2.1 carried through the
// solve -- with a rigorous rounding threshold; a workgroup with a mismatching
// right-hand side solves again from R (still intact in memory) and re-checks.  Faults are injected into the unknowns right after
// they are formed, so they propagate through the rest of the solve as a real
// fault would.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ftg_kernels.hpp"

namespace ftg {

namespace {

constexpr int kRhs = 32;      // right-hand sides per workgroup
constexpr int kMaxNb = 256;   // block size limit
constexpr int kHalf = 128;    // the solve runs on halves whose triangle fits in LDS
constexpr int kBatch = 16;    // global loads a thread issues before it uses them
constexpr int kChunk = 64;    // columns of an off-diagonal block staged at once
constexpr int kSub = 16;      // rows of a sub-block solved in registers

// Element (r, c) of the triangular block M.
__device__ inline double m_at(const TrsmDiag& d, int r, int c)
{
    if (d.unit && r == c) return 1.0;
    return d.trans ? d.M[c + (int64_t)r * d.ldm] : d.M[r + (int64_t)c * d.ldm];
}

// Offset of (r, c), r and c local to a half of hn rows, in the packed triangle:
// column c holds rows c..hn-1 (lower) or 0..c (upper), row r at
// tri_off(lower, hn, 0, c) + r.
__device__ inline int tri_off(bool lower, int hn, int r, int c)
{
    return lower ? c * hn - (c * (c - 1)) / 2 + (r - c) : (c * (c + 1)) / 2 + r;
}

template <bool LOWER>
__global__ __launch_bounds__(256) void trsm_diag_kernel(TrsmDiag d)
{
    __shared__ double Y[kMaxNb][kRhs + 1];
    __shared__ double Mp[kHalf * (kHalf + 1) / 2];
    __shared__ double w[kMaxNb], wa[kMaxNb];
    __shared__ double esum[kRhs], easum[kRhs];
    __shared__ int redo[kRhs];
    const int tid = threadIdx.x;
    const int nb = d.nb;
    constexpr bool lower = LOWER;
    const int64_t c0 = (int64_t)blockIdx.x * kRhs;
    const int nc = (int)(d.count - c0 < kRhs ? d.count - c0 : kRhs);
    // element (i, c) of R / Y in memory
    auto at = [&](int i, int c) -> double* { return d.R + (int64_t)i * d.rs + (c0 + c) * d.cs; };
    auto in_tri = [&](int r, int c) { return lower ? r >= c : r <= c; };

    // column sums of M (the checksum row e^T M) and of |M|, formed once per
    // block by trsm_colsum_kernel
    if (d.verify) {
        for (int c = tid; c < nb; c += 256) {
            w[c] = d.wsum[c];
            wa[c] = d.wsum[kMaxNb + c];
        }
    }

    // s R into LDS, coalesced along whichever index is contiguous in memory;
    // each thread issues kBatch loads before it stores any
    auto stage = [&]() {
        const int total = nb * kRhs;
        for (int e0 = tid; e0 < total; e0 += 256 * kBatch) {
            double v[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int e = e0 + 256 * u;
                const int i = d.rs == 1 ? e % nb : e / kRhs, c = d.rs == 1 ? e / nb : e % kRhs;
                v[u] = (e < total && c < nc) ? *at(i, c) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int e = e0 + 256 * u;
                const int i = d.rs == 1 ? e % nb : e / kRhs, c = d.rs == 1 ? e / nb : e % kRhs;
                if (e < total) Y[i][c] = d.scale * v[u];
            }
        }
        __syncthreads();
    };
    stage();
    // sums over the rows of each right-hand side, 8 threads per right-hand
    // side (rows p, p + 8, ...), their partial sums added in a fixed order
    __shared__ double part[2][8][kRhs];
    auto col_sums = [&](auto term_a, auto term_b, double* out_a, double* out_b) __attribute__((always_inline)) {
        const int c = tid % kRhs, p = tid / kRhs;
        double a = 0.0, b = 0.0;
        for (int i = p; i < nb; i += 8) {
            a += term_a(i, c);
            b += term_b(i, c);
        }
        part[0][p][c] = a;
        part[1][p][c] = b;
        __syncthreads();
        if (tid < kRhs) {
            double sa = 0.0, sb = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                sa += part[0][q][tid];
                sb += part[1][q][tid];
            }
            out_a[tid] = sa;
            out_b[tid] = sb;
        }
        __syncthreads();
    };
    if (d.verify)
        col_sums([&](int i, int c) { return Y[i][c]; }, [&](int i, int c) { return fabs(Y[i][c]); }, esum, easum);
    // planned faults of this workgroup's right-hand sides (slot = right-hand side)
    int f_step = -1, f_bit = 0, f_c = -1;
    if (d.inj.on && tid < nc) {
        Fault f[2];
        if (slot_faults(d.inj, (uint64_t)(c0 + tid), nb, 1, 0, nb, f) > 0) {
            f_step = f[0].row;
            f_bit = f[0].bit;
            f_c = tid;
        }
    }

    // the substitution, forward for a lower block and backward for an upper
    // one, over halves of at most kHalf rows: a half's triangle is staged in
    // LDS and solved step by step (the step's unknowns, then the rank-1 update
    // of the half's rows still to solve); the other half then takes the
    // half's contribution, with M read once from memory
    const int nh = (nb + kHalf - 1) / kHalf;
    int hit = 0;          // the planned flip of this lane's right-hand side happened
    double hit_old = 0.0;
    auto solve = [&](bool inject) {
        for (int hs = 0; hs < nh; ++hs) {
            const int h = lower ? hs : nh - 1 - hs;
            const int base = h * kHalf, hn = min(kHalf, nb - base);
            for (int e0 = tid; e0 < hn * hn; e0 += 256 * kBatch) {
                // the contiguous index of the stored block runs fastest
                double v[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int e = e0 + 256 * u, a = e % hn, b = e / hn;
                    const int r = d.trans ? b : a, c = d.trans ? a : b;
                    v[u] = (e < hn * hn && in_tri(r, c)) ? m_at(d, base + r, base + c) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int e = e0 + 256 * u, a = e % hn, b = e / hn;
                    const int r = d.trans ? b : a, c = d.trans ? a : b;
                    if (e < hn * hn && in_tri(r, c)) Mp[tri_off(lower, hn, r, c)] = v[u];
                }
            }
            __syncthreads();
            // the half in sub-blocks of kSub rows, in solve order: lanes 0..kRhs-1
            // of wave 0 solve a sub-block's unknowns in registers (no barrier
            // between its steps), then all threads update the half's rows
            // still to solve with the sub-block's unknowns
            const int nsb = (hn + kSub - 1) / kSub;
            for (int bs = 0; bs < nsb; ++bs) {
                const int sb = lower ? bs : nsb - 1 - bs;
                const int s0 = sb * kSub;
                // FULL: a whole sub-block of kSub rows, every bound known at compile time
                auto sub_block = [&](auto full) {
                    constexpr bool FULL = decltype(full)::value;
                    const int sn = FULL ? kSub : min(kSub, hn - s0);
                    // local row (in the half) of the sub-block's unknown solved at position ps
                    auto row_of = [&](int ps) { return s0 + (lower ? ps : sn - 1 - ps); };
                    auto in_sub = [&](int ps) { return FULL || ps < sn; };
                    // column j of the packed triangle holds row r at kcol[j] + r
                    int kcol[kSub];
#pragma unroll
                    for (int ps = 0; ps < kSub; ++ps) kcol[ps] = tri_off(lower, hn, 0, row_of(ps));
                    if (tid < kRhs) {
                        // each lane owns one right-hand side: the sub-block's unknowns
                        // are solved in registers, column by column (after an unknown
                        // is formed, the rows after it in solve order take its term:
                        // independent multiply-adds), without barriers
                        double v[kSub];
#pragma unroll
                        for (int ps = 0; ps < kSub; ++ps) v[ps] = in_sub(ps) ? Y[base + row_of(ps)][tid] : 0.0;
#pragma unroll
                        for (int qs = 0; qs < kSub; ++qs) {
                            if (in_sub(qs)) {
                                const int i = row_of(qs);
                                double mcol[kSub];
#pragma unroll
                                for (int ps = qs + 1; ps < kSub; ++ps)
                                    mcol[ps] = in_sub(ps) ? Mp[kcol[qs] + row_of(ps)] : 0.0;
                                double y = v[qs];
                                if (!d.unit) y = y / Mp[kcol[qs] + i];
                                if (inject && tid == f_c && base + i == f_step) {
                                    hit_old = y;
                                    y = flip_f64(y, f_bit);
                                    hit = 1;
                                }
                                v[qs] = y;
#pragma unroll
                                for (int ps = qs + 1; ps < kSub; ++ps) v[ps] = fma(-mcol[ps], y, v[ps]);
                            }
                        }
#pragma unroll
                        for (int ps = 0; ps < kSub; ++ps)
                            if (in_sub(ps)) Y[base + row_of(ps)][tid] = v[ps];
                    }
                    __syncthreads();
                    // the half's rows still to solve take the sub-block's terms,
                    // two rows per step (independent multiply-add chains)
                    const int r0 = lower ? s0 + sn : 0, rn = lower ? hn - r0 : s0;
                    if (rn > 0) {
                        const int c = tid % kRhs, g = tid / kRhs;
                        double yj[kSub];
#pragma unroll
                        for (int ps = 0; ps < kSub; ++ps) yj[ps] = in_sub(ps) ? Y[base + row_of(ps)][c] : 0.0;
                        constexpr int kStep = 256 / kRhs;
                        for (int rr = g; rr < rn; rr += 2 * kStep) {
                            const int ra = r0 + rr, rb = r0 + rr + kStep;
                            const bool has_b = rr + kStep < rn;
                            double ma[kSub], mb[kSub];
#pragma unroll
                            for (int ps = 0; ps < kSub; ++ps) {
                                ma[ps] = in_sub(ps) ? Mp[kcol[ps] + ra] : 0.0;
                                mb[ps] = (in_sub(ps) && has_b) ? Mp[kcol[ps] + rb] : 0.0;
                            }
                            double acc = Y[base + ra][c];
                            double acc2 = has_b ? Y[base + rb][c] : 0.0;
#pragma unroll
                            for (int ps = 0; ps < kSub; ++ps) {
                                acc = fma(-ma[ps], yj[ps], acc);
                                acc2 = fma(-mb[ps], yj[ps], acc2);
                            }
                            Y[base + ra][c] = acc;
                            if (has_b) Y[base + rb][c] = acc2;
                        }
                    }
                    __syncthreads();
                };
                if (s0 + kSub <= hn) sub_block(std::true_type{});
                else sub_block(std::false_type{});
            }
            // contribution of this half to the rows of the other half still to solve
            const bool more = lower ? h + 1 < nh : h > 0;
            if (more) {
                const int ob = lower ? base + hn : 0, on = lower ? nb - ob : base;
                const int r = tid % kHalf, cg = tid / kHalf;   // two groups of 16 right-hand sides
                double acc[kRhs / 2];
#pragma unroll
                for (int q = 0; q < kRhs / 2; ++q) acc[q] = r < on ? Y[ob + r][cg * (kRhs / 2) + q] : 0.0;
                // the on x hn block of M in chunks of kChunk columns staged in LDS
                // (Mp is free once the half is solved): Mp[j * kHalf + r]
                for (int j0 = 0; j0 < hn; j0 += kChunk) {
                    const int jn = min(kChunk, hn - j0);
                    for (int e0 = tid; e0 < kHalf * jn; e0 += 256 * kBatch) {
                        double v[kBatch];
#pragma unroll
                        for (int u = 0; u < kBatch; ++u) {
                            const int e = e0 + 256 * u;
                            const int rr = d.trans ? e / jn : e % kHalf, jj = d.trans ? e % jn : e / kHalf;
                            v[u] = (e < kHalf * jn && rr < on) ? m_at(d, ob + rr, base + j0 + jj) : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < kBatch; ++u) {
                            const int e = e0 + 256 * u;
                            const int rr = d.trans ? e / jn : e % kHalf, jj = d.trans ? e % jn : e / kHalf;
                            if (e < kHalf * jn) Mp[jj * kHalf + rr] = v[u];
                        }
                    }
                    __syncthreads();
                    for (int jj = 0; jj < jn; ++jj) {
                        const double mv = Mp[jj * kHalf + r];
#pragma unroll
                        for (int q = 0; q < kRhs / 2; ++q)
                            acc[q] = fma(-mv, Y[base + j0 + jj][cg * (kRhs / 2) + q], acc[q]);
                    }
                    __syncthreads();
                }
                if (r < on) {
#pragma unroll
                    for (int q = 0; q < kRhs / 2; ++q) Y[ob + r][cg * (kRhs / 2) + q] = acc[q];
                }
                __syncthreads();
            }
        }
    };
    solve(true);
    if (hit) {
        const double nv = flip_f64(hit_old, f_bit);
        push_inject(d.rep, 0, d.block, 0, 0, d.row0 + f_step, c0 + tid, f_step, f_bit, FTG_TARGET_ACC, hit_old, nv);
    }

    // verification of each right-hand side: e^T M y against e^T (s r).  The
    // threshold grows with the computed unknowns, so a fault that drives them
    // to overflow makes it infinite: such a check counts as failed too.
    auto bad = [](double dl, double tau) { return flagged(dl, tau) || !isfinite(tau); };
    __shared__ double cref[kRhs], cmag[kRhs];
    // (every thread takes part; the difference and threshold of right-hand
    // side c come out in thread c)
    auto check = [&](int c, double* dl, double* tau) __attribute__((always_inline)) {
        col_sums([&](int i, int cc) { return w[i] * Y[i][cc]; }, [&](int i, int cc) { return wa[i] * fabs(Y[i][cc]); },
                 cref, cmag);
        if (c < kRhs) {
            *dl = cref[c] - esum[c];
            *tau = tau_of(0, 0.0, 2 * (int64_t)nb + 8, cmag[c] + easum[c]);
        }
    };
    double ratio = 0.0, dl0 = 0.0, tau0 = 0.0;
    int flag = 0;
    if (d.verify) {
        check(tid, &dl0, &tau0);
        if (tid < nc) {
            flag = bad(dl0, tau0);
            if (!flag && tau0 > 0.0) ratio = fabs(dl0) / tau0;
        }
    }
    if (tid < kRhs) redo[tid] = flag;
    note_pass_ratio(d.rep, ratio);
    // a workgroup with a flagged right-hand side solves all of them again from
    // R (still intact in memory; the others come out the same) and re-checks
    if (__syncthreads_or(flag)) {
        stage();
        solve(false);
        double dl = 0.0, tau = 0.0;
        check(tid, &dl, &tau);
        if (tid < nc && redo[tid]) {
            const int kind = bad(dl, tau) ? FTG_KIND_UNCORRECTABLE : FTG_KIND_RECOMPUTE;
            atomicAdd(&d.rep->cnt[kDetected], 1ull);
            atomicAdd(&d.rep->cnt[kind == FTG_KIND_RECOMPUTE ? kCorrRecomp : kUncorrectable], 1ull);
            push_record(d.rep, 0, d.block, 0, 0, -1, c0 + tid, kind, dl0, tau0);
        }
        __syncthreads();
    }
    // write Y over R
    if (d.rs == 1) {
        for (int e = tid; e < nb * kRhs; e += 256) {
            const int i = e % nb, c = e / nb;
            if (c < nc) *at(i, c) = Y[i][c];
        }
    } else {
        for (int e = tid; e < nb * kRhs; e += 256) {
            const int c = e % kRhs, i = e / kRhs;
            if (c < nc) *at(i, c) = Y[i][c];
        }
    }
}

// Column sums e^T M and e^T |M| of one diagonal block into w[c] and
// w[kMaxNb + c]: without transpose a wave per column (contiguous in memory),
// transposed a lane per column with the rows split over the four waves.
__global__ __launch_bounds__(256) void trsm_colsum_kernel(TrsmDiag d, double* __restrict__ w)
{
    __shared__ double ps[4][64], pa[4][64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nb = d.nb;
    auto in_tri = [&](int r, int c) { return d.lower ? r >= c : r <= c; };
    if (!d.trans) {
        const int c = blockIdx.x * 4 + wv;
        if (c >= nb) return;  // a whole wave; this branch has no barrier
        double s = 0.0, sa = 0.0;
        for (int r = lane; r < nb; r += 64) {
            const double v = in_tri(r, c) ? m_at(d, r, c) : 0.0;
            s += v;
            sa += fabs(v);
        }
        s = group_sum<64>(s);
        sa = group_sum<64>(sa);
        if (lane == 0) {
            w[c] = s;
            w[kMaxNb + c] = sa;
        }
    } else {
        const int c = blockIdx.x * 64 + lane;
        double s = 0.0, sa = 0.0;
        if (c < nb) {
            for (int r = wv; r < nb; r += 4) {
                const double v = in_tri(r, c) ? m_at(d, r, c) : 0.0;
                s += v;
                sa += fabs(v);
            }
        }
        ps[wv][lane] = s;
        pa[wv][lane] = sa;
        __syncthreads();
        if (wv == 0 && c < nb) {
            w[c] = ((ps[0][lane] + ps[1][lane]) + ps[2][lane]) + ps[3][lane];
            w[kMaxNb + c] = ((pa[0][lane] + pa[1][lane]) + pa[2][lane]) + pa[3][lane];
        }
    }
}

}  // namespace

int trsm_diag_max_nb() { return kMaxNb; }

hipError_t launch_trsm_colsum(const TrsmDiag& d, double* w, hipStream_t s)
{
    if (d.nb <= 0) return hipSuccess;
    if (d.nb > kMaxNb) return hipErrorInvalidValue;
    const unsigned g = d.trans ? (unsigned)((d.nb + 63) / 64) : (unsigned)((d.nb + 3) / 4);
    hipLaunchKernelGGL(trsm_colsum_kernel, dim3(g), dim3(256), 0, s, d, w);
    return hipGetLastError();
}

hipError_t launch_trsm_diag(const TrsmDiag& d, hipStream_t s)
{
    if (d.count <= 0 || d.nb <= 0) return hipSuccess;
    if (d.nb > kMaxNb) return hipErrorInvalidValue;
    const int64_t g = (d.count + kRhs - 1) / kRhs;
    if (d.lower) hipLaunchKernelGGL(trsm_diag_kernel<true>, dim3((unsigned)g), dim3(256), 0, s, d);
    else hipLaunchKernelGGL(trsm_diag_kernel<false>, dim3((unsigned)g), dim3(256), 0, s, d);
    return hipGetLastError();
}

}  // namespace ftg
