// The unfused ABFT comparator: the online checksum scheme built around a GEMM
// that knows nothing of it (the "first trial" of §5.1, FT-BLAS building ABFT
// on a third-party library).  Whole-matrix checksum vectors are encoded
// before the product, updated after every rank-K_c update of C, and checked
// against reference checksums recomputed from C in memory:
//   encode    e^T op(A), op(B) e (k-vectors), C_in e and e^T C_in  (T_enc)
//   per slab  C += alpha op(A)[:, slab] op(B)[slab, :]             (our own
//             unprotected FP64 kernel)
//             C^r += alpha op(A)[:, slab] (op(B) e)[slab],
//             C^c += alpha (e^T op(A))[slab] op(B)[slab, :]         (T_update)
//             reference row sums C e, compared; only when a row mismatches,
//             reference column sums e^T C, compared, and the element at the
//             flagged row and column corrected                      (T_ref)
// Every pass is a matrix-vector product over data in HBM, so its cost is set
// by memory bandwidth: (6 + 2K/K_c) t_mv in the paper's model.
//
// The kernels below are the matrix-vector passes (both orientations of a
// column-major matrix), the two verification steps, the hand-off of a flagged
// slot to the repair kernel, and the injector of this scheme (bit flips of C
// in memory at the end of a slab, where the scheme can see C).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ftg_batched.hpp"
#include "ftg_kernels.hpp"

namespace ftg {

namespace {

constexpr int kUfColChunk = 512;  // columns of one partial row sum

// y_j (+)= sc * sum_i S(i, j) v_i and ya_j (+)= |sc| * sum_i |S(i, j)| va_i for
// the columns j of a column-major S (rows x cols); v = NULL means ones.  One
// wave per column: lanes stride the rows (coalesced), a fixed butterfly over
// the 64 lanes finishes the sum.
__global__ __launch_bounds__(256) void uf_dot_cols_kernel(const double* __restrict__ S, int64_t ld,
                                                          int64_t rows, int64_t cols,
                                                          const double* __restrict__ v,
                                                          const double* __restrict__ va, double sc,
                                                          double* y, double* ya, int accumulate,
                                                          const UfStatus* gate)
{
    if (gate && gate->nr == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= cols) return;
    const double* col = S + j * ld;
    double s = 0.0, sa = 0.0;
    int64_t i = lane;
    for (; i + 192 < rows; i += 256) {
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = col[i + 64 * u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double w = v ? v[i + 64 * u] : 1.0;
            const double wa = va ? va[i + 64 * u] : 1.0;
            s = fma(x[u], w, s);
            sa = fma(fabs(x[u]), wa, sa);
        }
    }
    for (; i < rows; i += 64) {
        const double x = col[i];
        s = fma(x, v ? v[i] : 1.0, s);
        sa = fma(fabs(x), va ? va[i] : 1.0, sa);
    }
    s = group_sum<64>(s);
    sa = group_sum<64>(sa);
    if (lane == 0) {
        const double r = sc * s, ra = fabs(sc) * sa;
        y[j] = accumulate ? y[j] + r : r;
        if (ya) ya[j] = accumulate ? ya[j] + ra : ra;
    }
}

// Partial row products of a column-major S (rows x cols): thread per row (the
// loads of a wave are one coalesced run of a column), columns in chunks of
// kUfColChunk; part[(chunk * rows + i) * 2 + {0, 1}].
__global__ __launch_bounds__(256) void uf_dot_rows_kernel(const double* __restrict__ S, int64_t ld,
                                                          int64_t rows, int64_t cols,
                                                          const double* __restrict__ v,
                                                          const double* __restrict__ va,
                                                          double* __restrict__ part)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * kUfColChunk;
    if (i >= rows) return;
    const int64_t c1 = c0 + kUfColChunk < cols ? c0 + kUfColChunk : cols;
    double s = 0.0, sa = 0.0;
    int64_t c = c0;
    for (; c + 7 < c1; c += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = S[i + (c + u) * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            s = fma(x[u], v ? v[c + u] : 1.0, s);
            sa = fma(fabs(x[u]), va ? va[c + u] : 1.0, sa);
        }
    }
    for (; c < c1; ++c) {
        const double x = S[i + c * ld];
        s = fma(x, v ? v[c] : 1.0, s);
        sa = fma(fabs(x), va ? va[c] : 1.0, sa);
    }
    part[(blockIdx.y * rows + i) * 2] = s;
    part[(blockIdx.y * rows + i) * 2 + 1] = sa;
}

// y_i (+)= sc * (sum of the chunks' partials in chunk order), and the absolute
// sums alike.
__global__ __launch_bounds__(256) void uf_rows_finish_kernel(const double* __restrict__ part, int64_t rows,
                                                             int chunks, double sc, double* y, double* ya,
                                                             int accumulate)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= rows) return;
    double s = 0.0, sa = 0.0;
    for (int c = 0; c < chunks; ++c) {
        s += part[((int64_t)c * rows + i) * 2];
        sa += part[((int64_t)c * rows + i) * 2 + 1];
    }
    const double r = sc * s, ra = fabs(sc) * sa;
    y[i] = accumulate ? y[i] + r : r;
    if (ya) ya[i] = accumulate ? ya[i] + ra : ra;
}

__global__ void uf_fill_kernel(double* x, int64_t n, double v)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        x[e] = v;
}

__global__ void uf_status_clear_kernel(UfStatus* st, int n)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        st[e].nr = 0;
        st[e].nc = 0;
        st[e].fi = 0x7FFFFFFF;
        st[e].fj = 0x7FFFFFFF;
    }
}

// Copies a column-major m x n block of C into out (leading dimension ldo).
__global__ __launch_bounds__(256) void uf_copy_kernel(const double* __restrict__ C, int64_t ldc, int64_t m,
                                                      int64_t n, double* __restrict__ out, int64_t ldo)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % m, j = e / m;
        out[i + j * ldo] = C[i + j * ldc];
    }
}

// One line check of the scheme: delta = reference - (maintained + beta C_in
// sum), flagged unless |delta| <= tau (NaN-safe); tau from the line's magnitude
// with pend + len + 8 terms, as for the fused kernels.
__device__ inline void uf_line(const UfLines& L, int64_t x, double* d, double* tau)
{
    const double ex = L.maint[x] + (L.cin ? L.beta * L.cin[x] : 0.0);
    const double mag = L.mag[x] + (L.cina ? fabs(L.beta) * L.cina[x] : 0.0);
    *d = L.ref[x] - ex;
    *tau = tau_of(0, 0.0, L.pend + L.len + 8, mag);
}

__global__ __launch_bounds__(256) void uf_verify_kernel(UfLines L, UfStatus* st, int cols, DevReport* rep)
{
    if (cols && st->nr == 0) return;  // columns are checked only after a row mismatch
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double ratio = 0.0;
    if (x < L.n) {
        double d, tau;
        uf_line(L, x, &d, &tau);
        if (flagged(d, tau)) {
            if (cols) {
                atomicAdd(&st->nc, 1);
                atomicMin(&st->fj, (int)x);
            } else {
                atomicAdd(&st->nr, 1);
                atomicMin(&st->fi, (int)x);
            }
        } else if (tau > 0.0) {
            ratio = fabs(d) / tau;
        }
    }
    note_pass_ratio(rep, ratio);
}

// Hands a flagged slot to the repair kernel (one thread), with the first
// flagged row and column; a row-only mismatch in a slab before the last
// re-bases the maintained row checksum on the data, as the fused kernels do.
__global__ void uf_handoff_kernel(UfLines R, UfLines Cl, UfStatus* st, int interval, int final,
                                  const double* cin_copy, int64_t m, DevReport* rep, double* maint_r)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int nr = st->nr, nc = st->nc;
    if (nr == 0 && nc == 0) return;
    RepairReq q;
    q.problem = 0; q.tm = 0; q.tn = 0; q.interval = interval;
    q.nr = nr; q.nc = nc;
    q.fi = nr ? st->fi : 0;
    q.fj = nc ? st->fj : 0;
    q.R = (int)R.n; q.Q = (int)Cl.n;
    q.whole = 0; q.pad1 = 0; q.m0 = 0; q.n0 = 0;
    q.dfi = q.tfi = q.dfj = q.tfj = 0.0;
    q.exp_row = q.exp_col = q.cin = 0.0;
    if (nr) {
        uf_line(R, q.fi, &q.dfi, &q.tfi);
        q.exp_row = R.maint[q.fi] + (R.cin ? R.beta * R.cin[q.fi] : 0.0);
    }
    if (nc) {
        uf_line(Cl, q.fj, &q.dfj, &q.tfj);
        q.exp_col = Cl.maint[q.fj] + (Cl.cin ? Cl.beta * Cl.cin[q.fj] : 0.0);
    }
    if (nr == 1 && nc == 1 && cin_copy) q.cin = cin_copy[q.fi + q.fj * m];
    if (nr == 1 && nc == 0 && !final) maint_r[q.fi] += q.dfi;
    push_repair(rep, q);
}

// Injection of this scheme: planned flips of C (or of the maintained row
// checksum) at the end of the slab, drawn with the same slot permutation and
// draws as the fused kernels' injector (one slot per slab).
__global__ void uf_inject_kernel(InjectParams ip, double* C, int64_t ldc, int64_t m, int64_t n,
                                 int interval, int64_t plo, int64_t phi, double* maint_r, DevReport* rep)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Fault f[2];
    const int nf = slot_faults(ip, (uint64_t)interval, (int)m, (int)n, plo, phi, f);
    for (int q = 0; q < nf; ++q) {
        if (ip.target == FTG_TARGET_CHECKSUM) {
            const double o = maint_r[f[q].row];
            const double nv = flip_f64(o, f[q].bit);
            maint_r[f[q].row] = nv;
            push_inject(rep, 0, 0, 0, interval, f[q].row, -1, phi - 1, f[q].bit, FTG_TARGET_CHECKSUM, o, nv);
        } else {
            double* c = C + f[q].row + (int64_t)f[q].col * ldc;
            const double o = *c;
            const double nv = flip_f64(o, f[q].bit);
            *c = nv;
            push_inject(rep, 0, 0, 0, interval, f[q].row, f[q].col, phi - 1, f[q].bit, FTG_TARGET_ACC, o, nv);
        }
    }
}

unsigned grid_of(int64_t n, int per)
{
    const int64_t g = (n + per - 1) / per;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t uf_dot_cols(const double* S, int64_t ld, int64_t rows, int64_t cols, const double* v,
                       const double* va, double sc, double* y, double* ya, int accumulate,
                       const UfStatus* gate, hipStream_t s)
{
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(uf_dot_cols_kernel, dim3(grid_of(cols, 4)), dim3(256), 0, s, S, ld, rows, cols, v, va,
                       sc, y, ya, accumulate, gate);
    return hipGetLastError();
}

hipError_t uf_dot_rows(const double* S, int64_t ld, int64_t rows, int64_t cols, const double* v,
                       const double* va, double sc, double* y, double* ya, int accumulate, double* part,
                       hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    const int chunks = (int)((cols + kUfColChunk - 1) / kUfColChunk);
    if (chunks > 0) {
        hipLaunchKernelGGL(uf_dot_rows_kernel, dim3(grid_of(rows, 256), (unsigned)chunks), dim3(256), 0, s, S, ld,
                           rows, cols, v, va, part);
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    }
    hipLaunchKernelGGL(uf_rows_finish_kernel, dim3(grid_of(rows, 256)), dim3(256), 0, s, part, rows, chunks, sc, y,
                       ya, accumulate);
    return hipGetLastError();
}

size_t uf_rows_part_doubles(int64_t rows, int64_t cols)
{
    return (size_t)rows * (size_t)((cols + kUfColChunk - 1) / kUfColChunk) * 2;
}

hipError_t uf_fill(double* x, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(uf_fill_kernel, dim3(grid_of(n, 256) > 1024 ? 1024 : grid_of(n, 256)), dim3(256), 0, s, x,
                       n, v);
    return hipGetLastError();
}

hipError_t uf_status_clear(UfStatus* st, int n, hipStream_t s)
{
    hipLaunchKernelGGL(uf_status_clear_kernel, dim3(grid_of(n, 256)), dim3(256), 0, s, st, n);
    return hipGetLastError();
}

hipError_t uf_copy2d(const double* C, int64_t ldc, int64_t m, int64_t n, double* out, int64_t ldo, hipStream_t s)
{
    const int64_t total = m * n;
    if (total <= 0) return hipSuccess;
    unsigned g = grid_of(total, 256);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(uf_copy_kernel, dim3(g), dim3(256), 0, s, C, ldc, m, n, out, ldo);
    return hipGetLastError();
}

hipError_t uf_copy(const double* C, int64_t ldc, int64_t m, int64_t n, double* out, hipStream_t s)
{
    return uf_copy2d(C, ldc, m, n, out, m, s);
}

hipError_t uf_verify(const UfLines& L, UfStatus* st, int cols, DevReport* rep, hipStream_t s)
{
    if (L.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(uf_verify_kernel, dim3(grid_of(L.n, 256)), dim3(256), 0, s, L, st, cols, rep);
    return hipGetLastError();
}

hipError_t uf_handoff(const UfLines& R, const UfLines& Cl, UfStatus* st, int interval, int final,
                      const double* cin_copy, int64_t m, DevReport* rep, double* maint_r, hipStream_t s)
{
    hipLaunchKernelGGL(uf_handoff_kernel, dim3(1), dim3(64), 0, s, R, Cl, st, interval, final, cin_copy, m, rep,
                       maint_r);
    return hipGetLastError();
}

hipError_t uf_inject(const InjectParams& ip, double* C, int64_t ldc, int64_t m, int64_t n, int interval,
                     int64_t plo, int64_t phi, double* maint_r, DevReport* rep, hipStream_t s)
{
    hipLaunchKernelGGL(uf_inject_kernel, dim3(1), dim3(64), 0, s, ip, C, ldc, m, n, interval, plo, phi, maint_r,
                       rep);
    return hipGetLastError();
}

}  // namespace ftg
