// Launch interfaces of the protected GEMM kernels (host side of the kernels,
// used by the C ABI in ftgemm_runtime.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ftg_common.hpp"

namespace ftg {

struct DGemmArgs {
    const double* A;
    const double* B;
    double* C;
    int lda, ldb, ldc;     // < 2^20 (buffer offsets are 32-bit)
    int m, n, k;           // < 2^31
    int kc;                // verification interval (>= k: one interval)
    int tiles_m, tiles_n;
    int ta, tb;
    int correct_policy, uncorrectable_policy;
    int problem;
    double alpha, beta;
    InjectParams inj;
    DevReport* rep;
    // checksum row/column of the encoded operands from the encode pass:
    // asp[(tile_m K + p) 2 + {0, 1}] = sum_{i in I} (a_ip, |a_ip|), bsp likewise
    // for the tile's columns; NULL = encode inside the k loop
    const double* asp;
    const double* bsp;
    int bm, bn;  // tile extent (panel rows of the encode pass)
    // 1: A and B are 16-byte aligned with even lda, ldb, so the 16-byte slots of
    // the operand panels can be loaded straight into LDS
    int lds_direct;
    int pad_;
};

inline int lds_direct_ok(const void* A, int64_t lda, const void* B, int64_t ldb)
{
    return ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && lda % 2 == 0 && ldb % 2 == 0;
}

// Encode pass of one FP64 operand: rows r (i of op(A) or j of op(B)) grouped in
// panels of `panel` rows (the output-tile extent), steps p; element (r, p) at
// X[p + r ld] when kcontig, else X[r + p ld].
struct DEncOperand {
    const double* X;
    int64_t ld;
    int rows, K, kcontig, panel, panels, chunks;
    double* out;  // out[(panel K + p) 2 + {0, 1}]
};
struct DEncArgs {
    DEncOperand op[2];
};
constexpr int kDEncChunk = 64;  // steps per encode workgroup
// items: workgroup items of the larger operand (panels * chunks)
hipError_t launch_dencode(const DEncArgs& e, int items, hipStream_t s);
// Encode pass of every problem of a batched call: workgroup item w is chunk c of
// panel q of the problem with efirst[p] <= w < efirst[p + 1] (panels 0 ..
// tiles_m - 1 of A, then tiles_n panels of B), writing desc[p].asp / bsp.
hipError_t launch_dencode_batched(const DGemmArgs* desc, const int* efirst, int count, int total,
                                  hipStream_t s);

// One persistent launch over the problems of a batched call that share a tile
// configuration and transposes (device tables written by the host).
struct BatchLaunch {
    const DGemmArgs* __restrict__ desc;  // problem descriptors, in work order
    const int* __restrict__ first;       // first work item of each problem (count + 1 entries)
    int count;                           // problems
    int total;                           // work items (tiles) = first[count]
    unsigned int* queue;                 // [0] next item - grid, [1] finished workgroups; zero at launch
};

// FP64 tile configurations (k-block 16): 1 = 256x128 on 4 waves, 2 = 128x128,
// 3 = 64x64, 4 = 256x128 on 8 waves, 5 = 128x128 on 8 waves.
// Verification intervals shorter than k need tile 2, 3 or 5.
template <int BM, int BN, int WGM, int WGN, bool IVL_OK, int MINB>
hipError_t launch_tile(const DGemmArgs& a, bool abft, hipStream_t s);
// each configuration is instantiated in its own translation unit (dgemm_t*.hip,
// dgemm_b*.hip); no other unit instantiates the kernel templates
extern template hipError_t launch_tile<256, 128, 2, 2, false, 1>(const DGemmArgs&, bool, hipStream_t);
extern template hipError_t launch_tile<128, 128, 2, 2, true, 2>(const DGemmArgs&, bool, hipStream_t);
extern template hipError_t launch_tile<64, 64, 2, 2, true, 2>(const DGemmArgs&, bool, hipStream_t);
extern template hipError_t launch_tile<256, 128, 4, 2, false, 1>(const DGemmArgs&, bool, hipStream_t);
extern template hipError_t launch_tile<128, 128, 4, 2, true, 1>(const DGemmArgs&, bool, hipStream_t);
extern template hipError_t launch_tile<128, 128, 4, 2, true, 0>(const DGemmArgs&, bool, hipStream_t);

inline hipError_t launch_dgemm(const DGemmArgs& a, int tile_id, bool abft, hipStream_t s)
{
    switch (tile_id) {
    case 1: return launch_tile<256, 128, 2, 2, false, 1>(a, abft, s);
    case 2: return launch_tile<128, 128, 2, 2, true, 2>(a, abft, s);
    case 3: return launch_tile<64, 64, 2, 2, true, 2>(a, abft, s);
    case 4: return launch_tile<256, 128, 4, 2, false, 1>(a, abft, s);
    case 5: {
        // Protected calls with beta != 0 whose epilogue outweighs the k loop
        // (short k, or at most one round of workgroups) run at one workgroup
        // per CU: the epilogue then holds the tile's C_in in registers for
        // both of its passes instead of reloading it in small batches.  So do
        // protected calls with verification intervals and direct staging: the
        // direct-staged interval kernel needs the whole register file.
        const bool direct = abft && a.asp != nullptr && a.lds_direct;
        const bool one_per_cu =
            direct && ((a.kc < a.k) ||
                       (a.beta != 0.0 && (a.k <= 256 || (int64_t)a.tiles_m * a.tiles_n <= 256)));
        return one_per_cu ? launch_tile<128, 128, 4, 2, true, 0>(a, abft, s)
                          : launch_tile<128, 128, 4, 2, true, 1>(a, abft, s);
    }
    default: return hipErrorInvalidValue;
    }
}
template <int BM, int BN, int WGM, int WGN, bool IVL_OK, int MINB>
hipError_t launch_batched(const BatchLaunch& L, int ta, int tb, bool abft, bool ivl, bool pre, bool lds_direct,
                          hipStream_t s);
extern template hipError_t launch_batched<128, 128, 2, 2, true, 2>(const BatchLaunch&, int, int, bool, bool,
                                                                   bool, bool, hipStream_t);
extern template hipError_t launch_batched<64, 64, 2, 2, true, 2>(const BatchLaunch&, int, int, bool, bool,
                                                                 bool, bool, hipStream_t);

// Batched launches exist for the configurations with verification intervals.
inline hipError_t launch_dgemm_batched(const BatchLaunch& L, int tile_id, int ta, int tb, bool abft,
                                       bool ivl, bool pre, bool lds_direct, hipStream_t s)
{
    switch (tile_id) {
    case 2: return launch_batched<128, 128, 2, 2, true, 2>(L, ta, tb, abft, ivl, pre, lds_direct, s);
    case 3: return launch_batched<64, 64, 2, 2, true, 2>(L, ta, tb, abft, ivl, pre, lds_direct, s);
    default: return hipErrorInvalidValue;
    }
}
inline bool dgemm_tile_intervals(int id) { return id == 2 || id == 3 || id == 5; }
hipError_t launch_dscale(double* C, int64_t m, int64_t n, int64_t ldc, double beta, hipStream_t s);

// ---- the unfused comparator (unfused.hip)
// Verification state of one slab: flagged row/column counts and the first
// (smallest) flagged row and column.
struct UfStatus {
    int nr, nc, fi, fj;
};
// The lines of one check direction: reference sums, maintained checksums (with
// alpha applied), magnitude sums, the C_in sums and their absolute sums (NULL
// when beta = 0), `n` lines of `len` elements after `pend` steps.
struct UfLines {
    const double* ref;
    const double* maint;
    const double* mag;
    const double* cin;
    const double* cina;
    double beta;
    int64_t n, len, pend;
};
// y_j (+)= sc sum_i S(i, j) v_i and ya_j (+)= |sc| sum_i |S(i, j)| va_i over the
// columns of a column-major rows x cols S (v, va NULL: ones; ya NULL: skipped);
// gate != NULL: nothing unless gate->nr > 0
hipError_t uf_dot_cols(const double* S, int64_t ld, int64_t rows, int64_t cols, const double* v,
                       const double* va, double sc, double* y, double* ya, int accumulate,
                       const UfStatus* gate, hipStream_t s);
// the same over the rows: y_i (+)= sc sum_j S(i, j) v_j, with a partial-sum
// buffer of uf_rows_part_doubles(rows, cols) doubles
hipError_t uf_dot_rows(const double* S, int64_t ld, int64_t rows, int64_t cols, const double* v,
                       const double* va, double sc, double* y, double* ya, int accumulate, double* part,
                       hipStream_t s);
size_t uf_rows_part_doubles(int64_t rows, int64_t cols);
hipError_t uf_fill(double* x, int64_t n, double v, hipStream_t s);
hipError_t uf_status_clear(UfStatus* st, int n, hipStream_t s);
hipError_t uf_copy(const double* C, int64_t ldc, int64_t m, int64_t n, double* out, hipStream_t s);
// flags the lines of one direction (cols = 1: columns, skipped unless a row was flagged)
hipError_t uf_verify(const UfLines& L, UfStatus* st, int cols, DevReport* rep, hipStream_t s);
// queues a flagged slab for the repair kernel
hipError_t uf_handoff(const UfLines& R, const UfLines& Cl, UfStatus* st, int interval, int final,
                      const double* cin_copy, int64_t m, DevReport* rep, double* maint_r, hipStream_t s);
hipError_t uf_inject(const InjectParams& ip, double* C, int64_t ldc, int64_t m, int64_t n, int interval,
                     int64_t plo, int64_t phi, double* maint_r, DevReport* rep, hipStream_t s);

// Dense column-major copy out (ld ldo) of an m x n block of C.
hipError_t uf_copy2d(const double* C, int64_t ldc, int64_t m, int64_t n, double* out, int64_t ldo, hipStream_t s);

// ---- packing of symmetric / triangular operands (level3.hip)
hipError_t launch_pack_sym(const double* A, int64_t lda, int64_t n, int lower, double* out, int64_t ldo,
                           hipStream_t s);
hipError_t launch_pack_tri(const double* A, int64_t lda, int64_t n, int lower, int unit, double* out, int64_t ldo,
                           hipStream_t s);

// ---- FT-DTRSM diagonal-block solve (trsm.hip)
// Solves M Y = scale * R in place for `count` right-hand sides: M is the
// nb x nb triangular block with element (r, c) at M[r + c ldm] (trans = 0) or
// M[c + r ldm] (trans = 1), lower or upper, unit diagonal optional; element
// (i, c) of R is R[i rs + c cs].  Faults: slots are right-hand sides; records
// and injection-log entries carry `block` as tile_m and global rows row0 + i.
struct TrsmDiag {
    const double* M;
    int64_t ldm;
    int nb, trans, lower, unit;
    double* R;
    int64_t rs, cs, count;
    double scale;
    InjectParams inj;
    DevReport* rep;
    int block;
    int verify;  // 0: no checksum verification (the unprotected solve)
    int64_t row0;
    const double* wsum;  // verify: e^T M at wsum[c], e^T |M| at wsum[trsm_diag_max_nb() + c]
};
int trsm_diag_max_nb();
hipError_t launch_trsm_diag(const TrsmDiag& d, hipStream_t s);
// The column sums a verified solve of block d reads through d.wsum, into w
// (2 * trsm_diag_max_nb() doubles).
hipError_t launch_trsm_colsum(const TrsmDiag& d, double* w, hipStream_t s);

// ---- duplicated-computation (DMR) Level-1/2 routines (dmr.hip)
// Injection plan of one call: up to kDmrMaxFaults verification units, each
// with the bit to flip.  The caller fills unit, bit and sub (DTRSV: the phase,
// 0 = residual, 1 = substitution); the launcher maps every unit to the thread
// (owner) and verification step of its kernel.
constexpr int kDmrMaxFaults = 64;
struct DmrFault {
    int64_t owner, unit;
    int step, sub, bit, pad;
};
struct DmrPlan {
    int n, target;
    DmrFault f[kDmrMaxFaults];
};
// Verification units of each routine (the injector's slot count).
int64_t dmr_units_vec(int64_t n);                                // DSCAL, DNRM2: elements
int64_t dmr_units_gemv(int trans, int64_t m, int64_t n);          // see ftg_dgemv
int64_t dmr_units_trsv(int64_t n);                               // elements of x
// Workspace bytes of a call (0 when none is needed).
size_t dmr_nrm2_work_bytes(int64_t n);
size_t dmr_gemv_work_bytes(int trans, int64_t m, int64_t n);
size_t dmr_trsv_work_bytes(int64_t n);
// x: element 0 of the vector, inc its stride (positive for DSCAL/DNRM2).
hipError_t launch_dmr_scal(double* x, int64_t n, int64_t inc, double alpha, bool dmr, DmrPlan plan,
                           DevReport* rep, hipStream_t s);
hipError_t launch_dmr_nrm2(const double* x, int64_t n, int64_t inc, double* out, double* work, bool dmr,
                           DmrPlan plan, DevReport* rep, hipStream_t s);
// y := alpha op(A) x + beta y with A m x n (lda), x/y element 0 and strides.
hipError_t launch_dmr_gemv(int trans, int64_t m, int64_t n, double alpha, const double* A, int64_t lda,
                           const double* x, int64_t incx, double beta, double* y, int64_t incy, double* work,
                           bool dmr, DmrPlan plan, DevReport* rep, hipStream_t s);
// x := op(A)^-1 x; lower = op(A) is lower triangular, trans = A read transposed.
hipError_t launch_dmr_trsv(int lower, int trans, int unit, int64_t n, const double* A, int64_t lda, double* x,
                           int64_t incx, double* work, bool dmr, DmrPlan plan, DevReport* rep, hipStream_t s);

inline void dgemm_tile_shape(int id, int* bm, int* bn, int* bk)
{
    *bk = 16;
    switch (id) {
    case 1: *bm = 256; *bn = 128; break;
    case 2: *bm = 128; *bn = 128; break;
    case 3: *bm = 64; *bn = 64; break;
    case 4: *bm = 256; *bn = 128; break;
    case 5: *bm = 128; *bn = 128; break;
    default: *bm = *bn = *bk = 0;
    }
}

}  // namespace ftg
