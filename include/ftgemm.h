/*
 * ftgemm.h -- C ABI of the checksum-protected GEMM for AMD MI355X (gfx950).
 *
 * Operation (BLAS dgemm semantics, column-major):
 *     C := alpha * op(A) * op(B) + beta * C,   op(X) = X or X^T,
 * with op(A) m x k, op(B) k x n, C m x n.  The product is protected by
 * algorithm-based fault tolerance (ABFT, Zhai et al., "FT-BLAS", ICS'21):
 *   - checksum encoding A^c = [A; e^T A], B^r = [B, B e]            (§2.1)
 *   - the relations e^T C = (e^T A) B and C e = A (B e) maintained
 *     through the rank-k updates of the k loop                       (§2.1)
 *   - the checksum row/column of the encoded operands summed per output
 *     tile, by default in one encode pass over A and B ahead of the
 *     product (optionally inside the k loop from the staged panels, the
 *     fused packing of §5.2); the maintained checksums, the encoding of
 *     C_in with the beta scaling and the reference sums of the computed C
 *     fused into the product kernel                                   (§5.2)
 *   - a mismatch above the round-off threshold locates the faulty row
 *     and column; the element is corrected by subtracting the error
 *     magnitude (§5.1, §6.3), one error per verification interval
 *     without checkpoint/rollback                                    (§2.1)
 * Checksums are kept per output tile (the unit each workgroup computes),
 * so every tile can correct one error per verification interval.
 *
 * Conventions for every entry point:
 *   - Matrix pointers are DEVICE pointers owned by the caller.  C is
 *     updated in place; C must not alias A or B.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Launches are
 *     asynchronous on it.  Device buffers belong to the handle.  A call
 *     that needs more workspace than the handle holds (the FP64 encode
 *     pass, the low-precision checksum pieces and packed operand copies)
 *     grows it first: that allocates and waits for the device.  Calls that
 *     fit the workspace allocate nothing and never synchronise; size it
 *     up front with ftg_workspace_reserve (or one call of the largest
 *     shape), and use ftg_dgemm_noalloc where no allocation may happen at
 *     all.  Growth is refused (FTG_ERR_UNSUPPORTED) under stream capture;
 *     a workspace that a captured graph has used is not freed when it is
 *     outgrown but kept until ftg_destroy (the graph replays with its
 *     address).  Otherwise only ftg_report_read, ftg_batched_reserve,
 *     ftg_workspace_reserve, ftg_timing_read and ftg_destroy wait for the
 *     device.
 *   - Argument errors return FTG_ERR_INVALID_ARG and set
 *     ftg_last_error_arg() to the BLAS xerbla position of the first bad
 *     argument of dgemm: 1 transa, 2 transb, 3 m, 4 n, 5 k, 8 lda,
 *     10 ldb, 13 ldc; 20 for an invalid ftg_config field.
 *   - Quick return, touching no memory, when m = 0, n = 0, or
 *     (alpha = 0 or k = 0) and beta = 1.  alpha = 0 (or k = 0) computes
 *     C := beta*C without reading A or B.  beta = 0 never reads C, so NaN
 *     or Inf in C on input do not propagate.
 *   - One handle per stream: calls that share a handle on different
 *     streams race on its fault report.  No C++ exception crosses the ABI.
 */
#ifndef FTGEMM_H
#define FTGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FTG_OP_N = 0, FTG_OP_T = 1 } ftg_op;
typedef enum { FTG_LEFT = 0, FTG_RIGHT = 1 } ftg_side;
typedef enum { FTG_LOWER = 0, FTG_UPPER = 1 } ftg_uplo;
typedef enum { FTG_NON_UNIT = 0, FTG_UNIT = 1 } ftg_diag;

/* operand element types (A and B share one type; C is FTG_F64 or FTG_F32) */
typedef enum { FTG_F64 = 0, FTG_F32 = 1, FTG_BF16 = 2, FTG_F8_E4M3 = 3 } ftg_dtype;

typedef enum {
    FTG_OK = 0,
    FTG_ERR_INVALID_ARG = 1,
    FTG_ERR_UNSUPPORTED = 2,
    FTG_ERR_HIP = 3,
    FTG_ERR_UNCORRECTED = 4 /* only from ftg_report_read */
} ftg_status;

/* fault-record kinds */
enum {
    FTG_KIND_SUBTRACT = 1,        /* located, corrected by subtracting delta   */
    FTG_KIND_RECOMPUTE = 2,       /* located, corrected by a fresh dot product */
    FTG_KIND_CHECKSUM_ONLY = 3,   /* one direction only: the checksum was hit  */
    FTG_KIND_UNCORRECTABLE = 4,   /* more than one error in the slot; reported */
    FTG_KIND_TILE_RECOMPUTED = 5  /* uncorrectable slot, tile recomputed       */
};

/* injection targets */
enum {
    FTG_TARGET_ACC = 0,         /* a bit of one accumulator element of C           */
    FTG_TARGET_CHECKSUM = 1,    /* a bit of the maintained row checksum of one row */
    FTG_TARGET_TWO_IN_SLOT = 2  /* two accumulator faults in one slot (distinct row
                                   and column): outside the one-error model        */
};

/* Seeded in-kernel fault injector (emulates the source-level injection of
 * §6.3 with single-bit flips of values held in registers).
 *
 * A "slot" is one (tile, verification interval) pair; slots are numbered
 * s = (tile_n * tiles_m + tile_m) * n_intervals + interval.  Fault r
 * (0 <= r < F, F = min(n_faults, #slots)) goes to slot (a*r + b) mod S,
 * a keyed bijection, so the F slots are distinct.  a and b come from
 * SplitMix64 (Steele, Lea & Flood 2014) seeded with `seed`: b is output 0
 * mod S, a the first of outputs 1..64 mapped to 1 + x mod (S-1) that is
 * coprime to S.  Fault r uses outputs x0..x7 numbered 1024+8r..1024+8r+7:
 * row = x0 mod rows-in-tile, col = x1 mod cols-in-tile,
 * step = interval start + x2 mod interval length,
 * bit = bit_lo + x3 mod (bit_hi - bit_lo + 1); the flip lands right after
 * the update of the rank-128 block of k holding `step`.  (TWO_IN_SLOT draws
 * its second fault from x4..x7.)  n_faults = 0 with per_mac_rate > 0 sets
 * F = ceil(m*n*k*per_mac_rate). */
typedef struct ftg_inject {
    uint64_t seed;
    uint32_t n_faults;
    uint32_t target;     /* FTG_TARGET_* */
    double per_mac_rate; /* used when n_faults == 0 */
    int32_t bit_lo;      /* flipped bit range of the 64-bit (FP64 path) or */
    int32_t bit_hi;      /* 32-bit (FP32-accumulating paths) value         */
} ftg_inject;

typedef struct ftg_config {
    int32_t abft;        /* 1: protected kernel; 0: the same kernel with the ABFT
                            code compiled out (for overhead measurement)        */
    int32_t interval_k;  /* verification interval in steps of k; 0 = the whole
                            k loop (one verification per tile); otherwise a
                            multiple of 128 (FP64: checks of the accumulators
                            in the k loop; BF16/FP8: rank-K_c updates of C,
                            see ftg_gemm_ex)                                    */
    double lambda;       /* threshold scale of the FP32-accumulating paths
                            (0 = ftg_default_lambda()); unused for FP64        */
    int32_t correct_policy;       /* 0: subtract, re-verify, else recompute;
                                     1: always recompute the located element    */
    int32_t uncorrectable_policy; /* 0: report only; 1: recompute the tile      */
    int32_t tile;        /* tile configuration id (0 = chosen by the tuning
                            table); see ftg_tile_info                           */
    int32_t encode_in_loop; /* FP64 single calls: 0 = the checksum row/column
                            of the encoded operands come from one encode pass
                            over A and B before the product (default); 1 =
                            summed from the staged panels inside the k loop
                            (§5.2's fused encoding).  Batched calls take the
                            same choice; low precision always uses its encode
                            pass                                                */
    const ftg_inject* inject; /* NULL = no injection (host memory, read at call) */
} ftg_config;

/* One detection outcome (per slot; for data faults, the located element). */
typedef struct ftg_fault_record {
    int32_t problem;   /* index in a batched call, 0 otherwise */
    int32_t tile_m, tile_n, interval;
    int64_t row, col;  /* global element position; -1 where not applicable */
    int32_t kind;      /* FTG_KIND_* */
    int32_t reserved;
    double delta;      /* checksum difference of the located row (or of the
                          flagged line for checksum-only/uncorrectable)      */
    double tau;        /* threshold it was compared with                     */
} ftg_fault_record;

/* One applied injection (written by the kernel as it flips the bit). */
typedef struct ftg_inject_record {
    int32_t problem;
    int32_t tile_m, tile_n, interval;
    int64_t row, col;  /* global element (row checksum target: col = -1) */
    int64_t pflip;     /* last k step whose update precedes the flip */
    int32_t bit, target;
    double old_val, new_val;
} ftg_inject_record;

/* Report accumulated on the handle since the last ftg_report_reset.
 * records/inject_log point to HOST arrays of `capacity` entries owned by
 * the caller; n_records/n_inject_log may exceed capacity (entries dropped;
 * the counters still count every slot).  The report capacity only bounds
 * the records kept: flagged slots are repaired through a separate queue of
 * max(report_capacity, 16384) entries per call, and a slot that finds that
 * queue full is counted uncorrectable and in `lost`. */
typedef struct ftg_fault_report {
    uint64_t injected, detected, corrected_subtract, corrected_recompute;
    uint64_t checksum_only, uncorrectable, tiles_recomputed;
    uint32_t n_records, n_inject_log, capacity;
    uint32_t lost;  /* flagged slots the handle's repair queue could not take
                       (counted in uncorrectable; their elements stay as the
                       kernel left them) */
    double max_pass_ratio; /* largest |delta| / tau among the checks that
                              passed: how close rounding noise came to the
                              threshold (the noise margin is its inverse) */
    ftg_fault_record* records;
    ftg_inject_record* inject_log;
} ftg_fault_report;

typedef struct ftg_handle_s* ftg_handle;

/* Creates a handle on the current HIP device: allocates the device fault
 * report with room for `report_capacity` records and injection-log entries,
 * and the device buffers of the batched entry point.  The report starts
 * empty. */
ftg_status ftg_create(ftg_handle* h, size_t report_capacity);
ftg_status ftg_destroy(ftg_handle h);

/* FP64 protected GEMM (the paper's FT-DGEMM, §5.2), see the file header. */
ftg_status ftg_dgemm(ftg_handle h, ftg_op transa, ftg_op transb, int64_t m, int64_t n,
                     int64_t k, double alpha, const double* A, int64_t lda, const double* B,
                     int64_t ldb, double beta, double* C, int64_t ldc, void* stream,
                     const ftg_config* cfg);

/* ftg_dgemm for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, semantics and fault report as ftg_dgemm, but the encode
 * pass writes into a fixed scratch buffer of ftg_dgemm_noalloc_max_bytes()
 * bytes (64 MiB) that the library holds per device until the process ends,
 * instead of the handle's growable workspace: the call never allocates,
 * frees or synchronises.  It needs (ceil(m/bm) + ceil(n/bn)) * k * 16 bytes
 * for the chosen tile (bm x bn; 128 x 128 by default from 2048^2 outputs
 * on), e.g. 16 MiB at 8192^3 and 64 MiB at 16384^3; a larger shape returns
 * FTG_ERR_UNSUPPORTED before anything is launched (encode_in_loop = 1 needs
 * no scratch at all).  Every call on a device shares that device's buffer:
 * calls that overlap on one device (several streams, or several handles)
 * race; serialise them. */
ftg_status ftg_dgemm_noalloc(ftg_handle h, ftg_op transa, ftg_op transb, int64_t m, int64_t n,
                             int64_t k, double alpha, const double* A, int64_t lda,
                             const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                             void* stream, const ftg_config* cfg);
size_t ftg_dgemm_noalloc_max_bytes(void);

/* The unfused comparator: the online ABFT of §5.1 built around an
 * unprotected GEMM (the paper's "first trial", FT-MKL), for measuring what
 * fusing saves.  Same arguments and BLAS semantics as ftg_dgemm.  The
 * checksums are whole-matrix vectors (e^T op(A), op(B) e, C_in e,
 * e^T C_in), encoded before the product.  The product runs as rank-K_c
 * updates C += alpha op(A)[:, slab] op(B)[slab, :] (K_c = cfg->interval_k,
 * a multiple of 128; 0 = one slab) by the unprotected FP64 kernel.  After
 * each slab, separate memory-bound passes update C^r and C^c, recompute the
 * reference row sums of C and check them; the reference column sums are
 * taken only after a row mismatch.  One flagged row and column locate an
 * element, which the repair kernel corrects as for ftg_dgemm (subtract the
 * difference, re-verify, else recompute from a fresh dot product).  So one
 * error per slab of the whole matrix is correctable (§2.1); more are
 * reported uncorrectable (uncorrectable_policy must be 0).  Thresholds
 * follow the FP64 rule with the whole row or column as the line.  The
 * injector draws from the same slot permutation as ftg_dgemm with one slot
 * per slab: a fault flips a bit of an element of C (or of the maintained
 * row checksum) in memory at the end of its slab, logged with pflip = the
 * slab's last step.  With beta != 0 the call keeps a copy of C_in in the
 * workspace (m * n doubles) for recomputed elements. */
ftg_status ftg_dgemm_unfused(ftg_handle h, ftg_op transa, ftg_op transb, int64_t m, int64_t n,
                             int64_t k, double alpha, const double* A, int64_t lda,
                             const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                             void* stream, const ftg_config* cfg);

/* FT-DSYMM (BLAS dsymm semantics, column-major; §6.2.3: DGEMM's protection
 * with modified packing): C := alpha A B + beta C (side = FTG_LEFT, A m x m)
 * or alpha B A + beta C (FTG_RIGHT, A n x n), A symmetric with only the
 * `uplo` triangle read.  A is first expanded into a dense copy in the
 * handle's workspace; the product then runs as one ftg_dgemm on it, with its
 * checksums, verification, correction, injection (cfg->inject) and report.
 * xerbla positions: 1 side, 2 uplo, 3 m, 4 n, 7 lda, 9 ldb, 12 ldc. */
ftg_status ftg_dsymm(ftg_handle h, ftg_side side, ftg_uplo uplo, int64_t m, int64_t n, double alpha,
                     const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                     int64_t ldc, void* stream, const ftg_config* cfg);

/* FT-DTRMM (BLAS dtrmm semantics; §6.2.3): B := alpha op(A) B (FTG_LEFT,
 * A m x m) or alpha B op(A) (FTG_RIGHT, A n x n), A triangular (`uplo`
 * triangle read; FTG_UNIT: the diagonal is taken as 1 and not read).  A is
 * expanded with zeros into a dense copy and B copied into the workspace; B
 * is then overwritten by protected products over blocks of 1024 output rows
 * (left) or columns (right), each with k cut to the nonzero part of op(A),
 * so about half the multiply-adds of a dense product run.  Every block is
 * one ftg_dgemm with `cfg` (an injector config applies to each block).
 * alpha = 0 sets B to 0 without reading A.  xerbla positions: 1 side,
 * 2 uplo, 3 transa, 4 diag, 5 m, 6 n, 9 lda, 11 ldb. */
ftg_status ftg_dtrmm(ftg_handle h, ftg_side side, ftg_uplo uplo, ftg_op transa, ftg_diag diag, int64_t m,
                     int64_t n, double alpha, const double* A, int64_t lda, double* B, int64_t ldb, void* stream,
                     const ftg_config* cfg);

/* FT-DTRSM (BLAS dtrsm semantics; §3.3.3, §6.2.3): B := alpha op(A)^-1 B
 * (FTG_LEFT, A m x m) or alpha B op(A)^-1 (FTG_RIGHT, A n x n), A
 * triangular (`uplo` triangle read; FTG_UNIT: unit diagonal, not read).
 * The solve is blocked along op(A): every block off the diagonal is an
 * update B_K := -op(A)[K, D] X_D + beta B_K by the protected GEMM (outer
 * blocks of 1024, inner blocks of 256), and every 256 x 256 block on the
 * diagonal is solved by a kernel that checks each right-hand side against
 * the column checksum relation e^T M Y = e^T R with a rigorous rounding
 * threshold and solves a mismatching one again (reported as
 * FTG_KIND_RECOMPUTE with row = -1 and col = the right-hand side; tile_m =
 * the diagonal block).  The result is only as accurate as op(A) is well
 * conditioned, as for any triangular solve.  cfg->abft = 0 runs the same
 * blocking unprotected.  With cfg->inject (target FTG_TARGET_ACC only),
 * every protected step -- each update and each diagonal solve, numbered s
 * in execution order -- draws its own plan from seed SplitMix64(seed,
 * 2^33 + s); a diagonal solve's slots are its right-hand sides, and a flip
 * hits an unknown right after it is formed.  n_faults applies to each step;
 * a per_mac_rate to the whole call: step s takes floor(d_s), d_s = its
 * multiply-adds (nb (nb + 1) / 2 per right-hand side for a diagonal solve)
 * times the rate plus d_{s-1} - floor(d_{s-1}).  alpha = 0 sets B to 0.
 * xerbla positions: 1 side, 2 uplo, 3 transa, 4 diag, 5 m, 6 n, 9 lda,
 * 11 ldb; 20 for an invalid injector. */
ftg_status ftg_dtrsm(ftg_handle h, ftg_side side, ftg_uplo uplo, ftg_op transa, ftg_diag diag, int64_t m,
                     int64_t n, double alpha, const double* A, int64_t lda, double* B, int64_t ldb, void* stream,
                     const ftg_config* cfg);

/* ---- Level-1 and Level-2 routines protected by duplicated computation
 * (DMR; §4): every floating-point operation runs twice, the two results
 * are compared bit for bit after each group of 8 operations of a lane (and
 * after every step of a reduction), and a mismatching group is recomputed
 * from the operands still in registers and compared again: agreement is
 * counted in corrected_recompute (record kind FTG_KIND_RECOMPUTE), a
 * second mismatch in uncorrectable.  Loads and stores are not duplicated.
 * cfg->abft = 0 runs the same kernels with one copy (the unprotected
 * baseline).  Vectors follow BLAS: n elements at stride inc, a negative
 * stride starting from the far end; the pointer is the lowest address of
 * the vector.  All pointers are device memory; the calls queue on `stream`
 * and return at once.
 *
 * Injector (cfg->inject): F = n_faults, or ceil(per_mac_rate x operation
 * count), distinct verification units (the routine's slots, drawn by the
 * same keyed bijection as the GEMM slots; F <= 64, else
 * FTG_ERR_UNSUPPORTED).  A fault flips bit b in [bit_lo, bit_hi] (default
 * 40..63) of the unit's first result (FTG_TARGET_ACC), of its duplicate
 * (FTG_TARGET_CHECKSUM), or of the first result in the computation and
 * again in the recomputation (FTG_TARGET_TWO_IN_SLOT: the unit then ends
 * uncorrectable).  Log entries carry the element in row/col and the
 * verification step in interval and pflip.  Invalid injector fields: xerbla
 * position 20. */

/* FT-DSCAL: x := alpha x.  Nothing for n <= 0 or incx <= 0 (BLAS).  Units:
 * the n elements (one product each); row = the element. */
ftg_status ftg_dscal(ftg_handle h, int64_t n, double alpha, double* x, int64_t incx, void* stream,
                     const ftg_config* cfg);

/* FT-DNRM2: *result (device) := the Euclidean norm of x, by Blue's scaled
 * sums of squares (no overflow or harmful underflow for any finite input);
 * NaN if an element is NaN, else +Inf if one is infinite; 0 for n <= 0 or
 * incx <= 0.  Workgroup sums go to the handle's workspace.  Units: the n
 * elements (a fault hits the sum that took the element). */
ftg_status ftg_dnrm2(ftg_handle h, int64_t n, const double* x, int64_t incx, double* result, void* stream,
                     const ftg_config* cfg);

/* FT-DGEMV: y := alpha op(A) x + beta y, A m x n column-major (BLAS dgemv;
 * y is not read when beta = 0; A and x are not read when alpha = 0).
 * Without transpose one lane owns a row and adds 8 columns per step;
 * transposed one wave owns an output element and each lane adds 8 rows 64
 * apart per step.  Long reductions are cut into chunks whose sums meet in a
 * second pass (workspace).  Units: without transpose (row i, columns
 * 8g..8g+7) as u = i + m g; transposed (output j, the rows 512 t + l + 64 v,
 * v < 8, of lane l in step t) as u = j + n (64 t + l) over the (t, l) with
 * 512 t + l < m.  xerbla positions: 1 trans, 2 m, 3 n, 6 lda, 8 incx,
 * 11 incy. */
ftg_status ftg_dgemv(ftg_handle h, ftg_op trans, int64_t m, int64_t n, double alpha, const double* A,
                     int64_t lda, const double* x, int64_t incx, double beta, double* y, int64_t incy,
                     void* stream, const ftg_config* cfg);

/* FT-DTRSV: x := op(A)^-1 x, A n x n triangular (the `uplo` triangle read;
 * FTG_UNIT: unit diagonal, not read).  Blocked as in §3.2, in one launch:
 * one workgroup per block of 128 rows, in solve order, adds the duplicated
 * products of its block row with every block solved before it (waiting for
 * each to be published), then solves its diagonal block by substitution,
 * multiplying by reciprocals of the diagonal (formed as the block is
 * staged).  The handle's workspace holds the blocks' flags.  Units: the n unknowns; a fault hits the unknown's
 * right-hand side after the update (phase 0) or the unknown as it is formed
 * (phase 1), chosen by the plan.  A corrected unknown is bitwise the
 * fault-free one.  xerbla positions: 1 uplo, 2 trans, 3 diag, 4 n, 6 lda,
 * 8 incx. */
ftg_status ftg_dtrsv(ftg_handle h, ftg_uplo uplo, ftg_op trans, ftg_diag diag, int64_t n, const double* A,
                     int64_t lda, double* x, int64_t incx, void* stream, const ftg_config* cfg);

/* Mixed-precision protected GEMM: A, B of type ab_type (FTG_BF16 or
 * FTG_F8_E4M3, OCP e4m3fn), FP32 accumulation on MFMA, FP32 maintained
 * checksums, FP64 reference sums and locate/correct; C of type c_type
 * (FTG_F32).  For FTG_F8_E4M3, scale_a and scale_b are DEVICE pointers to
 * one float each (per-tensor scales: the operand value is code * scale) and
 * the product is alpha * s_A * s_B * (A_q B_q) + beta * C; they are ignored
 * (may be NULL) for FTG_BF16.  The verification threshold uses the
 * probabilistic rounding bound lambda * sqrt(n) * 2^-24 in place of
 * gamma(n).  cfg->inject->bit_lo/hi refer to the FP32 accumulator.
 * cfg->interval_k = K_c < k runs the product as rank-K_c updates of C
 * (the K_c loop of the blocked GEMM, §5.1, checked after every update as in
 * §2.1): update t computes C := alpha op(A)[:, S_t] op(B)[S_t, :] + beta_t C
 * over the steps S_t = t K_c .. min(k, (t + 1) K_c) - 1, beta_t = beta for
 * the first update and 1 after, each verified with its own thresholds and
 * repaired before the next reads C.  So one error per 128 x 128 tile and
 * interval is corrected; injection slots, records and the log carry the
 * interval.  At most 128 intervals (else FTG_ERR_UNSUPPORTED). */
ftg_status ftg_gemm_ex(ftg_handle h, ftg_op transa, ftg_op transb, int64_t m, int64_t n,
                       int64_t k, ftg_dtype ab_type, ftg_dtype c_type, const float* scale_a,
                       const float* scale_b, float alpha, const void* A, int64_t lda,
                       const void* B, int64_t ldb, float beta, void* C, int64_t ldc,
                       void* stream, const ftg_config* cfg);

/* `count` independent FP64 protected GEMMs of arbitrary shapes (the
 * paper's DGEMM of §5.2 applied to each), run as persistent launches:
 * workgroups take (problem, tile) work items from a device counter, largest
 * k first.  Problems are grouped by tile configuration and transposes, one
 * launch per group present.  A problem's tile configuration is cfg->tile
 * (2 or 3; 1 and 4 give FTG_ERR_UNSUPPORTED), else an explicit tuning-table
 * entry of 2 or 3 for its (m, n, k), else 3 (64 x 64).
 * All arrays are HOST arrays of length count (the pointer arrays hold
 * DEVICE pointers); they are read during the call and may be reused at
 * once.  The call packs them into a pinned staging area of the handle and
 * copies that to the device with one asynchronous copy on `stream`; it
 * waits on the host only for the copy made two batched calls earlier.
 * Under stream capture the copy reads a staging area kept for captures, so
 * a captured graph replays the call as it was captured (one captured
 * batched call per handle).
 * BLAS argument checks and quick returns apply per problem; the first
 * invalid problem sets ftg_last_error_arg to the dgemm argument position;
 * count < 0 gives position 2; a NULL array gives 20.
 * Injection slots are numbered per problem as in ftg_inject; problem p
 * draws with seed SplitMix64(seed, 2^32 + p) (output of the generator for
 * that counter) and F_p = faults_per_problem[p] faults when that array is
 * given, else cfg->inject->n_faults (or the per-MAC rate) per problem.
 * count is limited by ftg_batched_reserve (1024 after ftg_create).  Fault
 * records and injection-log entries carry the problem index. */
ftg_status ftg_dgemm_batched_uneven(ftg_handle h, int64_t count, const ftg_op* transa,
                                    const ftg_op* transb, const int64_t* m, const int64_t* n,
                                    const int64_t* k, const double* alpha,
                                    const double* const* A, const int64_t* lda,
                                    const double* const* B, const int64_t* ldb,
                                    const double* beta, double* const* C, const int64_t* ldc,
                                    const uint32_t* faults_per_problem, void* stream,
                                    const ftg_config* cfg);

/* Grows the handle's workspace to at least `bytes` so that later calls up to
 * that size neither allocate nor synchronise (see the file header).
 * Allocates and waits for the device; not during stream capture. */
ftg_status ftg_workspace_reserve(ftg_handle h, size_t bytes);

/* Grows the batched descriptor table to `capacity` problems (at most
 * 2^24).  Allocates and waits for the device: not during stream capture. */
ftg_status ftg_batched_reserve(ftg_handle h, int64_t capacity);

/* Copies the device report into *out: the counters (after waiting for
 * `stream`, so every call queued on it before is included), then up to
 * out->capacity records and injection-log entries into out->records /
 * out->inject_log when those are non-NULL, with asynchronous copies on
 * `stream`; with sync = 1 it waits for those copies too.  Returns FTG_ERR_UNCORRECTED when
 * sync = 1 and some slot stayed uncorrectable (kind 4). */
ftg_status ftg_report_read(ftg_handle h, void* stream, ftg_fault_report* out, int sync);

/* Clears the device report with a kernel launched on `stream`
 * (graph-capturable). */
ftg_status ftg_report_reset(ftg_handle h, void* stream);

/* The threshold scale lambda that ftg_gemm_ex uses when cfg->lambda = 0. */
double ftg_default_lambda(void);

/* BLAS info of the last FTG_ERR_INVALID_ARG returned on this handle. */
int ftg_last_error_arg(ftg_handle h);

/* Tile configurations: id >= 1.  Writes the tile shape (rows, columns,
 * k-block) of configuration `id` for operand type `ab_type`; returns
 * FTG_ERR_INVALID_ARG for an unknown id.  For FTG_BF16 and FTG_F8_E4M3 the
 * shape is that of the checksum tile (the unit of verification, correction
 * and fault-injection slots), 128 x 128 for both configurations: id 1 runs
 * one such tile per workgroup, id 2 a 2 x 2 block of them (256 x 256
 * outputs, eight waves) when K is a multiple of its k-block (32 steps for
 * bf16) and the operands allow 16-byte loads, otherwise id 1's kernel.
 * For FTG_F64, id 5 (128 x 128 on eight waves) runs two workgroups per CU,
 * except protected calls with beta != 0 and k <= 256 or at most 256 tiles,
 * which run its kernel at one workgroup per CU (the epilogue's C_in kept in
 * registers). */
ftg_status ftg_tile_info(ftg_dtype ab_type, int32_t id, int32_t* bm, int32_t* bn, int32_t* bk);

/* Tuning table: the tile configuration used when cfg->tile == 0.  Entries
 * map a shape bucket (ceil(log2) of m, n and k, each clamped to [4, 15])
 * of one operand type to a configuration id.  ftg_tune_set overrides one
 * bucket; ftg_tune_get reads it (the built-in heuristic when unset). */
ftg_status ftg_tune_set(ftg_handle h, ftg_dtype ab_type, int64_t m, int64_t n, int64_t k,
                        int32_t id);
int32_t ftg_tune_get(ftg_handle h, ftg_dtype ab_type, int64_t m, int64_t n, int64_t k);

/* Optional timing of the product kernels.  With on = 1, every following
 * call records a pair of HIP events on its stream around its main GEMM
 * launch (the protected or unprotected product kernel; for a batched call
 * all of its persistent launches), up to 256 launches between reads and
 * never under stream capture; on = 0 stops.  Either resets the record
 * (creates the events on first use). */
ftg_status ftg_timing_enable(ftg_handle h, int on);

/* Waits for the recorded launches, returns their count and total duration
 * in milliseconds, and clears the record. */
ftg_status ftg_timing_read(ftg_handle h, int32_t* launches, double* total_ms);

/* Human-readable name of a status code (static storage). */
const char* ftg_status_string(ftg_status s);

#ifdef __cplusplus
}
#endif
#endif /* FTGEMM_H */
