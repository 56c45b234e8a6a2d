/*
 * CPU oracle for the checksum-protected GEMM -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file's library.  The GPU library neither includes,
 * links nor calls anything here, and this file includes nothing of the GPU
 * library: the two share no code.  Parity of every function below is pinned
 * in tests/test_oracle.py against closed forms, integer-exact brute force and
 * the worked fault example in tests/golden/ (see the header of that test).
 *
 * Precision: IEEE binary64 throughout, built with -O2 -ffp-contract=off and no
 * fast-math, so every sum below is evaluated in exactly the order written.
 *
 * What it computes (paper: Zhai et al., "FT-BLAS", ICS'21):
 *  - ftgo_gemm      C := alpha*op(A)*op(B) + beta*C, column-major, BLAS dgemm
 *                   semantics (§3.3.2 names the routine; §2.1 the product).
 *  - ftgo_abft      the online ABFT procedure applied per output tile:
 *                   checksum encoding A^c=[A; e^T A], B^r=[B, B e] (§2.1),
 *                   maintenance of the checksum relation after every rank-1
 *                   outer-product step (§2.1, second display equation),
 *                   verification at the end of every verification interval
 *                   against a round-off threshold (§2.1, §5.1), location of
 *                   one faulty element by intersecting the mismatching row and
 *                   column (§5.1), correction by subtracting the error
 *                   magnitude at that position (§6.3), one error corrected per
 *                   interval without checkpoint/rollback (§2.1), and the C
 *                   checksums of beta*C_in fused with the scaling (§5.2).
 *                   With `split` set, C itself is the accumulator across the
 *                   intervals, as in the K_c loop of the blocked GEMM (§5.1:
 *                   each rank-K_c update C := alpha A_t B_t + beta_t C is
 *                   checked on its own, beta_t = beta for the first and 1 after).
 *  - fault plan     the seeded injection plan: which (tile, interval) slots
 *                   receive a fault and the element, step and bit of each
 *                   (§6.3 injects one error per injection interval into a
 *                   randomly chosen element of C).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* operand access: column-major storage, op = identity (0) or transpose (1)  */
/* ------------------------------------------------------------------------ */
static double opA(int ta, const double* A, int64_t lda, int64_t i, int64_t p)
{
    return ta ? A[p + i * lda] : A[i + p * lda];
}

static double opB(int tb, const double* B, int64_t ldb, int64_t p, int64_t j)
{
    return tb ? B[j + p * ldb] : B[p + j * ldb];
}

static int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }
static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

/* BLAS xerbla numbering of dgemm's arguments; 0 when all are valid. */
static int gemm_arg_check(int ta, int tb, int64_t m, int64_t n, int64_t k,
                          int64_t lda, int64_t ldb, int64_t ldc)
{
    if (ta != 0 && ta != 1) return 1;
    if (tb != 0 && tb != 1) return 2;
    if (m < 0) return 3;
    if (n < 0) return 4;
    if (k < 0) return 5;
    if (lda < max64(1, ta ? k : m)) return 8;
    if (ldb < max64(1, tb ? n : k)) return 10;
    if (ldc < max64(1, m)) return 13;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 1. Plain GEMM: the result the protected method must reproduce.           */
/* ------------------------------------------------------------------------ */
int ftgo_gemm(int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb,
              double beta, double* C, int64_t ldc)
{
    int info = gemm_arg_check(ta, tb, m, n, k, lda, ldb, ldc);
    if (info) return info;
    if (m == 0 || n == 0 || ((alpha == 0.0 || k == 0) && beta == 1.0)) return 0;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            if (alpha != 0.0)
                for (int64_t p = 0; p < k; ++p)
                    s = s + opA(ta, A, lda, i, p) * opB(tb, B, ldb, p, j);
            double* c = &C[i + j * ldc];
            /* beta == 0: C is not read (BLAS), so NaN/Inf on input vanish */
            *c = (beta == 0.0) ? alpha * s : alpha * s + beta * (*c);
        }
    }
    return 0;
}

/* Selected entries only: out[e] = alpha*sum_p op(A)(i,p)op(B)(p,j) + beta*C(i,j)
 * for (i,j) = (rows[e], cols[e]); C is read only, and not at all when beta==0.
 * Serves the sampled parity checks at sizes the full triple loop cannot reach. */
int ftgo_gemm_entries(int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                      const double* A, int64_t lda, const double* B, int64_t ldb,
                      double beta, const double* C, int64_t ldc, int64_t count,
                      const int64_t* rows, const int64_t* cols, double* out)
{
    int info = gemm_arg_check(ta, tb, m, n, k, lda, ldb, ldc);
    if (info) return info;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; ++e) {
        int64_t i = rows[e], j = cols[e];
        double s = 0.0;
        if (alpha != 0.0)
            for (int64_t p = 0; p < k; ++p)
                s = s + opA(ta, A, lda, i, p) * opB(tb, B, ldb, p, j);
        out[e] = (beta == 0.0) ? alpha * s : alpha * s + beta * C[i + j * ldc];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 2. Bit flips (the fault model of §1: fail-continue soft errors that flip  */
/*    bits of values held in compute logic).                                */
/* ------------------------------------------------------------------------ */
double ftgo_flip64(double x, int bit)
{
    uint64_t u;
    memcpy(&u, &x, 8);
    u ^= (uint64_t)1 << bit;
    memcpy(&x, &u, 8);
    return x;
}

float ftgo_flip32(float x, int bit)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    u ^= (uint32_t)1 << bit;
    memcpy(&x, &u, 4);
    return x;
}

/* ------------------------------------------------------------------------ */
/* 3. Counter-based generator: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014). */
/*    Output number ctr of the stream seeded with `seed` is the SplitMix64   */
/*    finaliser applied to seed + (ctr+1) * 0x9E3779B97F4A7C15.              */
/* ------------------------------------------------------------------------ */
uint64_t ftgo_splitmix64(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

/* Keyed bijection of the slot ids [0,S): slot(r) = (a*r + b) mod S with
 * gcd(a,S) = 1.  b is output 0 of the stream; a is the first of outputs
 * 1..64 mapped to 1 + x mod (S-1) that is coprime to S (a = 1 if none is). */
void ftgo_slot_permutation(uint64_t seed, uint64_t S, uint64_t* a_out, uint64_t* b_out)
{
    uint64_t a = 1, b = 0;
    if (S > 1) {
        b = ftgo_splitmix64(seed, 0) % S;
        for (uint64_t t = 1; t <= 64; ++t) {
            uint64_t cand = 1 + ftgo_splitmix64(seed, t) % (S - 1);
            if (gcd_u64(cand, S) == 1) { a = cand; break; }
        }
    }
    *a_out = a;
    *b_out = b;
}

/* One planned fault.  row/col are tile-local; pflip is the global step after
 * whose update the value is flipped. */
typedef struct {
    int64_t tile_m, tile_n, interval;
    int64_t row, col, pflip;
    int32_t bit, target; /* target 0: accumulator C(i,j); 1: row checksum e_r(i) */
} ftgo_fault;

enum { FTGO_TARGET_ACC = 0, FTGO_TARGET_CHECKSUM = 1, FTGO_TARGET_TWO_IN_SLOT = 2 };

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

/* The injection plan.  Slots are (tile, interval) pairs, numbered
 * s = (tile_n*tiles_m + tile_m)*n_intervals + interval.  Fault r (r < F) goes
 * to slot (a*r+b) mod S, so the F slots are distinct.  Its draws are outputs
 * 1024+8r .. 1024+8r+7 of the stream:
 *   row  = x0 mod rows_in_tile,   col = x1 mod cols_in_tile,
 *   step = p_lo + x2 mod (p_hi - p_lo),  bit = bit_lo + x3 mod (bit_hi-bit_lo+1);
 * the flip lands after the update of the rank-kgran block holding `step`
 * (clipped to the interval).  Target TWO_IN_SLOT adds a second accumulator
 * fault in another row and column of the same slot from x4..x7.
 * Returns the number of entries written (F capped at S; two per slot for
 * TWO_IN_SLOT, whose slots need at least two rows and two columns). */
int64_t ftgo_fault_plan(uint64_t seed, int64_t n_faults, int32_t target, int32_t bit_lo,
                        int32_t bit_hi, int64_t m, int64_t n, int64_t k, int64_t bm,
                        int64_t bn, int64_t kc, int64_t kgran, ftgo_fault* out, int64_t cap)
{
    if (m <= 0 || n <= 0 || k <= 0 || n_faults <= 0) return 0;
    if (kc <= 0) kc = k;
    int64_t tiles_m = ceil_div(m, bm), tiles_n = ceil_div(n, bn), n_int = ceil_div(k, kc);
    uint64_t S = (uint64_t)(tiles_m * tiles_n * n_int);
    int64_t F = n_faults < (int64_t)S ? n_faults : (int64_t)S;
    uint64_t a, b;
    ftgo_slot_permutation(seed, S, &a, &b);
    int64_t w = 0;
    for (int64_t r = 0; r < F; ++r) {
        uint64_t s = (a * (uint64_t)r + b) % S;
        int64_t t = (int64_t)(s % (uint64_t)n_int);
        int64_t tile = (int64_t)(s / (uint64_t)n_int);
        int64_t tm = tile % tiles_m, tn = tile / tiles_m;
        int64_t rows = min64(bm, m - tm * bm), cols = min64(bn, n - tn * bn);
        int64_t plo = t * kc, phi = min64(k, plo + kc);
        uint64_t c0 = 1024 + 8 * (uint64_t)r;
        uint64_t x[8];
        for (int q = 0; q < 8; ++q) x[q] = ftgo_splitmix64(seed, c0 + (uint64_t)q);
        int32_t nbits = bit_hi - bit_lo + 1;
        ftgo_fault f;
        f.tile_m = tm; f.tile_n = tn; f.interval = t;
        f.row = (int64_t)(x[0] % (uint64_t)rows);
        f.col = (int64_t)(x[1] % (uint64_t)cols);
        int64_t step = plo + (int64_t)(x[2] % (uint64_t)(phi - plo));
        f.pflip = min64(phi, (step / kgran + 1) * kgran) - 1;
        f.bit = bit_lo + (int32_t)(x[3] % (uint64_t)nbits);
        f.target = (target == FTGO_TARGET_CHECKSUM) ? FTGO_TARGET_CHECKSUM : FTGO_TARGET_ACC;
        if (target == FTGO_TARGET_TWO_IN_SLOT) {
            if (rows < 2 || cols < 2) continue;
            if (w + 2 > cap) break;
            out[w++] = f;
            ftgo_fault g = f;
            g.row = (f.row + 1 + (int64_t)(x[4] % (uint64_t)(rows - 1))) % rows;
            g.col = (f.col + 1 + (int64_t)(x[5] % (uint64_t)(cols - 1))) % cols;
            int64_t step2 = plo + (int64_t)(x[6] % (uint64_t)(phi - plo));
            g.pflip = min64(phi, (step2 / kgran + 1) * kgran) - 1;
            g.bit = bit_lo + (int32_t)(x[7] % (uint64_t)nbits);
            out[w++] = g;
        } else {
            if (w + 1 > cap) break;
            out[w++] = f;
        }
    }
    return w;
}

/* ------------------------------------------------------------------------ */
/* 4. Round-off threshold (the paper requires a mismatch to exceed "the      */
/*    round-off threshold", §2.1, without giving it; this is the reading).  */
/*                                                                          */
/* gamma(n) = n u / (1 - n u), u = 2^-53 (binary64 accumulation).           */
/* For a tile row i, with M_i = sum_p |a_ip| * sum_{j in J} |b_pj| (+ the   */
/* |beta| |C_in| row sum at the final interval), both the reference sum of */
/* the computed row and the maintained checksum differ from the exact row  */
/* sum by at most gamma(p_end + ncols) M_i in any summation order, so       */
/*    tau_i = 2 gamma(p_end + ncols + 8) M_i (1 + 2^-20)                    */
/* can never be exceeded by rounding alone.  Columns: the same with nrows.   */
/* binary32 accumulation (low-precision operands): the probabilistic form  */
/* lambda sqrt(n) u32 replaces gamma(n), u32 = 2^-24.                        */
/* ------------------------------------------------------------------------ */
double ftgo_gamma(int64_t nterms)
{
    double nu = (double)nterms * 0x1p-53;
    return nu / (1.0 - nu);
}

double ftgo_tau(int acc32, double lambda, int64_t nterms, double mag)
{
    double g = acc32 ? lambda * sqrt((double)nterms) * 0x1p-24 : ftgo_gamma(nterms);
    return 2.0 * g * mag * (1.0 + 0x1p-20);
}

/* ------------------------------------------------------------------------ */
/* 5. The ABFT procedure, tile by tile.                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t ta, tb;
    int64_t m, n, k;
    double alpha, beta;
    int64_t lda, ldb, ldc;
    int64_t bm, bn;   /* output tile (the unit that carries its own checksums) */
    int64_t kc;       /* verification interval in steps of p; 0 = whole k */
    int32_t acc32;    /* 1: accumulator and maintained checksums are binary32 */
    double lambda;    /* threshold scale for acc32 */
    int32_t correct_policy;       /* 0: subtract, re-verify, recompute; 1: recompute */
    int32_t uncorrectable_policy; /* 0: report only; 1: recompute the tile */
    int32_t split;    /* 1: every interval is a product of its own (see ftgo_abft) */
} ftgo_params;

typedef struct {
    int64_t tile_m, tile_n, interval;
    int64_t row, col; /* global; -1 where not applicable */
    int32_t kind;
    double delta, tau;
} ftgo_record;

enum {
    FTGO_KIND_SUBTRACT = 1,
    FTGO_KIND_RECOMPUTE = 2,
    FTGO_KIND_CHECKSUM_ONLY = 3,
    FTGO_KIND_UNCORRECTABLE = 4,
    FTGO_KIND_TILE_RECOMPUTED = 5
};

typedef struct {
    int64_t injected, detected, corrected_subtract, corrected_recompute;
    int64_t checksum_only, uncorrectable, tiles_recomputed, n_records;
} ftgo_counts;

/* value of the accumulator after a flip of `bit` (binary32 path: of fl32(x)) */
static double flip_value(int acc32, double x, int bit)
{
    if (acc32) return (double)ftgo_flip32((float)x, bit);
    return ftgo_flip64(x, bit);
}

/* NaN-safe flag: set unless |d| <= tau holds (so NaN and Inf are flagged) */
static int flagged(double d, double tau) { return !(fabs(d) <= tau); }

/* Subtracting the error magnitude (§6.3) returns the true value only when the
 * faulty value still carries it.  The row threshold tau spreads over the q
 * elements of the row, so the subtraction is trusted while the rounding unit
 * of x (in the output's precision) stays within tau / (2 q); beyond that the
 * true value has been absorbed and the element is recomputed instead. */
static int absorbed(int acc32, double x, double tau, int64_t q)
{
    if (x == 0.0) return 0;
    double ulp = ldexp(1.0, ilogb(x) - (acc32 ? 23 : 52));
    return ulp > tau / (2.0 * (double)q);
}

typedef struct {
    /* tile geometry */
    int64_t i0, j0, R, Q;
    /* state, R x Q accumulator (column-major, leading dim R) */
    double *acc, *er, *ec, *mr, *mc;
    /* binary32 path: sum_p |a_ip|, sum_p |b_pj|, max_p sum_j |b_pj|, max_p sum_i |a_ip| */
    double *ra, *cb, mxb, mxa;
    /* per-verification scratch */
    double *rs, *cs, *out;
    const ftgo_params* P;
    const double *A, *B, *Cin;
    /* first step of the product being checked (0, or the interval's with
     * `split`) and the beta that scales C_in at its final check */
    int64_t plo;
    double beta_t;
} tile_state;

static double tA(const tile_state* T, int64_t i, int64_t p)
{
    return opA(T->P->ta, T->A, T->P->lda, T->i0 + i, p);
}
static double tB(const tile_state* T, int64_t p, int64_t j)
{
    return opB(T->P->tb, T->B, T->P->ldb, p, T->j0 + j);
}
static double tC(const tile_state* T, int64_t i, int64_t j)
{
    return T->Cin[(T->i0 + i) + (T->j0 + j) * T->P->ldc];
}

/* Rank-1 updates of steps p in [plo, phi): acc += a_p b_p^T together with the
 * checksum row e^T a_p and column b_p e of the encoded operands (§2.1) and the
 * magnitude sums that feed the threshold; planned faults flip after their step. */
static void advance(tile_state* T, int64_t plo, int64_t phi, const ftgo_fault* plan,
                    int64_t nplan, int inject, ftgo_counts* cnt)
{
    int64_t R = T->R, Q = T->Q;
    for (int64_t p = plo; p < phi; ++p) {
        double as = 0.0, asa = 0.0, bs = 0.0, bsa = 0.0;
        for (int64_t i = 0; i < R; ++i) { double a = tA(T, i, p); as = as + a; asa = asa + fabs(a); }
        for (int64_t j = 0; j < Q; ++j) { double b = tB(T, p, j); bs = bs + b; bsa = bsa + fabs(b); }
        for (int64_t j = 0; j < Q; ++j) {
            double b = tB(T, p, j);
            for (int64_t i = 0; i < R; ++i) T->acc[i + j * R] = T->acc[i + j * R] + tA(T, i, p) * b;
        }
        for (int64_t i = 0; i < R; ++i) {
            double a = tA(T, i, p);
            T->er[i] = T->er[i] + a * bs;
            T->mr[i] = T->mr[i] + fabs(a) * bsa;
            T->ra[i] = T->ra[i] + fabs(a);
        }
        for (int64_t j = 0; j < Q; ++j) {
            double b = tB(T, p, j);
            T->ec[j] = T->ec[j] + as * b;
            T->mc[j] = T->mc[j] + asa * fabs(b);
            T->cb[j] = T->cb[j] + fabs(b);
        }
        if (bsa > T->mxb) T->mxb = bsa;
        if (asa > T->mxa) T->mxa = asa;
        if (!inject) continue;
        for (int64_t f = 0; f < nplan; ++f) {
            if (plan[f].pflip != p) continue;
            if (plan[f].target == FTGO_TARGET_CHECKSUM) {
                T->er[plan[f].row] = flip_value(T->P->acc32, T->er[plan[f].row], plan[f].bit);
            } else {
                double* x = &T->acc[plan[f].row + plan[f].col * R];
                *x = flip_value(T->P->acc32, *x, plan[f].bit);
            }
            cnt->injected++;
        }
    }
}

/* Fresh dot product of row i and column j over steps [plo, pend), ascending. */
static double dot_fresh(const tile_state* T, int64_t i, int64_t j, int64_t pend)
{
    double s = 0.0;
    for (int64_t p = T->plo; p < pend; ++p) s = s + tA(T, i, p) * tB(T, p, j);
    return s;
}

/* Value the tile holds for element (i,j) at this verification: the
 * accumulator mid-way, alpha*acc + beta*C_in at the final interval (§5.2 fuses
 * the C checksums with the beta scaling, so the final check covers it). */
static double out_value(const tile_state* T, int final, double accv, int64_t i, int64_t j)
{
    if (!final) return accv;
    const ftgo_params* P = T->P;
    return (T->beta_t == 0.0) ? P->alpha * accv : P->alpha * accv + T->beta_t * tC(T, i, j);
}

typedef struct { double d, tau; } check;

/* delta and tau of row i (dir 0) or column j (dir 1) of the held values */
static check check_line(const tile_state* T, int final, int64_t pend, int dir, int64_t x)
{
    const ftgo_params* P = T->P;
    int64_t R = T->R, Q = T->Q;
    double ref = 0.0, cin = 0.0, cinabs = 0.0;
    int64_t len = dir == 0 ? Q : R;
    for (int64_t y = 0; y < len; ++y) {
        int64_t i = dir == 0 ? x : y, j = dir == 0 ? y : x;
        ref = ref + T->out[i + j * R];
        if (final && T->beta_t != 0.0) { double c = tC(T, i, j); cin = cin + c; cinabs = cinabs + fabs(c); }
    }
    double maint = dir == 0 ? T->er[x] : T->ec[x];
    double mag = dir == 0 ? T->mr[x] : T->mc[x];
    /* binary32 path: the bound (sum_p |a_ip|) max_p (sum_j |b_pj|) >= sum_p |a_ip| sum_j |b_pj|
     * (and alike for columns), which needs only per-line and per-panel sums */
    if (P->acc32) mag = dir == 0 ? T->ra[x] * T->mxb : T->cb[x] * T->mxa;
    double expect = maint;
    if (final) {
        expect = P->alpha * maint;
        mag = fabs(P->alpha) * mag;
        if (T->beta_t != 0.0) { expect = expect + T->beta_t * cin; mag = mag + fabs(T->beta_t) * cinabs; }
    }
    check c;
    c.d = ref - expect;
    c.tau = ftgo_tau(P->acc32, P->lambda, pend - T->plo + len + 8, mag);
    return c;
}

static void push_record(ftgo_record* recs, int64_t cap, ftgo_counts* cnt, const tile_state* T,
                        int64_t tm, int64_t tn, int64_t t, int64_t row, int64_t col, int kind,
                        double d, double tau)
{
    if (cnt->n_records < cap) {
        ftgo_record* r = &recs[cnt->n_records];
        r->tile_m = tm; r->tile_n = tn; r->interval = t;
        r->row = row < 0 ? -1 : T->i0 + row;
        r->col = col < 0 ? -1 : T->j0 + col;
        r->kind = kind; r->delta = d; r->tau = tau;
    }
    cnt->n_records++;
}

/* Sum of row x (dir 0) or column x (dir 1) of the held values, in the order
 * check_line forms its reference sum. */
static double held_line_sum(const tile_state* T, int dir, int64_t x)
{
    int64_t R = T->R, Q = T->Q;
    int64_t len = dir == 0 ? Q : R;
    double ref = 0.0;
    for (int64_t y = 0; y < len; ++y) {
        int64_t i = dir == 0 ? x : y, j = dir == 0 ? y : x;
        ref = ref + T->out[i + j * R];
    }
    return ref;
}

/* Verification of one (tile, interval) slot: flags, classification, correction. */
static void verify_slot(tile_state* T, int final, int64_t pend, int64_t tm, int64_t tn, int64_t t,
                        const ftgo_fault* plan, int64_t nplan, ftgo_record* recs, int64_t cap,
                        ftgo_counts* cnt)
{
    const ftgo_params* P = T->P;
    int64_t R = T->R, Q = T->Q;
    for (int64_t j = 0; j < Q; ++j)
        for (int64_t i = 0; i < R; ++i)
            T->out[i + j * R] = out_value(T, final, T->acc[i + j * R], i, j);

    int64_t nr = 0, nc = 0, fi = -1, fj = -1;
    double dri = 0.0, tri = 0.0, dcj = 0.0, tcj = 0.0;
    for (int64_t i = 0; i < R; ++i) {
        check c = check_line(T, final, pend, 0, i);
        if (flagged(c.d, c.tau)) { if (nr == 0) { fi = i; dri = c.d; tri = c.tau; } nr++; }
    }
    for (int64_t j = 0; j < Q; ++j) {
        check c = check_line(T, final, pend, 1, j);
        if (flagged(c.d, c.tau)) { if (nc == 0) { fj = j; dcj = c.d; tcj = c.tau; } nc++; }
    }
    if (nr == 0 && nc == 0) goto store;
    cnt->detected++;

    if (nr == 1 && nc == 1) {
        /* one faulty element located at the intersection (§5.1) */
        double* x = &T->out[fi + fj * R];
        int kind = 0;
        if (P->correct_policy == 0 && isfinite(dri) && isfinite(*x) && !absorbed(P->acc32, *x, tri, Q)) {
            double keep = *x;
            *x = *x - dri; /* subtract the error magnitude (§6.3) */
            check a = check_line(T, final, pend, 0, fi), b = check_line(T, final, pend, 1, fj);
            if (!flagged(a.d, a.tau) && !flagged(b.d, b.tau)) kind = FTGO_KIND_SUBTRACT;
            else *x = keep;
        }
        if (!kind) {
            double keep = *x;
            double fresh = dot_fresh(T, fi, fj, pend);
            *x = out_value(T, final, fresh, fi, fj);
            check a = check_line(T, final, pend, 0, fi), b = check_line(T, final, pend, 1, fj);
            kind = (!flagged(a.d, a.tau) && !flagged(b.d, b.tau)) ? FTGO_KIND_RECOMPUTE
                                                                  : FTGO_KIND_UNCORRECTABLE;
            if (kind == FTGO_KIND_UNCORRECTABLE) *x = keep; /* leave the data as found */
        }
        if (kind != FTGO_KIND_UNCORRECTABLE) {
            if (!final) T->acc[fi + fj * R] = *x; /* the held value carries on */
            if (kind == FTGO_KIND_SUBTRACT) cnt->corrected_subtract++;
            else cnt->corrected_recompute++;
            push_record(recs, cap, cnt, T, tm, tn, t, fi, fj, kind, dri, tri);
            goto store;
        }
    } else if (nr + nc == 1) {
        /* one direction only: the maintained checksum is the faulty value;
         * the data passed the other direction's check and is kept.  The
         * checksum is re-based on the data so later intervals start clean:
         * set to the line's sum of the held values (adding the mismatch
         * instead would lose the checksum's own value after a flip to a huge
         * value, and the later intervals would flag the line again). */
        if (nr) { if (!final) T->er[fi] = held_line_sum(T, 0, fi); }
        else    { if (!final) T->ec[fj] = held_line_sum(T, 1, fj); }
        cnt->checksum_only++;
        push_record(recs, cap, cnt, T, tm, tn, t, nr ? fi : -1, nr ? -1 : fj,
                    FTGO_KIND_CHECKSUM_ONLY, nr ? dri : dcj, nr ? tri : tcj);
        goto store;
    }

    /* more than one error in the interval: outside the model (§2.1) */
    cnt->uncorrectable++;
    if (P->uncorrectable_policy == 1) {
        /* recompute the tile from scratch, injection off (transient faults) */
        memset(T->acc, 0, sizeof(double) * R * Q);
        memset(T->er, 0, sizeof(double) * R);
        memset(T->ec, 0, sizeof(double) * Q);
        memset(T->mr, 0, sizeof(double) * R);
        memset(T->mc, 0, sizeof(double) * Q);
        memset(T->ra, 0, sizeof(double) * R);
        memset(T->cb, 0, sizeof(double) * Q);
        T->mxb = T->mxa = 0.0;
        advance(T, T->plo, pend, plan, nplan, 0, cnt);
        for (int64_t j = 0; j < Q; ++j)
            for (int64_t i = 0; i < R; ++i)
                T->out[i + j * R] = out_value(T, final, T->acc[i + j * R], i, j);
        cnt->tiles_recomputed++;
        push_record(recs, cap, cnt, T, tm, tn, t, -1, -1, FTGO_KIND_TILE_RECOMPUTED,
                    nr ? dri : dcj, nr ? tri : tcj);
    } else {
        push_record(recs, cap, cnt, T, tm, tn, t, -1, -1, FTGO_KIND_UNCORRECTABLE,
                    nr ? dri : dcj, nr ? tri : tcj);
    }

store:
    if (final) {
        double* C = (double*)T->Cin;
        for (int64_t j = 0; j < Q; ++j)
            for (int64_t i = 0; i < R; ++i) C[(T->i0 + i) + (T->j0 + j) * P->ldc] = T->out[i + j * R];
    }
}

/* Runs the protected product over all tiles and intervals.  C is updated in
 * place (it is C_in on entry).  plan/nplan: from ftgo_fault_plan (may be 0).
 * recs: capacity `cap`; counts->n_records may exceed cap (records dropped). */
int ftgo_abft(const ftgo_params* P, const double* A, const double* B, double* C,
              const ftgo_fault* plan, int64_t nplan, ftgo_record* recs, int64_t cap,
              ftgo_counts* counts)
{
    memset(counts, 0, sizeof(*counts));
    int info = gemm_arg_check(P->ta, P->tb, P->m, P->n, P->k, P->lda, P->ldb, P->ldc);
    if (info) return info;
    if (P->bm <= 0 || P->bn <= 0) return -1;
    if (P->m == 0 || P->n == 0) return 0;
    if (P->alpha == 0.0 || P->k == 0) /* no product: C := beta*C, nothing to protect */
        return ftgo_gemm(P->ta, P->tb, P->m, P->n, 0, 0.0, A, P->lda, B, P->ldb, P->beta, C, P->ldc);

    int64_t kc = P->kc > 0 ? P->kc : P->k;
    int64_t tiles_m = ceil_div(P->m, P->bm), tiles_n = ceil_div(P->n, P->bn);
    int64_t n_int = ceil_div(P->k, kc);
    int64_t R0 = P->bm, Q0 = P->bn;
    tile_state T;
    T.P = P; T.A = A; T.B = B; T.Cin = C;
    T.acc = (double*)malloc(sizeof(double) * R0 * Q0);
    T.out = (double*)malloc(sizeof(double) * R0 * Q0);
    T.er = (double*)malloc(sizeof(double) * R0);
    T.mr = (double*)malloc(sizeof(double) * R0);
    T.ec = (double*)malloc(sizeof(double) * Q0);
    T.mc = (double*)malloc(sizeof(double) * Q0);
    T.ra = (double*)malloc(sizeof(double) * R0);
    T.cb = (double*)malloc(sizeof(double) * Q0);
    ftgo_fault* sub = (ftgo_fault*)malloc(sizeof(ftgo_fault) * (nplan > 0 ? nplan : 1));
    if (!T.acc || !T.out || !T.er || !T.mr || !T.ec || !T.mc || !T.ra || !T.cb || !sub) return -2;

    for (int64_t tn = 0; tn < tiles_n; ++tn) {
        for (int64_t tm = 0; tm < tiles_m; ++tm) {
            T.i0 = tm * P->bm; T.j0 = tn * P->bn;
            T.R = min64(P->bm, P->m - T.i0); T.Q = min64(P->bn, P->n - T.j0);
            int64_t ns = 0; /* this tile's faults */
            for (int64_t f = 0; f < nplan; ++f)
                if (plan[f].tile_m == tm && plan[f].tile_n == tn) sub[ns++] = plan[f];
            T.plo = 0;
            T.beta_t = P->beta;
            for (int64_t t = 0; t < n_int; ++t) {
                int64_t plo = t * kc, phi = min64(P->k, plo + kc);
                if (t == 0 || P->split) {
                    /* a fresh accumulator, checksums and magnitude sums: the
                     * product's start (with `split`, every interval's, whose
                     * check then also covers C_in as left by the interval
                     * before, with beta_t = 1) */
                    memset(T.acc, 0, sizeof(double) * T.R * T.Q);
                    memset(T.er, 0, sizeof(double) * T.R);
                    memset(T.mr, 0, sizeof(double) * T.R);
                    memset(T.ec, 0, sizeof(double) * T.Q);
                    memset(T.mc, 0, sizeof(double) * T.Q);
                    memset(T.ra, 0, sizeof(double) * T.R);
                    memset(T.cb, 0, sizeof(double) * T.Q);
                    T.mxb = T.mxa = 0.0;
                }
                if (P->split) { T.plo = plo; T.beta_t = t == 0 ? P->beta : 1.0; }
                advance(&T, plo, phi, sub, ns, 1, counts);
                verify_slot(&T, P->split || t == n_int - 1, phi, tm, tn, t, sub, ns, recs, cap, counts);
            }
        }
    }
    free(T.acc); free(T.out); free(T.er); free(T.mr); free(T.ec); free(T.mc); free(T.ra); free(T.cb);
    free(sub);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 6. Level-3 routines that run on the protected product (§6.2.3): their    */
/*    plain definitions, reading only the referenced triangle of A.        */
/*    side 0 = left, 1 = right; uplo 0 = lower, 1 = upper; diag 1 = unit.   */
/* ------------------------------------------------------------------------ */

/* element (i, j) of a symmetric matrix stored in one triangle */
static double sym_at(int uplo, const double* A, int64_t lda, int64_t i, int64_t j)
{
    int stored = uplo == 0 ? i >= j : i <= j;
    return stored ? A[i + j * lda] : A[j + i * lda];
}

/* C := alpha A B + beta C (left, A m x m) or alpha B A + beta C (right, A n x n) */
int ftgo_dsymm(int side, int uplo, int64_t m, int64_t n, double alpha, const double* A, int64_t lda,
               const double* B, int64_t ldb, double beta, double* C, int64_t ldc)
{
    if (side != 0 && side != 1) return 1;
    if (uplo != 0 && uplo != 1) return 2;
    if (m < 0) return 3;
    if (n < 0) return 4;
    if (lda < max64(1, side == 0 ? m : n)) return 7;
    if (ldb < max64(1, m)) return 9;
    if (ldc < max64(1, m)) return 12;
    if (m == 0 || n == 0 || (alpha == 0.0 && beta == 1.0)) return 0;
    int64_t k = side == 0 ? m : n;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            if (alpha != 0.0)
                for (int64_t p = 0; p < k; ++p)
                    s = s + (side == 0 ? sym_at(uplo, A, lda, i, p) * B[p + j * ldb]
                                       : B[i + p * ldb] * sym_at(uplo, A, lda, p, j));
            double* c = &C[i + j * ldc];
            *c = (beta == 0.0) ? alpha * s : alpha * s + beta * (*c);
        }
    }
    return 0;
}

/* element (i, j) of op(A) for a triangular A: 0 outside the stored triangle,
 * 1 on a unit diagonal; *nz = 0 where the element is an implicit zero */
static double tri_op_at(int uplo, int ta, int diag, const double* A, int64_t lda, int64_t i, int64_t j, int* nz)
{
    int64_t r = ta ? j : i, c = ta ? i : j; /* position in the stored matrix */
    *nz = 1;
    if (r == c) return diag ? 1.0 : A[r + c * lda];
    if (uplo == 0 ? r > c : r < c) return A[r + c * lda];
    *nz = 0;
    return 0.0;
}

/* B := alpha op(A) B (left, A m x m) or alpha B op(A) (right, A n x n); only
 * the nonzero terms of op(A) enter the sums (ascending p) */
int ftgo_dtrmm(int side, int uplo, int ta, int diag, int64_t m, int64_t n, double alpha, const double* A,
               int64_t lda, double* B, int64_t ldb)
{
    if (side != 0 && side != 1) return 1;
    if (uplo != 0 && uplo != 1) return 2;
    if (ta != 0 && ta != 1) return 3;
    if (diag != 0 && diag != 1) return 4;
    if (m < 0) return 5;
    if (n < 0) return 6;
    if (lda < max64(1, side == 0 ? m : n)) return 9;
    if (ldb < max64(1, m)) return 11;
    if (m == 0 || n == 0) return 0;
    double* T = (double*)malloc(sizeof(double) * (size_t)(m * n));
    if (!T) return -2;
    int64_t k = side == 0 ? m : n;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            if (alpha != 0.0)
                for (int64_t p = 0; p < k; ++p) {
                    int nz;
                    double a = side == 0 ? tri_op_at(uplo, ta, diag, A, lda, i, p, &nz)
                                         : tri_op_at(uplo, ta, diag, A, lda, p, j, &nz);
                    if (!nz) continue;
                    s = s + (side == 0 ? a * B[p + j * ldb] : B[i + p * ldb] * a);
                }
            T[i + j * m] = alpha * s;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) B[i + j * ldb] = T[i + j * m];
    free(T);
    return 0;
}

/* B := alpha op(A)^-1 B (left, A m x m) or alpha B op(A)^-1 (right, A n x n),
 * A triangular: substitution in the order op(A) dictates, one right-hand
 * side at a time, subtracting the solved terms in ascending index order. */
int ftgo_dtrsm(int side, int uplo, int ta, int diag, int64_t m, int64_t n, double alpha, const double* A,
               int64_t lda, double* B, int64_t ldb)
{
    if (side != 0 && side != 1) return 1;
    if (uplo != 0 && uplo != 1) return 2;
    if (ta != 0 && ta != 1) return 3;
    if (diag != 0 && diag != 1) return 4;
    if (m < 0) return 5;
    if (n < 0) return 6;
    if (lda < max64(1, side == 0 ? m : n)) return 9;
    if (ldb < max64(1, m)) return 11;
    if (m == 0 || n == 0) return 0;
    /* op(A) is lower triangular when (lower, no transpose) or (upper, transpose) */
    int lower_op = (uplo == 0) == (ta == 0);
    if (side == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t q = 0; q < m; ++q) {
                int64_t i = lower_op ? q : m - 1 - q;
                double s = alpha * B[i + j * ldb];
                int64_t p0 = lower_op ? 0 : i + 1, p1 = lower_op ? i : m;
                for (int64_t p = p0; p < p1; ++p) {
                    int nz;
                    double a = tri_op_at(uplo, ta, diag, A, lda, i, p, &nz);
                    s = s - a * B[p + j * ldb];
                }
                if (!diag) { int nz; s = s / tri_op_at(uplo, ta, diag, A, lda, i, i, &nz); }
                B[i + j * ldb] = s;
            }
        }
    } else {
        /* X op(A) = alpha B: column j of X needs the columns p with op(A)(p, j)
         * nonzero: p > j when op(A) is lower (solve backward), p < j when upper */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t q = 0; q < n; ++q) {
                int64_t j = lower_op ? n - 1 - q : q;
                double s = alpha * B[i + j * ldb];
                int64_t p0 = lower_op ? j + 1 : 0, p1 = lower_op ? n : j;
                for (int64_t p = p0; p < p1; ++p) {
                    int nz;
                    double a = tri_op_at(uplo, ta, diag, A, lda, p, j, &nz);
                    s = s - B[i + p * ldb] * a;
                }
                if (!diag) { int nz; s = s / tri_op_at(uplo, ta, diag, A, lda, j, j, &nz); }
                B[i + j * ldb] = s;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Level-1 and Level-2 routines that FT-BLAS protects by duplicated
 * computation (§4), by their plain BLAS definitions.  Vectors are n
 * elements at stride inc; for a negative stride element 0 sits at the far
 * end (x + (1 - n) inc), as BLAS defines. */

static const double* vec0c(const double* x, int64_t n, int64_t inc) { return inc > 0 ? x : x + (1 - n) * inc; }
static double* vec0(double* x, int64_t n, int64_t inc) { return inc > 0 ? x : x + (1 - n) * inc; }

/* x := alpha x (nothing for n <= 0 or incx <= 0): one product per element. */
void ftgo_dscal(int64_t n, double alpha, double* x, int64_t incx)
{
    if (n <= 0 || incx <= 0) return;
    for (int64_t i = 0; i < n; ++i) x[i * incx] = alpha * x[i * incx];
}

/* Euclidean norm of n elements at stride incx (0 for n <= 0 or incx <= 0).
 * NaN if an element is NaN, else +Inf if one is infinite, else
 * 2^e sqrt(sum_i (x_i 2^-e)^2) with 2^e the power of two of the largest
 * magnitude.  Scaling by a power of two is exact, so no square overflows
 * (every scaled element is below 2 in magnitude) and the roundings are
 * those of the squares, the ascending sum and the square root. */
double ftgo_dnrm2(int64_t n, const double* x, int64_t incx)
{
    if (n <= 0 || incx <= 0) return 0.0;
    int has_nan = 0, has_inf = 0;
    double amax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double v = x[i * incx];
        if (isnan(v)) has_nan = 1;
        else if (isinf(v)) has_inf = 1;
        else if (fabs(v) > amax) amax = fabs(v);
    }
    if (has_nan) return NAN;
    if (has_inf) return INFINITY;
    if (amax == 0.0) return 0.0;
    int e = ilogb(amax);
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = ldexp(x[i * incx], -e);
        s = s + t * t;
    }
    return ldexp(sqrt(s), e);
}

/* y := alpha op(A) x + beta y (BLAS dgemv; A m x n column-major; x has n
 * elements without transpose, m with; y the other count).  Each element is
 * alpha times the ascending dot product plus beta y_i (y is not read when
 * beta = 0; A and x are not read when alpha = 0).  Returns the xerbla
 * position of an invalid argument, 0 otherwise. */
int ftgo_dgemv(int ta, int64_t m, int64_t n, double alpha, const double* A, int64_t lda, const double* x,
               int64_t incx, double beta, double* y, int64_t incy)
{
    if (ta != 0 && ta != 1) return 1;
    if (m < 0) return 2;
    if (n < 0) return 3;
    if (lda < max64(1, m)) return 6;
    if (incx == 0) return 8;
    if (incy == 0) return 11;
    if (m == 0 || n == 0 || (alpha == 0.0 && beta == 1.0)) return 0;
    int64_t lenx = ta ? m : n, leny = ta ? n : m;
    const double* x0 = vec0c(x, lenx, incx);
    double* y0 = vec0(y, leny, incy);
    for (int64_t i = 0; i < leny; ++i) {
        double s = 0.0;
        if (alpha != 0.0)
            for (int64_t p = 0; p < lenx; ++p) s = s + (ta ? A[p + i * lda] : A[i + p * lda]) * x0[p * incx];
        double by = beta == 0.0 ? 0.0 : beta * y0[i * incy];
        y0[i * incy] = alpha * s + by;
    }
    return 0;
}

/* x := op(A)^-1 x (BLAS dtrsv; A n x n triangular, the `uplo` triangle
 * read; diag = 1: unit diagonal, not read): substitution in the order op(A)
 * dictates, subtracting the solved terms in ascending index order, then
 * dividing by the diagonal. */
int ftgo_dtrsv(int uplo, int ta, int diag, int64_t n, const double* A, int64_t lda, double* x, int64_t incx)
{
    if (uplo != 0 && uplo != 1) return 1;
    if (ta != 0 && ta != 1) return 2;
    if (diag != 0 && diag != 1) return 3;
    if (n < 0) return 4;
    if (lda < max64(1, n)) return 6;
    if (incx == 0) return 8;
    if (n == 0) return 0;
    double* x0 = vec0(x, n, incx);
    int lower_op = (uplo == 0) == (ta == 0);
    for (int64_t q = 0; q < n; ++q) {
        int64_t i = lower_op ? q : n - 1 - q;
        double s = x0[i * incx];
        int64_t p0 = lower_op ? 0 : i + 1, p1 = lower_op ? i : n;
        for (int64_t p = p0; p < p1; ++p) {
            int nz;
            s = s - tri_op_at(uplo, ta, diag, A, lda, i, p, &nz) * x0[p * incx];
        }
        if (!diag) {
            int nz;
            s = s / tri_op_at(uplo, ta, diag, A, lda, i, i, &nz);
        }
        x0[i * incx] = s;
    }
    return 0;
}
