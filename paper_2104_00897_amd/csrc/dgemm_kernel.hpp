// FP64 checksum-protected GEMM kernel for gfx950 (CDNA4).
//
//   C := alpha op(A) op(B) + beta C, column-major, one workgroup per BM x BN
//   output tile, v_mfma_f64_16x16x4_f64 on 64-lane waves.
//
// ABFT (Zhai et al., FT-BLAS, ICS'21) fused into the tile computation:
//   a1  each k-block's A and B panels are staged in LDS; the checksum row
//       e^T A_I and column B_J e of the encoded operands A^c, B^r (§2.1) are
//       summed from the staged panels (with |.| sums for the threshold);
//   a2  MFMA accumulation acc += A_I B_J over the k loop;
//   a3  maintained checksums er = A_I (B_J e) and ec = (e^T A_I) B_J advanced
//       with every rank-16 update on the register-resident MFMA operands,
//       which keeps the outer-product relation of §2.1 true after each step;
//   a4  at the end, C_in is read once (skipped when beta = 0) and its row and
//       column sums enter the expected checksums, fused with the beta scaling
//       (§5.2);
//   a5  reference sums of the computed C from the accumulators in registers
//       (§5.2) via cross-lane and cross-wave reductions;
//   a6  mismatch beyond the round-off threshold (NaN-safe) flags a row/col;
//   a7  one flagged row and column locate the element, corrected by
//       subtracting the error magnitude (§6.3), re-verified, else recomputed;
//       a flag in one direction only is a checksum fault; more is reported
//       (and the tile recomputed under that policy);
//   a9  the seeded injector flips a bit of an accumulator (or checksum) after
//       the planned k-block;
//   a10 with a verification interval, a5-a7 also run on the accumulators at
//       the end of every interval (the online scheme of §2.1, one correction
//       per interval).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <utility>

#include "ftg_common.hpp"
#include "ftg_kernels.hpp"

namespace ftg {

typedef double d4v __attribute__((ext_vector_type(4)));

template <int BM, int BN, int WGM, int WGN, bool TA, bool TB>
struct DCfg {
    static constexpr int BK = 16;
    static constexpr int NW = WGM * WGN;
    static constexpr int NT = NW * 64;
    static constexpr int WM = BM / WGM, WN = BN / WGN;
    static constexpr int FM = WM / 16, FN = WN / 16;
    // LDS layouts: A as [p][i] (TA = 0) or [i][p] (TA = 1); B as [p][j] (TB = 1)
    // or [j][p], padded pitches.  Both are made of whole 16-byte slots (BK + 2 =
    // 9 slots per line along k), the unit of a direct global-to-LDS load.
    static constexpr int SA = TA ? (BK + 2) : (BM + 16);
    static constexpr int SB = TB ? (BN + 16) : (BK + 2);
    static constexpr int A_ELEMS = TA ? BM * SA : BK * SA;
    static constexpr int B_ELEMS = TB ? BK * SB : BN * SB;
    // direct-to-LDS staging: up to 1 KB (64 lanes x 16 bytes) per wave load
    static constexpr bool DIRECT = BM % 64 == 0 && BN % 64 == 0 && BK == 16;
    // protected kernels of small tiles run one copy of the k loop for all
    // waves also with register staging (their prefetch registers are few):
    // three workgroups per CU
    static constexpr bool ONE_COPY = BM * BN / NW <= 32 * 32;
    static constexpr int NA = BM * BK / NT, NB = BN * BK / NT;  // loads per thread
    static constexpr int PPW = BK / NW, LPP = 64 / PPW;        // encode: p's per wave, lanes per p
    static constexpr int GSH = FM / WGN, HSH = FN / WGM;        // checksum FMA shares per wave
    static_assert(BM * BK % NT == 0 && BN * BK % NT == 0, "load split");
    static_assert(BK % NW == 0 && FM % WGN == 0 && FN % WGM == 0, "checksum split");
    __device__ static int a_idx(int i, int p) { return TA ? i * SA + p : p * SA + i; }
    __device__ static int b_idx(int p, int j) { return TB ? p * SB + j : j * SB + p; }
};

// Per-tile verification bookkeeping in LDS.
template <int BM, int BN, int WGM, int WGN>
struct VerifyLds {
    double rsum[WGN][BM];
    double csum[WGM][BN];
    double cir[WGN][BM], cira[WGN][BM];  // C_in row sums (signed, abs)
    double cic[WGM][BN], cica[WGM][BN];  // C_in column sums
    double er[BM], mr[BM], ec[BN], mc[BN];
    double dfi, tfi, dfj, tfj, xold, dotv, cin;
    int nfr, nfc, fi, fj, xfinite, kind;
};

// The work of one workgroup on output tile (tm, tn) of one problem.  Shared by
// the one-launch-per-problem kernel and the persistent batched kernel.
// PRE: the checksum row/column of the encoded operands come from the encode
// pass (args.asp / args.bsp) and are staged with the operands; otherwise they
// are summed from the staged panels inside the k loop.
// DIR: full k-blocks of interior tiles are loaded straight into LDS (operands
// 16-byte aligned with even leading dimensions); otherwise every block is
// prefetched into registers one block ahead and stored after the MFMAs.
template <int BM, int BN, int WGM, int WGN, bool TA, bool TB, bool ABFT, bool IVL, bool PRE, bool DIR,
          bool WIDE_REGS = false>
__device__ __attribute__((always_inline)) inline void dgemm_tile(const DGemmArgs& args, const int tm,
                                                                 const int tn)
{
    using Cf = DCfg<BM, BN, WGM, WGN, TA, TB>;
    constexpr int BK = Cf::BK, NT = Cf::NT, FM = Cf::FM, FN = Cf::FN;
    constexpr int WM = Cf::WM, WN = Cf::WN;

    // Two staging buffers, each holding the A panel followed by the B panel of
    // one k-block.  The verification bookkeeping (VerifyLds) lives in a stage
    // that holds no live panel at the time (both after the k loop, the one not
    // holding the next block at an interval end), which keeps the workgroup's
    // LDS at the staging size and lets two workgroups share a CU.
    constexpr int SE = Cf::A_ELEMS + Cf::B_ELEMS;  // doubles per stage
    using VL = VerifyLds<BM, BN, WGM, WGN>;
    static_assert(sizeof(VL) <= SE * sizeof(double), "verification data must fit in one stage");
    __shared__ double stg[2][SE];
    __shared__ double sums[2][2][BK][2];  // [stage][A, B][p]: (e^T A_I, |A_I|), (B_J e, |B_J|)
    auto As = [&](int st) __attribute__((always_inline)) { return &stg[st][0]; };
    auto Bs = [&](int st) __attribute__((always_inline)) { return &stg[st][Cf::A_ELEMS]; };
    VL* Vp = reinterpret_cast<VL*>(&stg[0][0]);
    __shared__ int flt[kMaxIntervals][2][4];  // per interval: up to two faults (row, col, pflip, bit)
    __shared__ int fltn[kMaxIntervals];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / WGN, wc = wave % WGN;
    const int wm0 = wr * WM, wn0 = wc * WN;
    const int l16 = lane & 15, lq = lane >> 4;

    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int R = (int)min((int64_t)BM, (int64_t)args.m - m0);
    const int Q = (int)min((int64_t)BN, (int64_t)args.n - n0);
    const int64_t K = args.k;  // widened for index math
    const int nkb = (int)((K + BK - 1) / BK);
    const int64_t kc = args.kc;  // interval length (multiple of kKGran), >= K means one interval
    const int n_int = (int)((K + kc - 1) / kc);  // <= kMaxIntervals (checked by the host)

    const double* A = args.A;
    const double* B = args.B;

    d4v acc[FM][FN];
    double er[Cf::GSH], mr[Cf::GSH], ec[Cf::HSH], mc[Cf::HSH];
    double ra[Cf::NA], rb[Cf::NB];

    auto zero_state = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int g = 0; g < FM; ++g)
#pragma unroll
            for (int h = 0; h < FN; ++h) acc[g][h] = (d4v){0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < Cf::GSH; ++q) er[q] = mr[q] = 0.0;
#pragma unroll
        for (int q = 0; q < Cf::HSH; ++q) ec[q] = mc[q] = 0.0;
    };

    // ---- global -> registers.  Each thread stages a fixed line of the operand
    // panel and walks along the operand's contiguous dimension, so the q-th load
    // is the thread's byte offset plus the constant q*8 (an immediate operand of
    // the buffer instruction: no per-load scalar registers).  Elements outside
    // the matrix read 0 through an out-of-range offset.
    //   contiguous along the tile dimension (A with TA=0, B with TB=1):
    //     LPT = NT/BK lanes per k step, element q at tile index lane%LPT + LPT*q;
    //   contiguous along k (A with TA=1, B with TB=0):
    //     NT/ROWS threads per tile line, each reading BK*ROWS/NT consecutive steps.
    constexpr int LPT = NT / BK;
    static_assert(NT % BM == 0 && NT % BN == 0 && NT % BK == 0, "staging map");
    constexpr int APT = TA ? BK * BM / NT : BM / LPT;   // elements per thread
    constexpr int BPT = TB ? BN / LPT : BK * BN / NT;
    static_assert(APT == Cf::NA && BPT == Cf::NB, "staging count");
    const int64_t lda = args.lda, ldb = args.ldb;
    // the staging map of thread t_ (its first element of each panel)
    struct SMap { int ai0, ap0, bj0, bp0, a_voff, b_voff; };
    auto smap = [&](int t_) __attribute__((always_inline)) {
        SMap m;
        // A: TA=0 -> (i = t%LPT + LPT q, p = t/LPT); TA=1 -> (i = t%BM, p = (t/BM)*APT + q)
        m.ai0 = TA ? t_ % BM : t_ % LPT;
        m.ap0 = TA ? (t_ / BM) * APT : t_ / LPT;
        // B: TB=1 -> (j = t%LPT + LPT q, p = t/LPT); TB=0 -> (j = t%BN, p = (t/BN)*BPT + q)
        m.bj0 = TB ? t_ % LPT : t_ % BN;
        m.bp0 = TB ? t_ / LPT : (t_ / BN) * BPT;
        m.a_voff = (int)((TA ? (m.ap0 + (int64_t)m.ai0 * lda) : (m.ai0 + (int64_t)m.ap0 * lda)) * 8);
        m.b_voff = (int)((TB ? (m.bj0 + (int64_t)m.bp0 * ldb) : (m.bp0 + (int64_t)m.bj0 * ldb)) * 8);
        return m;
    };
    auto a_ip = [&](const SMap& M, int q, int* i, int* p) __attribute__((always_inline)) {
        if (TA) { *i = M.ai0; *p = M.ap0 + q; } else { *i = M.ai0 + LPT * q; *p = M.ap0; }
    };
    auto b_jp = [&](const SMap& M, int q, int* j, int* p) __attribute__((always_inline)) {
        if (TB) { *j = M.bj0 + LPT * q; *p = M.bp0; } else { *j = M.bj0; *p = M.bp0 + q; }
    };
    constexpr int a_qstep = TA ? 8 : 8 * LPT, b_qstep = TB ? 8 * LPT : 8;  // bytes per q
    const bool full_mn = (R == BM) && (Q == BN);
    const SMap M0 = smap(tid);  // register staging outside the direct kernels

    double rsum = 0.0;  // encode-pass value staged by threads tid < 4 BK
    auto load_global = [&](int kb, const SMap& M) __attribute__((always_inline)) {
        const int64_t k0 = (int64_t)kb * BK;
        const int kv = (int)min((int64_t)BK, K - k0);
        if constexpr (ABFT && PRE) {
            if (tid < 4 * BK) {
                const int p = tid >> 2, c = tid & 3;
                const double* src = c < 2 ? args.asp + ((int64_t)tm * K + k0 + p) * 2 + c
                                          : args.bsp + ((int64_t)tn * K + k0 + p) * 2 + (c - 2);
                rsum = p < kv ? *src : 0.0;
            }
        }  // valid steps in this block
        const __amdgpu_buffer_rsrc_t ra_ = make_rsrc(TA ? A + m0 * lda + k0 : A + m0 + k0 * lda);
        const __amdgpu_buffer_rsrc_t rb_ = make_rsrc(TB ? B + n0 + k0 * ldb : B + k0 + n0 * ldb);
        if (full_mn && kv == BK) {
#pragma unroll
            for (int q = 0; q < APT; ++q) ra[q] = buf_load_f64(ra_, M.a_voff + q * a_qstep, 0);
#pragma unroll
            for (int q = 0; q < BPT; ++q) rb[q] = buf_load_f64(rb_, M.b_voff + q * b_qstep, 0);
        } else {
#pragma unroll
            for (int q = 0; q < APT; ++q) {
                int i, p;
                a_ip(M, q, &i, &p);
                ra[q] = buf_load_f64(ra_, (i < R && p < kv) ? M.a_voff + q * a_qstep : kOOB, 0);
            }
#pragma unroll
            for (int q = 0; q < BPT; ++q) {
                int j, p;
                b_jp(M, q, &j, &p);
                rb[q] = buf_load_f64(rb_, (j < Q && p < kv) ? M.b_voff + q * b_qstep : kOOB, 0);
            }
        }
    };
    auto store_lds = [&](int st, const SMap& M) __attribute__((always_inline)) {
        if constexpr (ABFT && PRE) {
            if (tid < 4 * BK) sums[st][(tid & 3) >> 1][tid >> 2][tid & 1] = rsum;
        }
#pragma unroll
        for (int q = 0; q < APT; ++q) {
            int i, p;
            a_ip(M, q, &i, &p);
            As(st)[Cf::a_idx(i, p)] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            int j, p;
            b_jp(M, q, &j, &p);
            Bs(st)[Cf::b_idx(p, j)] = rb[q];
        }
    };
    // Direct staging of full k-block kb of an interior tile into stage st: each
    // active lane's 16-byte load lands in LDS at the wave load's base plus
    // 16 * lane, with no registers in between (the loads complete by the
    // barrier that publishes the stage).
    //   lines along the tile ([p][x], pitch X + 16): one wave load per 128
    //   elements of a step, all lanes active (64-element lines: one load per
    //   step with 32 lanes active);
    //   lines along k ([x][p], 9 slots per line): wave load I covers slots
    //   64 I .. 64 I + 63, lane l slot s = 64 I + l = line s / 9, step pair
    //   s % 9, the ninth (padding) slot of each line masked off.
    typedef __attribute__((address_space(3))) void* lds_ptr;
    auto direct_operand = [&]<bool KC, int X>(const double* base, int64_t ld, double* dst, int pitch)
        __attribute__((always_inline)) {
        const __amdgpu_buffer_rsrc_t r = make_rsrc(base);
        if constexpr (KC) {
            constexpr int NI = X * (BK / 2 + 1) / 64;  // wave loads per operand
            static_assert(X * (BK / 2 + 1) % 64 == 0, "whole wave loads");
#pragma unroll
            for (int q = 0; q < (NI + Cf::NW - 1) / Cf::NW; ++q) {
                const int I = wave + q * Cf::NW;
                if (I < NI) {
                    const int sl = 64 * I + lane;
                    const int x = sl / (BK / 2 + 1), pair = sl - x * (BK / 2 + 1);
                    if (pair < BK / 2)
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)(dst + 128 * I), 16,
                                                                 (int)(((int64_t)x * ld + 2 * pair) * 8), 0, 0, 0);
                }
            }
        } else if constexpr (X >= 128) {
            constexpr int PER = X / 128;  // wave loads per step
            constexpr int NL = BK * PER / Cf::NW;
            static_assert(BK * PER % Cf::NW == 0, "equal shares of wave loads");
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int L = wave * NL + q;
                const int p = L / PER, part = L % PER;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)(dst + p * pitch + part * 128), 16, lane * 16,
                                                         (int)(((int64_t)p * ld + part * 128) * 8), 0, 0);
            }
        } else {
            static_assert(X == 64 && BK % Cf::NW == 0, "64-element lines: one load per step");
            constexpr int NL = BK / Cf::NW;
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int p = wave * NL + q;
                if (lane < X / 2)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)(dst + p * pitch), 16, lane * 16,
                                                             (int)((int64_t)p * ld * 8), 0, 0);
            }
        }
    };
    auto direct_block = [&](int kb, int st) __attribute__((always_inline)) {
        const int64_t k0 = (int64_t)kb * BK;
        if constexpr (TA) direct_operand.template operator()<true, BM>(A + k0 + m0 * lda, lda, As(st), 0);
        else direct_operand.template operator()<false, BM>(A + m0 + k0 * lda, lda, As(st), Cf::SA);
        if constexpr (TB) direct_operand.template operator()<false, BN>(B + n0 + k0 * ldb, ldb, Bs(st), Cf::SB);
        else direct_operand.template operator()<true, BN>(B + k0 + n0 * ldb, ldb, Bs(st), 0);
        if constexpr (ABFT && PRE) {
            // encode-pass sums of the block's 16 steps: 16 lanes per operand
            if (wave == 0 && lane < BK) {
                __builtin_amdgcn_raw_ptr_buffer_load_lds(make_rsrc(args.asp + ((int64_t)tm * K + k0) * 2),
                                                         (lds_ptr)&sums[st][0][0][0], 16, lane * 16, 0, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(make_rsrc(args.bsp + ((int64_t)tn * K + k0) * 2),
                                                         (lds_ptr)&sums[st][1][0][0], 16, lane * 16, 0, 0, 0);
            }
        }
    };
    // full k-blocks, and whether this tile stages them directly
    const int full_kb = (int)(K / BK);
    static_assert(!DIR || (Cf::DIRECT && (!ABFT || PRE)), "direct staging configuration");
    const bool direct = DIR && full_mn;
    // stage block kb into st before any MFMA of the current block: directly, or
    // (edge tiles, the k tail) through registers whose live range ends here
    auto stage_now = [&](int kb, int st) __attribute__((always_inline)) {
        if (direct && kb < full_kb) {
            direct_block(kb, st);
        } else {
            // the staging map is rebuilt here from an opaque copy of the thread
            // id, so that none of it is hoisted into registers held across the
            // k loop (this path is rare: edge tiles and the k tail)
            int t_ = tid;
            asm volatile("" : "+v"(t_));
            const SMap M = smap(t_);
            load_global(kb, M);
            store_lds(st, M);
        }
    };
    // ---- a1: checksum row/column of the encoded operands for the staged k-block
    // Each wave owns PPW steps p of the block; LPP lanes per step sum the A
    // column and B row of that step, then reduce across the LPP lanes.  The
    // work is split in four slices so that the protected k loop can spread it
    // over the four rank-4 MFMA steps of the previous block (its LDS and
    // shuffle latency then hides under MFMA execution).
    struct EncAcc { double sa, saa, sb, sba; };
    auto encode_slice = [&](int st, int slice, EncAcc& e) __attribute__((always_inline)) {
        const int p = wave * Cf::PPW + lane / Cf::LPP;
        const int sub = lane % Cf::LPP;
        constexpr int UA = BM / Cf::LPP, UB = BN / Cf::LPP;
        if (slice == 0) {
            e.sa = e.saa = e.sb = e.sba = 0.0;
#pragma unroll
            for (int u = 0; u < UA / 2; ++u) {
                const double v = As(st)[Cf::a_idx(sub + u * Cf::LPP, p)];
                e.sa += v;
                e.saa += fabs(v);
            }
        } else if (slice == 1) {
#pragma unroll
            for (int u = UA / 2; u < UA; ++u) {
                const double v = As(st)[Cf::a_idx(sub + u * Cf::LPP, p)];
                e.sa += v;
                e.saa += fabs(v);
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const double v = Bs(st)[Cf::b_idx(p, sub + u * Cf::LPP)];
                e.sb += v;
                e.sba += fabs(v);
            }
        } else if (slice == 2) {
            e.sa = group_sum<Cf::LPP>(e.sa);
            e.saa = group_sum<Cf::LPP>(e.saa);
        } else {
            e.sb = group_sum<Cf::LPP>(e.sb);
            e.sba = group_sum<Cf::LPP>(e.sba);
            if (sub == 0) {
                sums[st][0][p][0] = e.sa;
                sums[st][0][p][1] = e.saa;
                sums[st][1][p][0] = e.sb;
                sums[st][1][p][1] = e.sba;
            }
        }
    };
    auto encode = [&](int st) __attribute__((always_inline)) {
        EncAcc e;
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) encode_slice(st, sl, e);
    };
    // ---- a2 + a3: one k-block of MFMA with the checksum updates.  Fragments of
    // the next rank-4 step are read from LDS while the current step's MFMAs run;
    // the scheduling fence keeps the compiler from hoisting further reads.
    // WRc, WCc: this wave's position, as compile-time constants so that its
    // share of the checksum updates is fixed at compile time (no selects), or
    // -1: one copy of the loop for all waves (its loop-invariant addresses do
    // not multiply), which reads the step's sums and its share's fragments
    // from LDS where the checksum updates use them (fewer live registers).
    auto mfma_block = [&]<int WRc, int WCc, bool ENC>(int st) __attribute__((always_inline)) {
        EncAcc enc;
        constexpr int NS = BK / 4;
        double a[2][FM], b[2][FN], sm[2][4];
        // the layouts are linear in both indices: one per-lane base per operand
        // and compile-time offsets for the fragment (g, h) and step s_
        const double* abase = As(st) + Cf::a_idx(wm0 + l16, lq);
        const double* bbase = Bs(st) + Cf::b_idx(lq, wn0 + l16);
        auto load_frag = [&](int s_, int buf) __attribute__((always_inline)) {
            const int p = 4 * s_ + lq;
#pragma unroll
            for (int g = 0; g < FM; ++g) a[buf][g] = abase[Cf::a_idx(16 * g, 4 * s_)];
#pragma unroll
            for (int h = 0; h < FN; ++h) b[buf][h] = bbase[Cf::b_idx(4 * s_, 16 * h)];
            if (ABFT && WRc >= 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) sm[buf][c] = sums[st][c >> 1][p][c & 1];
            }
        };
        // one-copy loop (run at four waves per SIMD): each step's fragments are
        // read at its start, the other waves' MFMAs cover the LDS latency;
        // otherwise the next step's fragments are read during this step's MFMAs
        constexpr bool JIT = WRc < 0;
        if (!JIT) load_frag(0, 0);
#pragma unroll
        for (int s_ = 0; s_ < NS; ++s_) {
            const int cur = JIT ? 0 : (s_ & 1);
            if (JIT) load_frag(s_, 0);
            else if (s_ + 1 < NS) load_frag(s_ + 1, cur ^ 1);
#pragma unroll
            for (int g = 0; g < FM; ++g)
#pragma unroll
                for (int h = 0; h < FN; ++h)
                    acc[g][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][g], b[cur][h], acc[g][h], 0, 0, 0);
            if (ABFT) {
                // this wave's share of the rows (columns) that the waves of its
                // wave-row (wave-column) have in common
                if constexpr (WRc < 0) {
                    const double* sp = &sums[st][0][lq][0] + 8 * s_;  // step 4 s_ + lq
                    const double as_ = sp[0], asa = sp[1];
                    const double bs_ = sp[2 * BK], bsa = sp[2 * BK + 1];
#pragma unroll
                    for (int q = 0; q < Cf::GSH; ++q) {
                        const double x = abase[Cf::a_idx(16 * (q * WGN + wc), 4 * s_)];
                        er[q] = fma(x, bs_, er[q]);
                        mr[q] = fma(fabs(x), bsa, mr[q]);
                    }
#pragma unroll
                    for (int q = 0; q < Cf::HSH; ++q) {
                        const double y = bbase[Cf::b_idx(4 * s_, 16 * (q * WGM + wr))];
                        ec[q] = fma(as_, y, ec[q]);
                        mc[q] = fma(asa, fabs(y), mc[q]);
                    }
                    // keep the updates in this step (sinking them out of the
                    // k-block would hold every step's operands live)
#pragma unroll
                    for (int q = 0; q < Cf::GSH; ++q) asm volatile("" : "+v"(er[q]), "+v"(mr[q]));
#pragma unroll
                    for (int q = 0; q < Cf::HSH; ++q) asm volatile("" : "+v"(ec[q]), "+v"(mc[q]));
                } else {
                    const double as_ = sm[cur][0], asa = sm[cur][1], bs_ = sm[cur][2], bsa = sm[cur][3];
#pragma unroll
                    for (int g = 0; g < FM; ++g)
                        if (g % WGN == WCc) {
                            er[g / WGN] = fma(a[cur][g], bs_, er[g / WGN]);
                            mr[g / WGN] = fma(fabs(a[cur][g]), bsa, mr[g / WGN]);
                        }
#pragma unroll
                    for (int h = 0; h < FN; ++h)
                        if (h % WGM == WRc) {
                            ec[h / WGM] = fma(as_, b[cur][h], ec[h / WGM]);
                            mc[h / WGM] = fma(asa, fabs(b[cur][h]), mc[h / WGM]);
                        }
                }
            }
            if (ENC) encode_slice(st ^ 1, s_, enc);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // ---- element access by a uniform tile position (rare paths only): a sweep of
    // selects over the accumulators keeps the code compact and free of
    // dynamically indexed register arrays.
    auto elem_index = [&](int row, int col) __attribute__((always_inline)) {
        const int rr = row % WM, cc = col % WN;
        return ((rr / 16) * FN + cc / 16) * 4 + (rr % 16) / 4;  // (g, h, r) flattened
    };
    auto owner_of = [&](int row, int col) __attribute__((always_inline)) {
        const int rr = row % WM, cc = col % WN;
        return (row / WM == wr) && (col / WN == wc) && lane == ((rr % 16) % 4) * 16 + (cc % 16);
    };
    auto get_elem = [&](int idx) __attribute__((always_inline)) {
        double v = 0.0;
#pragma unroll
        for (int g = 0; g < FM; ++g)
#pragma unroll
            for (int h = 0; h < FN; ++h)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if ((g * FN + h) * 4 + r == idx) v = acc[g][h][r];  // idx is uniform
        return v;
    };
    auto set_elem = [&](int idx, double v, bool own) __attribute__((always_inline)) {
#pragma unroll
        for (int g = 0; g < FM; ++g)
#pragma unroll
            for (int h = 0; h < FN; ++h)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if ((g * FN + h) * 4 + r == idx) acc[g][h][r] = own ? v : acc[g][h][r];
    };

    // ---- a9: apply a planned flip to the value it targets (owner lane only)
    auto apply_fault = [&](const Fault& f, int t) __attribute__((always_inline)) {
        double oldv = 0.0, newv = 0.0;
        bool own;
        const bool ck = args.inj.target == FTG_TARGET_CHECKSUM;
        if (ck) {
            const int g = (f.row % WM) / 16;
            own = (f.row / WM == wr) && (g % WGN == wc) && lane == (f.row % 16);
#pragma unroll
            for (int q = 0; q < Cf::GSH; ++q)
                if (q == g / WGN) {
                    oldv = er[q];
                    newv = flip_f64(oldv, f.bit);
                    er[q] = own ? newv : er[q];
                }
        } else {
            own = owner_of(f.row, f.col);
            const int idx = __builtin_amdgcn_readfirstlane(elem_index(f.row, f.col));
            // a uniform test per element (no select chains over all accumulators)
#pragma unroll
            for (int g = 0; g < FM; ++g)
#pragma unroll
                for (int h = 0; h < FN; ++h)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if ((g * FN + h) * 4 + r == idx) {
                            oldv = acc[g][h][r];
                            newv = flip_f64(oldv, f.bit);
                            if (own) acc[g][h][r] = newv;
                        }
        }
        if (own)
            push_inject(args.rep, args.problem, tm, tn, t, m0 + f.row, ck ? -1 : n0 + f.col, f.pflip,
                        f.bit, ck ? FTG_TARGET_CHECKSUM : FTG_TARGET_ACC, oldv, newv);
    };

    // ---- a4 + a5 + a6: reductions and flags; results in Vp->nfr / Vp->nfc (and the
    // first flagged row/column with its delta and tau).  On a final check acc
    // holds C_out and the C_in sums are in Vp->
    auto reduce_and_flag = [&](bool final, int64_t pend) __attribute__((always_inline)) {
        // (on the final check the row and column sums of C_out were taken by
        // finalize_output in the same pass that formed C_out)
        if (!final) {
#pragma unroll
        for (int g = 0; g < FM; ++g) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double s = 0.0;
#pragma unroll
                for (int h = 0; h < FN; ++h) s += acc[g][h][r];
                s = group_sum<16>(s);
                if (l16 == 0) Vp->rsum[wc][wm0 + 16 * g + 4 * r + lq] = s;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int h = 0; h < FN; ++h) {
            double s = 0.0;
#pragma unroll
            for (int g = 0; g < FM; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) s += acc[g][h][r];
            s = quarter_sum(s);
            if (lq == 0) Vp->csum[wr][wn0 + 16 * h + l16] = s;
        }
        }
        // maintained checksums: complete after summing the four p lanes
#pragma unroll
        for (int q = 0; q < Cf::GSH; ++q) {
            const double e = quarter_sum(er[q]), mm = quarter_sum(mr[q]);
            if (lq == 0) {
                const int row = wm0 + 16 * (q * WGN + wc) + l16;
                Vp->er[row] = e;
                Vp->mr[row] = mm;
            }
        }
#pragma unroll
        for (int q = 0; q < Cf::HSH; ++q) {
            const double e = quarter_sum(ec[q]), mm = quarter_sum(mc[q]);
            if (lq == 0) {
                const int col = wn0 + 16 * (q * WGM + wr) + l16;
                Vp->ec[col] = e;
                Vp->mc[col] = mm;
            }
        }
        if (tid == 0) { Vp->nfr = 0; Vp->nfc = 0; }
        __syncthreads();
        const bool cin = final && args.beta != 0.0;
        double pass_ratio = 0.0;
        for (int line = tid; line < BM + BN; line += NT) {
            const bool isrow = line < BM;
            const int x = isrow ? line : line - BM;
            if (x >= (isrow ? R : Q)) continue;
            double ref = 0.0, ci = 0.0, cia = 0.0;
            if (isrow) {
#pragma unroll
                for (int w = 0; w < WGN; ++w) {
                    ref += Vp->rsum[w][x];
                    if (cin) { ci += Vp->cir[w][x]; cia += Vp->cira[w][x]; }
                }
            } else {
#pragma unroll
                for (int w = 0; w < WGM; ++w) {
                    ref += Vp->csum[w][x];
                    if (cin) { ci += Vp->cic[w][x]; cia += Vp->cica[w][x]; }
                }
            }
            double ex = isrow ? Vp->er[x] : Vp->ec[x];
            double mag = isrow ? Vp->mr[x] : Vp->mc[x];
            if (final) {
                ex = args.alpha * ex;
                mag = fabs(args.alpha) * mag;
                if (cin) { ex += args.beta * ci; mag += fabs(args.beta) * cia; }
            }
            const double d = ref - ex;
            const double tau = tau_of(0, 0.0, pend + (isrow ? Q : R) + 8, mag);
            if (flagged(d, tau)) {
                if (isrow) {
                    if (atomicAdd(&Vp->nfr, 1) == 0) { Vp->fi = x; Vp->dfi = d; Vp->tfi = tau; }
                } else {
                    if (atomicAdd(&Vp->nfc, 1) == 0) { Vp->fj = x; Vp->dfj = d; Vp->tfj = tau; }
                }
            } else if (tau > 0.0) {
                pass_ratio = fmax(pass_ratio, fabs(d) / tau);
            }
        }
        note_pass_ratio(args.rep, pass_ratio);
        __syncthreads();
    };

    // fresh dot product of tile row fi and column fj over steps [0, pend), by wave 0
    auto fresh_dot = [&](int fi, int fj, int64_t pend) __attribute__((always_inline)) {
        if (wave == 0) {
            const int64_t gi = m0 + fi, gj = n0 + fj;
            double s = 0.0;
            for (int64_t p = lane; p < pend; p += 64) {
                const double a = TA ? A[p + gi * lda] : A[gi + p * lda];
                const double b = TB ? B[gj + p * ldb] : B[p + gj * ldb];
                s = fma(a, b, s);
            }
            s = group_sum<64>(s);
            if (lane == 0) Vp->dotv = s;
        }
        __syncthreads();
        return Vp->dotv;
    };

    // ---- a7: verification of one slot (a small state machine around one
    // reduce-and-flag pass): check -> subtract (§6.3) -> recompute -> give up.
    // Returns true when the tile must be recomputed (uncorrectable, policy 1).
    const int64_t ldc = args.ldc;
    // a tile is recomputed at most once: with non-finite inputs the checks can
    // never pass, and the second attempt is reported instead of repeated
    int redo_budget = 1;
    auto verify = [&](bool final, int64_t pend, int t) __attribute__((always_inline)) -> bool {
        int stage = 0;  // 0 first check, 1 after subtract, 2 after recompute
        int fi = 0, fj = 0, idx = 0;
        bool own = false;
        double dfi = 0.0, tfi = 0.0, xold = 0.0;
        for (;;) {
            reduce_and_flag(final, pend);
            const int nr = __builtin_amdgcn_readfirstlane(Vp->nfr);
            const int nc = __builtin_amdgcn_readfirstlane(Vp->nfc);
            int kind = 0;  // outcome to record; 0 = try the recompute next
            if (stage == 0) {
                if (nr == 0 && nc == 0) return false;
                if (tid == 0) atomicAdd(&args.rep->cnt[kDetected], 1ull);
                if (nr == 1 && nc == 1) {
                    fi = __builtin_amdgcn_readfirstlane(Vp->fi);
                    fj = __builtin_amdgcn_readfirstlane(Vp->fj);
                    dfi = Vp->dfi;
                    tfi = Vp->tfi;
                    own = owner_of(fi, fj);
                    idx = __builtin_amdgcn_readfirstlane(elem_index(fi, fj));
                    const double x = get_elem(idx);
                    __syncthreads();
                    if (own) { Vp->xold = x; Vp->xfinite = isfinite(x) ? 1 : 0; }
                    __syncthreads();
                    xold = Vp->xold;
                    stage = 1;
                    if (args.correct_policy == 0 && isfinite(dfi) &&
                        __builtin_amdgcn_readfirstlane(Vp->xfinite) && !absorbed(false, xold, tfi, Q)) {
                        set_elem(idx, xold - dfi, own);  // subtract the error (§6.3)
                        continue;
                    }
                } else if (nr + nc == 1) {
                    // one direction only: the maintained checksum is the faulty value;
                    // re-base it on the data for the following intervals
                    const int fr = __builtin_amdgcn_readfirstlane(Vp->fi);
                    const int fc = __builtin_amdgcn_readfirstlane(Vp->fj);
                    if (!final) {
                        // The line's checksum is the sum of its four lanes'
                        // partials; the first of them is set so that the sum
                        // is the line's reference sum (adding the mismatch
                        // instead would lose the checksum's own value after a
                        // flip to a huge value).  Both arrays are updated by
                        // value selects: conditional updates of either array
                        // were merged by the compiler into one through a
                        // selected pointer, which moved er and ec to scratch
                        // for the whole k loop.
                        const int g = (fr % WM) / 16, h = (fc % WN) / 16;
                        double rref = 0.0, cref = 0.0;
                        if (nr) {
#pragma unroll
                            for (int w = 0; w < WGN; ++w) rref += Vp->rsum[w][fr];
                        } else {
#pragma unroll
                            for (int w = 0; w < WGM; ++w) cref += Vp->csum[w][fc];
                        }
                        const bool rown = nr && fr / WM == wr && g % WGN == wc && lane == fr % 16;
                        const bool cown = !nr && fc / WN == wc && h % WGM == wr && lane == fc % 16;
#pragma unroll
                        for (int q = 0; q < Cf::GSH; ++q) {
                            const double others = quarter_sum(lq == 0 ? 0.0 : er[q]);
                            er[q] = (rown && q == g / WGN) ? rref - others : er[q];
                        }
#pragma unroll
                        for (int q = 0; q < Cf::HSH; ++q) {
                            const double others = quarter_sum(lq == 0 ? 0.0 : ec[q]);
                            ec[q] = (cown && q == h / WGM) ? cref - others : ec[q];
                        }
                    }
                    if (tid == 0) {
                        atomicAdd(&args.rep->cnt[kChecksumOnly], 1ull);
                        push_record(args.rep, args.problem, tm, tn, t, nr ? m0 + fr : -1,
                                    nr ? -1 : n0 + fc, FTG_KIND_CHECKSUM_ONLY, nr ? Vp->dfi : Vp->dfj,
                                    nr ? Vp->tfi : Vp->tfj);
                    }
                    __syncthreads();
                    return false;
                } else {
                    kind = FTG_KIND_UNCORRECTABLE;
                }
            } else if (nr == 0 && nc == 0) {
                kind = stage == 1 ? FTG_KIND_SUBTRACT : FTG_KIND_RECOMPUTE;
            } else {
                set_elem(idx, xold, own);  // undo the attempt
                if (stage == 2) kind = FTG_KIND_UNCORRECTABLE;
            }
            if (kind == 0) {
                // recompute the located element from a fresh dot product
                const double dot = fresh_dot(fi, fj, pend);
                double v = dot;
                if (final) {
                    v = args.alpha * dot;
                    if (args.beta != 0.0) v += args.beta * args.C[(m0 + fi) + (n0 + fj) * ldc];
                }
                set_elem(idx, v, own);
                stage = 2;
                continue;
            }
            bool redo = false;
            if (kind == FTG_KIND_UNCORRECTABLE && args.uncorrectable_policy == 1 && redo_budget > 0) {
                redo = true;
                kind = FTG_KIND_TILE_RECOMPUTED;
            }
            if (tid == 0) {
                if (kind == FTG_KIND_SUBTRACT) atomicAdd(&args.rep->cnt[kCorrSub], 1ull);
                if (kind == FTG_KIND_RECOMPUTE) atomicAdd(&args.rep->cnt[kCorrRecomp], 1ull);
                if (kind >= FTG_KIND_UNCORRECTABLE) atomicAdd(&args.rep->cnt[kUncorrectable], 1ull);
                if (kind == FTG_KIND_TILE_RECOMPUTED) atomicAdd(&args.rep->cnt[kTilesRecomputed], 1ull);
                const bool loc = kind == FTG_KIND_SUBTRACT || kind == FTG_KIND_RECOMPUTE;
                const double d = (stage > 0) ? dfi : (nr ? Vp->dfi : Vp->dfj);
                const double tt = (stage > 0) ? tfi : (nr ? Vp->tfi : Vp->tfj);
                push_record(args.rep, args.problem, tm, tn, t, loc ? m0 + fi : -1, loc ? n0 + fj : -1,
                            kind, d, tt);
            }
            __syncthreads();
            return redo;
        }
    };

    // ---- a4: C_out = alpha acc + beta C_in in registers, C_in sums to LDS.
    // Lane (lq, l16) holds rows wm0 + 16g + 4r + lq, columns wn0 + 16h + l16.
    // element (g, h, r): row bytes (16g + 4r)*8 < 4096 ride in the instruction's
    // immediate offset; the column step 16*h*ldc*8 is one uniform offset per h.
    const int c_voff = (int)((wm0 + lq + (int64_t)(wn0 + l16) * ldc) * 8);
    const int c_hstep = (int)(16 * ldc * 8);
    auto c_vo = [&](int g, int r, bool ok) __attribute__((always_inline)) {
        return ok ? c_voff + (16 * g + 4 * r) * 8 : kOOB;
    };
    auto c_ok = [&](int g, int h, int r) __attribute__((always_inline)) {
        return full_mn || ((wm0 + 16 * g + 4 * r + lq < R) && (wn0 + 16 * h + l16 < Q));
    };
    // C_out = alpha acc + beta C_in, and with ABFT the row and column sums of
    // C_in (a4) and of C_out (a5) into LDS.  Two passes, each with few values
    // live beside the accumulators: the C_in sums, then C_out with its sums
    // (the second pass re-reads C_in, from L2).  The C_in offset goes through
    // an opaque copy made here, so that the loads are issued after the k loop
    // (hoisted above it, their values would be held in scratch across the
    // whole loop); two rows of each fragment (2 FN values) load at a time.
    auto finalize_output = [&]() __attribute__((always_inline)) {
        const bool cin = args.beta != 0.0;
        int cvo = c_voff;
        asm volatile("" : "+v"(cvo));
        const __amdgpu_buffer_rsrc_t rc = make_rsrc(args.C + m0 + n0 * ldc);
        auto load_c = [&](double (&c)[2][FN], int g, int r0) __attribute__((always_inline)) {
#pragma unroll
            for (int rr = 0; rr < 2; ++rr)
#pragma unroll
                for (int h = 0; h < FN; ++h)
                    c[rr][h] = buf_load_f64(rc, c_ok(g, h, r0 + rr) ? cvo + (16 * g + 4 * (r0 + rr)) * 8 : kOOB,
                                            h * c_hstep);
        };
        // with the register file to itself, the workgroup requests the whole
        // of its C_in at once and keeps it for both passes
        double call[WIDE_REGS ? 2 * FM : 1][2][FN];
        if constexpr (WIDE_REGS) {
            if (cin) {
#pragma unroll
                for (int gr = 0; gr < 2 * FM; ++gr) load_c(call[gr], gr / 2, 2 * (gr % 2));
            }
        }
        if (ABFT && cin) {
            double cs[FN], csa[FN];
#pragma unroll
            for (int h = 0; h < FN; ++h) cs[h] = csa[h] = 0.0;
#pragma unroll
            for (int gr = 0; gr < 2 * FM; ++gr) {
                const int g = gr / 2, r0 = 2 * (gr % 2);
                double c[2][FN];
                if constexpr (WIDE_REGS) {
#pragma unroll
                    for (int rr = 0; rr < 2; ++rr)
#pragma unroll
                        for (int h = 0; h < FN; ++h) c[rr][h] = call[gr][rr][h];
                } else {
                    load_c(c, g, r0);
                }
#pragma unroll
                for (int rr = 0; rr < 2; ++rr) {
                    double s = 0.0, sa = 0.0;
#pragma unroll
                    for (int h = 0; h < FN; ++h) {
                        s += c[rr][h];
                        sa += fabs(c[rr][h]);
                        cs[h] += c[rr][h];
                        csa[h] += fabs(c[rr][h]);
                    }
                    s = group_sum<16>(s);
                    sa = group_sum<16>(sa);
                    if (l16 == 0) {
                        const int row = wm0 + 16 * g + 4 * (r0 + rr) + lq;
                        Vp->cir[wc][row] = s;
                        Vp->cira[wc][row] = sa;
                    }
                }
                // (one batch of C_in values at a time, unless the register
                // file is the workgroup's alone: then the loads run ahead)
                if constexpr (!WIDE_REGS) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int h = 0; h < FN; ++h) {
                const double s = quarter_sum(cs[h]), sa = quarter_sum(csa[h]);
                if (lq == 0) { Vp->cic[wr][wn0 + 16 * h + l16] = s; Vp->cica[wr][wn0 + 16 * h + l16] = sa; }
            }
        }
        double os[FN];
#pragma unroll
        for (int h = 0; h < FN; ++h) os[h] = 0.0;
#pragma unroll
        for (int gr = 0; gr < 2 * FM; ++gr) {
            const int g = gr / 2, r0 = 2 * (gr % 2);
            double c[2][FN];
            if constexpr (WIDE_REGS) {
#pragma unroll
                for (int rr = 0; rr < 2; ++rr)
#pragma unroll
                    for (int h = 0; h < FN; ++h) c[rr][h] = call[gr][rr][h];
            } else {
                if (cin) load_c(c, g, r0);
            }
#pragma unroll
            for (int rr = 0; rr < 2; ++rr) {
                const int r = r0 + rr;
                double o = 0.0;
#pragma unroll
                for (int h = 0; h < FN; ++h) {
                    const double v = cin ? args.alpha * acc[g][h][r] + args.beta * c[rr][h] : args.alpha * acc[g][h][r];
                    acc[g][h][r] = v;
                    o += v;
                    os[h] += v;
                }
                if (ABFT) {
                    o = group_sum<16>(o);
                    if (l16 == 0) Vp->rsum[wc][wm0 + 16 * g + 4 * r + lq] = o;
                }
            }
            if constexpr (!WIDE_REGS) __builtin_amdgcn_sched_barrier(0);
        }
        if (ABFT) {
#pragma unroll
            for (int h = 0; h < FN; ++h) {
                const double o = quarter_sum(os[h]);
                if (lq == 0) Vp->csum[wr][wn0 + 16 * h + l16] = o;
            }
        }
    };

    // ------------------------------------------------------------------ main loop
    // a9: the tile's injection plan, one thread per interval, kept in LDS so the
    // k loop only reads a few uniform values at interval starts.
    const bool inj = ABFT && args.inj.on;
    int inj_from = 0;  // intervals below this one replay fault-free after a recompute
    if (inj) {
        const uint64_t tile_id = (uint64_t)tn * args.tiles_m + tm;
        for (int tt = tid; tt < n_int; tt += NT) {
            const int64_t plo = (int64_t)tt * kc, phi = min(K, plo + kc);
            Fault f2[2];
            const int nf = slot_faults(args.inj, tile_id * n_int + tt, R, Q, plo, phi, f2);
            fltn[tt] = nf;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                flt[tt][q][0] = f2[q].row;
                flt[tt][q][1] = f2[q].col;
                flt[tt][q][2] = (int)f2[q].pflip;
                flt[tt][q][3] = f2[q].bit;
            }
        }
        __syncthreads();
    }
    // fault q of interval tt that lands after k-block kb (read from LDS when needed)
    auto fault_kb = [&](int tt, int q) __attribute__((always_inline)) {
        if (!inj || tt < inj_from || q >= fltn[tt]) return -1;
        return flt[tt][q][2] / BK;
    };
    auto load_fault = [&](int tt, int q) __attribute__((always_inline)) {
        Fault f;
        f.row = __builtin_amdgcn_readfirstlane(flt[tt][q][0]);
        f.col = __builtin_amdgcn_readfirstlane(flt[tt][q][1]);
        f.pflip = __builtin_amdgcn_readfirstlane(flt[tt][q][2]);
        f.bit = __builtin_amdgcn_readfirstlane(flt[tt][q][3]);
        return f;
    };

    // One pass of the k loop, repeated only when a slot turned out
    // uncorrectable and the policy asks for the tile to be recomputed.  The k
    // loop runs in segments that end where something has to happen to the
    // accumulators (a planned flip, an interval check), so the hot loop body
    // holds nothing but staging, encode and MFMA work.
    const int kb_per_int = (int)(kc / BK);
    int t = 0;
    for (;;) {
        zero_state();
        t = 0;
        if constexpr (DIR) stage_now(0, 0);
        else {
            load_global(0, M0);
            store_lds(0, M0);
        }
        __syncthreads();
        if (ABFT && !PRE) {
            encode(0);
            if (nkb > 1) load_global(1, M0);
            __syncthreads();
        }
        bool restart = false;
        int kb = 0;
        while (kb < nkb) {
            // end of this segment: the interval end or the next planned flip
            int seg = IVL ? min(nkb, (t + 1) * kb_per_int) : nkb;
            if (inj) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int fkb = __builtin_amdgcn_readfirstlane(fault_kb(t, q));
                    if (fkb >= kb && fkb + 1 < seg) seg = fkb + 1;
                }
            }
            // the hot loop, instantiated per wave position (uniform dispatch), or
            // once for all waves (W = -1) with direct staging
            auto hot = [&]<int W>() __attribute__((always_inline)) {
                constexpr int WR = W < 0 ? -1 : W / WGN, WC = W < 0 ? -1 : W % WGN;
                for (; kb < seg; ++kb) {
                    const int st = kb & 1;
                    if (DIR) {
                        if (kb + 1 < nkb) stage_now(kb + 1, st ^ 1);
                        mfma_block.template operator()<WR, WC, false>(st);
                        if (kb + 1 < nkb) __syncthreads();
                    } else if (!ABFT || PRE) {
                        // (with the encode pass, the checksum updates need no
                        // extra barrier: the sums travel with the operands)
                        if (kb + 1 < nkb) load_global(kb + 1, M0);
                        mfma_block.template operator()<WR, WC, false>(st);
                        if (kb + 1 < nkb) {
                            store_lds(st ^ 1, M0);
                            __syncthreads();
                        }
                    } else if (kb + 1 < nkb) {
                        // block kb+1: staged now, encoded while block kb's MFMAs run
                        store_lds(st ^ 1, M0);
                        __syncthreads();
                        if (kb + 2 < nkb) load_global(kb + 2, M0);
                        mfma_block.template operator()<WR, WC, true>(st);
                        __syncthreads();
                    } else {
                        mfma_block.template operator()<WR, WC, false>(st);
                    }
                }
            };
            if constexpr ((Cf::ONE_COPY && ABFT) || DIR) {
                hot.template operator()<-1>();
            } else {
                [&]<int... W>(std::integer_sequence<int, W...>) __attribute__((always_inline)) {
                    ((wave == W ? (hot.template operator()<W>(), 0) : 0), ...);
                }(std::make_integer_sequence<int, WGM * WGN>{});
            }
            if (!ABFT) continue;
            // accumulators now hold the sum over steps [0, kb * BK)
            if (inj) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    if (__builtin_amdgcn_readfirstlane(fault_kb(t, q)) == kb - 1)
                        apply_fault(load_fault(t, q), t);
            }
            if (IVL && kb < nkb && kb % kb_per_int == 0) {
                // a10: online verification of the accumulators at the interval end.
                // Stage kb & 1 holds block kb; the other stage is free.
                Vp = reinterpret_cast<VL*>(&stg[(kb - 1) & 1][0]);
                if (verify(false, (int64_t)kb * BK, t)) {
                    --redo_budget;
                    inj_from = t + 1;  // replay intervals 0..t fault-free
                    restart = true;
                    break;
                }
                ++t;
                __syncthreads();  // every read of the bookkeeping ends before the stage is refilled
            }
        }
        if (restart) { __syncthreads(); continue; }
        if (ABFT) {
            // the last block's fragment reads end before the bookkeeping reuses stage 0
            Vp = reinterpret_cast<VL*>(&stg[0][0]);
            __syncthreads();
        }
        finalize_output();
        if (!ABFT) break;
        // a5-a7 on the output: flags in registers; a located element is repaired
        // after the store, from global memory
        __syncthreads();
        reduce_and_flag(true, K);
        const int nr = __builtin_amdgcn_readfirstlane(Vp->nfr);
        const int nc = __builtin_amdgcn_readfirstlane(Vp->nfc);
        if (nr == 0 && nc == 0) break;
        const bool many = nr > 1 || nc > 1;
        if (many && args.uncorrectable_policy == 1 && redo_budget > 0) {
            // more than one error in the final slot: recompute the tile, no injection
            auto count_recomputed = [&]() {
                atomicAdd(&args.rep->cnt[kDetected], 1ull);
                atomicAdd(&args.rep->cnt[kUncorrectable], 1ull);
                atomicAdd(&args.rep->cnt[kTilesRecomputed], 1ull);
                push_record(args.rep, args.problem, tm, tn, t, -1, -1, FTG_KIND_TILE_RECOMPUTED,
                            nr ? Vp->dfi : Vp->dfj, nr ? Vp->tfi : Vp->tfj);
            };
            if constexpr (IVL) {
                if (tid == 0) count_recomputed();
                __syncthreads();
                --redo_budget;
                inj_from = n_int;
                continue;
            } else {
                // Without intervals the tile is recomputed by the repair kernel,
                // from the operands and C_in, which stays in place: the tile is
                // not stored.  (A restart here would make the k loop a loop body
                // whose invariants stay live through this epilogue.)
                if (tid == 0) {
                    RepairReq q;
                    q.problem = args.problem; q.tm = tm; q.tn = tn; q.interval = t;
                    q.nr = nr; q.nc = nc; q.fi = q.fj = 0; q.R = R; q.Q = Q;
                    q.whole = 1; q.pad1 = 0; q.m0 = m0; q.n0 = n0;
                    q.dfi = nr ? Vp->dfi : 0.0; q.tfi = nr ? Vp->tfi : 0.0;
                    q.dfj = nc ? Vp->dfj : 0.0; q.tfj = nc ? Vp->tfj : 0.0;
                    q.exp_row = q.exp_col = q.cin = 0.0;
                    // counted as recomputed only once the repair kernel will see it
                    if (push_repair(args.rep, q)) count_recomputed();
                }
                __syncthreads();
                return;
            }
        }
        // hand the slot to the repair kernel (it runs after this kernel on the
        // same stream and works on the stored tile in global memory)
        if (tid == 0) {
            RepairReq q;
            q.problem = args.problem; q.tm = tm; q.tn = tn; q.interval = t;
            q.nr = nr; q.nc = nc; q.fi = Vp->fi; q.fj = Vp->fj; q.R = R; q.Q = Q;
            q.whole = q.pad1 = 0; q.m0 = m0; q.n0 = n0;
            q.dfi = Vp->dfi; q.tfi = Vp->tfi; q.dfj = Vp->dfj; q.tfj = Vp->tfj;
            const bool cin = args.beta != 0.0;
            double cr = 0.0, cc = 0.0;
            q.exp_row = q.exp_col = 0.0;
            if (nr) {
#pragma unroll
                for (int w = 0; w < WGN; ++w) cr += Vp->cir[w][Vp->fi];
                q.exp_row = args.alpha * Vp->er[Vp->fi] + (cin ? args.beta * cr : 0.0);
            }
            if (nc) {
#pragma unroll
                for (int w = 0; w < WGM; ++w) cc += Vp->cic[w][Vp->fj];
                q.exp_col = args.alpha * Vp->ec[Vp->fj] + (cin ? args.beta * cc : 0.0);
            }
            q.cin = (cin && nr == 1 && nc == 1) ? args.C[(m0 + Vp->fi) + (n0 + Vp->fj) * ldc] : 0.0;
            push_repair(args.rep, q);
        }
        // C_in at the located element is read above before any wave stores
        // its part of the tile over it
        __syncthreads();
        break;
    }

    // ---- a8: store the tile
    {
        const __amdgpu_buffer_rsrc_t rc = make_rsrc(args.C + m0 + n0 * ldc);
#pragma unroll
        for (int g = 0; g < FM; ++g)
#pragma unroll
            for (int h = 0; h < FN; ++h)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    buf_store_f64(acc[g][h][r], rc, c_vo(g, r, c_ok(g, h, r)), h * c_hstep);
    }
}

// Occupancy target of a kernel (the second launch bound: waves per SIMD the
// register allocation must allow).  Kernels with one copy of the k loop
// (direct staging, or protected small tiles) whose accumulators take at most 64
// registers per lane aim at two workgroups per CU, at most 32 at three (their
// LDS fits that many times in 160 KB); the others use the configuration's MINB.
// MINB = 0 asks for one workgroup per CU: the whole register file per lane,
// for calls whose epilogue outweighs the k loop.
template <int BM, int BN, int WGM, int WGN, int MINB, bool DIR, bool ABFT>
constexpr int waves_per_simd()
{
    constexpr int NW = WGM * WGN;
    if constexpr (MINB == 0) return NW / 4;
    constexpr int accv = 2 * BM * BN / (NW * 64);  // accumulator VGPRs per lane
    constexpr bool one = DIR || (ABFT && DCfg<BM, BN, WGM, WGN, false, false>::ONE_COPY);
    constexpr int blocks = !one ? 0 : (accv <= 32 ? 3 : (accv <= 64 ? 2 : 0));
    return (blocks && (blocks * NW) % 4 == 0) ? blocks * NW / 4 : MINB;
}

// One problem, one workgroup per output tile.
template <int BM, int BN, int WGM, int WGN, bool TA, bool TB, bool ABFT, bool IVL, int MINB, bool PRE, bool DIR>
__global__ __launch_bounds__(WGM* WGN * 64, (waves_per_simd<BM, BN, WGM, WGN, MINB, DIR, ABFT>())) void dgemm_abft_kernel(
    DGemmArgs args)
{
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, args.tiles_m, args.tiles_n, 4, &tm, &tn);
    dgemm_tile<BM, BN, WGM, WGN, TA, TB, ABFT, IVL, PRE, DIR, MINB == 0>(args, tm, tn);
}

// Many problems in one persistent launch.  Work item w is tile
// w - first[p] (column-major over the problem's tile grid) of the problem p
// with first[p] <= w < first[p + 1]; the host orders the problems so that
// the most expensive tiles (largest k) are taken first.  Every workgroup
// starts with item blockIdx.x and then takes the next free item from a
// device counter until none is left; the last workgroup to finish resets the
// counter for the next launch.
template <int BM, int BN, int WGM, int WGN, bool TA, bool TB, bool ABFT, bool IVL, int MINB, bool PRE, bool DIR>
__global__ __launch_bounds__(WGM* WGN * 64, (waves_per_simd<BM, BN, WGM, WGN, MINB, DIR, ABFT>())) void dgemm_batched_kernel(
    BatchLaunch L)
{
    __shared__ int s_item;
    int item = blockIdx.x;
    for (;;) {
        if (item >= L.total) break;
        // problem of this item: binary search of the first-tile table
        int lo = 0, hi = L.count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.first[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const int p = __builtin_amdgcn_readfirstlane(lo);
        const DGemmArgs a = L.desc[p];
        const int local = item - L.first[p];
        const int tm = __builtin_amdgcn_readfirstlane(local % a.tiles_m);
        const int tn = __builtin_amdgcn_readfirstlane(local / a.tiles_m);
        dgemm_tile<BM, BN, WGM, WGN, TA, TB, ABFT, IVL, PRE, DIR>(a, tm, tn);
        // all LDS use of this tile ends before the next item is published
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)gridDim.x + (int)atomicAdd(&L.queue[0], 1u);
        __syncthreads();
        item = __builtin_amdgcn_readfirstlane(s_item);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&L.queue[1], 1u) == gridDim.x - 1) {
            atomicExch(&L.queue[0], 0u);
            atomicExch(&L.queue[1], 0u);
            __threadfence();
        }
    }
}

// ------------------------------------------------------------------ launchers
template <int BM, int BN, int WGM, int WGN, bool IVL_OK, int MINB>
hipError_t launch_tile(const DGemmArgs& a, bool abft, hipStream_t s)
{
    const dim3 grid(a.tiles_m * a.tiles_n), block(WGM * WGN * 64);
    const bool ivl = abft && a.kc < a.k;
    if (ivl && !IVL_OK) return hipErrorInvalidValue;
    const bool pre = abft && a.asp != nullptr;
    constexpr bool DOK = DCfg<BM, BN, WGM, WGN, false, false>::DIRECT;
    // direct staging with interval checks only at one workgroup per CU (the
    // interval kernels' restart path needs the whole register file)
    const bool dir = DOK && a.lds_direct && (!abft || (pre && (!ivl || MINB == 0)));
#define FTG_L(TA_, TB_, AB_, IV_, PR_, DR_)                                                                 \
    hipLaunchKernelGGL((dgemm_abft_kernel<BM, BN, WGM, WGN, TA_, TB_, AB_, IV_, MINB, PR_, DR_>), grid, block, 0, \
                       s, a)
#define FTG_T(AB_, IV_, PR_, DR_)                                       \
    do {                                                                \
        if (!a.ta && !a.tb) FTG_L(false, false, AB_, IV_, PR_, DR_);    \
        else if (a.ta && !a.tb) FTG_L(true, false, AB_, IV_, PR_, DR_); \
        else if (!a.ta && a.tb) FTG_L(false, true, AB_, IV_, PR_, DR_); \
        else FTG_L(true, true, AB_, IV_, PR_, DR_);                     \
    } while (0)
    if (!abft) {
        if constexpr (DOK) {
            if (dir) FTG_T(false, false, false, true);
            else FTG_T(false, false, false, false);
        } else FTG_T(false, false, false, false);
    } else if (!ivl) {
        if (pre) {
            if constexpr (DOK) {
                if (dir) FTG_T(true, false, true, true);
                else FTG_T(true, false, true, false);
            } else FTG_T(true, false, true, false);
        } else FTG_T(true, false, false, false);
    } else if constexpr (IVL_OK) {
        if (pre) {
            if constexpr (DOK && MINB == 0) {
                if (dir) FTG_T(true, true, true, true);
                else FTG_T(true, true, true, false);
            } else FTG_T(true, true, true, false);
        } else FTG_T(true, true, false, false);
    }
#undef FTG_T
#undef FTG_L
    return hipGetLastError();
}

// Persistent grid: as many workgroups as are resident on the device at once
// (from the kernel's register and LDS use), never more than there are work
// items.  Queried once per kernel instantiation.
template <int BM, int BN, int WGM, int WGN, bool TA, bool TB, bool AB, bool IV, int MINB, bool PR, bool DR>
int batched_grid(int total)
{
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, dgemm_batched_kernel<BM, BN, WGM, WGN, TA, TB, AB, IV, MINB, PR, DR>, WGM * WGN * 64, 0) !=
                hipSuccess)
            return std::min(total, 256);
        resident = std::max(1, cus) * std::max(1, per_cu);
    }
    return std::min(total, resident);
}

template <int BM, int BN, int WGM, int WGN, bool IVL_OK, int MINB>
hipError_t launch_batched(const BatchLaunch& L, int ta, int tb, bool abft, bool ivl, bool pre, bool lds_direct,
                          hipStream_t s)
{
    if (L.total <= 0) return hipSuccess;
    if (ivl && !IVL_OK) return hipErrorInvalidValue;
    const dim3 block(WGM * WGN * 64);
    constexpr bool DOK = DCfg<BM, BN, WGM, WGN, false, false>::DIRECT;
    const bool dir = DOK && lds_direct && (!abft || (pre && !ivl));
#define FTG_L(TA_, TB_, AB_, IV_, PR_, DR_)                                                                        \
    hipLaunchKernelGGL((dgemm_batched_kernel<BM, BN, WGM, WGN, TA_, TB_, AB_, IV_, MINB, PR_, DR_>),                 \
                       dim3(batched_grid<BM, BN, WGM, WGN, TA_, TB_, AB_, IV_, MINB, PR_, DR_>(L.total)), block, 0, \
                       s, L)
#define FTG_T(AB_, IV_, PR_, DR_)                                  \
    do {                                                           \
        if (!ta && !tb) FTG_L(false, false, AB_, IV_, PR_, DR_);   \
        else if (ta && !tb) FTG_L(true, false, AB_, IV_, PR_, DR_); \
        else if (!ta && tb) FTG_L(false, true, AB_, IV_, PR_, DR_); \
        else FTG_L(true, true, AB_, IV_, PR_, DR_);                \
    } while (0)
    if (!abft) {
        if constexpr (DOK) {
            if (dir) FTG_T(false, false, false, true);
            else FTG_T(false, false, false, false);
        } else FTG_T(false, false, false, false);
    } else if (!ivl) {
        if (pre) {
            if constexpr (DOK) {
                if (dir) FTG_T(true, false, true, true);
                else FTG_T(true, false, true, false);
            } else FTG_T(true, false, true, false);
        } else FTG_T(true, false, false, false);
    } else if constexpr (IVL_OK) {
        if (pre) FTG_T(true, true, true, false);
        else FTG_T(true, true, false, false);
    }
#undef FTG_T
#undef FTG_L
    return hipGetLastError();
}

}  // namespace ftg
