// Wide low-precision GEMM kernel for gfx950: 256 x 256 output tiles per
// workgroup, eight waves of 128 x 64, both operands k-contiguous (op(A) rows
// and op(B) columns along k, which every layout is after packing) and K a
// multiple of the k-block.
//
// Against the 128 x 128 kernel the wide tile halves the operand bytes moved
// per multiply-add (global to LDS: (256 + 256) rows per 256 x 256 outputs) and
// cuts the fragment reads from LDS by a quarter (128 + 64 rows per wave per
// 128 x 64 outputs), the two paths that bound the smaller tile.
//
// Protected mode keeps the 128 x 128 checksum tiles of the other kernel (the
// same slots, thresholds and repair requests; a workgroup checks its 2 x 2
// tiles) but folds the maintained checksums into the product (§5.2: the
// checksum updates reuse the operand panels already staged for the product):
//   row checksums A_I (B_J e): the three bf16 pieces of B_J e of the
//       workgroup's two tile columns ride along as six extra B rows of every
//       stage, multiplied by the A fragments already in registers;
//   column checksums (e^T A_I) B_J: the pieces of e^T A_I likewise as six
//       extra A rows, multiplied by the B fragments.
// A wave adds two MFMAs of each kind per k-step (36 instead of 32), FP32
// accumulation like the data path; the two thin checksum GEMMs of the
// 128 x 128 path and their re-reads of A and B are gone.
#pragma once
#include <type_traits>

#include "lowp_kernel.hpp"

namespace ftg {

typedef int i32x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// bf16: v_mfma_f32_16x16x32_bf16, 8 x 4 fragments of 16 x 16 per wave.
// fp8: the gfx950 full-rate v_mfma_scale_f32_32x32x64_f8f6f4 (e4m3 operands,
// unit block scales), 4 x 2 fragments of 32 x 32.  A lane holds row (column)
// lane % 32 of an operand fragment with steps 32 (lane / 32) .. + 31, and
// accumulator element q of rows 8 (q / 4) + 4 (lane / 32) + q % 4, column
// lane % 32 (checked on the device against a decoding product).
template <bool FP8>
struct WCfg {
    static constexpr int EB = FP8 ? 1 : 2;                   // bytes per element
    static constexpr int BM = 256, BN = 256, BK = 64 / EB;   // 64-byte k-block rows
    static constexpr int NT = 512;                           // eight waves: 2 (m) x 4 (n)
    static constexpr int WM = 128, WN = 64;
    static constexpr int ROWB = 64;
    static constexpr int A_BYTES = BM * ROWB, B_BYTES = BN * ROWB;  // 16 KB each
    // checksum pieces per panel sum (bf16: three of 2^0; fp8: eight e4m3 with
    // scales 2^(7 - 4 t)); their LDS rows per stage: 8 of e^T A_I then 8 of
    // B_J e (bf16, six used) or 16 and 16 (fp8)
    static constexpr int PIECES = FP8 ? 8 : 3;
    static constexpr int X_BYTES = FP8 ? 2048 : 1024;
    static constexpr int NSTAGE = 4;  // a power of two
    static constexpr int LPW = (A_BYTES + B_BYTES) / 1024 / 8;       // wave loads per stage
    static constexpr int FD = FP8 ? 32 : 16;                         // fragment edge
    static constexpr int FM = WM / FD, FN = WN / FD;
    using Frag = std::conditional_t<FP8, i32x8_t, bf16x8_t>;
    using Acc = std::conditional_t<FP8, f32x16_t, f32x4_t>;
    static constexpr int XF = FP8 ? 1 : 2;  // checksum fragments per wave and kind
};

// 16-byte chunk c of LDS row r is stored at chunk c ^ wide_swz<FP8>(r).
// Measured with SQ_LDS_BANK_CONFLICT: the bf16 fragment reads (16 lanes on
// consecutive rows per chunk) are conflict-free with (r >> 1) & 3 and take
// about 4 conflict cycles per read with (r >> 2) & 3; the fp8 reads (32 lanes
// on consecutive rows, two chunks each) the other way round.
template <bool FP8>
__device__ __attribute__((always_inline)) inline int wide_swz(int r)
{
    return FP8 ? (r >> 2) & 3 : (r >> 1) & 3;
}

// Waits until at most `later` blocks of this wave's loads (PER each) are in
// flight, and for its LDS reads; then a barrier publishes the block.
template <int PER>
__device__ __attribute__((always_inline)) inline void wide_wait_blocks(int later)
{
    static_assert(3 * PER <= 15, "vmcnt field");
    asm volatile("" ::: "memory");
    // s_waitcnt: vmcnt = later * PER, expcnt unconstrained, lgkmcnt = 0
    if (later >= 3) __builtin_amdgcn_s_waitcnt(0x70 | (3 * PER));
    else if (later == 2) __builtin_amdgcn_s_waitcnt(0x70 | (2 * PER));
    else if (later == 1) __builtin_amdgcn_s_waitcnt(0x70 | PER);
    else __builtin_amdgcn_s_waitcnt(0x70);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// The kernel arguments (the only explicit argument, at the start of the
// kernarg segment) through an opaque constant-space pointer: the epilogue's
// scalar loads of them then stay after the k loop instead of holding scalar
// registers through it.  (Taking the address of the argument itself would
// copy it to private memory.)
typedef const LowpArgs __attribute__((address_space(4)))* KArgsPtr;
__device__ __attribute__((always_inline)) inline KArgsPtr launder_args()
{
    KArgsPtr p = (KArgsPtr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return p;
}
__device__ __attribute__((always_inline)) inline InjectParams inject_of(KArgsPtr p)
{
    InjectParams ip;
    ip.on = p->inj.on; ip.target = p->inj.target; ip.bit_lo = p->inj.bit_lo; ip.bit_hi = p->inj.bit_hi;
    ip.seed = p->inj.seed; ip.S = p->inj.S; ip.F = p->inj.F; ip.a_inv = p->inj.a_inv; ip.b = p->inj.b;
    return ip;
}

// Epilogue staging: 16 columns of 128 rows per wave, 132 floats per column
// (the 4-float pad keeps the transposing writes and reads conflict-free).
constexpr int kWideCP = 132;
constexpr int kWideStgBytes = 8 * 16 * kWideCP * 4;

// Verification bookkeeping of the protected kernel (after the staging area).
template <int P>
struct WVerify {
    float er[256][2 * P];              // row checksum pieces: [row][P J + piece]
    float ec[256][2 * P];              // column checksum pieces: [column][P I + piece]
    double rs[4][256];                 // row sums over each wave column's 64 columns
    double cs[2][256];                 // column sums over each wave row's 128 rows
    double cir[4][256], cira[4][256];  // the same of C_in and abs(C_in)
    double cic[2][256], cica[2][256];
    double dfi[4], tfi[4], dfj[4], tfj[4], exi[4], exj[4];
    int nfr[4], nfc[4], fi[4], fj[4];
};

template <bool FP8, int MODE>
__global__ __launch_bounds__(512, 1) void lowp_wide_kernel(LowpArgs args)
{
    using Cf = WCfg<FP8>;
    constexpr int BM = Cf::BM, BN = Cf::BN, BK = Cf::BK, NS = Cf::NSTAGE;
    constexpr int STAGE = Cf::A_BYTES + Cf::B_BYTES + (MODE == 1 ? Cf::X_BYTES : 0);
    using Verify = WVerify<Cf::PIECES>;
    static_assert(kWideStgBytes + (MODE == 1 ? sizeof(Verify) : 0) <= NS * STAGE, "epilogue area");
    constexpr int FM = Cf::FM, FN = Cf::FN;
    using Frag = typename Cf::Frag;
    using Acc = typename Cf::Acc;
    __shared__ __attribute__((aligned(16))) unsigned char smem[NS * STAGE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave >> 2, wc = wave & 3;
    const int wm0 = wr * Cf::WM, wn0 = wc * Cf::WN;
    const int l16 = lane & 15, lq = lane >> 4;
    // Fragment order: A fragment g holds the wave's row block (g + rot_a) mod 8,
    // B fragment h its column block (h + rot_b) mod 4.  Protected mode rotates
    // them so that the row blocks whose checksums a wave updates (2 wc, 2 wc + 1)
    // and the column blocks (2 wr, 2 wr + 1) are fragments 0 and 1 of every
    // wave: the checksum MFMAs then take fixed registers (a uniform choice among
    // fragments would cost branches or selects in the loop).
    const int rot_a = MODE == 1 ? (FP8 ? wc : 2 * wc) : 0, rot_b = MODE == 1 ? (FP8 ? wr : 2 * wr) : 0;

    // wide tiles: (tiles_m + 1) / 2 x (tiles_n + 1) / 2 of the 128 x 128 tiles
    const int wtm = (args.tiles_m + 1) >> 1, wtn = (args.tiles_n + 1) >> 1;
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, wtm, wtn, 4, &tm, &tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int R = (int)min((int64_t)BM, (int64_t)args.m - m0);
    const int Q = (int)min((int64_t)BN, (int64_t)args.n - n0);
    const int K = args.k;
    const int ldxs = args.ldxs;  // elements between rows of the checksum pieces
    const int nkb = K / BK;
    const int64_t lda = args.lda, ldb = args.ldb;
    const unsigned char* A = (const unsigned char*)args.A;
    const unsigned char* B = (const unsigned char*)args.B;

    // ---- staging: per stage 16 wave loads of A rows then 16 of B rows, four
    // per wave; wave load I covers rows 16 I .. 16 I + 15 (slot = 64 I + lane,
    // row = slot / 4, chunk = slot % 4, stored at chunk ^ wide_swz<FP8>(row)).  A
    // wave's load u covers rows 64 (wave % 4) + 16 u + lane / 4: the same lane
    // offset from a resource that starts 16 u rows further and ends after the
    // last row of the matrix (the range check applies to the lane offset), so
    // loads of rows past the matrix return zeros; they only feed accumulators
    // that are never stored or checked.
    const bool a_wave = wave < 4;  // waves 0-3 load A, 4-7 load B
    const int64_t ldx = (a_wave ? lda : ldb) * Cf::EB;  // bytes between rows
    const int rows_left = (a_wave ? R : Q) - 64 * (wave & 3);
    int voff0;
    {
        const int x = lane / 4;
        voff0 = (int)((int64_t)x * ldx + 16 * ((lane & 3) ^ wide_swz<FP8>(x)));
    }
    const unsigned char* src0 = (a_wave ? A + m0 * lda * Cf::EB : B + n0 * ldb * Cf::EB) + 64 * (wave & 3) * ldx;
    // protected, bf16: wave 0 adds one load per stage of the checksum pieces
    // (k-major rows of K bf16), lanes 0-23 the six rows of e^T A_I of the
    // workgroup's two tile rows, lanes 32-55 the six of B_J e.  fp8: waves 0
    // and 1 add one each, the sixteen rows (K bytes) of e^T A_I and of B_J e.
    // A missing second tile reads the last rows (its checks are skipped).
    const bool xw = MODE == 1 && (FP8 ? wave < 2 : wave == 0);
    const unsigned char* XS = (const unsigned char*)(FP8 && wave == 1 ? args.XSB : args.XSA);
    int xoff = 0;
    bool xlane = false;
    // fp8: the first piece row and the last row of the wave's pieces (the lane
    // offset is formed at each load, keeping no register through the loop)
    const int x8_r0 = (FP8 && MODE == 1) ? 2 * Cf::PIECES * (wave == 1 ? tn : tm) : 0;
    const int x8_rmax = (FP8 && MODE == 1) ? Cf::PIECES * (wave == 1 ? args.tiles_n : args.tiles_m) - 1 : 0;
    if constexpr (MODE == 1 && !FP8) {
        const int64_t xsb = (const unsigned char*)args.XSB - XS;
        if (lane < 24) {
            const int r = min(6 * tm + lane / 4, 3 * args.tiles_m - 1);
            xoff = (int)((int64_t)r * args.ldxs * 2 + 16 * (lane % 4));
            xlane = true;
        } else if (lane >= 32 && lane < 56) {
            const int j = lane - 32, r = min(6 * tn + j / 4, 3 * args.tiles_n - 1);
            xoff = (int)(xsb + (int64_t)r * args.ldxs * 2 + 16 * (j % 4));
            xlane = true;
        }
    }
    auto issue = [&](int kb, int st) __attribute__((always_inline)) {
        unsigned char* base = smem + st * STAGE + (a_wave ? 0 : Cf::A_BYTES) + 4096 * (wave & 3);
        if (MODE == 1 && xw) {
            unsigned char* xd = smem + st * STAGE + Cf::A_BYTES + Cf::B_BYTES + (FP8 ? 1024 * wave : 0);
            if constexpr (FP8) {
                const int xo = min(x8_r0 + lane / 4, x8_rmax) * ldxs + 16 * (lane % 4);
                lds_dma16(make_rsrc(XS + (int64_t)kb * 64), xd, xo);
            } else if (xlane) {
                lds_dma16(make_rsrc(XS + (int64_t)kb * 64), xd, xoff);
            }
        }
#pragma unroll
        for (int u = 0; u < Cf::LPW; ++u) {
            // rows 16 u .. of this wave's 64 that exist: up to the last one's 64 bytes
            const int left = rows_left - 16 * u;
            const int nrec = left > 0 ? (int)((int64_t)(min(left, 16) - 1) * ldx + 64) : 0;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<unsigned char*>(src0 + 16 * u * ldx + (int64_t)kb * 64), (short)0, nrec, 0x00020000);
            lds_dma16(rs, base + 1024 * u, voff0);
        }
    };
    // wait for a block whose successors (this wave's loads of them) may stay
    // in flight, then publish it to every wave
    auto wait_blocks = [&](int later) __attribute__((always_inline)) {
        if (MODE == 1 && xw) wide_wait_blocks<Cf::LPW + 1>(later);
        else wide_wait_blocks<Cf::LPW>(later);
    };

    Acc acc[FM][FN];
#pragma unroll
    for (int g = 0; g < FM; ++g)
#pragma unroll
        for (int h = 0; h < FN; ++h) acc[g][h] = Acc{};
    // protected: row checksums of rows 16 (2 wc + i) + .. against the pieces of
    // B_J e (columns 3 J + piece), column checksums of columns 16 (2 wr + i) + ..
    // against the pieces of e^T A_I (rows 3 I + piece)
    Acc accr[Cf::XF], accc[Cf::XF];
#pragma unroll
    for (int i = 0; i < Cf::XF; ++i) accr[i] = accc[i] = Acc{};

    // ---- injection plan of this wave's checksum tile (I, J) = (wr, wc / 2):
    // up to two faults, applied to the accumulator after their k-block by the
    // wave whose 64 columns hold them (the checksum target is applied to the
    // expected sum in the epilogue).  Only the blocks stay live through the k
    // loop; the rest of the plan is drawn again when a fault is applied.
    const bool inj = MODE == 1 && args.inj.on;
    const int tmw = 2 * tm + wr, tnw = 2 * tn + (wc >> 1);  // this wave's checksum tile
    // (the slot of interval `it` of n_int: steps plo .. plo + k - 1)
    auto wave_faults = [&](const InjectParams& ip, int tiles_m, int tiles_n, int m, int n, int k, int n_int, int it,
                           int64_t plo, Fault* f2) __attribute__((always_inline)) {
        int nf = 0;
        if (ip.on && ip.target != FTG_TARGET_CHECKSUM && tmw < tiles_m && tnw < tiles_n)
            nf = slot_faults(ip, ((uint64_t)tnw * tiles_m + tmw) * n_int + it, min(128, m - 128 * tmw),
                             min(128, n - 128 * tnw), plo, plo + k, f2);
        return nf;
    };
    // (the same plan in every lane; read from the first so that the k loop's
    // control flow stays uniform)
    int fkb[2] = {-1, -1};
    if (inj) {
        Fault f2[2];
        const int nf = wave_faults(args.inj, args.tiles_m, args.tiles_n, args.m, args.n, K, args.n_int,
                                   args.interval, args.plo, f2);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            fkb[q] = __builtin_amdgcn_readfirstlane(
                q < nf && f2[q].col / 64 == (wc & 1) ? (int)((f2[q].pflip - args.plo) / BK) : -1);
    }
    auto apply_fault = [&](int q) __attribute__((always_inline)) {
        const KArgsPtr ar = launder_args();
        const InjectParams ip = inject_of(ar);
        Fault f2[2];
        wave_faults(ip, ar->tiles_m, ar->tiles_n, ar->m, ar->n, ar->k, ar->n_int, ar->interval, ar->plo, f2);
        const int rr = __builtin_amdgcn_readfirstlane(f2[q].row), col = __builtin_amdgcn_readfirstlane(f2[q].col);
        const int cc = col % 64, bit = __builtin_amdgcn_readfirstlane(f2[q].bit);
        const bool own = lane == ((rr % 16) / 4) * 16 + cc % 16;
        float oldv = 0.0f, newv = 0.0f;
        if constexpr (FP8) {
            // 32 x 32 fragments: block (rr / 32, cc / 32), lane (lh, cc % 32) with
            // lh = (rr % 32) / 4 % 2, element 4 ((rr % 32) / 8) + rr % 4
            const int i = rr % 32;
            const bool own8 = lane == 32 * ((i / 4) % 2) + cc % 32;
            const int gh = ((rr / 32 - rot_a) & 3) * 2 + ((cc / 32 - rot_b) & 1), qe = 4 * (i / 8) + i % 4;
#pragma unroll
            for (int g = 0; g < FM; ++g)
#pragma unroll
                for (int h = 0; h < FN; ++h)
                    if (g * FN + h == gh) {
                        Acc v = acc[g][h];
#pragma unroll
                        for (int e = 0; e < 16; ++e)
                            if (e == qe) oldv = v[e];
                        newv = flip_f32(oldv, bit);
#pragma unroll
                        for (int e = 0; e < 16; ++e)
                            if (e == qe && own8) v[e] = newv;
                        acc[g][h] = v;
                    }
            if (own8)
                push_inject(ar->rep, ar->problem, tmw, tnw, ar->interval, m0 + 128 * wr + rr, n0 + 128 * (wc >> 1) + col,
                            f2[q].pflip, bit, FTG_TARGET_ACC, (double)oldv, (double)newv);
            return;
        }
        // fragment (g, h) = (rr / 16, cc / 16) by a uniform branch, then the
        // element rr % 4 of the lane's four
        const int gh = ((rr / 16 - rot_a) & 7) * 4 + ((cc / 16 - rot_b) & 3), re = rr % 4;
#pragma unroll
        for (int g = 0; g < FM; ++g)
#pragma unroll
            for (int h = 0; h < FN; ++h)
                if constexpr (!FP8) if (g * 4 + h == gh) {
                    f32x4_t v = acc[g][h];
                    oldv = re == 0 ? v[0] : re == 1 ? v[1] : re == 2 ? v[2] : v[3];
                    newv = flip_f32(oldv, bit);
                    const float w = own ? newv : oldv;
                    v[0] = re == 0 ? w : v[0];
                    v[1] = re == 1 ? w : v[1];
                    v[2] = re == 2 ? w : v[2];
                    v[3] = re == 3 ? w : v[3];
                    acc[g][h] = v;
                }
        if (own)
            push_inject(ar->rep, ar->problem, tmw, tnw, ar->interval, m0 + 128 * wr + rr, n0 + 128 * (wc >> 1) + col,
                        f2[q].pflip, bit, FTG_TARGET_ACC, (double)oldv, (double)newv);
    };
    auto faults_after = [&](int kb) __attribute__((always_inline)) {
        if (MODE == 1) {
            if (kb == fkb[0]) apply_fault(0);
            if (kb == fkb[1]) apply_fault(1);
        }
    };

    // fragment read offset inside a row: chunk lq, swizzled by the row (l16)
    const int fo = 16 * (lq ^ wide_swz<FP8>(l16));
    // A fragments: one set, each refilled with the next block's as soon as
    // its four MFMAs are issued; B fragments: two sets; checksum-piece
    // fragments (x[0]: e^T A_I rows, x[1]: B_J e rows; rows 6 and 7 of each
    // only feed accumulator lanes that are never read): one set, refilled
    // after the block's last MFMA
    Frag fa[FM], fb[2][FN], fx[2];
    // fp8: the lane's 32 steps are chunks 2 (lane / 32) and + 1 of its row
    const int l32 = lane & 31, lh = lane >> 5;
    const int fo8a = 16 * ((2 * lh) ^ wide_swz<FP8>(l32)), fo8b = 16 * ((2 * lh + 1) ^ wide_swz<FP8>(l32));
    auto frag_at = [&](const unsigned char* rowp) __attribute__((always_inline)) {
        if constexpr (FP8) {
            const u32x4_t lo = *(const u32x4_t*)(rowp + fo8a), hi = *(const u32x4_t*)(rowp + fo8b);
            return (Frag){(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
        } else {
            return *(const Frag*)(rowp + fo);
        }
    };
    auto a_frag = [&](int st, int g) __attribute__((always_inline)) {
        if constexpr (FP8) return frag_at(smem + st * STAGE + (wm0 + 32 * ((g + rot_a) & 3) + l32) * 64);
        else return frag_at(smem + st * STAGE + (wm0 + 16 * ((g + rot_a) & 7) + l16) * 64);
    };
    auto read_b = [&](int st, Frag* b) __attribute__((always_inline)) {
        const unsigned char* tb = smem + st * STAGE + Cf::A_BYTES;
#pragma unroll
        for (int h = 0; h < FN; ++h) {
            if constexpr (FP8) b[h] = frag_at(tb + (wn0 + 32 * ((h + rot_b) & 1) + l32) * 64);
            else b[h] = frag_at(tb + (wn0 + 16 * ((h + rot_b) & 3) + l16) * 64);
        }
    };
    // fp8: piece fragment i (0: e^T A_I rows, 1: B_J e rows) of the block in
    // stage st, rows l32 % 16 (rows 16-31 of the fragment repeat 0-15: they
    // only feed accumulator lanes that are never read), steps 32 lh .. + 31
    auto x8_frag = [&](int st, int i) __attribute__((always_inline)) {
        const unsigned char* tx = smem + st * STAGE + Cf::A_BYTES + Cf::B_BYTES + 1024 * i + (l32 & 15) * 64 + 32 * lh;
        const u32x4_t lo = *(const u32x4_t*)tx, hi = *(const u32x4_t*)(tx + 16);
        return (i32x8_t){(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
    };
    auto read_x = [&](int st) __attribute__((always_inline)) {
        if constexpr (MODE == 1 && !FP8) {
            const unsigned char* tx = smem + st * STAGE + Cf::A_BYTES + Cf::B_BYTES + (l16 & 7) * 64 + 16 * lq;
            fx[0] = *(const Frag*)tx;
            fx[1] = *(const Frag*)(tx + 512);
        }
    };
    // MFMAs of the current block; with `refill` each A fragment is then
    // replaced by that of the block in stage st.  Protected: row checksums of
    // A fragments 0 and 1 against x[1] (row blocks 2 wc and 2 wc + 1 after the
    // rotation), column checksums of x[0] against B fragments 0 and 1 (column
    // blocks 2 wr and 2 wr + 1).
    auto mfmas = [&](const Frag* b, int st, auto refill, int st_cur) __attribute__((always_inline)) {
#pragma unroll
        for (int g = 0; g < FM; ++g) {
#pragma unroll
            for (int h = 0; h < FN; ++h) {
                if constexpr (FP8)
                    acc[g][h] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[g], b[h], acc[g][h], 0, 0, 0, 127, 0, 127);
                else
                    acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[g], b[h], acc[g][h], 0, 0, 0);
            }
            if constexpr (MODE == 1 && FP8) {
                // one piece-fragment register set: B_J e rows (read with the
                // block's first fragments), then e^T A_I rows (read here)
                if (g == 0) {
                    accr[0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[0], fx[0], accr[0], 0, 0, 0, 127, 0, 127);
                    fx[0] = x8_frag(st_cur, 0);
                }
                if (g == FM - 1) accc[0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fx[0], b[0], accc[0], 0, 0, 0, 127, 0, 127);
            } else if constexpr (MODE == 1) {
                if (g < 2) accr[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[g], fx[1], accr[g], 0, 0, 0);
                if (g == 7) {
                    accc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fx[0], b[0], accc[0], 0, 0, 0);
                    accc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fx[0], b[1], accc[1], 0, 0, 0);
                }
            }
            if constexpr (decltype(refill)::value) fa[g] = a_frag(st, g);
            // keep the written order: the scheduler would otherwise sink the
            // reads below the last MFMAs and expose their latency
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // Blocks loaded ahead: NS (each step refills the stage of the block whose
    // MFMAs it runs: its fragments were read in the step before), except for
    // protected fp8, which reads that block's checksum-piece fragments during
    // its step and refills the previous block's stage instead (NS - 1 ahead).
    constexpr int LA = (FP8 && MODE == 1) ? NS - 1 : NS;
    // ---- k loop over the ring, software-pipelined: block kb + 1's fragments
    // are read while block kb's MFMAs run.  The wait for block kb + 1 (its
    // loads by every wave, then a barrier) also retires every wave's reads of
    // block kb, whose stage then takes the load of block kb + NS: NS - 1
    // blocks stay in flight.  (The inner loop keeps its body free of branches
    // around LDS reads: the compiler's wait insertion merges states at such
    // joins and would then wait for the fragments just requested; injected
    // faults are applied between segments of that loop.)
    auto step = [&](int kb) __attribute__((always_inline)) {
        wait_blocks(min(nkb - 1, kb + LA - 1) - (kb + 1));
        // the wait above retired the reads of this block's fragments; pass
        // them through an empty asm so that no wait for them is placed after
        // the next block's reads
#pragma unroll
        for (int g = 0; g < FM; ++g) asm volatile("" : "+v"(fa[g]));
#pragma unroll
        for (int h = 0; h < FN; ++h) asm volatile("" : "+v"(fb[0][h]));
        if constexpr (MODE == 1 && !FP8) {
            asm volatile("" : "+v"(fx[0]));
            asm volatile("" : "+v"(fx[1]));
        }
        if (kb + LA < nkb) issue(kb + LA, (kb + LA) & (NS - 1));
        // (protected fp8 has no registers for a second B set: its next B
        // fragments are read after the block's last MFMA, during the wait
        // that follows)
        constexpr bool single_b = FP8 && MODE == 1;
        if constexpr (!single_b) read_b((kb + 1) & (NS - 1), fb[1]);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (FP8 && MODE == 1) fx[0] = x8_frag(kb & (NS - 1), 1);
        mfmas(fb[0], (kb + 1) & (NS - 1), std::true_type{}, kb & (NS - 1));
        if constexpr (single_b) {
            read_b((kb + 1) & (NS - 1), fb[0]);
        } else {
#pragma unroll
            for (int h = 0; h < FN; ++h) fb[0][h] = fb[1][h];
        }
        read_x((kb + 1) & (NS - 1));
    };
#pragma unroll 1
    for (int b = 0; b < LA && b < nkb; ++b) issue(b, b);
    // block 0: this wave's loads of blocks 1 .. NS - 1 may stay in flight
    wait_blocks(min(nkb - 1, LA - 1));
#pragma unroll
    for (int g = 0; g < FM; ++g) fa[g] = a_frag(0, g);
    read_b(0, fb[0]);
    read_x(0);
    // blocks 0 .. nkb - 2 (each with a successor) in segments that end at a
    // block after which a fault is applied (one copy of the block step: a
    // second one would not fit the registers), then the last block
    int kb = 0;
    while (kb <= nkb - 2) {
        int stop = nkb - 2;
        if (MODE == 1) {
            if (fkb[0] >= kb) stop = min(stop, fkb[0]);
            if (fkb[1] >= kb) stop = min(stop, fkb[1]);
        }
#pragma unroll 1
        for (; kb <= stop; ++kb) step(kb);
        faults_after(stop);
    }
    if constexpr (FP8 && MODE == 1) fx[0] = x8_frag((nkb - 1) & (NS - 1), 1);
    mfmas(fb[0], 0, std::false_type{}, (nkb - 1) & (NS - 1));
    faults_after(nkb - 1);

    // ---- epilogue.  Lane (lq, l16) of fragment (g, h) holds rows
    // wm0 + 16 g + 4 lq + (0 .. 3) of column wn0 + 16 h + l16.  Column-major C
    // takes the tile through LDS, 16 columns of a wave at a time: each store
    // then writes two whole 512-byte column runs (the fragment layout would
    // scatter every store over 16 columns, one ldc apart).
    const KArgsPtr ea = launder_args();
    const int64_t ldc = ea->ldc;
    const float as = ea->alpha * (ea->scale_a ? *ea->scale_a : 1.0f) * (ea->scale_b ? *ea->scale_b : 1.0f);
    const bool cin = ea->beta != 0.0f;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(ea->C + m0 + n0 * ldc);
    const bool vec_c = ea->vec_c;
    float* stg = (float*)smem + wave * (16 * kWideCP);
    // the lane's rows and column pair in the staged layout
    const int rl = 4 * (lane & 31), cl = lane >> 5;
    const int row = wm0 + rl;
    Verify& V = *(Verify*)(smem + kWideStgBytes);
    // scale of checksum piece t (the encode pass's split)
    auto piece_weight = [](int t) __attribute__((always_inline)) { return FP8 ? ldexp(1.0, 7 - 4 * t) : 1.0; };
    __syncthreads();  // every wave is done with the ring
    if constexpr (MODE == 1) {
        // expected pieces from the checksum accumulators
        if constexpr (FP8) {
            // accr: rows of row block wc x pieces (columns) l32; accc: pieces (rows)
            // x columns of column block wr
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int rq = 8 * (q / 4) + 4 * lh + q % 4;
                if (l32 < 16) V.er[wm0 + 32 * wc + rq][l32] = accr[0][q];
                if (rq < 16) V.ec[wn0 + 32 * wr + l32][rq] = accc[0][q];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (l16 < 6) V.er[wm0 + 16 * (2 * wc + i) + 4 * lq + r][l16] = accr[i][r];
                    if (4 * lq + r < 6) V.ec[wn0 + 16 * (2 * wr + i) + l16][4 * lq + r] = accc[i][r];
                }
        }
        if (tid < 4) { V.nfr[tid] = 0; V.nfc[tid] = 0; }
    }
    // One pass over the tile: the final values alpha s acc + beta C_in; with
    // `sums` their reference sums (binary64, §5.2; rows and columns outside the
    // matrix excluded) and those of C_in; with `store` the stores.
    auto pass = [&](bool store, bool sums) __attribute__((always_inline)) {
        double rsl[4] = {0.0, 0.0, 0.0, 0.0}, cirl[4] = {0.0, 0.0, 0.0, 0.0}, cial[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int hs = 0; hs < 4; ++hs) {
            auto col_of = [&](int p) __attribute__((always_inline)) {
                const int c = 2 * p + cl;
                return wn0 + (FP8 ? 32 * (((hs >> 1) + rot_b) & 1) + 16 * (hs & 1) : 16 * ((hs + rot_b) & 3)) + c;
            };
            // C_in of a group of kCinAhead column pairs, all requested before
            // any is used (one memory round trip per group instead of one per pair)
            constexpr int kCinAhead = 4;
            f32x4_t civ[kCinAhead];
            auto load_cin = [&](int p0) __attribute__((always_inline)) {
#pragma unroll
                for (int j = 0; j < kCinAhead; ++j) {
                    const int col = col_of(p0 + j);
                    const bool colok = col < Q;
                    const int vo = (int)(((int64_t)col * ldc + row) * 4);
                    if (vec_c && colok && row + 4 <= R) {
                        civ[j] = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rc, vo, 0, 0));
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            civ[j][r] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                                rc, colok && row + r < R ? vo + 4 * r : kOOB, 0, 0));
                    }
                }
            };
            // stage column block hs (16 columns) of the wave
            if constexpr (FP8) {
                // register fragment hs / 2 (column block (hs / 2 + rot_b) % 2), its
                // columns 16 (hs % 2) .. + 15
                const int h = hs >> 1;
                if ((l32 >> 4) == (hs & 1)) {
#pragma unroll
                    for (int g = 0; g < FM; ++g)
#pragma unroll
                        for (int rq = 0; rq < 4; ++rq)
                            *(f32x4_t*)(stg + (l32 & 15) * kWideCP + 32 * ((g + rot_a) & 3) + 8 * rq + 4 * lh) =
                                (f32x4_t){acc[g][h][4 * rq], acc[g][h][4 * rq + 1], acc[g][h][4 * rq + 2],
                                          acc[g][h][4 * rq + 3]};
                }
            } else {
#pragma unroll
                for (int g = 0; g < FM; ++g)
                    *(f32x4_t*)(stg + l16 * kWideCP + 16 * ((g + rot_a) & 7) + 4 * lq) = acc[g][hs];
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll 1
            for (int pg = 0; pg < 8; pg += kCinAhead) {
            if (cin) load_cin(pg);
#pragma unroll
            for (int j = 0; j < kCinAhead; ++j) {
                const int p = pg + j;
                const int c = 2 * p + cl;
                const int col = col_of(p);
                const f32x4_t v = *(const f32x4_t*)(stg + c * kWideCP + rl);
                const bool colok = col < Q;
                const bool full = colok && row + 4 <= R;
                const int vo = (int)(((int64_t)col * ldc + row) * 4);
                const f32x4_t ci = cin ? civ[j] : (f32x4_t){0.0f, 0.0f, 0.0f, 0.0f};
                f32x4_t x;
#pragma unroll
                for (int r = 0; r < 4; ++r) x[r] = cin ? fmaf(as, v[r], ea->beta * ci[r]) : as * v[r];
                if (MODE == 1 && sums) {
                    // row sums here; column sums here only with C_in (without,
                    // they were taken from the accumulators before staging)
                    double s = 0.0, sc = 0.0, sca = 0.0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const bool ok = colok && row + r < R;
                        const double xv = ok ? (double)x[r] : 0.0;
                        s += xv;
                        rsl[r] += xv;
                        if (cin) {
                            const double cv = ok ? (double)ci[r] : 0.0;
                            sc += cv;
                            sca += fabs(cv);
                            cirl[r] += cv;
                            cial[r] += fabs(cv);
                        }
                    }
                    if (cin) {
                        s = group_sum<32>(s);
                        sc = group_sum<32>(sc);
                        sca = group_sum<32>(sca);
                        if ((lane & 31) == 0) { V.cs[wr][col] = s; V.cic[wr][col] = sc; V.cica[wr][col] = sca; }
                    }
                }
                if (store) {
                    if (vec_c && full) {
                        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, x), rc, vo, 0, 0);
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x[r]), rc,
                                                                  colok && row + r < R ? vo + 4 * r : kOOB, 0, 0);
                    }
                }
                // one column pair at a time (interleaving them needs more registers)
                __builtin_amdgcn_sched_barrier(0);
            }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (MODE == 1 && sums) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                rsl[r] += __shfl_xor(rsl[r], 32);
                if (cin) {
                    cirl[r] += __shfl_xor(cirl[r], 32);
                    cial[r] += __shfl_xor(cial[r], 32);
                }
                if (lane < 32) {
                    V.rs[wc][row + r] = rsl[r];
                    if (cin) { V.cir[wc][row + r] = cirl[r]; V.cira[wc][row + r] = cial[r]; }
                }
            }
        }
    };
    if constexpr (MODE == 0) {
        pass(true, false);
    } else {
        if (FP8 && !cin) {
            // column sums of the final values alpha s acc over the wave's 128
            // rows, straight from the accumulators: the products are the ones
            // the pass below stores (the same binary32 multiply)
#pragma unroll
            for (int h = 0; h < FN; ++h) {
                const int col = wn0 + 32 * ((h + rot_b) & 1) + l32;
                double sh = 0.0;
#pragma unroll
                for (int g = 0; g < FM; ++g)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int rw = wm0 + 32 * ((g + rot_a) & 3) + 8 * (q / 4) + 4 * lh + q % 4;
                        sh += (rw < R && col < Q) ? (double)(as * acc[g][h][q]) : 0.0;
                    }
                sh += __shfl_xor(sh, 32);
                if (lh == 0) V.cs[wr][col] = sh;
            }
        } else if (!cin) {
            // the same for the 16 x 16 fragments
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int col = wn0 + 16 * ((h + rot_b) & 3) + l16;
                double sh = 0.0;
#pragma unroll
                for (int g = 0; g < 8; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int rw = wm0 + 16 * ((g + rot_a) & 7) + 4 * lq + r;
                        sh += (rw < R && col < Q) ? (double)(as * acc[g][h][r]) : 0.0;
                    }
                sh = quarter_sum(sh);
                if (lq == 0) V.cs[wr][col] = sh;
            }
        }
        // with beta != 0 the tile is stored by a second pass after the checks,
        // which read C_in at a located element
        const int npass = cin ? 2 : 1;
#pragma unroll 1
        for (int ps = 0; ps < npass; ++ps) {
        pass(ps == npass - 1, ps == 0);
        if (ps > 0) break;
        __syncthreads();
        const double asd = (double)as, bd = (double)ea->beta;
        double pass_ratio = 0.0;
        for (int line = tid; line < 1024; line += Cf::NT) {
            const int t = line >> 8, I = t >> 1, J = t & 1;
            const int tmc = 2 * tm + I, tnc = 2 * tn + J;
            if (tmc >= ea->tiles_m || tnc >= ea->tiles_n) continue;
            const int Rt = min(128, ea->m - 128 * tmc), Qt = min(128, ea->n - 128 * tnc);
            const bool isrow = (line & 255) < 128;
            const int xi = line & 127;
            if (xi >= (isrow ? Rt : Qt)) continue;
            double ref, ex, mag;
            if (isrow) {
                const int rw = 128 * I + xi;
                ref = V.rs[2 * J][rw] + V.rs[2 * J + 1][rw];
                double e = 0.0;
#pragma unroll
                for (int t = 0; t < Cf::PIECES; ++t) e += piece_weight(t) * (double)V.er[rw][Cf::PIECES * J + t];
                if (inj && ea->inj.target == FTG_TARGET_CHECKSUM) {
                    const InjectParams ipe = inject_of(ea);
                    Fault f2[2];
                    const int nf = slot_faults(ipe, ((uint64_t)tnc * ea->tiles_m + tmc) * ea->n_int + ea->interval,
                                               Rt, Qt, ea->plo, ea->plo + K, f2);
                    for (int q = 0; q < nf; ++q)
                        if (f2[q].row == xi) {
                            const float o = V.er[rw][Cf::PIECES * J];
                            const float nv = flip_f32(o, f2[q].bit);
                            e += piece_weight(0) * ((double)nv - (double)o);
                            push_inject(ea->rep, ea->problem, tmc, tnc, ea->interval, m0 + rw, -1, f2[q].pflip, f2[q].bit,
                                        FTG_TARGET_CHECKSUM, (double)o, (double)nv);
                        }
                }
                ex = asd * e;
                mag = fabs(asd) * (double)ea->RA[m0 + rw] * (double)ea->MB[tnc];
                if (cin) {
                    ex += bd * (V.cir[2 * J][rw] + V.cir[2 * J + 1][rw]);
                    mag += fabs(bd) * (V.cira[2 * J][rw] + V.cira[2 * J + 1][rw]);
                }
            } else {
                const int cw = 128 * J + xi;
                ref = V.cs[I][cw];
                double e = 0.0;
#pragma unroll
                for (int t = 0; t < Cf::PIECES; ++t) e += piece_weight(t) * (double)V.ec[cw][Cf::PIECES * I + t];
                ex = asd * e;
                mag = fabs(asd) * (double)ea->CB[n0 + cw] * (double)ea->MA[tmc];
                if (cin) { ex += bd * V.cic[I][cw]; mag += fabs(bd) * V.cica[I][cw]; }
            }
            const double d = ref - ex;
            const double tau = tau_of(1, ea->lambda, (int64_t)(K + (isrow ? Qt : Rt) + 8), mag);
            if (flagged(d, tau)) {
                if (isrow) {
                    if (atomicAdd(&V.nfr[t], 1) == 0) { V.fi[t] = xi; V.dfi[t] = d; V.tfi[t] = tau; V.exi[t] = ex; }
                } else {
                    if (atomicAdd(&V.nfc[t], 1) == 0) { V.fj[t] = xi; V.dfj[t] = d; V.tfj[t] = tau; V.exj[t] = ex; }
                }
            } else if (tau > 0.0) {
                pass_ratio = fmax(pass_ratio, fabs(d) / tau);
            }
        }
        note_pass_ratio(ea->rep, pass_ratio);
        __syncthreads();
        if (tid < 4) {
            const int t = tid, I = t >> 1, J = t & 1;
            const int tmc = 2 * tm + I, tnc = 2 * tn + J;
            const int nr = V.nfr[t], nc = V.nfc[t];
            if (tmc < ea->tiles_m && tnc < ea->tiles_n && (nr != 0 || nc != 0)) {
                RepairReq q;
                q.problem = ea->problem; q.tm = tmc; q.tn = tnc; q.interval = ea->interval;
                q.nr = nr; q.nc = nc; q.fi = V.fi[t]; q.fj = V.fj[t];
                q.R = min(128, ea->m - 128 * tmc); q.Q = min(128, ea->n - 128 * tnc);
                q.whole = q.pad1 = 0; q.m0 = 128 * (int64_t)tmc; q.n0 = 128 * (int64_t)tnc;
                q.dfi = V.dfi[t]; q.tfi = V.tfi[t]; q.dfj = V.dfj[t]; q.tfj = V.tfj[t];
                q.exp_row = nr ? V.exi[t] : 0.0;
                q.exp_col = nc ? V.exj[t] : 0.0;
                q.cin = (cin && nr == 1 && nc == 1) ? (double)ea->C[(q.m0 + q.fi) + (q.n0 + q.fj) * ldc] : 0.0;
                push_repair(ea->rep, q);
            }
        }
        __syncthreads();  // C_in at the located elements is read before the stores
        }
    }
}

template <bool FP8, int MODE>
hipError_t launch_lowp_wide_t(const LowpArgs& a, hipStream_t s)
{
    const int wt = ((a.tiles_m + 1) / 2) * ((a.tiles_n + 1) / 2);
    hipLaunchKernelGGL((lowp_wide_kernel<FP8, MODE>), dim3(wt), dim3(512), 0, s, a);
    return hipGetLastError();
}

}  // namespace ftg
