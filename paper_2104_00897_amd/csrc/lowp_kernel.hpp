// Low-precision (BF16 or FP8-e4m3 operands, FP32 accumulation) GEMM kernels for
// gfx950 and the checksum machinery of the protected variant.
//
// The protected product C := alpha s_A s_B op(A) op(B) + beta C runs as:
//   encode     one pass over A and B: for every output-tile panel the checksum
//              row e^T A_I and column B_J e of the encoded operands (§2.1),
//              kept as three bf16 pieces whose sum is the binary64 value to
//              2^-24 relative, plus the magnitude sums of the threshold;
//   checksum   the maintained checksums A_I (B_J e) and (e^T A_I) B_J of every
//   products   tile as two thin MFMA GEMMs against those pieces (FP32
//              accumulation, like the data path);
//   main GEMM  v_mfma_f32_16x16x32_{bf16,fp8}, and in its epilogue the
//              reference sums of the stored FP32 tile in binary64 (§5.2),
//              compared with the expected sums; flagged tiles are queued for
//              the repair kernel (locate, subtract, recompute; §5.1, §6.3).
// On this chip the 16x16x32 bf16 MFMA retires 512 multiply-adds per cycle per
// SIMD against 16 lanes of FP32 vector arithmetic, so summing the staged
// panels inside the k loop (as the FP64 kernel does) would cost more than the
// product itself; the encode is one memory-bound pass instead and the checksum
// updates ride on the matrix cores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <utility>

#include "ftg_common.hpp"
#include "ftg_lowp.hpp"

namespace ftg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));


// OCP e4m3fn code -> bf16 bits (exact: 3 mantissa bits fit in 7, exponent
// 2^-9 .. 2^8 fits in bf16's range).
__host__ __device__ inline uint16_t e4m3_to_bf16(uint32_t q)
{
    const uint32_t s = (q & 0x80u) << 8, e = (q >> 3) & 0xFu, f = q & 7u;
    if (e == 0xFu && f == 7u) return (uint16_t)(s | 0x7FC0u);  // NaN
    if (e != 0) return (uint16_t)(s | ((e + 120u) << 7) | (f << 4));
    if (f == 0) return (uint16_t)s;
    // subnormal f * 2^-9: normalise
    int sh = 0;
    uint32_t mm = f;
    while (!(mm & 4u)) { mm <<= 1; ++sh; }
    return (uint16_t)(s | ((118u + 2u - (uint32_t)sh) << 7) | ((mm & 3u) << 5));
}

__host__ __device__ inline float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

// value of a stored element as binary32 (exact)
template <typename ST>
__device__ inline float st_to_f32(uint32_t raw)
{
    if constexpr (ST::bytes == 2) return bf16_bits_to_f32(raw);
    else return bf16_bits_to_f32(e4m3_to_bf16(raw));
}

// binary32 -> bf16 bits, round to nearest even (finite inputs)
__device__ inline uint16_t f32_to_bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// binary64 -> e4m3fn code, round to nearest even, for abs(x) <= 448 (the
// largest finite e4m3fn value; bias 7, 3 mantissa bits, subnormals k 2^-9)
__device__ inline uint32_t f64_to_e4m3_rne(double x)
{
    const uint32_t sgn = x < 0.0 ? 0x80u : 0u;
    const double a = fabs(x);
    if (a == 0.0) return sgn;
    int e2;
    (void)frexp(a, &e2);
    int E = e2 - 1;  // a in [2^E, 2^(E+1))
    if (E < -6) {
        const double m = rint(a * 512.0);  // subnormal steps of 2^-9 (8 steps: the smallest normal)
        return sgn | (uint32_t)m;
    }
    double m = rint(ldexp(a, 3 - E));  // 8 .. 16
    if (m >= 16.0) { m = 8.0; ++E; }
    return sgn | ((uint32_t)(E + 7) << 3) | ((uint32_t)m - 8u);
}

// The same rounding, also giving the code's value (exact in binary64): for
// abs(x) <= 448, *val = the e4m3fn value nearest x (ties to even)
__device__ inline uint32_t f64_to_e4m3_rne(double x, double* val)
{
    const uint32_t sgn = x < 0.0 ? 0x80u : 0u;
    const double a = fabs(x);
    if (a == 0.0) { *val = 0.0; return sgn; }
    int e2;
    (void)frexp(a, &e2);
    int E = e2 - 1;
    if (E < -6) {
        const double m = rint(a * 512.0);
        *val = copysign(m * 0x1p-9, x);
        return sgn | (uint32_t)m;
    }
    double m = rint(ldexp(a, 3 - E));
    if (m >= 16.0) { m = 8.0; ++E; }
    *val = copysign(ldexp(m, E - 3), x);
    return sgn | ((uint32_t)(E + 7) << 3) | ((uint32_t)m - 8u);
}

// binary64 -> binary32 rounded towards +infinity (for magnitude bounds, x >= 0)
__device__ inline float f64_to_f32_up(double x)
{
    float f = (float)x;
    if ((double)f < x) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

// ---------------------------------------------------------------- GEMM
// RING: both operands k-contiguous; k-blocks of BK steps go straight from
// memory to a ring of four LDS stages (three blocks in flight, two workgroups
// per CU) in the stored type: 64-byte rows for bf16 (BK = 32) and for fp8 on
// the fp8 MFMA (BK = 64); an fp8 operand of a bf16 product (the fp8 checksum
// products) keeps 32-byte rows and is widened to bf16 exactly when its
// fragments are read.  Ring rows are not padded: 16-byte chunk c of row r sits
// at chunk c ^ ring_swz(r), chosen per row size and fragment read width;
// measured, the swizzles keep the reads free of bank conflicts, while padded
// 80-byte rows cost four conflict cycles per 16-byte read.
template <int ROWB, int W>
__device__ __attribute__((always_inline)) inline int ring_swz(int r)
{
    if constexpr (ROWB == 64) return (r >> (W == 16 ? 1 : 2)) & 3;
    else return (r >> 3) & 1;
}

template <typename STA, typename STB, bool F8MMA, bool TA, bool TB, bool RING = false>
struct LCfg {
    static constexpr int MB = F8MMA ? 1 : 2;              // bytes of an MFMA operand element
    static constexpr int BM = 128, BN = 128, BK = RING ? 64 / MB : 64;
    static constexpr int NSTAGE = RING ? 4 : 2;
    static constexpr int NT = 256, WGM = 2, WGN = 2;
    static constexpr int WM = 64, WN = 64, FM = 4, FN = 4;
    static constexpr bool SWZ = RING;                       // swizzled, unpadded rows
    static constexpr int PITCH = BK * MB + (SWZ ? 0 : 16);  // LDS row pitch in bytes (16-byte aligned rows)
    // LDS rows of A and B: the MFMA type, or in the ring the stored type
    static constexpr int PA = RING ? BK * STA::bytes : PITCH, PB = RING ? BK * STB::bytes : PITCH;
    static constexpr bool CVA = RING && !F8MMA && STA::bytes == 1;  // fp8 widened at the fragment read
    static constexpr bool CVB = RING && !F8MMA && STB::bytes == 1;
    static constexpr int WA = (F8MMA || CVA) ? 8 : 16, WB = (F8MMA || CVB) ? 8 : 16;  // fragment read bytes
    static constexpr int A_BYTES = BM * PA, B_BYTES = BN * PB;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int LA = A_BYTES / 1024, LB = B_BYTES / 1024;  // ring: wave loads per stage
    static constexpr int LPW = (LA + LB) / 4;                        // ring: loads per wave per stage
    static_assert(!RING || (TA && !TB && (STA::bytes == MB || CVA) && (STB::bytes == MB || CVB) &&
                            !(CVA && CVB) && (LA + LB) % 4 == 0), "ring staging");
    // operand staging: k-contiguous rows (A with TA=1, B with TB=0) or not
    static constexpr bool AKC = TA, BKC = !TB;
    // k-contiguous: 16-byte loads along k; otherwise each thread stages an
    // 8-row x 4-step block (four loads of 8 consecutive rows) and transposes it
    // in registers, so that every LDS row is written with one 4-step store
    static constexpr int VA = AKC ? 16 / STA::bytes : 8, VB = BKC ? 16 / STB::bytes : 8;
    static constexpr int NVA = AKC ? BM * BK / VA / NT : 4, NVB = BKC ? BN * BK / VB / NT : 4;
    static_assert(NVA >= 1 && NVB >= 1, "staging split");
    static_assert(AKC || (BM / 8) * (BK / 4) == NT, "column staging map");
    static_assert(BKC || (BN / 8) * (BK / 4) == NT, "column staging map");
};

// Writes one 16-byte load of k-contiguous stored elements (row r, steps p ..)
// to the k-contiguous LDS tile of the MFMA type (fp8 staged as bf16 when the
// product runs on the bf16 MFMA).
template <typename ST, bool F8MMA, int PITCH, bool RAW = false>
__device__ __attribute__((always_inline)) inline void lds_put16(unsigned char* tile, int r, int p, const u32x4_t v)
{
    if constexpr (RAW || F8MMA || ST::bytes == 2) {
        // the stored type (the MFMA type unless RAW keeps fp8 for a bf16 product)
        *(u32x4_t*)(tile + r * PITCH + p * ST::bytes) = v;
    } else {
        uint16_t h[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) h[e] = e4m3_to_bf16((v[e / 4] >> (8 * (e % 4))) & 0xFFu);
        u32x4_t w0, w1;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            w0[d] = (uint32_t)h[2 * d] | ((uint32_t)h[2 * d + 1] << 16);
            w1[d] = (uint32_t)h[8 + 2 * d] | ((uint32_t)h[8 + 2 * d + 1] << 16);
        }
        *(u32x4_t*)(tile + r * PITCH + p * 2) = w0;
        *(u32x4_t*)(tile + r * PITCH + p * 2 + 16) = w1;
    }
}

// Writes an 8-row x 4-step block (v[q]: rows r0..r0+7 at step p0+q, storage
// type) into the k-contiguous LDS tile: one 4-step store per row.
template <typename ST, bool F8MMA, int PITCH>
__device__ __attribute__((always_inline)) inline void lds_put_cols(unsigned char* tile, int r0, int p0,
                                                                   const u32x4_t* v)
{
    auto elem = [&](int q, int e) __attribute__((always_inline)) -> uint32_t {
        if constexpr (ST::bytes == 2) return (v[q][e / 2] >> (16 * (e % 2))) & 0xFFFFu;
        else return (v[q][e / 4] >> (8 * (e % 4))) & 0xFFu;
    };
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        if constexpr (F8MMA) {
            const uint32_t w = elem(0, e) | (elem(1, e) << 8) | (elem(2, e) << 16) | (elem(3, e) << 24);
            *(uint32_t*)(tile + (r0 + e) * PITCH + p0) = w;
        } else {
            uint32_t hq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (ST::bytes == 2) hq[q] = elem(q, e);
                else hq[q] = e4m3_to_bf16(elem(q, e));
            }
            u32x2 w;
            w[0] = hq[0] | (hq[1] << 16);
            w[1] = hq[2] | (hq[3] << 16);
            *(u32x2*)(tile + (r0 + e) * PITCH + p0 * 2) = w;
        }
    }
}

// One 16-byte load per lane from global memory straight into LDS: lane l
// writes 16 bytes at dst + 16 l (lanes that do not issue write nothing).
__device__ __attribute__((always_inline)) inline void lds_dma16(__amdgpu_buffer_rsrc_t r, unsigned char* dst, int voff)
{
    typedef __attribute__((address_space(3))) void* lds_ptr;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)dst, 16, voff, 0, 0, 0);
}

// Eight e4m3fn codes (k order, lowest byte first) as bf16, exactly: every
// e4m3fn value, subnormals included, is a bf16 value.
__device__ __attribute__((always_inline)) inline bf16x8_t widen_fp8x8(u32x2 w)
{
    u32x4_t r;
    r[0] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w[0], 1.0f, false));
    r[1] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w[0], 1.0f, true));
    r[2] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w[1], 1.0f, false));
    r[3] = __builtin_bit_cast(unsigned int, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w[1], 1.0f, true));
    return __builtin_bit_cast(bf16x8_t, r);
}

// Verification bookkeeping (aliases the stage buffers after the k loop).
struct LVerify {
    double rsum[2][128], csum[2][128];
    double cir[2][128], cira[2][128], cic[2][128], cica[2][128];
    double dfi, tfi, dfj, tfj, exi, exj;
    int nfr, nfc, fi, fj;
};

// MODE 0: C := alpha scale acc + beta C (FP32 C; also the checksum products);
// MODE 1: the same, protected (injection, reference sums, flags, repair queue).
template <typename STA, typename STB, bool F8MMA, bool TA, bool TB, int MODE, bool RING>
__global__ __launch_bounds__(256, 2) void lowp_gemm_kernel(LowpArgs args)
{
    using Cf = LCfg<STA, STB, F8MMA, TA, TB, RING>;
    constexpr int BM = Cf::BM, BN = Cf::BN, BK = Cf::BK, PITCH = Cf::PITCH;
    constexpr int FM = Cf::FM, FN = Cf::FN, WM = Cf::WM, WN = Cf::WN;
    static_assert(sizeof(LVerify) <= Cf::NSTAGE * Cf::STAGE, "verify alias");

    __shared__ __attribute__((aligned(16))) unsigned char smem[Cf::NSTAGE * Cf::STAGE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / 2, wc = wave % 2;
    const int wm0 = wr * WM, wn0 = wc * WN;
    const int l16 = lane & 15, lq = lane >> 4;

    // split k (plain mode): workgroup -> (slice, tile)
    const int ntiles = args.tiles_m * args.tiles_n;
    int bid = blockIdx.x, nb = gridDim.x;
    int64_t kbeg = 0, kend = args.k;
    float* Cbase = args.C;
    if (MODE == 0 && args.ksplit > 1) {
        const int slice = bid / ntiles;
        bid -= slice * ntiles;
        nb = ntiles;
        const int64_t kchunk = ((args.k + args.ksplit - 1) / args.ksplit + BK - 1) / BK * BK;
        kbeg = min((int64_t)args.k, (int64_t)slice * kchunk);
        kend = min((int64_t)args.k, kbeg + kchunk);
        Cbase += slice * args.cslice;
    }
    int tm, tn;
    tile_of_block(bid, nb, args.tiles_m, args.tiles_n, 4, &tm, &tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int R = (int)min((int64_t)BM, (int64_t)args.m - m0);
    const int Q = (int)min((int64_t)BN, (int64_t)args.n - n0);
    const int64_t K = kend - kbeg;
    const int nkb = (int)((K + BK - 1) / BK);
    const int64_t lda = args.lda, ldb = args.ldb;

    const typename STA::T* A = (const typename STA::T*)args.A + (Cf::AKC ? kbeg : kbeg * lda);
    const typename STB::T* B = (const typename STB::T*)args.B + (Cf::BKC ? kbeg : kbeg * ldb);

    // ---- staging map: thread t, vector q -> (row, k) of the operand tile
    auto a_rp = [&](int q, int* r, int* p) __attribute__((always_inline)) {
        const int v = tid + Cf::NT * q;
        if (Cf::AKC) { *r = v / (BK / Cf::VA); *p = (v % (BK / Cf::VA)) * Cf::VA; }
        else { *r = (tid % (BM / 8)) * 8; *p = (tid / (BM / 8)) * 4 + q; }
    };
    auto b_rp = [&](int q, int* r, int* p) __attribute__((always_inline)) {
        const int v = tid + Cf::NT * q;
        if (Cf::BKC) { *r = v / (BK / Cf::VB); *p = (v % (BK / Cf::VB)) * Cf::VB; }
        else { *r = (tid % (BN / 8)) * 8; *p = (tid / (BN / 8)) * 4 + q; }
    };
    // swizzled rows: the step whose 16-byte chunk holds step p of row r
    auto swz_a = [&](int r, int p) __attribute__((always_inline)) {
        constexpr int PER = 16 / STA::bytes;  // steps per chunk
        return ((p / PER) ^ ring_swz<Cf::PA, Cf::WA>(r)) * PER + p % PER;
    };
    auto swz_b = [&](int r, int p) __attribute__((always_inline)) {
        constexpr int PER = 16 / STB::bytes;
        return ((p / PER) ^ ring_swz<Cf::PB, Cf::WB>(r)) * PER + p % PER;
    };
    u32x4_t ra[Cf::NVA], rb[Cf::NVB];
    const bool full_a = (R == BM) && args.vec_a;
    const bool full_b = (Q == BN) && args.vec_b;

    auto load_global = [&](int kb) __attribute__((always_inline)) {
        const int64_t k0 = (int64_t)kb * BK;
        const int kv = (int)min((int64_t)BK, K - k0);
        const __amdgpu_buffer_rsrc_t rsa = make_rsrc(Cf::AKC ? A + k0 + m0 * lda : A + m0 + k0 * lda);
        const __amdgpu_buffer_rsrc_t rsb = make_rsrc(Cf::BKC ? B + k0 + n0 * ldb : B + n0 + k0 * ldb);
#pragma unroll
        for (int q = 0; q < Cf::NVA; ++q) {
            int r, p;
            a_rp(q, &r, &p);
            const int off = (int)((Cf::AKC ? p + (int64_t)r * lda : r + (int64_t)p * lda) * STA::bytes);
            if (full_a && kv == BK) {
                if (Cf::AKC || STA::bytes == 2) {
                    ra[q] = __builtin_amdgcn_raw_buffer_load_b128(rsa, off, 0, 0);
                } else {
                    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rsa, off, 0, 0);
                    ra[q] = (u32x4_t){w[0], w[1], 0u, 0u};
                }
            } else if ((Cf::AKC || STA::bytes == 2) && args.vec_a && r + (Cf::AKC ? 1 : Cf::VA) <= R &&
                       p + (Cf::AKC ? Cf::VA : 1) <= kv) {
                // a whole vector inside the matrix (edge tiles)
                ra[q] = __builtin_amdgcn_raw_buffer_load_b128(rsa, off, 0, 0);
            } else if (r >= R || p >= kv) {
                ra[q] = (u32x4_t){0u, 0u, 0u, 0u};  // entirely outside
            } else {
                // element by element, zero outside the matrix
                uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int e = 0; e < Cf::VA; ++e) {
                    const int rr = Cf::AKC ? r : r + e, pp = Cf::AKC ? p + e : p;
                    const bool ok = rr < R && pp < kv;
                    const int eo = (int)((Cf::AKC ? pp + (int64_t)rr * lda : rr + (int64_t)pp * lda) * STA::bytes);
                    uint32_t x;
                    if constexpr (STA::bytes == 2) x = __builtin_amdgcn_raw_buffer_load_b16(rsa, ok ? eo : kOOB, 0, 0);
                    else x = __builtin_amdgcn_raw_buffer_load_b8(rsa, ok ? eo : kOOB, 0, 0);
                    w[(e * STA::bytes) / 4] |= x << (8 * ((e * STA::bytes) % 4));
                }
                ra[q] = (u32x4_t){w[0], w[1], w[2], w[3]};
            }
        }
#pragma unroll
        for (int q = 0; q < Cf::NVB; ++q) {
            int r, p;
            b_rp(q, &r, &p);
            const int off = (int)((Cf::BKC ? p + (int64_t)r * ldb : r + (int64_t)p * ldb) * STB::bytes);
            if (full_b && kv == BK) {
                if (Cf::BKC || STB::bytes == 2) {
                    rb[q] = __builtin_amdgcn_raw_buffer_load_b128(rsb, off, 0, 0);
                } else {
                    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rsb, off, 0, 0);
                    rb[q] = (u32x4_t){w[0], w[1], 0u, 0u};
                }
            } else if ((Cf::BKC || STB::bytes == 2) && args.vec_b && r + (Cf::BKC ? 1 : Cf::VB) <= Q &&
                       p + (Cf::BKC ? Cf::VB : 1) <= kv) {
                rb[q] = __builtin_amdgcn_raw_buffer_load_b128(rsb, off, 0, 0);
            } else if (r >= Q || p >= kv) {
                rb[q] = (u32x4_t){0u, 0u, 0u, 0u};
            } else {
                uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int e = 0; e < Cf::VB; ++e) {
                    const int rr = Cf::BKC ? r : r + e, pp = Cf::BKC ? p + e : p;
                    const bool ok = rr < Q && pp < kv;
                    const int eo = (int)((Cf::BKC ? pp + (int64_t)rr * ldb : rr + (int64_t)pp * ldb) * STB::bytes);
                    uint32_t x;
                    if constexpr (STB::bytes == 2) x = __builtin_amdgcn_raw_buffer_load_b16(rsb, ok ? eo : kOOB, 0, 0);
                    else x = __builtin_amdgcn_raw_buffer_load_b8(rsb, ok ? eo : kOOB, 0, 0);
                    w[(e * STB::bytes) / 4] |= x << (8 * ((e * STB::bytes) % 4));
                }
                rb[q] = (u32x4_t){w[0], w[1], w[2], w[3]};
            }
        }
    };
    auto store_lds = [&](int st) __attribute__((always_inline)) {
        unsigned char* ta = smem + st * Cf::STAGE;
        unsigned char* tb = ta + Cf::A_BYTES;
        if constexpr (Cf::AKC) {
#pragma unroll
            for (int q = 0; q < Cf::NVA; ++q) {
                int r, p;
                a_rp(q, &r, &p);
                if constexpr (Cf::SWZ) p = swz_a(r, p);
                lds_put16<STA, F8MMA, Cf::PA, RING>(ta, r, p, ra[q]);
            }
        } else {
            int r, p;
            a_rp(0, &r, &p);
            lds_put_cols<STA, F8MMA, PITCH>(ta, r, p, ra);
        }
        if constexpr (Cf::BKC) {
#pragma unroll
            for (int q = 0; q < Cf::NVB; ++q) {
                int r, p;
                b_rp(q, &r, &p);
                if constexpr (Cf::SWZ) p = swz_b(r, p);
                lds_put16<STB, F8MMA, Cf::PB, RING>(tb, r, p, rb[q]);
            }
        } else {
            int r, p;
            b_rp(0, &r, &p);
            lds_put_cols<STB, F8MMA, PITCH>(tb, r, p, rb);
        }
    };

    f32x4_t acc[FM][FN];
#pragma unroll
    for (int g = 0; g < FM; ++g)
#pragma unroll
        for (int h = 0; h < FN; ++h) acc[g][h] = (f32x4_t){0.0f, 0.0f, 0.0f, 0.0f};

    // one k-block: BK/32 rank-32 MFMA steps; fragment rows read 8 consecutive k
    auto mfma_block = [&](int st) __attribute__((always_inline)) {
        const unsigned char* ta = smem + st * Cf::STAGE;
        const unsigned char* tb = ta + Cf::A_BYTES;
#pragma unroll
        for (int s = 0; s < BK / 32; ++s) {
            // byte offsets of the lane's 8 steps in an A / B row; fragment rows
            // are 16g + l16 past a multiple of 16, so the swizzle depends on l16
            int oa = (32 * s + 8 * lq) * (RING ? STA::bytes : Cf::MB);
            int ob = (32 * s + 8 * lq) * (RING ? STB::bytes : Cf::MB);
            if constexpr (Cf::SWZ) {
                oa = (((oa >> 4) ^ ring_swz<Cf::PA, Cf::WA>(l16)) << 4) | (oa & 15);
                ob = (((ob >> 4) ^ ring_swz<Cf::PB, Cf::WB>(l16)) << 4) | (ob & 15);
            }
            if constexpr (F8MMA) {
                long a[FM], b[FN];
#pragma unroll
                for (int g = 0; g < FM; ++g) a[g] = *(const long*)(ta + (wm0 + 16 * g + l16) * Cf::PA + oa);
#pragma unroll
                for (int h = 0; h < FN; ++h) b[h] = *(const long*)(tb + (wn0 + 16 * h + l16) * Cf::PB + ob);
                if constexpr (RING && MODE == 1) {
#pragma unroll
                    for (int g = 0; g < FM; ++g) asm volatile("" : "+v"(a[g]));
                }
#pragma unroll
                for (int g = 0; g < FM; ++g)
#pragma unroll
                    for (int h = 0; h < FN; ++h)
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[g], b[h], acc[g][h], 0, 0, 0);
            } else {
                bf16x8_t a[FM], b[FN];
#pragma unroll
                for (int g = 0; g < FM; ++g) {
                    const unsigned char* q = ta + (wm0 + 16 * g + l16) * Cf::PA + oa;
                    if constexpr (Cf::CVA) a[g] = widen_fp8x8(*(const u32x2*)q);
                    else a[g] = __builtin_bit_cast(bf16x8_t, *(const u32x4_t*)q);
                }
#pragma unroll
                for (int h = 0; h < FN; ++h) {
                    const unsigned char* q = tb + (wn0 + 16 * h + l16) * Cf::PB + ob;
                    if constexpr (Cf::CVB) b[h] = widen_fp8x8(*(const u32x2*)q);
                    else b[h] = __builtin_bit_cast(bf16x8_t, *(const u32x4_t*)q);
                }
                if constexpr (RING && MODE == 1) {
                    // all A fragments of the step live together: at the protected
                    // kernels' register budget the compiler would otherwise read
                    // them one at a time, each read waited for before its MFMAs
#pragma unroll
                    for (int g = 0; g < FM; ++g) asm volatile("" : "+v"(a[g]));
                }
#pragma unroll
                for (int g = 0; g < FM; ++g)
#pragma unroll
                    for (int h = 0; h < FN; ++h)
                        acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[g], b[h], acc[g][h], 0, 0, 0);
            }
        }
    };

    // ---- injection plan of this tile (one slot per tile: the whole k loop),
    // drawn by every thread (the same values in all lanes)
    const bool inj = MODE == 1 && args.inj.on;
    int flt[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    int nflt = 0;
    if (inj) {
        Fault f2[2];
        const uint64_t tile_id = (uint64_t)tn * args.tiles_m + tm;
        // the slot of this launch's verification interval: steps plo .. plo + K - 1
        nflt = __builtin_amdgcn_readfirstlane(
            slot_faults(args.inj, tile_id * args.n_int + args.interval, R, Q, args.plo, args.plo + K, f2));
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (q < nflt) {
                flt[q][0] = __builtin_amdgcn_readfirstlane(f2[q].row);
                flt[q][1] = __builtin_amdgcn_readfirstlane(f2[q].col);
                flt[q][2] = __builtin_amdgcn_readfirstlane((int)f2[q].pflip);
                flt[q][3] = __builtin_amdgcn_readfirstlane(f2[q].bit);
            }
    }
    const int fkb0 = nflt > 0 ? (int)((flt[0][2] - args.plo) / BK) : -1;
    const int fkb1 = nflt > 1 ? (int)((flt[1][2] - args.plo) / BK) : -1;
    auto apply_fault = [&](int q) __attribute__((always_inline)) {
        const int row = q ? flt[1][0] : flt[0][0];
        const int col = q ? flt[1][1] : flt[0][1];
        const int bit = q ? flt[1][3] : flt[0][3];
        const int pfl = q ? flt[1][2] : flt[0][2];
        const bool ck = args.inj.target == FTG_TARGET_CHECKSUM;
        if (ck) return;  // the checksum target is applied to the expected sum in the epilogue
        const int rr = row % WM, cc = col % WN;
        const bool own = (row / WM == wr) && (col / WN == wc) && lane == ((rr % 16) / 4) * 16 + (cc % 16);
        const int idx = ((rr / 16) * FN + cc / 16) * 4 + (rr % 4);
        float oldv = 0.0f, newv = 0.0f;
#pragma unroll
        for (int g = 0; g < FM; ++g)
#pragma unroll
            for (int h = 0; h < FN; ++h)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if ((g * FN + h) * 4 + r == idx) {
                        oldv = acc[g][h][r];
                        newv = flip_f32(oldv, bit);
                        acc[g][h][r] = own ? newv : oldv;
                    }
        if (own)
            push_inject(args.rep, args.problem, tm, tn, args.interval, m0 + row, n0 + col, pfl, bit, FTG_TARGET_ACC,
                        (double)oldv, (double)newv);
    };

    if constexpr (RING) {
        // ---- k loop over a ring of NSTAGE stages, NSTAGE - 1 blocks in flight.
        // Full k-blocks go straight to LDS: per stage LA + LB wave loads of 64
        // slots of 16 bytes, LPW per wave; slot s of an operand with S slots
        // per row holds row s / S, chunk (s % S) ^ ring_swz(row).  The k tail, and in protected mode the
        // edge tiles, stage through registers, written before the block is needed.  The
        // wait for block kb leaves the later blocks' loads in flight (an
        // explicit count), then a plain barrier publishes the stage; a
        // fenced barrier would wait for every outstanding load.
        constexpr int NS = Cf::NSTAGE;
        // plain mode: edge tiles use the ring too; rows past the matrix load
        // its last row (they only feed accumulators the epilogue never stores)
        const bool ring = MODE == 0 ? (args.vec_a && args.vec_b) : (full_a && full_b);
        const int nfull = (int)(K / BK);
        auto ring_issue = [&](int kb, int st) __attribute__((always_inline)) {
            const int64_t k0 = (int64_t)kb * BK;
            unsigned char* base = smem + st * Cf::STAGE;
#pragma unroll
            for (int u = 0; u < Cf::LPW; ++u) {
                const int I = wave * Cf::LPW + u;  // A loads 0 .. LA-1, then B loads
                if (I < Cf::LA) {
                    constexpr int SPR = Cf::PA / 16;  // 16-byte slots per row
                    const int sl = 64 * I + lane, x = sl / SPR;
                    const int c = (sl % SPR) ^ ring_swz<Cf::PA, Cf::WA>(x);
                    lds_dma16(make_rsrc(A + k0 + m0 * lda), base + 1024 * I,
                              (int)(((int64_t)min(x, R - 1) * lda) * STA::bytes + 16 * c));
                } else {
                    constexpr int SPR = Cf::PB / 16;
                    const int J = I - Cf::LA;
                    const int sl = 64 * J + lane, x = sl / SPR;
                    const int c = (sl % SPR) ^ ring_swz<Cf::PB, Cf::WB>(x);
                    lds_dma16(make_rsrc(B + k0 + n0 * ldb), base + Cf::A_BYTES + 1024 * J,
                              (int)(((int64_t)min(x, Q - 1) * ldb) * STB::bytes + 16 * c));
                }
            }
        };
        auto stage_block = [&](int kb) __attribute__((always_inline)) {
            const int st = kb % NS;
            if (ring && kb < nfull) {
                ring_issue(kb, st);
            } else {
                load_global(kb);
                store_lds(st);
            }
        };
        auto sync_for = [&](int kb) __attribute__((always_inline)) {
            // this wave's loads of later blocks (LPW per block) may stay in flight
            const int hi = min(nkb - 1, kb + NS - 2);
            const int later = ring ? max(0, min(hi, nfull - 1) - kb) : 0;
            asm volatile("" ::: "memory");
            // s_waitcnt: vmcnt = later * LPW, expcnt unconstrained, lgkmcnt = 0
            static_assert(2 * Cf::LPW <= 15, "vmcnt field");
            if (later >= 2) __builtin_amdgcn_s_waitcnt(0x70 | (2 * Cf::LPW));
            else if (later == 1) __builtin_amdgcn_s_waitcnt(0x70 | Cf::LPW);
            else __builtin_amdgcn_s_waitcnt(0x70);
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
        };
#pragma unroll 1
        for (int b = 0; b < NS - 1 && b < nkb; ++b) stage_block(b);
        for (int kb = 0; kb < nkb; ++kb) {
            sync_for(kb);
            // the stage of block kb - 1 is free: every wave is past its MFMAs
            if (kb + NS - 1 < nkb) stage_block(kb + NS - 1);
            mfma_block(kb % NS);
            if (MODE == 1) {
                if (kb == fkb0) apply_fault(0);
                if (kb == fkb1) apply_fault(1);
            }
        }
        __syncthreads();
    } else {
    // ---- k loop: stage kb+1 in registers while block kb multiplies from LDS
    load_global(0);
    store_lds(0);
    __syncthreads();
    for (int kb = 0; kb < nkb; ++kb) {
        const int st = kb & 1;
        if (kb + 1 < nkb) load_global(kb + 1);
        mfma_block(st);
        if (MODE == 1) {
            if (kb == fkb0) apply_fault(0);
            if (kb == fkb1) apply_fault(1);
        }
        if (kb + 1 < nkb) store_lds(st ^ 1);
        __syncthreads();
    }
    }

    // ---- epilogue.  Lane (lq, l16) of fragment (g, h) holds rows
    // wm0 + 16g + 4lq + r and column wn0 + 16h + l16.
    const int64_t ldc = args.ldc;
    const float as = args.alpha * (args.scale_a ? *args.scale_a : 1.0f) * (args.scale_b ? *args.scale_b : 1.0f);
    const bool cin = args.beta != 0.0f;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(Cbase + m0 + n0 * ldc);
    const int c_voff = (int)((wm0 + 4 * lq + (int64_t)(wn0 + l16) * ldc) * 4);
    const int c_hstep = (int)(16 * ldc * 4);
    const bool full_mn = R == BM && Q == BN;
    auto c_ok = [&](int g, int h, int r) __attribute__((always_inline)) {
        return full_mn || ((wm0 + 16 * g + 4 * lq + r < R) && (wn0 + 16 * h + l16 < Q));
    };
    auto c_vo = [&](int g, int r, bool ok) __attribute__((always_inline)) {
        return ok ? c_voff + (16 * g + r) * 4 : kOOB;
    };
    LVerify& V = *(LVerify*)smem;
    double csc[FN], csa[FN];
#pragma unroll
    for (int h = 0; h < FN; ++h) csc[h] = csa[h] = 0.0;
#pragma unroll
    for (int g = 0; g < FM; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double s = 0.0, sa = 0.0;
#pragma unroll
            for (int h = 0; h < FN; ++h) {
                float c = 0.0f;
                if (cin) c = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, c_vo(g, r, c_ok(g, h, r)), h * c_hstep, 0));
                acc[g][h][r] = cin ? fmaf(as, acc[g][h][r], args.beta * c) : as * acc[g][h][r];
                if (MODE == 1) {
                    s += (double)c;
                    sa += fabs((double)c);
                    csc[h] += (double)c;
                    csa[h] += fabs((double)c);
                }
            }
            if (MODE == 1 && cin) {
                s = group_sum<16>(s);
                sa = group_sum<16>(sa);
                if (l16 == 0) {
                    V.cir[wc][wm0 + 16 * g + 4 * lq + r] = s;
                    V.cira[wc][wm0 + 16 * g + 4 * lq + r] = sa;
                }
            }
        }
    if (MODE == 1) {
        if (cin) {
#pragma unroll
            for (int h = 0; h < FN; ++h) {
                const double s = quarter_sum(csc[h]), sa = quarter_sum(csa[h]);
                if (lq == 0) { V.cic[wr][wn0 + 16 * h + l16] = s; V.cica[wr][wn0 + 16 * h + l16] = sa; }
            }
        }
        // reference sums of the FP32 outputs in binary64 (§5.2)
#pragma unroll
        for (int g = 0; g < FM; ++g)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double s = 0.0;
#pragma unroll
                for (int h = 0; h < FN; ++h) s += (double)acc[g][h][r];
                s = group_sum<16>(s);
                if (l16 == 0) V.rsum[wc][wm0 + 16 * g + 4 * lq + r] = s;
            }
#pragma unroll
        for (int h = 0; h < FN; ++h) {
            double s = 0.0;
#pragma unroll
            for (int g = 0; g < FM; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) s += (double)acc[g][h][r];
            s = quarter_sum(s);
            if (lq == 0) V.csum[wr][wn0 + 16 * h + l16] = s;
        }
        if (tid == 0) { V.nfr = 0; V.nfc = 0; }
        __syncthreads();
        // expected sums: alpha s (maintained checksum) + beta (C_in sums); threshold
        // from the magnitude bound (sum_p |a_ip|) max_p (sum_j |b_pj|) (and columns alike)
        const double asd = (double)as, bd = (double)args.beta;
        double pass_ratio = 0.0;
        for (int line = tid; line < BM + BN; line += Cf::NT) {
            const bool isrow = line < BM;
            const int x = isrow ? line : line - BM;
            if (x >= (isrow ? R : Q)) continue;
            double ref, ex, mag;
            if (isrow) {
                ref = V.rsum[0][x] + V.rsum[1][x];
                const float* er = args.ER + (m0 + x) + (int64_t)(3 * tn) * args.lder;
                double e = 0.0;
                for (int sl = 0; sl < args.slices; ++sl) {
                    const float* es = er + sl * args.er_stride;
                    e += (double)es[0] + (double)es[args.lder] + (double)es[2 * args.lder];
                }
                if (inj && args.inj.target == FTG_TARGET_CHECKSUM) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int fr = q ? flt[1][0] : flt[0][0], fb = q ? flt[1][3] : flt[0][3];
                        const int fp = q ? flt[1][2] : flt[0][2];
                        if (q < nflt && fr == x) {
                            const float o = er[0];
                            const float nv = flip_f32(o, fb);
                            e += (double)nv - (double)o;
                            push_inject(args.rep, args.problem, tm, tn, args.interval, m0 + x, -1, fp, fb, FTG_TARGET_CHECKSUM,
                                        (double)o, (double)nv);
                        }
                    }
                }
                ex = asd * e;
                mag = fabs(asd) * (double)args.RA[m0 + x] * (double)args.MB[tn];
                if (cin) { ex += bd * (V.cir[0][x] + V.cir[1][x]); mag += fabs(bd) * (V.cira[0][x] + V.cira[1][x]); }
            } else {
                ref = V.csum[0][x] + V.csum[1][x];
                const float* ec = args.EC + (int64_t)(3 * tm) + (n0 + x) * args.ldec;
                double e = 0.0;
                for (int sl = 0; sl < args.slices_c; ++sl) {
                    const float* es = ec + sl * args.ec_stride;
                    e += (double)es[0] + (double)es[1] + (double)es[2];
                }
                ex = asd * e;
                mag = fabs(asd) * (double)args.CB[n0 + x] * (double)args.MA[tm];
                if (cin) { ex += bd * (V.cic[0][x] + V.cic[1][x]); mag += fabs(bd) * (V.cica[0][x] + V.cica[1][x]); }
            }
            const double d = ref - ex;
            const double tau = tau_of(1, args.lambda, (int64_t)(K + (isrow ? Q : R) + 8), mag);
            if (flagged(d, tau)) {
                if (isrow) {
                    if (atomicAdd(&V.nfr, 1) == 0) { V.fi = x; V.dfi = d; V.tfi = tau; V.exi = ex; }
                } else {
                    if (atomicAdd(&V.nfc, 1) == 0) { V.fj = x; V.dfj = d; V.tfj = tau; V.exj = ex; }
                }
            } else if (tau > 0.0) {
                pass_ratio = fmax(pass_ratio, fabs(d) / tau);
            }
        }
        note_pass_ratio(args.rep, pass_ratio);
        __syncthreads();
        const int nr = __builtin_amdgcn_readfirstlane(V.nfr);
        const int nc = __builtin_amdgcn_readfirstlane(V.nfc);
        if (nr != 0 || nc != 0) {
            if (tid == 0) {
                RepairReq q;
                q.problem = args.problem; q.tm = tm; q.tn = tn; q.interval = args.interval;
                q.nr = nr; q.nc = nc; q.fi = V.fi; q.fj = V.fj; q.R = R; q.Q = Q;
                q.whole = q.pad1 = 0; q.m0 = m0; q.n0 = n0;
                q.dfi = V.dfi; q.tfi = V.tfi; q.dfj = V.dfj; q.tfj = V.tfj;
                q.exp_row = nr ? V.exi : 0.0;
                q.exp_col = nc ? V.exj : 0.0;
                q.cin = (cin && nr == 1 && nc == 1) ? (double)args.C[(m0 + V.fi) + (n0 + V.fj) * ldc] : 0.0;
                push_repair(args.rep, q);
            }
            // C_in at the located element is read above before the tile is stored
            __syncthreads();
        }
    }
    // ---- store the tile
#pragma unroll
    for (int g = 0; g < FM; ++g)
#pragma unroll
        for (int h = 0; h < FN; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                // (by value: a bit cast of a vector element lvalue would read element 0)
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((float)acc[g][h][r]), rc,
                                                      c_vo(g, r, c_ok(g, h, r)), h * c_hstep, 0);
}

// grid: one workgroup per output tile; the four transpose cases
template <typename STA, typename STB, bool F8MMA, int MODE>
hipError_t launch_lowp_t(const LowpArgs& a, int ta, int tb, hipStream_t s)
{
    const dim3 grid(a.tiles_m * a.tiles_n * (MODE == 0 && a.ksplit > 1 ? a.ksplit : 1)), block(256);
    // fp8 product: fp8 x fp8; bf16 product: bf16 x bf16, or one fp8 operand widened at the read
    constexpr bool ring_ok = F8MMA ? (STA::bytes == 1 && STB::bytes == 1) : (STA::bytes + STB::bytes >= 3);
    if (!ta && !tb) hipLaunchKernelGGL((lowp_gemm_kernel<STA, STB, F8MMA, false, false, MODE, false>), grid, block, 0, s, a);
    else if (ta && !tb) {
        if constexpr (ring_ok) {
            if (a.vec_a && a.vec_b)
                hipLaunchKernelGGL((lowp_gemm_kernel<STA, STB, F8MMA, true, false, MODE, true>), grid, block, 0, s, a);
            else
                hipLaunchKernelGGL((lowp_gemm_kernel<STA, STB, F8MMA, true, false, MODE, false>), grid, block, 0, s, a);
        } else {
            hipLaunchKernelGGL((lowp_gemm_kernel<STA, STB, F8MMA, true, false, MODE, false>), grid, block, 0, s, a);
        }
    }
    else if (!ta && tb) hipLaunchKernelGGL((lowp_gemm_kernel<STA, STB, F8MMA, false, true, MODE, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((lowp_gemm_kernel<STA, STB, F8MMA, true, true, MODE, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace ftg
