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
// checksum updates reuse operand panels already staged for the product):
//   row checksums A_I (B_J e):  the bf16 pieces of B_J e for the two tile
//       columns of the workgroup ride along as six extra rows of the B stage,
//       multiplied by the staged A fragments;
//   column checksums (e^T A_I) B_J: the pieces of e^T A_I as six extra rows of
//       the A stage, multiplied by the staged B fragments.
// A wave adds two such MFMAs of each kind per k-step (32 + 4 in all), in FP32
// accumulation like the data path.
#pragma once
#include "lowp_kernel.hpp"

namespace ftg {

template <bool FP8>
struct WCfg {
    static constexpr int EB = FP8 ? 1 : 2;                   // bytes per element
    static constexpr int BM = 256, BN = 256, BK = 64 / EB;   // 64-byte k-block rows
    static constexpr int NT = 512;                           // eight waves: 2 (m) x 4 (n)
    static constexpr int WM = 128, WN = 64;
    static constexpr int ROWB = 64;
    static constexpr int A_BYTES = BM * ROWB, B_BYTES = BN * ROWB;  // 16 KB each
    static constexpr int X_BYTES = 1024;                             // checksum-piece rows
    static constexpr int NSTAGE = 4;
    static constexpr int LPW = (A_BYTES + B_BYTES) / 1024 / 8;       // wave loads per stage
};

// 16-byte chunk c of LDS row r is stored at chunk c ^ wide_swz(r): a 16-lane
// fragment read (rows r0 .. r0 + 15, one chunk) then touches every bank once
// per pair of rows.
__device__ __attribute__((always_inline)) inline int wide_swz(int r) { return (r >> 1) & 3; }

template <bool FP8, int MODE>
__global__ __launch_bounds__(512, 1) void lowp_wide_kernel(LowpArgs args)
{
    using Cf = WCfg<FP8>;
    constexpr int BM = Cf::BM, BN = Cf::BN, BK = Cf::BK, NS = Cf::NSTAGE;
    constexpr int STAGE = Cf::A_BYTES + Cf::B_BYTES + (MODE == 1 ? Cf::X_BYTES : 0);
    __shared__ __attribute__((aligned(16))) unsigned char smem[NS * STAGE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave >> 2, wc = wave & 3;
    const int wm0 = wr * Cf::WM, wn0 = wc * Cf::WN;
    const int l16 = lane & 15, lq = lane >> 4;

    // wide tiles: (tiles_m + 1) / 2 x (tiles_n + 1) / 2 of the 128 x 128 tiles
    const int wtm = (args.tiles_m + 1) >> 1, wtn = (args.tiles_n + 1) >> 1;
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, wtm, wtn, 4, &tm, &tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int R = (int)min((int64_t)BM, (int64_t)args.m - m0);
    const int Q = (int)min((int64_t)BN, (int64_t)args.n - n0);
    const int nkb = args.k / BK;
    const int64_t lda = args.lda, ldb = args.ldb;
    const unsigned char* A = (const unsigned char*)args.A;
    const unsigned char* B = (const unsigned char*)args.B;

    // ---- staging: per stage 16 wave loads of A rows then 16 of B rows, four
    // per wave; wave load I covers rows 16 I .. 16 I + 15 (slot = 64 I + lane,
    // row = slot / 4, chunk = slot % 4, stored at chunk ^ wide_swz(row)).
    // Rows past the matrix load its last row: they only feed accumulators
    // that are never stored or checked.
    int voff[Cf::LPW];
#pragma unroll
    for (int u = 0; u < Cf::LPW; ++u) {
        const int I = wave * Cf::LPW + u;
        const int J = I & 15, sl = 64 * J + lane, x = sl >> 2;
        const int c = (sl & 3) ^ wide_swz(x);
        voff[u] = I < 16 ? (int)((int64_t)min(x, R - 1) * lda * Cf::EB + 16 * c)
                         : (int)((int64_t)min(x, Q - 1) * ldb * Cf::EB + 16 * c);
    }
    const bool a_wave = wave < 4;  // waves 0-3 load A, 4-7 load B
    const unsigned char* src0 = a_wave ? A + m0 * lda * Cf::EB : B + n0 * ldb * Cf::EB;
    auto issue = [&](int kb, int st) __attribute__((always_inline)) {
        unsigned char* base = smem + st * STAGE + (a_wave ? 0 : Cf::A_BYTES);
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(src0 + (int64_t)kb * 64);
#pragma unroll
        for (int u = 0; u < Cf::LPW; ++u) lds_dma16(rs, base + 1024 * ((wave * Cf::LPW + u) & 15), voff[u]);
    };

    f32x4_t acc[8][4];
#pragma unroll
    for (int g = 0; g < 8; ++g)
#pragma unroll
        for (int h = 0; h < 4; ++h) acc[g][h] = (f32x4_t){0.0f, 0.0f, 0.0f, 0.0f};

    // fragment read offset inside a row: chunk lq, swizzled by the row (l16)
    const int fo = 16 * (lq ^ wide_swz(l16));
    // A fragments: one set, each refilled with the next block's as soon as
    // its four MFMAs are issued; B fragments: two sets (every MFMA of a block
    // reads all four)
    bf16x8_t fa[8], fb[2][4];
    auto a_frag = [&](int st, int g) __attribute__((always_inline)) {
        return *(const bf16x8_t*)(smem + st * STAGE + (wm0 + 16 * g + l16) * 64 + fo);
    };
    auto read_b = [&](int st, bf16x8_t* b) __attribute__((always_inline)) {
        const unsigned char* tb = smem + st * STAGE + Cf::A_BYTES;
#pragma unroll
        for (int h = 0; h < 4; ++h) b[h] = *(const bf16x8_t*)(tb + (wn0 + 16 * h + l16) * 64 + fo);
    };
    // MFMAs of the current block; with st >= 0 each A fragment is then
    // replaced by that of the block in stage st
    auto mfmas = [&](const bf16x8_t* b, int st) __attribute__((always_inline)) {
#pragma unroll
        for (int g = 0; g < 8; ++g) {
#pragma unroll
            for (int h = 0; h < 4; ++h)
                acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[g], b[h], acc[g][h], 0, 0, 0);
            if (st >= 0) fa[g] = a_frag(st, g);
            // keep the written order: the scheduler would otherwise sink the
            // reads below the last MFMAs and expose their latency
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // ---- k loop over the ring, software-pipelined: block kb + 1's fragments
    // are read while block kb's MFMAs run.  The wait for block kb + 1 (its
    // loads by every wave, then a barrier) also retires every wave's reads of
    // block kb, whose stage then takes the load of block kb + NS: NS - 1
    // blocks stay in flight.
    auto sync_for = [&](int kb) __attribute__((always_inline)) {
        const int later = min(nkb - 1, kb + NS - 2) - kb;
        asm volatile("" ::: "memory");
        static_assert(2 * Cf::LPW <= 15, "vmcnt field");
        if (later >= 2) __builtin_amdgcn_s_waitcnt(0x70 | (2 * Cf::LPW));
        else if (later == 1) __builtin_amdgcn_s_waitcnt(0x70 | Cf::LPW);
        else __builtin_amdgcn_s_waitcnt(0x70);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    // one k-block with a successor.  (The loop below keeps this body free of
    // branches around LDS reads: the compiler's wait insertion merges states
    // at such joins and would then wait for the fragments just requested.)
    auto step = [&](int kb, bf16x8_t* cb, bf16x8_t* nb) __attribute__((always_inline)) {
        sync_for(kb + 1);
        // the wait above retired the reads of this block's fragments; pass
        // them through an empty asm so that no wait for them is placed after
        // the next block's reads
#pragma unroll
        for (int g = 0; g < 8; ++g) asm volatile("" : "+v"(fa[g]));
#pragma unroll
        for (int h = 0; h < 4; ++h) asm volatile("" : "+v"(cb[h]));
        if (kb + NS < nkb) issue(kb + NS, kb % NS);
        read_b((kb + 1) % NS, nb);
        __builtin_amdgcn_sched_barrier(0);
        mfmas(cb, (kb + 1) % NS);
    };
#pragma unroll 1
    for (int b = 0; b < NS && b < nkb; ++b) issue(b, b);
    // block 0: this wave's loads of blocks 1 .. NS - 1 may stay in flight
    {
        const int later = min(nkb - 1, NS - 1);
        asm volatile("" ::: "memory");
        static_assert(3 * Cf::LPW <= 15, "vmcnt field");
        if (later >= 3) __builtin_amdgcn_s_waitcnt(0x70 | (3 * Cf::LPW));
        else if (later == 2) __builtin_amdgcn_s_waitcnt(0x70 | (2 * Cf::LPW));
        else if (later == 1) __builtin_amdgcn_s_waitcnt(0x70 | Cf::LPW);
        else __builtin_amdgcn_s_waitcnt(0x70);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int g = 0; g < 8; ++g) fa[g] = a_frag(0, g);
    read_b(0, fb[0]);
#pragma unroll 1
    for (int kb = 0; kb + 1 < nkb; ++kb) {
        step(kb, fb[0], fb[1]);
#pragma unroll
        for (int h = 0; h < 4; ++h) fb[0][h] = fb[1][h];
    }
    mfmas(fb[0], -1);

    // ---- epilogue.  Lane (lq, l16) of fragment (g, h) holds rows
    // wm0 + 16 g + 4 lq + (0 .. 3) of column wn0 + 16 h + l16.  Column-major C
    // takes the tile through LDS, 16 columns of a wave at a time: each store
    // then writes two whole 512-byte column runs (the fragment layout would
    // scatter every store over 16 columns, one ldc apart).
    const int64_t ldc = args.ldc;
    const float as = args.alpha * (args.scale_a ? *args.scale_a : 1.0f) * (args.scale_b ? *args.scale_b : 1.0f);
    const bool cin = args.beta != 0.0f;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(args.C + m0 + n0 * ldc);
    const bool vec_c = args.vec_c;
    constexpr int CP = 132;  // LDS floats per staged column (128 rows + 4: conflict-free)
    float* stg = (float*)smem + wave * (16 * CP);
    // the lane's rows and column pair in the staged layout
    const int rl = 4 * (lane & 31), cl = lane >> 5;
    const int row = wm0 + rl;
    __syncthreads();  // every wave is done with the ring
#pragma unroll
    for (int h = 0; h < 4; ++h) {
#pragma unroll
        for (int g = 0; g < 8; ++g) *(f32x4_t*)(stg + l16 * CP + 16 * g + 4 * lq) = acc[g][h];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int c = 2 * p + cl;
            const int col = wn0 + 16 * h + c;
            f32x4_t v = *(const f32x4_t*)(stg + c * CP + rl);
            const bool colok = col < Q;
            const int vo = (int)(((int64_t)col * ldc + row) * 4);
            if (vec_c && colok && row + 4 <= R) {
                if (cin) {
                    const u32x4_t ci = __builtin_amdgcn_raw_buffer_load_b128(rc, vo, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = fmaf(as, v[r], args.beta * __uint_as_float(ci[r]));
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = as * v[r];
                }
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), rc, vo, 0, 0);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int o = colok && row + r < R ? vo + 4 * r : kOOB;
                    float x = as * v[r];
                    if (cin) x = fmaf(as, v[r], args.beta * __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rc, o, 0, 0)));
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), rc, o, 0, 0);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
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
