// Host runtime of the protected GEMM: the C ABI declared in include/ftgemm.h.
//
// A handle owns the device fault report (counters, record ring, injection
// log), the batched descriptor table and the tuning table.  Entry points
// check arguments with BLAS numbering, derive the injector parameters and
// launch the kernels asynchronously on the caller's stream; nothing is
// allocated per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/ftgemm.h"
#include "ftg_kernels.hpp"
#include "ftg_lowp.hpp"
#include "ftg_batched.hpp"

namespace {

using ftg::DevReport;

// Default threshold scale of the FP32-accumulating paths (ftg_config.lambda = 0).
constexpr double kDefaultLambda = 1.0;

constexpr int kTuneBuckets = 12;  // ceil(log2) of a dimension clamped to [4, 15]
constexpr int kDtypes = 4;

}  // namespace

struct ftg_handle_s {
    int device = 0;
    DevReport* rep = nullptr;              // device
    ftg_fault_record* d_records = nullptr;  // device
    ftg_inject_record* d_inject = nullptr;  // device
    ftg::RepairReq* d_repair = nullptr;     // device repair queue
    size_t capacity = 0;
    int last_info = 0;
    // batched calls: a device table (descriptors, first-tile tables, repair
    // table) filled by one copy per call from a pinned staging area; staging
    // slots 0 and 1 alternate between eager calls, slot 2 serves stream capture
    unsigned char* d_blob = nullptr;
    unsigned char* h_blob[3] = {nullptr, nullptr, nullptr};
    hipEvent_t blob_ev[2] = {nullptr, nullptr};
    bool blob_pending[2] = {false, false};
    int next_slot = 0;
    unsigned int* d_queue = nullptr;  // work counter of the persistent launch
    int64_t batch_cap = 0;
    // workspace of the low-precision protected path (checksum pieces, checksum
    // products, magnitude bounds); grows to the largest shape seen
    unsigned char* d_work = nullptr;
    size_t work_bytes = 0;
    bool work_captured = false;  // a captured graph holds the workspace's address
    static constexpr int kMaxRetired = 64;
    unsigned char* retired[kMaxRetired] = {};  // outgrown workspaces captured graphs may still use
    int n_retired = 0;
    void* scratch = nullptr;     // device address of the scratch-free entry point's buffer
    // optional timing of the product launches: event pairs on the call's stream
    bool timing = false;
    hipEvent_t tev[2 * 256] = {};
    int tev_used = 0;  // pairs recorded since the last read
    // tuning table: configuration id per (dtype, bucket m, n, k); 0 = heuristic
    int8_t tune[kDtypes][kTuneBuckets][kTuneBuckets][kTuneBuckets];
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int bucket(int64_t x)
{
    int b = 0;
    while ((int64_t(1) << b) < x && b < 62) ++b;
    return std::min(15, std::max(4, b)) - 4;
}

int heuristic_tile_f64(int64_t m, int64_t n, int64_t k, bool need_intervals)
{
    // One workgroup per tile, 256 CUs.  The 128 x 128 tile on 8 waves runs two
    // workgroups per CU (512 at once), the 64 x 64 tile three (768).  Measured
    // (protected, 8 waves vs 64 x 64): the large tile wins once it fills the
    // chip, unless its last round of resident tiles is nearly empty (3072^3:
    // 576 tiles, the second round one eighth full); otherwise the small tile
    // wins.  The 4-wave 128 x 128 tile never won; explicit choices (config tile
    // or the tuning table) may still pick any configuration.
    auto tiles = [&](int bm, int bn) { return ((m + bm - 1) / bm) * ((n + bn - 1) / bn); };
    (void)k;
    (void)need_intervals;
    const int64_t t5 = tiles(128, 128), last = t5 % 512;
    if (t5 >= 256 && (t5 <= 512 || last == 0 || last >= 256)) return 5;
    return 3;
}

ftg_status set_err(ftg_handle h, int info)
{
    if (h) h->last_info = info;
    return FTG_ERR_INVALID_ARG;
}

uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// modular inverse of a mod S (gcd(a, S) = 1), extended Euclid
uint64_t inv_mod(uint64_t a, uint64_t S)
{
    if (S <= 1) return 0;
    int64_t t = 0, nt = 1;
    int64_t r = (int64_t)S, nr = (int64_t)(a % S);
    while (nr != 0) {
        int64_t q = r / nr;
        int64_t tmp = t - q * nt;
        t = nt;
        nt = tmp;
        tmp = r - q * nr;
        r = nr;
        nr = tmp;
    }
    if (t < 0) t += (int64_t)S;
    return (uint64_t)t;
}

// The keyed bijection of the injector's slots: slot(r) = a r + b mod S with
// a coprime to S (drawn from the seed; a = 1 if no draw of 64 is coprime).
void slot_affine(uint64_t seed, uint64_t S, uint64_t* a, uint64_t* b)
{
    *a = 1;
    *b = 0;
    if (S <= 1) return;
    *b = ftg::splitmix64(seed, 0) % S;
    for (uint64_t t = 1; t <= 64; ++t) {
        const uint64_t cand = 1 + ftg::splitmix64(seed, t) % (S - 1);
        if (gcd_u64(cand, S) == 1) {
            *a = cand;
            return;
        }
    }
}

}  // namespace

namespace ftg {

// Injector parameters for one problem with the given slot count.
// Returns false when the slot count does not fit the 32-bit slot arithmetic.
bool make_inject(const ftg_inject* in, int64_t m, int64_t n, int64_t k, int64_t slots,
                 int default_lo, int default_hi, InjectParams* ip, uint32_t faults_override,
                 bool use_override)
{
    std::memset(ip, 0, sizeof(*ip));
    if (!in) return true;
    uint64_t F = in->n_faults;
    if (use_override) F = faults_override;
    else if (F == 0 && in->per_mac_rate > 0.0)
        F = (uint64_t)std::ceil((double)m * (double)n * (double)k * in->per_mac_rate);
    if (F == 0 || slots <= 0) return true;
    if (slots >= (int64_t(1) << 32)) return false;
    const uint64_t S = (uint64_t)slots;
    uint64_t a, b;
    slot_affine(in->seed, S, &a, &b);
    ip->on = 1;
    ip->target = (int)in->target;
    ip->bit_lo = in->bit_lo;
    ip->bit_hi = in->bit_hi;
    if (ip->bit_lo == 0 && ip->bit_hi == 0) {
        ip->bit_lo = default_lo;
        ip->bit_hi = default_hi;
    }
    ip->seed = in->seed;
    ip->S = (uint32_t)S;
    ip->F = (uint32_t)std::min<uint64_t>(F, S);
    ip->a_inv = (uint32_t)inv_mod(a, S);
    ip->b = (uint32_t)b;
    return true;
}

}  // namespace ftg

// ---------------------------------------------------------------- workspace
namespace {

// Replaces the workspace by one of `bytes` (waits for the device first: the
// old buffer may still be in use by queued work).  A buffer that a captured
// graph has used is not freed but kept until the handle is destroyed, since
// the graph replays with its address.
ftg_status grow_work(ftg_handle h, size_t bytes)
{
    if (hipDeviceSynchronize() != hipSuccess) return FTG_ERR_HIP;
    if (h->d_work) {
        if (h->work_captured) {
            if (h->n_retired == ftg_handle_s::kMaxRetired) return FTG_ERR_UNSUPPORTED;
            h->retired[h->n_retired++] = h->d_work;
        } else {
            hipFree(h->d_work);
        }
    }
    h->d_work = nullptr;
    h->work_bytes = 0;
    h->work_captured = false;
    if (hipMalloc(&h->d_work, bytes) != hipSuccess) return FTG_ERR_HIP;
    h->work_bytes = bytes;
    return FTG_OK;
}

// Makes the handle's device workspace hold `bytes` for the call about to be
// queued on `s`.  Growing allocates and synchronises the device, so it is
// refused under stream capture: reserve the largest shape first.
ftg_status ensure_work(ftg_handle h, size_t bytes, hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return FTG_ERR_HIP;
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (bytes <= h->work_bytes) {
        if (capturing) h->work_captured = true;
        return FTG_OK;
    }
    if (capturing) return FTG_ERR_UNSUPPORTED;
    return grow_work(h, bytes);
}

// Scratch of the scratch-free entry point: one copy per device, held until
// the process ends.  Host code never passes `scratch` itself to a kernel (in
// host code it names a host-side stand-in); it uses the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.
ftg_status scratch_address(int device, void** out)
{
    if (device < 0 || device >= kMaxDevices) return FTG_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FTG_ERR_HIP;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return FTG_OK;
}

// Records an event pair around one product launch when timing is on (not
// under stream capture, and only while pairs are free).
struct LaunchTimer {
    ftg_handle h;
    hipStream_t s;
    int pair = -1;
    LaunchTimer(ftg_handle h_, hipStream_t s_) : h(h_), s(s_)
    {
        if (!h->timing || h->tev_used >= 256) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        pair = h->tev_used++;
        hipEventRecord(h->tev[2 * pair], s);
    }
    void end()
    {
        if (pair >= 0) hipEventRecord(h->tev[2 * pair + 1], s);
        pair = -1;
    }
};

}  // namespace

extern "C" {

const char* ftg_status_string(ftg_status s)
{
    switch (s) {
    case FTG_OK: return "ok";
    case FTG_ERR_INVALID_ARG: return "invalid argument";
    case FTG_ERR_UNSUPPORTED: return "unsupported";
    case FTG_ERR_HIP: return "HIP error";
    case FTG_ERR_UNCORRECTED: return "uncorrected fault";
    }
    return "unknown status";
}

ftg_status ftg_create(ftg_handle* out, size_t report_capacity)
{
    if (!out) return FTG_ERR_INVALID_ARG;
    *out = nullptr;
    ftg_handle h = new (std::nothrow) ftg_handle_s();
    if (!h) return FTG_ERR_HIP;
    std::memset(h->tune, 0, sizeof(h->tune));
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; return FTG_ERR_HIP; }
    h->capacity = report_capacity;
    bool ok = hipMalloc(&h->rep, sizeof(DevReport)) == hipSuccess;
    ok = ok && hipMalloc(&h->d_records, sizeof(ftg_fault_record) * std::max<size_t>(1, report_capacity)) == hipSuccess;
    ok = ok && hipMalloc(&h->d_inject, sizeof(ftg_inject_record) * std::max<size_t>(1, report_capacity)) == hipSuccess;
    // the repair queue holds the flagged slots of one call; it is independent of
    // the record capacity so that a small report still repairs every slot
    const size_t rq_cap = std::max<size_t>(report_capacity, ftg::kMinRepairQueue);
    ok = ok && hipMalloc(&h->d_repair, sizeof(ftg::RepairReq) * rq_cap) == hipSuccess;
    if (ok) {
        DevReport r;
        std::memset(&r, 0, sizeof(r));
        r.capacity = (unsigned)report_capacity;
        r.records = h->d_records;
        r.inject_log = h->d_inject;
        r.rq_capacity = (unsigned)rq_cap;
        r.rq = h->d_repair;
        ok = hipMemcpy(h->rep, &r, sizeof(r), hipMemcpyHostToDevice) == hipSuccess;
    }
    if (ok) ok = ftg_batched_reserve(h, 1024) == FTG_OK;
    if (ok) ok = scratch_address(h->device, &h->scratch) == FTG_OK;
    if (!ok) { ftg_destroy(h); return FTG_ERR_HIP; }
    *out = h;
    return FTG_OK;
}

ftg_status ftg_destroy(ftg_handle h)
{
    if (!h) return FTG_OK;
    hipDeviceSynchronize();
    if (h->rep) hipFree(h->rep);
    if (h->d_records) hipFree(h->d_records);
    if (h->d_inject) hipFree(h->d_inject);
    if (h->d_repair) hipFree(h->d_repair);
    if (h->d_blob) hipFree(h->d_blob);
    if (h->d_queue) hipFree(h->d_queue);
    if (h->d_work) hipFree(h->d_work);
    for (int i = 0; i < h->n_retired; ++i) hipFree(h->retired[i]);
    for (auto& e : h->tev)
        if (e) hipEventDestroy(e);
    for (int i = 0; i < 3; ++i)
        if (h->h_blob[i]) hipHostFree(h->h_blob[i]);
    for (int i = 0; i < 2; ++i)
        if (h->blob_ev[i]) hipEventDestroy(h->blob_ev[i]);
    delete h;
    return FTG_OK;
}

int ftg_last_error_arg(ftg_handle h) { return h ? h->last_info : 0; }

double ftg_default_lambda(void) { return kDefaultLambda; }

ftg_status ftg_tile_info(ftg_dtype ab_type, int32_t id, int32_t* bm, int32_t* bn, int32_t* bk)
{
    int a = 0, b = 0, c = 0;
    if (ab_type == FTG_F64) ftg::dgemm_tile_shape(id, &a, &b, &c);
    else if (ab_type == FTG_BF16 || ab_type == FTG_F8_E4M3) ftg::lowp_tile_shape(ab_type, id, &a, &b, &c);
    if (a == 0) return FTG_ERR_INVALID_ARG;
    if (bm) *bm = a;
    if (bn) *bn = b;
    if (bk) *bk = c;
    return FTG_OK;
}

ftg_status ftg_tune_set(ftg_handle h, ftg_dtype t, int64_t m, int64_t n, int64_t k, int32_t id)
{
    if (!h || (int)t < 0 || (int)t >= kDtypes) return FTG_ERR_INVALID_ARG;
    int32_t a, b, c;
    if (id != 0 && ftg_tile_info(t, id, &a, &b, &c) != FTG_OK) return FTG_ERR_INVALID_ARG;
    h->tune[t][bucket(m)][bucket(n)][bucket(k)] = (int8_t)id;
    return FTG_OK;
}

int32_t ftg_tune_get(ftg_handle h, ftg_dtype t, int64_t m, int64_t n, int64_t k)
{
    if (!h || (int)t < 0 || (int)t >= kDtypes) return 0;
    const int v = h->tune[t][bucket(m)][bucket(n)][bucket(k)];
    if (v) return v;
    if (t == FTG_F64) return heuristic_tile_f64(m, n, k, false);
    return ftg::lowp_heuristic_tile(t, m, n, k);
}

// Shared argument checks (BLAS xerbla numbering of dgemm).
static ftg_status check_gemm(ftg_handle h, ftg_op ta, ftg_op tb, int64_t m, int64_t n, int64_t k,
                             int64_t lda, int64_t ldb, int64_t ldc, const ftg_config* cfg)
{
    if (ta != FTG_OP_N && ta != FTG_OP_T) return set_err(h, 1);
    if (tb != FTG_OP_N && tb != FTG_OP_T) return set_err(h, 2);
    if (m < 0) return set_err(h, 3);
    if (n < 0) return set_err(h, 4);
    if (k < 0) return set_err(h, 5);
    if (lda < std::max<int64_t>(1, ta == FTG_OP_N ? m : k)) return set_err(h, 8);
    if (ldb < std::max<int64_t>(1, tb == FTG_OP_N ? k : n)) return set_err(h, 10);
    if (ldc < std::max<int64_t>(1, m)) return set_err(h, 13);
    if (cfg) {
        if (cfg->interval_k < 0 || cfg->interval_k % ftg::kKGran != 0) return set_err(h, 20);
        if (cfg->correct_policy < 0 || cfg->correct_policy > 1) return set_err(h, 20);
        if (cfg->uncorrectable_policy < 0 || cfg->uncorrectable_policy > 1) return set_err(h, 20);
        if (cfg->inject) {
            const ftg_inject* in = cfg->inject;
            if (in->target > FTG_TARGET_TWO_IN_SLOT) return set_err(h, 20);
            if (in->bit_lo < 0 || in->bit_hi < in->bit_lo) return set_err(h, 20);
            if (in->per_mac_rate < 0.0) return set_err(h, 20);
        }
    }
    return FTG_OK;
}

}  // extern "C"

namespace {

// Where the FP64 encode pass writes the checksum row/column of the operands:
// the handle's workspace (grown on demand), or a fixed buffer of `cap` bytes
// that is never grown (the scratch-free entry point).
struct EncodeBuffer {
    double* fixed = nullptr;
    size_t cap = 0;
};

// Encode-pass bytes of one FP64 call with bm x bn tiles.
size_t dencode_bytes(int64_t m, int64_t n, int64_t k, int bm, int bn)
{
    return (size_t)(((m + bm - 1) / bm) + ((n + bn - 1) / bn)) * (size_t)k * 2 * sizeof(double);
}

ftg_status dgemm_impl(ftg_handle h, ftg_op ta, ftg_op tb, int64_t m, int64_t n, int64_t k,
                      double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double beta, double* C, int64_t ldc, void* stream, const ftg_config* cfg,
                      const EncodeBuffer& eb)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    ftg_status st = check_gemm(h, ta, tb, m, n, k, lda, ldb, ldc, cfg);
    if (st != FTG_OK) return st;
    if (cfg && cfg->inject && cfg->inject->bit_hi > 63) return set_err(h, 20);
    hipStream_t s = (hipStream_t)stream;
    if (m == 0 || n == 0 || ((alpha == 0.0 || k == 0) && beta == 1.0)) return FTG_OK;
    if (alpha == 0.0 || k == 0)
        return ftg::launch_dscale(C, m, n, ldc, beta, s) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
    // 32-bit buffer offsets: every in-tile byte offset stays below 2^31
    if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31) || k >= (int64_t(1) << 31) ||
        lda >= (1 << 20) || ldb >= (1 << 20) || ldc >= (1 << 20))
        return FTG_ERR_UNSUPPORTED;

    const bool abft = !cfg || cfg->abft;
    const int64_t kc = (cfg && cfg->interval_k > 0 && cfg->interval_k < k) ? cfg->interval_k : k;
    const bool intervals = kc < k;
    int tile = cfg && cfg->tile ? cfg->tile : 0;
    if (!tile) {
        tile = h->tune[FTG_F64][bucket(m)][bucket(n)][bucket(k)];
        if (!tile || (intervals && !ftg::dgemm_tile_intervals(tile)))
            tile = heuristic_tile_f64(m, n, k, intervals);
    }
    int bm, bn, bk;
    ftg::dgemm_tile_shape(tile, &bm, &bn, &bk);
    if (bm == 0) return set_err(h, 20);
    if (abft && intervals && !ftg::dgemm_tile_intervals(tile)) return FTG_ERR_UNSUPPORTED;

    ftg::DGemmArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = A; a.B = B; a.C = C;
    a.lda = (int)lda; a.ldb = (int)ldb; a.ldc = (int)ldc;
    a.m = (int)m; a.n = (int)n; a.k = (int)k;
    a.kc = (int)kc;
    a.tiles_m = (int)((m + bm - 1) / bm);
    a.tiles_n = (int)((n + bn - 1) / bn);
    a.ta = ta == FTG_OP_T; a.tb = tb == FTG_OP_T;
    a.alpha = alpha; a.beta = beta;
    a.correct_policy = cfg ? cfg->correct_policy : 0;
    a.uncorrectable_policy = cfg ? cfg->uncorrectable_policy : 0;
    a.problem = 0;
    a.rep = h->rep;
    a.bm = bm;
    a.bn = bn;
    a.lds_direct = ftg::lds_direct_ok(A, lda, B, ldb);
    const int64_t n_int = (k + kc - 1) / kc;
    if (abft && cfg && cfg->inject) {
        if (n_int > ftg::kMaxIntervals) return FTG_ERR_UNSUPPORTED;
        const int64_t slots = (int64_t)a.tiles_m * a.tiles_n * n_int;
        if (!ftg::make_inject(cfg->inject, m, n, k, slots, 40, 63, &a.inj, 0, false))
            return FTG_ERR_UNSUPPORTED;
    }
    if (abft && !(cfg && cfg->encode_in_loop)) {
        // encode pass: checksum row/column of both operands for every tile panel
        // (every entry is written, so the buffer needs no clearing)
        const size_t bytes = dencode_bytes(m, n, k, bm, bn);
        double* w;
        if (eb.fixed) {
            if (bytes > eb.cap) return FTG_ERR_UNSUPPORTED;
            w = eb.fixed;
        } else {
            if ((st = ensure_work(h, bytes, s)) != FTG_OK) return st;
            w = (double*)h->d_work;
        }
        ftg::DEncArgs e;
        std::memset(&e, 0, sizeof(e));
        const int chunks = (int)((k + ftg::kDEncChunk - 1) / ftg::kDEncChunk);
        e.op[0] = ftg::DEncOperand{A, lda, (int)m, (int)k, ta == FTG_OP_T, bm, a.tiles_m, chunks, w};
        e.op[1] = ftg::DEncOperand{B, ldb, (int)n, (int)k, tb == FTG_OP_N, bn, a.tiles_n, chunks,
                                   w + (size_t)a.tiles_m * k * 2};
        if (ftg::launch_dencode(e, std::max(a.tiles_m, a.tiles_n) * chunks, s) != hipSuccess) return FTG_ERR_HIP;
        a.asp = e.op[0].out;
        a.bsp = e.op[1].out;
    }
    LaunchTimer timer(h, s);
    hipError_t e = ftg::launch_dgemm(a, tile, abft, s);
    timer.end();
    if (e == hipSuccess && abft) {
        ftg::RepairProblem rp;
        std::memset(&rp, 0, sizeof(rp));
        rp.A = A; rp.B = B; rp.C = C;
        rp.lda = lda; rp.ldb = ldb; rp.ldc = ldc; rp.k = k;
        rp.ta = a.ta; rp.tb = a.tb; rp.correct_policy = a.correct_policy;
        rp.ab_type = FTG_F64; rp.c_type = FTG_F64;
        rp.alpha = alpha; rp.beta = beta; rp.scale_a = rp.scale_b = nullptr;
        e = ftg::launch_repair(h->rep, rp, nullptr, s);
    }
    return e == hipSuccess ? FTG_OK : FTG_ERR_HIP;
}

}  // namespace

extern "C" {

ftg_status ftg_dgemm(ftg_handle h, ftg_op ta, ftg_op tb, int64_t m, int64_t n, int64_t k,
                     double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                     double beta, double* C, int64_t ldc, void* stream, const ftg_config* cfg)
{
    return dgemm_impl(h, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream, cfg,
                      EncodeBuffer{});
}

ftg_status ftg_dgemm_noalloc(ftg_handle h, ftg_op ta, ftg_op tb, int64_t m, int64_t n, int64_t k,
                             double alpha, const double* A, int64_t lda, const double* B,
                             int64_t ldb, double beta, double* C, int64_t ldc, void* stream,
                             const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (!h->scratch) return FTG_ERR_HIP;
    return dgemm_impl(h, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream, cfg,
                      EncodeBuffer{(double*)h->scratch, kNoallocScratchBytes});
}

size_t ftg_dgemm_noalloc_max_bytes(void) { return kNoallocScratchBytes; }

ftg_status ftg_dgemm_unfused(ftg_handle h, ftg_op ta, ftg_op tb, int64_t m, int64_t n, int64_t k,
                             double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                             double beta, double* C, int64_t ldc, void* stream, const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    ftg_status st = check_gemm(h, ta, tb, m, n, k, lda, ldb, ldc, cfg);
    if (st != FTG_OK) return st;
    if (cfg && cfg->inject && cfg->inject->bit_hi > 63) return set_err(h, 20);
    if (cfg && cfg->uncorrectable_policy != 0) return FTG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (m == 0 || n == 0 || ((alpha == 0.0 || k == 0) && beta == 1.0)) return FTG_OK;
    if (alpha == 0.0 || k == 0)
        return ftg::launch_dscale(C, m, n, ldc, beta, s) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
    if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31) || k >= (int64_t(1) << 31) ||
        lda >= (1 << 20) || ldb >= (1 << 20) || ldc >= (1 << 20))
        return FTG_ERR_UNSUPPORTED;
    const bool abft = !cfg || cfg->abft;
    const int64_t kc = (cfg && cfg->interval_k > 0 && cfg->interval_k < k) ? cfg->interval_k : k;
    const int64_t n_int = (k + kc - 1) / kc;
    if (n_int >= (int64_t(1) << 20)) return FTG_ERR_UNSUPPORTED;
    int tile = cfg && cfg->tile ? cfg->tile : 0;
    if (!tile) {
        tile = h->tune[FTG_F64][bucket(m)][bucket(n)][bucket(kc)];
        if (!tile) tile = heuristic_tile_f64(m, n, kc, false);
    }
    int bm, bn, bk;
    ftg::dgemm_tile_shape(tile, &bm, &bn, &bk);
    if (bm == 0) return set_err(h, 20);

    ftg::DGemmArgs a;
    std::memset(&a, 0, sizeof(a));
    a.C = C;
    a.lda = (int)lda; a.ldb = (int)ldb; a.ldc = (int)ldc;
    a.m = (int)m; a.n = (int)n;
    a.tiles_m = (int)((m + bm - 1) / bm);
    a.tiles_n = (int)((n + bn - 1) / bn);
    a.ta = ta == FTG_OP_T; a.tb = tb == FTG_OP_T;
    a.alpha = alpha;
    a.rep = h->rep;
    a.bm = bm; a.bn = bn;
    // the product of one slab (rank-kc update) by the unprotected kernel
    auto slab_gemm = [&](int64_t p0, int64_t len, double b) {
        a.A = a.ta ? A + p0 : A + p0 * lda;
        a.B = a.tb ? B + p0 * ldb : B + p0;
        a.k = (int)len; a.kc = (int)len;
        a.beta = b;
        a.lds_direct = ftg::lds_direct_ok(a.A, lda, a.B, ldb);
        return ftg::launch_dgemm(a, tile, false, s);
    };
    if (!abft) {
        for (int64_t t = 0; t < n_int; ++t) {
            const int64_t p0 = t * kc, len = std::min(kc, k - p0);
            if (slab_gemm(p0, len, t == 0 ? beta : 1.0) != hipSuccess) return FTG_ERR_HIP;
        }
        return FTG_OK;
    }
    ftg::InjectParams ip;
    std::memset(&ip, 0, sizeof(ip));
    if (cfg && cfg->inject && !ftg::make_inject(cfg->inject, m, n, k, n_int, 40, 63, &ip, 0, false))
        return FTG_ERR_UNSUPPORTED;

    // workspace: checksum vectors, reference sums, partial sums, C_in copy, slab states
    const bool cin = beta != 0.0;
    const int64_t mx = std::max(m, n);
    size_t part = ftg::uf_rows_part_doubles(k, mx);
    part = std::max(part, ftg::uf_rows_part_doubles(mx, std::max(n, kc)));
    size_t off = 0;
    auto take = [&](size_t doubles) { const size_t at = off; off += (doubles + 31) / 32 * 32; return at; };
    const size_t o_ea = take(k), o_eaa = take(k), o_be = take(k), o_bea = take(k);
    const size_t o_er = take(m), o_mr = take(m), o_ec = take(n), o_mc = take(n);
    const size_t o_rs = take(m), o_cs = take(n);
    const size_t o_cr = take(cin ? m : 0), o_cra = take(cin ? m : 0);
    const size_t o_cc = take(cin ? n : 0), o_cca = take(cin ? n : 0);
    const size_t o_part = take(part);
    const size_t o_copy = take(cin ? (size_t)m * n : 0);
    const size_t o_st = take((size_t)n_int * 2);
    if ((st = ensure_work(h, off * sizeof(double), s)) != FTG_OK) return st;
    double* w = (double*)h->d_work;
    double *ea = w + o_ea, *eaa = w + o_eaa, *be = w + o_be, *bea = w + o_bea;
    double *er = w + o_er, *mr = w + o_mr, *ec = w + o_ec, *mc = w + o_mc, *rs = w + o_rs, *cs = w + o_cs;
    double *pw = w + o_part, *copy = cin ? w + o_copy : nullptr;
    auto* sts = (ftg::UfStatus*)(w + o_st);
    const int ita = a.ta, itb = a.tb;
    hipError_t e = ftg::uf_status_clear(sts, (int)n_int, s);
    // T_enc: e^T op(A) and op(B) e (k-vectors with their absolute sums) ...
    if (e == hipSuccess)
        e = ita ? ftg::uf_dot_rows(A, lda, k, m, nullptr, nullptr, 1.0, ea, eaa, 0, pw, s)
                : ftg::uf_dot_cols(A, lda, m, k, nullptr, nullptr, 1.0, ea, eaa, 0, nullptr, s);
    if (e == hipSuccess)
        e = itb ? ftg::uf_dot_cols(B, ldb, n, k, nullptr, nullptr, 1.0, be, bea, 0, nullptr, s)
                : ftg::uf_dot_rows(B, ldb, k, n, nullptr, nullptr, 1.0, be, bea, 0, pw, s);
    // ... and C_in e, e^T C_in (kept with a copy of C_in for recomputed elements)
    if (e == hipSuccess && cin) e = ftg::uf_dot_rows(C, ldc, m, n, nullptr, nullptr, 1.0, w + o_cr, w + o_cra, 0, pw, s);
    if (e == hipSuccess && cin)
        e = ftg::uf_dot_cols(C, ldc, m, n, nullptr, nullptr, 1.0, w + o_cc, w + o_cca, 0, nullptr, s);
    if (e == hipSuccess && cin) e = ftg::uf_copy(C, ldc, m, n, copy, s);
    if (e == hipSuccess) e = ftg::uf_fill(er, (int64_t)(o_mc + n - o_er), 0.0, s);  // er, mr, ec, mc
    ftg::UfLines Lr{rs, er, mr, cin ? w + o_cr : nullptr, cin ? w + o_cra : nullptr, beta, m, n, 0};
    ftg::UfLines Lc{cs, ec, mc, cin ? w + o_cc : nullptr, cin ? w + o_cca : nullptr, beta, n, m, 0};
    ftg::RepairProblem rp;
    std::memset(&rp, 0, sizeof(rp));
    rp.A = A; rp.B = B; rp.C = C;
    rp.lda = lda; rp.ldb = ldb; rp.ldc = ldc;
    rp.ta = ita; rp.tb = itb; rp.correct_policy = cfg ? cfg->correct_policy : 0;
    rp.ab_type = FTG_F64; rp.c_type = FTG_F64;
    rp.alpha = alpha; rp.beta = beta;
    for (int64_t t = 0; t < n_int && e == hipSuccess; ++t) {
        const int64_t p0 = t * kc, p1 = std::min(k, p0 + kc), len = p1 - p0;
        // the rank-kc update of C by the unprotected product
        if (slab_gemm(p0, len, t == 0 ? beta : 1.0) != hipSuccess) return FTG_ERR_HIP;
        // T_update: C^r += alpha op(A)[:, slab] (op(B) e)[slab], C^c += alpha (e^T op(A))[slab] op(B)[slab, :]
        e = ita ? ftg::uf_dot_cols(A + p0, lda, len, m, be + p0, bea + p0, alpha, er, mr, 1, nullptr, s)
                : ftg::uf_dot_rows(A + p0 * lda, lda, m, len, be + p0, bea + p0, alpha, er, mr, 1, pw, s);
        if (e == hipSuccess)
            e = itb ? ftg::uf_dot_rows(B + p0 * ldb, ldb, n, len, ea + p0, eaa + p0, alpha, ec, mc, 1, pw, s)
                    : ftg::uf_dot_cols(B + p0, ldb, len, n, ea + p0, eaa + p0, alpha, ec, mc, 1, nullptr, s);
        if (e == hipSuccess && ip.on) e = ftg::uf_inject(ip, C, ldc, m, n, (int)t, p0, p1, er, h->rep, s);
        // T_ref: reference row sums, checked; column sums only after a row mismatch
        Lr.pend = Lc.pend = p1;
        if (e == hipSuccess) e = ftg::uf_dot_rows(C, ldc, m, n, nullptr, nullptr, 1.0, rs, nullptr, 0, pw, s);
        if (e == hipSuccess) e = ftg::uf_verify(Lr, sts + t, 0, h->rep, s);
        if (e == hipSuccess) e = ftg::uf_dot_cols(C, ldc, m, n, nullptr, nullptr, 1.0, cs, nullptr, 0, sts + t, s);
        if (e == hipSuccess) e = ftg::uf_verify(Lc, sts + t, 1, h->rep, s);
        if (e == hipSuccess)
            e = ftg::uf_handoff(Lr, Lc, sts + t, (int)t, t == n_int - 1, copy, m, h->rep, er, s);
        rp.k = p1;
        if (e == hipSuccess) e = ftg::launch_repair(h->rep, rp, nullptr, s);
    }
    return e == hipSuccess ? FTG_OK : FTG_ERR_HIP;
}

// ---------------------------------------------------------------- FT-DSYMM, FT-DTRMM
// Both pack the symmetric or triangular operand into a dense copy at the front
// of the workspace and run the protected GEMM on it (§6.2.3: DGEMM's scheme
// with modified packing); the encode passes of those products use the rest of
// the workspace, sized up front so that nothing is reallocated in between.
static int64_t even_ld(int64_t x) { return std::max<int64_t>(2, (x + 1) / 2 * 2); }

// Upper bound of one protected product's encode-pass bytes (the smallest tile).
static size_t encode_bound(int64_t m, int64_t n, int64_t k)
{
    return dencode_bytes(m, n, k, 64, 64);
}

ftg_status ftg_dsymm(ftg_handle h, ftg_side side, ftg_uplo uplo, int64_t m, int64_t n, double alpha,
                     const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                     int64_t ldc, void* stream, const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (side != FTG_LEFT && side != FTG_RIGHT) return set_err(h, 1);
    if (uplo != FTG_LOWER && uplo != FTG_UPPER) return set_err(h, 2);
    if (m < 0) return set_err(h, 3);
    if (n < 0) return set_err(h, 4);
    const int64_t ka = side == FTG_LEFT ? m : n;
    if (lda < std::max<int64_t>(1, ka)) return set_err(h, 7);
    if (ldb < std::max<int64_t>(1, m)) return set_err(h, 9);
    if (ldc < std::max<int64_t>(1, m)) return set_err(h, 12);
    if (m == 0 || n == 0 || (alpha == 0.0 && beta == 1.0)) return FTG_OK;
    hipStream_t s = (hipStream_t)stream;
    if (alpha == 0.0) return ftg::launch_dscale(C, m, n, ldc, beta, s) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
    if (ka >= (1 << 20)) return FTG_ERR_UNSUPPORTED;
    const int64_t ldp = even_ld(ka);
    const size_t pack = align256((size_t)ldp * ka * sizeof(double));
    const size_t enc = encode_bound(m, n, ka);
    ftg_status st = ensure_work(h, pack + enc, s);
    if (st != FTG_OK) return st;
    double* Af = (double*)h->d_work;
    if (ftg::launch_pack_sym(A, lda, ka, uplo == FTG_LOWER, Af, ldp, s) != hipSuccess) return FTG_ERR_HIP;
    const EncodeBuffer eb{(double*)(h->d_work + pack), enc};
    if (side == FTG_LEFT)
        return dgemm_impl(h, FTG_OP_N, FTG_OP_N, m, n, m, alpha, Af, ldp, B, ldb, beta, C, ldc, stream, cfg, eb);
    return dgemm_impl(h, FTG_OP_N, FTG_OP_N, m, n, n, alpha, B, ldb, Af, ldp, beta, C, ldc, stream, cfg, eb);
}

ftg_status ftg_dtrmm(ftg_handle h, ftg_side side, ftg_uplo uplo, ftg_op transa, ftg_diag diag, int64_t m,
                     int64_t n, double alpha, const double* A, int64_t lda, double* B, int64_t ldb, void* stream,
                     const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (side != FTG_LEFT && side != FTG_RIGHT) return set_err(h, 1);
    if (uplo != FTG_LOWER && uplo != FTG_UPPER) return set_err(h, 2);
    if (transa != FTG_OP_N && transa != FTG_OP_T) return set_err(h, 3);
    if (diag != FTG_NON_UNIT && diag != FTG_UNIT) return set_err(h, 4);
    if (m < 0) return set_err(h, 5);
    if (n < 0) return set_err(h, 6);
    const int64_t ka = side == FTG_LEFT ? m : n;
    if (lda < std::max<int64_t>(1, ka)) return set_err(h, 9);
    if (ldb < std::max<int64_t>(1, m)) return set_err(h, 11);
    if (m == 0 || n == 0) return FTG_OK;
    hipStream_t s = (hipStream_t)stream;
    if (alpha == 0.0) return ftg::launch_dscale(B, m, n, ldb, 0.0, s) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
    if (ka >= (1 << 20) || m >= (1 << 20)) return FTG_ERR_UNSUPPORTED;
    const int64_t ldp = even_ld(ka), ldq = even_ld(m);
    const size_t pack = align256((size_t)ldp * ka * sizeof(double));
    const size_t copy = align256((size_t)ldq * n * sizeof(double));
    const size_t enc = encode_bound(m, n, ka);
    ftg_status st = ensure_work(h, pack + copy + enc, s);
    if (st != FTG_OK) return st;
    double* Af = (double*)h->d_work;
    double* Bc = (double*)(h->d_work + pack);
    if (ftg::launch_pack_tri(A, lda, ka, uplo == FTG_LOWER, diag == FTG_UNIT, Af, ldp, s) != hipSuccess)
        return FTG_ERR_HIP;
    if (ftg::uf_copy2d(B, ldb, m, n, Bc, ldq, s) != hipSuccess) return FTG_ERR_HIP;
    const EncodeBuffer eb{(double*)(h->d_work + pack + copy), enc};
    // op(A) is lower triangular when (lower, N) or (upper, T): row i of op(A) is
    // nonzero for columns p <= i only; otherwise for p >= i.  The product runs in
    // blocks of output rows (left) or columns (right) with k cut to the nonzero
    // range, which halves the multiply-adds of a dense product.
    const bool lower_eff = (uplo == FTG_LOWER) == (transa == FTG_OP_N);
    const int64_t nb = 1024;
    const int ta = transa == FTG_OP_T;
    // element (r, c) of op(Af) and its address
    auto opa = [&](int64_t r, int64_t c) { return ta ? Af + c + r * ldp : Af + r + c * ldp; };
    if (side == FTG_LEFT) {
        for (int64_t i0 = 0; i0 < m; i0 += nb) {
            const int64_t rows = std::min(nb, m - i0);
            const int64_t k0 = lower_eff ? 0 : i0, k1 = lower_eff ? i0 + rows : m;
            st = dgemm_impl(h, transa, FTG_OP_N, rows, n, k1 - k0, alpha, opa(i0, k0), ldp, Bc + k0, ldq, 0.0,
                            B + i0, ldb, stream, cfg, eb);
            if (st != FTG_OK) return st;
        }
    } else {
        for (int64_t j0 = 0; j0 < n; j0 += nb) {
            const int64_t cols = std::min(nb, n - j0);
            // column j of op(A) is nonzero for rows p >= j (lower) or p <= j (upper)
            const int64_t k0 = lower_eff ? j0 : 0, k1 = lower_eff ? n : j0 + cols;
            st = dgemm_impl(h, FTG_OP_N, transa, m, cols, k1 - k0, alpha, Bc + k0 * ldq, ldq, opa(k0, j0), ldp, 0.0,
                            B + j0 * ldb, ldb, stream, cfg, eb);
            if (st != FTG_OK) return st;
        }
    }
    return FTG_OK;
}

// ---------------------------------------------------------------- FT-DTRSM
// B := alpha op(A)^-1 B (left) or alpha B op(A)^-1 (right), blocked as in
// §3.3.3: blocks on the diagonal are solved by the checksum-verified
// diagonal kernel, every other block of the solve is an update
// B_K := -op(A)[K, D] X_D + beta B_K on the protected GEMM.  Outer blocks of
// 1024 make those updates large products; inside an outer block, inner
// blocks of 256 are solved in turn with smaller updates.  The first update
// that touches a block applies alpha (as beta); a block that no update
// touches (the very first one) gets alpha in the diagonal solve.
ftg_status ftg_dtrsm(ftg_handle h, ftg_side side, ftg_uplo uplo, ftg_op transa, ftg_diag diag, int64_t m,
                     int64_t n, double alpha, const double* A, int64_t lda, double* B, int64_t ldb, void* stream,
                     const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (side != FTG_LEFT && side != FTG_RIGHT) return set_err(h, 1);
    if (uplo != FTG_LOWER && uplo != FTG_UPPER) return set_err(h, 2);
    if (transa != FTG_OP_N && transa != FTG_OP_T) return set_err(h, 3);
    if (diag != FTG_NON_UNIT && diag != FTG_UNIT) return set_err(h, 4);
    if (m < 0) return set_err(h, 5);
    if (n < 0) return set_err(h, 6);
    const int64_t ka = side == FTG_LEFT ? m : n;
    if (lda < std::max<int64_t>(1, ka)) return set_err(h, 9);
    if (ldb < std::max<int64_t>(1, m)) return set_err(h, 11);
    if (cfg) {
        if (cfg->inject && (cfg->inject->target != FTG_TARGET_ACC || cfg->inject->bit_hi > 63 ||
                            cfg->inject->bit_lo < 0 || cfg->inject->bit_hi < cfg->inject->bit_lo))
            return set_err(h, 20);
    }
    if (m == 0 || n == 0) return FTG_OK;
    hipStream_t s = (hipStream_t)stream;
    if (alpha == 0.0) return ftg::launch_dscale(B, m, n, ldb, 0.0, s) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
    if (ka >= (int64_t(1) << 31) || lda >= (1 << 20) || ldb >= (1 << 20)) return FTG_ERR_UNSUPPORTED;
    const bool abft = !cfg || cfg->abft;
    const int64_t rhs = side == FTG_LEFT ? n : m;   // right-hand sides
    const size_t enc = encode_bound(side == FTG_LEFT ? 1024 : m, side == FTG_LEFT ? n : 1024, ka);
    // after the encode region: the column sums of the diagonal block being solved
    const size_t colsum_bytes = 2 * (size_t)ftg::trsm_diag_max_nb() * sizeof(double);
    ftg_status st = ensure_work(h, enc + colsum_bytes, s);
    if (st != FTG_OK) return st;
    const EncodeBuffer eb{(double*)h->d_work, enc};
    double* colsum = (double*)((char*)h->d_work + enc);
    const int ta = transa == FTG_OP_T;
    // op(A) lower triangular: the solve runs forward (left) / backward (right)
    const bool lower_eff = (uplo == FTG_LOWER) == (transa == FTG_OP_N);
    const bool forward = side == FTG_LEFT ? lower_eff : !lower_eff;
    auto opa = [&](int64_t r, int64_t c) { return ta ? A + c + r * lda : A + r + c * lda; };
    const int64_t NB = 1024, nbd = ftg::trsm_diag_max_nb();
    int step = 0;  // protected steps so far: each draws its own injection plan
    // a per-MAC rate applies to the whole call: each step takes the whole
    // faults its multiply-adds are due, the fraction carried to the next step
    // (rounding each step up would multiply the rate of the many small steps)
    double carry = 0.0;
    auto step_cfg = [&](ftg_config* c, ftg_inject* in, double macs) -> const ftg_config* {
        if (!cfg) return nullptr;
        *c = *cfg;
        if (cfg->inject) {
            *in = *cfg->inject;
            in->seed = ftg::splitmix64(cfg->inject->seed, (uint64_t(1) << 33) + (uint64_t)step);
            if (in->n_faults == 0 && in->per_mac_rate > 0.0) {
                const double due = macs * in->per_mac_rate + carry;
                const double f = std::floor(due);
                carry = due - f;
                in->n_faults = (uint32_t)f;
                in->per_mac_rate = 0.0;
            }
            c->inject = in->n_faults ? in : nullptr;
        }
        ++step;
        return c;
    };
    // update of the blocks in [k0, k1) by the solved range [d0, d1)
    auto update = [&](int64_t k0, int64_t k1, int64_t d0, int64_t d1, double beta) -> ftg_status {
        if (d1 <= d0) return FTG_OK;
        ftg_config c;
        ftg_inject in;
        const ftg_config* pc = step_cfg(&c, &in, (double)(k1 - k0) * (double)(d1 - d0) * (double)rhs);
        if (side == FTG_LEFT)
            return dgemm_impl(h, transa, FTG_OP_N, k1 - k0, n, d1 - d0, -1.0, opa(k0, d0), lda, B + d0, ldb, beta,
                              B + k0, ldb, stream, pc, eb);
        return dgemm_impl(h, FTG_OP_N, transa, m, k1 - k0, d1 - d0, -1.0, B + d0 * ldb, ldb, opa(d0, k0), lda, beta,
                          B + k0 * ldb, ldb, stream, pc, eb);
    };
    auto solve = [&](int64_t k0, int64_t k1, double scale, int block) -> ftg_status {
        ftg::TrsmDiag d;
        std::memset(&d, 0, sizeof(d));
        // left: M = op(A)[K, K]; right: M = op(A)[K, K]^T (rows of B solved from the right)
        d.M = A + k0 + k0 * lda;
        d.ldm = lda;
        d.nb = (int)(k1 - k0);
        d.trans = side == FTG_LEFT ? ta : !ta;
        d.lower = forward;
        d.unit = diag == FTG_UNIT;
        d.R = side == FTG_LEFT ? B + k0 : B + k0 * ldb;
        d.rs = side == FTG_LEFT ? 1 : ldb;
        d.cs = side == FTG_LEFT ? ldb : 1;
        d.count = rhs;
        d.scale = scale;
        d.rep = h->rep;
        d.block = block;
        d.verify = abft;
        d.row0 = k0;
        d.wsum = colsum;
        ftg_config c;
        ftg_inject in;
        const ftg_config* pc = step_cfg(&c, &in, 0.5 * (double)d.nb * (double)(d.nb + 1) * (double)rhs);
        if (abft && pc && pc->inject &&
            !ftg::make_inject(pc->inject, d.nb, rhs, d.nb, rhs, 40, 63, &d.inj, 0, false))
            return FTG_ERR_UNSUPPORTED;
        if (abft && ftg::launch_trsm_colsum(d, colsum, s) != hipSuccess) return FTG_ERR_HIP;
        return ftg::launch_trsm_diag(d, s) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
    };
    // blocks in solve order
    const int64_t nouter = (ka + NB - 1) / NB;
    for (int64_t oi = 0; oi < nouter; ++oi) {
        const int64_t ob = forward ? oi : nouter - 1 - oi;
        const int64_t K0 = ob * NB, K1 = std::min(ka, K0 + NB);
        // outer update by everything solved before this block
        const bool first_outer = oi == 0;
        if (!first_outer) {
            st = forward ? update(K0, K1, 0, K0, alpha) : update(K0, K1, K1, ka, alpha);
            if (st != FTG_OK) return st;
        }
        const int64_t ninner = (K1 - K0 + nbd - 1) / nbd;
        for (int64_t ii = 0; ii < ninner; ++ii) {
            const int64_t ib = forward ? ii : ninner - 1 - ii;
            const int64_t k0 = K0 + ib * nbd, k1 = std::min(K1, k0 + nbd);
            if (ii > 0) {
                // inner update by the blocks of this outer block solved so far
                const double beta = first_outer ? alpha : 1.0;
                st = forward ? update(k0, k1, K0, k0, beta) : update(k0, k1, k1, K1, beta);
                if (st != FTG_OK) return st;
            }
            const double scale = (first_outer && ii == 0) ? alpha : 1.0;
            st = solve(k0, k1, scale, (int)(k0 / nbd));
            if (st != FTG_OK) return st;
        }
    }
    return FTG_OK;
}

}  // extern "C"

namespace {

// Injector of a duplicated-computation routine: F distinct verification
// units out of S (F = n_faults, or ceil(ops * per_mac_rate)), unit r of the
// plan = a r + b mod S by the slot bijection, each with a bit in
// [bit_lo, bit_hi] (default 40..63) and a phase bit.  Empty when the routine
// runs unprotected or without injector; false when F exceeds the plan's room.
bool make_dmr_plan(const ftg_config* cfg, bool dmr, uint64_t S, double ops, ftg::DmrPlan* p)
{
    std::memset(p, 0, sizeof(*p));
    if (!dmr || !cfg || !cfg->inject || S == 0) return true;
    const ftg_inject* in = cfg->inject;
    uint64_t F = in->n_faults;
    if (F == 0 && in->per_mac_rate > 0.0) F = (uint64_t)std::ceil(ops * in->per_mac_rate);
    if (F == 0) return true;
    if (F > S) F = S;
    if (F > (uint64_t)ftg::kDmrMaxFaults) return false;
    uint64_t a, b;
    slot_affine(in->seed, S, &a, &b);
    int lo = in->bit_lo, hi = in->bit_hi;
    if (lo == 0 && hi == 0) {
        lo = 40;
        hi = 63;
    }
    for (uint64_t r = 0; r < F; ++r) {
        ftg::DmrFault& f = p->f[r];
        f.unit = (int64_t)(((unsigned __int128)a * r + b) % S);
        f.bit = lo + (int)(ftg::splitmix64(in->seed, 1024 + 8 * r + 3) % (uint64_t)(hi - lo + 1));
        f.sub = (int)(ftg::splitmix64(in->seed, 1024 + 8 * r + 4) & 1);
    }
    p->n = (int)F;
    p->target = (int)in->target;
    return true;
}

// Injector checks shared by the duplicated-computation routines.
bool dmr_inject_ok(const ftg_config* cfg)
{
    if (!cfg || !cfg->inject) return true;
    const ftg_inject* in = cfg->inject;
    return in->target <= FTG_TARGET_TWO_IN_SLOT && in->bit_lo >= 0 && in->bit_hi <= 63 &&
           in->bit_lo <= in->bit_hi && in->per_mac_rate >= 0.0;
}

// Element 0 of a BLAS vector of n elements at stride inc (for a negative
// stride, the last element in memory).
template <typename T>
T* vec_first(T* x, int64_t n, int64_t inc)
{
    return inc > 0 ? x : x + (1 - n) * inc;
}

}  // namespace

extern "C" {

ftg_status ftg_dscal(ftg_handle h, int64_t n, double alpha, double* x, int64_t incx, void* stream,
                     const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (!dmr_inject_ok(cfg)) return set_err(h, 20);
    if (n <= 0 || incx <= 0) return FTG_OK;
    if (n >= (int64_t(1) << 40) || incx >= (int64_t(1) << 20)) return FTG_ERR_UNSUPPORTED;
    const bool dmr = !cfg || cfg->abft;
    ftg::DmrPlan plan;
    if (!make_dmr_plan(cfg, dmr, (uint64_t)ftg::dmr_units_vec(n), (double)n, &plan)) return FTG_ERR_UNSUPPORTED;
    return ftg::launch_dmr_scal(x, n, incx, alpha, dmr, plan, h->rep, (hipStream_t)stream) == hipSuccess
               ? FTG_OK
               : FTG_ERR_HIP;
}

ftg_status ftg_dnrm2(ftg_handle h, int64_t n, const double* x, int64_t incx, double* result, void* stream,
                     const ftg_config* cfg)
{
    if (!h || !result) return FTG_ERR_INVALID_ARG;
    if (!dmr_inject_ok(cfg)) return set_err(h, 20);
    hipStream_t s = (hipStream_t)stream;
    if (n <= 0 || incx <= 0) return ftg::launch_dscale(result, 1, 1, 1, 0.0, s) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
    if (n >= (int64_t(1) << 40) || incx >= (int64_t(1) << 20)) return FTG_ERR_UNSUPPORTED;
    const bool dmr = !cfg || cfg->abft;
    ftg::DmrPlan plan;
    if (!make_dmr_plan(cfg, dmr, (uint64_t)ftg::dmr_units_vec(n), (double)n, &plan)) return FTG_ERR_UNSUPPORTED;
    const ftg_status st = ensure_work(h, ftg::dmr_nrm2_work_bytes(n), s);
    if (st != FTG_OK) return st;
    return ftg::launch_dmr_nrm2(x, n, incx, result, (double*)h->d_work, dmr, plan, h->rep, s) == hipSuccess
               ? FTG_OK
               : FTG_ERR_HIP;
}

ftg_status ftg_dgemv(ftg_handle h, ftg_op trans, int64_t m, int64_t n, double alpha, const double* A,
                     int64_t lda, const double* x, int64_t incx, double beta, double* y, int64_t incy,
                     void* stream, const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (trans != FTG_OP_N && trans != FTG_OP_T) return set_err(h, 1);
    if (m < 0) return set_err(h, 2);
    if (n < 0) return set_err(h, 3);
    if (lda < std::max<int64_t>(1, m)) return set_err(h, 6);
    if (incx == 0) return set_err(h, 8);
    if (incy == 0) return set_err(h, 11);
    if (!dmr_inject_ok(cfg)) return set_err(h, 20);
    if (m == 0 || n == 0 || (alpha == 0.0 && beta == 1.0)) return FTG_OK;
    if (m >= (int64_t(1) << 36) || n >= (int64_t(1) << 36) || std::abs(incx) >= (int64_t(1) << 20) ||
        std::abs(incy) >= (int64_t(1) << 20))
        return FTG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const bool dmr = !cfg || cfg->abft;
    const int ta = trans == FTG_OP_T;
    const int64_t lenx = ta ? m : n, leny = ta ? n : m;
    if (alpha == 0.0) {
        // y := beta y without reading A or x: the same elements in memory order
        // (y is the lowest address of the vector for either sign of incy)
        double* ylo = y;
        const int64_t ainc = incy > 0 ? incy : -incy;
        if (beta == 0.0) return ftg::launch_dscale(ylo, 1, leny, ainc, 0.0, s) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
        ftg::DmrPlan none;
        std::memset(&none, 0, sizeof(none));
        return ftg::launch_dmr_scal(ylo, leny, ainc, beta, dmr, none, h->rep, s) == hipSuccess ? FTG_OK
                                                                                             : FTG_ERR_HIP;
    }
    ftg::DmrPlan plan;
    if (!make_dmr_plan(cfg, dmr, (uint64_t)ftg::dmr_units_gemv(ta, m, n), (double)m * (double)n, &plan))
        return FTG_ERR_UNSUPPORTED;
    const ftg_status st = ensure_work(h, ftg::dmr_gemv_work_bytes(ta, m, n), s);
    if (st != FTG_OK) return st;
    return ftg::launch_dmr_gemv(ta, m, n, alpha, A, lda, vec_first(x, lenx, incx), incx, beta,
                                vec_first(y, leny, incy), incy, (double*)h->d_work, dmr, plan, h->rep,
                                s) == hipSuccess
               ? FTG_OK
               : FTG_ERR_HIP;
}

ftg_status ftg_dtrsv(ftg_handle h, ftg_uplo uplo, ftg_op trans, ftg_diag diag, int64_t n, const double* A,
                     int64_t lda, double* x, int64_t incx, void* stream, const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (uplo != FTG_LOWER && uplo != FTG_UPPER) return set_err(h, 1);
    if (trans != FTG_OP_N && trans != FTG_OP_T) return set_err(h, 2);
    if (diag != FTG_NON_UNIT && diag != FTG_UNIT) return set_err(h, 3);
    if (n < 0) return set_err(h, 4);
    if (lda < std::max<int64_t>(1, n)) return set_err(h, 6);
    if (incx == 0) return set_err(h, 8);
    if (!dmr_inject_ok(cfg)) return set_err(h, 20);
    if (n == 0) return FTG_OK;
    if (n >= (int64_t(1) << 31) || std::abs(incx) >= (int64_t(1) << 20)) return FTG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const bool dmr = !cfg || cfg->abft;
    ftg::DmrPlan plan;
    if (!make_dmr_plan(cfg, dmr, (uint64_t)ftg::dmr_units_trsv(n), 0.5 * (double)n * (double)n, &plan))
        return FTG_ERR_UNSUPPORTED;
    const ftg_status st = ensure_work(h, ftg::dmr_trsv_work_bytes(n), s);
    if (st != FTG_OK) return st;
    const int lower_eff = (uplo == FTG_LOWER) == (trans == FTG_OP_N);
    return ftg::launch_dmr_trsv(lower_eff, trans == FTG_OP_T, diag == FTG_UNIT, n, A, lda, vec_first(x, n, incx),
                                incx, (double*)h->d_work, dmr, plan, h->rep, s) == hipSuccess
               ? FTG_OK
               : FTG_ERR_HIP;
}

ftg_status ftg_workspace_reserve(ftg_handle h, size_t bytes)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (bytes <= h->work_bytes) return FTG_OK;
    return grow_work(h, bytes);
}


// ---------------------------------------------------------------- low precision
namespace {

struct LowpLayout {
    size_t xs_a, xs_b, xs8_a, xs8_b, xrp_a, xrp_b, xmp_a, xmp_b, ra, cb, ma, mb, er, ec, total;
};

// k slices of the checksum products: enough workgroups to fill the chip twice,
// each slice at least 512 steps long
int lowp_ksplit(int64_t tiles, int64_t k)
{
    int s = (int)std::min<int64_t>(16, std::max<int64_t>(1, (512 + tiles - 1) / std::max<int64_t>(1, tiles)));
    while (s > 1 && k / s < 512) --s;
    return s;
}

LowpLayout lowp_layout(int64_t m, int64_t n, int64_t k, int ks_r, int ks_c, int64_t n_int)
{
    const int64_t tm = (m + ftg::kLowpTile - 1) / ftg::kLowpTile, tn = (n + ftg::kLowpTile - 1) / ftg::kLowpTile;
    const int64_t ch = (k + ftg::kLowpChunk - 1) / ftg::kLowpChunk;
    LowpLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.xs_a = take((size_t)(3 * tm * k) * 2);
    L.xs_b = take((size_t)(3 * tn * k) * 2);
    L.xs8_a = take((size_t)(ftg::kFp8Pieces * tm * k));
    L.xs8_b = take((size_t)(ftg::kFp8Pieces * tn * k));
    L.xrp_a = take((size_t)(ch * m) * 4);
    L.xrp_b = take((size_t)(ch * n) * 4);
    L.xmp_a = take((size_t)(tm * ch) * 4);
    L.xmp_b = take((size_t)(tn * ch) * 4);
    L.ra = take((size_t)(n_int * m) * 4);  // one set of magnitude sums per interval
    L.cb = take((size_t)(n_int * n) * 4);
    L.ma = take((size_t)(n_int * tm) * 4);
    L.mb = take((size_t)(n_int * tn) * 4);
    L.er = take((size_t)ks_r * (size_t)(m * 3 * tn) * 4);
    L.ec = take((size_t)ks_c * (size_t)(3 * tm * n) * 4);
    L.total = o;
    return L;
}

bool vec_ok(const void* p, int64_t ld, int bytes)
{
    return ((uintptr_t)p % 16 == 0) && ((ld * bytes) % 16 == 0);
}

}  // namespace

ftg_status ftg_gemm_ex(ftg_handle h, ftg_op ta, ftg_op tb, int64_t m, int64_t n, int64_t k,
                       ftg_dtype ab_type, ftg_dtype c_type, const float* scale_a,
                       const float* scale_b, float alpha, const void* A, int64_t lda,
                       const void* B, int64_t ldb, float beta, void* C, int64_t ldc,
                       void* stream, const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    ftg_status st = check_gemm(h, ta, tb, m, n, k, lda, ldb, ldc, cfg);
    if (st != FTG_OK) return st;
    if (ab_type != FTG_BF16 && ab_type != FTG_F8_E4M3) return FTG_ERR_UNSUPPORTED;
    if (c_type != FTG_F32) return FTG_ERR_UNSUPPORTED;
    if (ab_type == FTG_F8_E4M3 && (!scale_a || !scale_b)) return set_err(h, 20);
    if (cfg && cfg->inject && cfg->inject->bit_hi > 31) return set_err(h, 20);
    if (cfg && cfg->lambda < 0.0) return set_err(h, 20);
    hipStream_t s = (hipStream_t)stream;
    if (m == 0 || n == 0 || ((alpha == 0.0f || k == 0) && beta == 1.0f)) return FTG_OK;
    if (alpha == 0.0f || k == 0)
        return ftg::launch_sscale((float*)C, m, n, ldc, beta, s) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
    if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31) || k >= (int64_t(1) << 31) ||
        lda >= (1 << 20) || ldb >= (1 << 20) || ldc >= (1 << 20))
        return FTG_ERR_UNSUPPORTED;
    const bool abft = !cfg || cfg->abft;
    // verification intervals (K_c, a multiple of 128): the product runs as
    // rank-K_c updates of C, each protected and verified on its own
    const int64_t kc = (abft && cfg && cfg->interval_k > 0 && cfg->interval_k < k) ? cfg->interval_k : k;
    const int64_t n_int = (k + kc - 1) / kc;
    if (n_int > ftg::kMaxIntervals) return FTG_ERR_UNSUPPORTED;
    int tile = cfg && cfg->tile ? cfg->tile : h->tune[ab_type][bucket(m)][bucket(n)][bucket(k)];
    if (!tile) tile = ftg::lowp_heuristic_tile(ab_type, m, n, k);
    int bm, bn, bk;
    ftg::lowp_tile_shape(ab_type, tile, &bm, &bn, &bk);
    if (bm == 0) return set_err(h, 20);
    const int eb = ab_type == FTG_BF16 ? 2 : 1;

    ftg::LowpArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = A; a.B = B; a.C = (float*)C;
    a.lda = (int)lda; a.ldb = (int)ldb; a.ldc = (int)ldc;
    a.m = (int)m; a.n = (int)n; a.k = (int)k;
    a.tiles_m = (int)((m + bm - 1) / bm);
    a.tiles_n = (int)((n + bn - 1) / bn);
    a.vec_a = vec_ok(A, lda, eb);
    a.vec_b = vec_ok(B, ldb, eb);
    a.vec_c = vec_ok(C, ldc, 4);
    a.alpha = alpha; a.beta = beta;
    a.scale_a = ab_type == FTG_F8_E4M3 ? scale_a : nullptr;
    a.scale_b = ab_type == FTG_F8_E4M3 ? scale_b : nullptr;
    a.rep = h->rep;
    a.n_int = 1; a.ldxs = (int)k;
    // Operands whose rows are contiguous (op(A) = A, op(B) = B^T) are first
    // packed into k-major copies in the workspace: the product kernels stage
    // k-contiguous operands without register transposes (about twice as fast).
    // Everything after the pack (encode, checksum products, product, repair)
    // reads the packed copies.
    const int ita0 = ta == FTG_OP_T, itb0 = tb == FTG_OP_T;
    const bool pack_a = !ita0, pack_b = itb0 != 0;
    const int64_t ldp = (k + 15) / 16 * 16;
    if ((pack_a || pack_b) && ldp >= (1 << 20)) return FTG_ERR_UNSUPPORTED;
    const size_t pa_bytes = pack_a ? align256((size_t)m * ldp * eb) : 0;
    const size_t pb_bytes = pack_b ? align256((size_t)n * ldp * eb) : 0;
    size_t work_base = 0;  // workspace bytes before the packed copies
    const int64_t chk_tiles_r = (int64_t)a.tiles_m * ((3 * a.tiles_n + bn - 1) / bn);
    const int64_t chk_tiles_c = (int64_t)((3 * a.tiles_m + bm - 1) / bm) * a.tiles_n;
    const int ks_r = lowp_ksplit(chk_tiles_r, k), ks_c = lowp_ksplit(chk_tiles_c, k);
    const LowpLayout L = lowp_layout(m, n, k, ks_r, ks_c, n_int);
    if (abft) work_base = align256(L.total);
    // workspace (grows; allocation is not allowed under stream capture)
    if ((st = ensure_work(h, work_base + pa_bytes + pb_bytes, s)) != FTG_OK) return st;
    unsigned char* w = h->d_work;
    if (pack_a) {
        void* P = w + work_base;
        if (ftg::launch_lowp_pack(A, lda, m, k, eb, P, ldp, a.vec_a, s) != hipSuccess) return FTG_ERR_HIP;
        a.A = P; a.lda = (int)ldp; a.vec_a = vec_ok(P, ldp, eb);
    }
    if (pack_b) {
        void* P = w + work_base + pa_bytes;
        if (ftg::launch_lowp_pack(B, ldb, n, k, eb, P, ldp, a.vec_b, s) != hipSuccess) return FTG_ERR_HIP;
        a.B = P; a.ldb = (int)ldp; a.vec_b = vec_ok(P, ldp, eb);
    }
    const int ita = 1, itb = 0;  // op(A) rows and op(B) columns are k-contiguous from here on
    const bool wide = tile == ftg::kLowpWideTile && ftg::lowp_wide_ok(a, ab_type, abft ? 1 : 0);
    if (!abft) {
        LaunchTimer timer(h, s);
        const hipError_t e = wide ? ftg::launch_lowp_wide(a, ab_type, 0, s)
                                  : ftg::launch_lowp_gemm(a, ab_type, ab_type, ita, itb, 0, s);
        timer.end();
        return e == hipSuccess ? FTG_OK : FTG_ERR_HIP;
    }
    const int chunks = (int)((k + ftg::kLowpChunk - 1) / ftg::kLowpChunk);

    // Interval t is the update C := alpha op(A)[:, S_t] op(B)[S_t, :] + beta_t C
    // over the steps S_t = plo .. plo + kt - 1 (beta_t = beta for the first, 1
    // after): the operands and checksum pieces are read from step plo on, the
    // thresholds use the interval's own magnitude sums, and the repair of its
    // flagged slots runs before the next interval reads C.
    auto interval_args = [&](int64_t t) {
        ftg::LowpArgs at = a;
        const int64_t plo = t * kc, kt = std::min(kc, k - plo);
        at.A = (const unsigned char*)a.A + plo * eb;
        at.B = (const unsigned char*)a.B + plo * eb;
        at.k = (int)kt;
        at.vec_a = vec_ok(at.A, at.lda, eb);
        at.vec_b = vec_ok(at.B, at.ldb, eb);
        at.beta = t == 0 ? beta : 1.0f;
        at.n_int = (int)n_int; at.interval = (int)t; at.plo = plo;
        at.ldxs = (int)k;
        return at;
    };
    auto interval_wide = [&](const ftg::LowpArgs& at) {
        return tile == ftg::kLowpWideTile && ftg::lowp_wide_ok(at, ab_type, 1);
    };
    bool any_wide = false, any_narrow = false;
    for (int64_t t = 0; t < n_int; ++t) (interval_wide(interval_args(t)) ? any_wide : any_narrow) = true;

    // encode: checksum pieces and magnitude sums of both operands
    ftg::EncArgs e;
    std::memset(&e, 0, sizeof(e));
    ftg::EncOperand& ea = e.op[0];
    ea.X = a.A; ea.ld = a.lda; ea.rows = (int)m; ea.K = (int)k; ea.kcontig = ita; ea.vec = a.vec_a;
    ea.panels = a.tiles_m; ea.chunks = chunks;
    ea.XS = (uint16_t*)(w + L.xs_a); ea.XRp = (float*)(w + L.xrp_a); ea.XMp = (float*)(w + L.xmp_a);
    ea.XR = (float*)(w + L.ra); ea.XM = (float*)(w + L.ma);
    ftg::EncOperand& eb_ = e.op[1];
    eb_.X = a.B; eb_.ld = a.ldb; eb_.rows = (int)n; eb_.K = (int)k; eb_.kcontig = !itb; eb_.vec = a.vec_b;
    eb_.panels = a.tiles_n; eb_.chunks = chunks;
    eb_.XS = (uint16_t*)(w + L.xs_b); eb_.XRp = (float*)(w + L.xrp_b); eb_.XMp = (float*)(w + L.xmp_b);
    eb_.XR = (float*)(w + L.cb); eb_.XM = (float*)(w + L.mb);
    // magnitude sums per interval (kc is a multiple of the chunk when n_int > 1)
    ea.ichunks = eb_.ichunks = (int)((kc + ftg::kLowpChunk - 1) / ftg::kLowpChunk);
    if (ab_type == FTG_F8_E4M3) {
        // the fp8 wide product multiplies e4m3 pieces on the fp8 MFMA; the
        // 128 x 128 tile's checksum products take bf16 pieces
        if (any_wide) { ea.XS8 = w + L.xs8_a; eb_.XS8 = w + L.xs8_b; }
        if (!any_narrow) { ea.XS = nullptr; eb_.XS = nullptr; }
    }
    const int gx = std::max(a.tiles_m, a.tiles_n) * chunks;
    const int fx = (int)((std::max(m, n) + 255) / 256);
    if (ftg::launch_lowp_encode(e, ab_type, gx, fx, s) != hipSuccess) return FTG_ERR_HIP;

    ftg::InjectParams inj;
    std::memset(&inj, 0, sizeof(inj));
    if (cfg && cfg->inject) {
        // one slot per (128 x 128 tile, interval)
        const int64_t slots = (int64_t)a.tiles_m * a.tiles_n * n_int;
        if (!ftg::make_inject(cfg->inject, m, n, k, slots, 13, 31, &inj, 0, false)) return FTG_ERR_UNSUPPORTED;
    }
    for (int64_t t = 0; t < n_int; ++t) {
        ftg::LowpArgs at = interval_args(t);
        const int64_t plo = at.plo, kt = at.k;
        const bool wide = interval_wide(at);
        if (wide) {
            // the wide tile multiplies the checksum pieces inside the product
            at.XSA = ab_type == FTG_F8_E4M3 ? (const void*)(ea.XS8 + plo) : (const void*)(ea.XS + plo);
            at.XSB = ab_type == FTG_F8_E4M3 ? (const void*)(eb_.XS8 + plo) : (const void*)(eb_.XS + plo);
        } else {
            // checksum products: ER = op(A) [B_J e pieces], EC = [e^T A_I pieces]^T op(B)
            const int ksr = lowp_ksplit(chk_tiles_r, kt), ksc = lowp_ksplit(chk_tiles_c, kt);
            ftg::LowpArgs c1;
            std::memset(&c1, 0, sizeof(c1));
            c1.A = at.A; c1.lda = at.lda; c1.B = eb_.XS + plo; c1.ldb = (int)k;
            c1.C = (float*)(w + L.er); c1.ldc = (int)m;
            c1.m = (int)m; c1.n = 3 * a.tiles_n; c1.k = (int)kt;
            c1.tiles_m = a.tiles_m; c1.tiles_n = (c1.n + bn - 1) / bn;
            c1.vec_a = at.vec_a; c1.vec_b = vec_ok(c1.B, k, 2);
            c1.alpha = 1.0f; c1.beta = 0.0f;
            c1.ksplit = ksr; c1.cslice = (int64_t)m * 3 * a.tiles_n;
            if (ftg::launch_lowp_gemm(c1, ab_type, FTG_BF16, ita, 0, 0, s) != hipSuccess) return FTG_ERR_HIP;
            ftg::LowpArgs c2;
            std::memset(&c2, 0, sizeof(c2));
            c2.A = ea.XS + plo; c2.lda = (int)k; c2.B = at.B; c2.ldb = at.ldb;
            c2.C = (float*)(w + L.ec); c2.ldc = 3 * a.tiles_m;
            c2.m = 3 * a.tiles_m; c2.n = (int)n; c2.k = (int)kt;
            c2.tiles_m = (c2.m + bm - 1) / bm; c2.tiles_n = a.tiles_n;
            c2.vec_a = vec_ok(c2.A, k, 2); c2.vec_b = at.vec_b;
            c2.alpha = 1.0f; c2.beta = 0.0f;
            c2.ksplit = ksc; c2.cslice = (int64_t)3 * a.tiles_m * n;
            if (ftg::launch_lowp_gemm(c2, FTG_BF16, ab_type, 1, itb, 0, s) != hipSuccess) return FTG_ERR_HIP;
            at.ER = c1.C; at.lder = (int)m;
            at.EC = c2.C; at.ldec = 3 * a.tiles_m;
            at.slices = ksr;
            at.slices_c = ksc;
            at.er_stride = c1.cslice;
            at.ec_stride = c2.cslice;
        }

        // protected product of this interval
        at.RA = ea.XR + t * m; at.MA = ea.XM + t * a.tiles_m;
        at.CB = eb_.XR + t * n; at.MB = eb_.XM + t * a.tiles_n;
        at.lambda = (cfg && cfg->lambda > 0.0) ? cfg->lambda : kDefaultLambda;
        at.problem = 0;
        at.inj = inj;
        {
            LaunchTimer timer(h, s);
            const hipError_t e2 = wide ? ftg::launch_lowp_wide(at, ab_type, 1, s)
                                       : ftg::launch_lowp_gemm(at, ab_type, ab_type, ita, itb, 1, s);
            timer.end();
            if (e2 != hipSuccess) return FTG_ERR_HIP;
        }
        ftg::RepairProblem rp;
        std::memset(&rp, 0, sizeof(rp));
        rp.A = at.A; rp.B = at.B; rp.C = C;  // the packed copies are still in the workspace
        rp.lda = at.lda; rp.ldb = at.ldb; rp.ldc = ldc; rp.k = kt;
        rp.ta = ita; rp.tb = itb; rp.correct_policy = cfg ? cfg->correct_policy : 0;
        rp.ab_type = ab_type; rp.c_type = FTG_F32;
        rp.alpha = alpha; rp.beta = at.beta;
        rp.scale_a = a.scale_a; rp.scale_b = a.scale_b;
        if (ftg::launch_repair(h->rep, rp, nullptr, s) != hipSuccess) return FTG_ERR_HIP;
    }
    return FTG_OK;
}

// ---------------------------------------------------------------- batched
namespace {

constexpr int kMaxGroups = 8;  // (tile 2 or 3) x 4 transpose pairs

// Bytes of the batched table for `count` problems: descriptors, first-tile
// tables of up to kMaxGroups groups, repair table.
void blob_layout(int64_t count, size_t* off_first, size_t* off_efirst, size_t* off_rep, size_t* total)
{
    *off_first = align256((size_t)count * sizeof(ftg::DGemmArgs));
    *off_efirst = align256(*off_first + (size_t)(count + kMaxGroups) * sizeof(int));
    *off_rep = align256(*off_efirst + (size_t)(count + 1) * sizeof(int));
    *total = *off_rep + (size_t)count * sizeof(ftg::RepairProblem);
}

}  // namespace

ftg_status ftg_batched_reserve(ftg_handle h, int64_t capacity)
{
    if (!h || capacity < 0 || capacity > (int64_t(1) << 24)) return FTG_ERR_INVALID_ARG;
    if (capacity <= h->batch_cap && h->d_blob) return FTG_OK;
    if (hipDeviceSynchronize() != hipSuccess) return FTG_ERR_HIP;
    size_t of, oe, orp, bytes;
    blob_layout(std::max<int64_t>(1, capacity), &of, &oe, &orp, &bytes);
    if (h->d_blob) { hipFree(h->d_blob); h->d_blob = nullptr; }
    for (int i = 0; i < 3; ++i)
        if (h->h_blob[i]) { hipHostFree(h->h_blob[i]); h->h_blob[i] = nullptr; }
    h->batch_cap = 0;
    bool ok = hipMalloc(&h->d_blob, bytes) == hipSuccess;
    for (int i = 0; i < 3 && ok; ++i) ok = hipHostMalloc(&h->h_blob[i], bytes, hipHostMallocDefault) == hipSuccess;
    if (ok && !h->d_queue) {
        ok = hipMalloc(&h->d_queue, 2 * sizeof(unsigned int)) == hipSuccess;
        ok = ok && hipMemset(h->d_queue, 0, 2 * sizeof(unsigned int)) == hipSuccess;
    }
    for (int i = 0; i < 2 && ok; ++i)
        if (!h->blob_ev[i]) ok = hipEventCreateWithFlags(&h->blob_ev[i], hipEventDisableTiming) == hipSuccess;
    if (ok) ok = hipDeviceSynchronize() == hipSuccess;
    if (!ok) return FTG_ERR_HIP;
    h->blob_pending[0] = h->blob_pending[1] = false;
    h->batch_cap = std::max<int64_t>(1, capacity);
    return FTG_OK;
}

ftg_status ftg_dgemm_batched_uneven(ftg_handle h, int64_t count, const ftg_op* transa,
                                    const ftg_op* transb, const int64_t* m, const int64_t* n,
                                    const int64_t* k, const double* alpha,
                                    const double* const* A, const int64_t* lda,
                                    const double* const* B, const int64_t* ldb,
                                    const double* beta, double* const* C, const int64_t* ldc,
                                    const uint32_t* faults_per_problem, void* stream,
                                    const ftg_config* cfg)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (count < 0) return set_err(h, 2);
    if (count == 0) return FTG_OK;
    if (!transa || !transb || !m || !n || !k || !alpha || !A || !lda || !B || !ldb || !beta || !C || !ldc)
        return set_err(h, 20);
    if (count > h->batch_cap) return FTG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const bool abft = !cfg || cfg->abft;
    if (cfg && cfg->tile && cfg->tile != 2 && cfg->tile != 3) return FTG_ERR_UNSUPPORTED;

    // per problem: checks, tile configuration, group
    struct Item { int64_t p; int group; int64_t k; };
    Item* items = new (std::nothrow) Item[(size_t)count];
    if (!items) return FTG_ERR_HIP;
    struct Guard { Item* p; ~Guard() { delete[] p; } } guard{items};
    int64_t n_items = 0;
    for (int64_t p = 0; p < count; ++p) {
        ftg_status st = check_gemm(h, transa[p], transb[p], m[p], n[p], k[p], lda[p], ldb[p], ldc[p], cfg);
        if (st != FTG_OK) return st;
        if (cfg && cfg->inject && cfg->inject->bit_hi > 63) return set_err(h, 20);
        if (m[p] >= (int64_t(1) << 31) || n[p] >= (int64_t(1) << 31) || k[p] >= (int64_t(1) << 31) ||
            lda[p] >= (1 << 20) || ldb[p] >= (1 << 20) || ldc[p] >= (1 << 20))
            return FTG_ERR_UNSUPPORTED;
        if (m[p] == 0 || n[p] == 0 || ((alpha[p] == 0.0 || k[p] == 0) && beta[p] == 1.0)) continue;
        int tile = cfg && cfg->tile ? cfg->tile : h->tune[FTG_F64][bucket(m[p])][bucket(n[p])][bucket(k[p])];
        if (tile != 2 && tile != 3) tile = 3;
        const int g = (tile - 2) * 4 + (transa[p] == FTG_OP_T) * 2 + (transb[p] == FTG_OP_T);
        items[n_items++] = Item{p, g, alpha[p] == 0.0 ? 0 : k[p]};
    }
    if (n_items == 0) return FTG_OK;
    // group by configuration, most expensive tiles (largest k) first
    std::sort(items, items + n_items, [](const Item& x, const Item& y) {
        return x.group != y.group ? x.group < y.group : (x.k != y.k ? x.k > y.k : x.p < y.p);
    });

    // staging slot: wait until the copy that last read it has run
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return FTG_ERR_HIP;
    const bool capturing = cs != hipStreamCaptureStatusNone;
    const int slot = capturing ? 2 : h->next_slot;
    if (!capturing) {
        if (h->blob_pending[slot] && hipEventSynchronize(h->blob_ev[slot]) != hipSuccess) return FTG_ERR_HIP;
        h->next_slot ^= 1;
    }
    size_t off_first, off_efirst, off_rep, bytes;
    blob_layout(count, &off_first, &off_efirst, &off_rep, &bytes);
    unsigned char* hb = h->h_blob[slot];
    auto* hdesc = (ftg::DGemmArgs*)hb;
    auto* hfirst = (int*)(hb + off_first);
    auto* hefirst = (int*)(hb + off_efirst);

    // encode pass workspace: per problem, both operands' panel sums
    const bool pre = abft && !(cfg && cfg->encode_in_loop);
    size_t enc_doubles = 0;
    if (pre) {
        for (int64_t it = 0; it < n_items; ++it) {
            int ebm, ebn, ebk;
            ftg::dgemm_tile_shape(items[it].group / 4 + 2, &ebm, &ebn, &ebk);
            const int64_t p = items[it].p, kk = items[it].k;
            enc_doubles += (size_t)(((m[p] + ebm - 1) / ebm) + ((n[p] + ebn - 1) / ebn)) * (size_t)kk * 2;
        }
        const ftg_status ws = ensure_work(h, std::max<size_t>(enc_doubles, 1) * sizeof(double), s);
        if (ws != FTG_OK) return ws;
    }
    size_t enc_off = 0;
    int64_t enc_items = 0;
    auto* hrep = (ftg::RepairProblem*)(hb + off_rep);
    std::memset(hrep, 0, (size_t)count * sizeof(ftg::RepairProblem));

    struct Group { int64_t d0, d1; int f0; int tile, ta, tb; bool ivl, direct; };
    Group groups[kMaxGroups];
    int ng = 0;
    int nfirst = 0;
    int64_t total = 0;
    for (int64_t it = 0; it < n_items; ++it) {
        const int64_t p = items[it].p;
        if (ng == 0 || groups[ng - 1].tile * 4 + groups[ng - 1].ta * 2 + groups[ng - 1].tb - 8 != items[it].group) {
            if (ng > 0) hfirst[nfirst++] = (int)total;  // closing entry of the previous group
            Group& G = groups[ng++];
            G.d0 = it; G.d1 = it; G.f0 = nfirst;
            G.tile = items[it].group / 4 + 2; G.ta = (items[it].group >> 1) & 1; G.tb = items[it].group & 1;
            G.ivl = false;
            G.direct = true;
            total = 0;
        }
        Group& G = groups[ng - 1];
        int bm, bn, bk;
        ftg::dgemm_tile_shape(G.tile, &bm, &bn, &bk);
        const int64_t kk = items[it].k;
        // one interval: a multiple of 128 no shorter than k, so that problems of
        // both kinds can share a launch with interval checks compiled in
        const int64_t kc = (cfg && cfg->interval_k > 0 && cfg->interval_k < kk)
                               ? cfg->interval_k
                               : (std::max<int64_t>(kk, 1) + ftg::kKGran - 1) / ftg::kKGran * ftg::kKGran;
        ftg::DGemmArgs& a = hdesc[it];
        std::memset(&a, 0, sizeof(a));
        a.A = A[p]; a.B = B[p]; a.C = C[p];
        a.lda = (int)lda[p]; a.ldb = (int)ldb[p]; a.ldc = (int)ldc[p];
        a.m = (int)m[p]; a.n = (int)n[p]; a.k = (int)kk;
        a.kc = (int)kc;
        a.tiles_m = (int)((m[p] + bm - 1) / bm);
        a.tiles_n = (int)((n[p] + bn - 1) / bn);
        a.ta = G.ta; a.tb = G.tb;
        a.alpha = alpha[p]; a.beta = beta[p];
        a.correct_policy = cfg ? cfg->correct_policy : 0;
        a.uncorrectable_policy = cfg ? cfg->uncorrectable_policy : 0;
        a.problem = (int)p;
        a.rep = h->rep;
        a.bm = bm;
        a.bn = bn;
        a.lds_direct = ftg::lds_direct_ok(a.A, a.lda, a.B, a.ldb);
        G.direct = G.direct && a.lds_direct;
        hefirst[it] = (int)enc_items;
        if (pre && kk > 0) {
            double* w = (double*)h->d_work + enc_off;
            a.asp = w;
            a.bsp = w + (size_t)a.tiles_m * kk * 2;
            enc_off += (size_t)(a.tiles_m + a.tiles_n) * kk * 2;
            enc_items += (int64_t)(a.tiles_m + a.tiles_n) * ((kk + ftg::kDEncChunk - 1) / ftg::kDEncChunk);
            if (enc_items >= (int64_t(1) << 31)) return FTG_ERR_UNSUPPORTED;
        }
        if (kc < kk) G.ivl = true;
        const int64_t n_int = (kk + kc - 1) / kc;
        if (abft && cfg && cfg->inject && kk > 0) {
            if (n_int > ftg::kMaxIntervals) return FTG_ERR_UNSUPPORTED;
            ftg_inject in = *cfg->inject;
            in.seed = ftg::splitmix64(cfg->inject->seed, (uint64_t(1) << 32) + (uint64_t)p);
            const int64_t slots = (int64_t)a.tiles_m * a.tiles_n * n_int;
            if (!ftg::make_inject(&in, m[p], n[p], kk, slots, 40, 63, &a.inj,
                                  faults_per_problem ? faults_per_problem[p] : 0u, faults_per_problem != nullptr))
                return FTG_ERR_UNSUPPORTED;
        }
        hfirst[nfirst++] = (int)total;
        total += (int64_t)a.tiles_m * a.tiles_n;
        if (total >= (int64_t(1) << 31)) return FTG_ERR_UNSUPPORTED;
        G.d1 = it + 1;
        ftg::RepairProblem& rp = hrep[p];
        rp.A = a.A; rp.B = a.B; rp.C = a.C;
        rp.lda = lda[p]; rp.ldb = ldb[p]; rp.ldc = ldc[p]; rp.k = kk;
        rp.ta = a.ta; rp.tb = a.tb; rp.correct_policy = a.correct_policy;
        rp.ab_type = FTG_F64; rp.c_type = FTG_F64;
        rp.alpha = alpha[p]; rp.beta = beta[p]; rp.scale_a = rp.scale_b = nullptr;
    }
    hfirst[nfirst++] = (int)total;
    hefirst[n_items] = (int)enc_items;

    if (hipMemcpyAsync(h->d_blob, hb, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return FTG_ERR_HIP;
    if (!capturing) {
        if (hipEventRecord(h->blob_ev[slot], s) != hipSuccess) return FTG_ERR_HIP;
        h->blob_pending[slot] = true;
    }
    const auto* ddesc = (const ftg::DGemmArgs*)h->d_blob;
    const auto* dfirst = (const int*)(h->d_blob + off_first);
    if (pre && enc_items > 0 &&
        ftg::launch_dencode_batched(ddesc, (const int*)(h->d_blob + off_efirst), (int)n_items, (int)enc_items, s) !=
            hipSuccess)
        return FTG_ERR_HIP;
    LaunchTimer timer(h, s);
    for (int g = 0; g < ng; ++g) {
        const Group& G = groups[g];
        ftg::BatchLaunch L;
        L.desc = ddesc + G.d0;
        L.first = dfirst + G.f0;
        L.count = (int)(G.d1 - G.d0);
        L.total = hfirst[G.f0 + L.count];
        L.queue = h->d_queue;
        hipError_t e = ftg::launch_dgemm_batched(L, G.tile, G.ta, G.tb, abft, abft && G.ivl, pre, G.direct, s);
        if (e != hipSuccess) return FTG_ERR_HIP;
    }
    timer.end();
    if (abft) {
        ftg::RepairProblem none;
        std::memset(&none, 0, sizeof(none));
        if (ftg::launch_repair(h->rep, none, (const ftg::RepairProblem*)(h->d_blob + off_rep), s) != hipSuccess)
            return FTG_ERR_HIP;
    }
    return FTG_OK;
}

ftg_status ftg_timing_enable(ftg_handle h, int on)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    if (on && !h->tev[0]) {
        for (auto& e : h->tev)
            if (hipEventCreate(&e) != hipSuccess) return FTG_ERR_HIP;
    }
    h->timing = on != 0;
    h->tev_used = 0;
    return FTG_OK;
}

ftg_status ftg_timing_read(ftg_handle h, int32_t* launches, double* total_ms)
{
    if (!h || !launches || !total_ms) return FTG_ERR_INVALID_ARG;
    double t = 0.0;
    for (int i = 0; i < h->tev_used; ++i) {
        if (hipEventSynchronize(h->tev[2 * i + 1]) != hipSuccess) return FTG_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, h->tev[2 * i], h->tev[2 * i + 1]) != hipSuccess) return FTG_ERR_HIP;
        t += ms;
    }
    *launches = h->tev_used;
    *total_ms = t;
    h->tev_used = 0;
    return FTG_OK;
}

ftg_status ftg_report_read(ftg_handle h, void* stream, ftg_fault_report* out, int sync)
{
    if (!h || !out) return FTG_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    DevReport r;
    if (hipMemcpyAsync(&r, h->rep, sizeof(r), hipMemcpyDeviceToHost, s) != hipSuccess) return FTG_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return FTG_ERR_HIP;
    out->injected = r.cnt[ftg::kInjected];
    out->detected = r.cnt[ftg::kDetected];
    out->corrected_subtract = r.cnt[ftg::kCorrSub];
    out->corrected_recompute = r.cnt[ftg::kCorrRecomp];
    out->checksum_only = r.cnt[ftg::kChecksumOnly];
    out->uncorrectable = r.cnt[ftg::kUncorrectable];
    out->tiles_recomputed = r.cnt[ftg::kTilesRecomputed];
    out->lost = r.rq_lost;
    std::memcpy(&out->max_pass_ratio, &r.cnt[ftg::kMaxPassRatio], sizeof(double));
    out->n_records = r.n_records;
    out->n_inject_log = r.n_inject;
    const size_t nr = std::min<size_t>({(size_t)r.n_records, (size_t)out->capacity, h->capacity});
    const size_t ni = std::min<size_t>({(size_t)r.n_inject, (size_t)out->capacity, h->capacity});
    if (out->records && nr)
        if (hipMemcpyAsync(out->records, h->d_records, nr * sizeof(ftg_fault_record),
                           hipMemcpyDeviceToHost, s) != hipSuccess)
            return FTG_ERR_HIP;
    if (out->inject_log && ni)
        if (hipMemcpyAsync(out->inject_log, h->d_inject, ni * sizeof(ftg_inject_record),
                           hipMemcpyDeviceToHost, s) != hipSuccess)
            return FTG_ERR_HIP;
    if (sync) {
        if (hipStreamSynchronize(s) != hipSuccess) return FTG_ERR_HIP;
        // uncorrectable slots left as they were (not recomputed), including
        // slots the full repair queue could not take
        if (out->uncorrectable > out->tiles_recomputed || out->lost) return FTG_ERR_UNCORRECTED;
    }
    return FTG_OK;
}

ftg_status ftg_report_reset(ftg_handle h, void* stream)
{
    if (!h) return FTG_ERR_INVALID_ARG;
    return ftg::launch_report_reset(h->rep, (hipStream_t)stream) == hipSuccess ? FTG_OK : FTG_ERR_HIP;
}

}  // extern "C"
