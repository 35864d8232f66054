// pk_runtime.cpp -- host side of the C ABI declared in include/pk.h.
//
// The runtime holds no device code of its own: every kernel, including the
// built-in defaults, is a gfx950 code object loaded with hipModuleLoadData
// and launched with hipModuleLaunchKernel.  The defaults are embedded in this
// library at build time; tuned variants arrive through pk_variant_load.  Each
// code object exports `pk_knobs` (its family and compile-time knobs), read
// once at load time; launch geometry and workspace layout are derived from it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pk.h"
#include "pk_internal.h"
#include "pk_kernel_abi.h"

static_assert((int)PK_FAMILY_COUNT == (int)PKF_COUNT, "family enums out of sync");

// embedded default code objects (generated at build time)
struct pk_embedded_co {
    int family;
    const unsigned char *data;
    size_t size;
};
extern "C" const pk_embedded_co pk_embedded[];
extern "C" const int pk_embedded_count;

namespace {

thread_local std::string g_err;

pk_status fail(pk_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

// A failed HIP call also leaves its code as the thread's last HIP error, which the
// caller's next unrelated check (torch's launch checks, for one) would report as its
// own: take it off before returning the status.
pk_status hip_fail(hipError_t e, const char *what) {
    (void)hipGetLastError();
    return fail(PK_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define PK_HIP(call)                                  \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess)                         \
            return hip_fail(e_, #call);               \
    } while (0)

// the API boundary: no exception escapes
#define PK_GUARD_BEGIN try {
#define PK_GUARD_END                                                              \
    }                                                                             \
    catch (const std::exception &ex) {                                            \
        return fail(PK_ERR_INVALID_ARG, "internal error: %s", ex.what());         \
    }                                                                             \
    catch (...) {                                                                 \
        return fail(PK_ERR_INVALID_ARG, "internal error");                        \
    }

uint64_t fnv1a(const void *p, size_t n) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

const char *const kFnNames[PKF_COUNT][2] = {
    {"pk_gemm", nullptr},                              // GEMM_F32
    {"pk_gemm", nullptr},                              // GEMM_BF16
    {"pk_gemm", nullptr},                              // GEMM_SPLIT
    {"pk_gemv", nullptr},                              // GEMV
    {"pk_gemvt_partial", "pk_colsum_reduce"},          // GEMV_T
    {"pk_gemv_pair_partial", "pk_colsum_reduce"},      // GEMV_PAIR
    {"pk_conv2d", nullptr},                            // CONV2D
    {"pk_conv3d", nullptr},                            // CONV3D
    {"pk_colstats_partial", "pk_colstats_merge"},      // COLSTATS
    {"pk_syrk", nullptr},                              // SYRK_F32
    {"pk_gemm_bf", "pk_corr_prep"},                    // SYRK_BF16
    {"pk_gemm_bf", "pk_corr_prep"},                    // SYRK_SPLIT
    {"pk_convert", "pk_fill"},                         // CONVERT
    {"pk_rankk_syrk", "pk_rankk_syr2k"},               // RANKK
    {"pk_gesummv", "pk_colsum_accumulate"},            // GESUMMV
    {"pk_fdtd_e", "pk_fdtd_h"},                        // FDTD
    {"pk_gemm_bf", "pk_gemm_prep"},                    // GEMM_BF16_WS
    {"pk_gemm_bf", "pk_gemm_prep"},                    // GEMM_SPLIT_WS
    {"pk_stream_read", "pk_stream_copy"},              // STREAM
};

// smallest row-block / segment a gemv_t, gemv_pair or colstats variant may use
// and the narrowest column strip; workspace bounds follow from these
constexpr int kMinRowBlock = 16;
constexpr int kMinStrip = 64;
// the fixed-order reduce of the transposed matvec's partials and the column
// statistics' merge: blocks of 8 wavefronts over 64 columns
constexpr int kReduceThreads = 512;

struct Variant {
    int family = -1;
    hipModule_t mod = nullptr;
    hipFunction_t fn[2] = {nullptr, nullptr};
    int32_t knobs[PK_NKNOBS] = {0};
    uint64_t hash = 0;
    bool builtin = false;
};

}  // namespace

struct pk_context {
    int device = 0;
    std::mutex mu;
    std::vector<std::unique_ptr<Variant>> variants;
    pk_variant_id def[PKF_COUNT];
    pk_variant_id forced[PKF_COUNT];
    std::map<std::pair<int, int>, pk_variant_id> best;
    bool checks = true;
    void *flush_buf = nullptr;
    size_t flush_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct pk_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// read and check the knob record of a freshly loaded module
pk_status load_module(pk_context *ctx, const void *code, size_t bytes, bool builtin, pk_variant_id *out) {
    if (!code || bytes < 64)
        return fail(PK_ERR_INVALID_ARG, "variant code object is empty");
    auto v = std::make_unique<Variant>();
    hipError_t e = hipModuleLoadData(&v->mod, code);
    if (e != hipSuccess) {
        (void)hipGetLastError();    // not the caller's error to find later (see hip_fail)
        return fail(PK_ERR_NO_VARIANT, "hipModuleLoadData: %s", hipGetErrorString(e));
    }
    hipDeviceptr_t kp = nullptr;
    size_t ksz = 0;
    e = hipModuleGetGlobal(&kp, &ksz, v->mod, "pk_knobs");
    if (e != hipSuccess || ksz != sizeof(v->knobs)) {
        (void)hipGetLastError();
        (void)hipModuleUnload(v->mod);
        return fail(PK_ERR_NO_VARIANT, "code object has no pk_knobs record");
    }
    e = hipMemcpyDtoH(v->knobs, kp, sizeof(v->knobs));
    if (e != hipSuccess) {
        (void)hipModuleUnload(v->mod);
        return hip_fail(e, "reading pk_knobs");
    }
    const int32_t *k = v->knobs;
    const int fam = k[PK_K_FAMILY];
    bool ok = fam >= 0 && fam < PKF_COUNT && k[PK_K_ABI] == PK_KERNEL_ABI_VERSION &&
              k[PK_K_THREADS] >= 64 && k[PK_K_THREADS] <= 1024 && k[PK_K_THREADS] % 64 == 0;
    if (ok) {
        switch (fam) {
        case PKF_GEMM_F32: case PKF_GEMM_BF16: case PKF_GEMM_SPLIT: case PKF_SYRK_F32:
            ok = k[PK_K_TM] >= 16 && k[PK_K_TN] >= 16 && k[PK_K_TK] >= 4;
            break;
        case PKF_GEMM_BF16_WS: case PKF_GEMM_SPLIT_WS: case PKF_SYRK_BF16: case PKF_SYRK_SPLIT:
            // + the transposing preparation's rows per block (0: 64), a multiple of 32
            ok = k[PK_K_TM] >= 16 && k[PK_K_TN] >= 16 && k[PK_K_TK] >= 4 && k[PK_K_X3] >= 0 &&
                 k[PK_K_X3] <= 1024 && k[PK_K_X3] % 32 == 0;
            break;
        case PKF_GEMV:
            ok = k[PK_K_TM] >= 1 && k[PK_K_WAVES_M] >= 1;
            break;
        case PKF_GEMV_T: case PKF_GEMV_PAIR:
            // one-launch variants (X3 = 1) are one wavefront strip wide
            ok = k[PK_K_TM] >= kMinRowBlock && k[PK_K_TN] >= kMinStrip && k[PK_K_X1] >= kMinStrip &&
                 k[PK_K_TN] % k[PK_K_X1] == 0 && k[PK_K_X2] * 64 == kReduceThreads &&
                 (k[PK_K_X3] == 0 || (k[PK_K_X3] == 1 && k[PK_K_TN] == k[PK_K_X1]));
            break;
        case PKF_COLSTATS:
            ok = k[PK_K_TM] >= kMinRowBlock && k[PK_K_TN] >= kMinStrip && k[PK_K_X2] * 64 == kReduceThreads &&
                 (k[PK_K_X3] == 0 || k[PK_K_X3] == 1);
            break;
        case PKF_CONV2D: case PKF_CONV3D:
            ok = k[PK_K_TM] >= 1 && k[PK_K_TN] >= 1 && k[PK_K_TK] >= 1;
            break;
        case PKF_RANKK:
            ok = k[PK_K_TM] >= 16 && k[PK_K_TK] >= 16;
            break;
        case PKF_GESUMMV:
            ok = k[PK_K_TM] >= 1 && k[PK_K_WAVES_M] >= 1;
            break;
        case PKF_FDTD:
            ok = k[PK_K_TM] >= 1 && k[PK_K_TN] >= 1;
            break;
        default:
            ok = k[PK_K_VEC] >= 1;
        }
    }
    if (!ok) {
        (void)hipModuleUnload(v->mod);
        return fail(PK_ERR_NO_VARIANT, "code object knob record is invalid (family %d)", fam);
    }
    v->family = fam;
    for (int i = 0; i < 2; ++i) {
        const char *name = kFnNames[fam][i];
        if (!name)
            continue;
        e = hipModuleGetFunction(&v->fn[i], v->mod, name);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            (void)hipModuleUnload(v->mod);
            return fail(PK_ERR_NO_VARIANT, "code object lacks entry point %s", name);
        }
    }
    v->hash = fnv1a(code, bytes);
    v->builtin = builtin;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->variants.push_back(std::move(v));
    *out = (pk_variant_id)(ctx->variants.size() - 1);
    return PK_OK;
}

const Variant *get_variant(pk_context *ctx, pk_variant_id id) {
    if (id < 0 || (size_t)id >= ctx->variants.size())
        return nullptr;
    return ctx->variants[id].get();
}

int32_t bucket_of(int64_t d) {
    int32_t b = 0;
    while (b < 62 && ((int64_t)1 << b) < d)
        ++b;
    return b;
}

const Variant *pick(pk_context *ctx, int family, int64_t largest) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    pk_variant_id id = ctx->forced[family];
    if (id < 0) {
        auto it = ctx->best.find({family, bucket_of(largest)});
        if (it != ctx->best.end())
            id = it->second;
    }
    const Variant *v = get_variant(ctx, id);
    if (!v)
        v = get_variant(ctx, ctx->def[family]);
    return v;
}

pk_status launch(const Variant *v, int fn, int64_t grid, int threads, void *args, size_t args_size,
                 hipStream_t s) {
    if (grid <= 0)
        return PK_OK;
    if (grid > 0x7fffffffll)
        return fail(PK_ERR_SHAPE, "problem too large for one launch (%lld blocks)", (long long)grid);
    void *cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &args_size,
                   HIP_LAUNCH_PARAM_END};
    hipError_t e = hipModuleLaunchKernel(v->fn[fn], (unsigned)grid, 1, 1, (unsigned)threads, 1, 1, 0, s,
                                         nullptr, cfg);
    if (e != hipSuccess)
        return hip_fail(e, "hipModuleLaunchKernel");
    return PK_OK;
}

// ---- argument checks -------------------------------------------------------------

bool aligned16(const void *p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// the extent [p, p + bytes) must be device memory inside one allocation
pk_status check_ptr(pk_context *ctx, const void *p, size_t bytes, const char *name) {
    if (bytes == 0)
        return PK_OK;
    if (!p)
        return fail(PK_ERR_INVALID_ARG, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) & 3u)
        return fail(PK_ERR_INVALID_ARG, "%s is not 4-byte aligned", name);
    if (!ctx->checks)
        return PK_OK;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PK_ERR_INVALID_ARG, "%s is not HIP-allocated memory", name);
    }
    if (attr.type != hipMemoryTypeDevice)
        return fail(PK_ERR_INVALID_ARG, "%s is not device memory", name);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return PK_OK;   // range query unsupported for this allocation: type check only
    }
    const uintptr_t lo = reinterpret_cast<uintptr_t>(base), hi = lo + size;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    if (a < lo || a + bytes > hi)
        return fail(PK_ERR_INVALID_ARG, "%s: %zu bytes overrun its allocation", name, bytes);
    return PK_OK;
}

// bytes spanned by a rows x cols matrix with row stride ld
size_t mat_bytes(int64_t rows, int64_t cols, int64_t ld) {
    if (rows <= 0 || cols <= 0)
        return 0;
    return (size_t)((rows - 1) * ld + cols) * sizeof(float);
}

pk_status check_ctx(pk_context *ctx) {
    if (!ctx)
        return fail(PK_ERR_INVALID_ARG, "context is NULL");
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != ctx->device)
        PK_HIP(hipSetDevice(ctx->device));
    return PK_OK;
}

#define PK_TRY(x)                  \
    do {                           \
        pk_status s_ = (x);        \
        if (s_ != PK_OK)           \
            return s_;             \
    } while (0)

// ---- workspace bounds ------------------------------------------------------------------

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
// bytes per ticket cell of the one-launch reductions
constexpr size_t kCellStride = PK_CELL_STRIDE;
// row stride of the partial-sum rows: rows start 256 bytes apart (the one-launch
// variants read them back with 16-byte loads); matches the kernels' pk_part_ld
int64_t part_ld(int64_t n) { return (n + 63) & ~(int64_t)63; }

// Transposed matvec / pair workspace: [part2: rb rows of part_ld(N)][ticket cells:
// one per column strip (+ one per row block for the pair), PK_CELL_STRIDE bytes
// apart][part1 (pair): wstrips rows of M].  The bound covers every variant (row
// blocks of at least kMinRowBlock rows, strips of at least kMinStrip columns).
struct GemvtLayout {
    size_t part2, cells, part1;
    size_t total() const { return part2 + cells + part1; }
};
GemvtLayout gemvt_layout(bool pair, int64_t M, int64_t N, int64_t rb, int64_t strips, int64_t wstrips) {
    GemvtLayout l;
    l.part2 = align256((size_t)rb * (size_t)part_ld(N) * 4);
    l.cells = (size_t)(strips + (pair ? rb : 0)) * kCellStride;
    l.part1 = pair ? (size_t)wstrips * (size_t)M * 4 : 0;
    return l;
}
size_t ws_gemv_t(int64_t M, int64_t N) {
    return gemvt_layout(false, M, N, cdiv(M, kMinRowBlock), cdiv(N, kMinStrip), 0).total();
}
size_t ws_gemv_pair(int64_t M, int64_t N) {
    const int64_t rb = cdiv(M, kMinRowBlock), st = cdiv(N, kMinStrip);
    return gemvt_layout(true, M, N, rb, st, st).total();
}
// Column statistics workspace: [segments][3][part_ld(m)] partials, then one ticket
// cell per column strip (PK_CELL_STRIDE bytes apart)
size_t colstats_bytes(int64_t segs, int64_t m, int64_t strips) {
    return align256((size_t)segs * 3 * (size_t)part_ld(m) * 4) + (size_t)strips * kCellStride;
}
size_t ws_colstats(int64_t n, int64_t m) { return colstats_bytes(cdiv(n, kMinRowBlock), m, cdiv(m, kMinStrip)); }

// The ticket tag of one call of a one-launch reduction: distinct for every call of
// the process (a bijective mix of a counter, so consecutive calls differ in every
// bit), never 0 (a cleared ticket cell holds tag 0).  `bits` 32 or 31.
uint32_t next_tag(int bits) {
    static std::atomic<uint32_t> counter{0};
    const uint32_t mask = bits >= 32 ? 0xffffffffu : ((1u << bits) - 1u);
    for (;;) {
        uint32_t x = counter.fetch_add(1, std::memory_order_relaxed) + 1u;
        x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
        x &= mask;
        if (x != 0)
            return x;
    }
}
bool one_launch(const Variant *v) { return v->knobs[PK_K_X3] == 1; }

// a one-launch variant needs its workspace 16-byte aligned (64-bit ticket cells,
// 16-byte partial loads); with a less aligned workspace the family's built-in
// default (partials + reduce) runs instead
pk_status one_launch_ok(pk_context *ctx, const Variant *&v, int family, const void *ws) {
    if (!v)
        return fail(PK_ERR_NO_VARIANT, "no variant for family %d", family);
    if (!one_launch(v) || (reinterpret_cast<uintptr_t>(ws) & 15u) == 0)
        return PK_OK;
    const Variant *d = get_variant(ctx, ctx->def[family]);
    if (!d || one_launch(d))
        return fail(PK_ERR_ALIGNMENT, "this variant needs a 16-byte aligned workspace");
    v = d;
    return PK_OK;
}
size_t ws_covar(int64_t n, int64_t m) { return align256(ws_colstats(n, m)) + 2 * align256((size_t)m * 4); }

// ---- launches ----------------------------------------------------------------------------

pk_status run_gemm(pk_context *ctx, int family, int64_t M, int64_t N, int64_t K, float alpha,
                   const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
                   const float *C, int64_t ldc, float *D, int64_t ldd, hipStream_t s) {
    const Variant *v = pick(ctx, family, std::max(M, std::max(N, K)));
    if (!v)
        return fail(PK_ERR_NO_VARIANT, "no variant for family %d", family);
    pk_gemm_args a{};
    a.A = A; a.B = B; a.C = C; a.D = D;
    a.M = M; a.N = N; a.K = K;
    a.lda = lda; a.ldb = ldb; a.ldc = ldc; a.ldd = ldd;
    a.alpha = alpha; a.beta = beta;
    a.aligned = aligned16(A) && aligned16(B) && aligned16(C) && aligned16(D) && lda % 4 == 0 &&
                ldb % 4 == 0 && ldc % 4 == 0 && ldd % 4 == 0;
    const int64_t grid = cdiv(M, v->knobs[PK_K_TM]) * cdiv(N, v->knobs[PK_K_TN]);
    return launch(v, 0, grid, v->knobs[PK_K_THREADS], &a, sizeof a, s);
}

size_t ws_gemm_bf(pk_precision prec, int64_t M, int64_t N, int64_t K);
int64_t prep_kp(int64_t K);
// chained product: T (M x L, FP32), then for bf16 / split the larger of the two
// products' prepared operands
size_t ws_gemm3_t(pk_precision prec, int64_t M, int64_t N, int64_t K, int64_t L) {
    const size_t t = (size_t)M * (size_t)L * 4;
    if (prec == PK_FP32)
        return t;
    return align256(t) + std::max(ws_gemm_bf(prec, M, L, K), ws_gemm_bf(prec, M, N, L));
}
// bf16 / split with T written straight as the second product's prepared A operand:
// T's planes (M rows of Kp2 = L rounded up to 64, hi then lo), then the larger of the
// first product's prepared operands and the second product's prepared C^T
size_t ws_gemm3_direct(pk_precision prec, int64_t M, int64_t N, int64_t K, int64_t L) {
    const size_t planes = prec == PK_SPLIT_BF16 ? 2 : 1;
    const size_t kp2 = (size_t)prep_kp(L);
    return align256(planes * (size_t)M * kp2 * 2) +
           std::max(ws_gemm_bf(prec, M, L, K), planes * align256((size_t)N * kp2 * 2));
}
size_t ws_gemm3(pk_precision prec, int64_t M, int64_t N, int64_t K, int64_t L) {
    if (prec == PK_FP32)
        return ws_gemm3_t(prec, M, N, K, L);
    return std::max(ws_gemm3_t(prec, M, N, K, L), ws_gemm3_direct(prec, M, N, K, L));
}

int gemm_family(pk_precision p) {
    return p == PK_FP32 ? PKF_GEMM_F32 : (p == PK_BF16 ? PKF_GEMM_BF16 : PKF_GEMM_SPLIT);
}

// ---- bf16 / split GEMM from prepared operands --------------------------------------------
// workspace: [A hi][A lo][B^T hi][B^T lo] (lo planes for split only), bf16 rows of Kp
int64_t prep_kp(int64_t K) { return cdiv(std::max<int64_t>(K, 1), 64) * 64; }
// source rows per block of a code object's transposing preparation (its knob record)
int64_t prep_rows(const Variant *v) { return v->knobs[PK_K_X3] > 0 ? v->knobs[PK_K_X3] : 64; }
size_t ws_gemm_bf(pk_precision prec, int64_t M, int64_t N, int64_t K) {
    if (prec == PK_FP32)
        return 0;
    const size_t planes = prec == PK_SPLIT_BF16 ? 2 : 1;
    const size_t kp = (size_t)prep_kp(K);
    return planes * (align256((size_t)M * kp * 2) + align256((size_t)N * kp * 2));
}

// D = alpha A B + beta C from operands prepared in `ws` (A as [M][Kp], B^T as [N][Kp]).
// With `pre_h` (and `pre_l` for split) A is already prepared there ([M][Kp] rows, as the
// preparation writes them) and only B^T is prepared, at the start of `ws`.  With `out_t`
// the result is not stored to D but written as the next product's prepared A operand:
// M rows of `out_kp` bf16 values (the hi plane, then for split the lo plane right
// after it), which the variant must support (knob slot X2 = 3).
pk_status run_gemm_bf(pk_context *ctx, pk_precision prec, int64_t M, int64_t N, int64_t K, float alpha,
                      const float *A, int64_t lda, const float *B, int64_t ldb, float beta, const float *C,
                      int64_t ldc, float *D, int64_t ldd, void *ws, hipStream_t s,
                      const uint16_t *pre_h = nullptr, const uint16_t *pre_l = nullptr,
                      uint16_t *out_t = nullptr, int64_t out_kp = 0) {
    const int family = prec == PK_BF16 ? PKF_GEMM_BF16_WS : PKF_GEMM_SPLIT_WS;
    const Variant *v = pick(ctx, family, std::max(M, std::max(N, K)));
    if (!v)
        return fail(PK_ERR_NO_VARIANT, "no variant for family %d", family);
    if (out_t && v->knobs[PK_K_X2] != 3)
        return fail(PK_ERR_NO_VARIANT, "variant cannot write a prepared operand");
    const bool split = prec == PK_SPLIT_BF16;
    const int64_t kp = prep_kp(K);
    char *w = static_cast<char *>(ws);
    const size_t a_pl = align256((size_t)M * (size_t)kp * 2), b_pl = align256((size_t)N * (size_t)kp * 2);
    const uint16_t *Ah, *Al;
    uint16_t *Bh, *Bl;
    if (pre_h) {
        Ah = pre_h;
        Al = split ? pre_l : nullptr;
        Bh = reinterpret_cast<uint16_t *>(w);
        Bl = split ? reinterpret_cast<uint16_t *>(w + b_pl) : nullptr;
    } else {
        uint16_t *ah = reinterpret_cast<uint16_t *>(w);
        uint16_t *al = split ? reinterpret_cast<uint16_t *>(w + a_pl) : nullptr;
        Ah = ah;
        Al = al;
        Bh = reinterpret_cast<uint16_t *>(w + (split ? 2 : 1) * a_pl);
        Bl = split ? reinterpret_cast<uint16_t *>(w + 2 * a_pl + b_pl) : nullptr;
        pk_gemmprep_args pa{};
        pa.src = A; pa.hi = ah; pa.lo = al; pa.rows = M; pa.cols = K; pa.ld = std::max<int64_t>(lda, 1);
        pa.ldo = kp; pa.transpose = 0; pa.split = split ? 1 : 0;
        PK_TRY(launch(v, 1, std::min<int64_t>(cdiv(M * (kp / 8), 256), 16384), 256, &pa, sizeof pa, s));
    }
    pk_gemmprep_args pb{};
    pb.src = B; pb.hi = Bh; pb.lo = Bl; pb.rows = K; pb.cols = N; pb.ld = ldb;
    pb.ldo = kp; pb.transpose = 1; pb.split = split ? 1 : 0;
    PK_TRY(launch(v, 1, cdiv(kp, prep_rows(v)) * cdiv(N, 64), 256, &pb, sizeof pb, s));
    pk_gemmbf_args a{};
    a.Ah = Ah; a.Al = Al; a.Bh = Bh; a.Bl = Bl; a.C = C; a.D = D;
    a.M = M; a.N = N; a.Kp = kp; a.ldc = ldc; a.ldd = ldd; a.alpha = alpha; a.beta = beta;
    if (out_t) {
        a.C = nullptr; a.beta = 0.f;
        a.D = reinterpret_cast<float *>(out_t);
        a.ldd = -out_kp;                                   // the prepared-operand epilogue
    }
    const int64_t grid = cdiv(M, v->knobs[PK_K_TM]) * cdiv(N, v->knobs[PK_K_TN]);
    return launch(v, 0, grid, v->knobs[PK_K_THREADS], &a, sizeof a, s);
}
int syrk_family(pk_precision p) {
    return p == PK_FP32 ? PKF_SYRK_F32 : (p == PK_BF16 ? PKF_SYRK_BF16 : PKF_SYRK_SPLIT);
}

// ---- bf16 / split rank-k product of the correlation and covariance ----------------------
// Z^T planes: [m][np] bf16 (hi, then lo for split), np = n rounded up to 64
size_t ws_zplanes(pk_precision prec, int64_t n, int64_t m) {
    if (prec == PK_FP32)
        return 0;
    return (prec == PK_SPLIT_BF16 ? 2 : 1) * align256((size_t)m * (size_t)prep_kp(n) * 2);
}
size_t ws_corr(pk_precision prec, int64_t n, int64_t m) {
    return prec == PK_FP32 ? ws_colstats(n, m) : align256(ws_colstats(n, m)) + ws_zplanes(prec, n, m);
}
size_t ws_covar_p(pk_precision prec, int64_t n, int64_t m) { return ws_covar(n, m) + ws_zplanes(prec, n, m); }

// R = Z^T Z * (1/(n-1)), Z = (X - mean) * (1/sd), lower-triangle tiles mirrored;
// zws: the Z^T planes (256-byte aligned)
pk_status run_syrk_bf(pk_context *ctx, pk_precision prec, int64_t n, int64_t m, const float *X, int64_t ldx,
                      const float *mean, const float *sd, float *R, int64_t ldr, char *zws, hipStream_t s) {
    const Variant *v = pick(ctx, syrk_family(prec), std::max(n, m));
    if (!v)
        return fail(PK_ERR_NO_VARIANT, "no variant for family %d", syrk_family(prec));
    const bool split = prec == PK_SPLIT_BF16;
    const int64_t np = prep_kp(n);
    const size_t pl = align256((size_t)m * (size_t)np * 2);
    uint16_t *Zh = reinterpret_cast<uint16_t *>(zws);
    uint16_t *Zl = split ? reinterpret_cast<uint16_t *>(zws + pl) : nullptr;
    pk_corrprep_args pa{};
    pa.X = X; pa.mean = mean; pa.std = sd; pa.hi = Zh; pa.lo = Zl;
    pa.n = n; pa.m = m; pa.ldx = ldx; pa.ldo = np; pa.split = split ? 1 : 0;
    PK_TRY(launch(v, 1, cdiv(np, prep_rows(v)) * cdiv(m, 64), 256, &pa, sizeof pa, s));
    pk_gemmbf_args a{};
    a.Ah = Zh; a.Al = Zl; a.Bh = Zh; a.Bl = Zl; a.C = nullptr; a.D = R;
    a.M = m; a.N = m; a.Kp = np; a.ldc = ldr; a.ldd = ldr;
    a.alpha = 1.0f / (float)(n - 1); a.beta = 0.0f;
    const int64_t nt = cdiv(m, v->knobs[PK_K_TM]);
    return launch(v, 0, nt * (nt + 1) / 2, v->knobs[PK_K_THREADS], &a, sizeof a, s);
}

pk_status run_colstats(pk_context *ctx, int64_t n, int64_t m, const float *X, int64_t ldx, float eps,
                       float *mean, float *sd, void *ws, size_t ws_bytes, hipStream_t s) {
    const Variant *v = pick(ctx, PKF_COLSTATS, std::max(n, m));
    if (!v)
        return fail(PK_ERR_NO_VARIANT, "no colstats variant");
    PK_TRY(one_launch_ok(ctx, v, PKF_COLSTATS, ws));
    const int rows = v->knobs[PK_K_TM];
    const int64_t segs = cdiv(n, rows);
    const int64_t strips = cdiv(m, v->knobs[PK_K_TN]);
    if (colstats_bytes(segs, m, strips) > ws_bytes)
        return fail(PK_ERR_INVALID_ARG, "workspace too small for colstats");
    if (segs > 0x7fffffff)
        return fail(PK_ERR_SHAPE, "too many segments");
    pk_colstats_args a{};
    a.X = X; a.part = (float *)ws; a.mean = mean; a.std = sd;
    a.n = n; a.m = m; a.ldx = ldx; a.eps = eps;
    a.segments = (int32_t)segs; a.seg_rows = rows;
    a.aligned = aligned16(X) && ldx % 4 == 0;
    if (one_launch(v)) {
        a.aligned |= (int32_t)(next_tag(31) << 1);
        return launch(v, 0, segs * strips, v->knobs[PK_K_THREADS], &a, sizeof a, s);
    }
    PK_TRY(launch(v, 0, segs * strips, v->knobs[PK_K_THREADS], &a, sizeof a, s));
    return launch(v, 1, std::min<int64_t>(cdiv(m, 64), 65535), kReduceThreads, &a, sizeof a, s);
}

}  // namespace

// ---- shared implementations (pk_internal.h) ---------------------------------------------

pk_status pk_internal_fail(pk_status s, const char *msg) { return fail(s, "%s", msg); }

pk_status pk_internal_device(pk_context *ctx, int *device) {
    PK_TRY(check_ctx(ctx));
    *device = ctx->device;
    return PK_OK;
}

size_t pk_internal_corr_ws(pk_precision prec, int64_t n, int64_t m) { return ws_corr(prec, n, m); }

pk_status pk_internal_corr(pk_context *ctx, pk_precision prec, int64_t n, int64_t m, const float *X,
                           int64_t ldx, float eps, float *mean, float *std_, float *R, int64_t ldr,
                           void *ws, size_t ws_bytes, bool ws_owned, hipStream_t s) {
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (prec < PK_FP32 || prec > PK_SPLIT_BF16)
        return fail(PK_ERR_INVALID_ARG, "bad precision %d", (int)prec);
    if (n < 0 || m < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (m > 0 && n < 2)
        return fail(PK_ERR_SHAPE, "correlation needs n >= 2 samples");
    if (ldx < std::max<int64_t>(m, 1) || ldr < std::max<int64_t>(m, 1))
        return fail(PK_ERR_SHAPE, "leading dimension smaller than m");
    if (!(eps >= 0.f))
        return fail(PK_ERR_INVALID_ARG, "eps must be >= 0");
    if (m == 0)
        return PK_OK;
    if (ws_owned && ws_corr(prec, n, m) > ws_bytes)
        return fail(PK_ERR_SHAPE, "n = %lld, m = %lld needs %zu bytes of scratch; the library's scratch holds %zu",
                    (long long)n, (long long)m, ws_corr(prec, n, m), ws_bytes);
    PK_TRY(check_ptr(ctx, X, mat_bytes(n, m, ldx), "X"));
    PK_TRY(check_ptr(ctx, mean, (size_t)m * 4, "mean"));
    PK_TRY(check_ptr(ctx, std_, (size_t)m * 4, "std"));
    PK_TRY(check_ptr(ctx, R, mat_bytes(m, m, ldr), "R"));
    if (prec != PK_FP32) {
        const size_t need = ws_corr(prec, n, m);
        if (ws_bytes < need)
            return fail(PK_ERR_INVALID_ARG, "workspace too small: %zu < %zu bytes", ws_bytes, need);
        if (!ws_owned)
            PK_TRY(check_ptr(ctx, ws, need, "workspace"));
        if (reinterpret_cast<uintptr_t>(ws) & 255u)
            return fail(PK_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
        const size_t part = align256(ws_colstats(n, m));
        PK_TRY(run_colstats(ctx, n, m, X, ldx, eps, mean, std_, ws, part, s));
        return run_syrk_bf(ctx, prec, n, m, X, ldx, mean, std_, R, ldr, static_cast<char *>(ws) + part, s);
    }
    if (!ws_owned)
        PK_TRY(check_ptr(ctx, ws, std::min(ws_bytes, ws_colstats(n, m)), "workspace"));
    PK_TRY(run_colstats(ctx, n, m, X, ldx, eps, mean, std_, ws, ws_bytes, s));
    const Variant *v = pick(ctx, syrk_family(prec), std::max(n, m));
    pk_syrk_args a{};
    a.X = X; a.mean = mean; a.std = std_; a.R = R;
    a.n = n; a.m = m; a.ldx = ldx; a.ldr = ldr;
    a.aligned = aligned16(X) && ldx % 4 == 0;
    const int64_t nt = cdiv(m, v->knobs[PK_K_TM]);
    return launch(v, 0, nt * (nt + 1) / 2, v->knobs[PK_K_THREADS], &a, sizeof a, s);
}


// ==========================================================================================
// C ABI
// ==========================================================================================

extern "C" {

const char *pk_status_string(pk_status s) {
    switch (s) {
    case PK_OK: return "ok";
    case PK_ERR_INVALID_ARG: return "invalid argument";
    case PK_ERR_SHAPE: return "invalid shape";
    case PK_ERR_ALIGNMENT: return "misaligned operand";
    case PK_ERR_UNSUPPORTED: return "unsupported";
    case PK_ERR_HIP: return "HIP error";
    case PK_ERR_NO_VARIANT: return "no usable variant";
    case PK_ERR_COMPILE: return "compile failure";
    case PK_ERR_TIMEOUT: return "timeout";
    case PK_ERR_VALIDATION: return "validation failure";
    case PK_ERR_IO: return "I/O error";
    }
    return "unknown status";
}

const char *pk_last_error(void) { return g_err.c_str(); }

int pk_abi_version(void) { return PK_ABI_VERSION; }

int32_t pk_size_bucket(int64_t d) { return bucket_of(d); }

pk_status pk_context_create(int device, pk_context **out) {
    PK_GUARD_BEGIN
    g_err.clear();
    if (!out)
        return fail(PK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0)
        return fail(PK_ERR_HIP, "no HIP device available");
    if (device < 0 || device >= count)
        return fail(PK_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, count);
    PK_HIP(hipSetDevice(device));
    auto ctx = std::make_unique<pk_context>();
    ctx->device = device;
    for (int f = 0; f < PKF_COUNT; ++f) {
        ctx->def[f] = -1;
        ctx->forced[f] = -1;
    }
    for (int i = 0; i < pk_embedded_count; ++i) {
        pk_variant_id id = -1;
        pk_status s = load_module(ctx.get(), pk_embedded[i].data, pk_embedded[i].size, true, &id);
        if (s != PK_OK)
            return s;
        const int fam = ctx->variants[id]->family;
        if (fam != pk_embedded[i].family)
            return fail(PK_ERR_NO_VARIANT, "embedded code object %d reports family %d", i, fam);
        ctx->def[fam] = id;
    }
    for (int f = 0; f < PKF_COUNT; ++f)
        if (ctx->def[f] < 0)
            return fail(PK_ERR_NO_VARIANT, "no built-in code object for family %d", f);
    PK_HIP(hipEventCreate(&ctx->ev0));
    PK_HIP(hipEventCreate(&ctx->ev1));
    // the allocation-free entry points' scratch: its device address is taken here, once
    // per device; a failure is reported by those entry points, not by the context
    (void)pk_internal_scratch_setup(device);
    g_err.clear();
    *out = ctx.release();
    return PK_OK;
    PK_GUARD_END
}

void pk_context_destroy(pk_context *ctx) {
    if (!ctx)
        return;
    try {
        (void)hipSetDevice(ctx->device);
        for (auto &v : ctx->variants)
            if (v && v->mod)
                (void)hipModuleUnload(v->mod);
        if (ctx->flush_buf)
            (void)hipFree(ctx->flush_buf);
        if (ctx->ev0)
            (void)hipEventDestroy(ctx->ev0);
        if (ctx->ev1)
            (void)hipEventDestroy(ctx->ev1);
        delete ctx;
    } catch (...) {
    }
}

pk_status pk_context_set_checks(pk_context *ctx, int enabled) {
    if (!ctx)
        return fail(PK_ERR_INVALID_ARG, "context is NULL");
    ctx->checks = enabled != 0;
    return PK_OK;
}

pk_status pk_workspace_bytes(pk_kernel kernel, const int64_t *dims, int ndims, pk_precision prec,
                             size_t *out) {
    PK_GUARD_BEGIN
    if (!out || (!dims && ndims > 0))
        return fail(PK_ERR_INVALID_ARG, "NULL argument");
    if (prec < PK_FP32 || prec > PK_SPLIT_BF16)
        return fail(PK_ERR_INVALID_ARG, "bad precision %d", (int)prec);
    for (int i = 0; i < ndims; ++i)
        if (dims[i] < 0)
            return fail(PK_ERR_SHAPE, "negative dimension");
    auto need = [&](int n) { return ndims >= n; };
    switch (kernel) {
    case PK_KERNEL_GEMM:
        // pk_sgemm needs none; pk_sgemm_ws takes this much for bf16 / split (0 for FP32)
        if (!need(3)) break;
        *out = ws_gemm_bf(prec, dims[0], dims[1], dims[2]);
        return PK_OK;
    case PK_KERNEL_GEMV: case PK_KERNEL_CONV2D: case PK_KERNEL_CONV3D: case PK_KERNEL_CONVERT:
        *out = 0;
        return PK_OK;
    case PK_KERNEL_GEMM3:
        if (!need(4)) break;
        *out = ws_gemm3(prec, dims[0], dims[1], dims[2], dims[3]);
        return PK_OK;
    case PK_KERNEL_GEMV_T:
        if (!need(2)) break;
        *out = ws_gemv_t(dims[0], dims[1]);
        return PK_OK;
    case PK_KERNEL_GEMV_PAIR:
        if (!need(2)) break;
        *out = ws_gemv_pair(dims[0], dims[1]);
        return PK_OK;
    case PK_KERNEL_COLSTATS:
        if (!need(2)) break;
        *out = ws_colstats(dims[0], dims[1]);
        return PK_OK;
    case PK_KERNEL_CORR:
        // bf16 / split also hold the prepared Z^T planes
        if (!need(2)) break;
        *out = ws_corr(prec, dims[0], dims[1]);
        return PK_OK;
    case PK_KERNEL_COVAR:
        if (!need(2)) break;
        *out = ws_covar_p(prec, dims[0], dims[1]);
        return PK_OK;
    case PK_KERNEL_MVT:
        if (!need(1)) break;
        *out = ws_gemv_pair(dims[0], dims[0]);
        return PK_OK;
    case PK_KERNEL_SYRK: case PK_KERNEL_SYR2K: case PK_KERNEL_GESUMMV: case PK_KERNEL_FDTD2D:
        *out = 0;
        return PK_OK;
    default:
        return fail(PK_ERR_INVALID_ARG, "bad kernel id %d", (int)kernel);
    }
    return fail(PK_ERR_INVALID_ARG, "too few dims for kernel %d", (int)kernel);
    PK_GUARD_END
}

pk_status pk_sgemm(pk_context *ctx, pk_precision prec, int64_t M, int64_t N, int64_t K, float alpha,
                   const float *A, int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                   int64_t ldc, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (prec < PK_FP32 || prec > PK_SPLIT_BF16)
        return fail(PK_ERR_INVALID_ARG, "bad precision %d", (int)prec);
    if (M < 0 || N < 0 || K < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if ((M > 0 && lda < std::max<int64_t>(K, 1)) || ldb < std::max<int64_t>(N, 1) ||
        ldc < std::max<int64_t>(N, 1))
        return fail(PK_ERR_SHAPE, "leading dimension smaller than the row length");
    if (M == 0 || N == 0)
        return PK_OK;
    PK_TRY(check_ptr(ctx, A, mat_bytes(M, K, lda), "A"));
    PK_TRY(check_ptr(ctx, B, mat_bytes(K, N, ldb), "B"));
    PK_TRY(check_ptr(ctx, C, mat_bytes(M, N, ldc), "C"));
    return run_gemm(ctx, gemm_family(prec), M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, C, ldc,
                    (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_sgemm_ws(pk_context *ctx, pk_precision prec, int64_t M, int64_t N, int64_t K, float alpha,
                      const float *A, int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                      int64_t ldc, void *ws, size_t ws_bytes, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (prec < PK_FP32 || prec > PK_SPLIT_BF16)
        return fail(PK_ERR_INVALID_ARG, "bad precision %d", (int)prec);
    if (M < 0 || N < 0 || K < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if ((M > 0 && lda < std::max<int64_t>(K, 1)) || ldb < std::max<int64_t>(N, 1) ||
        ldc < std::max<int64_t>(N, 1))
        return fail(PK_ERR_SHAPE, "leading dimension smaller than the row length");
    if (M == 0 || N == 0)
        return PK_OK;
    const size_t need = ws_gemm_bf(prec, M, N, K);
    if (ws_bytes < need)
        return fail(PK_ERR_INVALID_ARG, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    PK_TRY(check_ptr(ctx, A, mat_bytes(M, K, lda), "A"));
    PK_TRY(check_ptr(ctx, B, mat_bytes(K, N, ldb), "B"));
    PK_TRY(check_ptr(ctx, C, mat_bytes(M, N, ldc), "C"));
    if (prec == PK_FP32)
        return run_gemm(ctx, PKF_GEMM_F32, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, C, ldc,
                        (hipStream_t)stream);
    PK_TRY(check_ptr(ctx, ws, need, "workspace"));
    if (reinterpret_cast<uintptr_t>(ws) & 255u)
        return fail(PK_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
    return run_gemm_bf(ctx, prec, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, C, ldc, ws,
                       (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_sgemm3(pk_context *ctx, pk_precision prec, int64_t M, int64_t N, int64_t K, int64_t L,
                    float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
                    const float *Cm, int64_t ldcm, float beta, float *D, int64_t ldd, void *ws,
                    size_t ws_bytes, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (prec < PK_FP32 || prec > PK_SPLIT_BF16)
        return fail(PK_ERR_INVALID_ARG, "bad precision %d", (int)prec);
    if (M < 0 || N < 0 || K < 0 || L < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (lda < std::max<int64_t>(K, 1) || ldb < std::max<int64_t>(L, 1) ||
        ldcm < std::max<int64_t>(N, 1) || ldd < std::max<int64_t>(N, 1))
        return fail(PK_ERR_SHAPE, "leading dimension smaller than the row length");
    if (M == 0 || N == 0)
        return PK_OK;
    // bf16 / split: T goes straight into the second product's prepared operand when the
    // first product's variant can write that layout (the preparation pass of T is saved)
    bool direct = false;
    if (prec != PK_FP32 && L > 0) {
        const Variant *v1 = pick(ctx, prec == PK_BF16 ? PKF_GEMM_BF16_WS : PKF_GEMM_SPLIT_WS,
                                 std::max(M, std::max(L, K)));
        direct = v1 && v1->knobs[PK_K_X2] == 3 && v1->knobs[PK_K_TN] % 64 == 0;   // tiles cover Kp2
    }
    const size_t need = direct ? ws_gemm3_direct(prec, M, N, K, L) : ws_gemm3_t(prec, M, N, K, L);
    if (ws_bytes < need)
        return fail(PK_ERR_INVALID_ARG, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    PK_TRY(check_ptr(ctx, A, mat_bytes(M, K, lda), "A"));
    PK_TRY(check_ptr(ctx, B, mat_bytes(K, L, ldb), "B"));
    PK_TRY(check_ptr(ctx, Cm, mat_bytes(L, N, ldcm), "Cm"));
    PK_TRY(check_ptr(ctx, D, mat_bytes(M, N, ldd), "D"));
    PK_TRY(check_ptr(ctx, ws, need, "workspace"));
    float *T = static_cast<float *>(ws);
    hipStream_t s = (hipStream_t)stream;
    if (direct) {
        if (reinterpret_cast<uintptr_t>(ws) & 255u)
            return fail(PK_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
        const bool split = prec == PK_SPLIT_BF16;
        const int64_t kp2 = prep_kp(L);
        uint16_t *th = static_cast<uint16_t *>(ws);
        uint16_t *tl = split ? th + M * kp2 : nullptr;
        void *rest = static_cast<char *>(ws) + align256((split ? 2 : 1) * (size_t)M * (size_t)kp2 * 2);
        PK_TRY(run_gemm_bf(ctx, prec, M, L, K, 1.0f, A, lda, B, ldb, 0.0f, nullptr, L, nullptr, L, rest, s,
                           nullptr, nullptr, th, kp2));
        return run_gemm_bf(ctx, prec, M, N, L, alpha, nullptr, 0, Cm, ldcm, beta, D, ldd, D, ldd, rest, s, th, tl);
    }
    if (prec != PK_FP32) {
        if (reinterpret_cast<uintptr_t>(ws) & 255u)
            return fail(PK_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
        // both products from prepared operands; T stays FP32 and is rounded (bf16) or
        // re-split (split) when it is prepared for the second product
        void *prep = static_cast<char *>(ws) + align256((size_t)M * (size_t)L * 4);
        if (L > 0)
            PK_TRY(run_gemm_bf(ctx, prec, M, L, K, 1.0f, A, lda, B, ldb, 0.0f, nullptr, L, T, L, prep, s));
        return run_gemm_bf(ctx, prec, M, N, L, alpha, T, std::max<int64_t>(L, 1), Cm, ldcm, beta, D, ldd, D,
                           ldd, prep, s);
    }
    const int fam = gemm_family(prec);
    if (L > 0)
        PK_TRY(run_gemm(ctx, fam, M, L, K, 1.0f, A, lda, B, ldb, 0.0f, nullptr, L, T, L, s));
    return run_gemm(ctx, fam, M, N, L, alpha, T, std::max<int64_t>(L, 1), Cm, ldcm, beta, D, ldd, D,
                    ldd, s);
    PK_GUARD_END
}

pk_status pk_sgemv(pk_context *ctx, int64_t M, int64_t N, const float *A, int64_t lda, const float *x,
                   float *y, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (M < 0 || N < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (lda < std::max<int64_t>(N, 1))
        return fail(PK_ERR_SHAPE, "lda smaller than N");
    if (M == 0)
        return PK_OK;
    PK_TRY(check_ptr(ctx, A, mat_bytes(M, N, lda), "A"));
    PK_TRY(check_ptr(ctx, x, (size_t)N * 4, "x"));
    PK_TRY(check_ptr(ctx, y, (size_t)M * 4, "y"));
    const Variant *v = pick(ctx, PKF_GEMV, std::max(M, N));
    pk_gemv_args a{};
    a.A = A; a.x = x; a.y = y; a.M = M; a.N = N; a.lda = lda;
    a.aligned = aligned16(A) && aligned16(x) && lda % 4 == 0;
    const int64_t rows_per_block = (int64_t)v->knobs[PK_K_TM] * v->knobs[PK_K_WAVES_M];
    return launch(v, 0, cdiv(M, rows_per_block), v->knobs[PK_K_THREADS], &a, sizeof a,
                  (hipStream_t)stream);
    PK_GUARD_END
}

static pk_status gemvt_common(pk_context *ctx, bool pair, int64_t M, int64_t N, const float *A,
                              int64_t lda, const float *x, const float *z, float *y1, float *y2,
                              void *ws, size_t ws_bytes, hipStream_t s) {
    if (M < 0 || N < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (lda < std::max<int64_t>(N, 1))
        return fail(PK_ERR_SHAPE, "lda smaller than N");
    if (M == 0 && N == 0)
        return PK_OK;
    const int family = pair ? PKF_GEMV_PAIR : PKF_GEMV_T;
    const Variant *v = pick(ctx, family, std::max(M, N));
    PK_TRY(one_launch_ok(ctx, v, family, ws));
    const int64_t rb = cdiv(M, v->knobs[PK_K_TM]);
    const int64_t strips = cdiv(N, v->knobs[PK_K_TN]);       // blocks per row block
    const int64_t wstrips = cdiv(N, v->knobs[PK_K_X1]);      // wavefront strips (rows of part1)
    const GemvtLayout lay = gemvt_layout(pair, M, N, rb, strips, wstrips);
    if (ws_bytes < lay.total())
        return fail(PK_ERR_INVALID_ARG, "workspace too small: %zu < %zu bytes", ws_bytes, lay.total());
    PK_TRY(check_ptr(ctx, A, mat_bytes(M, N, lda), "A"));
    PK_TRY(check_ptr(ctx, z, (size_t)M * 4, "z"));
    PK_TRY(check_ptr(ctx, y2, (size_t)N * 4, "y2"));
    if (pair) {
        PK_TRY(check_ptr(ctx, x, (size_t)N * 4, "x"));
        PK_TRY(check_ptr(ctx, y1, (size_t)M * 4, "y1"));
    }
    PK_TRY(check_ptr(ctx, ws, lay.total(), "workspace"));
    if (M == 0 || N == 0) {
        // degenerate: y2 (length N) is all zero when M == 0; y1 (length M) when N == 0.
        // Use the reduce kernel with zero rows, which writes zeros.
        pk_reduce_args r{};
        r.P1 = nullptr; r.y1 = y2; r.n1 = N; r.rows1 = 0;
        r.P2 = nullptr; r.y2 = pair ? y1 : nullptr; r.n2 = pair ? M : 0; r.rows2 = 0;
        return launch(v, 1, cdiv(r.n1, 64) + cdiv(r.n2, 64), kReduceThreads, &r, sizeof r, s);
    }
    if (rb > 0x7fffffff || strips > 0x7fffffff)
        return fail(PK_ERR_SHAPE, "problem too large");
    pk_gemvt_args a{};
    a.A = A; a.x = x; a.z = z; a.y1 = y1; a.y2 = y2;
    a.part2 = (float *)ws;
    a.part1 = pair ? (float *)((char *)ws + lay.part2 + lay.cells) : nullptr;
    a.M = M; a.N = N; a.lda = lda;
    a.aligned = aligned16(A) && lda % 4 == 0;
    a.row_blocks = (int32_t)rb;
    a.col_strips = (int32_t)wstrips;
    if (one_launch(v)) {
        a.tag = next_tag(32);
        return launch(v, 0, rb * strips, v->knobs[PK_K_THREADS], &a, sizeof a, s);
    }
    PK_TRY(launch(v, 0, rb * strips, v->knobs[PK_K_THREADS], &a, sizeof a, s));
    pk_reduce_args r{};
    r.P1 = a.part2; r.y1 = y2; r.n1 = N; r.rows1 = (int32_t)rb;
    if (pair) {
        r.P2 = a.part1; r.y2 = y1; r.n2 = M; r.rows2 = (int32_t)wstrips;
    }
    return launch(v, 1, cdiv(r.n1, 64) + (pair ? cdiv(r.n2, 64) : 0), kReduceThreads, &r, sizeof r, s);
}

pk_status pk_sgemv_t(pk_context *ctx, int64_t M, int64_t N, const float *A, int64_t lda, const float *z,
                     float *y, void *ws, size_t ws_bytes, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    return gemvt_common(ctx, false, M, N, A, lda, nullptr, z, nullptr, y, ws, ws_bytes,
                        (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_sgemv_pair(pk_context *ctx, int64_t M, int64_t N, const float *A, int64_t lda,
                        const float *x, const float *z, float *y1, float *y2, void *ws,
                        size_t ws_bytes, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    return gemvt_common(ctx, true, M, N, A, lda, x, z, y1, y2, ws, ws_bytes, (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_conv2d_3x3(pk_context *ctx, int64_t H, int64_t W, const float w[9], const float *in,
                        int64_t ldi, float *out, int64_t ldo, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (H < 0 || W < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (ldi < std::max<int64_t>(W, 1) || ldo < std::max<int64_t>(W, 1))
        return fail(PK_ERR_SHAPE, "leading dimension smaller than W");
    if (!w)
        return fail(PK_ERR_INVALID_ARG, "w is NULL");
    if (H == 0 || W == 0)
        return PK_OK;
    PK_TRY(check_ptr(ctx, in, mat_bytes(H, W, ldi), "in"));
    PK_TRY(check_ptr(ctx, out, mat_bytes(H, W, ldo), "out"));
    const Variant *v = pick(ctx, PKF_CONV2D, std::max(H, W));
    pk_conv2d_args a{};
    a.in = in; a.out = out; a.H = H; a.W = W; a.ldi = ldi; a.ldo = ldo;
    std::memcpy(a.w, w, sizeof a.w);
    a.aligned = aligned16(in) && aligned16(out) && ldi % 4 == 0 && ldo % 4 == 0;
    const int64_t grid = cdiv(W, v->knobs[PK_K_TN]) * cdiv(H, v->knobs[PK_K_TM]);
    return launch(v, 0, grid, v->knobs[PK_K_THREADS], &a, sizeof a, (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_conv3d_3x3x3(pk_context *ctx, int64_t D, int64_t H, int64_t W, const float w[27],
                          const float *in, float *out, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (D < 0 || H < 0 || W < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (!w)
        return fail(PK_ERR_INVALID_ARG, "w is NULL");
    if (D == 0 || H == 0 || W == 0)
        return PK_OK;
    const size_t bytes = (size_t)D * (size_t)H * (size_t)W * 4;
    PK_TRY(check_ptr(ctx, in, bytes, "in"));
    PK_TRY(check_ptr(ctx, out, bytes, "out"));
    const Variant *v = pick(ctx, PKF_CONV3D, std::max(D, std::max(H, W)));
    pk_conv3d_args a{};
    a.in = in; a.out = out; a.D = D; a.H = H; a.W = W;
    std::memcpy(a.w, w, sizeof a.w);
    a.aligned = aligned16(in) && aligned16(out) && W % 4 == 0;
    const int64_t grid = cdiv(W, v->knobs[PK_K_TN]) * cdiv(H, v->knobs[PK_K_TM]) * cdiv(D, v->knobs[PK_K_TK]);
    return launch(v, 0, grid, v->knobs[PK_K_THREADS], &a, sizeof a, (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_colstats(pk_context *ctx, int64_t n, int64_t m, const float *X, int64_t ldx, float eps,
                      float *mean, float *std_, void *ws, size_t ws_bytes, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (n < 0 || m < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (m > 0 && n < 2)
        return fail(PK_ERR_SHAPE, "column deviation needs n >= 2 samples");
    if (ldx < std::max<int64_t>(m, 1))
        return fail(PK_ERR_SHAPE, "ldx smaller than m");
    if (!(eps >= 0.f))
        return fail(PK_ERR_INVALID_ARG, "eps must be >= 0");
    if (m == 0)
        return PK_OK;
    PK_TRY(check_ptr(ctx, X, mat_bytes(n, m, ldx), "X"));
    PK_TRY(check_ptr(ctx, mean, (size_t)m * 4, "mean"));
    PK_TRY(check_ptr(ctx, std_, (size_t)m * 4, "std"));
    PK_TRY(check_ptr(ctx, ws, std::min(ws_bytes, ws_colstats(n, m)), "workspace"));
    return run_colstats(ctx, n, m, X, ldx, eps, mean, std_, ws, ws_bytes, (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_corr(pk_context *ctx, pk_precision prec, int64_t n, int64_t m, const float *X, int64_t ldx,
                  float eps, float *mean, float *std_, float *R, int64_t ldr, void *ws, size_t ws_bytes,
                  pk_stream stream) {
    PK_GUARD_BEGIN
    return pk_internal_corr(ctx, prec, n, m, X, ldx, eps, mean, std_, R, ldr, ws, ws_bytes, false,
                            (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_convert_bf16(pk_context *ctx, int64_t n, const float *x, uint16_t *hi, uint16_t *lo,
                          pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (n < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (n == 0)
        return PK_OK;
    PK_TRY(check_ptr(ctx, x, (size_t)n * 4, "x"));
    if (!hi || (reinterpret_cast<uintptr_t>(hi) & 1u) || (lo && (reinterpret_cast<uintptr_t>(lo) & 1u)))
        return fail(PK_ERR_INVALID_ARG, "hi/lo must be non-NULL (hi) and 2-byte aligned");
    if (ctx->checks) {
        // 2-byte outputs: reuse the extent check on a 4-byte-aligned view when possible
        const size_t b = (size_t)n * 2;
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, hi) != hipSuccess || attr.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            return fail(PK_ERR_INVALID_ARG, "hi is not device memory");
        }
        if (lo && (hipPointerGetAttributes(&attr, lo) != hipSuccess || attr.type != hipMemoryTypeDevice)) {
            (void)hipGetLastError();
            return fail(PK_ERR_INVALID_ARG, "lo is not device memory");
        }
        hipDeviceptr_t base;
        size_t size;
        if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)hi) == hipSuccess &&
            reinterpret_cast<uintptr_t>(hi) + b > reinterpret_cast<uintptr_t>(base) + size)
            return fail(PK_ERR_INVALID_ARG, "hi overruns its allocation");
        if (lo && hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)lo) == hipSuccess &&
            reinterpret_cast<uintptr_t>(lo) + b > reinterpret_cast<uintptr_t>(base) + size)
            return fail(PK_ERR_INVALID_ARG, "lo overruns its allocation");
        (void)hipGetLastError();
    }
    const Variant *v = pick(ctx, PKF_CONVERT, n);
    pk_convert_args a{};
    a.x = x; a.hi = hi; a.lo = lo; a.n = n; a.mode = lo ? 1 : 0;
    const int64_t per_block = (int64_t)v->knobs[PK_K_THREADS] * v->knobs[PK_K_VEC];
    return launch(v, 0, cdiv(n, per_block), v->knobs[PK_K_THREADS], &a, sizeof a, (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_covar(pk_context *ctx, pk_precision prec, int64_t n, int64_t m, const float *X, int64_t ldx,
                   float *mean, float *C, int64_t ldc, void *ws, size_t ws_bytes, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (prec < PK_FP32 || prec > PK_SPLIT_BF16)
        return fail(PK_ERR_INVALID_ARG, "bad precision %d", (int)prec);
    if (n < 0 || m < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (m > 0 && n < 2)
        return fail(PK_ERR_SHAPE, "covariance needs n >= 2 samples");
    if (ldx < std::max<int64_t>(m, 1) || ldc < std::max<int64_t>(m, 1))
        return fail(PK_ERR_SHAPE, "leading dimension smaller than m");
    if (m == 0)
        return PK_OK;
    const size_t need = ws_covar_p(prec, n, m);
    if (ws_bytes < need)
        return fail(PK_ERR_INVALID_ARG, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    PK_TRY(check_ptr(ctx, X, mat_bytes(n, m, ldx), "X"));
    PK_TRY(check_ptr(ctx, mean, (size_t)m * 4, "mean"));
    PK_TRY(check_ptr(ctx, C, mat_bytes(m, m, ldc), "C"));
    PK_TRY(check_ptr(ctx, ws, need, "workspace"));
    if (prec != PK_FP32 && (reinterpret_cast<uintptr_t>(ws) & 255u))
        return fail(PK_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *w = static_cast<char *>(ws);
    const size_t part = align256(ws_colstats(n, m));
    float *sd = reinterpret_cast<float *>(w + part);
    float *ones = reinterpret_cast<float *>(w + part + align256((size_t)m * 4));
    PK_TRY(run_colstats(ctx, n, m, X, ldx, 0.0f, mean, sd, ws, part, s));
    const Variant *fv = get_variant(ctx, ctx->def[PKF_CONVERT]);
    struct {
        float *p;
        int64_t n;
        float value;
        int32_t pad;
    } fa{ones, m, 1.0f, 0};
    PK_TRY(launch(fv, 1, std::min<int64_t>(cdiv(m, 1024), 4096), 256, &fa, sizeof fa, s));
    if (prec != PK_FP32)
        return run_syrk_bf(ctx, prec, n, m, X, ldx, mean, ones, C, ldc, w + ws_covar(n, m), s);
    const Variant *v = pick(ctx, syrk_family(prec), std::max(n, m));
    pk_syrk_args a{};
    a.X = X; a.mean = mean; a.std = ones; a.R = C;
    a.n = n; a.m = m; a.ldx = ldx; a.ldr = ldc;
    a.aligned = aligned16(X) && ldx % 4 == 0;
    const int64_t nt = cdiv(m, v->knobs[PK_K_TM]);
    return launch(v, 0, nt * (nt + 1) / 2, v->knobs[PK_K_THREADS], &a, sizeof a, s);
    PK_GUARD_END
}

static pk_status rankk_common(pk_context *ctx, int mode, int64_t N, int64_t K, float alpha, const float *A,
                              int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                              hipStream_t s) {
    if (N < 0 || K < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (lda < std::max<int64_t>(K, 1) || (mode == 1 && ldb < std::max<int64_t>(K, 1)) ||
        ldc < std::max<int64_t>(N, 1))
        return fail(PK_ERR_SHAPE, "leading dimension smaller than the row length");
    if (N == 0)
        return PK_OK;
    PK_TRY(check_ptr(ctx, A, mat_bytes(N, K, lda), "A"));
    if (mode == 1)
        PK_TRY(check_ptr(ctx, B, mat_bytes(N, K, ldb), "B"));
    PK_TRY(check_ptr(ctx, C, mat_bytes(N, N, ldc), "C"));
    const Variant *v = pick(ctx, PKF_RANKK, std::max(N, K));
    pk_rankk_args a{};
    a.A = A; a.B = mode == 1 ? B : A; a.C = C;
    a.N = N; a.K = K; a.lda = lda; a.ldb = mode == 1 ? ldb : lda; a.ldc = ldc;
    a.alpha = alpha; a.beta = beta;
    a.aligned = aligned16(A) && aligned16(a.B) && lda % 4 == 0 && a.ldb % 4 == 0;
    const int64_t nt = cdiv(N, v->knobs[PK_K_TM]);
    return launch(v, mode, nt * (nt + 1) / 2, v->knobs[PK_K_THREADS], &a, sizeof a, s);
}

pk_status pk_ssyrk(pk_context *ctx, int64_t N, int64_t K, float alpha, const float *A, int64_t lda, float beta,
                   float *C, int64_t ldc, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    return rankk_common(ctx, 0, N, K, alpha, A, lda, nullptr, 0, beta, C, ldc, (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_ssyr2k(pk_context *ctx, int64_t N, int64_t K, float alpha, const float *A, int64_t lda,
                    const float *B, int64_t ldb, float beta, float *C, int64_t ldc, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    return rankk_common(ctx, 1, N, K, alpha, A, lda, B, ldb, beta, C, ldc, (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_sgesummv(pk_context *ctx, int64_t N, float alpha, const float *A, int64_t lda, float beta,
                      const float *B, int64_t ldb, const float *x, float *y, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (N < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (lda < std::max<int64_t>(N, 1) || ldb < std::max<int64_t>(N, 1))
        return fail(PK_ERR_SHAPE, "leading dimension smaller than N");
    if (N == 0)
        return PK_OK;
    PK_TRY(check_ptr(ctx, A, mat_bytes(N, N, lda), "A"));
    PK_TRY(check_ptr(ctx, B, mat_bytes(N, N, ldb), "B"));
    PK_TRY(check_ptr(ctx, x, (size_t)N * 4, "x"));
    PK_TRY(check_ptr(ctx, y, (size_t)N * 4, "y"));
    const Variant *v = pick(ctx, PKF_GESUMMV, N);
    pk_gesummv_args a{};
    a.A = A; a.B = B; a.x = x; a.y = y; a.N = N; a.lda = lda; a.ldb = ldb;
    a.alpha = alpha; a.beta = beta;
    a.aligned = aligned16(A) && aligned16(B) && aligned16(x) && lda % 4 == 0 && ldb % 4 == 0;
    const int64_t rows_per_block = (int64_t)v->knobs[PK_K_TM] * v->knobs[PK_K_WAVES_M];
    return launch(v, 0, cdiv(N, rows_per_block), v->knobs[PK_K_THREADS], &a, sizeof a, (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_smvt(pk_context *ctx, int64_t N, const float *A, int64_t lda, const float *y1, const float *y2,
                  float *x1, float *x2, void *ws, size_t ws_bytes, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (N < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (lda < std::max<int64_t>(N, 1))
        return fail(PK_ERR_SHAPE, "lda smaller than N");
    if (N == 0)
        return PK_OK;
    const Variant *v = pick(ctx, PKF_GEMV_PAIR, N);
    PK_TRY(one_launch_ok(ctx, v, PKF_GEMV_PAIR, ws));
    const int64_t rb = cdiv(N, v->knobs[PK_K_TM]);
    const int64_t strips = cdiv(N, v->knobs[PK_K_TN]);
    const int64_t wstrips = cdiv(N, v->knobs[PK_K_X1]);
    const GemvtLayout lay = gemvt_layout(true, N, N, rb, strips, wstrips);
    if (ws_bytes < lay.total())
        return fail(PK_ERR_INVALID_ARG, "workspace too small: %zu < %zu bytes", ws_bytes, lay.total());
    PK_TRY(check_ptr(ctx, A, mat_bytes(N, N, lda), "A"));
    PK_TRY(check_ptr(ctx, y1, (size_t)N * 4, "y1"));
    PK_TRY(check_ptr(ctx, y2, (size_t)N * 4, "y2"));
    PK_TRY(check_ptr(ctx, x1, (size_t)N * 4, "x1"));
    PK_TRY(check_ptr(ctx, x2, (size_t)N * 4, "x2"));
    PK_TRY(check_ptr(ctx, ws, lay.total(), "workspace"));
    if (rb > 0x7fffffff || wstrips > 0x7fffffff)
        return fail(PK_ERR_SHAPE, "problem too large");
    hipStream_t s = (hipStream_t)stream;
    // the fused pair: part1 = row dots with y1 (A y1), part2 = column sums with y2 (A^T y2)
    pk_gemvt_args a{};
    a.A = A; a.x = y1; a.z = y2; a.y1 = nullptr; a.y2 = nullptr;
    a.part2 = (float *)ws;
    a.part1 = (float *)((char *)ws + lay.part2 + lay.cells);
    a.M = N; a.N = N; a.lda = lda;
    a.aligned = aligned16(A) && lda % 4 == 0;
    a.row_blocks = (int32_t)rb;
    a.col_strips = (int32_t)wstrips;
    if (one_launch(v)) {
        // one launch: the folds add into x1 (A y1) and x2 (A^T y2)
        a.y1 = x1; a.y2 = x2;
        a.aligned |= 2;
        a.tag = next_tag(32);
        return launch(v, 0, rb * strips, v->knobs[PK_K_THREADS], &a, sizeof a, s);
    }
    PK_TRY(launch(v, 0, rb * strips, v->knobs[PK_K_THREADS], &a, sizeof a, s));
    const Variant *g = get_variant(ctx, ctx->def[PKF_GESUMMV]);
    pk_reduce_args r{};
    r.P1 = a.part1; r.y1 = x1; r.n1 = N; r.rows1 = (int32_t)wstrips;
    r.P2 = a.part2; r.y2 = x2; r.n2 = N; r.rows2 = (int32_t)rb;
    return launch(g, 1, cdiv(N, 16) * 2, 256, &r, sizeof r, s);
    PK_GUARD_END
}

pk_status pk_fdtd2d(pk_context *ctx, int64_t T, int64_t NX, int64_t NY, const float *fict, float *ex, float *ey,
                    float *hz, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (T < 0 || NX < 0 || NY < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (T == 0 || NX == 0 || NY == 0)
        return PK_OK;
    const size_t f = (size_t)NX * (size_t)NY * 4;
    PK_TRY(check_ptr(ctx, fict, (size_t)T * 4, "fict"));
    PK_TRY(check_ptr(ctx, ex, f, "ex"));
    PK_TRY(check_ptr(ctx, ey, f, "ey"));
    PK_TRY(check_ptr(ctx, hz, f, "hz"));
    const Variant *v = pick(ctx, PKF_FDTD, std::max(NX, NY));
    const int64_t grid = cdiv(NY, v->knobs[PK_K_TN]) * cdiv(NX, v->knobs[PK_K_TM]);
    hipStream_t s = (hipStream_t)stream;
    for (int64_t t = 0; t < T; ++t) {
        pk_fdtd_args a{ex, ey, hz, fict, NX, NY, t};
        PK_TRY(launch(v, 0, grid, v->knobs[PK_K_THREADS], &a, sizeof a, s));
        PK_TRY(launch(v, 1, grid, v->knobs[PK_K_THREADS], &a, sizeof a, s));
    }
    return PK_OK;
    PK_GUARD_END
}

// ---- variants ----------------------------------------------------------------------------

pk_status pk_variant_load(pk_context *ctx, const void *code, size_t bytes, pk_variant_id *out) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (!out)
        return fail(PK_ERR_INVALID_ARG, "out is NULL");
    *out = -1;
    return load_module(ctx, code, bytes, false, out);
    PK_GUARD_END
}

pk_status pk_variant_unload(pk_context *ctx, pk_variant_id id) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    std::lock_guard<std::mutex> lk(ctx->mu);
    const Variant *v = get_variant(ctx, id);
    if (!v)
        return fail(PK_ERR_NO_VARIANT, "unknown variant %d", id);
    if (v->builtin)
        return fail(PK_ERR_INVALID_ARG, "built-in variant %d cannot be unloaded", id);
    for (int f = 0; f < PKF_COUNT; ++f)
        if (ctx->forced[f] == id)
            ctx->forced[f] = -1;
    for (auto it = ctx->best.begin(); it != ctx->best.end();)
        it = (it->second == id) ? ctx->best.erase(it) : std::next(it);
    (void)hipModuleUnload(v->mod);
    ctx->variants[id].reset();
    return PK_OK;
    PK_GUARD_END
}

pk_status pk_variant_info(pk_context *ctx, pk_variant_id id, int32_t *family, int32_t knobs[PK_NKNOBS],
                          uint64_t *code_hash) {
    if (!ctx)
        return fail(PK_ERR_INVALID_ARG, "context is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    const Variant *v = get_variant(ctx, id);
    if (!v)
        return fail(PK_ERR_NO_VARIANT, "unknown variant %d", id);
    if (family)
        *family = v->family;
    if (knobs)
        std::memcpy(knobs, v->knobs, sizeof v->knobs);
    if (code_hash)
        *code_hash = v->hash;
    return PK_OK;
}

pk_status pk_variant_default(pk_context *ctx, int32_t family, pk_variant_id *out) {
    if (!ctx || !out)
        return fail(PK_ERR_INVALID_ARG, "NULL argument");
    if (family < 0 || family >= PKF_COUNT)
        return fail(PK_ERR_INVALID_ARG, "bad family %d", family);
    *out = ctx->def[family];
    return PK_OK;
}

pk_status pk_variant_select(pk_context *ctx, int32_t family, pk_variant_id id) {
    if (!ctx)
        return fail(PK_ERR_INVALID_ARG, "context is NULL");
    if (family < 0 || family >= PKF_COUNT)
        return fail(PK_ERR_INVALID_ARG, "bad family %d", family);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (id >= 0) {
        const Variant *v = get_variant(ctx, id);
        if (!v)
            return fail(PK_ERR_NO_VARIANT, "unknown variant %d", id);
        if (v->family != family)
            return fail(PK_ERR_INVALID_ARG, "variant %d is of family %d, not %d", id, v->family, family);
    }
    ctx->forced[family] = id < 0 ? -1 : id;
    return PK_OK;
}

pk_status pk_variant_set_best(pk_context *ctx, int32_t family, int32_t bucket, pk_variant_id id) {
    if (!ctx)
        return fail(PK_ERR_INVALID_ARG, "context is NULL");
    if (family < 0 || family >= PKF_COUNT)
        return fail(PK_ERR_INVALID_ARG, "bad family %d", family);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (id < 0) {
        ctx->best.erase({family, bucket});
        return PK_OK;
    }
    const Variant *v = get_variant(ctx, id);
    if (!v)
        return fail(PK_ERR_NO_VARIANT, "unknown variant %d", id);
    if (v->family != family)
        return fail(PK_ERR_INVALID_ARG, "variant %d is of family %d, not %d", id, v->family, family);
    ctx->best[{family, bucket}] = id;
    return PK_OK;
}

// ---- graphs --------------------------------------------------------------------------------

pk_status pk_graph_begin(pk_context *ctx, pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (!stream)
        return fail(PK_ERR_INVALID_ARG, "graph capture needs a non-default stream");
    PK_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return PK_OK;
    PK_GUARD_END
}

pk_status pk_graph_end(pk_context *ctx, pk_stream stream, pk_graph **out) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (!stream || !out)
        return fail(PK_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    auto g = std::make_unique<pk_graph>();
    PK_HIP(hipStreamEndCapture((hipStream_t)stream, &g->graph));
    hipError_t e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = g.release();
    return PK_OK;
    PK_GUARD_END
}

pk_status pk_graph_launch(pk_graph *g, pk_stream stream) {
    if (!g || !g->exec)
        return fail(PK_ERR_INVALID_ARG, "graph is NULL");
    PK_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return PK_OK;
}

void pk_graph_destroy(pk_graph *g) {
    if (!g)
        return;
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    delete g;
}

// ---- timing ----------------------------------------------------------------------------------

pk_status pk_timer_start(pk_context *ctx, pk_stream stream) {
    PK_TRY(check_ctx(ctx));
    PK_HIP(hipEventRecord(ctx->ev0, (hipStream_t)stream));
    return PK_OK;
}

pk_status pk_timer_stop(pk_context *ctx, pk_stream stream, double *ms) {
    PK_TRY(check_ctx(ctx));
    if (!ms)
        return fail(PK_ERR_INVALID_ARG, "ms is NULL");
    PK_HIP(hipEventRecord(ctx->ev1, (hipStream_t)stream));
    PK_HIP(hipEventSynchronize(ctx->ev1));
    float t = 0.f;
    PK_HIP(hipEventElapsedTime(&t, ctx->ev0, ctx->ev1));
    *ms = t;
    return PK_OK;
}

pk_status pk_graph_time(pk_context *ctx, pk_graph *g, int reps, pk_stream stream, double *ms) {
    PK_TRY(check_ctx(ctx));
    if (!g || !ms || reps <= 0)
        return fail(PK_ERR_INVALID_ARG, "bad argument");
    PK_HIP(hipEventRecord(ctx->ev0, (hipStream_t)stream));
    for (int i = 0; i < reps; ++i)
        PK_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    PK_HIP(hipEventRecord(ctx->ev1, (hipStream_t)stream));
    PK_HIP(hipEventSynchronize(ctx->ev1));
    float t = 0.f;
    PK_HIP(hipEventElapsedTime(&t, ctx->ev0, ctx->ev1));
    *ms = t / reps;
    return PK_OK;
}

pk_status pk_cache_flush(pk_context *ctx, pk_stream stream) {
    PK_GUARD_BEGIN
    PK_TRY(check_ctx(ctx));
    const size_t bytes = (size_t)512 << 20;
    if (!ctx->flush_buf) {
        PK_HIP(hipMalloc(&ctx->flush_buf, bytes));
        ctx->flush_bytes = bytes;
    }
    const Variant *v = get_variant(ctx, ctx->def[PKF_CONVERT]);
    struct {
        float *p;
        int64_t n;
        float value;
        int32_t pad;
    } a{(float *)ctx->flush_buf, (int64_t)(ctx->flush_bytes / 4), 0.f, 0};
    return launch(v, 1, 4096, 256, &a, sizeof a, (hipStream_t)stream);
    PK_GUARD_END
}

pk_status pk_stream_probe(pk_context *ctx, int kind, const float *src, float *dst, int64_t n,
                          pk_stream stream) {
    PK_GUARD_BEGIN
    g_err.clear();
    PK_TRY(check_ctx(ctx));
    if (kind < 0 || kind > 3)
        return fail(PK_ERR_INVALID_ARG, "bad probe kind %d", kind);
    if (n < 0)
        return fail(PK_ERR_SHAPE, "negative size");
    if (!aligned16(src) || !aligned16(dst))
        return fail(PK_ERR_ALIGNMENT, "probe buffers must be 16-byte aligned");
    PK_TRY(check_ptr(ctx, src, (size_t)n * 4, "src"));
    const int copy = kind & 1;
    PK_TRY(check_ptr(ctx, dst, copy ? (size_t)n * 4 : (size_t)PK_STREAM_BLOCKS * 4, "dst"));
    const Variant *v = get_variant(ctx, ctx->def[PKF_STREAM]);
    pk_stream_args a{src, dst, n, kind >> 1, 0};
    return launch(v, copy, PK_STREAM_BLOCKS, v->knobs[PK_K_THREADS], &a, sizeof a, (hipStream_t)stream);
    PK_GUARD_END
}

}  // extern "C"
