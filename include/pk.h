/*
 * pk.h -- C ABI of the MI355X (gfx950) kernel library for the data-parallel
 * kernel family of Nobre, Reis and Cardoso, "Improving OpenCL Performance by
 * Specializing Compiler Phase Selection and Ordering" (arXiv 1810.10496).
 *
 * The paper (Sec. 2.2) evaluates the PolyBench/GPU kernels; this library
 * implements the dense products (GEMM, 2MM/3MM), the matrix-vector pairs
 * (ATAX, BICG, MVT), the 3x3 and 3x3x3 stencils (2DCONV, 3DCONV) and the
 * correlation kernels (CORR: column mean/deviation, then a symmetric rank-k
 * product), plus the machinery its method needs: loading alternative compiled
 * versions ("variants") of each kernel, choosing between them, and running
 * mixed batches as captured HIP graphs.
 *
 * Conventions for every kernel entry point:
 *   - All matrices are FP32, row-major; `ld*` is the row stride in elements
 *     and must be >= the number of columns.  Sizes are int64_t.
 *   - Data pointers are caller-owned DEVICE memory (hipMalloc or a torch CUDA
 *     tensor).  They must stay valid until the enqueued work has completed
 *     (for a captured graph: for the graph's lifetime).  Host arrays of
 *     coefficients (`w`) are copied by value at call time.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *     asynchronous on it; nothing synchronises the host.
 *   - A call either enqueues its whole work and returns PK_OK, or enqueues
 *     nothing and returns an error; details via pk_last_error() (thread-local).
 *     Negative sizes, ld smaller than the row length, null pointers for a
 *     non-empty operand, pointers that are not device memory or whose extent
 *     overruns their allocation, and bad enum values are rejected this way.
 *     A size of zero in an output dimension is a legal no-op.  Device faults
 *     surface at the caller's next synchronisation, as for any HIP launch.
 *   - No entry point allocates device memory on the launch path; kernels that
 *     need scratch take a caller workspace (size from pk_workspace_bytes).
 *   - No C++ exception crosses the ABI; nothing aborts the process.
 */
#ifndef PK_H
#define PK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PK_ABI_VERSION 1

typedef enum pk_status {
    PK_OK = 0,
    PK_ERR_INVALID_ARG = 1,  /* null/invalid pointer, bad enum, workspace too small */
    PK_ERR_SHAPE = 2,        /* negative size or ld < row length */
    PK_ERR_ALIGNMENT = 3,    /* a workspace that must be 256-byte aligned is not (operands
                                need only 4-byte alignment) */
    PK_ERR_UNSUPPORTED = 4,  /* precision not offered by this kernel */
    PK_ERR_HIP = 5,          /* HIP runtime call failed */
    PK_ERR_NO_VARIANT = 6,   /* unknown variant id / code object not usable */
    PK_ERR_COMPILE = 7,      /* reserved for the variant compiler */
    PK_ERR_TIMEOUT = 8,      /* reserved for the variant evaluator */
    PK_ERR_VALIDATION = 9,   /* reserved for the variant evaluator */
    PK_ERR_IO = 10           /* reserved */
} pk_status;

/* Arithmetic of the contractions (gemm, gemm3, corr's rank-k product).
 * FP32: FP32 operands on v_mfma_f32_16x16x4_f32.
 * BF16: operands rounded to bfloat16 (nearest-even), FP32 accumulation.
 * SPLIT_BF16: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); the product
 *   hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32 accumulation (close to FP32
 *   accuracy at BF16 matrix-core rate).
 * Every other kernel is FP32 only and rejects other values (PK_ERR_UNSUPPORTED). */
typedef enum pk_precision {
    PK_FP32 = 0,
    PK_BF16 = 1,
    PK_SPLIT_BF16 = 2
} pk_precision;

/* Operations (for pk_workspace_bytes). */
typedef enum pk_kernel {
    PK_KERNEL_GEMM = 0,
    PK_KERNEL_GEMM3 = 1,
    PK_KERNEL_GEMV = 2,
    PK_KERNEL_GEMV_T = 3,
    PK_KERNEL_GEMV_PAIR = 4,
    PK_KERNEL_CONV2D = 5,
    PK_KERNEL_CONV3D = 6,
    PK_KERNEL_COLSTATS = 7,
    PK_KERNEL_CORR = 8,
    PK_KERNEL_CONVERT = 9,
    PK_KERNEL_COVAR = 10,
    PK_KERNEL_SYRK = 11,
    PK_KERNEL_SYR2K = 12,
    PK_KERNEL_GESUMMV = 13,
    PK_KERNEL_MVT = 14,
    PK_KERNEL_FDTD2D = 15
} pk_kernel;

/* Kernel families: one compiled code object implements one family. */
typedef enum pk_family {
    PK_FAMILY_GEMM_F32 = 0,
    PK_FAMILY_GEMM_BF16 = 1,
    PK_FAMILY_GEMM_SPLIT = 2,
    PK_FAMILY_GEMV = 3,
    PK_FAMILY_GEMV_T = 4,
    PK_FAMILY_GEMV_PAIR = 5,
    PK_FAMILY_CONV2D = 6,
    PK_FAMILY_CONV3D = 7,
    PK_FAMILY_COLSTATS = 8,
    PK_FAMILY_SYRK_F32 = 9,
    PK_FAMILY_SYRK_BF16 = 10,
    PK_FAMILY_SYRK_SPLIT = 11,
    PK_FAMILY_CONVERT = 12,
    PK_FAMILY_RANKK = 13,
    PK_FAMILY_GESUMMV = 14,
    PK_FAMILY_FDTD = 15,
    PK_FAMILY_GEMM_BF16_WS = 16,   /* bf16 GEMM from prepared operands (pk_sgemm_ws) */
    PK_FAMILY_GEMM_SPLIT_WS = 17,  /* split-bf16 GEMM from prepared operands (pk_sgemm_ws) */
    PK_FAMILY_STREAM = 18,         /* bandwidth probes (pk_stream_probe) */
    PK_FAMILY_COUNT = 19
} pk_family;

typedef struct pk_context pk_context;
typedef struct pk_graph pk_graph;
typedef void *pk_stream;        /* hipStream_t */
typedef int32_t pk_variant_id;  /* -1 = none */

#define PK_NKNOBS 16

/* ---- status ---------------------------------------------------------------- */
const char *pk_status_string(pk_status s);
/* Detail of the last error on the calling thread ("" if none).  Valid until the
 * next pk_* call on the same thread. */
const char *pk_last_error(void);
int pk_abi_version(void);

/* ---- context ---------------------------------------------------------------
 * A context binds one HIP device and owns the loaded code objects: the
 * built-in default variant of every family (embedded in this library and
 * loaded here) and any variants loaded later.  Launch calls on one context
 * may come from several threads; variant loading/selection must not race
 * with launches of the same family. */
pk_status pk_context_create(int device, pk_context **out);
void pk_context_destroy(pk_context *ctx);
/* Enable (default) or disable the per-call pointer checks (device memory,
 * extent within allocation). */
pk_status pk_context_set_checks(pk_context *ctx, int enabled);

/* ---- workspace --------------------------------------------------------------
 * Bytes of caller workspace an operation needs, an upper bound valid for every
 * variant of its family.  dims:
 *   GEMM {M,N,K} (pk_sgemm_ws; pk_sgemm takes none)  GEMM3 {M,N,K,L}  GEMV/GEMV_T/GEMV_PAIR {M,N}
 *   CONV2D {H,W}  CONV3D {D,H,W}  COLSTATS/CORR/COVAR {n,m}  CONVERT {n}
 *   SYRK/SYR2K {N,K}  GESUMMV {N}  MVT {N}  FDTD2D {T,NX,NY} */
pk_status pk_workspace_bytes(pk_kernel kernel, const int64_t *dims, int ndims,
                             pk_precision prec, size_t *out);

/* ---- kernels ------------------------------------------------------------------ */

/* GEMM (Sec. 2.2): C <- alpha * A B + beta * C.  A is M x K, B is K x N, C is
 * M x N, updated in place.  When beta == 0, C is not read (BLAS convention).
 * K == 0 gives C <- beta * C. */
pk_status pk_sgemm(pk_context *ctx, pk_precision prec, int64_t M, int64_t N, int64_t K,
                   float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
                   float beta, float *C, int64_t ldc, pk_stream stream);

/* GEMM as pk_sgemm, with a caller workspace (pk_workspace_bytes(PK_KERNEL_GEMM,
 * {M,N,K}, prec); 256-byte aligned; none needed for FP32).  For BF16 and
 * SPLIT_BF16 the operands are first rounded once into the workspace (A as
 * [M][Kp], B transposed to [N][Kp], Kp = K rounded up to 64, zero padded; hi and
 * lo planes for split), then multiplied from there: the same arithmetic as
 * pk_sgemm (RNE bf16 operands, FP32 accumulation; split = hi*hi + hi*lo + lo*hi)
 * with the rounding taken out of the product's inner loop.  The workspace is
 * overwritten; calls sharing one workspace must not overlap. */
pk_status pk_sgemm_ws(pk_context *ctx, pk_precision prec, int64_t M, int64_t N, int64_t K,
                      float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
                      float beta, float *C, int64_t ldc, void *ws, size_t ws_bytes,
                      pk_stream stream);

/* Chained product (2MM/3MM, Sec. 2.2): D <- alpha * (A B) Cm + beta * D with A
 * M x K, B K x L, Cm L x N, D M x N.  T = A B is formed first, as FP32, in the
 * workspace (M*L floats); alpha is applied once, in the second product.  For
 * BF16 / SPLIT_BF16 both products run as in pk_sgemm_ws (T is rounded, or
 * re-split, for the second product: by the first product's epilogue straight into
 * the second's prepared operand when the selected variant can, else by a separate
 * preparation of the FP32 T; the results are the same bit for bit) and the
 * workspace (pk_workspace_bytes(PK_KERNEL_GEMM3, ...), which covers both) must be
 * 256-byte aligned. */
pk_status pk_sgemm3(pk_context *ctx, pk_precision prec, int64_t M, int64_t N, int64_t K,
                    int64_t L, float alpha, const float *A, int64_t lda, const float *B,
                    int64_t ldb, const float *Cm, int64_t ldcm, float beta, float *D,
                    int64_t ldd, void *ws, size_t ws_bytes, pk_stream stream);

/* Matrix-vector (ATAX/BICG/MVT, Sec. 2.2): y = A x, A is M x N. */
pk_status pk_sgemv(pk_context *ctx, int64_t M, int64_t N, const float *A, int64_t lda,
                   const float *x, float *y, pk_stream stream);

/* Transpose matrix-vector: y = A^T z (z has M entries, y has N).  Column sums
 * are formed per row block in the workspace and reduced in a fixed order
 * (bitwise reproducible): by a second launch, or, with a one-launch variant, by the
 * last row block of each column strip to finish.  The workspace needs no clearing
 * (whatever it held before is overwritten or read as empty); a one-launch variant
 * needs it 16-byte aligned and otherwise the two-launch default runs instead.
 * Calls sharing one workspace must not overlap. */
pk_status pk_sgemv_t(pk_context *ctx, int64_t M, int64_t N, const float *A, int64_t lda,
                     const float *z, float *y, void *ws, size_t ws_bytes, pk_stream stream);

/* The BiCG pair in one pass over A: y1 = A x and y2 = A^T z (workspace as for
 * pk_sgemv_t). */
pk_status pk_sgemv_pair(pk_context *ctx, int64_t M, int64_t N, const float *A, int64_t lda,
                        const float *x, const float *z, float *y1, float *y2, void *ws,
                        size_t ws_bytes, pk_stream stream);

/* 2DCONV (Sec. 2.2): out[i][j] = sum_{di,dj in -1..1} w[(di+1)*3+(dj+1)] *
 * in[i+di][j+dj] for 1 <= i <= H-2, 1 <= j <= W-2 (no flip); every border cell
 * of out is written as 0.  in and out must not overlap. */
pk_status pk_conv2d_3x3(pk_context *ctx, int64_t H, int64_t W, const float w[9],
                        const float *in, int64_t ldi, float *out, int64_t ldo, pk_stream stream);

/* 3DCONV (Sec. 2.2): dense D x H x W volumes (x fastest), 27 taps indexed
 * (dz+1)*9 + (dy+1)*3 + (dx+1), no flip; every cell on a face of out is 0. */
pk_status pk_conv3d_3x3x3(pk_context *ctx, int64_t D, int64_t H, int64_t W, const float w[27],
                          const float *in, float *out, pk_stream stream);

/* CORR's mean/deviation kernels (Sec. 3.4): for the n x m matrix X (n samples,
 * m features), mean_j = (1/n) sum_i x_ij and std_j = max(sqrt((1/(n-1))
 * sum_i (x_ij - mean_j)^2), eps), in FP32 with compensated summation.
 * Requires n >= 2.  Per-segment partials in the workspace are merged in a fixed
 * order, by a second launch or, with a one-launch variant, by the last segment of
 * each column strip to finish (workspace rules as for pk_sgemv_t). */
pk_status pk_colstats(pk_context *ctx, int64_t n, int64_t m, const float *X, int64_t ldx,
                      float eps, float *mean, float *std, void *ws, size_t ws_bytes,
                      pk_stream stream);

/* CORR (Sec. 2.2): mean and std as pk_colstats, then R = Z^T Z / (n-1) with
 * Z = (X - mean) / std (R is m x m).  Only lower-triangle tiles are computed;
 * each value is written at (j,k) and (k,j), so R is exactly symmetric.  The
 * diagonal is computed, not forced to 1.  Requires n >= 2.
 * Workspace: pk_workspace_bytes(PK_KERNEL_CORR, {n,m}, prec).  For BF16 and
 * SPLIT_BF16 it also holds Z^T rounded (split) once, [m][np] bf16 with np = n
 * rounded up to 64 and zero padded, from which the product is formed
 * (z = (x - mean) * (1/std) in FP32, then rounded); the workspace must then be
 * 256-byte aligned (else PK_ERR_ALIGNMENT) and at least that size (else
 * PK_ERR_INVALID_ARG). */
pk_status pk_corr(pk_context *ctx, pk_precision prec, int64_t n, int64_t m, const float *X,
                  int64_t ldx, float eps, float *mean, float *std, float *R, int64_t ldr,
                  void *ws, size_t ws_bytes, pk_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): pk_corr without a workspace
 * argument.  The workspace pk_corr would take is the library's own static
 * device array of PK_NOALLOC_SCRATCH_BYTES per device, whose address is taken
 * once per device when the first context on it is created and which is held
 * until the process ends.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and otherwise behaves as pk_corr: same kernels,
 * same results, same argument checks; X, mean, std and R are the caller's.
 * A problem whose pk_corr workspace (pk_workspace_bytes(PK_KERNEL_CORR, {n,m},
 * prec)) exceeds the scratch is rejected with PK_ERR_SHAPE before anything is
 * enqueued.  Every call on one device shares that device's scratch and leaves
 * its contents behind (each call writes all it reads), so calls that overlap
 * on one device -- on two streams, or from two threads -- race and must be
 * serialised by the caller. */
#define PK_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
pk_status pk_corr_noalloc(pk_context *ctx, pk_precision prec, int64_t n, int64_t m,
                          const float *X, int64_t ldx, float eps, float *mean, float *std,
                          float *R, int64_t ldr, pk_stream stream);

/* COVAR (Sec. 2.2; same mean kernel as CORR, Sec. 3.4): mean as pk_colstats,
 * then C = (X - mean)^T (X - mean) / (n-1), m x m, lower-triangle tiles
 * mirrored (exactly symmetric), in the requested precision.  Requires n >= 2.
 * Workspace: pk_workspace_bytes(PK_KERNEL_COVAR, {n,m}, prec); BF16 and
 * SPLIT_BF16 prepare the centred operand in it as pk_corr does (256-byte
 * aligned). */
pk_status pk_covar(pk_context *ctx, pk_precision prec, int64_t n, int64_t m, const float *X,
                   int64_t ldx, float *mean, float *C, int64_t ldc, void *ws, size_t ws_bytes,
                   pk_stream stream);

/* SYRK (Sec. 2.2): C <- alpha A A^T + beta C, A is N x K, C is N x N (updated in
 * place; C need not be symmetric: each of C[i][j], C[j][i] keeps its own beta
 * term).  When beta == 0, C is not read.  FP32. */
pk_status pk_ssyrk(pk_context *ctx, int64_t N, int64_t K, float alpha, const float *A, int64_t lda,
                   float beta, float *C, int64_t ldc, pk_stream stream);

/* SYR2K (Sec. 2.2): C <- alpha (A B^T + B A^T) + beta C, A and B N x K.  FP32. */
pk_status pk_ssyr2k(pk_context *ctx, int64_t N, int64_t K, float alpha, const float *A, int64_t lda,
                    const float *B, int64_t ldb, float beta, float *C, int64_t ldc, pk_stream stream);

/* GESUMMV (Sec. 2.2): y = alpha A x + beta B x, A and B N x N; one pass over each. */
pk_status pk_sgesummv(pk_context *ctx, int64_t N, float alpha, const float *A, int64_t lda,
                      float beta, const float *B, int64_t ldb, const float *x, float *y,
                      pk_stream stream);

/* MVT (Sec. 2.2), accumulate form: x1 += A y1 and x2 += A^T y2 in one pass over
 * A (N x N).  Workspace as for PK_KERNEL_GEMV_PAIR / PK_KERNEL_MVT. */
pk_status pk_smvt(pk_context *ctx, int64_t N, const float *A, int64_t lda, const float *y1,
                  const float *y2, float *x1, float *x2, void *ws, size_t ws_bytes, pk_stream stream);

/* FDTD-2D (Sec. 2.2): T time steps on NX x NY fields ex, ey, hz (dense, updated
 * in place); fict holds T device floats, the source row of each step.  Each
 * step enqueues two kernels (E update, then H update). */
pk_status pk_fdtd2d(pk_context *ctx, int64_t T, int64_t NX, int64_t NY, const float *fict, float *ex,
                    float *ey, float *hz, pk_stream stream);

/* FP32 -> bfloat16 bits (round to nearest even): hi[i] = bf16(x[i]); if lo is
 * not NULL also lo[i] = bf16(x[i] - hi[i]).  The contractions apply the same
 * rounding internally. */
pk_status pk_convert_bf16(pk_context *ctx, int64_t n, const float *x, uint16_t *hi,
                          uint16_t *lo, pk_stream stream);

/* ---- variants ------------------------------------------------------------------
 * A variant is a gfx950 code object (ELF, or an offload bundle holding one)
 * built from this library's kernel source for one family with some knob
 * values and some LLVM pass pipeline.  Each code object records its family
 * and knobs (exported array `pk_knobs`), from which launch geometry follows.
 * Which variant a launch uses: the family's selected variant if set
 * (pk_variant_select), else the best variant registered for the problem's
 * size bucket (pk_variant_set_best), else the built-in default. */

/* Load a code object (copied).  Fails with PK_ERR_NO_VARIANT if it has no
 * valid knob record or lacks the family's entry points. */
pk_status pk_variant_load(pk_context *ctx, const void *code, size_t bytes, pk_variant_id *out);
/* Release a loaded variant (not a built-in default).  Its id becomes invalid;
 * selections and best-table entries naming it are cleared.  The caller must
 * ensure no enqueued work still uses it. */
pk_status pk_variant_unload(pk_context *ctx, pk_variant_id id);
/* Family, knobs and a 64-bit FNV-1a hash of the code object bytes. */
pk_status pk_variant_info(pk_context *ctx, pk_variant_id id, int32_t *family,
                          int32_t knobs[PK_NKNOBS], uint64_t *code_hash);
pk_status pk_variant_default(pk_context *ctx, int32_t family, pk_variant_id *out);
/* Force every launch of `family` to use `id` (-1 clears the selection). */
pk_status pk_variant_select(pk_context *ctx, int32_t family, pk_variant_id id);
/* Register `id` as the best variant of `family` for problems of `bucket`
 * (-1 clears).  See pk_size_bucket. */
pk_status pk_variant_set_best(pk_context *ctx, int32_t family, int32_t bucket, pk_variant_id id);
/* Size bucket of a problem: ceil(log2(largest dimension)), 0 for <= 1. */
int32_t pk_size_bucket(int64_t largest_dim);

/* ---- graphs ------------------------------------------------------------------------
 * Capture everything enqueued on `stream` between begin and end into a HIP
 * graph (stream capture; `stream` must not be NULL). */
pk_status pk_graph_begin(pk_context *ctx, pk_stream stream);
pk_status pk_graph_end(pk_context *ctx, pk_stream stream, pk_graph **out);
pk_status pk_graph_launch(pk_graph *g, pk_stream stream);
void pk_graph_destroy(pk_graph *g);

/* ---- timing helpers --------------------------------------------------------------
 * HIP-event timer on `stream`: start records an event, stop records a second
 * one, waits for it and returns the elapsed milliseconds. */
pk_status pk_timer_start(pk_context *ctx, pk_stream stream);
pk_status pk_timer_stop(pk_context *ctx, pk_stream stream, double *ms);
/* Launch `g` `reps` times back to back and return the mean milliseconds per
 * launch (HIP events on `stream`). */
pk_status pk_graph_time(pk_context *ctx, pk_graph *g, int reps, pk_stream stream, double *ms);
/* Evict caches (L2 and the Infinity Cache) by writing a 512 MiB scratch
 * buffer owned by the context (allocated on first use). */
pk_status pk_cache_flush(pk_context *ctx, pk_stream stream);
/* Bandwidth probes, the ceilings the memory-bound kernels are reported against
 * (not one of the paper's kernels).  kind 0 (read): every one of the n floats
 * of src is read once with 16-byte loads and dst[b] receives the sum of what
 * block b read, for b < PK_STREAM_BLOCKS (dst must hold that many floats);
 * kind 1 (copy): dst[i] = src[i] for i < n (src and dst must not overlap);
 * kinds 2 and 3: the same with non-temporal loads (and stores).
 * src and dst must be 16-byte aligned (else PK_ERR_ALIGNMENT); n >= 0. */
#define PK_STREAM_BLOCKS 2048
pk_status pk_stream_probe(pk_context *ctx, int kind, const float *src, float *dst, int64_t n,
                          pk_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* PK_H */
