// pk_kernel_abi.h -- argument blocks and knob layout shared by the host
// runtime and the device kernels.
//
// Every kernel entry point takes exactly one of these plain structs by value,
// so the runtime can launch any code object (built-in or tuned) through
// hipModuleLaunchKernel with a single parameter.  Every code object also
// exports `pk_knobs`, an int array holding the compile-time knobs it was built
// with (layout below); the runtime reads it at load time and derives the
// launch geometry from it, so a code object always describes itself.
#pragma once
#include <stdint.h>

#define PK_NKNOBS 16

// knob slots
enum {
    PK_K_FAMILY = 0,   // pk_family (below)
    PK_K_TM = 1,       // rows of the block tile / rows per block
    PK_K_TN = 2,       // columns of the block tile / columns per thread group
    PK_K_TK = 3,       // contraction tile depth / rows per segment
    PK_K_WAVES_M = 4,  // waves along the tile's rows (contractions) / waves per block
    PK_K_WAVES_N = 5,  // waves along the tile's columns (contractions)
    PK_K_VEC = 6,      // elements per vector memory access (1, 2, 4)
    PK_K_UNROLL = 7,   // unroll factor of the main loop
    PK_K_LDS = 8,      // 1: stage operands through LDS, 0: read them from memory directly
    PK_K_ORDER = 9,    // loop / tile-raster order
    PK_K_X1 = 10,      // family-specific extra knob
    PK_K_X2 = 11,      // family-specific extra knob
    PK_K_THREADS = 12, // threads per block (derived, checked at load)
    PK_K_LDS_BYTES = 13,
    PK_K_ABI = 14,     // PK_KERNEL_ABI_VERSION
    PK_K_X3 = 15       // family-specific: bf16 GEMM / rank-k families: source rows per block
                       // of the transposing operand preparation (0 means 64); transposed
                       // matvec, pair and column statistics: 1 = one launch (the last
                       // block of each group folds the partials), 0 = partials + reduce
};

#define PK_KERNEL_ABI_VERSION 3

// bytes between the ticket cells of the one-launch reductions (transposed matvec,
// pair, column statistics): one cache line and channel per group
#define PK_CELL_STRIDE 256

// kernel families: one code object implements one family
enum pk_family_id {
    PKF_GEMM_F32 = 0,
    PKF_GEMM_BF16 = 1,
    PKF_GEMM_SPLIT = 2,
    PKF_GEMV = 3,
    PKF_GEMV_T = 4,
    PKF_GEMV_PAIR = 5,
    PKF_CONV2D = 6,
    PKF_CONV3D = 7,
    PKF_COLSTATS = 8,
    PKF_SYRK_F32 = 9,
    PKF_SYRK_BF16 = 10,
    PKF_SYRK_SPLIT = 11,
    PKF_CONVERT = 12,
    PKF_RANKK = 13,      // SYRK / SYR2K (C = alpha A A^T + beta C, alpha (A B^T + B A^T) + beta C)
    PKF_GESUMMV = 14,    // y = alpha A x + beta B x; accumulating column-sum reduce (MVT)
    PKF_FDTD = 15,       // FDTD-2D field updates
    PKF_GEMM_BF16_WS = 16,   // bf16 GEMM from operands prepared in a workspace (+ the preparation)
    PKF_GEMM_SPLIT_WS = 17,  // split-bf16 GEMM from prepared operands (+ the preparation)
    PKF_STREAM = 18,         // bandwidth probes (read-only and copy ceilings)
    PKF_COUNT = 19
};

// C <- alpha * A B + beta * C   (row-major, FP32 storage)
struct pk_gemm_args {
    const float *A;
    const float *B;
    const float *C;   // read only when beta != 0
    float *D;         // output (may equal C)
    int64_t M, N, K;
    int64_t lda, ldb, ldc, ldd;
    float alpha, beta;
    int32_t aligned;  // 1: every row start is 16-byte aligned (vector path allowed)
    int32_t pad_;
};

// y = A x   (A is M x N row-major)
struct pk_gemv_args {
    const float *A;
    const float *x;
    float *y;
    int64_t M, N, lda;
    int32_t aligned;
    int32_t pad_;
};

// y2 = A^T z (and, for the pair, y1 = A x) via per-block partial sums
struct pk_gemvt_args {
    const float *A;
    const float *x;     // pair only
    const float *z;
    float *y1;          // pair only
    float *y2;
    float *part1;       // pair only: [col_strips][M]
    float *part2;       // [row_blocks][N]
    int64_t M, N, lda;
    int32_t aligned;    // bit 0: rows of A start 16-byte aligned; bit 1 (one-launch variants):
                        // add the results to y1 / y2 instead of storing them (MVT's x += A y)
    int32_t row_blocks; // number of row blocks (rows of part2)
    int32_t col_strips; // number of column strips (rows of part1)
    uint32_t tag;       // one-launch variants: the call's ticket tag (never 0)
};

// fixed-order column sums of a partial-sum matrix: y[j] = sum_r P[r][j]
struct pk_reduce_args {
    const float *P1;
    float *y1;
    int64_t n1;        // columns of P1
    int32_t rows1;     // rows of P1
    int32_t pad1_;
    const float *P2;   // optional second matrix (pair): may be null
    float *y2;
    int64_t n2;
    int32_t rows2;
    int32_t pad2_;
};

// bandwidth probes: read n floats of src (dst: one float per block) or copy them to dst
struct pk_stream_args {
    const float *src;
    float *dst;
    int64_t n;
    int32_t nt;        // 1: non-temporal loads and stores
    int32_t pad_;
};

// 3x3 stencil
struct pk_conv2d_args {
    const float *in;
    float *out;
    int64_t H, W, ldi, ldo;
    float w[9];
    int32_t aligned;
};

// 3x3x3 stencil on a dense D x H x W volume
struct pk_conv3d_args {
    const float *in;
    float *out;
    int64_t D, H, W;
    float w[27];
    int32_t aligned;
};

// column statistics, stage 1 (per row segment) and stage 2 (merge)
struct pk_colstats_args {
    const float *X;
    float *part;       // [segments][3][m]: compensated sum (hi, lo), M2 about the segment mean
    float *mean;
    float *std;
    int64_t n, m, ldx;
    float eps;
    int32_t segments;
    int32_t seg_rows;  // rows per segment
    int32_t aligned;   // bit 0: rows of X start 16-byte aligned; bits 1-31 (one-launch
                       // variants): the call's ticket tag (never 0)
};

// R = Z^T Z / (n-1), Z = (X - mean) / std, lower-triangle tiles mirrored
struct pk_syrk_args {
    const float *X;
    const float *mean;
    const float *std;
    float *R;
    int64_t n, m, ldx, ldr;
    int32_t aligned;
    int32_t pad_;
};

// lower-triangle rank-k / rank-2k update of an N x N matrix C (in place):
//   mode 0: C = alpha A A^T + beta C          mode 1: C = alpha (A B^T + B A^T) + beta C
// A and B are N x K row-major; C may be non-symmetric on input (each of C[i][j]
// and C[j][i] gets its own beta term; the product part is shared).
struct pk_rankk_args {
    const float *A;
    const float *B;
    float *C;
    int64_t N, K, lda, ldb, ldc;
    float alpha, beta;
    int32_t aligned;
    int32_t pad_;
};

// y = alpha A x + beta B x  (A, B N x N row-major)
struct pk_gesummv_args {
    const float *A;
    const float *B;
    const float *x;
    float *y;
    int64_t N, lda, ldb;
    float alpha, beta;
    int32_t aligned;
    int32_t pad_;
};

// FDTD-2D fields, NX x NY row-major, one time step t (fict on the device)
struct pk_fdtd_args {
    float *ex;
    float *ey;
    float *hz;
    const float *fict;
    int64_t NX, NY, t;
};

// FP32 -> bfloat16 (RNE); mode 0: hi only, 1: hi and lo = bf16(x - hi)
struct pk_convert_args {
    const float *x;
    uint16_t *hi;
    uint16_t *lo;
    int64_t n;
    int32_t mode;
    int32_t pad_;
};

// D <- alpha * A B + beta * C from prepared bf16 operands: A as [M][Kp], B as
// B^T [N][Kp] (hi planes; lo planes for split, else unused), Kp a multiple of 64
// with zeros beyond K
struct pk_gemmbf_args {
    const uint16_t *Ah;
    const uint16_t *Al;
    const uint16_t *Bh;
    const uint16_t *Bl;
    const float *C;   // read only when beta != 0
    float *D;
    int64_t M, N, Kp;
    int64_t ldc, ldd;
    float alpha, beta;
};

// FP32 rows x cols (row stride ld) -> bf16 hi (and lo when split) with row
// stride ldo; transpose != 0 writes the transpose ([cols][ldo])
struct pk_gemmprep_args {
    const float *src;
    uint16_t *hi;
    uint16_t *lo;
    int64_t rows, cols, ld, ldo;
    int32_t transpose;
    int32_t split;
};

// Correlation / covariance operand: X is n samples x m features (row stride
// ldx); writes Z^T as bf16 hi (and lo when split), [m][ldo], with
// z_ij = (x_ij - mean_j) * (1 / std_j) for i < n and 0 for n <= i < ldo
struct pk_corrprep_args {
    const float *X;
    const float *mean;
    const float *std;
    uint16_t *hi;
    uint16_t *lo;
    int64_t n, m, ldx, ldo;
    int32_t split;
    int32_t pad;
};
