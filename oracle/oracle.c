/*
 * oracle.c -- plain FP64 CPU oracle for the data-parallel kernel family.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this file: it is used by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg, and by nothing else.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What it computes.  The paper (Sec. 2.2) names its kernels (GEMM, 2MM/3MM,
 * ATAX/BICG/MVT, 2DCONV/3DCONV, CORR) but does not print their definitions,
 * so each function below is the textbook definition of the operation, written
 * as plainly as possible:
 *   - every input is the FP32 array the GPU sees, widened exactly to double;
 *     scalars are their FP32 values widened (beta = (double)1.2f, ...);
 *   - every sum runs in ascending index order in double, so the result does
 *     not depend on the number of OpenMP threads (only the outermost output
 *     index is split between threads);
 *   - there is no blocking, fusion or reordering beyond a transposed copy of
 *     an operand so that a dot product reads contiguous memory (the order of
 *     the additions is unchanged by it).
 *
 * All output arrays are dense, row-major, caller-allocated doubles.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops that follow (n >= 1); the results do not depend
 * on it (every sum runs in a fixed order inside one thread). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Dense product (GEMM, Sec. 2.2):  r_ij = alpha * sum_k a_ik b_kj + beta * c_ij
 * A is M x K (row stride lda), B is K x N (ldb), C is M x N (ldc).
 * ------------------------------------------------------------------------ */
void oracle_gemm(int64_t M, int64_t N, int64_t K, float alpha,
                 const float *A, int64_t lda, const float *B, int64_t ldb,
                 float beta, const float *C, int64_t ldc, double *out)
{
    double *Bt = (double *)malloc(sizeof(double) * (size_t)(N * K + 1));
    for (int64_t k = 0; k < K; ++k)
        for (int64_t j = 0; j < N; ++j)
            Bt[j * K + k] = (double)B[k * ldb + j];
    const double a = (double)alpha, b = (double)beta;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            double acc = 0.0;
            const double *bt = Bt + j * K;
            for (int64_t k = 0; k < K; ++k)
                acc += (double)A[i * lda + k] * bt[k];
            out[i * N + j] = a * acc + b * (double)C[i * ldc + j];
        }
    }
    free(Bt);
}

/* ------------------------------------------------------------------------
 * Chained product (2MM/3MM family, Sec. 2.2):
 *   t_il = sum_k a_ik b_kl             (kept in double, never rounded)
 *   r_ij = alpha * sum_l t_il c_lj + beta * d_ij
 * A M x K, B K x L, C L x N, D M x N.
 * ------------------------------------------------------------------------ */
void oracle_gemm3(int64_t M, int64_t N, int64_t K, int64_t L, float alpha,
                  const float *A, int64_t lda, const float *B, int64_t ldb,
                  const float *C, int64_t ldc, float beta, const float *D,
                  int64_t ldd, double *out)
{
    double *Bt = (double *)malloc(sizeof(double) * (size_t)(L * K + 1));
    double *Ct = (double *)malloc(sizeof(double) * (size_t)(N * L + 1));
    double *T = (double *)malloc(sizeof(double) * (size_t)(M * L + 1));
    for (int64_t k = 0; k < K; ++k)
        for (int64_t l = 0; l < L; ++l)
            Bt[l * K + k] = (double)B[k * ldb + l];
    for (int64_t l = 0; l < L; ++l)
        for (int64_t j = 0; j < N; ++j)
            Ct[j * L + l] = (double)C[l * ldc + j];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t l = 0; l < L; ++l) {
            double acc = 0.0;
            for (int64_t k = 0; k < K; ++k)
                acc += (double)A[i * lda + k] * Bt[l * K + k];
            T[i * L + l] = acc;
        }
    const double a = (double)alpha, b = (double)beta;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int64_t l = 0; l < L; ++l)
                acc += T[i * L + l] * Ct[j * L + l];
            out[i * N + j] = a * acc + b * (double)D[i * ldd + j];
        }
    free(Bt);
    free(Ct);
    free(T);
}

/* ------------------------------------------------------------------------
 * Matrix-vector pair (ATAX / BICG / MVT, Sec. 2.2):
 *   y1_i = sum_j a_ij x_j      (A is M x N)
 *   y2_j = sum_i a_ij z_i
 * ------------------------------------------------------------------------ */
void oracle_gemv(int64_t M, int64_t N, const float *A, int64_t lda,
                 const float *x, double *y1)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < N; ++j)
            acc += (double)A[i * lda + j] * (double)x[j];
        y1[i] = acc;
    }
}

void oracle_gemv_t(int64_t M, int64_t N, const float *A, int64_t lda,
                   const float *z, double *y2)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        double acc = 0.0;
        for (int64_t i = 0; i < M; ++i)
            acc += (double)A[i * lda + j] * (double)z[i];
        y2[j] = acc;
    }
}

/* ------------------------------------------------------------------------
 * 3x3 stencil (2DCONV, Sec. 2.2), no kernel flip:
 *   r_ij = sum_{di,dj in -1..1} w[(di+1)*3 + (dj+1)] * x[i+di][j+dj]
 * for 1 <= i <= H-2 and 1 <= j <= W-2; every border cell of r is 0.
 * ------------------------------------------------------------------------ */
void oracle_conv2d(int64_t H, int64_t W, const float *w, const float *in,
                   int64_t ldi, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < H; ++i)
        for (int64_t j = 0; j < W; ++j) {
            if (i == 0 || j == 0 || i == H - 1 || j == W - 1) {
                out[i * W + j] = 0.0;
                continue;
            }
            double acc = 0.0;
            for (int di = -1; di <= 1; ++di)
                for (int dj = -1; dj <= 1; ++dj)
                    acc += (double)w[(di + 1) * 3 + (dj + 1)] *
                           (double)in[(i + di) * ldi + (j + dj)];
            out[i * W + j] = acc;
        }
}

/* ------------------------------------------------------------------------
 * 3x3x3 stencil (3DCONV, Sec. 2.2), dense D x H x W volume, no flip:
 *   r_zyx = sum_{dz,dy,dx} w[(dz+1)*9 + (dy+1)*3 + (dx+1)] * x[z+dz][y+dy][x+dx]
 * on the interior; every cell on a face of the volume is 0.
 * ------------------------------------------------------------------------ */
void oracle_conv3d(int64_t D, int64_t H, int64_t W, const float *w,
                   const float *in, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < D; ++z)
        for (int64_t y = 0; y < H; ++y)
            for (int64_t x = 0; x < W; ++x) {
                int64_t o = (z * H + y) * W + x;
                if (z == 0 || y == 0 || x == 0 || z == D - 1 || y == H - 1 ||
                    x == W - 1) {
                    out[o] = 0.0;
                    continue;
                }
                double acc = 0.0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx)
                            acc += (double)w[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] *
                                   (double)in[((z + dz) * H + (y + dy)) * W + (x + dx)];
                out[o] = acc;
            }
}

/* ------------------------------------------------------------------------
 * Column statistics (CORR's mean and deviation kernels, Sec. 3.4):
 *   mu_j    = (1/n) sum_i x_ij
 *   sigma_j = sqrt( (1/(n-1)) sum_i (x_ij - mu_j)^2 )   (two passes)
 *   sigma_j = max(sigma_j, eps)
 * X is n samples (rows) x m features (columns), row stride ldx.
 * ------------------------------------------------------------------------ */
void oracle_colstats(int64_t n, int64_t m, const float *X, int64_t ldx,
                     float eps, double *mean, double *std)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i)
            s += (double)X[i * ldx + j];
        double mu = s / (double)n;
        double q = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double d = (double)X[i * ldx + j] - mu;
            q += d * d;
        }
        double sd = sqrt(q / (double)(n - 1));
        if (sd < (double)eps)
            sd = (double)eps;
        mean[j] = mu;
        std[j] = sd;
    }
}

/* ------------------------------------------------------------------------
 * Correlation (CORR, Sec. 2.2 / 3.4):
 *   z_ij  = (x_ij - mu_j) / sigma_j           (mu, sigma from oracle_colstats)
 *   R_jk  = (1/(n-1)) sum_i z_ij z_ik         for every j, k (full matrix)
 * and the matching error scale  S_jk = (1/(n-1)) sum_i |z_ij z_ik|.
 * R and S are m x m; S may be NULL.
 * ------------------------------------------------------------------------ */
void oracle_corr(int64_t n, int64_t m, const float *X, int64_t ldx, float eps,
                 double *R, double *S)
{
    double *mean = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *std = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *Zt = (double *)malloc(sizeof(double) * (size_t)(m * n + 1));
    oracle_colstats(n, m, X, ldx, eps, mean, std);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i < n; ++i)
            Zt[j * n + i] = ((double)X[i * ldx + j] - mean[j]) / std[j];
    const double inv = 1.0 / (double)(n - 1);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j)
        for (int64_t k = 0; k < m; ++k) {
            const double *zj = Zt + j * n, *zk = Zt + k * n;
            double acc = 0.0, aabs = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                acc += zj[i] * zk[i];
                aabs += fabs(zj[i] * zk[i]);
            }
            R[j * m + k] = acc * inv;
            if (S)
                S[j * m + k] = aabs * inv;
        }
    free(mean);
    free(std);
    free(Zt);
}

/* ------------------------------------------------------------------------
 * BF16 rounding and the split representation used by the reduced-precision
 * contractions.
 *
 * bf16_rne(x): x rounded to the nearest value with an 8-bit significand
 * (bfloat16), ties to even.  Written from that definition in double: with
 * e = floor(log2|x|) the spacing of bfloat16 values around |x| is 2^(e-7)
 * (2^-133 for the subnormal range, the FP32 subnormal spacing is 2^-149 and
 * bfloat16 keeps 7 fraction bits); |x| / spacing is rounded to the nearest
 * integer, ties to even, and scaled back.  Finite inputs only; results that
 * exceed the largest bfloat16 become infinite.
 *
 * split: hi = bf16_rne(x), lo = bf16_rne(x - hi) (x - hi is exact in FP32).
 * ------------------------------------------------------------------------ */
static double round_half_even(double v)
{
    double f = floor(v);
    double r = v - f;
    if (r > 0.5)
        return f + 1.0;
    if (r < 0.5)
        return f;
    return (fmod(f, 2.0) == 0.0) ? f : f + 1.0;
}

float oracle_bf16_rne(float x)
{
    double a = fabs((double)x);
    if (a == 0.0)
        return x;
    int e;
    frexp(a, &e);              /* a = f * 2^e, f in [0.5, 1) -> floor(log2 a) = e - 1 */
    int ulp_exp = (e - 1) - 7; /* spacing of 8-bit significands at this binade */
    if (ulp_exp < -133)
        ulp_exp = -133;        /* bfloat16 subnormal spacing */
    double q = round_half_even(ldexp(a, -ulp_exp));
    double r = ldexp(q, ulp_exp);
    /* largest finite bfloat16 is (2 - 2^-7) * 2^127 */
    if (r > ldexp(2.0 - ldexp(1.0, -7), 127))
        r = INFINITY;
    return (float)(x < 0 ? -r : r);
}

void oracle_bf16_rne_array(int64_t n, const float *in, float *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = oracle_bf16_rne(in[i]);
}

void oracle_split_bf16(int64_t n, const float *in, float *hi, float *lo)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float h = oracle_bf16_rne(in[i]);
        hi[i] = h;
        lo[i] = oracle_bf16_rne(in[i] - h);
    }
}

/* ------------------------------------------------------------------------
 * Split-product diagnostic: the exact (double) value of the three-term
 * product alpha * sum_k (ah bh + ah bl + al bh) + beta * c, i.e. the product
 * the split path evaluates before any accumulation rounding.  Separates the
 * truncation error of dropping al*bl from the GPU's accumulation error.
 * ------------------------------------------------------------------------ */
void oracle_gemm_split3(int64_t M, int64_t N, int64_t K, float alpha,
                        const float *A, int64_t lda, const float *B, int64_t ldb,
                        float beta, const float *C, int64_t ldc, double *out)
{
    float *Ah = (float *)malloc(sizeof(float) * (size_t)(M * K + 1));
    float *Al = (float *)malloc(sizeof(float) * (size_t)(M * K + 1));
    float *Bh = (float *)malloc(sizeof(float) * (size_t)(K * N + 1));
    float *Bl = (float *)malloc(sizeof(float) * (size_t)(K * N + 1));
    for (int64_t i = 0; i < M; ++i)
        for (int64_t k = 0; k < K; ++k) {
            float x = A[i * lda + k], h = oracle_bf16_rne(x);
            Ah[i * K + k] = h;
            Al[i * K + k] = oracle_bf16_rne(x - h);
        }
    for (int64_t k = 0; k < K; ++k)
        for (int64_t j = 0; j < N; ++j) {
            float x = B[k * ldb + j], h = oracle_bf16_rne(x);
            Bh[j * K + k] = h;
            Bl[j * K + k] = oracle_bf16_rne(x - h);
        }
    const double a = (double)alpha, b = (double)beta;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                double ah = Ah[i * K + k], al = Al[i * K + k];
                double bh = Bh[j * K + k], bl = Bl[j * K + k];
                acc += ah * bh + ah * bl + al * bh;
            }
            out[i * N + j] = a * acc + b * (double)C[i * ldc + j];
        }
    free(Ah);
    free(Al);
    free(Bh);
    free(Bl);
}

/* ------------------------------------------------------------------------
 * Covariance (COVAR, Sec. 2.2; same mean kernel as CORR, Sec. 3.4):
 *   C_jk = (1/(n-1)) sum_i (x_ij - mu_j)(x_ik - mu_k)
 * ------------------------------------------------------------------------ */
void oracle_covar(int64_t n, int64_t m, const float *X, int64_t ldx, double *C)
{
    double *mean = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *Dt = (double *)malloc(sizeof(double) * (size_t)(m * n + 1));
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i)
            s += (double)X[i * ldx + j];
        mean[j] = s / (double)n;
        for (int64_t i = 0; i < n; ++i)
            Dt[j * n + i] = (double)X[i * ldx + j] - mean[j];
    }
    const double inv = 1.0 / (double)(n - 1);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j)
        for (int64_t k = 0; k < m; ++k) {
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i)
                acc += Dt[j * n + i] * Dt[k * n + i];
            C[j * m + k] = acc * inv;
        }
    free(mean);
    free(Dt);
}

/* ------------------------------------------------------------------------
 * Symmetric rank-k update (SYRK, Sec. 2.2), A is N x K:
 *   r_ij = alpha * sum_k a_ik a_jk + beta * c_ij          (every i, j)
 * Symmetric rank-2k update (SYR2K):
 *   r_ij = alpha * sum_k (a_ik b_jk + b_ik a_jk) + beta * c_ij
 * ------------------------------------------------------------------------ */
void oracle_syrk(int64_t N, int64_t K, float alpha, const float *A, int64_t lda,
                 float beta, const float *C, int64_t ldc, double *out)
{
    const double a = (double)alpha, b = (double)beta;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < K; ++k)
                acc += (double)A[i * lda + k] * (double)A[j * lda + k];
            out[i * N + j] = a * acc + b * (double)C[i * ldc + j];
        }
}

void oracle_syr2k(int64_t N, int64_t K, float alpha, const float *A, int64_t lda,
                  const float *B, int64_t ldb, float beta, const float *C, int64_t ldc,
                  double *out)
{
    const double a = (double)alpha, b = (double)beta;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < K; ++k)
                acc += (double)A[i * lda + k] * (double)B[j * ldb + k] +
                       (double)B[i * ldb + k] * (double)A[j * lda + k];
            out[i * N + j] = a * acc + b * (double)C[i * ldc + j];
        }
}

/* ------------------------------------------------------------------------
 * Scalar, vector and matrix multiplication (GESUMMV, Sec. 2.2), A, B N x N:
 *   y_i = alpha * sum_j a_ij x_j + beta * sum_j b_ij x_j
 * Matrix-vector product and transpose (MVT), accumulate form:
 *   x1_i += sum_j a_ij y1_j ;   x2_i += sum_j a_ji y2_j
 * ------------------------------------------------------------------------ */
void oracle_gesummv(int64_t N, float alpha, const float *A, int64_t lda, float beta,
                    const float *B, int64_t ldb, const float *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double sa = 0.0, sb = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            sa += (double)A[i * lda + j] * (double)x[j];
            sb += (double)B[i * ldb + j] * (double)x[j];
        }
        y[i] = (double)alpha * sa + (double)beta * sb;
    }
}

void oracle_mvt(int64_t N, const float *A, int64_t lda, const float *y1, const float *y2,
                const float *x1, const float *x2, double *x1_out, double *x2_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double s1 = 0.0, s2 = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            s1 += (double)A[i * lda + j] * (double)y1[j];
            s2 += (double)A[j * lda + i] * (double)y2[j];
        }
        x1_out[i] = (double)x1[i] + s1;
        x2_out[i] = (double)x2[i] + s2;
    }
}

/* ------------------------------------------------------------------------
 * 2D finite-difference time domain (FDTD-2D, Sec. 2.2), NX x NY fields,
 * T steps; for each step t, in this order:
 *   ey[0][j]  = fict[t]                                         (all j)
 *   ey[i][j] -= 0.5 (hz[i][j] - hz[i-1][j])                     (i >= 1)
 *   ex[i][j] -= 0.5 (hz[i][j] - hz[i][j-1])                     (j >= 1)
 *   hz[i][j] -= c (ex[i][j+1] - ex[i][j] + ey[i+1][j] - ey[i][j])
 *                                                   (i < NX-1, j < NY-1)
 * with c = 0.7 as the FP32 value the GPU multiplies by, widened.
 * Fields are updated in place (inputs are copied to the double outputs first).
 * If sex/sey/shz are not NULL they receive each element's error scale.  An
 * update's own scale is the sum of the magnitudes of its terms (for ey[i][j]:
 * |ey| + 0.5(|hz[i][j]| + |hz[i-1][j]|), with the values it read).  A rounding
 * error committed anywhere travels on through every later update that reads
 * the element, so an element's error scale is the largest own scale of any
 * update in its domain of dependence: the maximum of its update's own scale and
 * the error scales of the elements that update read.  The initial values (and
 * the source assignments of row 0 of ey) carry their own magnitudes.
 * ------------------------------------------------------------------------ */
void oracle_fdtd2d(int64_t T, int64_t NX, int64_t NY, const float *fict, const float *ex0,
                   const float *ey0, const float *hz0, double *ex, double *ey, double *hz,
                   double *sex, double *sey, double *shz)
{
    const double c = (double)0.7f;
    const int scales = sex != NULL && sey != NULL && shz != NULL;
    for (int64_t i = 0; i < NX * NY; ++i) {
        ex[i] = (double)ex0[i];
        ey[i] = (double)ey0[i];
        hz[i] = (double)hz0[i];
        if (scales) {
            sex[i] = fabs(ex[i]);
            sey[i] = fabs(ey[i]);
            shz[i] = fabs(hz[i]);
        }
    }
    for (int64_t t = 0; t < T; ++t) {
        for (int64_t j = 0; j < NY; ++j) {
            ey[j] = (double)fict[t];
            if (scales)
                sey[j] = fabs(ey[j]);
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 1; i < NX; ++i)
            for (int64_t j = 0; j < NY; ++j) {
                const int64_t o = i * NY + j;
                if (scales)
                    sey[o] = fmax(fmax(fabs(ey[o]) + 0.5 * (fabs(hz[o]) + fabs(hz[o - NY])), sey[o]),
                                  fmax(shz[o], shz[o - NY]));
                ey[o] -= 0.5 * (hz[o] - hz[o - NY]);
            }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < NX; ++i)
            for (int64_t j = 1; j < NY; ++j) {
                const int64_t o = i * NY + j;
                if (scales)
                    sex[o] = fmax(fmax(fabs(ex[o]) + 0.5 * (fabs(hz[o]) + fabs(hz[o - 1])), sex[o]),
                                  fmax(shz[o], shz[o - 1]));
                ex[o] -= 0.5 * (hz[o] - hz[o - 1]);
            }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < NX - 1; ++i)
            for (int64_t j = 0; j < NY - 1; ++j) {
                const int64_t o = i * NY + j;
                if (scales) {
                    const double own = fabs(hz[o]) + c * (fabs(ex[o + 1]) + fabs(ex[o]) + fabs(ey[o + NY]) + fabs(ey[o]));
                    const double rd = fmax(fmax(sex[o + 1], sex[o]), fmax(sey[o + NY], sey[o]));
                    shz[o] = fmax(fmax(own, shz[o]), rd);
                }
                hz[o] -= c * (ex[o + 1] - ex[o] + ey[o + NY] - ey[o]);
            }
    }
}
