// gesummv.hip -- GESUMMV and the accumulate half of MVT (Sec. 2.2).
//
//   pk_gesummv:           y = alpha A x + beta B x    (A, B N x N)
//   pk_colsum_accumulate: y[j] += sum_r P[r][j]       (MVT: x1 += A y1, x2 += A^T y2,
//                         from the partial sums of the fused matrix-vector pair)
//
// GESUMMV reads A and B once each: a wavefront walks ROWS rows of both with
// VEC-wide loads, keeps both sums in registers and stores y once (the
// paper's finding for this kernel, Sec. 3.4, is exactly that store).
#include "pk_device.h"

#ifndef VEC
#define VEC 4
#endif
#ifndef WAVES
#define WAVES 4
#endif
#ifndef ROWS
#define ROWS 1
#endif
#ifndef UNROLL
#define UNROLL 4
#endif
#ifndef NTL           // 1: the streamed matrices are read with the non-temporal hint
#define NTL 0
#endif
#if NTL
#define PK_LDM pk_ldv_nt
#else
#define PK_LDM pk_ldv
#endif

constexpr int NT = 64 * WAVES;

PK_DEFINE_KNOBS(PKF_GESUMMV, ROWS, 64 * VEC, 0, WAVES, 1, VEC, UNROLL, 0, 0, 0, 0, NT, 0,
                PK_KERNEL_ABI_VERSION, 0)

template <int V>
__device__ __forceinline__ void gesummv_body(const pk_gesummv_args &a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t row0 = ((int64_t)blockIdx.x * WAVES + wave) * ROWS;
    if (row0 >= a.N)
        return;
    float sa[ROWS], sb[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        sa[r] = 0.f;
        sb[r] = 0.f;
    }
#pragma unroll UNROLL
    for (int64_t j0 = 0; j0 < a.N; j0 += 64 * V) {
        const int64_t j = j0 + lane * V;
        if (j + V <= a.N) {
            float xv[V];
            pk_ldv<V>(a.x + j, xv);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t row = min(row0 + r, a.N - 1);
                float av[V], bv[V];
                PK_LDM<V>(a.A + row * a.lda + j, av);
                PK_LDM<V>(a.B + row * a.ldb + j, bv);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    sa[r] += av[e] * xv[e];
                    sb[r] += bv[e] * xv[e];
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                if (j + e < a.N) {
                    const float xe = a.x[j + e];
#pragma unroll
                    for (int r = 0; r < ROWS; ++r) {
                        const int64_t row = min(row0 + r, a.N - 1);
                        sa[r] += a.A[row * a.lda + j + e] * xe;
                        sb[r] += a.B[row * a.ldb + j + e] * xe;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const float ta = pk_wave_sum(sa[r]);
        const float tb = pk_wave_sum(sb[r]);
        if (lane == 0 && row0 + r < a.N)
            a.y[row0 + r] = a.alpha * ta + a.beta * tb;
    }
}

extern "C" __global__ void __launch_bounds__(NT) pk_gesummv(pk_gesummv_args a) {
    if (blockDim.x != NT)
        return;
    if (VEC > 1 && a.aligned)
        gesummv_body<VEC>(a);
    else
        gesummv_body<1>(a);
}

// y[j] += sum_r P[r][j]: 16 columns x 16 sub-lanes per block, sub-lane u adds
// rows u, u+16, ... in ascending order, the 16 partials are added in a fixed
// order, then added to y.  Blocks [0, ceil(n1/16)) handle (P1, y1), the rest
// (P2, y2).
extern "C" __global__ void __launch_bounds__(256) pk_colsum_accumulate(pk_reduce_args a) {
    const int cl = threadIdx.x % 16;
    const int u = threadIdx.x / 16;
    const int64_t b1 = (a.n1 + 15) / 16;
    const float *P;
    float *y;
    int64_t n, j;
    int rows;
    if ((int64_t)blockIdx.x < b1) {
        P = a.P1; y = a.y1; n = a.n1; rows = a.rows1;
        j = (int64_t)blockIdx.x * 16 + cl;
    } else {
        P = a.P2; y = a.y2; n = a.n2; rows = a.rows2;
        j = ((int64_t)blockIdx.x - b1) * 16 + cl;
    }
    __shared__ float sh[16][16];
    float s = 0.f;
    if (y != nullptr && j < n) {
#pragma unroll 4
        for (int r = u; r < rows; r += 16)
            s += P[(int64_t)r * n + j];
    }
    sh[u][cl] = s;
    __syncthreads();
    if (u == 0 && y != nullptr && j < n) {
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            t += sh[q][cl];
        y[j] += t;
    }
}
