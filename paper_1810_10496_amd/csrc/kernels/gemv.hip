// gemv.hip -- matrix-vector pair kernels (ATAX / BICG / MVT family, Sec. 2.2).
//
//   GEMV_KIND 0: y1 = A x                  (pk_gemv; one wavefront per ROWS rows)
//   GEMV_KIND 1: y2 = A^T z                (pk_gemvt_partial + pk_colsum_reduce)
//   GEMV_KIND 2: y1 = A x and y2 = A^T z   (pk_gemv_pair_partial + pk_colsum_reduce),
//                one pass over A
//
// All three are bound by reading A once from HBM.  Rows are streamed with
// VEC-wide loads, every sum stays in registers until one store (the paper's
// main finding for these kernels, Sec. 3.4), and the column sums of A^T z use
// per-block partials reduced in a fixed order, so results are bitwise
// reproducible (no floating-point atomics).
#include "pk_device.h"

#ifndef GEMV_KIND
#define GEMV_KIND 0
#endif
#ifndef VEC
#define VEC 4
#endif
#ifndef WAVES
#define WAVES 4
#endif
#ifndef UNROLL        // kind 0: column loop; kind 1: row loop (the pair unrolls fully)
#define UNROLL 4
#endif
#ifndef ROWS          // kind 0: rows per wavefront; kinds 1/2: rows per block
#define ROWS ((GEMV_KIND) == 0 ? 1 : 64)
#endif
#ifndef USE_LDS       // kind 0: stage x in LDS; kinds 1/2: reduce waves through LDS (always)
#define USE_LDS 0
#endif
#ifndef ORDER         // kinds 1/2: 0 = column strips fastest, 1 = row blocks fastest
#define ORDER 0
#endif
#ifndef FUSE          // kinds 1/2: 1 = one launch (the partials are folded by the last
#define FUSE 0        // block of each strip / row block), 0 = partials + pk_colsum_reduce
#endif
#ifndef NTL           // 1: the streamed matrix is read with the non-temporal hint
#define NTL 0
#endif
#if NTL
#define PK_LDM pk_ldv_nt
#else
#define PK_LDM pk_ldv
#endif

constexpr int NT = 64 * WAVES;
constexpr int XMAX = 4096;   // x staged in LDS when N <= XMAX

#if GEMV_KIND == 0
#define FAMILY PKF_GEMV
#elif GEMV_KIND == 1
#define FAMILY PKF_GEMV_T
#else
#define FAMILY PKF_GEMV_PAIR
#endif

// wavefronts per block of the partial-sum reduce (kinds 1/2, pk_colsum_reduce)
constexpr int RW = 8;

#if FUSE && GEMV_KIND == 0
#error "FUSE applies to the transposed matvec and the pair only"
#endif

// TM: rows per wavefront (kind 0) or per block (kinds 1/2); TN: columns per
// block (kinds 1/2; one wavefront wide in the one-launch form, whose wavefronts
// share the block's columns); X1: columns per wavefront (rows of the pair's part1
// = N / X1); X2: the reduce's wavefronts per block (kinds 1/2), which the runtime
// launches with; X3: FUSE
PK_DEFINE_KNOBS(FAMILY, ROWS, (GEMV_KIND) == 0 ? 64 * VEC : (FUSE ? 64 * VEC : WAVES * 64 * VEC), 0, WAVES, 1,
                VEC, UNROLL, USE_LDS, ORDER, 64 * VEC, (GEMV_KIND) == 0 ? 0 : RW, NT, 0, PK_KERNEL_ABI_VERSION,
                FUSE)

#if GEMV_KIND == 0
// ---------------------------------------------------------------- y = A x --
template <int V>
__device__ __forceinline__ void gemv_body(const pk_gemv_args &a, float *xs) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t row0 = ((int64_t)blockIdx.x * WAVES + wave) * ROWS;
#if USE_LDS
    const bool staged = a.N <= XMAX;
    if (staged) {
        for (int64_t j = threadIdx.x; j < a.N; j += NT)
            xs[j] = a.x[j];
        __syncthreads();
    }
    const float *xp = staged ? (const float *)xs : a.x;
#else
    const float *xp = a.x;
#endif
    if (row0 >= a.M)
        return;
    float acc[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
        acc[r] = 0.f;
#pragma unroll UNROLL
    for (int64_t j0 = 0; j0 < a.N; j0 += 64 * V) {
        const int64_t j = j0 + lane * V;
        float xv[V];
        if (j + V <= a.N) {
            pk_ldv<V>(xp + j, xv);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t row = min(row0 + r, a.M - 1);
                float av[V];
                PK_LDM<V>(a.A + row * a.lda + j, av);
#pragma unroll
                for (int e = 0; e < V; ++e)
                    acc[r] += av[e] * xv[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                if (j + e < a.N) {
                    const float xe = xp[j + e];
#pragma unroll
                    for (int r = 0; r < ROWS; ++r) {
                        const int64_t row = min(row0 + r, a.M - 1);
                        acc[r] += a.A[row * a.lda + j + e] * xe;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const float s = pk_wave_sum(acc[r]);
        if (lane == 0 && row0 + r < a.M)
            a.y[row0 + r] = s;
    }
}

extern "C" __global__ void __launch_bounds__(NT) pk_gemv(pk_gemv_args a) {
    if (blockDim.x != NT)
        return;
#if USE_LDS
    __shared__ __attribute__((aligned(16))) float xs[XMAX];
#else
    float *xs = nullptr;
#endif
    if (VEC > 1 && a.aligned)
        gemv_body<VEC>(a, xs);
    else
        gemv_body<1>(a, xs);
}

#else
// ------------------------------------------------- y2 = A^T z (and y1 = A x) --
// A block is WAVES wavefronts side by side; wavefront w owns the strip of
// 64*VEC columns [(blk*WAVES + w)*64*VEC, ...) and walks the block's ROWS rows,
// so each row segment a block reads is WAVES*64*VEC*4 contiguous bytes and no
// cross-wavefront reduction is needed.  part2[rb][col] receives the strip's
// column sums of the row block; for the pair, part1[wstrip][row] receives the
// strip's contribution to each row's dot product with x.
constexpr int WSTRIP = 64 * VEC;          // columns per wavefront
constexpr int STRIP = WAVES * WSTRIP;     // columns per block
// rows are read in chunks of RC = UNROLL rows (loads of a chunk are in flight
// together); for the pair each chunk's per-row dot products are reduced at once
constexpr int RC = UNROLL;
static_assert(RC >= 1 && RC <= 64 && (RC & (RC - 1)) == 0, "UNROLL must be a power of two <= 64");
static_assert(ROWS % RC == 0, "ROWS must be a multiple of UNROLL");
#if GEMV_KIND == 2
constexpr int LOGR = __builtin_ctz(RC);

// Sum each of the RC values v[q] over the 64 lanes.  Each halving step
// trades half of the remaining values with the partner lane (CNT values left,
// exchange distance OFF), so lane l ends up holding the total of row
// (l >> (6 - LOGR)); lanes whose low 6-LOGR bits are zero report it.
template <int CNT, int OFF>
__device__ __forceinline__ void rows_reduce_step(float *v, int lane) {
    if constexpr (OFF >= 1) {
        if constexpr (CNT > 1) {
            constexpr int H = CNT / 2;
            const bool upper = (lane & OFF) != 0;
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const float send = upper ? v[i] : v[i + H];
                const float keep = upper ? v[i + H] : v[i];
                v[i] = keep + __shfl_xor(send, OFF, 64);
            }
            rows_reduce_step<H, OFF / 2>(v, lane);
        } else {
            v[0] += __shfl_xor(v[0], OFF, 64);
            rows_reduce_step<1, OFF / 2>(v, lane);
        }
    }
}

__device__ __forceinline__ float rows_reduce(float *v, int lane) {
    rows_reduce_step<RC, 32>(v, lane);
    return v[0];
}
#endif

template <int V>
__device__ __forceinline__ void colblock_body(const pk_gemvt_args &a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int strips = (int)((a.N + STRIP - 1) / STRIP);
    int strip, rb;
    if (ORDER == 0) {
        strip = blockIdx.x % strips;
        rb = blockIdx.x / strips;
    } else {
        rb = blockIdx.x % a.row_blocks;
        strip = blockIdx.x / a.row_blocks;
    }
    if (rb >= a.row_blocks || strip >= strips)
        return;
    const int64_t wstrip = (int64_t)strip * WAVES + wave;
    const int64_t c0 = wstrip * WSTRIP + lane * VEC;     // this lane's VEC columns
    if (wstrip * WSTRIP >= a.N)
        return;                                          // no barrier below: wavefronts may leave
    const int64_t r0 = (int64_t)rb * ROWS;
    const int64_t rend = min(r0 + (int64_t)ROWS, a.M);
    const bool full = c0 + VEC <= a.N;

    float acc2[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        acc2[e] = 0.f;
#if GEMV_KIND == 2
    float xv[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        xv[e] = (c0 + e < a.N) ? a.x[c0 + e] : 0.f;
#endif
    for (int q0 = 0; q0 < ROWS; q0 += RC) {
        if (r0 + q0 >= rend)
            break;
#if GEMV_KIND == 2
        float rs[RC];
#endif
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            const int64_t i = r0 + q0 + q;
            float av[VEC];
            float zi = 0.f;
            if (i < rend) {
                zi = a.z[i];
                if (full) {
#pragma unroll
                    for (int e = 0; e < VEC; e += V)
                        PK_LDM<V>(a.A + i * a.lda + c0 + e, av + e);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        av[e] = (c0 + e < a.N) ? a.A[i * a.lda + c0 + e] : 0.f;
                }
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    av[e] = 0.f;
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                acc2[e] += av[e] * zi;
#if GEMV_KIND == 2
            float t = 0.f;
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                t += av[e] * xv[e];
            rs[q] = t;
#endif
        }
#if GEMV_KIND == 2
        const float s = rows_reduce(rs, lane);
        const int64_t i = r0 + q0 + (lane >> (6 - LOGR));
        if ((lane & ((1 << (6 - LOGR)) - 1)) == 0 && i < rend)
            a.part1[wstrip * a.M + i] = s;
#endif
    }
    float *p2 = a.part2 + (int64_t)rb * a.N;
    if (full) {
#pragma unroll
        for (int e = 0; e < VEC; e += V)
            pk_stv<V>(p2 + c0 + e, acc2 + e);
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (c0 + e < a.N)
                p2[c0 + e] = acc2[e];
    }
}

#if FUSE
// ------------------------------------------------------------ one launch --
// The block is WAVES wavefronts stacked over ROWS rows of one strip of SW = 64*VEC
// columns: wavefront w takes the block's rows w, w+WAVES, ... (RC of them in flight).
// The wavefronts' column sums are added through LDS in the order w = 0..WAVES-1 and
// stored as the block's row of part2; for the pair, each row's dot product over the
// strip goes to part1[strip][row].  Then the block takes a ticket for its strip: the
// last of the strip's row blocks adds the strip's part2 rows into y2 (wavefront w the
// rows k = w, w+WAVES, ... in ascending order, then the WAVES sums in order w = 0..).
// For the pair it also takes a ticket for its row block: the last of the row block's
// strips adds part1's strips into y1 the same way.  Bit 1 of `aligned` adds the
// results to y1 / y2 instead of storing them.
constexpr int SW = 64 * VEC;
constexpr int RPW = ROWS / WAVES;     // rows per wavefront
constexpr int FB = 16;                // partial loads in flight per thread in a fold
static_assert(ROWS % WAVES == 0 && RPW % RC == 0, "one launch: ROWS / WAVES must be a multiple of UNROLL");
#if GEMV_KIND == 2
constexpr int RT = NT < ROWS ? NT : ROWS;   // y1 fold: threads along the rows
constexpr int G = NT / RT;                  // y1 fold: groups of strips
#endif

template <int V>
__device__ __forceinline__ void fused_body(const pk_gemvt_args &a) {
    __shared__ __attribute__((aligned(16))) float red[WAVES][SW];
#if GEMV_KIND == 2
    __shared__ float red1[G][ROWS];
#endif
    __shared__ int flag;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int strips = (int)((a.N + SW - 1) / SW);
    int strip, rb;
    if (ORDER == 0) {
        strip = blockIdx.x % strips;
        rb = blockIdx.x / strips;
    } else {
        rb = blockIdx.x % a.row_blocks;
        strip = blockIdx.x / a.row_blocks;
    }
    if (rb >= a.row_blocks || strip >= strips)
        return;                                          // never taken: the grid is exact
    const bool accumulate = (a.aligned & 2) != 0;
    const int64_t ldp = pk_part_ld(a.N);
    const int64_t c0 = (int64_t)strip * SW + lane * VEC;
    const bool full = c0 + VEC <= a.N;
    const int64_t r0 = (int64_t)rb * ROWS;
    const int64_t rend = min(r0 + (int64_t)ROWS, a.M);

    float acc2[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        acc2[e] = 0.f;
#if GEMV_KIND == 2
    float xv[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        xv[e] = (c0 + e < a.N) ? a.x[c0 + e] : 0.f;
#endif
    for (int q0 = 0; q0 < RPW; q0 += RC) {
        if (r0 + wave + (int64_t)q0 * WAVES >= rend)
            break;                                       // wavefront-uniform
#if GEMV_KIND == 2
        float rs[RC];
#endif
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            const int64_t i = r0 + wave + (int64_t)(q0 + q) * WAVES;
            float av[VEC];
            float zi = 0.f;
            if (i < rend) {
                zi = a.z[i];
                if (full) {
#pragma unroll
                    for (int e = 0; e < VEC; e += V)
                        PK_LDM<V>(a.A + i * a.lda + c0 + e, av + e);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        av[e] = (c0 + e < a.N) ? a.A[i * a.lda + c0 + e] : 0.f;
                }
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    av[e] = 0.f;
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                acc2[e] += av[e] * zi;
#if GEMV_KIND == 2
            float t = 0.f;
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                t += av[e] * xv[e];
            rs[q] = t;
#endif
        }
#if GEMV_KIND == 2
        const float s = rows_reduce(rs, lane);
        const int64_t i = r0 + wave + (int64_t)(q0 + (lane >> (6 - LOGR))) * WAVES;
        if ((lane & ((1 << (6 - LOGR)) - 1)) == 0 && i < rend) {
            if (strips == 1)                              // one strip: the dot product is y1's
                a.y1[i] = accumulate ? a.y1[i] + s : s;
            else
                pk_part_store(a.part1 + (int64_t)strip * a.M + i, s);
        }
#endif
    }

    // the block's column sums: wavefronts added in order, one row of part2 (with one
    // row block they are y2 itself, and no group needs a ticket)
    const bool single = a.row_blocks == 1;
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        red[wave][lane * VEC + e] = acc2[e];
    __syncthreads();
    for (int col = threadIdx.x; col < SW; col += NT) {
        float t = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w)
            t += red[w][col];
        const int64_t j = (int64_t)strip * SW + col;
        if (j < a.N) {
            if (single)
                a.y2[j] = accumulate ? a.y2[j] + t : t;
            else
                pk_part_store(a.part2 + (int64_t)rb * ldp + j, t);
        }
    }
    unsigned long long *cells = reinterpret_cast<unsigned long long *>(a.part2 + (int64_t)a.row_blocks * ldp);

    if (!single && pk_ticket_last(cells, strip, (uint32_t)rb, a.tag, (uint32_t)a.row_blocks, &flag)) {
        const bool pal = (reinterpret_cast<uintptr_t>(a.part2) & 15) == 0;
        float t[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            t[e] = 0.f;
        for (int k0 = wave; k0 < a.row_blocks; k0 += FB * WAVES) {
            float v[FB][VEC];
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                const int k = k0 + f * WAVES;
                const float *p = a.part2 + (int64_t)min(k, a.row_blocks - 1) * ldp;
                if (full && pal) {
                    pk_part_loadv<VEC>(p + c0, v[f]);    // rows start 256 bytes apart
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        v[f][e] = (c0 + e < a.N) ? pk_part_load(p + c0 + e) : 0.f;
                }
            }
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                if (k0 + f * WAVES < a.row_blocks) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        t[e] += v[f][e];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            red[wave][lane * VEC + e] = t[e];
        __syncthreads();
        for (int col = threadIdx.x; col < SW; col += NT) {
            float u = 0.f;
#pragma unroll
            for (int w = 0; w < WAVES; ++w)
                u += red[w][col];
            const int64_t j = (int64_t)strip * SW + col;
            if (j < a.N)
                a.y2[j] = accumulate ? a.y2[j] + u : u;
        }
    }
#if GEMV_KIND == 2
    if (strips > 1 && pk_ticket_last(cells, strips + rb, (uint32_t)strip, a.tag, (uint32_t)strips, &flag)) {
        const int rt = threadIdx.x % RT;
        const int g = threadIdx.x / RT;
        for (int j = rt; j < ROWS; j += RT) {
            const int64_t i = r0 + j;
            float u = 0.f;
            if (i < rend) {
                for (int s0 = g; s0 < strips; s0 += FB * G) {
                    float v[FB];
#pragma unroll
                    for (int f = 0; f < FB; ++f)
                        v[f] = pk_part_load(a.part1 + (int64_t)min(s0 + f * G, strips - 1) * a.M + i);
#pragma unroll
                    for (int f = 0; f < FB; ++f)
                        if (s0 + f * G < strips)
                            u += v[f];
                }
            }
            red1[g][j] = u;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < ROWS; j += NT) {
            const int64_t i = r0 + j;
            if (i < rend) {
                float u = 0.f;
#pragma unroll
                for (int q = 0; q < G; ++q)
                    u += red1[q][j];
                a.y1[i] = accumulate ? a.y1[i] + u : u;
            }
        }
    }
#endif
}
#endif

#if GEMV_KIND == 1
extern "C" __global__ void __launch_bounds__(NT) pk_gemvt_partial(pk_gemvt_args a) {
#else
extern "C" __global__ void __launch_bounds__(NT) pk_gemv_pair_partial(pk_gemvt_args a) {
#endif
    if (blockDim.x != NT)
        return;
#if FUSE
    if (VEC > 1 && (a.aligned & 1))
        fused_body<VEC>(a);
    else
        fused_body<1>(a);
#else
    if (VEC > 1 && a.aligned)
        colblock_body<VEC>(a);
    else
        colblock_body<1>(a);
#endif
}

// y[j] = sum_r P[r][j].  A block is RW wavefronts over 64 columns (lane = column):
// wavefront w adds the rows r = w, w+RW, ... in ascending order, issuing a batch of
// RB rows' loads before the first add of the batch (the partials were just written
// and sit in the L2 or the Infinity Cache, so what costs is the wait, not the
// bytes), and the RW wavefront sums of a column are added in the order w = 0..RW-1:
// the result does not depend on timing.  Blocks [0, ceil(n1/64)) handle P1, the
// rest P2 (when present).
constexpr int RB = 16;
extern "C" __global__ void __launch_bounds__(64 * RW) pk_colsum_reduce(pk_reduce_args a) {
    if (blockDim.x != 64 * RW)
        return;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t b1 = (a.n1 + 63) / 64;
    const float *P;
    float *y;
    int64_t n, j;
    int rows;
    if ((int64_t)blockIdx.x < b1) {
        P = a.P1; y = a.y1; n = a.n1; rows = a.rows1;
        j = (int64_t)blockIdx.x * 64 + lane;
    } else {
        P = a.P2; y = a.y2; n = a.n2; rows = a.rows2;
        j = ((int64_t)blockIdx.x - b1) * 64 + lane;
    }
    __shared__ float sh[RW][64];
    float s = 0.f;
    if (y != nullptr && j < n) {
        for (int r0 = w; r0 < rows; r0 += RB * RW) {      // rows == 0 leaves zeros (empty sums)
            float v[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int r = r0 + q * RW;
                v[q] = r < rows ? P[(int64_t)r * n + j] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < RB; ++q)
                s += v[q];
        }
    }
    sh[w][lane] = s;
    __syncthreads();
    if (w == 0 && y != nullptr && j < n) {
        float t = sh[0][lane];
#pragma unroll
        for (int q = 1; q < RW; ++q)
            t += sh[q][lane];
        y[j] = t;
    }
}
#endif
