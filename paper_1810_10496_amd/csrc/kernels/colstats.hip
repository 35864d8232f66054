// colstats.hip -- column mean and standard deviation (CORR's mean and
// deviation kernels, Sec. 3.4), in FP32 with compensated summation.
//
//   mu_j    = (1/n) sum_i x_ij
//   sigma_j = sqrt( (1/(n-1)) sum_i (x_ij - mu_j)^2 ),  then max(sigma_j, eps)
//
// Stage 1 (pk_colstats_partial): a block owns a segment of seg_rows rows and a
// strip of 64*VEC columns.  Each thread keeps its rows' values in registers,
// so the segment is read from memory once: a Neumaier-compensated sum gives
// the segment mean, then the squared deviations about that mean are summed
// from the same registers.  Per segment it writes (sum_hi, sum_lo, M2).
// Stage 2 (pk_colstats_merge): per column, segments are folded in a fixed
// order: the total sum by Neumaier summation of every (hi, lo) term, the mean
// from it, and M2 = sum_b [M2_b + n_b (mu_b - mu)^2] (all terms >= 0, so the
// large column offsets never cancel).
#include "pk_device.h"

#ifndef VEC
#define VEC 4
#endif
#ifndef WAVES
#define WAVES 4
#endif
#ifndef ROWS        // rows per segment (block)
#define ROWS 64
#endif
#ifndef ORDER       // 0: column strips fastest, 1: segments fastest
#define ORDER 0
#endif
#ifndef FUSE        // 1: one launch (the last segment of each strip merges), 0: + pk_colstats_merge
#define FUSE 0
#endif
#ifndef MG          // the two-launch merge: 0 = two passes about the total mean, 1 = one pass
#define MG 0        // (pairwise count / mean / M2 combination), loading only existing segments
#endif
#ifndef NTL           // 1: the data matrix is read with the non-temporal hint
#define NTL 0
#endif
#if NTL
#define PK_LDM pk_ldv_nt
#else
#define PK_LDM pk_ldv
#endif

constexpr int NT = 64 * WAVES;
constexpr int RPW = (ROWS + WAVES - 1) / WAVES;
constexpr int STRIP = 64 * VEC;

// wavefronts per block of the merge (pk_colstats_merge); recorded in knob X2, which
// the runtime launches it with
constexpr int MW = 8;

PK_DEFINE_KNOBS(PKF_COLSTATS, ROWS, STRIP, ROWS, WAVES, 1, VEC, 1, 1, ORDER, 0, MW, NT,
                3 * WAVES * STRIP * 4, PK_KERNEL_ABI_VERSION, FUSE)

#if FUSE
// partial loads in flight per thread in the one-launch merge
constexpr int FB = 8;
__device__ __forceinline__ void fused_merge(const pk_colstats_args &a, int strip, int seg,
                                            float (*red)[WAVES][STRIP], float *smean);
#endif

template <int V>
__device__ __forceinline__ void partial_body(const pk_colstats_args &a, float (*red)[WAVES][STRIP],
                                             float *smean) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int strips = (int)((a.m + STRIP - 1) / STRIP);
    int strip, seg;
    if (ORDER == 0) {
        strip = blockIdx.x % strips;
        seg = blockIdx.x / strips;
    } else {
        seg = blockIdx.x % a.segments;
        strip = blockIdx.x / a.segments;
    }
    if (seg >= a.segments)
        return;
    const int64_t r0 = (int64_t)seg * a.seg_rows;
    const int64_t rend = min(r0 + (int64_t)a.seg_rows, a.n);
    const int64_t c0 = (int64_t)strip * STRIP + lane * VEC;
    const bool full = c0 + VEC <= a.m;

    float v[RPW][VEC];
    float s[VEC], c[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        s[e] = 0.f;
        c[e] = 0.f;
    }
    // every row's loads are issued before the first sum needs one (summing in
    // the same loop made each row wait for its own load)
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int64_t i = r0 + wave + (int64_t)q * WAVES;
        if (i < rend) {
            if (full) {
#pragma unroll
                for (int e = 0; e < VEC; e += V)
                    PK_LDM<V>(a.X + i * a.ldx + c0 + e, v[q] + e);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    v[q][e] = (c0 + e < a.m) ? a.X[i * a.ldx + c0 + e] : 0.f;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int64_t i = r0 + wave + (int64_t)q * WAVES;
        if (i < rend) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                pk_neumaier(s[e], c[e], v[q][e]);
        }
    }

    // combine the wavefronts' compensated sums in a fixed order
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        red[0][wave][lane * VEC + e] = s[e];
        red[1][wave][lane * VEC + e] = c[e];
    }
    __syncthreads();
    const float nb = (float)(rend - r0);
    for (int col = threadIdx.x; col < STRIP; col += NT) {
        float hi = 0.f, lo = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            pk_neumaier(hi, lo, red[0][w][col]);
            lo += red[1][w][col];
        }
        // renormalise (hi, lo) so hi carries the rounded total
        const float t = hi + lo;
        lo = lo - (t - hi);
        hi = t;
        red[0][0][col] = hi;
        red[1][0][col] = lo;
        smean[col] = (hi + lo) / nb;
    }
    __syncthreads();

    float q2[VEC], qc[VEC], mu[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        q2[e] = 0.f;
        qc[e] = 0.f;
        mu[e] = smean[lane * VEC + e];
    }
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int64_t i = r0 + wave + (int64_t)q * WAVES;
        if (i < rend) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const float d = v[q][e] - mu[e];
                pk_neumaier(q2[e], qc[e], d * d);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        red[2][wave][lane * VEC + e] = q2[e] + qc[e];
    __syncthreads();
#if FUSE
    const int64_t ldp = pk_part_ld(a.m);       // one-launch layout: rows 256 bytes apart
#else
    const int64_t ldp = a.m;
#endif
    for (int col = threadIdx.x; col < STRIP; col += NT) {
        float m2 = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w)
            m2 += red[2][w][col];
        const int64_t j = (int64_t)strip * STRIP + col;
        if (j < a.m) {
            float *p = a.part + (int64_t)seg * 3 * ldp;
#if FUSE
            if (a.segments == 1) {        // one segment: its statistics are the column's
                a.mean[j] = smean[col];
                a.std[j] = fmaxf(sqrtf(m2 / (float)(a.n - 1)), a.eps);
                continue;
            }
            pk_part_store(p + j, red[0][0][col]);
            pk_part_store(p + ldp + j, red[1][0][col]);
            pk_part_store(p + 2 * ldp + j, m2);
#else
            p[j] = red[0][0][col];
            p[ldp + j] = red[1][0][col];
            p[2 * ldp + j] = m2;
#endif
        }
    }
#if FUSE
    if (a.segments > 1)
        fused_merge(a, strip, seg, red, smean);
#endif
}

#if FUSE
// The one-launch merge: the last segment of a strip to finish (its ticket) merges
// the strip's segments the way pk_colstats_merge does, wavefront w taking the
// segments b = w, w+WAVES, ... in ascending order and the WAVES results combined in
// the order w = 0..WAVES-1: first the compensated total of every (hi, lo) term and
// the mean from it, then M2 = sum_b [M2_b + n_b (mu_b - mu)^2].  The result does not
// depend on which segment finishes last.
// (hi, lo, M2) of segment b for this lane's VEC columns (vector loads when `full`)
__device__ __forceinline__ void merge_load(const pk_colstats_args &a, int64_t ldp, int64_t c0, bool full, int b,
                                           float (&h)[VEC], float (&l)[VEC], float (&q)[VEC]) {
    const float *p = a.part + (int64_t)min(b, a.segments - 1) * 3 * ldp;
    if (full) {
        pk_part_loadv<VEC>(p + c0, h);
        pk_part_loadv<VEC>(p + ldp + c0, l);
        pk_part_loadv<VEC>(p + 2 * ldp + c0, q);
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const bool ok = c0 + e < a.m;
            h[e] = ok ? pk_part_load(p + c0 + e) : 0.f;
            l[e] = ok ? pk_part_load(p + ldp + c0 + e) : 0.f;
            q[e] = ok ? pk_part_load(p + 2 * ldp + c0 + e) : 0.f;
        }
    }
}

__device__ __forceinline__ void fused_merge(const pk_colstats_args &a, int strip, int seg,
                                            float (*red)[WAVES][STRIP], float *smean) {
    __shared__ int flag;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t ldp = pk_part_ld(a.m);
    const uint32_t tag = (uint32_t)a.aligned >> 1;
    unsigned long long *cells =
        reinterpret_cast<unsigned long long *>(a.part + (int64_t)a.segments * 3 * ldp);
    if (!pk_ticket_last(cells, strip, (uint32_t)seg, tag, (uint32_t)a.segments, &flag))
        return;
    const int64_t c0 = (int64_t)strip * STRIP + lane * VEC;
    const bool full = c0 + VEC <= a.m && (reinterpret_cast<uintptr_t>(a.part) & 15) == 0;
    float hi[VEC], lo[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        hi[e] = 0.f;
        lo[e] = 0.f;
    }
    float hv[FB][VEC], lv[FB][VEC], mv[FB][VEC];
    const bool one_batch = a.segments <= FB * WAVES;
    for (int b0 = wave; b0 < a.segments; b0 += FB * WAVES) {
#pragma unroll
        for (int f = 0; f < FB; ++f)
            merge_load(a, ldp, c0, full, b0 + f * WAVES, hv[f], lv[f], mv[f]);
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            if (b0 + f * WAVES < a.segments) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    pk_neumaier(hi[e], lo[e], hv[f][e]);
                    pk_neumaier(hi[e], lo[e], lv[f][e]);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        red[0][wave][lane * VEC + e] = hi[e];
        red[1][wave][lane * VEC + e] = lo[e];
    }
    __syncthreads();
    for (int col = threadIdx.x; col < STRIP; col += NT) {
        float th = 0.f, tl = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            pk_neumaier(th, tl, red[0][w][col]);
            pk_neumaier(th, tl, red[1][w][col]);
        }
        smean[col] = (th + tl) / (float)a.n;
    }
    __syncthreads();
    float mu[VEC], m2[VEC], m2c[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        mu[e] = smean[lane * VEC + e];
        m2[e] = 0.f;
        m2c[e] = 0.f;
    }
    for (int b0 = wave; b0 < a.segments; b0 += FB * WAVES) {
        if (!one_batch) {
#pragma unroll
            for (int f = 0; f < FB; ++f)
                merge_load(a, ldp, c0, full, b0 + f * WAVES, hv[f], lv[f], mv[f]);
        }
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            const int b = b0 + f * WAVES;
            if (b < a.segments) {
                const int64_t r0 = (int64_t)b * a.seg_rows;
                const float nb = (float)(min(r0 + (int64_t)a.seg_rows, a.n) - r0);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const float d = (hv[f][e] + lv[f][e]) / nb - mu[e];
                    pk_neumaier(m2[e], m2c[e], mv[f][e]);
                    pk_neumaier(m2[e], m2c[e], nb * d * d);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        red[0][wave][lane * VEC + e] = m2[e];
        red[1][wave][lane * VEC + e] = m2c[e];
    }
    __syncthreads();
    for (int col = threadIdx.x; col < STRIP; col += NT) {
        const int64_t j = (int64_t)strip * STRIP + col;
        if (j < a.m) {
            float M = 0.f, Mc = 0.f;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                pk_neumaier(M, Mc, red[0][w][col]);
                pk_neumaier(M, Mc, red[1][w][col]);
            }
            a.mean[j] = smean[col];
            a.std[j] = fmaxf(sqrtf((M + Mc) / (float)(a.n - 1)), a.eps);
        }
    }
}
#endif

extern "C" __global__ void __launch_bounds__(NT) pk_colstats_partial(pk_colstats_args a) {
    if (blockDim.x != NT)
        return;
    __shared__ float red[3][WAVES][STRIP];
    __shared__ float smean[STRIP];
#if FUSE
    const bool aligned = (a.aligned & 1) != 0;     // the upper bits carry the ticket tag
#else
    const bool aligned = a.aligned != 0;
#endif
    if (VEC > 1 && aligned)
        partial_body<VEC>(a, red, smean);
    else
        partial_body<1>(a, red, smean);
}

#if MG
// The merge in one pass: a block is MW wavefronts over 64 columns (lane = column).
// Wavefront w folds the segments b = w, w+MW, ... in ascending order, loading only those
// that exist (the bound is the same for the whole wavefront), MQ1 at a time, into
//  - a compensated total: the (hi, lo) terms by Neumaier summation, from which the mean
//    is taken, and
//  - the pairwise combination of (count, mean, M2) (Chan, Golub and LeVeque): a
//    segment's mean is its compensated sum over its rows, and merging (n_a, mu_a, M2_a)
//    with (n_b, mu_b, M2_b) gives M2_a + M2_b + d^2 n_a n_b / (n_a + n_b), d = mu_b - mu_a
//    (every term >= 0, so the large column offsets never cancel).
// After one barrier the MW partial results of a column are combined in the order
// w = 0..MW-1, so the result does not depend on timing.
constexpr int MQ1 = 8;

__device__ __forceinline__ void chan_merge(float &cnt, float &mu, float &m2, float nb, float mb, float m2b) {
    if (nb > 0.f) {
        if (cnt == 0.f) {
            cnt = nb;
            mu = mb;
            m2 = m2b;
        } else {
            const float t = cnt + nb;
            const float rt = 1.0f / t;
            const float d = mb - mu;
            mu += d * nb * rt;
            m2 += m2b + d * d * (cnt * nb * rt);
            cnt = t;
        }
    }
}

extern "C" __global__ void __launch_bounds__(64 * MW) pk_colstats_merge(pk_colstats_args a) {
    if (blockDim.x != 64 * MW)
        return;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    __shared__ float sh[5][MW][64];
    for (int64_t c0 = (int64_t)blockIdx.x * 64; c0 < a.m; c0 += (int64_t)gridDim.x * 64) {
        const int64_t j = c0 + lane;
        const bool valid = j < a.m;
        const int64_t jr = valid ? j : a.m - 1;          // lanes past m read column m-1
        float hi = 0.f, lo = 0.f, cnt = 0.f, mu = 0.f, m2 = 0.f;
        for (int b0 = w; b0 < a.segments; b0 += MQ1 * MW) {
            float hv[MQ1], lv[MQ1], mv[MQ1];
#pragma unroll
            for (int q = 0; q < MQ1; ++q) {
                const int b = b0 + q * MW;
                if (b < a.segments) {
                    const float *p = a.part + (int64_t)b * 3 * a.m;
                    hv[q] = p[jr];
                    lv[q] = p[a.m + jr];
                    mv[q] = p[2 * a.m + jr];
                }
            }
#pragma unroll
            for (int q = 0; q < MQ1; ++q) {
                const int b = b0 + q * MW;
                if (b < a.segments) {
                    pk_neumaier(hi, lo, hv[q]);
                    pk_neumaier(hi, lo, lv[q]);
                    const int64_t r0 = (int64_t)b * a.seg_rows;
                    const float nb = (float)(min(r0 + (int64_t)a.seg_rows, a.n) - r0);
                    chan_merge(cnt, mu, m2, nb, (hv[q] + lv[q]) / nb, mv[q]);
                }
            }
        }
        sh[0][w][lane] = hi;
        sh[1][w][lane] = lo;
        sh[2][w][lane] = cnt;
        sh[3][w][lane] = mu;
        sh[4][w][lane] = m2;
        __syncthreads();
        if (w == 0 && valid) {
            float th = 0.f, tl = 0.f, tc = 0.f, tm = 0.f, t2 = 0.f;
#pragma unroll
            for (int q = 0; q < MW; ++q) {
                pk_neumaier(th, tl, sh[0][q][lane]);
                pk_neumaier(th, tl, sh[1][q][lane]);
                chan_merge(tc, tm, t2, sh[2][q][lane], sh[3][q][lane], sh[4][q][lane]);
            }
            a.mean[j] = (th + tl) / (float)a.n;
            a.std[j] = fmaxf(sqrtf(t2 / (float)(a.n - 1)), a.eps);
        }
        __syncthreads();
    }
}
#else
// The merge: a block is MW wavefronts over 64 columns (lane = column).  Wavefront w
// takes the segments b = w, w+MW, ... in ascending order; it loads the (hi, lo, M2)
// of up to MQ of them at once into registers and folds them from there, so both
// passes of a batch wait for memory once (and the second pass reads nothing when
// a wavefront has at most MQ segments).  The MW results of a column are combined
// in the order w = 0..MW-1, so the result does not depend on timing.
constexpr int MQ = 16;
extern "C" __global__ void __launch_bounds__(64 * MW) pk_colstats_merge(pk_colstats_args a) {
    if (blockDim.x != 64 * MW)
        return;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    __shared__ float sh[2][MW][64];
    __shared__ float smu[64];
    const bool one_batch = a.segments <= MW * MQ;
    for (int64_t c0 = (int64_t)blockIdx.x * 64; c0 < a.m; c0 += (int64_t)gridDim.x * 64) {
        const int64_t j = c0 + lane;
        const bool valid = j < a.m;
        float hv[MQ], lv[MQ], mv[MQ];
        float hi = 0.f, lo = 0.f;
        if (valid) {
            for (int b0 = w; b0 < a.segments; b0 += MQ * MW) {
#pragma unroll
                for (int q = 0; q < MQ; ++q) {
                    const int b = b0 + q * MW;
                    const float *p = a.part + (int64_t)min(b, a.segments - 1) * 3 * a.m;
                    hv[q] = p[j];
                    lv[q] = p[a.m + j];
                    mv[q] = p[2 * a.m + j];
                }
#pragma unroll
                for (int q = 0; q < MQ; ++q) {
                    if (b0 + q * MW < a.segments) {
                        pk_neumaier(hi, lo, hv[q]);
                        pk_neumaier(hi, lo, lv[q]);
                    }
                }
            }
        }
        sh[0][w][lane] = hi;
        sh[1][w][lane] = lo;
        __syncthreads();
        if (w == 0) {
            float th = 0.f, tl = 0.f;
#pragma unroll
            for (int q = 0; q < MW; ++q) {
                pk_neumaier(th, tl, sh[0][q][lane]);
                pk_neumaier(th, tl, sh[1][q][lane]);
            }
            smu[lane] = (th + tl) / (float)a.n;
        }
        __syncthreads();
        const float mu = smu[lane];
        float m2 = 0.f, m2c = 0.f;
        if (valid) {
            for (int b0 = w; b0 < a.segments; b0 += MQ * MW) {
                if (!one_batch) {
#pragma unroll
                    for (int q = 0; q < MQ; ++q) {
                        const int b = b0 + q * MW;
                        const float *p = a.part + (int64_t)min(b, a.segments - 1) * 3 * a.m;
                        hv[q] = p[j];
                        lv[q] = p[a.m + j];
                        mv[q] = p[2 * a.m + j];
                    }
                }
#pragma unroll
                for (int q = 0; q < MQ; ++q) {
                    const int b = b0 + q * MW;
                    if (b < a.segments) {
                        const int64_t r0 = (int64_t)b * a.seg_rows;
                        const float nb = (float)(min(r0 + (int64_t)a.seg_rows, a.n) - r0);
                        const float d = (hv[q] + lv[q]) / nb - mu;
                        pk_neumaier(m2, m2c, mv[q]);
                        pk_neumaier(m2, m2c, nb * d * d);
                    }
                }
            }
        }
        __syncthreads();
        sh[0][w][lane] = m2;
        sh[1][w][lane] = m2c;
        __syncthreads();
        if (w == 0 && valid) {
            float M = 0.f, Mc = 0.f;
#pragma unroll
            for (int q = 0; q < MW; ++q) {
                pk_neumaier(M, Mc, sh[0][q][lane]);
                pk_neumaier(M, Mc, sh[1][q][lane]);
            }
            const float sd = sqrtf((M + Mc) / (float)(a.n - 1));
            a.mean[j] = mu;
            a.std[j] = fmaxf(sd, a.eps);
        }
        __syncthreads();
    }
}
#endif
