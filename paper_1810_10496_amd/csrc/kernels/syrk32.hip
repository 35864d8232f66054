// syrk32.hip -- correlation rank-k update in FP32 (CORR, Sec. 2.2 / 3.4):
//
//   z_ij  = (x_ij - mu_j) / sigma_j
//   R_jk  = (1/(n-1)) sum_i z_ij z_ik
//
// X is n samples x m features, row-major.  Only lower-triangle T x T tiles of R
// are computed (grid = nt(nt+1)/2 blocks); each result is stored at (j, k) and
// (k, j), so R is bitwise symmetric.  The normalisation is fused into the tile
// loads, as (x - mu) * (1/sigma) with the reciprocal taken once per column.
//
// The contraction index is the sample, which is the slow index of X.  An FP32
// MFMA (v_mfma_f32_16x16x4_f32) takes one k value per lane per instruction, so
// the tiles can stay in X's own layout in LDS ([sample][feature]): the global
// loads are whole row segments (one 16-byte load per lane, a wavefront reading
// contiguous rows), the LDS writes are plain 16-byte stores, and a fragment is
// one 4-byte LDS read in which 16 lanes read 16 consecutive features of one
// sample.  With k slot g (lane group) of step s mapped to sample 4s + g, the
// four lane groups read four rows whose offsets differ by LDR = BT + 16 words
// (BT + 32 for tiles that are odd multiples of 16),
// which puts them on disjoint bank ranges.  Two LDS stages let the next tile
// be written while the current one is read (one barrier per step), and the
// global loads for the tile after next are in flight meanwhile.
#include "pk_device.h"

#ifndef BT           // square output tile
#define BT 64
#endif
#ifndef BK           // samples per step
#define BK 16
#endif
#ifndef WAVES_M
#define WAVES_M 2
#endif
#ifndef WAVES_N
#define WAVES_N 2
#endif
#ifndef VEC
#define VEC 4
#endif
#ifndef STAGES
#define STAGES 2
#endif
#ifndef ORDER        // 0: triangle rows in order, 2: XCD-aware groups of 8 tile rows
#define ORDER 0
#endif
#ifndef IL           // two stages: 1 = full tiles run a branch-free k loop whose LDS stores and
#define IL 0         // global loads are interleaved with the MFMAs (below); 2 = the same for any
#endif               // n (samples past n read the last one and are zeroed); 3 = as 1, with the
                     // column statistics kept in the second stage (less LDS per block)

constexpr int NT = 64 * WAVES_M * WAVES_N;
constexpr int WTM = BT / WAVES_M;
constexpr int WTN = BT / WAVES_N;
constexpr int FM = WTM / 16;
constexpr int FN = WTN / 16;
// LDS row stride (floats): the four lane groups of a fragment read rows
// g * LDR apart, which must start 16, 32, 48 banks apart (LDR = 16 or 48 mod 64)
constexpr int LDR = BT + ((BT % 32 == 0) ? 16 : 32);
constexpr int TILE = BK * LDR;                   // one operand tile
constexpr int LDS_FLOATS = STAGES * 2 * TILE;
static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be a multiple of 16");
static_assert(BK % 4 == 0, "BK must be a multiple of 4");
static_assert(BT % VEC == 0, "bad VEC");
static_assert(STAGES == 1 || STAGES == 2, "bad STAGES");
static_assert(IL == 0 || (STAGES == 2 && (BK * BT / 4) % NT == 0), "IL: two stages, whole chunks per thread");
// the general loop's stages: one when the statistics live in the second stage (IL 3)
constexpr int GST = IL == 3 ? 1 : STAGES;

// knob slot X2 records 1, + 1000 with IL
PK_DEFINE_KNOBS(PKF_SYRK_F32, BT, BT, BK, WAVES_M, WAVES_N, VEC, 1, STAGES, ORDER, 0, 1 + 1000 * IL, NT,
                LDS_FLOATS * 4 + (IL == 3 ? 0 : 4 * BT * 4), PK_KERNEL_ABI_VERSION, 0)

// block index -> lower-triangle tile (bj >= bk)
__device__ __forceinline__ void tri_tile(int b, int nt, int &bj, int &bk) {
    if (ORDER == 2) {
        // Blocks are dealt to the 8 XCDs in turn; each XCD gets a contiguous
        // range of logical tiles (a bijection on [0, nb)), and the logical order
        // walks groups of 8 tile rows column by column, so the blocks an XCD
        // runs together share their column strips of X in its L2.
        const int nb = nt * (nt + 1) / 2;
        const int q = nb / 8, rem = nb % 8, x = b % 8;
        int L = x * q + min(x, rem) + b / 8;
        constexpr int G = 8;
        for (int g0 = 0; g0 < nt; g0 += G) {
            const int gend = min(g0 + G, nt);
            const int cnt = (gend * (gend + 1) - g0 * (g0 + 1)) / 2;
            if (L < cnt) {
                for (int c = 0; c < gend; ++c) {
                    const int h = gend - max(c, g0);
                    if (L < h) {
                        bk = c;
                        bj = max(c, g0) + L;
                        return;
                    }
                    L -= h;
                }
            }
            L -= cnt;
        }
        bj = bk = 0;   // not reached: L < nb
        return;
    }
    int r = (int)((sqrtf(8.f * b + 1.f) - 1.f) * 0.5f);
    while (r * (r + 1) / 2 > b) --r;
    while ((r + 1) * (r + 2) / 2 <= b) ++r;
    bj = r;
    bk = b - r * (r + 1) / 2;
}

// BK samples x BT features of X in registers, V consecutive features per load.
// The registers hold the raw values (the mean where the element is outside X,
// so that it normalises to exactly 0); the normalisation happens when the tile
// is written to LDS, so the loads for the next tile stay in flight during the
// current tile's MFMAs instead of being waited for right after they are issued.
template <int V> struct ZTile {
    static constexpr int CPR = BT / V;              // chunks per sample row
    static constexpr int CH = BK * CPR;
    static constexpr int PER = (CH + NT - 1) / NT;
    float v[PER][V];
    __device__ __forceinline__ void load(const pk_syrk_args &a, int64_t col0, int64_t i0, int tid,
                                         const float *smu) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int q = p * NT + tid;
            const int r = q / CPR;
            const int c = (q % CPR) * V;
            const int64_t i = i0 + r, col = col0 + c;
            if (q < CH && i < a.n && col + V <= a.m) {
                pk_ldv<V>(a.X + i * a.ldx + col, v[p]);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e)
                    v[p][e] = (q < CH && i < a.n && col + e < a.m) ? a.X[i * a.ldx + col + e]
                                                                   : ((q < CH) ? smu[c + e] : 0.f);
            }
        }
    }
    __device__ __forceinline__ void store(float *S, int tid, const float *smu, const float *srs) const {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int q = p * NT + tid;
            if (q >= CH)
                break;
            const int c = (q % CPR) * V;
            float z[V];
#pragma unroll
            for (int e = 0; e < V; ++e)
                z[e] = (v[p][e] - smu[c + e]) * srs[c + e];
            pk_stv<V>(S + (q / CPR) * LDR + c, z);
        }
    }
};

#if IL
// The k loop of a full tile (its features inside X, n a multiple of BK, 16-byte aligned
// rows, at least two k tiles), separately for diagonal blocks (one operand tile) and the
// others: no bounds checks, so one step is one basic block, and the scheduling-group
// barriers lay it out as: the step's fragment reads, then its MFMAs with the next tile's
// normalised LDS stores (from registers) and the following tile's global loads (into the
// same registers, after their stores) placed between them, then the barrier.  The last
// step stores into the idle stage and re-loads the last tile (clamped), which nothing
// reads.  Each thread's columns are fixed, so their means and reciprocal deviations are
// taken from LDS once, before the loop.
constexpr int IL_P = BK * BT / 4 / NT;           // 16-byte chunks of one operand tile per thread

__device__ __forceinline__ void il_load(const pk_syrk_args &a, int64_t col0, int64_t i0, int tid, f32x4 *r) {
#pragma unroll
    for (int p = 0; p < IL_P; ++p) {
        const int q = p * NT + tid;
#if IL == 2
        // a sample past n reads the last one (its normalised value is zeroed at the store)
        r[p] = *reinterpret_cast<const f32x4 *>(a.X + min(i0 + q / (BT / 4), a.n - 1) * a.ldx + col0 +
                                                (q % (BT / 4)) * 4);
#else
        r[p] = *reinterpret_cast<const f32x4 *>(a.X + (i0 + q / (BT / 4)) * a.ldx + col0 + (q % (BT / 4)) * 4);
#endif
    }
}

#if IL == 2
__device__ __forceinline__ void il_store(float *S, int tid, const f32x4 *r, const f32x4 *mu, const f32x4 *rs,
                                         int64_t i0, int64_t n) {
#pragma unroll
    for (int p = 0; p < IL_P; ++p) {
        const int q = p * NT + tid;
        const f32x4 z = (r[p] - mu[p]) * rs[p];
        const uint32_t keep = 0u - (uint32_t)(i0 + q / (BT / 4) < n);     // samples past n add zeros
        *reinterpret_cast<f32x4 *>(S + (q / (BT / 4)) * LDR + (q % (BT / 4)) * 4) =
            __builtin_bit_cast(f32x4, __builtin_bit_cast(u32x4, z) & keep);
    }
}
#else
__device__ __forceinline__ void il_store(float *S, int tid, const f32x4 *r, const f32x4 *mu, const f32x4 *rs) {
#pragma unroll
    for (int p = 0; p < IL_P; ++p) {
        const int q = p * NT + tid;
        *reinterpret_cast<f32x4 *>(S + (q / (BT / 4)) * LDR + (q % (BT / 4)) * 4) = (r[p] - mu[p]) * rs[p];
    }
}
#endif

#if IL == 2
#define IL_STORE(S, r, mu, rs, i0) il_store(S, tid, r, mu, rs, i0, a.n)
#else
#define IL_STORE(S, r, mu, rs, i0) il_store(S, tid, r, mu, rs)
#endif

template <bool DIAG>
__device__ __forceinline__ void il_main(const pk_syrk_args &a, float *lds, int64_t j0, int64_t k0, int tid,
                                        int wm, int wn, int g, int l16, float (*stat)[BT], f32x4 (&acc)[FM][FN]) {
    constexpr int OPS = DIAG ? 1 : 2;
    constexpr int DSR = (BK / 4) * (FM + FN);    // fragment reads per step
    constexpr int MMA = (BK / 4) * FM * FN;      // MFMAs per step
    constexpr int DSW = OPS * IL_P;              // LDS stores per step
    constexpr int VMR = OPS * IL_P;              // global loads per step
    constexpr int MW = MMA / (2 * DSW) > 0 ? MMA / (2 * DSW) : 1;
    constexpr int MV = MMA / (4 * VMR) > 0 ? MMA / (4 * VMR) : 1;
    constexpr int REST = MMA - DSW * MW - VMR * MV;
    f32x4 muj[IL_P], rsj[IL_P], muk[IL_P], rsk[IL_P];
#pragma unroll
    for (int p = 0; p < IL_P; ++p) {
        const int c = ((p * NT + tid) % (BT / 4)) * 4;
        muj[p] = f32x4{stat[0][c], stat[0][c + 1], stat[0][c + 2], stat[0][c + 3]};
        rsj[p] = f32x4{stat[1][c], stat[1][c + 1], stat[1][c + 2], stat[1][c + 3]};
        muk[p] = f32x4{stat[2][c], stat[2][c + 1], stat[2][c + 2], stat[2][c + 3]};
        rsk[p] = f32x4{stat[3][c], stat[3][c + 1], stat[3][c + 2], stat[3][c + 3]};
    }
#if IL == 2
    const int64_t nk = (a.n + BK - 1) / BK;
#else
    const int64_t nk = a.n / BK;
#endif
    f32x4 rj[IL_P], rk[IL_P];
    il_load(a, j0, 0, tid, rj);
    if (!DIAG)
        il_load(a, k0, 0, tid, rk);
    IL_STORE(lds, rj, muj, rsj, 0);
    if (!DIAG)
        IL_STORE(lds + TILE, rk, muk, rsk, 0);
    il_load(a, j0, BK, tid, rj);
    if (!DIAG)
        il_load(a, k0, BK, tid, rk);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const float *Sj = lds + 2 * cur * TILE, *Sk = DIAG ? Sj : Sj + TILE;
        float *Nj = lds + 2 * (cur ^ 1) * TILE, *Nk = Nj + TILE;
        float fa[BK / 4][FM], fb[BK / 4][FN];
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
                fa[s][i] = Sj[(4 * s + g) * LDR + wm * WTM + i * 16 + l16];
#pragma unroll
            for (int j = 0; j < FN; ++j)
                fb[s][j] = Sk[(4 * s + g) * LDR + wn * WTN + j * 16 + l16];
        }
#pragma unroll
        for (int s = 0; s < BK / 4; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s][i], fb[s][j], acc[i][j], 0, 0, 0);
        IL_STORE(Nj, rj, muj, rsj, (kt + 1) * BK);               // tile kt+1
        if (!DIAG)
            IL_STORE(Nk, rk, muk, rsk, (kt + 1) * BK);
        const int64_t i2 = min(kt + 2, nk - 1) * BK;             // tile kt+2
        il_load(a, j0, i2, tid, rj);
        if (!DIAG)
            il_load(a, k0, i2, tid, rk);
        __builtin_amdgcn_sched_group_barrier(0x100, DSR, 0);     // the fragment reads
#pragma unroll
        for (int w = 0; w < DSW; ++w) {
            __builtin_amdgcn_sched_group_barrier(0x008, MW, 0);  // MFMAs, then one LDS store
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
        }
#pragma unroll
        for (int v = 0; v < VMR; ++v) {
            __builtin_amdgcn_sched_group_barrier(0x008, MV, 0);  // MFMAs, then one global load
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, REST, 0);
        __syncthreads();
    }
}
#endif

template <int V>
__device__ __forceinline__ void syrk32_body(const pk_syrk_args &a, float *lds, float (*stat)[BT]) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WAVES_N;
    const int wn = wave % WAVES_N;
    const int g = lane >> 4;
    const int l16 = lane & 15;
    const int nt = (int)((a.m + BT - 1) / BT);
    if ((int)blockIdx.x >= nt * (nt + 1) / 2)
        return;
    int bj, bk;
    tri_tile(blockIdx.x, nt, bj, bk);
    const bool diag = (bj == bk);
    const int64_t j0 = (int64_t)bj * BT;
    const int64_t k0 = (int64_t)bk * BT;

    for (int c = tid; c < BT; c += NT) {
        stat[0][c] = (j0 + c < a.m) ? a.mean[j0 + c] : 0.f;
        stat[1][c] = (j0 + c < a.m) ? 1.0f / a.std[j0 + c] : 1.f;
        stat[2][c] = (k0 + c < a.m) ? a.mean[k0 + c] : 0.f;
        stat[3][c] = (k0 + c < a.m) ? 1.0f / a.std[k0 + c] : 1.f;
    }
    __syncthreads();

    // stage s: the j tile at lds + 2*s*TILE, the k tile right after it
    // (a diagonal block reads its j tile for both operands)
    auto jt = [&](int s) { return lds + 2 * s * TILE; };
    auto kt_ = [&](int s) { return diag ? lds + 2 * s * TILE : lds + (2 * s + 1) * TILE; };

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

#if IL
#if IL == 2
    if (j0 + BT <= a.m && k0 + BT <= a.m && a.n > BK && a.aligned && V == 4) {
#else
    if (j0 + BT <= a.m && k0 + BT <= a.m && a.n % BK == 0 && a.n >= 2 * BK && a.aligned && V == 4) {
#endif
        if (diag)
            il_main<true>(a, lds, j0, k0, tid, wm, wn, g, l16, stat, acc);
        else
            il_main<false>(a, lds, j0, k0, tid, wm, wn, g, l16, stat, acc);
    } else {
#endif
    const int64_t nk = (a.n + BK - 1) / BK;
    ZTile<V> tj, tk;
    tj.load(a, j0, 0, tid, stat[0]);
    if (!diag)
        tk.load(a, k0, 0, tid, stat[2]);
    if (GST == 2) {
        tj.store(jt(0), tid, stat[0], stat[1]);
        if (!diag)
            tk.store(kt_(0), tid, stat[2], stat[3]);
        if (nk > 1) {
            tj.load(a, j0, BK, tid, stat[0]);
            if (!diag)
                tk.load(a, k0, BK, tid, stat[2]);
        }
        __syncthreads();
    }

    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (GST == 2) ? (int)(kt & 1) : 0;
        if (GST == 1) {
            tj.store(jt(0), tid, stat[0], stat[1]);
            if (!diag)
                tk.store(kt_(0), tid, stat[2], stat[3]);
            __syncthreads();
            if (kt + 1 < nk) {
                tj.load(a, j0, (kt + 1) * BK, tid, stat[0]);
                if (!diag)
                    tk.load(a, k0, (kt + 1) * BK, tid, stat[2]);
            }
        }
        const float *Sj = jt(cur), *Sk = kt_(cur);
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
            const int kk = 4 * s + g;                 // sample of k slot g in step s
            float fa[FM], fb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                fa[i] = Sj[kk * LDR + wm * WTM + i * 16 + l16];
#pragma unroll
            for (int j = 0; j < FN; ++j)
                fb[j] = Sk[kk * LDR + wn * WTN + j * 16 + l16];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        if (GST == 2 && kt + 1 < nk) {
            // registers hold tile kt+1: write it to the other stage (its last
            // readers finished before the previous barrier), fetch tile kt+2
            tj.store(jt(cur ^ 1), tid, stat[0], stat[1]);
            if (!diag)
                tk.store(kt_(cur ^ 1), tid, stat[2], stat[3]);
            if (kt + 2 < nk) {
                tj.load(a, j0, (kt + 2) * BK, tid, stat[0]);
                if (!diag)
                    tk.load(a, k0, (kt + 2) * BK, tid, stat[2]);
            }
        }
        __syncthreads();
    }
#if IL
    }
#endif

    const float denom = (float)(a.n - 1);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t k = k0 + wn * WTN + j * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = j0 + wm * WTM + i * 16 + 4 * g + r;
                if (row < a.m && k < a.m && (!diag || row >= k)) {
                    const float v = acc[i][j][r] / denom;
                    a.R[row * a.ldr + k] = v;
                    a.R[k * a.ldr + row] = v;
                }
            }
        }
}

extern "C" __global__ void __launch_bounds__(NT) pk_syrk(pk_syrk_args a) {
    if (blockDim.x != NT)
        return;
    __shared__ __attribute__((aligned(16))) float lds[LDS_FLOATS];
#if IL == 3
    // the statistics in the second stage: the general loop (edge tiles) uses the first
    // only, and the interleaved loop reads them into registers before it first writes
    // the second (after a barrier), so the two stages are the block's whole LDS
    float (*stat)[BT] = reinterpret_cast<float (*)[BT]>(lds + 2 * TILE);
#else
    __shared__ float stat[4][BT];   // mean and 1/std of the j columns, then of the k columns
#endif
    if (VEC > 1 && a.aligned)
        syrk32_body<VEC>(a, lds, stat);
    else
        syrk32_body<1>(a, lds, stat);
}
