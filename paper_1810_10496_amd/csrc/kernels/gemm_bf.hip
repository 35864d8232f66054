// gemm_bf.hip -- D = alpha * A B + beta * C on bf16 MFMA from prepared operands.
//
// The GEMM of the paper's suite (Sec. 2.2) in its reduced-precision forms,
// split into two kernels:
//
//   pk_gemm_prep  rounds an FP32 operand to bf16 once (PREC 1: hi = bf16(x);
//                 PREC 2 also lo = bf16(x - hi)) into a caller workspace, with
//                 the contraction index contiguous: A [M][Kp] as it is, B
//                 transposed to [N][Kp] through an LDS tile; k in [K, Kp) is
//                 zero, Kp a multiple of 64.
//   pk_gemm_bf    the product of the prepared operands: both tiles are plain
//                 16-byte row copies into LDS (no conversion, no transpose in
//                 the main loop, half the bytes of FP32 operands), two LDS
//                 stages with one barrier per k-step, and the global loads
//                 for step k+2 in flight during step k+1's MFMAs.
//                 v_mfma_f32_16x16x32_bf16 with FP32 accumulation; split
//                 issues hi*hi + hi*lo + lo*hi per fragment pair.
//
// Built with SYRK=1 the same file is the bf16 / split rank-k product of the
// correlation and covariance (CORR, Sec. 2.2 / 3.4): pk_corr_prep writes
// Z^T = ((X - mean) / std)^T with the sample index contiguous, and pk_gemm_bf
// multiplies it by itself over the lower-triangle tiles only (square tiles,
// A = B), scaling by 1/(n-1) and storing each value at (j, k) and (k, j).
//
// Fragment scheme as in the other MFMA kernels: lane l supplies row l % 16 of
// a 16-row block, lane group g = l / 16 takes the contiguous k range
// [g*BK/4, (g+1)*BK/4) of the tile (eight k per MFMA), and receives rows
// 4g .. 4g+3 of output column l % 16.  The LDS row stride is BK + LDS_PAD bf16
// (16-byte rows); the padding is a tuning knob, because which stride keeps the
// 16-byte fragment reads and row stores off each other's banks is measured,
// not derived (a pad of 16 cuts the bank-conflict cycles per access from 1.0 to
// 0.33 for 32-deep tiles).
#include "pk_device.h"

#ifndef PREC
#define PREC 1
#endif
#ifndef BM
#define BM 256
#endif
#ifndef BN
#define BN 256
#endif
#ifndef BK
#define BK 64
#endif
#ifndef WAVES_M
#define WAVES_M 2
#endif
#ifndef WAVES_N
#define WAVES_N 4
#endif
#ifndef ORDER
#define ORDER 3
#endif
#ifndef LDS_PAD      // row padding of the LDS tiles, in bf16 elements (a multiple of 8)
#define LDS_PAD 8
#endif
#ifndef PIPE         // 0: tiles staged through registers; 1: direct-to-LDS loads, swizzled tiles;
#define PIPE 0       // 2: as 1, with the next k-step's fragments read during this one's MFMAs;
#endif               // 3: as 1, two wave groups alternating compute and memory phases (ping-pong)
#ifndef DSTAGES      // LDS stages of the direct-to-LDS pipelines (PIPE 1: 2 or 3; PIPE 2, 3: 3 or 4)
#define DSTAGES 3
#endif
#ifndef SCHED        // 1: a scheduling fence between a k-step's fragment reads and its MFMAs
#define SCHED 0      // (PIPE 3: raised issue priority during the compute phase)
#endif
#ifndef SYRK         // 1: the correlation / covariance rank-k form (below)
#define SYRK 0
#endif
#ifndef EPI          // 1: the epilogue can also write the result as the next product's prepared
#define EPI 0        // operand (bf16 rows, hi and lo planes for split): chained products
#endif
static_assert(EPI == 0 || !SYRK, "EPI applies to the GEMM form");

#if SYRK
#define FAMILY ((PREC) == 1 ? PKF_SYRK_BF16 : PKF_SYRK_SPLIT)
#else
#define FAMILY ((PREC) == 1 ? PKF_GEMM_BF16_WS : PKF_GEMM_SPLIT_WS)
#endif

constexpr int NT = 64 * WAVES_M * WAVES_N;
constexpr int WTM = BM / WAVES_M;
constexpr int WTN = BN / WAVES_N;
constexpr int FM = WTM / 16;
constexpr int FN = WTN / 16;
constexpr int KG = BK / 4;
constexpr int STEPS = BK / 32;
constexpr int PLANES = (PREC == 2) ? 2 : 1;
constexpr int LDK = BK + LDS_PAD;
constexpr int TILE_ELEMS = (BM + BN) * LDK;
constexpr int LDS_ELEMS = 2 * PLANES * TILE_ELEMS;
static_assert(PREC == 1 || PREC == 2, "PREC must be 1 or 2");
static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be a multiple of 16");
static_assert(BK == 32 || BK == 64, "BK must be 32 or 64");
static_assert(LDS_PAD % 8 == 0, "rows must stay 16-byte aligned");

// direct-to-LDS pipeline: a stage holds, per plane, the A tile then the B tile,
// each BK bf16 per row without padding.  The 16-byte chunks of a tile are
// numbered row by row (chunk q = row * CPR + k / 8) and stored XOR-swizzled in
// 128-byte lines: chunk q sits at slot (q % 8) ^ ((q / 8) % 8) of line q / 8,
// so the 16 rows a fragment read touches spread over all banks.
constexpr int CPR = BK / 8;
constexpr int STAGE_ELEMS = PLANES * (BM + BN) * BK;
constexpr int LPA = BM * CPR / NT;                 // direct loads per thread and plane, A tile
constexpr int LPB = BN * CPR / NT;
constexpr int LPT = PLANES * (LPA + LPB);          // direct loads per thread and k-tile
constexpr int LDS_TOTAL = (PIPE >= 1) ? DSTAGES * STAGE_ELEMS : LDS_ELEMS;
static_assert(PIPE >= 0 && PIPE <= 3, "PIPE must be 0, 1, 2 or 3");
static_assert(PIPE != 3 || ((DSTAGES == 3 || DSTAGES == 4) && (WAVES_M * WAVES_N) % 2 == 0),
              "PIPE 3: DSTAGES 3 or 4 and an even number of waves");
static_assert(PIPE != 3 || (DSTAGES - 2) * LPT <= 63, "PIPE 3: outstanding loads beyond the wait counter");
static_assert(PIPE == 0 || ((BM * CPR) % NT == 0 && (BN * CPR) % NT == 0),
              "direct loads: the tile chunks must divide evenly over the threads");
static_assert(PIPE != 1 || DSTAGES == 2 || DSTAGES == 3, "PIPE 1: DSTAGES must be 2 or 3");
static_assert(PIPE != 2 || DSTAGES == 3 || DSTAGES == 4, "PIPE 2: DSTAGES must be 3 or 4");
static_assert(PIPE == 0 || LPT <= 63, "outstanding loads beyond the wait counter");
static_assert(LDS_TOTAL * 2 <= 163840, "LDS over the 160 KiB per workgroup");
static_assert(!SYRK || (BM == BN && (ORDER == 0 || ORDER == 2)), "rank-k form: square tiles, ORDER 0 or 2");

constexpr int PT = 64;    // transposing preparation: source columns per block
constexpr int PTK = 64;   // ... and source rows per block (recorded in the knob record)

// knob slot X2: 2, or 3 when the epilogue can write the prepared-operand layout (EPI)
PK_DEFINE_KNOBS(FAMILY, BM, BN, BK, WAVES_M, WAVES_N, 8, 1, 2, ORDER, PREC, 2 + EPI, NT, LDS_TOTAL * 2,
                PK_KERNEL_ABI_VERSION, PTK)

__device__ __forceinline__ void tile_of(int bid, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int nb = tiles_m * tiles_n;
    if (ORDER == 3 && (nb % 8) == 0)             // consecutive blocks go to different XCDs:
        bid = (bid % 8) * (nb / 8) + bid / 8;    // give each XCD a contiguous run of tiles
    if (ORDER == 0) {
        tm = bid / tiles_n;
        tn = bid % tiles_n;
    } else if (ORDER == 1) {
        tn = bid / tiles_m;
        tm = bid % tiles_m;
    } else {                                     // groups of 8 tile rows sweep the columns
        const int G = 8;
        const int group = bid / (G * tiles_n);
        const int first = group * G;
        const int gsz = min(tiles_m - first, G);
        const int r = bid - group * G * tiles_n;
        tm = first + r % gsz;
        tn = r / gsz;
    }
}

#if SYRK
// block index -> lower-triangle tile (bj >= bk) of an nt x nt tile grid
__device__ __forceinline__ void tri_tile(int b, int nt, int &bj, int &bk) {
    if (ORDER == 2) {
        // Blocks are dealt to the 8 XCDs in turn; each XCD gets a contiguous
        // range of logical tiles, and the logical order walks groups of 8 tile
        // rows column by column, so the tiles an XCD runs together share their
        // operand rows in its L2.
        const int nb = nt * (nt + 1) / 2;
        const int q = nb / 8, rem = nb % 8, x = b % 8;
        int L = x * q + min(x, rem) + b / 8;
        for (int g0 = 0; g0 < nt; g0 += 8) {
            const int gend = min(g0 + 8, nt);
            const int cnt = (gend * (gend + 1) - g0 * (g0 + 1)) / 2;   // tiles in rows [g0, gend)
            if (L < cnt) {
                for (int c = 0; c < gend; ++c) {
                    const int h = gend - max(c, g0);                   // of them in column c
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
    while (r * (r + 1) / 2 > b)
        --r;
    while ((r + 1) * (r + 2) / 2 <= b)
        ++r;
    bj = r;
    bk = b - r * (r + 1) / 2;
}
#endif

// ROWS rows x BK bf16 of a prepared operand ([rows][Kp]), 16-byte chunks
template <int ROWS> struct Tile {
    static constexpr int CPR = BK / 8;            // chunks per row
    static constexpr int CH = ROWS * CPR;
    static constexpr int PER = (CH + NT - 1) / NT;
    u32x4 v[PLANES][PER];
    __device__ __forceinline__ void load(const uint16_t *H, const uint16_t *L, int64_t rows, int64_t ld,
                                         int64_t row0, int64_t k0, int tid) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int q = p * NT + tid;
            const int64_t row = row0 + q / CPR;
            const int64_t off = row * ld + k0 + (q % CPR) * 8;
            const bool in = q < CH && row < rows;
            v[0][p] = in ? *reinterpret_cast<const u32x4 *>(H + off) : u32x4{0u, 0u, 0u, 0u};
            if (PLANES == 2)
                v[PLANES - 1][p] = in ? *reinterpret_cast<const u32x4 *>(L + off) : u32x4{0u, 0u, 0u, 0u};
        }
    }
    __device__ __forceinline__ void store(uint16_t *S, uint16_t *S2, int tid) const {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int q = p * NT + tid;
            if (q >= CH)
                break;
            const int o = (q / CPR) * LDK + (q % CPR) * 8;
            *reinterpret_cast<u32x4 *>(S + o) = v[0][p];
            if (PLANES == 2)
                *reinterpret_cast<u32x4 *>(S2 + o) = v[PLANES - 1][p];
        }
    }
};

__device__ __forceinline__ bf16x8 frag(const uint16_t *S, int row, int g, int s) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(S + row * LDK + g * KG + s * 8));
}

__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

#if PIPE >= 1
typedef __attribute__((address_space(3))) void pk_lds_void;
typedef __attribute__((address_space(1))) void pk_glb_void;

// chunk number <-> stored position (the swizzle is its own inverse).  A
// 16-byte fragment read is served 16 lanes at a time, lanes 0-7 with 16-23 and
// so on (measured: this is the grouping under which the bank-conflict counter
// reads zero for 32-deep tiles and two-way conflicts for plainer 64-deep
// layouts), over 64 four-byte banks.  With 32-deep tiles a line holds two rows
// and the slot is XORed with the line number; with 64-deep tiles (one row per
// line) it is XORed with row & 6, and lane groups g and g ^ 1 read chunks that
// differ in bit 0, so the 16 reads of each pass cover all 64 banks.
__device__ __forceinline__ int swz(int q) {
    const int line = q >> 3;
    const int f = (CPR == 8) ? (line & 6) : (line & 7);
    return (q & ~7) | ((q ^ f) & 7);
}

// chunk of a tile row that lane group g reads in k-step s
__device__ __forceinline__ int kchunk(int g, int s) { return (CPR == 8) ? s * 4 + g : g * STEPS + s; }

// wait until at most N vector-memory operations of this wave are outstanding
template <int N> __device__ __forceinline__ void wait_loads() {
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | (((N >> 4) & 3) << 14));
}

// Workgroup barrier without a memory fence: __syncthreads() would also wait for
// every outstanding global load, the next tile's included.  The LDS side is
// covered by hand: each wave waits for its own direct loads (wait_loads) and
// has consumed its fragment reads before it arrives; the empty asm statements
// keep the compiler from moving LDS accesses across the barrier.
__device__ __forceinline__ void barrier_lds() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ bf16x8 frag_at(const uint16_t *S, int off) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(S + off));
}
#endif

extern "C" __global__ void __launch_bounds__(NT) pk_gemm_bf(pk_gemmbf_args a) {
    if (blockDim.x != NT)
        return;
    __shared__ __attribute__((aligned(16))) uint16_t lds[LDS_TOTAL];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WAVES_N;
    const int wn = wave % WAVES_N;
    const int g = lane >> 4;
    const int l16 = lane & 15;

#if SYRK
    // lower-triangle tiles of the m x m result (M = N = m, A = B = Z^T)
    const int nt = (int)((a.M + BM - 1) / BM);
    if ((int)blockIdx.x >= nt * (nt + 1) / 2)
        return;
    int tm, tn;
    tri_tile(blockIdx.x, nt, tm, tn);
    const bool diag = (tm == tn);
#else
    const int tiles_m = (int)((a.M + BM - 1) / BM);
    const int tiles_n = (int)((a.N + BN - 1) / BN);
    int tm, tn;
    tile_of(blockIdx.x, tiles_m, tiles_n, tm, tn);
    if (tm >= tiles_m || tn >= tiles_n)
        return;
#endif
    const int64_t row0 = (int64_t)tm * BM;
    const int64_t col0 = (int64_t)tn * BN;

    // stage s, plane p: A rows at lds + (s*PLANES + p)*TILE_ELEMS, B rows right after
    auto a_pl = [&](int s, int p) { return lds + (s * PLANES + p) * TILE_ELEMS; };
    auto b_pl = [&](int s, int p) { return lds + (s * PLANES + p) * TILE_ELEMS + BM * LDK; };

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int64_t nk = a.Kp / BK;
#if PIPE >= 1
    // Each wave's direct load fills 64 consecutive stored chunks (1 KiB at a
    // wave-uniform LDS address); a lane fetches the chunk that belongs at its
    // position.  Rows past M (N) read row M-1 (N-1): they only feed outputs
    // that are never stored.
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    int64_t oa[LPA], ob[LPB];
#pragma unroll
    for (int p = 0; p < LPA; ++p) {
        const int q = swz((p * (NT / 64) + wave_u) * 64 + lane);
        oa[p] = min(row0 + q / CPR, a.M - 1) * a.Kp + (q % CPR) * 8;
    }
#pragma unroll
    for (int p = 0; p < LPB; ++p) {
        const int q = swz((p * (NT / 64) + wave_u) * 64 + lane);
        ob[p] = min(col0 + q / CPR, a.N - 1) * a.Kp + (q % CPR) * 8;
    }
    auto issue = [&](int64_t kt, int st) {
        const int64_t k0 = kt * BK;
#pragma unroll
        for (int pl = 0; pl < PLANES; ++pl) {
            const uint16_t *sa = (pl == 0) ? a.Ah : a.Al;
            const uint16_t *sb = (pl == 0) ? a.Bh : a.Bl;
            uint16_t *da = lds + st * STAGE_ELEMS + pl * (BM + BN) * BK;
            uint16_t *db = da + BM * BK;
#pragma unroll
            for (int p = 0; p < LPA; ++p)
                __builtin_amdgcn_global_load_lds((pk_glb_void *)(sa + oa[p] + k0),
                                                 (pk_lds_void *)(da + (p * (NT / 64) + wave_u) * 512), 16, 0, 0);
#pragma unroll
            for (int p = 0; p < LPB; ++p)
                __builtin_amdgcn_global_load_lds((pk_glb_void *)(sb + ob[p] + k0),
                                                 (pk_lds_void *)(db + (p * (NT / 64) + wave_u) * 512), 16, 0, 0);
        }
    };
    // fragment 0 of k-step s (lane group g reads chunk kchunk(g, s) of its row);
    // fragment i is 16 rows further, which leaves the swizzle unchanged
    int fa0[STEPS], fb0[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        fa0[s] = swz((wm * WTM + l16) * CPR + kchunk(g, s)) * 8;
        fb0[s] = BM * BK + swz((wn * WTN + l16) * CPR + kchunk(g, s)) * 8;
    }
    constexpr int FRAG_STRIDE = 16 * CPR * 8;
    constexpr int PLANE = (BM + BN) * BK;
#endif
#if PIPE == 2
    // Fragments of one k-step in registers.  Step u's MFMAs run on one set while
    // the reads of step u+1 fill the other; when u+1 starts a new tile, the
    // wait for that tile and the barrier come first, so a tile's LDS reads
    // overlap the previous tile's MFMAs instead of following a barrier alone.
    struct Frags {
        bf16x8 a[FM], b[FN];
#if PREC == 2
        bf16x8 a2[FM], b2[FN];
#endif
    };
    auto read = [&](Frags &f, int st, int s) {
        const uint16_t *S = lds + st * STAGE_ELEMS;
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            f.a[i] = frag_at(S, fa0[s] + i * FRAG_STRIDE);
#if PREC == 2
            f.a2[i] = frag_at(S, PLANE + fa0[s] + i * FRAG_STRIDE);
#endif
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            f.b[j] = frag_at(S, fb0[s] + j * FRAG_STRIDE);
#if PREC == 2
            f.b2[j] = frag_at(S, PLANE + fb0[s] + j * FRAG_STRIDE);
#endif
        }
    };
    auto mfmas = [&](const Frags &f) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
#if PREC == 2
                acc[i][j] = mma(f.a2[i], f.b[j], acc[i][j]);
                acc[i][j] = mma(f.a[i], f.b2[j], acc[i][j]);
#endif
                acc[i][j] = mma(f.a[i], f.b[j], acc[i][j]);
            }
    };
    (void)PLANE;
    // stages: tile k in st_c, tile k+1 in st_n; st_i = (k - 1) mod DSTAGES receives
    // tile k + DSTAGES - 1 (its fragments were read two tiles ago)
    int st_c = 0, st_n = 1, st_i = DSTAGES - 1;
    auto adv = [](int x) { return (x + 1 == DSTAGES) ? 0 : x + 1; };
    // step (k, s): MFMAs on `cur`; first the reads of the following step into `nxt`
    auto step = [&](Frags &cur, Frags &nxt, int64_t k, int s) {
        if (s + 1 < STEPS) {
            read(nxt, st_c, s + 1);
        } else {
            if (k + 1 < nk) {
                // tile k+1 has landed once only tiles past k+1 are outstanding
                if (DSTAGES == 4 && k + 2 < nk)
                    wait_loads<LPT>();
                else
                    wait_loads<0>();
                barrier_lds();   // every wave's part of tile k+1 is in; stage st_i is free
                if (k + DSTAGES - 1 < nk)
                    issue(k + DSTAGES - 1, st_i);
            }
            // unconditional, so that the LDS wait counts stay exact on every path
            // (after the last tile the values read are never used)
            read(nxt, st_n, 0);
        }
        if (SCHED)
            __builtin_amdgcn_sched_barrier(0);
        mfmas(cur);
        if (s + 1 == STEPS) {
            st_c = st_n;
            st_n = adv(st_n);
            st_i = adv(st_i);
        }
    };
    if (nk > 0) {
        for (int t = 0; t < DSTAGES - 1; ++t)
            if (t < nk)
                issue(t, t);
        wait_loads<0>();
        barrier_lds();
        Frags f0, f1;
        read(f0, 0, 0);
        if (STEPS == 2) {
            for (int64_t k = 0; k < nk; ++k) {
                step(f0, f1, k, 0);
                step(f1, f0, k, STEPS - 1);
            }
        } else {
            int64_t k = 0;
            for (; k + 1 < nk; k += 2) {
                step(f0, f1, k, 0);
                step(f1, f0, k + 1, 0);
            }
            if (k < nk)
                step(f0, f1, k, 0);
        }
    }
#endif
#if PIPE == 1

    for (int s = 0; s < DSTAGES - 1; ++s)
        if (s < nk)
            issue(s, s);
    int st_c = 0, st_i = DSTAGES - 1;
    for (int64_t kt = 0; kt < nk; ++kt) {
        // tile kt has landed once only the later tiles' loads are outstanding
        if (DSTAGES == 3 && kt + 1 < nk)
            wait_loads<LPT>();
        else
            wait_loads<0>();
        barrier_lds();       // every wave's part of tile kt is in; stage st_i is no longer read
        if (kt + DSTAGES - 1 < nk)
            issue(kt + DSTAGES - 1, st_i);
        const uint16_t *S = lds + st_c * STAGE_ELEMS;
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            bf16x8 fa[FM], fb[FN];
#if PREC == 2
            bf16x8 fa2[FM], fb2[FN];
#endif
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                fa[i] = frag_at(S, fa0[s] + i * FRAG_STRIDE);
#if PREC == 2
                fa2[i] = frag_at(S, PLANE + fa0[s] + i * FRAG_STRIDE);
#endif
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                fb[j] = frag_at(S, fb0[s] + j * FRAG_STRIDE);
#if PREC == 2
                fb2[j] = frag_at(S, PLANE + fb0[s] + j * FRAG_STRIDE);
#endif
            }
            if (SCHED)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
#if PREC == 2
                    acc[i][j] = mma(fa2[i], fb[j], acc[i][j]);
                    acc[i][j] = mma(fa[i], fb2[j], acc[i][j]);
#endif
                    acc[i][j] = mma(fa[i], fb[j], acc[i][j]);
                }
        }
        (void)PLANE;
        st_c = (st_c + 1 == DSTAGES) ? 0 : st_c + 1;
        st_i = (st_i + 1 == DSTAGES) ? 0 : st_i + 1;
    }
#elif PIPE == 3
    // Ping-pong: the first half of the waves (group 0) and the second half
    // (group 1) take turns, so that on each SIMD one wave runs MFMAs while the
    // other reads LDS and issues loads.  Every wave works tile k in a memory
    // phase (read all of the tile's fragments into registers, issue the direct
    // loads of tile k + DSTAGES - 1) and then a compute phase (the tile's
    // MFMAs), with a barrier after each phase.  Group 1 passes one barrier
    // before its first phase and group 0 one after its last, so each barrier
    // ends a memory phase of one group and a compute phase of the other.
    //   Counting barriers from the one after the prologue (0): group 0's memory
    // phase for tile k ends at barrier 2k+1 and its compute phase at 2k+2;
    // group 1's at 2k+2 and 2k+3.  Tile k+1 is first read after barrier 2k+2,
    // so every wave has waited for its own loads of tiles <= k+1 before it
    // (group 0 at the end of compute phase k, group 1 at the end of memory
    // phase k).  The stage that tile k + DSTAGES - 1 overwrites held tile k-1,
    // whose last fragment reads (group 1's, completed before barrier 2k) precede
    // both groups' issues of it (after barriers 2k and 2k+1).
    constexpr int DA = DSTAGES - 1;              // tiles issued ahead of the one being read
    const int grp = wave_u / (NT / 128);
    struct Frags {
        bf16x8 a[STEPS][FM], b[STEPS][FN];
#if PREC == 2
        bf16x8 a2[STEPS][FM], b2[STEPS][FN];
#endif
    } f;
    auto read_tile = [&](int st) {
        const uint16_t *S = lds + st * STAGE_ELEMS;
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                f.a[s][i] = frag_at(S, fa0[s] + i * FRAG_STRIDE);
#if PREC == 2
                f.a2[s][i] = frag_at(S, PLANE + fa0[s] + i * FRAG_STRIDE);
#endif
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                f.b[s][j] = frag_at(S, fb0[s] + j * FRAG_STRIDE);
#if PREC == 2
                f.b2[s][j] = frag_at(S, PLANE + fb0[s] + j * FRAG_STRIDE);
#endif
            }
        }
    };
    auto mfma_tile = [&]() {
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
#if PREC == 2
                    acc[i][j] = mma(f.a2[s][i], f.b[s][j], acc[i][j]);
                    acc[i][j] = mma(f.a[s][i], f.b2[s][j], acc[i][j]);
#endif
                    acc[i][j] = mma(f.a[s][i], f.b[s][j], acc[i][j]);
                }
    };
    // tiles <= k+1 complete (the later ones may still be in flight)
    auto wait_next = [&](int64_t k) {
        if (k + DA < nk)
            wait_loads<(DA - 1) * LPT>();
        else
            wait_loads<0>();
    };
    auto phase_end = [&]() {
        __builtin_amdgcn_sched_barrier(0);
        barrier_lds();
        __builtin_amdgcn_sched_barrier(0);
    };
    (void)PLANE;
    if (nk > 0) {
        for (int t = 0; t < DA; ++t)
            if (t < nk)
                issue(t, t);
        if (nk >= DA)
            wait_loads<(DA - 1) * LPT>();
        else
            wait_loads<0>();
        phase_end();                              // barrier 0: tile 0 is in
        if (grp == 1)
            phase_end();                          // barrier 1 (group 0 ends memory phase 0 there)
        int st = 0;                               // stage of tile k
        for (int64_t k = 0; k < nk; ++k) {
            // memory phase
            read_tile(st);
            if (k + DA < nk)
                issue(k + DA, (st + DA) % DSTAGES);
            __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's fragment reads are done
            if (grp == 1)
                wait_next(k);
            phase_end();
            // compute phase
            if (SCHED)
                __builtin_amdgcn_s_setprio(1);
            mfma_tile();
            if (SCHED)
                __builtin_amdgcn_s_setprio(0);
            if (grp == 0)
                wait_next(k);
            phase_end();
            st = (st + 1 == DSTAGES) ? 0 : st + 1;
        }
        if (grp == 0)
            phase_end();
    }
#elif PIPE == 0
    Tile<BM> ta;
    Tile<BN> tb;
    if (nk > 0) {
        ta.load(a.Ah, a.Al, a.M, a.Kp, row0, 0, tid);
        tb.load(a.Bh, a.Bl, a.N, a.Kp, col0, 0, tid);
        ta.store(a_pl(0, 0), a_pl(0, PLANES - 1), tid);
        tb.store(b_pl(0, 0), b_pl(0, PLANES - 1), tid);
        if (nk > 1) {
            ta.load(a.Ah, a.Al, a.M, a.Kp, row0, BK, tid);
            tb.load(a.Bh, a.Bl, a.N, a.Kp, col0, BK, tid);
        }
        __syncthreads();
    }
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const uint16_t *As = a_pl(cur, 0), *Bs = b_pl(cur, 0);
        const uint16_t *As2 = a_pl(cur, PLANES - 1), *Bs2 = b_pl(cur, PLANES - 1);
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            bf16x8 fa[FM], fb[FN];
#if PREC == 2
            bf16x8 fa2[FM], fb2[FN];
#endif
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                fa[i] = frag(As, wm * WTM + i * 16 + l16, g, s);
#if PREC == 2
                fa2[i] = frag(As2, wm * WTM + i * 16 + l16, g, s);
#endif
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                fb[j] = frag(Bs, wn * WTN + j * 16 + l16, g, s);
#if PREC == 2
                fb2[j] = frag(Bs2, wn * WTN + j * 16 + l16, g, s);
#endif
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
#if PREC == 2
                    acc[i][j] = mma(fa2[i], fb[j], acc[i][j]);
                    acc[i][j] = mma(fa[i], fb2[j], acc[i][j]);
#endif
                    acc[i][j] = mma(fa[i], fb[j], acc[i][j]);
                }
        }
        (void)As2;
        (void)Bs2;
        if (kt + 1 < nk) {
            // registers hold tile kt+1: write it to the other stage (its last
            // readers finished before the previous barrier), then fetch kt+2
            ta.store(a_pl(cur ^ 1, 0), a_pl(cur ^ 1, PLANES - 1), tid);
            tb.store(b_pl(cur ^ 1, 0), b_pl(cur ^ 1, PLANES - 1), tid);
            if (kt + 2 < nk) {
                ta.load(a.Ah, a.Al, a.M, a.Kp, row0, (kt + 2) * BK, tid);
                tb.load(a.Bh, a.Bl, a.N, a.Kp, col0, (kt + 2) * BK, tid);
            }
        }
        __syncthreads();
    }
#endif

#if SYRK
    // each value at (row, col) and (col, row): the result is exactly symmetric
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t col = col0 + wn * WTN + j * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + wm * WTM + i * 16 + 4 * g + r;
                if (row < a.M && col < a.N && (!diag || row >= col)) {
                    const float v = a.alpha * acc[i][j][r];
                    a.D[row * a.ldd + col] = v;
                    a.D[col * a.ldd + row] = v;
                }
            }
        }
#else
#if EPI
    if (a.ldd < 0) {
        // the result as the next product's prepared operand: rows of -ldd bf16 values
        // (a multiple of 64 covered by the tile columns), RNE hi and, for split, lo =
        // bf16(v - hi) one plane of M rows further; zeros beyond column N
        const int64_t ldt = -a.ldd;
        uint16_t *th = reinterpret_cast<uint16_t *>(a.D);
        uint16_t *tl = th + a.M * ldt;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int64_t col = col0 + wn * WTN + j * 16 + l16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row0 + wm * WTM + i * 16 + 4 * g + r;
                    if (row < a.M && col < ldt) {
                        const float v = col < a.N ? a.alpha * acc[i][j][r] : 0.f;
                        uint32_t hb, lb;
                        pk_split(v, hb, lb);
                        th[row * ldt + col] = (uint16_t)hb;
                        if (PLANES == 2)
                            tl[row * ldt + col] = (uint16_t)lb;
                    }
                }
            }
        return;
    }
#endif
    const bool use_c = a.beta != 0.f;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t col = col0 + wn * WTN + j * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + wm * WTM + i * 16 + 4 * g + r;
                if (row < a.M && col < a.N) {
                    float v = a.alpha * acc[i][j][r];
                    if (use_c)
                        v += a.beta * a.C[row * a.ldc + col];
                    a.D[row * a.ldd + col] = v;
                }
            }
        }
#endif
}

// ---- operand preparation ----------------------------------------------------------------
// transpose == 0: dst[r][k] = src[r][k] for r < rows, k < cols; 0 for cols <= k < ldo
// transpose == 1: dst[c][k] = src[k][c] for c < cols, k < rows; 0 for rows <= k < ldo
// (src is rows x cols with row stride ld; dst has row stride ldo, a multiple of 64)

// eight consecutive values -> eight bf16 (hi) and, for split, eight lo, as 16-byte words
__device__ __forceinline__ void prep_pack8(const float *x, bool split, u32x4 &h, u32x4 &l) {
    uint32_t hb[8], lb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        if (split) {
            pk_split(x[e], hb[e], lb[e]);
        } else {
            hb[e] = pk_bf16_bits(x[e]);
            lb[e] = 0u;
        }
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        h[w] = hb[2 * w] | (hb[2 * w + 1] << 16);
        l[w] = lb[2 * w] | (lb[2 * w + 1] << 16);
    }
}

#if !SYRK
extern "C" __global__ void __launch_bounds__(256) pk_gemm_prep(pk_gemmprep_args a) {
    if (blockDim.x != 256)
        return;
    __shared__ float tile[PTK][PT + 1];
    if (!a.transpose) {
        // 8 consecutive k per item (two 16-byte loads where the source allows,
        // one 16-byte store per plane), grid-stride over rows x (ldo / 8)
        const bool vec = ((reinterpret_cast<uintptr_t>(a.src) & 15) == 0) && ((a.ld & 3) == 0);
        const int64_t per_row = a.ldo / 8;
        const int64_t total = a.rows * per_row;
        for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
            const int64_t r = q / per_row, k = (q % per_row) * 8;
            const float *src = a.src + r * a.ld + k;
            float x[8];
            if (vec && k + 8 <= a.cols) {
                const f32x4 v0 = *reinterpret_cast<const f32x4 *>(src);
                const f32x4 v1 = *reinterpret_cast<const f32x4 *>(src + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    x[e] = v0[e];
                    x[4 + e] = v1[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    x[e] = (k + e < a.cols) ? src[e] : 0.f;
            }
            u32x4 h, l;
            prep_pack8(x, a.split != 0, h, l);
            *reinterpret_cast<u32x4 *>(a.hi + r * a.ldo + k) = h;
            if (a.split)
                *reinterpret_cast<u32x4 *>(a.lo + r * a.ldo + k) = l;
        }
        return;
    }
    // transpose: block = one PTK x 64 tile (k0 .. k0+PTK-1 of src rows, c0 .. c0+63 of
    // src columns); a destination row gets PTK * 2 contiguous bytes from one block
    const int64_t tiles_c = (a.cols + PT - 1) / PT;
    const int64_t k0 = (int64_t)(blockIdx.x / tiles_c) * PTK;
    const int64_t c0 = (int64_t)(blockIdx.x % tiles_c) * PT;
    if (k0 >= a.ldo)
        return;
    const int tx = threadIdx.x % PT, ty = threadIdx.x / PT;   // 64 x 4
    {
        // all of a thread's loads are issued before the first LDS store
        float v[PTK / 4];
        const int64_t c = c0 + tx;
#pragma unroll
        for (int q = 0; q < PTK / 4; ++q) {
            const int64_t k = k0 + q * 4 + ty;
            v[q] = (k < a.rows && c < a.cols) ? a.src[k * a.ld + c] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < PTK / 4; ++q)
            tile[q * 4 + ty][tx] = v[q];
    }
    __syncthreads();
    // thread -> destination row c0 + t/4, k0 + 32q + 8*(t%4) + {0..7}: in each store
    // the four lanes of a row write 64 contiguous bytes, so the 128-byte lines of
    // the destination are filled by whole halves (split stores per lane left
    // partly written lines and extra write traffic)
    const int cc = threadIdx.x / 4, seg = threadIdx.x % 4;
    const int64_t c = c0 + cc;
    if (c >= a.cols)
        return;
#pragma unroll
    for (int half = 0; half < PTK / 32; ++half) {
        const int kk = half * 32 + seg * 8;
        if (k0 + kk >= a.ldo)           // ldo is a multiple of 64, not of PTK
            break;
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            x[e] = tile[kk + e][cc];
        u32x4 h, l;
        prep_pack8(x, a.split != 0, h, l);
        *reinterpret_cast<u32x4 *>(a.hi + c * a.ldo + k0 + kk) = h;
        if (a.split)
            *reinterpret_cast<u32x4 *>(a.lo + c * a.ldo + k0 + kk) = l;
    }
}
#else
// The rank-k operand: Z^T with the sample index contiguous.  Block = PTK samples
// x 64 features of X read row by row (coalesced) into an LDS tile; each thread
// then normalises PTK/4 samples of one feature with that feature's mean and
// 1/std and writes them as 16-byte bf16 chunks, 32 samples apart, so that the
// four lanes of a destination row write 64 contiguous bytes per store.
// Samples n .. ldo-1 are written as 0.
extern "C" __global__ void __launch_bounds__(256) pk_corr_prep(pk_corrprep_args a) {
    if (blockDim.x != 256)
        return;
    __shared__ float tile[PTK][PT + 1];
    const int64_t tiles_c = (a.m + PT - 1) / PT;
    const int64_t i0 = (int64_t)(blockIdx.x / tiles_c) * PTK;
    const int64_t c0 = (int64_t)(blockIdx.x % tiles_c) * PT;
    if (i0 >= a.ldo)
        return;
    const int tx = threadIdx.x % PT, ty = threadIdx.x / PT;
    {
        // all of a thread's loads are issued before the first LDS store
        float v[PTK / 4];
        const int64_t c = c0 + tx;
#pragma unroll
        for (int q = 0; q < PTK / 4; ++q) {
            const int64_t i = i0 + q * 4 + ty;
            v[q] = (i < a.n && c < a.m) ? a.X[i * a.ldx + c] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < PTK / 4; ++q)
            tile[q * 4 + ty][tx] = v[q];
    }
    __syncthreads();
    const int cc = threadIdx.x / 4, seg = threadIdx.x % 4;
    const int64_t c = c0 + cc;
    if (c >= a.m)
        return;
    const float mu = a.mean[c];
    const float rs = 1.0f / a.std[c];
#pragma unroll
    for (int half = 0; half < PTK / 32; ++half) {
        const int kk = half * 32 + seg * 8;
        if (i0 + kk >= a.ldo)
            break;
        float z[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            z[e] = (i0 + kk + e < a.n) ? (tile[kk + e][cc] - mu) * rs : 0.f;
        u32x4 h, l;
        prep_pack8(z, a.split != 0, h, l);
        *reinterpret_cast<u32x4 *>(a.hi + c * a.ldo + i0 + kk) = h;
        if (a.split)
            *reinterpret_cast<u32x4 *>(a.lo + c * a.ldo + i0 + kk) = l;
    }
}
#endif
