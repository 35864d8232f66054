// gemm.hip -- dense product D = alpha * A B + beta * C on MFMA (gfx950).
//
// The GEMM kernel of the paper's suite (Sec. 2.2).  The paper traces most of
// its phase-order gains on this kernel to keeping the running sum in a
// register and storing once, to the unroll factor, and to the address pattern
// of the loads (Sec. 3.4); here the sum lives in MFMA accumulators from the
// start, so what is left to tune is the tiling, the vector width, LDS staging,
// the tile raster order and the LLVM pass pipeline.
//
// Precision (compile-time PREC):
//   0  FP32 operands, v_mfma_f32_16x16x4_f32
//   1  BF16 operands (RNE from FP32 on the way into LDS), v_mfma_f32_16x16x32_bf16
//   2  split BF16: x = hi + lo, product = hi*hi + hi*lo + lo*hi, three
//      v_mfma_f32_16x16x32_bf16 into one FP32 accumulator
// Accumulation is FP32 in every case.
//
// MFMA 16x16 operand layout (one 16x16 output block per wave instruction):
// lane l supplies row (l % 16) of the A block and column (l % 16) of the B
// block, for the k slots of lane group g = l / 16; it receives rows
// 4g .. 4g+3 of output column (l % 16).  Because the instruction sums over
// all k slots, any assignment of real k indices to slots works as long as A
// and B use the same one: lane group g takes the contiguous k range
// [g*BK/4, (g+1)*BK/4) of the tile, so each lane's operands are one
// contiguous run in LDS (a single 16-byte read per fragment).
// With MF = 32 (FP32 only, v_mfma_f32_32x32x2_f32) a block is 32x32: lane l
// supplies row (and column) l % 32 for the k slot of lane group l / 32, the
// two groups take the two halves of the tile's k range, and lane l receives
// column l % 32 of rows 8 (r / 4) + 4 (l / 32) + r % 4, r = 0..15.
#include "pk_device.h"

#ifndef PREC
#define PREC 0
#endif
#ifndef BM
#define BM 128
#endif
#ifndef BN
#define BN 128
#endif
#ifndef BK
#define BK ((PREC) == 0 ? 16 : 32)
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
#ifndef UNROLL
#define UNROLL 1
#endif
#ifndef USE_LDS
#define USE_LDS 1
#endif
#ifndef ORDER
#define ORDER 3
#endif
#ifndef MF           // FP32: output block of one MFMA, 16 (v_mfma_f32_16x16x4_f32) or 32
#define MF 16        // (v_mfma_f32_32x32x2_f32: half the instructions for one wave tile)
#endif
#ifndef FC           // FP32: 0 reads a k-step's fragments all at once; 4 reads them four k at a
#define FC 0         // time, each chunk's MFMAs right after it (deep k-steps in fewer registers)
#endif
#ifndef IL           // FP32, two LDS stages: 1 = full interior tiles run a branch-free k loop whose
#define IL 0         // LDS stores and global loads are interleaved with the MFMAs (below); 2 = the
#endif               // same for K any multiple of 4 (the partial last k tile masked)
#ifndef DK           // FP32 without LDS: 1 = branch-free fragment loads (address clamped into the
#define DK 0         // matrix, value zeroed outside it), so an unrolled k loop is straight-line
#endif               // code whose loads can all be issued ahead of the MFMAs

#define FAMILY ((PREC) == 0 ? PKF_GEMM_F32 : ((PREC) == 1 ? PKF_GEMM_BF16 : PKF_GEMM_SPLIT))

static_assert(MF == 16 || (MF == 32 && PREC == 0), "MF 32 is an FP32 form");
constexpr int NT = 64 * WAVES_M * WAVES_N;
constexpr int WTM = BM / WAVES_M;
constexpr int WTN = BN / WAVES_N;
constexpr int BLK = MF;                   // rows / columns of one MFMA output block
constexpr int NG = 64 / BLK;              // lane groups (k slots of one MFMA)
constexpr int FM = WTM / BLK;
constexpr int FN = WTN / BLK;
constexpr int KI = (PREC == 0) ? NG : 32; // depth of one MFMA
constexpr int KG = BK / NG;               // contiguous k per lane group
constexpr int STEPS = BK / KI;            // MFMAs per fragment pair per tile
static_assert(WTM % BLK == 0 && WTN % BLK == 0, "wave tile must be a multiple of the MFMA block");
static_assert(PREC != 0 || STEPS % 4 == 0, "FP32 fragments are read four k at a time");
static_assert(FC == 0 || (FC == 4 && PREC == 0 && STEPS % FC == 0), "FC is 0, or 4 for FP32");
static_assert(IL == 0 || (PREC == 0 && USE_LDS == 2 && FC == 0), "IL: FP32 with two LDS stages");
static_assert(DK == 0 || (PREC == 0 && USE_LDS == 0 && MF == 16), "DK: FP32 without LDS, 16x16 blocks");
static_assert(BK % KI == 0 && BK % VEC == 0, "bad BK");
static_assert(VEC == 1 || VEC == 2 || VEC == 4, "bad VEC");
static_assert(BN % VEC == 0, "bad BN");

// LDS element: FP32 for PREC 0, bf16 bits otherwise.  Rows are k-contiguous
// (A as [m][k], B transposed to [n][k]); the padding keeps 16-byte fragment
// reads of 8 consecutive lanes on distinct banks.
#ifndef LDS_PAD      // FP32: row padding of the LDS tiles, in elements (a multiple of 4)
#define LDS_PAD 4
#endif
#if PREC == 0
typedef float lds_t;
constexpr int PADK = LDS_PAD;
#else
typedef uint16_t lds_t;
constexpr int PADK = 8;
#endif
constexpr int LDK = BK + PADK;
constexpr int NSPLIT = (PREC == 2) ? 2 : 1;
constexpr int LDS_STAGES = (USE_LDS == 2) ? 2 : 1;
constexpr int LDS_BYTES = USE_LDS ? LDS_STAGES * NSPLIT * (BM + BN) * LDK * (int)sizeof(lds_t) : 0;

// knob slot X2 records MF when it is not 16 (+ 1000 with IL), slot X3 FC
PK_DEFINE_KNOBS(FAMILY, BM, BN, BK, WAVES_M, WAVES_N, VEC, UNROLL, USE_LDS, ORDER, PREC,
                (MF == 16 ? 0 : MF) + 1000 * IL, NT, LDS_BYTES, PK_KERNEL_ABI_VERSION, FC)

// map a block index to a (tile row, tile column)
__device__ __forceinline__ void tile_of(int bid, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int nb = tiles_m * tiles_n;
    if (ORDER == 3 && (nb % 8) == 0)   // blocks are dealt round-robin to 8 XCDs:
        bid = (bid % 8) * (nb / 8) + bid / 8;   // give each XCD a contiguous run
    if (ORDER == 0) {
        tm = bid / tiles_n;
        tn = bid % tiles_n;
    } else if (ORDER == 1) {
        tn = bid / tiles_m;
        tm = bid % tiles_m;
    } else {   // grouped: 8 tile rows sweep the columns together (L2 reuse of B)
        const int G = 8;
        const int per_group = G * tiles_n;
        const int group = bid / per_group;
        const int first = group * G;
        const int gsz = min(tiles_m - first, G);
        const int r = bid - group * per_group;
        tm = first + r % gsz;
        tn = r / gsz;
    }
}

// ---- global -> registers ----------------------------------------------------
// A tile: BM rows x BK k, loaded V-wide along k.
template <int V> struct ATile {
    static constexpr int CH = BM * (BK / V);
    static constexpr int PER = (CH + NT - 1) / NT;
    float v[PER][V];
    __device__ __forceinline__ void load(const pk_gemm_args &a, int row0, int64_t k0, int tid) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int q = p * NT + tid;
            const int r = q / (BK / V);
            const int c = (q % (BK / V)) * V;
            const int64_t row = row0 + r;
            const int64_t k = k0 + c;
            if (q < CH && row < a.M && k + V <= a.K) {
                pk_ldv<V>(a.A + row * a.lda + k, v[p]);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e)
                    v[p][e] = (q < CH && row < a.M && k + e < a.K) ? a.A[row * a.lda + k + e] : 0.f;
            }
        }
    }
};

// B tile: BK k x BN columns, loaded V-wide along n, KB consecutive k rows per
// chunk.  Consecutive threads take consecutive k (then the next V columns), so
// the transposed LDS stores below hit consecutive banks.
constexpr int KB = (PREC == 0) ? 1 : 2;
template <int V> struct BTile {
    static constexpr int CH = (BK / KB) * (BN / V);
    static constexpr int PER = (CH + NT - 1) / NT;
    float v[PER][KB][V];
    __device__ __forceinline__ void load(const pk_gemm_args &a, int col0, int64_t k0, int tid) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int q = p * NT + tid;
            const int kk = (q % (BK / KB)) * KB;
            const int c = (q / (BK / KB)) * V;
            const int64_t col = col0 + c;
#pragma unroll
            for (int h = 0; h < KB; ++h) {
                const int64_t k = k0 + kk + h;
                if (q < CH && k < a.K && col + V <= a.N) {
                    pk_ldv<V>(a.B + k * a.ldb + col, v[p][h]);
                } else {
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        v[p][h][e] = (q < CH && k < a.K && col + e < a.N) ? a.B[k * a.ldb + col + e] : 0.f;
                }
            }
        }
    }
};

// ---- registers -> LDS ---------------------------------------------------------
template <int V>
__device__ __forceinline__ void store_a(const ATile<V> &t, lds_t *As, lds_t *As2, int tid) {
#pragma unroll
    for (int p = 0; p < ATile<V>::PER; ++p) {
        const int q = p * NT + tid;
        if (q >= ATile<V>::CH)
            break;
        const int r = q / (BK / V);
        const int c = (q % (BK / V)) * V;
#if PREC == 0
        pk_stv<V>(As + r * LDK + c, t.v[p]);
#else
#pragma unroll
        for (int e = 0; e < V; ++e) {
#if PREC == 1
            As[r * LDK + c + e] = (uint16_t)pk_bf16_bits(t.v[p][e]);
#else
            uint32_t hb, lb;
            pk_split(t.v[p][e], hb, lb);
            As[r * LDK + c + e] = (uint16_t)hb;
            As2[r * LDK + c + e] = (uint16_t)lb;
#endif
        }
#endif
    }
}

template <int V>
__device__ __forceinline__ void store_b(const BTile<V> &t, lds_t *Bs, lds_t *Bs2, int tid) {
#pragma unroll
    for (int p = 0; p < BTile<V>::PER; ++p) {
        const int q = p * NT + tid;
        if (q >= BTile<V>::CH)
            break;
        const int kk = (q % (BK / KB)) * KB;
        const int c = (q / (BK / KB)) * V;
#pragma unroll
        for (int e = 0; e < V; ++e) {
#if PREC == 0
            Bs[(c + e) * LDK + kk] = t.v[p][0][e];
#elif PREC == 1
            *reinterpret_cast<uint32_t *>(Bs + (c + e) * LDK + kk) = pk_pack_bf16(t.v[p][0][e], t.v[p][1][e]);
#else
            uint32_t h0, l0, h1, l1;
            pk_split(t.v[p][0][e], h0, l0);
            pk_split(t.v[p][1][e], h1, l1);
            *reinterpret_cast<uint32_t *>(Bs + (c + e) * LDK + kk) = h0 | (h1 << 16);
            *reinterpret_cast<uint32_t *>(Bs2 + (c + e) * LDK + kk) = l0 | (l1 << 16);
#endif
        }
    }
}

// ---- fragments + MFMA -----------------------------------------------------------
#if PREC == 0
typedef float frag_t;   // one k slot per MFMA
#else
typedef bf16x8 frag_t;  // eight k slots per MFMA
#endif
#if MF == 32
// 32x32 output block: lane l holds column l % 32, rows 8 (r / 4) + 4 (l / 32) + r % 4
typedef f32x16 acc_t;
constexpr int ACCN = 16;
#else
// 16x16 output block: lane l holds column l % 16, rows 4 (l / 16) + r
typedef f32x4 acc_t;
constexpr int ACCN = 4;
#endif

__device__ __forceinline__ acc_t mma(frag_t a, frag_t b, acc_t c) {
#if PREC == 0 && MF == 32
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
#elif PREC == 0
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
#else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
#endif
}

// read the STEPS fragments of one 16-row block from a k-contiguous LDS tile
__device__ __forceinline__ void read_frag(const lds_t *S, int row, int g, frag_t *f) {
#if PREC == 0
    const float *p = S + row * LDK + g * KG;
#pragma unroll
    for (int s = 0; s < STEPS; s += 4) {
        f32x4 v = *reinterpret_cast<const f32x4 *>(p + s);
        f[s] = v[0];
        f[s + 1] = v[1];
        f[s + 2] = v[2];
        f[s + 3] = v[3];
    }
#else
    const uint16_t *p = S + row * LDK + g * KG;
#pragma unroll
    for (int s = 0; s < STEPS; ++s)
        f[s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(p + s * 8));
#endif
}

// FC = 4: fragments for k slots s0 .. s0+3 of one block row (one 16-byte read)
__device__ __forceinline__ void read_frag4(const lds_t *S, int row, int g, int s0, frag_t *f) {
    const f32x4 v = *reinterpret_cast<const f32x4 *>(S + row * LDK + g * KG + s0);
    f[0] = v[0];
    f[1] = v[1];
    f[2] = v[2];
    f[3] = v[3];
}

// direct (no LDS) fragment loads from global memory
__device__ __forceinline__ void global_frag_a(const pk_gemm_args &a, int64_t row, int64_t kbase,
                                              frag_t *f, frag_t *f2) {
    float t[KG];
#if DK
    // the value is masked with an AND (a select would let the compiler move the load
    // under a branch on the condition, where each load waits for itself)
    const int64_t rc = min(row, a.M - 1);
#pragma unroll
    for (int e = 0; e < KG; ++e) {
        const float v = a.A[rc * a.lda + min(kbase + e, a.K - 1)];
        const uint32_t keep = 0u - (uint32_t)((row < a.M) & (kbase + e < a.K));
        t[e] = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) & keep);
    }
#else
#pragma unroll
    for (int e = 0; e < KG; ++e)
        t[e] = (row < a.M && kbase + e < a.K) ? a.A[row * a.lda + kbase + e] : 0.f;
#endif
#if PREC == 0
#pragma unroll
    for (int s = 0; s < STEPS; ++s)
        f[s] = t[s];
#else
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        u16x8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
#if PREC == 1
            h[e] = (uint16_t)pk_bf16_bits(t[s * 8 + e]);
#else
            uint32_t hb, lb;
            pk_split(t[s * 8 + e], hb, lb);
            h[e] = (uint16_t)hb;
            l[e] = (uint16_t)lb;
#endif
        }
        f[s] = __builtin_bit_cast(bf16x8, h);
#if PREC == 2
        f2[s] = __builtin_bit_cast(bf16x8, l);
#endif
    }
#endif
}

__device__ __forceinline__ void global_frag_b(const pk_gemm_args &a, int64_t col, int64_t kbase,
                                              frag_t *f, frag_t *f2) {
    float t[KG];
#if DK
    const int64_t cc = min(col, a.N - 1);
#pragma unroll
    for (int e = 0; e < KG; ++e) {
        const float v = a.B[min(kbase + e, a.K - 1) * a.ldb + cc];
        const uint32_t keep = 0u - (uint32_t)((col < a.N) & (kbase + e < a.K));
        t[e] = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) & keep);
    }
#else
#pragma unroll
    for (int e = 0; e < KG; ++e)
        t[e] = (col < a.N && kbase + e < a.K) ? a.B[(kbase + e) * a.ldb + col] : 0.f;
#endif
#if PREC == 0
#pragma unroll
    for (int s = 0; s < STEPS; ++s)
        f[s] = t[s];
#else
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        u16x8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
#if PREC == 1
            h[e] = (uint16_t)pk_bf16_bits(t[s * 8 + e]);
#else
            uint32_t hb, lb;
            pk_split(t[s * 8 + e], hb, lb);
            h[e] = (uint16_t)hb;
            l[e] = (uint16_t)lb;
#endif
        }
        f[s] = __builtin_bit_cast(bf16x8, h);
#if PREC == 2
        f2[s] = __builtin_bit_cast(bf16x8, l);
#endif
    }
#endif
}

#if IL
// The k loop of a full interior tile (rows 16-byte aligned, K a multiple of BK, at least
// two k tiles): no bounds checks, so one iteration is one basic block, and the
// scheduling-group barriers below lay it out as: the tile's fragment reads, then its
// MFMAs with the next tile's LDS stores (from registers) and the following tile's global
// loads (into the same registers, after their stores) interleaved among them, then the
// barrier.  The last iterations store into the idle stage and re-load the last tile
// (clamped), which nothing reads.
constexpr int IL_PA = BM * (BK / 4) / NT;        // A chunks (16 bytes) per thread
constexpr int IL_PB = BK * (BN / 4) / NT;        // B chunks per thread
static_assert(IL == 0 || (BM * (BK / 4) % NT == 0 && BK * (BN / 4) % NT == 0), "IL: chunks must divide evenly");
constexpr int IL_DSR = (FM + FN) * (STEPS / 4);  // 16-byte fragment reads per k tile
constexpr int IL_MMA = STEPS * FM * FN;          // MFMAs per k tile
constexpr int IL_DSW = IL_PA + 4 * IL_PB;        // LDS stores per k tile (B is transposed, 4 each)
constexpr int IL_VMR = IL_PA + IL_PB;            // global loads per k tile
constexpr int IL_MW = IL_MMA / (2 * IL_DSW) > 0 ? IL_MMA / (2 * IL_DSW) : 1;   // MFMAs before each store
constexpr int IL_MV = IL_MMA / (4 * IL_VMR) > 0 ? IL_MMA / (4 * IL_VMR) : 1;   // ... before each load
constexpr int IL_REST = IL_MMA - IL_DSW * IL_MW - IL_VMR * IL_MV;

__device__ __forceinline__ void il_load(const pk_gemm_args &a, int row0, int col0, int64_t k0, int tid,
                                        f32x4 *ra, f32x4 *rb) {
#if IL == 2
    // K a multiple of 4, the last k tile partial: a chunk past K reads the last one in
    // the row (A) or the last row (B) and is masked to zeros with an AND (no branch)
#pragma unroll
    for (int p = 0; p < IL_PA; ++p) {
        const int q = p * NT + tid;
        const int64_t k = k0 + (q % (BK / 4)) * 4;
        const f32x4 v = *reinterpret_cast<const f32x4 *>(a.A + (int64_t)(row0 + q / (BK / 4)) * a.lda + min(k, a.K - 4));
        ra[p] = __builtin_bit_cast(f32x4, __builtin_bit_cast(u32x4, v) & (0u - (uint32_t)(k < a.K)));
    }
#pragma unroll
    for (int p = 0; p < IL_PB; ++p) {
        const int q = p * NT + tid;
        const int64_t k = k0 + q % BK;
        const f32x4 v = *reinterpret_cast<const f32x4 *>(a.B + min(k, a.K - 1) * a.ldb + col0 + (q / BK) * 4);
        rb[p] = __builtin_bit_cast(f32x4, __builtin_bit_cast(u32x4, v) & (0u - (uint32_t)(k < a.K)));
    }
#else
#pragma unroll
    for (int p = 0; p < IL_PA; ++p) {
        const int q = p * NT + tid;
        ra[p] = *reinterpret_cast<const f32x4 *>(a.A + (int64_t)(row0 + q / (BK / 4)) * a.lda + k0 + (q % (BK / 4)) * 4);
    }
#pragma unroll
    for (int p = 0; p < IL_PB; ++p) {
        const int q = p * NT + tid;
        rb[p] = *reinterpret_cast<const f32x4 *>(a.B + (k0 + q % BK) * a.ldb + col0 + (q / BK) * 4);
    }
#endif
}

__device__ __forceinline__ void il_store(float *As, float *Bs, int tid, const f32x4 *ra, const f32x4 *rb) {
#pragma unroll
    for (int p = 0; p < IL_PA; ++p) {
        const int q = p * NT + tid;
        *reinterpret_cast<f32x4 *>(As + (q / (BK / 4)) * LDK + (q % (BK / 4)) * 4) = ra[p];
    }
#pragma unroll
    for (int p = 0; p < IL_PB; ++p) {
        const int q = p * NT + tid;
        const int kk = q % BK, c = (q / BK) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            Bs[(c + e) * LDK + kk] = rb[p][e];
    }
}

__device__ __forceinline__ void il_main(const pk_gemm_args &a, float *lds, int row0, int col0, int tid, int wm,
                                        int wn, int g, int lr, acc_t (&acc)[FM][FN]) {
    constexpr int STAGE = (BM + BN) * LDK;
#if IL == 2
    const int64_t nk = (a.K + BK - 1) / BK;
#else
    const int64_t nk = a.K / BK;
#endif
    f32x4 ra[IL_PA], rb[IL_PB];
    il_load(a, row0, col0, 0, tid, ra, rb);
    il_store(lds, lds + BM * LDK, tid, ra, rb);
    il_load(a, row0, col0, BK, tid, ra, rb);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const float *As = lds + cur * STAGE, *Bs = lds + cur * STAGE + BM * LDK;
        float *An = lds + (cur ^ 1) * STAGE, *Bn = lds + (cur ^ 1) * STAGE + BM * LDK;
        frag_t fa[FM][STEPS], fb[FN][STEPS];
#pragma unroll
        for (int i = 0; i < FM; ++i)
            read_frag(As, wm * WTM + i * BLK + lr, g, fa[i]);
#pragma unroll
        for (int j = 0; j < FN; ++j)
            read_frag(Bs, wn * WTN + j * BLK + lr, g, fb[j]);
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = mma(fa[i][s], fb[j][s], acc[i][j]);
        il_store(An, Bn, tid, ra, rb);                              // tile kt+1
        il_load(a, row0, col0, min(kt + 2, nk - 1) * BK, tid, ra, rb);  // tile kt+2
        __builtin_amdgcn_sched_group_barrier(0x100, IL_DSR, 0);    // the fragment reads
#pragma unroll
        for (int w = 0; w < IL_DSW; ++w) {
            __builtin_amdgcn_sched_group_barrier(0x008, IL_MW, 0); // MFMAs, then one LDS store
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
        }
#pragma unroll
        for (int v = 0; v < IL_VMR; ++v) {
            __builtin_amdgcn_sched_group_barrier(0x008, IL_MV, 0); // MFMAs, then one global load
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, IL_REST, 0);
        __syncthreads();
    }
}
#endif

#if DK
// one group of UNROLL k tiles starting at k0, read straight from memory into fragments
// (rows r0 + i*BLK of A, columns c0 + j*BLK of B for this lane), then the MFMAs
template <bool INK>
__device__ __forceinline__ void dk_group(const pk_gemm_args &a, int64_t k0, int64_t r0, int64_t c0, int g,
                                         acc_t (&acc)[FM][FN]) {
    constexpr int NLD = UNROLL * (FM + FN) * KG;     // loads of the group
    float ta[UNROLL][FM][KG], tb[UNROLL][FN][KG];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int64_t r = r0 + i * BLK;
        const float *pa = a.A + min(r, a.M - 1) * a.lda;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int e = 0; e < KG; ++e) {
                const int64_t k = k0 + u * BK + g * KG + e;
                ta[u][i][e] = pa[INK ? k : min(k, a.K - 1)];
            }
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int64_t c = min(c0 + j * BLK, a.N - 1);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int e = 0; e < KG; ++e) {
                const int64_t k = k0 + u * BK + g * KG + e;
                tb[u][j][e] = a.B[(INK ? k : min(k, a.K - 1)) * a.ldb + c];
            }
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u)
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    // masks by AND: a select on a loaded value can be turned into a
                    // branch around the load, where each load waits for itself
                    const int64_t k = k0 + u * BK + g * KG + s;
                    const uint32_t kin = INK ? 1u : (uint32_t)(k < a.K);
                    const uint32_t mx = 0u - (kin & (uint32_t)(r0 + i * BLK < a.M));
                    const uint32_t my = 0u - (kin & (uint32_t)(c0 + j * BLK < a.N));
                    const float x = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, ta[u][i][s]) & mx);
                    const float y = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, tb[u][j][s]) & my);
                    acc[i][j] = mma(x, y, acc[i][j]);
                }
    // the groups take their members from the code above: all of the loads, then the MFMAs
    __builtin_amdgcn_sched_group_barrier(0x020, NLD, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, UNROLL * STEPS * FM * FN, 0);
}
#endif

template <int V>
__device__ __forceinline__ void gemm_body(const pk_gemm_args &a, lds_t *lds) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WAVES_N;
    const int wn = wave % WAVES_N;
#if MF == 32
    const int g = lane >> 5;                   // lane group: its k slot of each MFMA
    const int lr = lane & 31;                  // row / column of the lane within a block
#else
    const int g = lane >> 4;
    const int lr = lane & 15;
#endif

    const int tiles_m = (int)((a.M + BM - 1) / BM);
    const int tiles_n = (int)((a.N + BN - 1) / BN);
    int tm, tn;
    tile_of(blockIdx.x, tiles_m, tiles_n, tm, tn);
    if (tm >= tiles_m || tn >= tiles_n)
        return;
    const int row0 = tm * BM;
    const int col0 = tn * BN;

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#if MF == 32
            acc[i][j] = f32x16{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#else
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#endif

    const int64_t nk = (a.K + BK - 1) / BK;

#if IL
#if IL == 2
    if (row0 + BM <= a.M && col0 + BN <= a.N && a.K % 4 == 0 && nk >= 2 && a.aligned && V == 4) {
#else
    if (row0 + BM <= a.M && col0 + BN <= a.N && a.K % BK == 0 && nk >= 2 && a.aligned && V == 4) {
#endif
        il_main(a, lds, row0, col0, tid, wm, wn, g, lr, acc);
    } else {
#endif
#if USE_LDS == 2
    // two LDS stages: tile kt+1 is written to the other stage while tile kt is
    // read (its last readers finished before the previous barrier), and the
    // global loads for tile kt+2 are in flight meanwhile; one barrier per step
    constexpr int STAGE = NSPLIT * (BM + BN) * LDK;
    auto As_ = [&](int st) { return lds + st * STAGE; };
    auto Bs_ = [&](int st) { return lds + st * STAGE + BM * LDK; };
    auto As2_ = [&](int st) { return lds + st * STAGE + (BM + BN) * LDK; };
    auto Bs2_ = [&](int st) { return lds + st * STAGE + (BM + BN) * LDK + BM * LDK; };
    ATile<V> ta;
    BTile<V> tb;
    ta.load(a, row0, 0, tid);
    tb.load(a, col0, 0, tid);
    store_a<V>(ta, As_(0), As2_(0), tid);
    store_b<V>(tb, Bs_(0), Bs2_(0), tid);
    if (nk > 1) {
        ta.load(a, row0, BK, tid);
        tb.load(a, col0, BK, tid);
    }
    __syncthreads();
#pragma unroll UNROLL
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
#if FC
#pragma unroll
        for (int s0 = 0; s0 < STEPS; s0 += FC) {
            frag_t fa[FM][FC], fb[FN][FC];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                read_frag4(As_(cur), wm * WTM + i * BLK + lr, g, s0, fa[i]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                read_frag4(Bs_(cur), wn * WTN + j * BLK + lr, g, s0, fb[j]);
#pragma unroll
            for (int s = 0; s < FC; ++s)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = mma(fa[i][s], fb[j][s], acc[i][j]);
            // keep the next chunk's fragment reads after these MFMAs are issued, so a
            // deep k-step holds one chunk of fragments at a time
            __builtin_amdgcn_sched_barrier(0);
        }
#else
        frag_t fa[FM][STEPS], fb[FN][STEPS];
#if PREC == 2
        frag_t fa2[FM][STEPS], fb2[FN][STEPS];
#endif
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            read_frag(As_(cur), wm * WTM + i * BLK + lr, g, fa[i]);
#if PREC == 2
            read_frag(As2_(cur), wm * WTM + i * BLK + lr, g, fa2[i]);
#endif
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            read_frag(Bs_(cur), wn * WTN + j * BLK + lr, g, fb[j]);
#if PREC == 2
            read_frag(Bs2_(cur), wn * WTN + j * BLK + lr, g, fb2[j]);
#endif
        }
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
#if PREC == 2
                    acc[i][j] = mma(fa2[i][s], fb[j][s], acc[i][j]);
                    acc[i][j] = mma(fa[i][s], fb2[j][s], acc[i][j]);
#endif
                    acc[i][j] = mma(fa[i][s], fb[j][s], acc[i][j]);
                }
#endif
        if (kt + 1 < nk) {
            store_a<V>(ta, As_(cur ^ 1), As2_(cur ^ 1), tid);
            store_b<V>(tb, Bs_(cur ^ 1), Bs2_(cur ^ 1), tid);
            if (kt + 2 < nk) {
                ta.load(a, row0, (kt + 2) * BK, tid);
                tb.load(a, col0, (kt + 2) * BK, tid);
            }
        }
        __syncthreads();
    }
#elif USE_LDS
    lds_t *As = lds;
    lds_t *Bs = lds + BM * LDK;
    lds_t *As2 = lds + (BM + BN) * LDK;   // lo parts (split only)
    lds_t *Bs2 = As2 + BM * LDK;

    ATile<V> ta;
    BTile<V> tb;
    ta.load(a, row0, 0, tid);
    tb.load(a, col0, 0, tid);
#pragma unroll UNROLL
    for (int64_t kt = 0; kt < nk; ++kt) {
        store_a<V>(ta, As, As2, tid);
        store_b<V>(tb, Bs, Bs2, tid);
        __syncthreads();
        if (kt + 1 < nk) {   // next tile's loads overlap this tile's MFMAs
            ta.load(a, row0, (kt + 1) * BK, tid);
            tb.load(a, col0, (kt + 1) * BK, tid);
        }
#if FC
#pragma unroll
        for (int s0 = 0; s0 < STEPS; s0 += FC) {
            frag_t fa[FM][FC], fb[FN][FC];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                read_frag4(As, wm * WTM + i * BLK + lr, g, s0, fa[i]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                read_frag4(Bs, wn * WTN + j * BLK + lr, g, s0, fb[j]);
#pragma unroll
            for (int s = 0; s < FC; ++s)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = mma(fa[i][s], fb[j][s], acc[i][j]);
            // keep the next chunk's fragment reads after these MFMAs are issued, so a
            // deep k-step holds one chunk of fragments at a time
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
    }
#else
        frag_t fa[FM][STEPS], fb[FN][STEPS];
#if PREC == 2
        frag_t fa2[FM][STEPS], fb2[FN][STEPS];
#endif
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            read_frag(As, wm * WTM + i * BLK + lr, g, fa[i]);
#if PREC == 2
            read_frag(As2, wm * WTM + i * BLK + lr, g, fa2[i]);
#endif
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            read_frag(Bs, wn * WTN + j * BLK + lr, g, fb[j]);
#if PREC == 2
            read_frag(Bs2, wn * WTN + j * BLK + lr, g, fb2[j]);
#endif
        }
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
#if PREC == 2
                    acc[i][j] = mma(fa2[i][s], fb[j][s], acc[i][j]);
                    acc[i][j] = mma(fa[i][s], fb2[j][s], acc[i][j]);
#endif
                    acc[i][j] = mma(fa[i][s], fb[j][s], acc[i][j]);
                }
        __syncthreads();
    }
#endif
#else
#if DK
    // k tiles in groups of UNROLL: every fragment of a group is loaded into registers
    // first (a scheduling-group barrier keeps all those loads ahead of the rest, in
    // flight together), then the group's MFMAs run.  A group inside K reads its rows
    // and columns at constant offsets; the last group, if it reaches past K, reads
    // clamped addresses masked to zero in both operands (exact zeros).
    for (int64_t ku = 0; ku < (nk + UNROLL - 1) / UNROLL; ++ku) {
        if ((ku + 1) * UNROLL * BK <= a.K)
            dk_group<true>(a, ku * UNROLL * BK, row0 + wm * WTM + lr, col0 + wn * WTN + lr, g, acc);
        else
            dk_group<false>(a, ku * UNROLL * BK, row0 + wm * WTM + lr, col0 + wn * WTN + lr, g, acc);
    }
#else
#pragma unroll UNROLL
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int64_t kbase = kt * BK + g * KG;
        frag_t fa[FM][STEPS], fb[FN][STEPS];
        frag_t fa2[FM][STEPS], fb2[FN][STEPS];
#pragma unroll
        for (int i = 0; i < FM; ++i)
            global_frag_a(a, row0 + wm * WTM + i * BLK + lr, kbase, fa[i], fa2[i]);
#pragma unroll
        for (int j = 0; j < FN; ++j)
            global_frag_b(a, col0 + wn * WTN + j * BLK + lr, kbase, fb[j], fb2[j]);
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
#if PREC == 2
                    acc[i][j] = mma(fa2[i][s], fb[j][s], acc[i][j]);
                    acc[i][j] = mma(fa[i][s], fb2[j][s], acc[i][j]);
#endif
                    acc[i][j] = mma(fa[i][s], fb[j][s], acc[i][j]);
                }
    }
#endif
    (void)V;
#endif
#if IL
    }
#endif

    // epilogue: one store per output element
    const bool use_c = a.beta != 0.f;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t col = col0 + wn * WTN + j * BLK + lr;
#pragma unroll
            for (int r = 0; r < ACCN; ++r) {
#if MF == 32
                const int64_t row = row0 + wm * WTM + i * 32 + 8 * (r / 4) + 4 * g + (r % 4);
#else
                const int64_t row = row0 + wm * WTM + i * 16 + 4 * g + r;
#endif
                if (row < a.M && col < a.N) {
                    float v = a.alpha * acc[i][j][r];
                    if (use_c)
                        v += a.beta * a.C[row * a.ldc + col];
                    a.D[row * a.ldd + col] = v;
                }
            }
        }
}

extern "C" __global__ void __launch_bounds__(NT) pk_gemm(pk_gemm_args a) {
    if (blockDim.x != NT)
        return;
#if USE_LDS
    __shared__ __attribute__((aligned(16))) lds_t lds[LDS_STAGES * NSPLIT * (BM + BN) * LDK];
#else
    lds_t *lds = nullptr;
#endif
    if (VEC > 1 && a.aligned)
        gemm_body<VEC>(a, lds);
    else
        gemm_body<1>(a, lds);
}
