// conv.hip -- 3x3 (2DCONV) and 3x3x3 (3DCONV) stencils, Sec. 2.2.
//
//   out[i][j]    = sum_{di,dj}    w[(di+1)*3+(dj+1)]          * in[i+di][j+dj]
//   out[z][y][x] = sum_{dz,dy,dx} w[(dz+1)*9+(dy+1)*3+(dx+1)] * in[z+dz][y+dy][x+dx]
// on the interior (no flip); every border cell is written as 0.
//
// Both are bound by one read of the input and one write of the output
// (Sec. 3.4 finds 3DCONV dominated by its global loads).  Each thread owns
// VEC adjacent outputs along x and marches along y (2D) or z (3D) keeping a
// sliding window of input rows/planes in registers, so each input row is
// fetched from memory by one thread column and reused from registers.  The
// 2D kernel can instead stage a haloed tile in LDS (USE_LDS=1).
#include "pk_device.h"

#ifndef CONV_KIND
#define CONV_KIND 2
#endif
#ifndef VEC
#define VEC 4
#endif
#ifndef TX          // threads along x
#define TX 64
#endif
#ifndef TY          // threads along y
#define TY 4
#endif
#ifndef ROWS        // outputs per thread along the marching axis (y for 2D, z for 3D)
#define ROWS ((CONV_KIND) == 2 ? 8 : 16)
#endif
#ifndef UNROLL
#define UNROLL 1
#endif
#ifndef USE_LDS
#define USE_LDS 0
#endif
#ifndef ORDER       // 0: x tiles fastest, 1: y tiles fastest, 2: x fastest, XCD-contiguous
#define ORDER 0
#endif
#ifndef NTL         // 1: the input's row segments are read with the non-temporal hint
#define NTL 0
#endif
#if NTL
#define PK_LDM pk_ldv_nt
#else
#define PK_LDM pk_ldv
#endif

constexpr int NT = TX * TY;
static_assert(NT % 64 == 0, "block must be whole wavefronts");
constexpr int BX = TX * VEC;

// ORDER 2: blocks are dealt to the 8 XCDs in turn; give each XCD a contiguous
// range of tiles (a bijection on [0, nb)) so neighbouring tiles, which share
// halo rows, meet in the same L2.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t nb) {
    const int64_t q = nb / 8, rem = nb % 8, x = b % 8;
    return x * q + min(x, rem) + b / 8;
}

#if CONV_KIND == 2
constexpr int BY = TY * ROWS;
constexpr int LDS_BYTES = USE_LDS ? (BY + 2) * (BX + 4) * 4 : 0;
PK_DEFINE_KNOBS(PKF_CONV2D, BY, BX, ROWS, TY, TX, VEC, UNROLL, USE_LDS, ORDER, 0, 0, NT,
                LDS_BYTES, PK_KERNEL_ABI_VERSION, 0)

// one input row segment [x0-1, x0+V] of row y (zeros outside the grid)
template <int V>
__device__ __forceinline__ void load_seg(const pk_conv2d_args &a, int64_t y, int64_t x0, float *s) {
    if (y < 0 || y >= a.H) {
#pragma unroll
        for (int e = 0; e < VEC + 2; ++e)
            s[e] = 0.f;
        return;
    }
    const float *row = a.in + y * a.ldi;
    s[0] = (x0 - 1 >= 0 && x0 - 1 < a.W) ? row[x0 - 1] : 0.f;
    if (x0 + VEC <= a.W) {
#pragma unroll
        for (int e = 0; e < VEC; e += V)
            PK_LDM<V>(row + x0 + e, s + 1 + e);
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            s[1 + e] = (x0 + e < a.W) ? row[x0 + e] : 0.f;
    }
    s[VEC + 1] = (x0 + VEC < a.W) ? row[x0 + VEC] : 0.f;
}

template <int V>
__device__ __forceinline__ void store_seg(const pk_conv2d_args &a, int64_t y, int64_t x0, float *o) {
    float *row = a.out + y * a.ldo;
    if (x0 + VEC <= a.W) {
#pragma unroll
        for (int e = 0; e < VEC; e += V)
            pk_stv<V>(row + x0 + e, o + e);
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (x0 + e < a.W)
                row[x0 + e] = o[e];
    }
}

template <int V>
__device__ __forceinline__ void conv2d_body(const pk_conv2d_args &a, float *tile) {
    constexpr int BXV = TX * VEC;
    const int tx = threadIdx.x % TX;
    const int ty = threadIdx.x / TX;
    const int64_t nbx = (a.W + BXV - 1) / BXV;
    const int64_t nby = (a.H + BY - 1) / BY;
    int64_t bx, by;
    if (ORDER == 2) {
        const int64_t L = xcd_contiguous(blockIdx.x, nbx * nby);
        bx = L % nbx;
        by = L / nbx;
    } else if (ORDER == 0) {
        bx = blockIdx.x % nbx;
        by = blockIdx.x / nbx;
    } else {
        by = blockIdx.x % nby;
        bx = blockIdx.x / nby;
    }
    if (by >= nby)
        return;
    const int64_t x0 = bx * BXV + (int64_t)tx * VEC;
    const int64_t y0 = by * BY + (int64_t)ty * ROWS;
    float w[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
        w[t] = a.w[t];

#if USE_LDS
    constexpr int LW = TX * VEC + 4;   // staged columns: [bx*BXV - 1, bx*BXV + BXV + 1) padded
    {
        const int64_t gx0 = bx * BXV - 1;
        const int64_t gy0 = by * BY - 1;
        for (int idx = threadIdx.x; idx < (BY + 2) * (BXV + 2); idx += NT) {
            const int ry = idx / (BXV + 2);
            const int rx = idx % (BXV + 2);
            const int64_t gy = gy0 + ry, gx = gx0 + rx;
            tile[ry * LW + rx] = (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) ? a.in[gy * a.ldi + gx] : 0.f;
        }
        __syncthreads();
    }
#endif
    if (x0 >= a.W)
        return;

#if USE_LDS
#pragma unroll UNROLL
    for (int r = 0; r < ROWS; ++r) {
        const int64_t y = y0 + r;
        if (y >= a.H)
            break;
        const int ly = ty * ROWS + r + 1;   // tile row of y
        const int lx = tx * VEC + 1;        // tile column of x0
        float o[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            float acc = 0.f;
#pragma unroll
            for (int di = -1; di <= 1; ++di)
#pragma unroll
                for (int dj = -1; dj <= 1; ++dj)
                    acc += w[(di + 1) * 3 + (dj + 1)] * tile[(ly + di) * LW + lx + e + dj];
            const int64_t x = x0 + e;
            o[e] = (y == 0 || y == a.H - 1 || x == 0 || x >= a.W - 1) ? 0.f : acc;
        }
        store_seg<V>(a, y, x0, o);
    }
#else
    float s0[VEC + 2], s1[VEC + 2], s2[VEC + 2];
    load_seg<V>(a, y0 - 1, x0, s0);
    load_seg<V>(a, y0, x0, s1);
    load_seg<V>(a, y0 + 1, x0, s2);
#pragma unroll UNROLL
    for (int r = 0; r < ROWS; ++r) {
        const int64_t y = y0 + r;
        if (y >= a.H)
            break;
        float o[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            float acc = w[0] * s0[e] + w[1] * s0[e + 1] + w[2] * s0[e + 2];
            acc += w[3] * s1[e] + w[4] * s1[e + 1] + w[5] * s1[e + 2];
            acc += w[6] * s2[e] + w[7] * s2[e + 1] + w[8] * s2[e + 2];
            const int64_t x = x0 + e;
            o[e] = (y == 0 || y == a.H - 1 || x == 0 || x >= a.W - 1) ? 0.f : acc;
        }
        store_seg<V>(a, y, x0, o);
        if (r + 1 < ROWS) {
#pragma unroll
            for (int e = 0; e < VEC + 2; ++e) {
                s0[e] = s1[e];
                s1[e] = s2[e];
            }
            load_seg<V>(a, y + 2, x0, s2);
        }
    }
#endif
}

extern "C" __global__ void __launch_bounds__(NT) pk_conv2d(pk_conv2d_args a) {
    if (blockDim.x != NT)
        return;
#if USE_LDS
    __shared__ __attribute__((aligned(16))) float tile[(BY + 2) * (TX * VEC + 4)];
#else
    float *tile = nullptr;
#endif
    if (VEC > 1 && a.aligned)
        conv2d_body<VEC>(a, tile);
    else
        conv2d_body<1>(a, tile);
}

#else   // ------------------------------------------------------------- 3D --

#if USE_LDS == 2
// Staged variant: a block owns BX columns x BYT = TY*YR rows and marches ROWS
// planes along z.  Each plane's haloed (BYT+2) x (BX+2) tile is fetched with
// 16-byte loads into registers one plane ahead and written to a ring of four
// LDS slots, so every input element is read from memory once per block and the
// y halo costs 2/BYT.  A thread computes a VEC x YR patch of outputs.
#ifndef YR
#define YR 4
#endif
#ifndef PF          // planes fetched ahead into registers: 1, or 2 (two register tiles in turn)
#define PF 1
#endif
static_assert(PF == 1 || PF == 2, "PF must be 1 or 2");
constexpr int BYT = TY * YR;
constexpr int LW4 = BX + 8;                 // tile row: halo at 3, interior at 4 .. BX+3, halo at BX+4
constexpr int LP4 = (BYT + 2) * LW4;
// knob slot X2 records PF when it is not 1
PK_DEFINE_KNOBS(PKF_CONV3D, BYT, BX, ROWS, TY, TX, VEC, UNROLL, 2, ORDER, YR, (PF == 1 ? 0 : PF), NT, 4 * LP4 * 4,
                PK_KERNEL_ABI_VERSION, 0)
#else
// LDS variant: a ring of three haloed (TY+2) x (BX+2) plane tiles
constexpr int LW3 = TX * VEC + 4;
constexpr int LP3 = (TY + 2) * LW3;
constexpr int LDS3_BYTES = USE_LDS ? 3 * LP3 * 4 : 0;
PK_DEFINE_KNOBS(PKF_CONV3D, TY, BX, ROWS, TY, TX, VEC, UNROLL, USE_LDS, ORDER, 0, 0, NT, LDS3_BYTES,
                PK_KERNEL_ABI_VERSION, 0)
#endif

// rows y-1, y, y+1 of plane z, columns [x0-1, x0+V] (zeros outside the volume)
template <int V>
__device__ __forceinline__ void load_plane(const pk_conv3d_args &a, int64_t z, int64_t y, int64_t x0,
                                           float (*p)[VEC + 2]) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
        const int64_t yy = y - 1 + dy;
        if (z < 0 || z >= a.D || yy < 0 || yy >= a.H) {
#pragma unroll
            for (int e = 0; e < VEC + 2; ++e)
                p[dy][e] = 0.f;
            continue;
        }
        const float *row = a.in + (z * a.H + yy) * a.W;
        p[dy][0] = (x0 >= 1) ? row[x0 - 1] : 0.f;
        if (x0 + VEC <= a.W) {
#pragma unroll
            for (int e = 0; e < VEC; e += V)
                PK_LDM<V>(row + x0 + e, p[dy] + 1 + e);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                p[dy][1 + e] = (x0 + e < a.W) ? row[x0 + e] : 0.f;
        }
        p[dy][VEC + 1] = (x0 + VEC < a.W) ? row[x0 + VEC] : 0.f;
    }
}

template <int V>
__device__ __forceinline__ void conv3d_body(const pk_conv3d_args &a) {
    constexpr int BXV = TX * VEC;
    const int tx = threadIdx.x % TX;
    const int ty = threadIdx.x / TX;
    const int64_t nbx = (a.W + BXV - 1) / BXV;
    const int64_t nby = (a.H + TY - 1) / TY;
    const int64_t nbz = (a.D + ROWS - 1) / ROWS;
    int64_t b = blockIdx.x, bx, by, bz;
    if (ORDER == 2)
        b = xcd_contiguous(b, nbx * nby * nbz);
    if (ORDER == 0 || ORDER == 2) {
        bx = b % nbx; b /= nbx;
        by = b % nby; bz = b / nby;
    } else {
        by = b % nby; b /= nby;
        bx = b % nbx; bz = b / nbx;
    }
    if (bz >= nbz)
        return;
    const int64_t x0 = bx * BXV + (int64_t)tx * VEC;
    const int64_t y = by * TY + ty;
    const int64_t z0 = bz * ROWS;
    if (x0 >= a.W || y >= a.H)
        return;
    float w[27];
#pragma unroll
    for (int t = 0; t < 27; ++t)
        w[t] = a.w[t];
    float p0[3][VEC + 2], p1[3][VEC + 2], p2[3][VEC + 2];
    load_plane<V>(a, z0 - 1, y, x0, p0);
    load_plane<V>(a, z0, y, x0, p1);
    load_plane<V>(a, z0 + 1, y, x0, p2);
    const bool yborder = (y == 0 || y == a.H - 1);
#pragma unroll UNROLL
    for (int r = 0; r < ROWS; ++r) {
        const int64_t z = z0 + r;
        if (z >= a.D)
            break;
        float o[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            float acc = 0.f;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    acc += w[0 * 9 + dy * 3 + dx] * p0[dy][e + dx];
                    acc += w[1 * 9 + dy * 3 + dx] * p1[dy][e + dx];
                    acc += w[2 * 9 + dy * 3 + dx] * p2[dy][e + dx];
                }
            const int64_t x = x0 + e;
            o[e] = (yborder || z == 0 || z == a.D - 1 || x == 0 || x >= a.W - 1) ? 0.f : acc;
        }
        float *orow = a.out + (z * a.H + y) * a.W;
        if (x0 + VEC <= a.W) {
#pragma unroll
            for (int e = 0; e < VEC; e += V)
                pk_stv<V>(orow + x0 + e, o + e);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (x0 + e < a.W)
                    orow[x0 + e] = o[e];
        }
        if (r + 1 < ROWS) {
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int e = 0; e < VEC + 2; ++e) {
                    p0[dy][e] = p1[dy][e];
                    p1[dy][e] = p2[dy][e];
                }
            load_plane<V>(a, z + 2, y, x0, p2);
        }
    }
}

#if USE_LDS == 1
// 2.5D blocking: the block marches along z keeping planes z-1, z, z+1 of its
// haloed (x, y) tile in an LDS ring; each input plane tile is read from memory
// once per block and every thread takes its 27 taps from LDS.
template <int V>
__device__ __forceinline__ void load_tile3(const pk_conv3d_args &a, int64_t z, int64_t gy0, int64_t gx0,
                                           float *t) {
    constexpr int TW = TX * VEC + 2;           // tile columns: x in [gx0, gx0 + TW)
    for (int idx = threadIdx.x; idx < (TY + 2) * TW; idx += NT) {
        const int ry = idx / TW, rx = idx % TW;
        const int64_t gy = gy0 + ry, gx = gx0 + rx;
        t[ry * LW3 + rx] = (z >= 0 && z < a.D && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
                               ? a.in[(z * a.H + gy) * a.W + gx] : 0.f;
    }
}

template <int V>
__device__ __forceinline__ void conv3d_lds_body(const pk_conv3d_args &a, float *ring) {
    constexpr int BXV = TX * VEC;
    const int tx = threadIdx.x % TX;
    const int ty = threadIdx.x / TX;
    const int64_t nbx = (a.W + BXV - 1) / BXV;
    const int64_t nby = (a.H + TY - 1) / TY;
    const int64_t nbz = (a.D + ROWS - 1) / ROWS;
    int64_t b = blockIdx.x, bx, by, bz;
    if (ORDER == 2)
        b = xcd_contiguous(b, nbx * nby * nbz);
    if (ORDER == 0 || ORDER == 2) {
        bx = b % nbx; b /= nbx;
        by = b % nby; bz = b / nby;
    } else {
        by = b % nby; b /= nby;
        bx = b % nbx; bz = b / nbx;
    }
    if (bz >= nbz)
        return;
    const int64_t gx0 = bx * BXV - 1, gy0 = by * TY - 1;
    const int64_t x0 = bx * BXV + (int64_t)tx * VEC;
    const int64_t y = by * TY + ty;
    const int64_t z0 = bz * ROWS;
    float w[27];
#pragma unroll
    for (int t = 0; t < 27; ++t)
        w[t] = a.w[t];
    load_tile3<V>(a, z0 - 1, gy0, gx0, ring);
    load_tile3<V>(a, z0, gy0, gx0, ring + LP3);
    const bool active = x0 < a.W && y < a.H;
    const bool yborder = (y == 0 || y == a.H - 1);
    for (int r = 0; r < ROWS; ++r) {
        const int64_t z = z0 + r;
        if (z >= a.D)
            break;                                         // uniform across the block
        load_tile3<V>(a, z + 1, gy0, gx0, ring + ((r + 2) % 3) * LP3);
        __syncthreads();
        const float *pm = ring + (r % 3) * LP3, *pc = ring + ((r + 1) % 3) * LP3, *pp = ring + ((r + 2) % 3) * LP3;
        if (active) {
            float o[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                float acc = 0.f;
#pragma unroll
                for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        const int off = (ty + dy) * LW3 + tx * VEC + e + dx;
                        acc += w[0 * 9 + dy * 3 + dx] * pm[off];
                        acc += w[1 * 9 + dy * 3 + dx] * pc[off];
                        acc += w[2 * 9 + dy * 3 + dx] * pp[off];
                    }
                const int64_t x = x0 + e;
                o[e] = (yborder || z == 0 || z == a.D - 1 || x == 0 || x >= a.W - 1) ? 0.f : acc;
            }
            float *orow = a.out + (z * a.H + y) * a.W;
            if (x0 + VEC <= a.W) {
#pragma unroll
                for (int e = 0; e < VEC; e += V)
                    pk_stv<V>(orow + x0 + e, o + e);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (x0 + e < a.W)
                        orow[x0 + e] = o[e];
            }
        }
        __syncthreads();                                   // the oldest plane's slot is reloaded next
    }
}
#endif

#if USE_LDS == 2
// one plane's haloed tile in registers: CV-float chunks of the interior, then
// the left and right halo columns
template <int CV> struct PlaneTile {
    static constexpr int NV = (BYT + 2) * (BX / CV);
    static constexpr int PERV = (NV + NT - 1) / NT;
    static constexpr int NH = 2 * (BYT + 2);
    static constexpr int PERH = (NH + NT - 1) / NT;
    float v[PERV][CV];
    float h[PERH];
    __device__ __forceinline__ void load(const pk_conv3d_args &a, int64_t z, int64_t gy0, int64_t gx0) {
        const bool zin = z >= 0 && z < a.D;
#pragma unroll
        for (int p = 0; p < PERV; ++p) {
            const int q = p * NT + (int)threadIdx.x;
            const int r = q / (BX / CV), c = (q % (BX / CV)) * CV;
            const int64_t gy = gy0 + r, gx = gx0 + c;
            if (q < NV && zin && gy >= 0 && gy < a.H && gx + CV <= a.W) {
                PK_LDM<CV>(a.in + (z * a.H + gy) * a.W + gx, v[p]);
            } else {
#pragma unroll
                for (int e = 0; e < CV; ++e)
                    v[p][e] = (q < NV && zin && gy >= 0 && gy < a.H && gx + e < a.W)
                                  ? a.in[(z * a.H + gy) * a.W + gx + e] : 0.f;
            }
        }
#pragma unroll
        for (int p = 0; p < PERH; ++p) {
            const int q = p * NT + (int)threadIdx.x;
            const int r = q >> 1;
            const int64_t gy = gy0 + r, gx = (q & 1) ? gx0 + BX : gx0 - 1;
            h[p] = (q < NH && zin && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
                       ? a.in[(z * a.H + gy) * a.W + gx] : 0.f;
        }
    }
    __device__ __forceinline__ void store(float *t) const {
#pragma unroll
        for (int p = 0; p < PERV; ++p) {
            const int q = p * NT + (int)threadIdx.x;
            if (q < NV)
                pk_stv<CV>(t + (q / (BX / CV)) * LW4 + 4 + (q % (BX / CV)) * CV, v[p]);
        }
#pragma unroll
        for (int p = 0; p < PERH; ++p) {
            const int q = p * NT + (int)threadIdx.x;
            if (q < NH)
                t[(q >> 1) * LW4 + ((q & 1) ? 4 + BX : 3)] = h[p];
        }
    }
};

#if PF == 2
// output plane z (step r: its input planes z-1, z, z+1 sit in ring slots r, r+1, r+2
// mod 4): each thread's VEC x YR patch from the 27 taps, then stored
template <int CV>
__device__ __forceinline__ void staged_plane(const pk_conv3d_args &a, const float *ring, int r, int64_t z,
                                             int64_t x0, int64_t y0, int tx, int ty, const float *w) {
    if (x0 >= a.W || y0 >= a.H)
        return;
    float acc[YR][VEC];
#pragma unroll
    for (int i = 0; i < YR; ++i)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            acc[i][e] = 0.f;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
        const float *pl = ring + ((r + dz) % 4) * LP4 + 3 + tx * VEC;
#pragma unroll
        for (int rr = 0; rr < YR + 2; ++rr) {              // tile row ty*YR + rr = output row y0 + rr - 1
            float v[VEC + 2];
#pragma unroll
            for (int d = 0; d < VEC + 2; ++d)
                v[d] = pl[(ty * YR + rr) * LW4 + d];
#pragma unroll
            for (int i = 0; i < YR; ++i) {
                const int dy = rr - i;                      // input row y0+i-1+dy
                if (dy < 0 || dy > 2)
                    continue;
#pragma unroll
                for (int e = 0; e < VEC; ++e)
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx)
                        acc[i][e] += w[dz * 9 + dy * 3 + dx] * v[e + dx];
            }
        }
    }
    const bool zb = (z == 0 || z == a.D - 1);
#pragma unroll
    for (int i = 0; i < YR; ++i) {
        const int64_t y = y0 + i;
        if (y >= a.H)
            break;
        float o[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int64_t x = x0 + e;
            o[e] = (zb || y == 0 || y == a.H - 1 || x == 0 || x >= a.W - 1) ? 0.f : acc[i][e];
        }
        float *orow = a.out + (z * a.H + y) * a.W;
        if (CV > 1 && x0 + VEC <= a.W) {
#pragma unroll
            for (int e = 0; e < VEC; e += (VEC < CV ? VEC : CV))
                pk_stv<(VEC < CV ? VEC : CV)>(orow + x0 + e, o + e);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (x0 + e < a.W)
                    orow[x0 + e] = o[e];
        }
    }
}
#endif

template <int CV>
__device__ __forceinline__ void conv3d_staged_body(const pk_conv3d_args &a, float *ring) {
    const int tx = threadIdx.x % TX;
    const int ty = threadIdx.x / TX;
    const int64_t nbx = (a.W + BX - 1) / BX;
    const int64_t nby = (a.H + BYT - 1) / BYT;
    const int64_t nbz = (a.D + ROWS - 1) / ROWS;
    int64_t b = blockIdx.x, bx, by, bz;
    if (ORDER == 2)
        b = xcd_contiguous(b, nbx * nby * nbz);
    if (ORDER == 0 || ORDER == 2) {
        bx = b % nbx; b /= nbx;
        by = b % nby; bz = b / nby;
    } else {
        by = b % nby; b /= nby;
        bx = b % nbx; bz = b / nbx;
    }
    if (bz >= nbz)
        return;
    const int64_t gx0 = bx * BX, gy0 = by * BYT - 1;      // tile origin (interior column 0, halo row 0)
    const int64_t x0 = gx0 + (int64_t)tx * VEC;
    const int64_t y0 = by * BYT + (int64_t)ty * YR;
    const int64_t z0 = bz * ROWS;
    float w[27];
#pragma unroll
    for (int t = 0; t < 27; ++t)
        w[t] = a.w[t];

#if PF == 2
    // two register tiles in turn: the loads for plane z0 + r + 4 are issued during
    // step r and stored to LDS at the end of step r + 2, so two planes' arithmetic
    // covers each plane's load latency (slot k % 4 holds plane z0 - 1 + k as below)
    PlaneTile<CV> pa, pb;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        pa.load(a, z0 - 1 + k, gy0, gx0);
        pa.store(ring + k * LP4);
    }
    __syncthreads();
    pa.load(a, z0 + 2, gy0, gx0);
    pb.load(a, z0 + 3, gy0, gx0);
    for (int r = 0; r < ROWS; r += 2) {
        if (z0 + r >= a.D)
            break;                                          // uniform across the block
        staged_plane<CV>(a, ring, r, z0 + r, x0, y0, tx, ty, w);
        if (r + 1 < ROWS)
            pa.store(ring + ((r + 3) % 4) * LP4);           // plane z0 + r + 2
        __syncthreads();
        if (r + 3 < ROWS)
            pa.load(a, z0 + r + 4, gy0, gx0);
        if (r + 1 >= ROWS || z0 + r + 1 >= a.D)
            break;
        staged_plane<CV>(a, ring, r + 1, z0 + r + 1, x0, y0, tx, ty, w);
        if (r + 2 < ROWS)
            pb.store(ring + ((r + 4) % 4) * LP4);           // plane z0 + r + 3
        __syncthreads();
        if (r + 4 < ROWS)
            pb.load(a, z0 + r + 5, gy0, gx0);
    }
#else
    // slot k % 4 holds plane z0 - 1 + k
    PlaneTile<CV> pt;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        pt.load(a, z0 - 1 + k, gy0, gx0);
        pt.store(ring + k * LP4);
    }
    __syncthreads();
    pt.load(a, z0 + 2, gy0, gx0);
    for (int r = 0; r < ROWS; ++r) {
        const int64_t z = z0 + r;
        if (z >= a.D)
            break;                                          // uniform across the block
        if (x0 < a.W && y0 < a.H) {
            float acc[YR][VEC];
#pragma unroll
            for (int i = 0; i < YR; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    acc[i][e] = 0.f;
#pragma unroll
            for (int dz = 0; dz < 3; ++dz) {
                const float *pl = ring + ((r + dz) % 4) * LP4 + 3 + tx * VEC;
#pragma unroll
                for (int rr = 0; rr < YR + 2; ++rr) {      // tile row ty*YR + rr = output row y0 + rr - 1
                    float v[VEC + 2];
#pragma unroll
                    for (int d = 0; d < VEC + 2; ++d)
                        v[d] = pl[(ty * YR + rr) * LW4 + d];
#pragma unroll
                    for (int i = 0; i < YR; ++i) {
                        const int dy = rr - i;              // input row y0+i-1+dy
                        if (dy < 0 || dy > 2)
                            continue;
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
#pragma unroll
                            for (int dx = 0; dx < 3; ++dx)
                                acc[i][e] += w[dz * 9 + dy * 3 + dx] * v[e + dx];
                    }
                }
            }
            const bool zb = (z == 0 || z == a.D - 1);
#pragma unroll
            for (int i = 0; i < YR; ++i) {
                const int64_t y = y0 + i;
                if (y >= a.H)
                    break;
                float o[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int64_t x = x0 + e;
                    o[e] = (zb || y == 0 || y == a.H - 1 || x == 0 || x >= a.W - 1) ? 0.f : acc[i][e];
                }
                float *orow = a.out + (z * a.H + y) * a.W;
                if (CV > 1 && x0 + VEC <= a.W) {
#pragma unroll
                    for (int e = 0; e < VEC; e += (VEC < CV ? VEC : CV))
                        pk_stv<(VEC < CV ? VEC : CV)>(orow + x0 + e, o + e);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        if (x0 + e < a.W)
                            orow[x0 + e] = o[e];
                }
            }
        }
        if (r + 1 < ROWS)
            pt.store(ring + ((r + 3) % 4) * LP4);           // plane z0 + r + 2 (slot last read for output r - 1)
        __syncthreads();
        if (r + 2 < ROWS)
            pt.load(a, z0 + r + 3, gy0, gx0);
    }
#endif
}
#endif

extern "C" __global__ void __launch_bounds__(NT) pk_conv3d(pk_conv3d_args a) {
    if (blockDim.x != NT)
        return;
#if USE_LDS == 2
    __shared__ __attribute__((aligned(16))) float ring[4 * LP4];
    if (a.aligned)
        conv3d_staged_body<4>(a, ring);
    else
        conv3d_staged_body<1>(a, ring);
#elif USE_LDS
    __shared__ __attribute__((aligned(16))) float ring[3 * LP3];
    if (VEC > 1 && a.aligned)
        conv3d_lds_body<VEC>(a, ring);
    else
        conv3d_lds_body<1>(a, ring);
#else
    if (VEC > 1 && a.aligned)
        conv3d_body<VEC>(a);
    else
        conv3d_body<1>(a);
#endif
}
#endif
