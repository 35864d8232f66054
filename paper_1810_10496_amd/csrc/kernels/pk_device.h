// pk_device.h -- device-side helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../pk_kernel_abi.h"

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

#define PK_WAVE 64

// Every code object records the knobs it was compiled with.  `used` keeps the
// array alive through any optimisation pipeline the tuner applies.
#define PK_DEFINE_KNOBS(...)                                                   \
    extern "C" __device__ __attribute__((used, visibility("default")))         \
    const int pk_knobs[PK_NKNOBS] = {__VA_ARGS__};

// FP32 -> bfloat16 bits, round to nearest, ties to even (finite inputs; values
// beyond the largest bfloat16 become infinity).  Integer arithmetic only, so
// the result does not depend on the floating-point mode of the kernel.
__device__ __forceinline__ uint32_t pk_bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ float pk_bf16_to_f32(uint32_t b) {
    return __uint_as_float(b << 16);
}

// two bf16 values packed low/high into one 32-bit word
__device__ __forceinline__ uint32_t pk_pack_bf16(float lo, float hi) {
    return pk_bf16_bits(lo) | (pk_bf16_bits(hi) << 16);
}

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi); x - hi is exact in FP32
__device__ __forceinline__ void pk_split(float x, uint32_t &hb, uint32_t &lb) {
    hb = pk_bf16_bits(x);
    lb = pk_bf16_bits(x - pk_bf16_to_f32(hb));
}

__device__ __forceinline__ float pk_wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, PK_WAVE);
    return v;
}

// Neumaier compensated accumulation: (s, c) += x
__device__ __forceinline__ void pk_neumaier(float &s, float &c, float x) {
    float t = s + x;
    if (fabsf(s) >= fabsf(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

template <int V> struct pk_vec;
template <> struct pk_vec<1> { typedef float T; };
template <> struct pk_vec<2> { typedef f32x2 T; };
template <> struct pk_vec<4> { typedef f32x4 T; };

// load V consecutive floats (p must be V*4-byte aligned)
template <int V>
__device__ __forceinline__ void pk_ldv(const float *p, float *dst) {
    typedef typename pk_vec<V>::T T;
    T v = *reinterpret_cast<const T *>(p);
    if constexpr (V == 1) {
        dst[0] = v;
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i)
            dst[i] = v[i];
    }
}

// the same load with the non-temporal hint, for data read once: its lines need not
// displace reusable ones from the caches
template <int V>
__device__ __forceinline__ void pk_ldv_nt(const float *p, float *dst) {
    typedef typename pk_vec<V>::T T;
    T v = __builtin_nontemporal_load(reinterpret_cast<const T *>(p));
    if constexpr (V == 1) {
        dst[0] = v;
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i)
            dst[i] = v[i];
    }
}

template <int V>
__device__ __forceinline__ void pk_stv(float *p, const float *src) {
    typedef typename pk_vec<V>::T T;
    T v;
    if constexpr (V == 1) {
        v = src[0];
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i)
            v[i] = src[i];
    }
    *reinterpret_cast<T *>(p) = v;
}

// ---- one-launch reductions ------------------------------------------------------------
// A kernel that writes per-block partial sums can fold them in the same launch: the
// last block of a group to finish (a column strip, a row block) reads the group's
// partials in a fixed order and writes the result, so the output does not depend on
// which block that is.  Each group has a 64-bit ticket cell: the call's tag in the
// high half and the number of the group's blocks that have arrived in that call in
// the low half.  A cell whose tag is not the call's, or whose count is not below the
// group size, reads as empty, so the cells need no clearing before a call (a tag is a
// value the library never used before); the block that completes a group clears its
// cell, so a captured graph that replays one tag starts every replay from empty cells.
//
// The partials' writers and their reader may sit on different XCDs, whose L2 caches
// are not coherent with each other.  The partials therefore travel as device-scope
// relaxed atomic stores and loads, which bypass the non-coherent caches, and each
// wavefront waits for its stores to complete before the block's barrier and ticket.
// (Plain stores with device-scope release and acquire fences were measured 1.1-2.7x
// slower per call: each release writes back the XCD's whole L2.)  Cells sit
// PK_CELL_STRIDE bytes apart: device-scope atomics on one cache line queue behind
// each other.

__device__ __forceinline__ void pk_part_store(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float pk_part_load(const float *p) {
    return __hip_atomic_load(const_cast<float *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// V consecutive partials (p 4V-byte aligned)
template <int V>
__device__ __forceinline__ void pk_part_loadv(const float *p, float *dst) {
#pragma unroll
    for (int i = 0; i < V; ++i)
        dst[i] = pk_part_load(p + i);
}

// Called by every thread of the block after its partial stores (block-uniform
// arguments); returns true in every thread of the block that completed the group.
// The compare-and-swap loop is lock free: each failed attempt means another block of
// the group got its ticket, so a block retries at most group-size - 1 times.
// `cells` is the group array, `group` the block's group, `guess` the number of the
// group's blocks expected to have arrived before this one (0 for the first): the
// first compare-and-swap assumes it, so a block that arrives in that order takes its
// ticket with one atomic operation.
__device__ __forceinline__ bool pk_ticket_last(unsigned long long *cells, int group, uint32_t guess,
                                               uint32_t tag, uint32_t total, int *flag) {
    unsigned long long *cell = cells + (int64_t)group * (PK_CELL_STRIDE / 8);
    __builtin_amdgcn_s_waitcnt(0);          // this wavefront's partial stores have completed
    __syncthreads();
    if (threadIdx.x == 0) {
        bool last = true;
        if (total > 1) {
            unsigned long long old = guess == 0 ? 0ull : (((unsigned long long)tag << 32) | guess);
            uint32_t cnt;
            for (;;) {
                const bool ours = (uint32_t)(old >> 32) == tag && (uint32_t)old < total;
                cnt = (ours ? (uint32_t)old : 0u) + 1u;
                const unsigned long long want = ((unsigned long long)tag << 32) | cnt;
                const unsigned long long prev = atomicCAS(cell, old, want);
                if (prev == old)
                    break;
                old = prev;
            }
            last = cnt == total;
            if (last)
                __hip_atomic_store(cell, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        *flag = last ? 1 : 0;
    }
    __syncthreads();
    return *flag != 0;
}

// row stride (floats) of the partial-sum rows a one-launch reduction writes: rows
// start 256-byte aligned, so a fold reads them with 16-byte loads
__host__ __device__ __forceinline__ int64_t pk_part_ld(int64_t n) { return (n + 63) & ~(int64_t)63; }
