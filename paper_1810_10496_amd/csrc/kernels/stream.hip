// stream.hip -- bandwidth probes: the ceilings the memory-bound kernels are
// measured against on this chip.  Not part of any of the paper's kernels.
//
//   pk_stream_read: every element of src read once with 16-byte loads (UNROLL
//                   loads in flight per thread); each block writes the sum of
//                   what it read to dst[blockIdx.x], so no load can be dropped
//   pk_stream_copy: dst[i] = src[i] with 16-byte loads and stores
//
// Both walk the buffer in grid-stride order: consecutive threads take
// consecutive 16-byte chunks, so every wavefront access is 1 KiB contiguous.
// With `nt` set the accesses carry the non-temporal hint (streamed past the
// caches instead of allocated in them); the caller takes the faster form.
#include "pk_device.h"

#ifndef NTHREADS
#define NTHREADS 256
#endif
#ifndef UNROLL
#define UNROLL 4
#endif

PK_DEFINE_KNOBS(PKF_STREAM, 0, 0, 0, NTHREADS / 64, 1, 4, UNROLL, 0, 0, 0, 0, NTHREADS, 0,
                PK_KERNEL_ABI_VERSION, 0)

template <bool NT>
__device__ __forceinline__ f32x4 ld(const f32x4 *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT>
__device__ __forceinline__ void st(f32x4 *p, f32x4 v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <bool NT>
__device__ __forceinline__ f32x4 read_body(const pk_stream_args &a, int64_t nv) {
    const int64_t stride = (int64_t)gridDim.x * NTHREADS;
    const f32x4 *src = reinterpret_cast<const f32x4 *>(a.src);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    int64_t i = (int64_t)blockIdx.x * NTHREADS + threadIdx.x;
    for (; i + (UNROLL - 1) * stride < nv; i += UNROLL * stride) {
        f32x4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            v[u] = ld<NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            acc += v[u];
    }
    for (; i < nv; i += stride)
        acc += ld<NT>(src + i);
    return acc;
}

template <bool NT>
__device__ __forceinline__ void copy_body(const pk_stream_args &a, int64_t nv) {
    const int64_t stride = (int64_t)gridDim.x * NTHREADS;
    const f32x4 *src = reinterpret_cast<const f32x4 *>(a.src);
    f32x4 *dst = reinterpret_cast<f32x4 *>(a.dst);
    int64_t i = (int64_t)blockIdx.x * NTHREADS + threadIdx.x;
    for (; i + (UNROLL - 1) * stride < nv; i += UNROLL * stride) {
        f32x4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            v[u] = ld<NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            st<NT>(dst + i + u * stride, v[u]);
    }
    for (; i < nv; i += stride)
        st<NT>(dst + i, ld<NT>(src + i));
}

extern "C" __global__ void __launch_bounds__(NTHREADS) pk_stream_read(pk_stream_args a) {
    if (blockDim.x != NTHREADS)
        return;
    const int64_t nv = a.n / 4;                                   // whole 16-byte chunks
    const f32x4 acc = a.nt ? read_body<true>(a, nv) : read_body<false>(a, nv);
    float s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    // the tail of fewer than 4 elements: block 0
    if (blockIdx.x == 0 && threadIdx.x < (int)(a.n - nv * 4))
        s += a.src[nv * 4 + threadIdx.x];
    s = pk_wave_sum(s);
    __shared__ float ws[NTHREADS / 64];
    if ((threadIdx.x & 63) == 0)
        ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
#pragma unroll
        for (int w = 0; w < NTHREADS / 64; ++w)
            t += ws[w];
        a.dst[blockIdx.x] = t;
    }
}

extern "C" __global__ void __launch_bounds__(NTHREADS) pk_stream_copy(pk_stream_args a) {
    if (blockDim.x != NTHREADS)
        return;
    const int64_t nv = a.n / 4;
    if (a.nt)
        copy_body<true>(a, nv);
    else
        copy_body<false>(a, nv);
    if (blockIdx.x == 0 && threadIdx.x < (int)(a.n - nv * 4))
        a.dst[nv * 4 + threadIdx.x] = a.src[nv * 4 + threadIdx.x];
}
