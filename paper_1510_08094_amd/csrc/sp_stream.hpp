// Streaming kernels that measure the achievable HBM bandwidth of the device:
// a copy, a read (each workgroup reduces its chunk to one partial sum) and a
// write (fill).  Each thread moves 4 x 16 bytes per direction with 128-bit
// accesses, all loads issued before the first store; workgroups take
// consecutive 16 KiB chunks, so a wavefront reads whole 128-byte lines.  NT
// selects non-temporal accesses (the data is touched once).  The tail that
// does not fill a whole chunk is handled element by element.
#pragma once
#include <hip/hip_runtime.h>

namespace sp {

typedef double vd2 __attribute__((ext_vector_type(2)));   // one 128-bit access

constexpr int kStreamThreads = 256;
constexpr int kStreamVec = 4;                                        // vd2 per thread
constexpr int kStreamChunk = kStreamThreads * kStreamVec * 2;        // doubles per workgroup

template <bool NT>
__device__ __forceinline__ vd2 stream_ld(const vd2* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT>
__device__ __forceinline__ void stream_st(vd2* p, vd2 v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <bool NT>
__global__ void __launch_bounds__(kStreamThreads) k_stream_copy(const double* __restrict__ x, double* __restrict__ y,
                                                                 size_t count) {
    const size_t base = (size_t)blockIdx.x * kStreamChunk;
    if (base + kStreamChunk <= count) {
        const vd2* xs = reinterpret_cast<const vd2*>(x + base) + threadIdx.x;
        vd2* ys = reinterpret_cast<vd2*>(y + base) + threadIdx.x;
        vd2 v[kStreamVec];
#pragma unroll
        for (int e = 0; e < kStreamVec; ++e) v[e] = stream_ld<NT>(xs + e * kStreamThreads);
#pragma unroll
        for (int e = 0; e < kStreamVec; ++e) stream_st<NT>(ys + e * kStreamThreads, v[e]);
    } else {
        for (size_t i = base + threadIdx.x; i < count; i += kStreamThreads) y[i] = x[i];
    }
}

template <bool NT>
__global__ void __launch_bounds__(kStreamThreads) k_stream_read(const double* __restrict__ x,
                                                                 double* __restrict__ partial, size_t count) {
    __shared__ double red[kStreamThreads / 64];
    const size_t base = (size_t)blockIdx.x * kStreamChunk;
    double s = 0.0;
    if (base + kStreamChunk <= count) {
        const vd2* xs = reinterpret_cast<const vd2*>(x + base) + threadIdx.x;
        vd2 v[kStreamVec];
#pragma unroll
        for (int e = 0; e < kStreamVec; ++e) v[e] = stream_ld<NT>(xs + e * kStreamThreads);
#pragma unroll
        for (int e = 0; e < kStreamVec; ++e) s += v[e].x + v[e].y;
    } else {
        for (size_t i = base + threadIdx.x; i < count; i += kStreamThreads) s += x[i];
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kStreamThreads / 64; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

template <bool NT>
__global__ void __launch_bounds__(kStreamThreads) k_stream_write(double* __restrict__ y, double value, size_t count) {
    const size_t base = (size_t)blockIdx.x * kStreamChunk;
    if (base + kStreamChunk <= count) {
        vd2* ys = reinterpret_cast<vd2*>(y + base) + threadIdx.x;
        const vd2 v = {value, value};
#pragma unroll
        for (int e = 0; e < kStreamVec; ++e) stream_st<NT>(ys + e * kStreamThreads, v);
    } else {
        for (size_t i = base + threadIdx.x; i < count; i += kStreamThreads) y[i] = value;
    }
}

}  // namespace sp
