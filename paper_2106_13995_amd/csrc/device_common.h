// Device helpers shared by the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsim {

template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };

template <typename T> using c2_t = typename C2<T>::type;

// acc += u * v for complex numbers held as (re, im) pairs.
template <typename T>
__device__ __forceinline__ void cfma(T &accr, T &acci, T ur, T ui, T vr, T vi) {
    accr = fma(ur, vr, accr);
    accr = fma(-ui, vi, accr);
    acci = fma(ur, vi, acci);
    acci = fma(ui, vr, acci);
}

// Inserts a zero bit at each of the ascending positions pos[0..np-1].
__device__ __forceinline__ uint64_t insert_zeros(uint64_t x, const int *pos, int np) {
    for (int i = 0; i < np; ++i) {
        const uint64_t lo = x & ((1ull << pos[i]) - 1ull);
        x = ((x - lo) << 1) | lo;
    }
    return x;
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Loads and stores of one or two amplitudes; NT marks them nontemporal
// (streamed once through HBM, not worth keeping in the caches).
template <bool NT, typename V>
__device__ __forceinline__ V ld(const void *p) {
    if constexpr (NT) return __builtin_nontemporal_load(static_cast<const V *>(p));
    else return *static_cast<const V *>(p);
}
template <bool NT, typename V>
__device__ __forceinline__ void st(void *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, static_cast<V *>(p));
    else *static_cast<V *>(p) = v;
}

constexpr int kBlockThreads = 256;

// Sum of one double per thread over a 256-thread block (four 64-wide waves);
// the result is valid in thread 0.  Fixed order: bitwise reproducible.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kBlockThreads / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlockThreads / 64; ++i) t += red[i];
    return t;
}

}  // namespace qsim
