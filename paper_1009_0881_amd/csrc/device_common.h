// Small device helpers shared by the HIP kernels of libnmf (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace nmf {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Global-memory view of a pointer.  Pointers read from a job table are generic
// to the compiler, which then issues FLAT loads: they count against both the
// vector-memory and the LDS counters, so every wait on them becomes a full
// wait and loads issued ahead cannot stay in flight.  Through this view the
// compiler issues global_load / global_store, counted precisely.
template <class T>
using gmem = __attribute__((address_space(1))) T;

template <class T>
__device__ __forceinline__ gmem<T> *to_global(T *p) {
    return (gmem<T> *)p;
}

__device__ __forceinline__ bool stopped(const int32_t *stop) {
    return stop != nullptr && *stop != 0;
}

// Error-free accumulation of an FP32 partial sum p into the pair (hi, lo):
// hi + lo carries the running sum with the rounding error of every addition
// kept in lo (Knuth's TwoSum).  Used to merge short MFMA accumulation chains.
__device__ __forceinline__ void two_sum_acc(v4f &hi, v4f &lo, v4f p) {
    const v4f s = hi + p;
    const v4f bp = s - hi;
    const v4f e = (hi - (s - bp)) + (p - bp);
    hi = s;
    lo += e;
}

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

__device__ __forceinline__ float wave_sum_f32(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// Block-wide FP64 sum with a fixed reduction order (deterministic).  All
// threads of the block must call it; the result is valid in every thread.
template <int NT>
__device__ __forceinline__ double block_sum_f64(double x, double *scratch /* NT/64 */) {
    x = wave_sum_f64(x);
    const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    __syncthreads();
    if (lane == 0) scratch[wid] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) t += scratch[i];
    return t;
}

}  // namespace nmf
