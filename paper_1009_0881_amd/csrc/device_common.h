// Small device helpers shared by the HIP kernels of libnmf (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace nmf {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// f(integral_constant<int, I>) for I = 0..N-1, unrolled at compile time.
template <int N, int I = 0, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

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

// Position of entry k within a row of Wt (the transposed W, rpad = 16 rt
// entries per row): interleaved so that entries 16t + p, t = 0..rt-1, of lane
// p are contiguous and one vector load gives a lane all of its W operands.
__host__ __device__ __forceinline__ int wt_pos(int k, int rt) { return (k & 15) * rt + (k >> 4); }

// The RT operands 16t + li (t = 0..RT-1) of a row of Wt.
template <int RT>
__device__ __forceinline__ void load_wt(gmem<const float> *row, int li, float (&out)[RT]) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    gmem<const float> *p = row + li * RT;
    if constexpr (RT == 4) {
        const v4f x = *(gmem<const v4f> *)p;
        out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
    } else if constexpr (RT == 2) {
        const v2 x = *(gmem<const v2> *)p;
        out[0] = x[0]; out[1] = x[1];
    } else {
#pragma unroll
        for (int t = 0; t < RT; ++t) out[t] = p[t];
    }
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
