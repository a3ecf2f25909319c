// Device helpers shared by the sweep kernels (regular and streaming):
// operand types, BF16 rounding, the per-block job lookup, row broadcasts, the
// factor-row update of Alg. 2 / Alg. 3, Gram staging and strided sums.
#pragma once

#include <type_traits>

#include "device_common.h"
#include "job.h"
#include "nmf_internal.h"

namespace nmf {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

constexpr int MODE_HALS = 0, MODE_MU = 1, MODE_STORE = 2, MODE_INIT = 3;

template <int N, int I = 0, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

// (job, tile) of this block: entry blockIdx.x of the launch's block map, or
// (0, blockIdx.x) for a launch over a single job (null map).
__device__ __forceinline__ int2 block_job(const int2 *bmap) {
    return bmap ? bmap[blockIdx.x] : make_int2(0, (int)blockIdx.x);
}

// Broadcast lane N of every row of 16 consecutive lanes to the whole row
// (DPP row_newbcast).
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + N, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + N, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int N>
__device__ __forceinline__ float row_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + N, 0xF, 0xF, false));
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Returns v unchanged, but only once dep has been computed: an empty asm that
// takes dep as an input orders the instructions that use the result after
// those that produce dep.  No instruction is emitted.
template <class T>
__device__ __forceinline__ int ordered_after(int v, T dep) {
    asm("" : "+v"(v) : "v"(dep));
    return v;
}

// HALS / MU update of one factor row held by a row of 16 lanes, lane p
// holding entries k = 16t + p.  G is the r x r FP64 Gram of the other factor
// in LDS (row stride gs, zero-padded to RPAD), gi[k] = 1/G_kk (0 when
// G_kk = 0 or k >= r), a[t] entry 16t + p of the matching row of the product.  The
// r x r-sized update arithmetic runs in T: FP64 in the FP32 mode (the
// numerator a_k - sum_l x_l G_lk cancels as the iterate converges), FP32 in
// the BF16 mode; the row is read from and written back to FP32 storage by the
// caller.
//
// HALS (Alg. 3): x_k <- max(0, (a_k - sum_{l != k} x_l G_lk) / G_kk) for
// k = 1..r in order, G_kk = 0 keeping x_k.  Computed in the equivalent
// gradient form: g = a - G x once, then for each k the owner lane sets
// x_k <- max(0, x_k + g_k / G_kk), broadcasts the change d to its row, and
// every lane applies g_l -= d G_kl for its l > k.
// MU (Alg. 2): x_k <- x_k a_k / (sum_l x_l G_lk); a zero denominator keeps x_k.
template <int RT, int MODE, class T = double>
__device__ __forceinline__ void row_update(T (&x)[RT], const T *G, int gs, const T *gi,
                                           const T (&a)[RT], int r, int p) {
    constexpr int RPAD = 16 * RT;
    T acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = T(0);
    // acc_k = sum_l x_l G_lk.  Padded entries (k >= r) have x_k = 0, zero Gram
    // rows and 1/G_kk = 0: the mat-vec skips whole groups of 4 of them, the
    // HALS loop runs over all RPAD entries with no runtime bound.
    static_for<RPAD / 4>([&](auto lg_c) {
        constexpr int lg = decltype(lg_c)::value;
        if (4 * lg < r) {
            static_for<4>([&](auto lq_c) {
                constexpr int l = 4 * lg + decltype(lq_c)::value;
                const T xl = row_bcast<l % 16>(x[l / 16]);
                const T *gr = G + l * gs + p;
#pragma unroll
                for (int t = 0; t < RT; ++t) acc[t] = fma_t(xl, gr[16 * t], acc[t]);
            });
        }
    });
    if constexpr (MODE == MODE_HALS) {
        T g[RT], ginv[RT], row0[RT], row1[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + p;
            g[t] = k < r ? a[t] - acc[t] : T(0);
            ginv[t] = gi[k];
            row0[t] = G[k];                  // Gram row 0
            row1[t] = G[gs + k];             // Gram row 1
        }
        // Each step loads the Gram row of step k+2 behind ordered_after() on
        // the previous step's broadcast: loads run two steps ahead, hiding LDS
        // latency, and the compiler cannot hoist all of them (and spill).
        T dprev = acc[0];
        static_for<RPAD>([&](auto k_c) {
            constexpr int k = decltype(k_c)::value, kt = k / 16, pk = k % 16;
            T row2[RT];
            if constexpr (k + 2 < RPAD) {
                const T *gr = G + ordered_after((k + 2) * gs + p, dprev);
#pragma unroll
                for (int t = (k + 2) / 16; t < RT; ++t) row2[t] = gr[16 * t];
            }
            const bool own = p == pk && ginv[kt] > T(0);
            const T c0 = fma_t(g[kt], ginv[kt], x[kt]);
            const T cand = c0 > T(0) ? c0 : T(0);
            T d = own ? cand - x[kt] : T(0);
            x[kt] = own ? cand : x[kt];
            d = row_bcast<pk>(d);
            dprev = d;
            g[kt] = p > pk ? fma_t(-d, row0[kt], g[kt]) : g[kt];
#pragma unroll
            for (int t = kt + 1; t < RT; ++t) g[t] = fma_t(-d, row0[t], g[t]);
#pragma unroll
            for (int t = (k + 1) / 16; t < RT; ++t) {
                row0[t] = row1[t];
                if constexpr (k + 2 < RPAD) row1[t] = row2[t];
            }
        });
    } else {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + p;
            if (k < r && acc[t] > T(0)) x[t] = x[t] * a[t] / acc[t];
        }
    }
}

// Load an r x r FP64 Gram (row-major, stride r) into LDS zero-padded to
// RPAD x RPAD (stride gs), and its inverse diagonal.
template <int RPAD, class T = double>
__device__ __forceinline__ void load_gram(const double *__restrict__ Gd, int r, T *Gs, int gs,
                                          T *gi) {
    const auto G = to_global(Gd);
    for (int e = threadIdx.x; e < RPAD * RPAD; e += blockDim.x) {
        const int a = e / RPAD, b = e % RPAD;
        Gs[a * gs + b] = (a < r && b < r) ? (T)G[a * r + b] : T(0);
    }
    for (int k = threadIdx.x; k < RPAD; k += blockDim.x) {
        const double g = (k < r) ? G[k * r + k] : 0.0;
        gi[k] = g > 0.0 ? (T)(1.0 / g) : T(0);
    }
}

// Sum of `count` FP64 values p0[0], p0[stride], ... in index order, with up
// to 16 loads in flight.
__device__ __forceinline__ double sum_strided(const double *__restrict__ pg, int64_t stride,
                                              int count) {
    const auto p0 = to_global(pg);
    double s = 0.0;
    int p = 0;
    for (; p + 16 <= count; p += 16) {
        double t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) t[u] = p0[(p + u) * stride];
#pragma unroll
        for (int u = 0; u < 16; ++u) s += t[u];
    }
    for (; p + 4 <= count; p += 4) {
        double t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = p0[(p + u) * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) s += t[u];
    }
    for (; p < count; ++p) s += p0[p * stride];
    return s;
}


}  // namespace

}  // namespace nmf
