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

// Prefetch distance (in HALS steps) of the Gram rows in row_update.
constexpr int kGramAhead = 2;

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

// acc[t] = sum_l x_l G[l][16t + p] for a factor row held by a row of 16 lanes
// (lane p holding entries 16t + p) and the r x r Gram G in LDS (row stride
// gs, zero-padded).  Padded entries (l >= r) are zero and skipped in whole
// groups of 4.
template <int RT, class T>
__device__ __forceinline__ void gram_matvec(const T (&x)[RT], const T *G, int gs, int r, int p,
                                            T (&acc)[RT]) {
    constexpr int RPAD = 16 * RT;
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = T(0);
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
    // acc_k = sum_l x_l G_lk; the HALS loop then runs over the RPAD entries
    // with the padded ones (x_k = 0, zero Gram rows, 1/G_kk = 0) skipped.
    T acc[RT];
    gram_matvec<RT>(x, G, gs, r, p, acc);
    if constexpr (MODE == MODE_HALS) {
        // Gram rows ahead of step k: rows[i] holds row k + i.  Step k loads
        // row k + PD behind ordered_after() on the previous step's broadcast,
        // so loads run PD steps ahead (hiding LDS latency) and the compiler
        // cannot hoist all of them (and spill).  Steps k >= r change nothing
        // (padded entries) and are skipped: each step runs the next one only
        // while k + 1 < r, a nest of uniform branches.
        constexpr int PD = kGramAhead < RPAD ? kGramAhead : RPAD;
        T g[RT], ginv[RT], rows[PD][RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + p;
            g[t] = k < r ? a[t] - acc[t] : T(0);
            ginv[t] = gi[k];
#pragma unroll
            for (int i = 0; i < PD; ++i) rows[i][t] = G[i * gs + k];
        }
        T dprev = acc[0];
        auto step = [&](auto self, auto k_c) -> void {
            constexpr int k = decltype(k_c)::value, kt = k / 16, pk = k % 16;
            T rnew[RT];
            if constexpr (k + PD < RPAD) {
                const T *gr = G + ordered_after((k + PD) * gs + p, dprev);
#pragma unroll
                for (int t = (k + PD) / 16; t < RT; ++t) rnew[t] = gr[16 * t];
            }
            const bool own = p == pk && ginv[kt] > T(0);
            const T c0 = fma_t(g[kt], ginv[kt], x[kt]);
            const T cand = c0 > T(0) ? c0 : T(0);
            T d = own ? cand - x[kt] : T(0);
            x[kt] = own ? cand : x[kt];
            d = row_bcast<pk>(d);
            dprev = d;
            g[kt] = p > pk ? fma_t(-d, rows[0][kt], g[kt]) : g[kt];
#pragma unroll
            for (int t = kt + 1; t < RT; ++t) g[t] = fma_t(-d, rows[0][t], g[t]);
#pragma unroll
            for (int t = (k + 1) / 16; t < RT; ++t) {
#pragma unroll
                for (int i = 0; i + 1 < PD; ++i) rows[i][t] = rows[i + 1][t];
                if constexpr (k + PD < RPAD) rows[PD - 1][t] = rnew[t];
            }
            if constexpr (k + 1 < RPAD) {
                if (k + 1 < r) self(self, std::integral_constant<int, k + 1>{});
            }
        };
        if (r > 0) step(step, std::integral_constant<int, 0>{});
    } else {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + p;
            if (k < r && acc[t] > T(0)) x[t] = x[t] * a[t] / acc[t];
        }
    }
}

// Load an r x r FP64 Gram (row-major, stride r) into LDS zero-padded to
// RPAD x RPAD (stride gs), and its inverse diagonal.  Blocks of 256 threads:
// every thread issues all of its loads before its first store, so the block
// waits for one memory latency.
template <int RPAD, class T = double>
__device__ __forceinline__ void load_gram(const double *__restrict__ Gd, int r, T *Gs, int gs,
                                          T *gi) {
    constexpr int PER = (RPAD * RPAD + 255) / 256;
    const auto G = to_global(Gd);
    const int tid = threadIdx.x;
    double v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = tid + 256 * i, a = e / RPAD, b = e % RPAD;
        v[i] = (e < RPAD * RPAD && a < r && b < r) ? G[a * r + b] : 0.0;
    }
    const double g = (tid < r) ? G[tid * r + tid] : 0.0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = tid + 256 * i, a = e / RPAD, b = e % RPAD;
        if (e < RPAD * RPAD) Gs[a * gs + b] = (T)v[i];
    }
    if (tid < RPAD) gi[tid] = g > 0.0 ? (T)(1.0 / g) : T(0);
}

// Sum of `count` values p0[0], p0[stride], ... (FP64 or FP32) in FP64, in
// index order, with up to W loads in flight.
template <int W = 16, class T = double>
__device__ __forceinline__ double sum_strided(const T *__restrict__ pg, int64_t stride,
                                              int count) {
    const auto p0 = to_global(pg);
    double s = 0.0;
    int p = 0;
    for (; p + W <= count; p += W) {
        double t[W];
#pragma unroll
        for (int u = 0; u < W; ++u) t[u] = (double)p0[(p + u) * stride];
#pragma unroll
        for (int u = 0; u < W; ++u) s += t[u];
    }
    if (p < count) {   // the rest in one batch
        double t[W];
#pragma unroll
        for (int u = 0; u < W; ++u) t[u] = (p + u < count) ? (double)p0[(p + u) * stride] : 0.0;
#pragma unroll
        for (int u = 0; u < W; ++u)
            if (p + u < count) s += t[u];
    }
    return s;
}

// Sums of `count` values (FP64 or FP32) for N outputs at once, in FP64:
// out[e] = sum over p = 0..count-1 of pg[e][p * stride] in index order (pg[e]
// null: 0).  The loads of all N outputs go out together in batches of B.
template <int N, int B = 16, class T = double>
__device__ __forceinline__ void sum_strided_n(const T *const (&pg)[N], int64_t stride, int count,
                                              double (&out)[N]) {
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = 0.0;
    for (int p = 0; p < count; p += B) {
        double t[N][B];
#pragma unroll
        for (int e = 0; e < N; ++e)
#pragma unroll
            for (int u = 0; u < B; ++u)
                t[e][u] = (pg[e] && p + u < count)
                              ? (double)to_global(pg[e])[(int64_t)(p + u) * stride]
                              : 0.0;
#pragma unroll
        for (int e = 0; e < N; ++e)
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (p + u < count) out[e] += t[e][u];
    }
}

}  // namespace

}  // namespace nmf
