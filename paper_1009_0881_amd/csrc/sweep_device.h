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
__device__ __forceinline__ double max_t(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float max_t(float a, float b) { return __builtin_fmaxf(a, b); }

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
//
// The Gram rows are read in batches of GB rows, each batch issued one batch
// ahead of the FMAs that use it (scheduling barriers keep the reads there;
// left alone, the compiler waits on every read next to its use).  Rows
// l >= r are zero in LDS: their batches are read but not used.
template <int RT, class T>
__device__ __forceinline__ void gram_matvec(const T (&x)[RT], const T *G, int gs, int r, int p,
                                            T (&acc)[RT]) {
    constexpr int RPAD = 16 * RT, GB = 8, NB = RPAD / GB;
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = T(0);
    T buf[2][GB][RT];
    auto fetch = [&](auto b_c) {
        constexpr int b = decltype(b_c)::value;
#pragma unroll
        for (int i = 0; i < GB; ++i)
#pragma unroll
            for (int t = 0; t < RT; ++t) buf[b & 1][i][t] = G[(GB * b + i) * gs + p + 16 * t];
    };
    fetch(std::integral_constant<int, 0>{});
    static_for<NB>([&](auto b_c) {
        constexpr int b = decltype(b_c)::value;
        if constexpr (b + 1 < NB) fetch(std::integral_constant<int, b + 1>{});
        __builtin_amdgcn_sched_barrier(0);
        if (GB * b < r) {
            static_for<GB>([&](auto i_c) {
                constexpr int i = decltype(i_c)::value, l = GB * b + i;
                const T xl = row_bcast<l % 16>(x[l / 16]);
#pragma unroll
                for (int t = 0; t < RT; ++t) acc[t] = fma_t(xl, buf[b & 1][i][t], acc[t]);
            });
        }
        __builtin_amdgcn_sched_barrier(0);
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
                // keep the loads here: the scheduler would otherwise sink them to
                // their use PD steps later and wait for LDS there
                __builtin_amdgcn_sched_barrier(0);
            }
            // Only the owner lane's d is broadcast.  With 1/G_kk = 0 (G_kk = 0)
            // c0 = x_k and the floor is x_k itself, so d = 0 and x_k keeps its
            // value; the floor is chosen off the dependency chain.  Lanes
            // p <= pk update a g entry they no longer read.
            const T lo = ginv[kt] > T(0) ? T(0) : x[kt];
            const T c0 = fma_t(g[kt], ginv[kt], x[kt]);
            const T cand = max_t(c0, lo);
            T d = cand - x[kt];
            x[kt] = p == pk ? cand : x[kt];
            d = row_bcast<pk>(d);
            dprev = d;
            g[kt] = fma_t(-d, rows[0][kt], g[kt]);
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

// An r x r FP64 Gram (row-major, stride r) staged through registers: thread
// tid holds entries tid + 256 i of the RPAD x RPAD zero-padded matrix and
// diagonal entry tid.  gram_fetch issues the loads (clamped addresses, no
// value depends on them yet); gram_put masks and stores them into LDS (stride
// gs) with the inverse diagonal, so the loads can be in flight while other
// work runs in between.  Blocks of 256 threads.
template <int RPAD>
struct GramRegs {
    static constexpr int PER = (RPAD * RPAD + 255) / 256;
    double v[PER];
    double g;
};

template <int RPAD>
__device__ __forceinline__ void gram_fetch(const double *__restrict__ Gd, int r,
                                           GramRegs<RPAD> &R) {
    const auto G = to_global(Gd);
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < GramRegs<RPAD>::PER; ++i) {
        const int e = tid + 256 * i, a = e / RPAD, b = e % RPAD;
        R.v[i] = G[(e < RPAD * RPAD && a < r && b < r) ? a * r + b : 0];
    }
    R.g = G[tid < r ? tid * r + tid : 0];
}

template <int RPAD, class T = double>
__device__ __forceinline__ void gram_put(const GramRegs<RPAD> &R, int r, T *Gs, int gs, T *gi) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < GramRegs<RPAD>::PER; ++i) {
        const int e = tid + 256 * i, a = e / RPAD, b = e % RPAD;
        if (e < RPAD * RPAD) Gs[a * gs + b] = (a < r && b < r) ? (T)R.v[i] : T(0);
    }
    if (tid < RPAD) gi[tid] = (tid < r && R.g > 0.0) ? (T)(1.0 / R.g) : T(0);
}

// Load an r x r FP64 Gram into LDS zero-padded to RPAD x RPAD (stride gs),
// and its inverse diagonal: every thread issues all of its loads before its
// first store, so the block waits for one memory latency.
template <int RPAD, class T = double>
__device__ __forceinline__ void load_gram(const double *__restrict__ Gd, int r, T *Gs, int gs,
                                          T *gi) {
    GramRegs<RPAD> R;
    gram_fetch<RPAD>(Gd, r, R);
    gram_put<RPAD, T>(R, r, Gs, gs, gi);
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
// out[e] = sum over p = 0..count-1 of pg[e][p * stride] in index order, for
// the outputs with ok[e] (the others are 0; pg[e] must still point at `count`
// readable values).  The loads of all N outputs go out together in batches of
// B, from clamped indices as in sum_strided.
template <int N, int B = 16, class T = double>
__device__ __forceinline__ void sum_strided_n(const T *const (&pg)[N], const bool (&ok)[N],
                                              int64_t stride, int count, double (&out)[N]) {
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = 0.0;
    for (int p = 0; p < count; p += B) {
        double t[N][B];
#pragma unroll
        for (int e = 0; e < N; ++e)
#pragma unroll
            for (int u = 0; u < B; ++u)
                t[e][u] = (double)to_global(pg[e])[(int64_t)(p + u < count ? p + u : count - 1) * stride];
#pragma unroll
        for (int e = 0; e < N; ++e)
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (ok[e] && p + u < count) out[e] += t[e][u];
    }
}

}  // namespace

}  // namespace nmf
