// One NMF iteration on one level: the two M-streaming products and the
// factor updates of Alg. 2 (MU) and Alg. 3 (HALS), plus the residual.
//
//   k_apass    A = M W^T (m x r), V update fused as epilogue
//   k_cpass    split-m partials of C = V^T M, and of D = V^T V (FP64)
//   k_reduce   D = sum of partials (fixed order)
//   k_cfinal   C = sum of partials, W update, partials of W W^T and of the
//              residual terms
//   k_reduce   B = W W^T, plus rel_err = sqrt(||M||^2 - 2<C,W> + <D,B>)/||M||
//
// Every kernel takes a job table (one entry per problem and level, see job.h)
// and a block map: block b works on tile bmap[b].y of job bmap[b].x, so one
// launch per phase serves a single solve or a whole batch of uneven problems.
//
// Both products run on the FP32 matrix cores (v_mfma_f32_16x16x4f32); the
// Gram V^T V on the FP64 ones (v_mfma_f64_16x16x4f64).  Lane layout on a
// 64-wide wave: lane l supplies A[l%16][l/16] and B[l/16][l%16] for both;
// accumulator register v of lane l holds D[4*(l/16)+v][l%16] for the FP32
// instruction and D[4*v+l/16][l%16] for the FP64 one.
//
// Each MFMA accumulator chain covers 16 products; chain results are merged
// with TwoSum into an FP32 (hi, lo) pair and handed on in FP64, so the products
// carry about one FP32 rounding instead of the sqrt(length) growth of one long
// chain (the HALS numerator a_k - sum_l x_l G_lk cancels and would amplify
// that error).
//
// Factor updates: one factor row (a row of V, or a column of W) is owned by 16
// consecutive lanes, lane p holding the entries k = p (mod 16).  HALS walks
// k = 1..r in order using already-updated entries (Gauss-Seidel, Alg. 3);
// MU updates all entries from the old values (Alg. 2).

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

// ---------------------------------------------------------------------------
// A-pass tile.  Block = 4 waves; the waves form WR = 4/WN row groups of RW
// 16-row tiles each, and the WN waves of a row group split the n columns into
// contiguous ranges.  M (column j of a 16-row tile: 16 consecutive floats) and
// the transposed factor Wt (n x RPAD, row j = column j of W) are loaded
// straight into registers, S 4-column steps at a time, double buffered.  The
// WN partial tiles are added in LDS (fixed order) before the epilogue.
// ---------------------------------------------------------------------------
template <int RT, int RW, int WN>
constexpr int apass_lds_doubles(bool upd) {
    return (upd ? (RT * 16) * (RT * 16 + 1) + RT * 16 : 0) + 4 * 16 * RW * (RT * 16 + 1);
}

template <int RT, int RW, int WN, int S, int MODE, bool BF>
__device__ void apass_tile(const Job &J, int tile, double *smem) {
    constexpr int RPAD = RT * 16, WR = 4 / WN, TMW = 16 * RW, TM = TMW * WR;
    constexpr int AS = RPAD + 1, GS = RPAD + 1;
    constexpr bool UPD = MODE != MODE_STORE;
    double *Gs = smem;
    double *Gi = Gs + (UPD ? RPAD * GS : 0);
    double *As = Gi + (UPD ? RPAD : 0);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = wave / WN, wn = wave % WN;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m = J.m, n = J.n, ldm = J.ldm;
    const int r = J.r;
    const int64_t brow = (int64_t)tile * TM;
    const int64_t row0 = brow + wr * TMW;
    const auto Wt = to_global(J.Wt);
    const auto Vg = to_global(J.V);

    const int64_t nsteps = (n + 3) >> 2;
    const int64_t per = (nsteps + WN - 1) / WN;
    const int64_t s_begin = wn * per;
    const int64_t s_end = (s_begin + per < nsteps) ? s_begin + per : nsteps;
    gmem<const float> *Mr[RW];
    bool rok[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int64_t row = row0 + 16 * q + li;
        rok[q] = row < m;
        Mr[q] = to_global(J.M) + (rok[q] ? row : 0);
    }
    v4f hi[RW][RT], lo[RW][RT];
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
        for (int t = 0; t < RT; ++t) hi[q][t] = lo[q][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};

    float a0[S][RW], b0[S][RT], a1[S][RW], b1[S][RT];
    auto load = [&](int64_t s, float (&a)[S][RW], float (&b)[S][RT]) {
#pragma unroll
        for (int u = 0; u < S; ++u) {
            const int64_t j = 4 * (s + u) + lk;
            const bool ok = (s + u) < s_end && j < n;
#pragma unroll
            for (int q = 0; q < RW; ++q) a[u][q] = (ok && rok[q]) ? Mr[q][j * ldm] : 0.0f;
            {
                float w[RT];
                load_wt<RT>(Wt + (ok ? j : 0) * RPAD, li, w);
#pragma unroll
                for (int t = 0; t < RT; ++t) b[u][t] = ok ? w[t] : 0.0f;
            }
        }
    };
    auto compute = [&](const float (&a)[S][RW], const float (&b)[S][RT]) {
#pragma unroll
        for (int u0 = 0; u0 < S; u0 += 4) {      // 4 steps = 16 products per chain
            v4f acc[RW][RT];
#pragma unroll
            for (int q = 0; q < RW; ++q)
#pragma unroll
                for (int t = 0; t < RT; ++t) acc[q][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int u = u0; u < u0 + 4; ++u)
#pragma unroll
                for (int q = 0; q < RW; ++q)
#pragma unroll
                    for (int t = 0; t < RT; ++t)
                        acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][q], b[u][t],
                                                                         acc[q][t], 0, 0, 0);
#pragma unroll
            for (int q = 0; q < RW; ++q)
#pragma unroll
                for (int t = 0; t < RT; ++t) two_sum_acc(hi[q][t], lo[q][t], acc[q][t]);
        }
    };
    // factor rows of the epilogue: 16 lanes per row, rows tid/16 + 16i
    constexpr int EPR = TM / 16;
    double xv[UPD ? EPR : 1][RT];
    if constexpr (UPD) {
#pragma unroll
        for (int i = 0; i < EPR; ++i) {
            const int64_t vrow = brow + (tid >> 4) + 16 * i;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + (tid & 15);
                xv[i][t] = (vrow < m && k < r) ? (double)Vg[vrow + (int64_t)k * m] : 0.0;
            }
        }
    }
    double *Aw = As + wave * TMW * AS;
    if constexpr (!BF) {
        if (s_begin < s_end) load(s_begin, a0, b0);
        // the Gram goes to LDS while the first operand batch is in flight
        if constexpr (UPD) load_gram<RPAD>(J.Bd, r, Gs, GS, Gi);
        for (int64_t s = s_begin; s < s_end; s += 2 * S) {
            if (s + S < s_end) load(s + S, a1, b1);
            compute(a0, b0);
            if (s + S >= s_end) break;
            if (s + 2 * S < s_end) load(s + 2 * S, a0, b0);
            compute(a1, b1);
        }
        // hi[q][t][v] + lo[q][t][v] = A[row0 + 16q + 4*lk + v][16t + li]
#pragma unroll
        for (int q = 0; q < RW; ++q)
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Aw[(16 * q + 4 * lk + v) * AS + 16 * t + li] = (double)hi[q][t][v] + (double)lo[q][t][v];
    } else {
        // BF16 operands (v_mfma_f32_16x16x32_bf16, FP32 accumulation): K-steps of
        // 32 columns; lane (li, lk) supplies row li of a 16-row panel at columns
        // 8*lk..8*lk+7 from the K-packed copy of M (16 bytes), and row 16t + li of
        // W at the same columns from its BF16 copy.
        constexpr int SB = 2;
        const int64_t ksteps = J.npad / 32, kper = (ksteps + WN - 1) / WN;
        const int64_t k_begin = wn * kper;
        const int64_t k_end = (k_begin + kper < ksteps) ? k_begin + kper : ksteps;
        const int64_t G = J.npad / 8;
        gmem<const uint16_t> *Mp[RW];
        bool pok[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const int64_t pr = row0 + 16 * q;          // first row of the panel
            pok[q] = pr < m;
            Mp[q] = to_global(J.Mbp) + (pok[q] ? ((pr / 16) * G * 16 + li) * 8 + lk * 128 : 0);
        }
        gmem<const uint16_t> *Wr[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) Wr[t] = to_global(J.Wb) + (int64_t)(16 * t + li) * J.npad + 8 * lk;
        v4f acc[RW][RT];
#pragma unroll
        for (int q = 0; q < RW; ++q)
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[q][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        bf16x8 ma0[SB][RW], wb0[SB][RT], ma1[SB][RW], wb1[SB][RT];
        const bf16x8 z8 = {};
        auto loadb = [&](int64_t k0, bf16x8 (&a)[SB][RW], bf16x8 (&b)[SB][RT]) {
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int64_t kk = k0 + u;
                const bool ok = kk < k_end;
#pragma unroll
                for (int q = 0; q < RW; ++q)
                    a[u][q] = (ok && pok[q]) ? *(gmem<const bf16x8> *)(Mp[q] + kk * 512) : z8;
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    b[u][t] = ok ? *(gmem<const bf16x8> *)(Wr[t] + 32 * kk) : z8;
            }
        };
        auto computeb = [&](const bf16x8 (&a)[SB][RW], const bf16x8 (&b)[SB][RT]) {
#pragma unroll
            for (int u = 0; u < SB; ++u)
#pragma unroll
                for (int q = 0; q < RW; ++q)
#pragma unroll
                    for (int t = 0; t < RT; ++t)
                        acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][q], b[u][t],
                                                                            acc[q][t], 0, 0, 0);
        };
        if (k_begin < k_end) loadb(k_begin, ma0, wb0);
        if constexpr (UPD) load_gram<RPAD>(J.Bd, r, Gs, GS, Gi);
        for (int64_t k0 = k_begin; k0 < k_end; k0 += 2 * SB) {
            if (k0 + SB < k_end) loadb(k0 + SB, ma1, wb1);
            computeb(ma0, wb0);
            if (k0 + SB >= k_end) break;
            if (k0 + 2 * SB < k_end) loadb(k0 + 2 * SB, ma0, wb0);
            computeb(ma1, wb1);
        }
        // acc[q][t][v] = A[row0 + 16q + 4*lk + v][16t + li]
#pragma unroll
        for (int q = 0; q < RW; ++q)
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Aw[(16 * q + 4 * lk + v) * AS + 16 * t + li] = (double)acc[q][t][v];
    }
    __syncthreads();
    if constexpr (WN > 1) {
        for (int e = tid; e < TM * RPAD; e += 256) {
            const int row = e / RPAD, k = e % RPAD;
            const int g = row / TMW, rr = row % TMW;
            double s = 0.0;
#pragma unroll
            for (int w2 = 0; w2 < WN; ++w2) s += As[((g * WN + w2) * TMW + rr) * AS + k];
            As[(g * WN * TMW + rr) * AS + k] = s;
        }
        __syncthreads();
    }
    auto arow = [&](int row) { return As + ((row / TMW) * WN * TMW + row % TMW) * AS; };

    if constexpr (MODE == MODE_STORE) {
        for (int e = tid; e < TM * r; e += 256) {
            const int rr = e % TM, k = e / TM;
            const int64_t row = brow + rr;
            if (row < m) to_global(J.A)[row + (int64_t)k * m] = (float)arow(rr)[k];
        }
    } else {
#pragma unroll
        for (int i = 0; i < EPR; ++i) {
            const int er = (tid >> 4) + 16 * i, p = tid & 15;
            const int64_t vrow = brow + er;
            double av[RT];
#pragma unroll
            for (int t = 0; t < RT; ++t) av[t] = arow(er)[16 * t + p];
            row_update<RT, MODE>(xv[i], Gs, GS, Gi, av, r, p);
            if (vrow < m) {
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const int k = 16 * t + p;
                    if (k < r) Vg[vrow + (int64_t)k * m] = (float)xv[i][t];
                    // BF16 copy of the new row for the C-pass (k >= r stays 0)
                    if constexpr (BF)
                        to_global(J.Vb)[vrow + (int64_t)k * J.mpad] = bf16_rne((float)xv[i][t]);
                }
            }
        }
    }
}

template <int RT, int RW, int WN, int S, int MODE, bool BF>
__global__ __launch_bounds__(256) void k_apass(const Job *__restrict__ jobs,
                                               const int2 *__restrict__ bmap) {
    extern __shared__ double smem[];
    int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (!bmap) {
        // single problem: XCD x (= block % 8) takes a contiguous range of row
        // tiles, so neighbouring tiles, which share 128-byte lines of M, meet
        // in one L2
        const int per = (J.nA + 7) / 8;
        jt.y = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
        if (jt.y >= J.nA) return;
    }
    if (J.st->stop) return;
    apass_tile<RT, RW, WN, S, MODE, BF>(J, jt.y, smem);
}

// ---------------------------------------------------------------------------
// C-pass tile: (x = 64-column tile of n, y = chunk of m rows).  Each wave owns
// 16 columns; a lane loads 4 consecutive rows of M and of the r columns of V
// (float4 each) and feeds them to 4 MFMAs, so the k-index of MFMA s maps to
// row i0 + 4*(lane/16) + s.  Loads are double buffered two 16-row steps deep.
// The same V registers feed the FP64 MFMAs of the chunk's partial V^T V: its
// upper-triangle 16x16 tiles are spread over the waves of the chunk's tiles.
// ---------------------------------------------------------------------------
template <int RT, int SB, bool BF>
__device__ void cpass_tile(const Job &J, int tx, int ty, int ntx) {
    constexpr int RPAD = RT * 16, DMAX = 3;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lj = lane & 15, lg = lane >> 4;
    const int64_t m = J.m, n = J.n, ldm = J.ldm;
    const int r = J.r;
    const auto V = to_global(J.V);
    const int64_t jb = (int64_t)tx * 64 + wave * 16;
    const int64_t i_begin = (int64_t)ty * J.chunk;
    const int64_t i_end = (i_begin + J.chunk < m) ? i_begin + J.chunk : m;
    const int64_t j = jb + lj;
    const bool jok = j < n;
    const auto Mc = to_global(J.M) + (jok ? j : 0) * ldm;
    const bool vec = ((ldm & 3) == 0) && ((m & 3) == 0) &&
                     (((uintptr_t)J.M & 15) == 0) && (((uintptr_t)V & 15) == 0);
    const int slot = tx * 4 + wave, nslots = ntx * 4;
    int dta[DMAX], dtb[DMAX];
    int nd = 0;
    {
        int idx = 0;
        for (int ta = 0; ta < RT; ++ta)
            for (int tb = ta; tb < RT; ++tb, ++idx)
                if (idx % nslots == slot && nd < DMAX) {
                    dta[nd] = ta;
                    dtb[nd] = tb;
                    ++nd;
                }
    }
    v4f hi[RT], lo[RT];
    v4d dacc[DMAX];
#pragma unroll
    for (int t = 0; t < RT; ++t) hi[t] = lo[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int d = 0; d < DMAX; ++d) dacc[d] = v4d{0.0, 0.0, 0.0, 0.0};

    auto load1 = [&](int64_t i0, v4f &mv, v4f (&vv)[RT]) {
        const int64_t ib = i0 + 4 * lg;
        if (vec && ib + 3 < i_end) {
            mv = jok ? *(gmem<const v4f> *)(Mc + ib) : v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + lj;
                vv[t] = (k < r) ? *(gmem<const v4f> *)(V + ib + (int64_t)k * m)
                                : v4f{0.0f, 0.0f, 0.0f, 0.0f};
            }
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int64_t i = ib + s;
                const bool iok = i < i_end;
                mv[s] = (jok && iok) ? Mc[i] : 0.0f;
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const int k = 16 * t + lj;
                    vv[t][s] = (k < r && iok) ? V[i + (int64_t)k * m] : 0.0f;
                }
            }
        }
    };
    auto load = [&](int64_t i0, v4f (&mv)[SB], v4f (&vv)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) load1(i0 + 16 * u, mv[u], vv[u]);
    };
    auto compute = [&](const v4f (&mvs)[SB], const v4f (&vvs)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            v4f acc[RT];
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(mvs[u][s], vvs[u][t][s], acc[t], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < RT; ++t) two_sum_acc(hi[t], lo[t], acc[t]);
#pragma unroll
            for (int d = 0; d < DMAX; ++d) {
                if (d < nd) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        double va = 0.0, vb = 0.0;
#pragma unroll
                        for (int t = 0; t < RT; ++t) {
                            if (t == dta[d]) va = (double)vvs[u][t][s];
                            if (t == dtb[d]) vb = (double)vvs[u][t][s];
                        }
                        dacc[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(va, vb, dacc[d], 0, 0, 0);
                    }
                }
            }
        }
    };
    if constexpr (!BF) {
        if (i_begin < i_end) {
            v4f m0[SB], m1[SB], v0[SB][RT], v1[SB][RT];
            load(i_begin, m0, v0);
            for (int64_t i0 = i_begin; i0 < i_end; i0 += 32 * SB) {
                const bool more = i0 + 16 * SB < i_end;
                if (more) load(i0 + 16 * SB, m1, v1);
                compute(m0, v0);
                if (!more) break;
                if (i0 + 32 * SB < i_end) load(i0 + 32 * SB, m0, v0);
                compute(m1, v1);
            }
        }
    } else {
        // C on BF16 operands, K-steps of 32 rows (chunks are multiples of 32,
        // the copies are zero past row m): lane (lj, lg) supplies rows
        // i0 + 8*lg..+7 of column j from the column-major BF16 M, and of
        // column 16t + lj from the BF16 V (16 bytes each).
        constexpr int KB = 2;
        const int64_t mp = J.mpad;
        const auto Mb = to_global(J.Mbc) + (jok ? j : 0) * mp + 8 * lg;
        gmem<const uint16_t> *Vr[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) Vr[t] = to_global(J.Vb) + (int64_t)(16 * t + lj) * mp + 8 * lg;
        const bf16x8 z8 = {};
        v4f acc[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        bf16x8 ma0[KB], vb0[KB][RT], ma1[KB], vb1[KB][RT];
        auto loadb = [&](int64_t i0, bf16x8 (&a)[KB], bf16x8 (&b)[KB][RT]) {
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                const int64_t ik = i0 + 32 * u;
                const bool ok = ik < i_end;
                a[u] = (ok && jok) ? *(gmem<const bf16x8> *)(Mb + ik) : z8;
#pragma unroll
                for (int t = 0; t < RT; ++t) b[u][t] = ok ? *(gmem<const bf16x8> *)(Vr[t] + ik) : z8;
            }
        };
        auto computeb = [&](const bf16x8 (&a)[KB], const bf16x8 (&b)[KB][RT]) {
#pragma unroll
            for (int u = 0; u < KB; ++u)
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], b[u][t], acc[t], 0, 0, 0);
        };
        if (i_begin < i_end) {
            loadb(i_begin, ma0, vb0);
            for (int64_t i0 = i_begin; i0 < i_end; i0 += 64 * KB) {
                const bool more = i0 + 32 * KB < i_end;
                if (more) loadb(i0 + 32 * KB, ma1, vb1);
                computeb(ma0, vb0);
                if (!more) break;
                if (i0 + 64 * KB < i_end) loadb(i0 + 64 * KB, ma0, vb0);
                computeb(ma1, vb1);
            }
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) hi[t] = acc[t];
        // D = V^T V partial in FP64 from the FP32 V (waves that own D tiles)
        if (nd > 0) {
            for (int64_t i0 = i_begin; i0 < i_end; i0 += 16) {
#pragma unroll
                for (int d = 0; d < DMAX; ++d) {
                    if (d < nd) {
                        const int ka = 16 * dta[d] + lj, kb = 16 * dtb[d] + lj;
#pragma unroll
                        for (int s2 = 0; s2 < 4; ++s2) {
                            const int64_t i = i0 + 4 * lg + s2;
                            const bool iok = i < i_end;
                            const double va = (iok && ka < r) ? (double)V[i + (int64_t)ka * m] : 0.0;
                            const double vb = (iok && kb < r) ? (double)V[i + (int64_t)kb * m] : 0.0;
                            dacc[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(va, vb, dacc[d], 0, 0, 0);
                        }
                    }
                }
            }
        }
    }
    // hi[t][v] + lo[t][v] = C[k = 16t + lj][j = jb + 4*lg + v]
    const auto out = to_global(J.Cp) + (int64_t)ty * r * n;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int k = 16 * t + lj;
        if (k < r) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t jj = jb + 4 * lg + v;
                if (jj < n) out[(int64_t)k * n + jj] = (double)hi[t][v] + (double)lo[t][v];
            }
        }
    }
    // dacc[d][v] = D[16*dta + 4*v + lg][16*dtb + lj]
    const auto dout = to_global(J.Dp) + (int64_t)ty * RPAD * RPAD;
#pragma unroll
    for (int d = 0; d < DMAX; ++d) {
        if (d < nd) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
                dout[(16 * dta[d] + 4 * v + lg) * RPAD + 16 * dtb[d] + lj] = dacc[d][v];
        }
    }
}

template <int RT, int SB, bool BF>
__global__ __launch_bounds__(256) void k_cpass(const Job *__restrict__ jobs,
                                               const int2 *__restrict__ bmap) {
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    int tx = jt.y % J.nCx, ty = jt.y / J.nCx;
    if (!bmap) {
        // single problem: all column tiles of a row chunk run on one XCD
        // (= block % 8), so the chunk's V rows are read from HBM once
        const int l = (int)(blockIdx.x >> 3);
        ty = (int)(blockIdx.x & 7) + 8 * (l / J.nCx);
        tx = l % J.nCx;
        if (ty >= J.chunks) return;
    }
    if (J.st->stop) return;
    cpass_tile<RT, SB, BF>(J, tx, ty, J.nCx);
}

// ---------------------------------------------------------------------------
// Sum of FP64 Gram partials stored as upper-triangle 16x16 tiles (row stride
// rpad): G[a][b] = sum_p parts[p][min(a,b)][max(a,b)], added in index order.
// which = 0: D from the C-pass partials.  which = 1: B from the W-update
// partials, and tile 0 also assembles the residual of the iteration,
// e^2 = ||M_d||^2 + sum_b rparts[b] (the partials carry <D,B_b> - 2<C_b,W_b>),
// logs rel_err and sets the stop flag.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(const Job *__restrict__ jobs,
                                                const int2 *__restrict__ bmap,
                                                int which) {
    __shared__ double red[4];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (J.st->stop) return;
    const int tile = jt.y;
    const int r = J.r, rpad = J.rpad;
    const int e = tile * 256 + threadIdx.x;
    const double *parts = which ? J.Bp : J.Dp;
    const int nparts = which ? J.nF : J.chunks;   // which 2: W W^T only (start of a solve)
    if (e < r * r) {
        const int a = e / r, b = e % r;
        const int ua = a < b ? a : b, ub = a < b ? b : a;
        const double s = sum_strided(parts + ua * rpad + ub, (int64_t)rpad * rpad, nparts);
        (which ? J.Bd : J.Dd)[e] = s;
    }
    if (which == 1 && tile == 0) {
        double s = 0.0;
        for (int i = threadIdx.x; i < J.nF; i += 256) s += to_global(J.rparts)[i];
        s = block_sum_f64<256>(s, red);
        if (threadIdx.x == 0) {
            DevState *st = J.st;
            const double nm = *J.normM2;
            const double e2 = nm + s;
            const double e2c = e2 > 0.0 ? e2 : 0.0;
            const double rel = nm > 0.0 ? sqrt(e2c / nm) : sqrt(e2c);
            const int idx = st->log_len;
            if (idx < J.log_cap) {
                J.log_rel[idx] = rel;
                J.log_depth[idx] = J.depth;
            }
            st->log_len = idx + 1;
            st->last_rel = rel;
            if (!isfinite(e2)) {
                st->status = NMF_E_NONFINITE;
                st->stop = 1;
            } else if (J.depth == 0 && J.prec == 0 && J.tol > 0.0 && rel <= J.tol) {
                st->stopped = 1;
                st->stop = 1;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// W-update tile: reduce the C partials of 16 columns (fixed order) and update
// those columns of W (and of its transposed copy Wt).  Also emits this
// tile's FP64 partial of B = W W^T (upper-triangle tiles) and the residual
// scalar <D, B_tile> - 2 <C_tile, W_tile>.
// ---------------------------------------------------------------------------
template <int RT, int MODE>
__device__ void cfinal_tile(const Job &J, int tile, double *smem) {
    constexpr int RPAD = RT * 16, GS = RPAD + 1, CS = RPAD + 1;
    constexpr bool UPD = MODE == MODE_HALS || MODE == MODE_MU;
    constexpr bool INIT = MODE == MODE_INIT;     // no C, no update: Wt and W W^T partials
    double *Gs = smem;
    double *Gi = Gs + (UPD ? RPAD * GS : 0);
    double *Cs = Gi + (UPD ? RPAD : 0);
    double *Wn = Cs + (INIT ? 0 : 16 * CS);
    double *red = Wn + (MODE == MODE_STORE ? 0 : 16 * CS);
    const int tid = threadIdx.x;
    const int64_t n = J.n;
    const int r = J.r;
    const int64_t j0 = (int64_t)tile * 16;
    // factor columns of the update: 16 lanes per column, column j0 + tid/16
    double xw[RT];
    if constexpr (MODE != MODE_STORE) {
        const int64_t j = j0 + (tid >> 4);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + (tid & 15);
            xw[t] = (j < n && k < r) ? (double)to_global(J.W)[(int64_t)k * n + j] : 0.0;
        }
    }
    if constexpr (!INIT) {
        for (int e = tid; e < 16 * RPAD; e += 256) {
            const int jj = e & 15, k = e >> 4;
            const int64_t j = j0 + jj;
            double s = 0.0;
            if (k < r && j < n) s = sum_strided(J.Cp + (int64_t)k * n + j, (int64_t)r * n, J.chunks);
            Cs[jj * CS + k] = s;
        }
    }
    if constexpr (UPD) load_gram<RPAD>(J.Dd, r, Gs, GS, Gi);
    if constexpr (!INIT) __syncthreads();
    if constexpr (MODE == MODE_STORE) {
        for (int e = tid; e < 16 * r; e += 256) {
            const int jj = e & 15, k = e >> 4;
            const int64_t j = j0 + jj;
            if (j < n) to_global(J.C)[(int64_t)k * n + j] = (float)Cs[jj * CS + k];
        }
    } else {
        double part_cw = 0.0;
        {
            const int jj = tid >> 4, p = tid & 15;
            const int64_t j = j0 + jj;
            const bool ok = j < n;
            if constexpr (UPD) {
                double cv[RT];
#pragma unroll
                for (int t = 0; t < RT; ++t) cv[t] = Cs[jj * CS + 16 * t + p];
                row_update<RT, MODE>(xw, Gs, GS, Gi, cv, r, p);
            }
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + p;
                const float xf = (ok && k < r) ? (float)xw[t] : 0.0f;
                Wn[jj * CS + k] = (double)xf;
                if (ok) {
                    to_global(J.Wt)[j * RPAD + wt_pos(k, RT)] = xf;
                    if (J.Wb) to_global(J.Wb)[(int64_t)k * J.npad + j] = bf16_rne(xf);   // BF16 mode
                    if (UPD && k < r) {
                        to_global(J.W)[(int64_t)k * n + j] = xf;
                        part_cw += Cs[jj * CS + k] * (double)xf;
                    }
                }
            }
        }
        __syncthreads();
        double part_db = 0.0;
        const auto bout = to_global(J.Bp) + (int64_t)tile * RPAD * RPAD;
        for (int e = tid; e < RPAD * RPAD; e += 256) {
            const int a = e / RPAD, b = e % RPAD;
            if (a <= b) {
                double s = 0.0;
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) s = fma(Wn[jj * CS + a], Wn[jj * CS + b], s);
                bout[a * RPAD + b] = s;
                if constexpr (UPD) part_db += (a == b ? 1.0 : 2.0) * Gs[a * GS + b] * s;
            }
        }
        if constexpr (UPD) {
            const double tot = block_sum_f64<256>(part_db - 2.0 * part_cw, red);
            if (tid == 0) to_global(J.rparts)[tile] = tot;
        }
    }
}

template <int RT, int MODE>
__global__ __launch_bounds__(256) void k_cfinal(const Job *__restrict__ jobs,
                                                const int2 *__restrict__ bmap) {
    extern __shared__ double smem[];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (J.st->stop) return;
    cfinal_tile<RT, MODE>(J, jt.y, smem);
}

__global__ __launch_bounds__(256) void k_make_wt(const float *__restrict__ W, int64_t n, int r,
                                                 int rpad, float *__restrict__ Wt) {
    const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (e >= n * rpad) return;
    const int64_t j = e / rpad;
    const int k = (int)(e % rpad);
    Wt[j * rpad + wt_pos(k, rpad / 16)] = k < r ? W[(int64_t)k * n + j] : 0.0f;
}

__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ rparts, int nparts,
                                                  const double *__restrict__ Dd,
                                                  const double *__restrict__ Bd, int r,
                                                  const double *__restrict__ normM2, int depth,
                                                  double *__restrict__ log_rel,
                                                  int32_t *__restrict__ log_depth, int log_cap,
                                                  DevState *st, double tol) {
    __shared__ double red[4];
    if (st->stop) return;
    const int tid = threadIdx.x;
    double s1 = 0.0, s2 = 0.0;
    for (int i = tid; i < nparts; i += 256) s1 += rparts[i];
    for (int e = tid; e < r * r; e += 256) s2 += Dd[e] * Bd[e];
    s1 = block_sum_f64<256>(s1, red);
    s2 = block_sum_f64<256>(s2, red);
    if (tid == 0) {
        const double nm = normM2[depth];
        const double e2 = nm - 2.0 * s1 + s2;
        const double e2c = e2 > 0.0 ? e2 : 0.0;
        const double rel = nm > 0.0 ? sqrt(e2c / nm) : sqrt(e2c);
        const int idx = st->log_len;
        if (idx < log_cap) {
            log_rel[idx] = rel;
            log_depth[idx] = depth;
        }
        st->log_len = idx + 1;
        st->last_rel = rel;
        if (!isfinite(e2)) {
            st->status = NMF_E_NONFINITE;
            st->stop = 1;
        } else if (depth == 0 && tol > 0.0 && rel <= tol) {
            st->stopped = 1;
            st->stop = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Streaming passes for large levels in BF16 mode (job.stream = 1).
//
// A-pass: a block of 4 waves owns 256 rows; each wave owns 64 rows (four
// 16-row panels) over all of n, so every W operand feeds four MFMAs and no
// partial tiles are combined.  Operands are loaded two 32-column K-steps per
// batch, double buffered.  The wave's A rows then go to a wave-private LDS
// region (FP32) and are updated four at a time: row 16q + 4lk + v over the 16
// lanes of lane group lk, entry 16t + li in lane li (the layout of
// row_update).  The next row group's V entries are loaded while the current
// one is updated.
// ---------------------------------------------------------------------------
template <int RT, int MODE>
__device__ void apass_stream_tile(const Job &J, int tile, double *smem) {
    constexpr int RPAD = RT * 16, GS = RPAD + 1, AS = RPAD + 1, RW = 4, SB = 2;
    float *Gs = reinterpret_cast<float *>(smem);   // FP32 update arithmetic (BF16 mode)
    float *Gi = Gs + RPAD * GS;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m = J.m;
    const int r = J.r;
    const int64_t row0 = (int64_t)tile * 256 + wave * 64;
    // npad is a multiple of 128: ksteps is a multiple of 2 * SB and every load
    // of the loop below is in bounds (panels past m read the last panel; their
    // rows are not written back)
    const int64_t ksteps = J.npad / 32, G = J.npad / 8;
    const int64_t lastp = (m - 1) / 16;
    gmem<const uint16_t> *Mp[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int64_t pr = (row0 + 16 * q) / 16;
        Mp[q] = to_global(J.Mbp) + ((pr < lastp ? pr : lastp) * G * 16 + li) * 8 + lk * 128;
    }
    gmem<const uint16_t> *Wr[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) Wr[t] = to_global(J.Wb) + (int64_t)(16 * t + li) * J.npad + 8 * lk;
    v4f acc[RW][RT];
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[q][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 a0[SB][RW], b0[SB][RT], a1[SB][RW], b1[SB][RT];
    auto load = [&](int64_t k0, bf16x8 (&a)[SB][RW], bf16x8 (&b)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int64_t kk = k0 + u;
#pragma unroll
            for (int q = 0; q < RW; ++q) a[u][q] = *(gmem<const bf16x8> *)(Mp[q] + kk * 512);
#pragma unroll
            for (int t = 0; t < RT; ++t) b[u][t] = *(gmem<const bf16x8> *)(Wr[t] + 32 * kk);
        }
    };
    auto compute = [&](const bf16x8 (&a)[SB][RW], const bf16x8 (&b)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u)
#pragma unroll
            for (int q = 0; q < RW; ++q)
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][q], b[u][t], acc[q][t],
                                                                        0, 0, 0);
    };
    load(0, a0, b0);
    load_gram<RPAD, float>(J.Bd, r, Gs, GS, Gi);
    int64_t k0 = 0;
    for (; k0 + 2 * SB < ksteps; k0 += 2 * SB) {
        load(k0 + SB, a1, b1);
        compute(a0, b0);
        load(k0 + 2 * SB, a0, b0);
        compute(a1, b1);
    }
    load(k0 + SB, a1, b1);
    compute(a0, b0);
    compute(a1, b1);
    float *Aw = Gi + RPAD + wave * 64 * AS;
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) Aw[(16 * q + 4 * lk + v) * AS + 16 * t + li] = acc[q][t][v];
    __syncthreads();   // Gram and A rows in LDS
    auto load_x = [&](int g, float (&x)[RT]) {
        const int64_t row = row0 + 16 * (g >> 2) + 4 * lk + (g & 3);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + li;
            x[t] = (row < m && k < r) ? to_global(J.V)[row + (int64_t)k * m] : 0.0f;
        }
    };
    float xc[RT], xn[RT];
    load_x(0, xc);
#pragma unroll 1
    for (int g = 0; g < RW * 4; ++g) {
        const int q = g >> 2, v = g & 3;
        if (g + 1 < RW * 4) load_x(g + 1, xn);
        float a[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) a[t] = Aw[(16 * q + 4 * lk + v) * AS + 16 * t + li];
        row_update<RT, MODE, float>(xc, Gs, GS, Gi, a, r, li);
        const int64_t row = row0 + 16 * q + 4 * lk + v;
        if (row < m) {
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + li;
                if (k < r) to_global(J.V)[row + (int64_t)k * m] = xc[t];
                to_global(J.Vb)[row + (int64_t)k * J.mpad] = bf16_rne(xc[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) xc[t] = xn[t];
    }
}

template <int RT, int MODE>
__global__ __launch_bounds__(256) void k_apass_stream(const Job *__restrict__ jobs,
                                                      const int2 *__restrict__ bmap) {
    extern __shared__ double smem[];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (jt.y >= J.nA || J.st->stop) return;
    apass_stream_tile<RT, MODE>(J, jt.y, smem);
}

// C-pass: a block of 4 waves owns 256 columns of one row chunk; each wave owns
// 64 columns (four 16-column tiles), so every V operand feeds four MFMAs.  The
// first column block of each chunk also forms the chunk's partial D = V^T V
// from the same V operands (upper-triangle 16x16 tiles spread over its waves).
template <int RT>
__device__ void cpass_stream_tile(const Job &J, int tx, int ty) {
    constexpr int RPAD = RT * 16, RN = 4, SB = 2, DMAX = 3;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lj = lane & 15, lg = lane >> 4;
    const int64_t m = J.m, n = J.n, mp = J.mpad;
    const int r = J.r;
    const int64_t jb = (int64_t)tx * 256 + wave * 64;
    // chunks and mpad are multiples of 128 rows: [i_begin, i_stop) is a whole
    // number of double-buffered pairs of K-steps and every load is in bounds
    // (rows past m are zero; columns past n read column n-1 and are not stored)
    const int64_t i_begin = (int64_t)ty * J.chunk;
    const int64_t i_stop = (i_begin + J.chunk < mp) ? i_begin + J.chunk : mp;
    gmem<const uint16_t> *Mb[RN];
#pragma unroll
    for (int c = 0; c < RN; ++c) {
        const int64_t j = jb + 16 * c + lj;
        Mb[c] = to_global(J.Mbc) + (j < n ? j : n - 1) * mp + 8 * lg;
    }
    gmem<const uint16_t> *Vr[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) Vr[t] = to_global(J.Vb) + (int64_t)(16 * t + lj) * mp + 8 * lg;
    int dta[DMAX], dtb[DMAX], nd = 0;
    if (tx == 0) {
        int idx = 0;
        for (int ta = 0; ta < RT; ++ta)
            for (int tb = ta; tb < RT; ++tb, ++idx)
                if (idx % 4 == wave && nd < DMAX) {
                    dta[nd] = ta;
                    dtb[nd] = tb;
                    ++nd;
                }
    }
    v4f acc[RN][RT], dacc[DMAX];
#pragma unroll
    for (int c = 0; c < RN; ++c)
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[c][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int d = 0; d < DMAX; ++d) dacc[d] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    const bf16x8 z8 = {};
    bf16x8 a0[SB][RN], b0[SB][RT], a1[SB][RN], b1[SB][RT];
    auto load = [&](int64_t i0, bf16x8 (&a)[SB][RN], bf16x8 (&b)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int64_t ik = i0 + 32 * u;
#pragma unroll
            for (int c = 0; c < RN; ++c) a[u][c] = *(gmem<const bf16x8> *)(Mb[c] + ik);
#pragma unroll
            for (int t = 0; t < RT; ++t) b[u][t] = *(gmem<const bf16x8> *)(Vr[t] + ik);
        }
    };
    auto compute = [&](const bf16x8 (&a)[SB][RN], const bf16x8 (&b)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
#pragma unroll
            for (int c = 0; c < RN; ++c)
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][c], b[u][t], acc[c][t],
                                                                        0, 0, 0);
#pragma unroll
            for (int d = 0; d < DMAX; ++d) {
                if (d < nd) {
                    bf16x8 va = z8, vb = z8;
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        if (t == dta[d]) va = b[u][t];
                        if (t == dtb[d]) vb = b[u][t];
                    }
                    dacc[d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, dacc[d], 0, 0, 0);
                }
            }
        }
    };
    if (i_begin < i_stop) {
        load(i_begin, a0, b0);
        int64_t i0 = i_begin;
        for (; i0 + 64 * SB < i_stop; i0 += 64 * SB) {
            load(i0 + 32 * SB, a1, b1);
            compute(a0, b0);
            load(i0 + 64 * SB, a0, b0);
            compute(a1, b1);
        }
        load(i0 + 32 * SB, a1, b1);
        compute(a0, b0);
        compute(a1, b1);
    }
    // acc[c][t][v] = C[k = 16t + lj][j = jb + 16c + 4lg + v]
    const auto out = to_global(J.Cp) + (int64_t)ty * r * n;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int k = 16 * t + lj;
        if (k < r) {
#pragma unroll
            for (int c = 0; c < RN; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t j = jb + 16 * c + 4 * lg + v;
                    if (j < n) out[(int64_t)k * n + j] = (double)acc[c][t][v];
                }
        }
    }
    // dacc[d][v] = D[16 dta + 4lg + v][16 dtb + lj]
    const auto dout = to_global(J.Dp) + (int64_t)ty * RPAD * RPAD;
#pragma unroll
    for (int d = 0; d < DMAX; ++d) {
        if (d < nd) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
                dout[(16 * dta[d] + 4 * lg + v) * RPAD + 16 * dtb[d] + lj] = (double)dacc[d][v];
        }
    }
}

template <int RT>
__global__ __launch_bounds__(256) void k_cpass_stream(const Job *__restrict__ jobs,
                                                      const int2 *__restrict__ bmap) {
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    int tx = jt.y % J.nCx, ty = jt.y / J.nCx;
    if (!bmap) {   // single problem: the column blocks of a chunk run on one XCD
        const int l = (int)(blockIdx.x >> 3);
        ty = (int)(blockIdx.x & 7) + 8 * (l / J.nCx);
        tx = l % J.nCx;
    }
    if (ty >= J.chunks || J.st->stop) return;
    cpass_stream_tile<RT>(J, tx, ty);
}

// ---------------------------------------------------------------------------
// Streaming passes for large levels in FP32 mode (job.stream = 1, prec = 0):
// m >= kStreamMinRows, m and the column stride of M multiples of 4, M 16-byte
// aligned.  FP32 products are MFMA-bound (v_mfma_f32_16x16x4f32), so the
// design keeps the matrix cores busy and M in flight to feed them: batches of
// 4 K-steps, double buffered in registers.
//
// A-pass: a wave owns 32 rows.  Lane (li, lk) loads rows row0 + 2li, 2li + 1
// of column 4ks + lk (8 bytes) and feeds them to two MFMAs, so MFMA s maps its
// row index li to row row0 + 2li + s; its accumulator v of lane (li', lk')
// holds A[row0 + 8lk' + 2v + s][16t + li'].  Every 4 K-steps (16 products per
// chain) the accumulators are added into FP64 sums.  Past n the W operand is
// zero (the M column read is clamped), so no load is conditional.  The V
// update (FP64, as in the regular kernels) takes the wave's rows 4 at a time
// from a wave-private LDS slot, one s at a time.
// ---------------------------------------------------------------------------
template <int RT, int MODE>
__device__ void apass_s32_tile(const Job &J, int tile, double *smem) {
    constexpr int RPAD = RT * 16, GS = RPAD + 1, AS = RPAD + 1, RS = 2, SB = 4;
    typedef float v2f __attribute__((ext_vector_type(2)));
    double *Gs = smem;
    double *Gi = Gs + RPAD * GS;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m = J.m, n = J.n, ldm = J.ldm;
    const int r = J.r;
    const int64_t row0 = (int64_t)tile * 128 + wave * 32;
    const int64_t rl = row0 + 2 * li;
    const auto Mw = to_global(J.M) + (rl < m ? rl : m - 2);
    const auto Wt = to_global(J.Wt);
    const int64_t nsteps = (n + 3) / 4;
    const int64_t nb = (nsteps + SB - 1) / SB;            // batches (last one padded)
    v4f acc[RS][RT];
    double hs[RS][RT][4];
#pragma unroll
    for (int s2 = 0; s2 < RS; ++s2)
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            acc[s2][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int v = 0; v < 4; ++v) hs[s2][t][v] = 0.0;
        }
    v2f a0[SB], a1[SB];
    float b0[SB][RT], b1[SB][RT];
    auto load = [&](int64_t bidx, v2f (&a)[SB], float (&b)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int64_t j = 4 * (bidx * SB + u) + lk;
            const int64_t jc = j < n ? j : n - 1;
            a[u] = *(gmem<const v2f> *)(Mw + jc * ldm);
            float w[RT];
            load_wt<RT>(Wt + jc * RPAD, li, w);
#pragma unroll
            for (int t = 0; t < RT; ++t) b[u][t] = j < n ? w[t] : 0.0f;
        }
    };
    auto compute = [&](const v2f (&a)[SB], const float (&b)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
#pragma unroll
            for (int s2 = 0; s2 < RS; ++s2)
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][s2], b[u][t], acc[s2][t], 0, 0, 0);
            if ((u & 3) == 3) {        // chains of 4 K-steps (16 products) into FP64
#pragma unroll
                for (int s2 = 0; s2 < RS; ++s2)
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) hs[s2][t][v] += (double)acc[s2][t][v];
                        acc[s2][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
                    }
            }
        }
    };
    load(0, a0, b0);
    if constexpr (MODE != MODE_STORE) load_gram<RPAD>(J.Bd, r, Gs, GS, Gi);
    int64_t bi = 0;
    for (; bi + 2 < nb; bi += 2) {
        load(bi + 1, a1, b1);
        compute(a0, b0);
        load(bi + 2, a0, b0);
        compute(a1, b1);
    }
    if (bi + 1 < nb) {
        load(bi + 1, a1, b1);
        compute(a0, b0);
        compute(a1, b1);
    } else {
        compute(a0, b0);
    }
    double *Aw = Gi + RPAD + wave * 16 * AS;   // 16 rows of this wave (one s)
    __syncthreads();                            // Gram in LDS
    auto load_x = [&](int g, double (&x)[RT]) {   // g = 4 s + v: rows row0 + 8lk + 2v + s
        const int64_t row = row0 + 8 * lk + 2 * (g & 3) + (g >> 2);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + li;
            x[t] = (row < m && k < r) ? (double)to_global(J.V)[row + (int64_t)k * m] : 0.0;
        }
    };
    double xc[RT], xn[RT];
    load_x(0, xc);
    static_for<RS>([&](auto s_c) {
        constexpr int s2 = decltype(s_c)::value;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) Aw[(4 * lk + v) * AS + 16 * t + li] = hs[s2][t][v];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 1
        for (int v = 0; v < 4; ++v) {
            const int g = 4 * s2 + v;
            if (g + 1 < RS * 4) load_x(g + 1, xn);
            double a[RT];
#pragma unroll
            for (int t = 0; t < RT; ++t) a[t] = Aw[(4 * lk + v) * AS + 16 * t + li];
            const int64_t row = row0 + 8 * lk + 2 * v + s2;
            if constexpr (MODE == MODE_STORE) {
                if (row < m) {
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        const int k = 16 * t + li;
                        if (k < r) to_global(J.A)[row + (int64_t)k * m] = (float)a[t];
                    }
                }
            } else {
                row_update<RT, MODE>(xc, Gs, GS, Gi, a, r, li);
                if (row < m) {
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        const int k = 16 * t + li;
                        if (k < r) to_global(J.V)[row + (int64_t)k * m] = (float)xc[t];
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < RT; ++t) xc[t] = xn[t];
        }
    });
}

template <int RT, int MODE>
__global__ __launch_bounds__(256) void k_apass_s32(const Job *__restrict__ jobs,
                                                   const int2 *__restrict__ bmap) {
    extern __shared__ double smem[];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (jt.y >= J.nA || J.st->stop) return;
    apass_s32_tile<RT, MODE>(J, jt.y, smem);
}

// C-pass (FP32): a block of 4 waves owns 128 columns of one row chunk; a wave
// owns 32 columns (two 16-column tiles).  Per 16-row step a lane loads 4
// consecutive rows of M (per column tile) and of V (per rank tile) as float4
// and feeds them to 4 MFMAs, whose K index lk maps to row i0 + 4lk + s.  Each
// step's chains (16 products) are added into FP64 sums.  Rows past the chunk
// read a clamped row with a zero V operand.  The first column block of each
// chunk also forms the chunk's V^T V partial on the FP64 matrix cores.
template <int RT>
__device__ void cpass_s32_tile(const Job &J, int tx, int ty) {
    constexpr int RPAD = RT * 16, RN = 2, SB = 2, DMAX = 3;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lj = lane & 15, lg = lane >> 4;
    const int64_t m = J.m, n = J.n, ldm = J.ldm;
    const int r = J.r;
    const auto V = to_global(J.V);
    const int64_t jb = (int64_t)tx * 128 + wave * 32;
    const int64_t i_begin = (int64_t)ty * J.chunk;
    const int64_t i_end = (i_begin + J.chunk < m) ? i_begin + J.chunk : m;
    const int64_t nsteps = (i_end - i_begin + 15) / 16;
    gmem<const float> *Mc[RN];
#pragma unroll
    for (int c = 0; c < RN; ++c) {
        const int64_t j = jb + 16 * c + lj;
        Mc[c] = to_global(J.M) + (j < n ? j : n - 1) * ldm;
    }
    int dta[DMAX], dtb[DMAX], nd = 0;
    if (tx == 0) {
        int idx = 0;
        for (int ta = 0; ta < RT; ++ta)
            for (int tb = ta; tb < RT; ++tb, ++idx)
                if (idx % 4 == wave && nd < DMAX) {
                    dta[nd] = ta;
                    dtb[nd] = tb;
                    ++nd;
                }
    }
    v4f acc[RN][RT];
    double hs[RN][RT][4];
    v4d dacc[DMAX];
#pragma unroll
    for (int c = 0; c < RN; ++c)
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            acc[c][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int v = 0; v < 4; ++v) hs[c][t][v] = 0.0;
        }
#pragma unroll
    for (int d = 0; d < DMAX; ++d) dacc[d] = v4d{0.0, 0.0, 0.0, 0.0};
    v4f ma0[SB][RN], vb0[SB][RT], ma1[SB][RN], vb1[SB][RT];
    auto load = [&](int64_t st0, v4f (&a)[SB][RN], v4f (&b)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int64_t ib = i_begin + 16 * (st0 + u) + 4 * lg;   // rows ib .. ib+3
            const bool ok = ib < i_end;                             // whole groups of 4 (m % 4 == 0)
            const int64_t ic = ok ? ib : i_begin;
#pragma unroll
            for (int c = 0; c < RN; ++c) a[u][c] = *(gmem<const v4f> *)(Mc[c] + ic);
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + lj;
                const v4f x = *(gmem<const v4f> *)(V + ic + (int64_t)(k < r ? k : 0) * m);
                b[u][t] = (ok && k < r) ? x : v4f{0.0f, 0.0f, 0.0f, 0.0f};
            }
        }
    };
    auto compute = [&](const v4f (&a)[SB][RN], const v4f (&b)[SB][RT]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < RN; ++c)
#pragma unroll
                    for (int t = 0; t < RT; ++t)
                        acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][c][s], b[u][t][s], acc[c][t], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < RN; ++c)
#pragma unroll
                for (int t = 0; t < RT; ++t) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) hs[c][t][v] += (double)acc[c][t][v];
                    acc[c][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
                }
#pragma unroll
            for (int d = 0; d < DMAX; ++d) {
                if (d < nd) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        double va = 0.0, vb = 0.0;
#pragma unroll
                        for (int t = 0; t < RT; ++t) {
                            if (t == dta[d]) va = (double)b[u][t][s];
                            if (t == dtb[d]) vb = (double)b[u][t][s];
                        }
                        dacc[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(va, vb, dacc[d], 0, 0, 0);
                    }
                }
            }
        }
    };
    const int64_t nb = (nsteps + SB - 1) / SB;
    if (nb > 0) {
        load(0, ma0, vb0);
        int64_t bi = 0;
        for (; bi + 2 < nb; bi += 2) {
            load(SB * (bi + 1), ma1, vb1);
            compute(ma0, vb0);
            load(SB * (bi + 2), ma0, vb0);
            compute(ma1, vb1);
        }
        if (bi + 1 < nb) {
            load(SB * (bi + 1), ma1, vb1);
            compute(ma0, vb0);
            compute(ma1, vb1);
        } else {
            compute(ma0, vb0);
        }
    }
    // hs[c][t][v] = C[k = 16t + lj][j = jb + 16c + 4lg + v]
    const auto out = to_global(J.Cp) + (int64_t)ty * r * n;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int k = 16 * t + lj;
        if (k < r) {
#pragma unroll
            for (int c = 0; c < RN; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t j = jb + 16 * c + 4 * lg + v;
                    if (j < n) out[(int64_t)k * n + j] = hs[c][t][v];
                }
        }
    }
    // dacc[d][v] = D[16 dta + 4v + lg][16 dtb + lj]  (FP64 MFMA layout)
    const auto dout = to_global(J.Dp) + (int64_t)ty * RPAD * RPAD;
#pragma unroll
    for (int d = 0; d < DMAX; ++d) {
        if (d < nd) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
                dout[(16 * dta[d] + 4 * v + lg) * RPAD + 16 * dtb[d] + lj] = dacc[d][v];
        }
    }
}

template <int RT>
__global__ __launch_bounds__(256) void k_cpass_s32(const Job *__restrict__ jobs,
                                                   const int2 *__restrict__ bmap) {
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    int tx = jt.y % J.nCx, ty = jt.y / J.nCx;
    if (!bmap) {   // single problem: the column blocks of a chunk run on one XCD
        const int l = (int)(blockIdx.x >> 3);
        ty = (int)(blockIdx.x & 7) + 8 * (l / J.nCx);
        tx = l % J.nCx;
    }
    if (ty >= J.chunks || J.st->stop) return;
    cpass_s32_tile<RT>(J, tx, ty);
}

}  // namespace

// ---- host side -------------------------------------------------------------

int apass_rows_per_block(int64_t m) { return m >= 32768 ? 64 : 16; }

size_t apass_lds_bytes(int rpad, int tm, int mode) {
    const bool upd = mode != MODE_STORE;
    const int rw = tm == 16 ? 1 : 2;
    return sizeof(double) * ((upd ? rpad * (rpad + 1) + rpad : 0) + 4 * 16 * rw * (rpad + 1));
}

size_t cfinal_lds_bytes(int rpad, int mode) {
    const bool upd = mode == MODE_HALS || mode == MODE_MU;
    const size_t g = upd ? (size_t)rpad * (rpad + 1) + rpad : 0;     // Gram and 1/G_kk
    const size_t c = mode == MODE_INIT ? 0 : 16 * (size_t)(rpad + 1);  // C rows
    const size_t w = mode == MODE_STORE ? 0 : 16 * (size_t)(rpad + 1); // new W rows
    return sizeof(double) * (g + c + w + 4);
}

// Tile configurations of the A-pass, by rank class and rows per tile: 16-row
// tiles whose 4 waves split n with deep register batches (small m, latency
// bound), or 64-row tiles of two 32-row groups with two waves each (large m).
template <int RT, int MODE, bool BF>
static void apass_launch(int tm, const Job *jobs, const int2 *bmap, int blocks,
                         size_t lds, hipStream_t s) {
    constexpr int S16 = 4;
    constexpr int S64 = 4;
    if (tm == 16) k_apass<RT, 1, 4, S16, MODE, BF><<<blocks, 256, lds, s>>>(jobs, bmap);
    else k_apass<RT, 2, 2, S64, MODE, BF><<<blocks, 256, lds, s>>>(jobs, bmap);
}

template <int RT>
static void apass_launch_mode(int mode, int tm, bool bf, const Job *jobs, const int2 *bmap,
                              int blocks, size_t lds, hipStream_t s) {
    if (bf) {
        if (mode == MODE_HALS) apass_launch<RT, MODE_HALS, true>(tm, jobs, bmap, blocks, lds, s);
        else apass_launch<RT, MODE_MU, true>(tm, jobs, bmap, blocks, lds, s);
    } else if (mode == MODE_HALS) {
        apass_launch<RT, MODE_HALS, false>(tm, jobs, bmap, blocks, lds, s);
    } else if (mode == MODE_MU) {
        apass_launch<RT, MODE_MU, false>(tm, jobs, bmap, blocks, lds, s);
    } else {
        apass_launch<RT, MODE_STORE, false>(tm, jobs, bmap, blocks, lds, s);
    }
}

hipError_t launch_apass_jobs(int mode, int rpad, int tm, const Job *jobs, const int2 *bmap,
                             int blocks, size_t lds, hipStream_t s, bool bf) {
    if (blocks <= 0) return hipSuccess;
    if (bf && mode == MODE_STORE) return hipErrorInvalidValue;
    switch (rpad) {
        case 16: apass_launch_mode<1>(mode, tm, bf, jobs, bmap, blocks, lds, s); break;
        case 32: apass_launch_mode<2>(mode, tm, bf, jobs, bmap, blocks, lds, s); break;
        case 48: apass_launch_mode<3>(mode, tm, bf, jobs, bmap, blocks, lds, s); break;
        case 64: apass_launch_mode<4>(mode, tm, bf, jobs, bmap, blocks, lds, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cpass_jobs(int rpad, const Job *jobs, const int2 *bmap, int blocks,
                             hipStream_t s, bool bf) {
    if (blocks <= 0) return hipSuccess;
    switch (rpad) {
        case 16:
            if (bf) k_cpass<1, 2, true><<<blocks, 256, 0, s>>>(jobs, bmap);
            else k_cpass<1, 2, false><<<blocks, 256, 0, s>>>(jobs, bmap);
            break;
        case 32:
            if (bf) k_cpass<2, 2, true><<<blocks, 256, 0, s>>>(jobs, bmap);
            else k_cpass<2, 2, false><<<blocks, 256, 0, s>>>(jobs, bmap);
            break;
        case 48:
            if (bf) k_cpass<3, 1, true><<<blocks, 256, 0, s>>>(jobs, bmap);
            else k_cpass<3, 1, false><<<blocks, 256, 0, s>>>(jobs, bmap);
            break;
        case 64:
            if (bf) k_cpass<4, 1, true><<<blocks, 256, 0, s>>>(jobs, bmap);
            else k_cpass<4, 1, false><<<blocks, 256, 0, s>>>(jobs, bmap);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_jobs(int which, const Job *jobs, const int2 *bmap, int blocks,
                              hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    k_reduce<<<blocks, 256, 0, s>>>(jobs, bmap, which);
    return hipGetLastError();
}

template <int RT>
static void cfinal_launch(int mode, const Job *jobs, const int2 *bmap, int blocks,
                          size_t lds, hipStream_t s) {
    if (mode == MODE_HALS) k_cfinal<RT, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap);
    else if (mode == MODE_MU) k_cfinal<RT, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap);
    else if (mode == MODE_INIT) k_cfinal<RT, MODE_INIT><<<blocks, 256, lds, s>>>(jobs, bmap);
    else k_cfinal<RT, MODE_STORE><<<blocks, 256, lds, s>>>(jobs, bmap);
}

hipError_t launch_cfinal_jobs(int mode, int rpad, const Job *jobs, const int2 *bmap,
                              int blocks, size_t lds, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    switch (rpad) {
        case 16: cfinal_launch<1>(mode, jobs, bmap, blocks, lds, s); break;
        case 32: cfinal_launch<2>(mode, jobs, bmap, blocks, lds, s); break;
        case 48: cfinal_launch<3>(mode, jobs, bmap, blocks, lds, s); break;
        case 64: cfinal_launch<4>(mode, jobs, bmap, blocks, lds, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_make_wt(const float *W, int64_t n, int r, int rpad, float *Wt, hipStream_t s) {
    const int64_t total = n * rpad;
    if (total == 0) return hipSuccess;
    k_make_wt<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(W, n, r, rpad, Wt);
    return hipGetLastError();
}

hipError_t launch_residual(const double *rparts, int nparts, const double *Dd, const double *Bd,
                           int r, const double *normM2, int depth, double *log_rel,
                           int32_t *log_depth, int log_cap, DevState *st, double tol,
                           hipStream_t s) {
    k_residual<<<1, 256, 0, s>>>(rparts, nparts, Dd, Bd, r, normM2, depth, log_rel, log_depth,
                                 log_cap, st, tol);
    return hipGetLastError();
}

int cpass_final_blocks(int64_t n) { return (int)((n + 15) / 16); }

int apass_grid_single(int nA) { return 8 * ((nA + 7) / 8); }

int cpass_stream_grid(int nCx, int chunks) { return 8 * nCx * ((chunks + 7) / 8); }

// FP64 Gram and 1/G_kk, then 4 waves x 16 rows of A (FP64, stride rpad + 1).
size_t apass_s32_lds_bytes(int rpad) {
    return sizeof(double) * ((size_t)rpad * (rpad + 1) + rpad + 4 * 16 * (size_t)(rpad + 1));
}

hipError_t launch_apass_s32(int mode, int rpad, const Job *jobs, const int2 *bmap, int blocks,
                            hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (mode != MODE_HALS && mode != MODE_MU) return hipErrorInvalidValue;
    const size_t lds = apass_s32_lds_bytes(rpad);
    const bool h = mode == MODE_HALS;
    switch (rpad) {
        case 16: h ? k_apass_s32<1, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_apass_s32<1, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 32: h ? k_apass_s32<2, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_apass_s32<2, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 48: h ? k_apass_s32<3, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_apass_s32<3, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 64: h ? k_apass_s32<4, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_apass_s32<4, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cpass_s32(int rpad, const Job *jobs, const int2 *bmap, int blocks,
                            hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    switch (rpad) {
        case 16: k_cpass_s32<1><<<blocks, 256, 0, s>>>(jobs, bmap); break;
        case 32: k_cpass_s32<2><<<blocks, 256, 0, s>>>(jobs, bmap); break;
        case 48: k_cpass_s32<3><<<blocks, 256, 0, s>>>(jobs, bmap); break;
        case 64: k_cpass_s32<4><<<blocks, 256, 0, s>>>(jobs, bmap); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Gram and 1/G_kk, then 4 waves x 64 rows of A (all FP32, stride rpad + 1).
size_t apass_stream_lds_bytes(int rpad) {
    return sizeof(float) * ((size_t)rpad * (rpad + 1) + rpad) +
           sizeof(float) * 4 * 64 * (size_t)(rpad + 1);
}

hipError_t launch_apass_stream(int mode, int rpad, const Job *jobs, const int2 *bmap, int blocks,
                               hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (mode != MODE_HALS && mode != MODE_MU) return hipErrorInvalidValue;
    const size_t lds = apass_stream_lds_bytes(rpad);
    const bool h = mode == MODE_HALS;
    switch (rpad) {
        case 16: h ? k_apass_stream<1, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_apass_stream<1, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 32: h ? k_apass_stream<2, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_apass_stream<2, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 48: h ? k_apass_stream<3, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_apass_stream<3, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 64: h ? k_apass_stream<4, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_apass_stream<4, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cpass_stream(int rpad, const Job *jobs, const int2 *bmap, int blocks,
                               hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    switch (rpad) {
        case 16: k_cpass_stream<1><<<blocks, 256, 0, s>>>(jobs, bmap); break;
        case 32: k_cpass_stream<2><<<blocks, 256, 0, s>>>(jobs, bmap); break;
        case 48: k_cpass_stream<3><<<blocks, 256, 0, s>>>(jobs, bmap); break;
        case 64: k_cpass_stream<4><<<blocks, 256, 0, s>>>(jobs, bmap); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int cpass_grid_single(int nCx, int chunks) { return 8 * nCx * ((chunks + 7) / 8); }

// Allow the sweep kernels the LDS sizes apass_lds_bytes / cfinal_lds_bytes
// can ask for (above the 64 KB default).
template <int RT, int MODE>
static void lds_attr(hipError_t &e) {
    constexpr int S16 = 4;
    constexpr int S64 = 4;
    const int bytes = 160 * 1024;
    auto set = [&](const void *f) {
        hipError_t x = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (x != hipSuccess && e == hipSuccess) e = x;
    };
    set((const void *)k_apass<RT, 1, 4, S16, MODE, false>);
    set((const void *)k_apass<RT, 2, 2, S64, MODE, false>);
    if constexpr (MODE != MODE_STORE) {
        set((const void *)k_apass<RT, 1, 4, S16, MODE, true>);
        set((const void *)k_apass<RT, 2, 2, S64, MODE, true>);
    }
    set((const void *)k_cfinal<RT, MODE>);
}

template <int RT>
static void lds_attr_modes(hipError_t &e) {
    lds_attr<RT, MODE_HALS>(e);
    lds_attr<RT, MODE_MU>(e);
    lds_attr<RT, MODE_STORE>(e);
    hipError_t x = hipFuncSetAttribute((const void *)k_cfinal<RT, MODE_INIT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (x != hipSuccess && e == hipSuccess) e = x;
    for (const void *f : {(const void *)k_apass_stream<RT, MODE_HALS>,
                          (const void *)k_apass_stream<RT, MODE_MU>,
                          (const void *)k_apass_s32<RT, MODE_HALS>,
                          (const void *)k_apass_s32<RT, MODE_MU>}) {
        x = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (x != hipSuccess && e == hipSuccess) e = x;
    }
}

hipError_t enable_large_lds() {
    static hipError_t done = [] {
        hipError_t e = hipSuccess;
        lds_attr_modes<1>(e);
        lds_attr_modes<2>(e);
        lds_attr_modes<3>(e);
        lds_attr_modes<4>(e);
        return e;
    }();
    return done;
}

}  // namespace nmf
