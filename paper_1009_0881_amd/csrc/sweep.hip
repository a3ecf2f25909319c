// One NMF iteration on one level: the two M-streaming products and the
// factor updates of Alg. 2 (MU) and Alg. 3 (HALS), plus the residual.
//
//   k_apass          A = M W^T (m x r), V update fused as epilogue
//   k_cpass_partial  split-m partials of C = V^T M, and of D = V^T V (FP64)
//   k_reduce_gram    D = sum of partials (fixed order)
//   k_cpass_final    C = sum of partials, W update, partials of W W^T and of
//                    the residual terms
//   k_reduce_gram    B = W W^T, plus rel_err = sqrt(||M||^2 - 2<C,W> + <D,B>)/||M||
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
// Factor updates: one factor row (a row of V, or a column of W) is owned by 4
// consecutive lanes, lane q holding the entries k = q (mod 4).  HALS walks
// k = 1..r in order using already-updated entries (Gauss-Seidel, Alg. 3);
// MU updates all entries from the old values (Alg. 2).

#include "device_common.h"
#include "nmf_internal.h"

namespace nmf {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int MODE_HALS = 0, MODE_MU = 1, MODE_STORE = 2;

// HALS / MU update of one factor row held by 4 lanes.  G is the r x r FP64
// Gram of the other factor in LDS (row stride gs, zero-padded to RPAD), gi[k]
// = 1/G_kk (0 when G_kk = 0), a[k] the matching row of the product (FP64,
// LDS).  The r x r-sized update arithmetic runs in FP64 (the numerator
// a_k - sum_l x_l G_lk cancels as the iterate converges); the row is read
// from and written back to FP32 storage.
//   HALS: x_k <- max(0, (a_k - sum_{l != k} x_l G_lk) / G_kk); G_kk = 0 keeps x_k.
//   MU:   x_k <- x_k a_k / (sum_l x_l G_lk); a zero denominator keeps x_k.
template <int RPAD, int MODE>
__device__ __forceinline__ void row_update(double (&x)[RPAD / 4], const double *G, int gs,
                                           const double *gi, const double *a, int r, int q) {
    if constexpr (MODE == MODE_HALS) {
#pragma unroll
        for (int k = 0; k < RPAD; ++k) {
            if (k < r) {
                double s = 0.0;
#pragma unroll
                for (int jj = 0; jj < RPAD / 4; ++jj) {
                    const int l = 4 * jj + q;
                    if (l != k) s = fma(x[jj], G[l * gs + k], s);
                }
                s += __shfl_xor(s, 1, kWave);
                s += __shfl_xor(s, 2, kWave);
                const double inv = gi[k];
                if (inv > 0.0) {
                    const double nv = fmax(0.0, (a[k] - s) * inv);
                    if (q == (k & 3)) x[k >> 2] = nv;
                }
            }
        }
    } else {
        double nx[RPAD / 4];
#pragma unroll
        for (int jj = 0; jj < RPAD / 4; ++jj) nx[jj] = x[jj];
#pragma unroll
        for (int k = 0; k < RPAD; ++k) {
            if (k < r) {
                double den = 0.0;
#pragma unroll
                for (int jj = 0; jj < RPAD / 4; ++jj) den = fma(x[jj], G[(4 * jj + q) * gs + k], den);
                den += __shfl_xor(den, 1, kWave);
                den += __shfl_xor(den, 2, kWave);
                if (q == (k & 3) && den > 0.0) nx[k >> 2] = x[k >> 2] * a[k] / den;
            }
        }
#pragma unroll
        for (int jj = 0; jj < RPAD / 4; ++jj) x[jj] = nx[jj];
    }
}

// Load an r x r FP64 Gram (row-major, stride r) into LDS zero-padded to
// RPAD x RPAD (stride gs), and its inverse diagonal.
template <int RPAD>
__device__ __forceinline__ void load_gram(const double *__restrict__ Gd, int r, double *Gs, int gs,
                                          double *gi) {
    for (int e = threadIdx.x; e < RPAD * RPAD; e += blockDim.x) {
        const int a = e / RPAD, b = e % RPAD;
        Gs[a * gs + b] = (a < r && b < r) ? Gd[a * r + b] : 0.0;
    }
    for (int k = threadIdx.x; k < RPAD; k += blockDim.x) {
        const double g = (k < r) ? Gd[k * r + k] : 0.0;
        gi[k] = g > 0.0 ? 1.0 / g : 0.0;
    }
}

// ---------------------------------------------------------------------------
// A-pass.  Block = 4 waves; the waves form WR = 4/WN row groups of RW 16-row
// tiles each, and the WN waves of a row group split the n columns into
// contiguous ranges.  M (column j of a 16-row tile: 16 consecutive floats) and
// the transposed factor Wt (n x RPAD, row j = column j of W) are loaded
// straight into registers, four 4-column steps at a time, double buffered.
// The WN partial tiles are added in LDS (fixed order) before the epilogue.
// ---------------------------------------------------------------------------
template <int RT, int RW, int WN, int MODE>
__global__ __launch_bounds__(256) void k_apass(const float *__restrict__ M, int64_t ldm,
                                               int64_t m, int64_t n,
                                               const float *__restrict__ Wt,
                                               const double *__restrict__ Bd,
                                               float *__restrict__ V, float *__restrict__ Aout,
                                               int r, const int32_t *stop) {
    constexpr int RPAD = RT * 16, WR = 4 / WN, TMW = 16 * RW, TM = TMW * WR;
    constexpr int AS = RPAD + 1, GS = RPAD + 1;
    constexpr bool UPD = MODE != MODE_STORE;
    __shared__ double Gs[UPD ? RPAD * GS : 1];
    __shared__ double Gi[UPD ? RPAD : 1];
    __shared__ double As[4 * TMW * AS];
    if (stopped(stop)) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = wave / WN, wn = wave % WN;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t brow = (int64_t)blockIdx.x * TM;
    const int64_t row0 = brow + wr * TMW;
    if constexpr (UPD) load_gram<RPAD>(Bd, r, Gs, GS, Gi);

    const int64_t nsteps = (n + 3) >> 2;
    const int64_t per = (nsteps + WN - 1) / WN;
    const int64_t s_begin = wn * per;
    const int64_t s_end = (s_begin + per < nsteps) ? s_begin + per : nsteps;
    const float *Mr[RW];
    bool rok[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int64_t row = row0 + 16 * q + li;
        rok[q] = row < m;
        Mr[q] = M + (rok[q] ? row : 0);
    }
    v4f hi[RW][RT], lo[RW][RT];
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
        for (int t = 0; t < RT; ++t) hi[q][t] = lo[q][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};

    float a0[4][RW], b0[4][RT], a1[4][RW], b1[4][RT];
    auto load = [&](int64_t s, float (&a)[4][RW], float (&b)[4][RT]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = 4 * (s + u) + lk;
            const bool ok = (s + u) < s_end && j < n;
#pragma unroll
            for (int q = 0; q < RW; ++q) a[u][q] = (ok && rok[q]) ? Mr[q][j * ldm] : 0.0f;
#pragma unroll
            for (int t = 0; t < RT; ++t) b[u][t] = ok ? Wt[j * RPAD + 16 * t + li] : 0.0f;
        }
    };
    auto compute = [&](const float (&a)[4][RW], const float (&b)[4][RT]) {
        v4f acc[RW][RT];
#pragma unroll
        for (int q = 0; q < RW; ++q)
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[q][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < RW; ++q)
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][q], b[u][t], acc[q][t], 0, 0, 0);
#pragma unroll
        for (int q = 0; q < RW; ++q)
#pragma unroll
            for (int t = 0; t < RT; ++t) two_sum_acc(hi[q][t], lo[q][t], acc[q][t]);
    };
    if (s_begin < s_end) {
        load(s_begin, a0, b0);
        for (int64_t s = s_begin; s < s_end; s += 8) {
            load(s + 4, a1, b1);
            compute(a0, b0);
            if (s + 4 >= s_end) break;
            load(s + 8, a0, b0);
            compute(a1, b1);
        }
    }
    // hi[q][t][v] + lo[q][t][v] = A[row0 + 16q + 4*lk + v][16t + li]
    double *Aw = As + wave * TMW * AS;
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Aw[(16 * q + 4 * lk + v) * AS + 16 * t + li] = (double)hi[q][t][v] + (double)lo[q][t][v];
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
            if (row < m) Aout[row + (int64_t)k * m] = (float)arow(rr)[k];
        }
    } else {
        if (tid < 4 * TM) {
            const int er = tid >> 2, q = tid & 3;
            const int64_t vrow = brow + er;
            const bool ok = vrow < m;
            double x[RPAD / 4];
#pragma unroll
            for (int jj = 0; jj < RPAD / 4; ++jj) {
                const int k = 4 * jj + q;
                x[jj] = (ok && k < r) ? (double)V[vrow + (int64_t)k * m] : 0.0;
            }
            row_update<RPAD, MODE>(x, Gs, GS, Gi, arow(er), r, q);
#pragma unroll
            for (int jj = 0; jj < RPAD / 4; ++jj) {
                const int k = 4 * jj + q;
                if (ok && k < r) V[vrow + (int64_t)k * m] = (float)x[jj];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// C-pass partials: block (x = 64-column tile of n, y = chunk of m rows).
// Each wave owns 16 columns; a lane loads 4 consecutive rows of M and of the
// r columns of V (float4 each) and feeds them to 4 MFMAs, so the k-index of
// MFMA s maps to row i0 + 4*(lane/16) + s.  Loads are double buffered.
// The same V registers feed the FP64 MFMAs of the chunk's partial V^T V: its
// upper-triangle 16x16 tiles are spread over the waves of the chunk's blocks.
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(256) void k_cpass_partial(const float *__restrict__ M, int64_t ldm,
                                                       int64_t m, int64_t n,
                                                       const float *__restrict__ V, int r,
                                                       int64_t chunk, double *__restrict__ Cp,
                                                       double *__restrict__ Dp,
                                                       const int32_t *stop) {
    constexpr int RPAD = RT * 16, DMAX = 3;
    if (stopped(stop)) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lj = lane & 15, lg = lane >> 4;
    const int64_t jb = (int64_t)blockIdx.x * 64 + wave * 16;
    const int64_t i_begin = (int64_t)blockIdx.y * chunk;
    const int64_t i_end = (i_begin + chunk < m) ? i_begin + chunk : m;
    const int64_t j = jb + lj;
    const bool jok = j < n;
    const float *Mc = M + (jok ? j : 0) * ldm;
    const bool vec = ((ldm & 3) == 0) && ((m & 3) == 0) &&
                     (((uintptr_t)M & 15) == 0) && (((uintptr_t)V & 15) == 0);
    // Gram tiles owned by this wave: tile indices slot, slot + nslots, ...
    const int slot = blockIdx.x * 4 + wave, nslots = gridDim.x * 4;
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

    auto load = [&](int64_t i0, v4f &mv, v4f (&vv)[RT]) {
        const int64_t ib = i0 + 4 * lg;
        if (vec && ib + 3 < i_end) {
            mv = jok ? *(const v4f *)(Mc + ib) : v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + lj;
                vv[t] = (k < r) ? *(const v4f *)(V + ib + (int64_t)k * m)
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
    auto compute = [&](const v4f &mv, const v4f (&vv)[RT]) {
        v4f acc[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(mv[s], vv[t][s], acc[t], 0, 0, 0);
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
                        if (t == dta[d]) va = (double)vv[t][s];
                        if (t == dtb[d]) vb = (double)vv[t][s];
                    }
                    dacc[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(va, vb, dacc[d], 0, 0, 0);
                }
            }
        }
    };
    if (i_begin < i_end) {
        v4f m0, m1, v0[RT], v1[RT];
        load(i_begin, m0, v0);
        for (int64_t i0 = i_begin; i0 < i_end; i0 += 32) {
            const bool more = i0 + 16 < i_end;
            if (more) load(i0 + 16, m1, v1);
            compute(m0, v0);
            if (!more) break;
            if (i0 + 32 < i_end) load(i0 + 32, m0, v0);
            compute(m1, v1);
        }
    }
    // hi[t][v] + lo[t][v] = C[k = 16t + lj][j = jb + 4*lg + v]
    double *out = Cp + (int64_t)blockIdx.y * r * n;
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
    double *dout = Dp + (int64_t)blockIdx.y * RPAD * RPAD;
#pragma unroll
    for (int d = 0; d < DMAX; ++d) {
        if (d < nd) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
                dout[(16 * dta[d] + 4 * v + lg) * RPAD + 16 * dtb[d] + lj] = dacc[d][v];
        }
    }
}

// ---------------------------------------------------------------------------
// Sum of FP64 Gram partials stored as upper-triangle 16x16 tiles (row stride
// rpad): G[a][b] = sum_p parts[p][min(a,b)][max(a,b)], added in index order.
// With `resid` set, block 0 also assembles the residual of the iteration:
// e^2 = ||M_d||^2 + sum_b rparts[b] (the partials carry <D, B_b> - 2 <C_b, W_b>).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_gram(const double *__restrict__ parts, int nparts,
                                                     int rpad, int r, double *__restrict__ Gd,
                                                     int resid, const double *__restrict__ rparts,
                                                     int nr, const double *__restrict__ normM2,
                                                     int depth, double *__restrict__ log_rel,
                                                     int32_t *__restrict__ log_depth, int log_idx,
                                                     int log_cap, DevState *st, double tol) {
    __shared__ double red[4];
    if (st->stop) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < r * r) {
        const int a = e / r, b = e % r;
        const int ua = a < b ? a : b, ub = a < b ? b : a;
        const double *p0 = parts + ua * rpad + ub;
        const int64_t stride = (int64_t)rpad * rpad;
        double s = 0.0;
        int p = 0;
        for (; p + 8 <= nparts; p += 8) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = p0[(p + u) * stride];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += t[u];
        }
        for (; p < nparts; ++p) s += p0[p * stride];
        Gd[e] = s;
    }
    if (resid && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nr; i += 256) s += rparts[i];
        s = block_sum_f64<256>(s, red);
        if (threadIdx.x == 0) {
            const double nm = normM2[depth];
            const double e2 = nm + s;
            const double e2c = e2 > 0.0 ? e2 : 0.0;
            const double rel = nm > 0.0 ? sqrt(e2c / nm) : sqrt(e2c);
            if (log_idx < log_cap) {
                log_rel[log_idx] = rel;
                log_depth[log_idx] = depth;
            }
            st->log_len = log_idx + 1;
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
}

// ---------------------------------------------------------------------------
// Reduce the C partials of 16 columns (fixed order) and update those columns
// of W (and of its transposed copy Wt).  Also emits this block's FP64 partial
// of B = W W^T (upper-triangle tiles) and the residual scalar
// <D, B_block> - 2 <C_block, W_block>.
// ---------------------------------------------------------------------------
template <int RT, int MODE>
__global__ __launch_bounds__(256) void k_cpass_final(const double *__restrict__ Cp, int chunks,
                                                     int64_t n, int r,
                                                     const double *__restrict__ Dd,
                                                     float *__restrict__ W, float *__restrict__ Wt,
                                                     float *__restrict__ Cout,
                                                     double *__restrict__ Bp,
                                                     double *__restrict__ rparts,
                                                     const int32_t *stop) {
    constexpr int RPAD = RT * 16, GS = RPAD + 1, CS = RPAD + 1;
    constexpr bool UPD = MODE != MODE_STORE;
    __shared__ double Gs[UPD ? RPAD * GS : 1];
    __shared__ double Gi[UPD ? RPAD : 1];
    __shared__ double Cs[16 * CS];
    __shared__ double Wn[UPD ? 16 * CS : 1];
    __shared__ double red[4];
    if (stopped(stop)) return;
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * 16;
    if constexpr (UPD) load_gram<RPAD>(Dd, r, Gs, GS, Gi);
    for (int e = tid; e < 16 * RPAD; e += 256) {
        const int jj = e & 15, k = e >> 4;
        const int64_t j = j0 + jj;
        double s = 0.0;
        if (k < r && j < n) {
            const double *p0 = Cp + (int64_t)k * n + j;
            const int64_t stride = (int64_t)r * n;
            int p = 0;
            for (; p + 8 <= chunks; p += 8) {
                double t[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) t[u] = p0[(p + u) * stride];
#pragma unroll
                for (int u = 0; u < 8; ++u) s += t[u];
            }
            for (; p < chunks; ++p) s += p0[p * stride];
        }
        Cs[jj * CS + k] = s;
    }
    __syncthreads();
    if constexpr (MODE == MODE_STORE) {
        for (int e = tid; e < 16 * r; e += 256) {
            const int jj = e & 15, k = e >> 4;
            const int64_t j = j0 + jj;
            if (j < n) Cout[(int64_t)k * n + j] = (float)Cs[jj * CS + k];
        }
    } else {
        double part_cw = 0.0;
        if (tid < 64) {
            const int jj = tid >> 2, q = tid & 3;
            const int64_t j = j0 + jj;
            const bool ok = j < n;
            double x[RPAD / 4];
#pragma unroll
            for (int t = 0; t < RPAD / 4; ++t) {
                const int k = 4 * t + q;
                x[t] = (ok && k < r) ? (double)W[(int64_t)k * n + j] : 0.0;
            }
            row_update<RPAD, MODE>(x, Gs, GS, Gi, Cs + jj * CS, r, q);
#pragma unroll
            for (int t = 0; t < RPAD / 4; ++t) {
                const int k = 4 * t + q;
                const float xf = (ok && k < r) ? (float)x[t] : 0.0f;
                Wn[jj * CS + k] = (double)xf;
                if (ok) {
                    Wt[j * RPAD + k] = xf;
                    if (k < r) {
                        W[(int64_t)k * n + j] = xf;
                        part_cw += Cs[jj * CS + k] * (double)xf;
                    }
                }
            }
        }
        __syncthreads();
        double part_db = 0.0;
        double *bout = Bp + (int64_t)blockIdx.x * RPAD * RPAD;
        for (int e = tid; e < RPAD * RPAD; e += 256) {
            const int a = e / RPAD, b = e % RPAD;
            if (a <= b) {
                double s = 0.0;
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) s = fma(Wn[jj * CS + a], Wn[jj * CS + b], s);
                bout[a * RPAD + b] = s;
                part_db += (a == b ? 1.0 : 2.0) * Gs[a * GS + b] * s;
            }
        }
        const double tot = block_sum_f64<256>(part_db - 2.0 * part_cw, red);
        if (tid == 0) rparts[blockIdx.x] = tot;
    }
}

__global__ __launch_bounds__(256) void k_make_wt(const float *__restrict__ W, int64_t n, int r,
                                                 int rpad, float *__restrict__ Wt) {
    const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (e >= n * rpad) return;
    const int64_t j = e / rpad;
    const int k = (int)(e % rpad);
    Wt[e] = k < r ? W[(int64_t)k * n + j] : 0.0f;
}

__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ rparts, int nparts,
                                                  const double *__restrict__ Dd,
                                                  const double *__restrict__ Bd, int r,
                                                  const double *__restrict__ normM2, int depth,
                                                  double *__restrict__ log_rel,
                                                  int32_t *__restrict__ log_depth, int log_idx,
                                                  int log_cap, DevState *st, double tol) {
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
        if (log_idx < log_cap) {
            log_rel[log_idx] = rel;
            log_depth[log_idx] = depth;
        }
        st->log_len = log_idx + 1;
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

template <int RT, int RW, int WN>
void apass_launch(int mode, int grid, hipStream_t s, const float *M, int64_t ldm, int64_t m,
                  int64_t n, const float *Wt, const double *Bd, float *V, float *Aout, int r,
                  const int32_t *stop) {
    if (mode == MODE_HALS)
        k_apass<RT, RW, WN, MODE_HALS><<<grid, 256, 0, s>>>(M, ldm, m, n, Wt, Bd, V, Aout, r, stop);
    else if (mode == MODE_MU)
        k_apass<RT, RW, WN, MODE_MU><<<grid, 256, 0, s>>>(M, ldm, m, n, Wt, Bd, V, Aout, r, stop);
    else
        k_apass<RT, RW, WN, MODE_STORE><<<grid, 256, 0, s>>>(M, ldm, m, n, Wt, Bd, V, Aout, r, stop);
}

}  // namespace

int cpass_final_blocks(int64_t n) { return (int)((n + 15) / 16); }

// Rows per A-pass block: 16-row blocks whose 4 waves split n for small m (the
// sweep is latency bound there), 64-row blocks of two 32-row groups with two
// waves each for large m (more reuse of each loaded W value).
int apass_rows_per_block(int64_t m) { return m >= 32768 ? 64 : 16; }

#define NMF_DISPATCH_RT(rpad, MACRO) \
    switch (rpad) {                  \
        case 16: MACRO(1); break;    \
        case 32: MACRO(2); break;    \
        case 48: MACRO(3); break;    \
        case 64: MACRO(4); break;    \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_apass(int rpad, int mode, const float *M, int64_t ldm, int64_t m, int64_t n,
                        const float *Wt, const double *Bd, float *V, float *Aout, int r,
                        const int32_t *stop, hipStream_t s) {
    const int tm = apass_rows_per_block(m);
    const int grid = (int)((m + tm - 1) / tm);
    if (grid == 0) return hipSuccess;
#define L_APASS(RT)                                                                              \
    if (tm == 16) apass_launch<RT, 1, 4>(mode, grid, s, M, ldm, m, n, Wt, Bd, V, Aout, r, stop); \
    else apass_launch<RT, 2, 2>(mode, grid, s, M, ldm, m, n, Wt, Bd, V, Aout, r, stop);
    NMF_DISPATCH_RT(rpad, L_APASS)
#undef L_APASS
    return hipGetLastError();
}

hipError_t launch_cpass_partial(int rpad, const float *M, int64_t ldm, int64_t m, int64_t n,
                                const float *V, int r, int chunks, int64_t chunk, double *Cp,
                                double *Dp, const int32_t *stop, hipStream_t s) {
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)chunks);
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
#define L_CPART(RT) \
    k_cpass_partial<RT><<<grid, 256, 0, s>>>(M, ldm, m, n, V, r, chunk, Cp, Dp, stop);
    NMF_DISPATCH_RT(rpad, L_CPART)
#undef L_CPART
    return hipGetLastError();
}

hipError_t launch_reduce_gram(const double *parts, int nparts, int rpad, int r, double *Gd,
                              bool resid, const double *rparts, int nr, const double *normM2,
                              int depth, double *log_rel, int32_t *log_depth, int log_idx,
                              int log_cap, DevState *st, double tol, hipStream_t s) {
    const int grid = (r * r + 255) / 256;
    k_reduce_gram<<<grid, 256, 0, s>>>(parts, nparts, rpad, r, Gd, resid ? 1 : 0, rparts, nr,
                                       normM2, depth, log_rel, log_depth, log_idx, log_cap, st,
                                       tol);
    return hipGetLastError();
}

hipError_t launch_cpass_final(int rpad, int mode, const double *Cp, int chunks, int64_t n, int r,
                              const double *Dd, float *W, float *Wt, float *Cout, double *Bp,
                              double *rparts, const int32_t *stop, hipStream_t s) {
    const int grid = cpass_final_blocks(n);
    if (grid == 0) return hipSuccess;
#define L_CFIN(RT)                                                                          \
    if (mode == MODE_HALS)                                                                  \
        k_cpass_final<RT, MODE_HALS><<<grid, 256, 0, s>>>(Cp, chunks, n, r, Dd, W, Wt, Cout, Bp, rparts, stop); \
    else if (mode == MODE_MU)                                                               \
        k_cpass_final<RT, MODE_MU><<<grid, 256, 0, s>>>(Cp, chunks, n, r, Dd, W, Wt, Cout, Bp, rparts, stop);   \
    else                                                                                    \
        k_cpass_final<RT, MODE_STORE><<<grid, 256, 0, s>>>(Cp, chunks, n, r, Dd, W, Wt, Cout, Bp, rparts, stop);
    NMF_DISPATCH_RT(rpad, L_CFIN)
#undef L_CFIN
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
                           int32_t *log_depth, int log_idx, int log_cap, DevState *st, double tol,
                           hipStream_t s) {
    k_residual<<<1, 256, 0, s>>>(rparts, nparts, Dd, Bd, r, normM2, depth, log_rel, log_depth,
                                 log_idx, log_cap, st, tol);
    return hipGetLastError();
}

}  // namespace nmf
