// One NMF iteration on one level: the two M-streaming products and the
// factor updates of Alg. 2 (MU) and Alg. 3 (HALS), plus the residual.
//
//   A = M W^T   (m x r)  -> V update fused as epilogue   [k_apass]
//   C = V^T M   (r x n)  -> split-m partials             [k_cpass_partial]
//                        -> reduce + W update            [k_cpass_final]
//   rel_err from ||M||^2 - 2 <C, W> + <V^T V, W W^T>     [k_residual]
//
// Both products run on the FP32 matrix cores (v_mfma_f32_16x16x4f32).  Lane
// layout of that instruction on a 64-wide wave: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; accumulator register v of lane l holds D[4*(l/16)+v][l%16].
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

constexpr int MODE_HALS = 0, MODE_MU = 1, MODE_STORE = 2;

// HALS / MU update of one factor row held by 4 lanes.  G is the r x r FP64
// Gram of the other factor in LDS (row stride gs, zero-padded to RPAD), a[k]
// the matching row of the FP32 product (M W^T or V^T M, LDS).  Entries beyond
// r are 0.  The r x r-sized update arithmetic runs in FP64 (the numerator
// a_k - sum_l x_l G_lk cancels as the iterate converges); the row is read
// from and written back to FP32 storage.
//   HALS: x_k <- max(0, (a_k - sum_{l != k} x_l G_lk) / G_kk); G_kk = 0 keeps x_k.
//   MU:   x_k <- x_k a_k / (sum_l x_l G_lk); a zero denominator keeps x_k.
template <int RPAD, int MODE>
__device__ __forceinline__ void row_update(double (&x)[RPAD / 4], const double *G, int gs,
                                           const double *a, int r, int q) {
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
                const double gkk = G[k * gs + k];
                if (gkk > 0.0) {
                    const double nv = fmax(0.0, (a[k] - s) / gkk);
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

// ---------------------------------------------------------------------------
// A-pass: block = 4 waves = 64 rows of M; each wave owns 16 rows and the full
// n reduction.  W is staged through LDS in chunks of KC columns.
// ---------------------------------------------------------------------------
template <int RT, int MODE>
__global__ __launch_bounds__(256) void k_apass(const float *__restrict__ M, int64_t ldm,
                                               int64_t m, int64_t n,
                                               const float *__restrict__ W,
                                               const double *__restrict__ Bd,
                                               float *__restrict__ V, float *__restrict__ Aout,
                                               int r, const int32_t *stop) {
    constexpr int RPAD = RT * 16, KC = 64, WS = KC + 2, GS = RPAD + 1, AS = RPAD + 1;
    __shared__ float Ws[RPAD * WS];
    __shared__ double Gs[(MODE == MODE_STORE) ? 1 : RPAD * GS];
    __shared__ double As[4 * 16 * AS];
    if (stopped(stop)) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t row0 = (int64_t)blockIdx.x * 64 + wave * 16;

    if constexpr (MODE != MODE_STORE) {
        for (int e = tid; e < RPAD * RPAD; e += 256) {
            const int a = e / RPAD, b = e % RPAD;
            Gs[a * GS + b] = (a < r && b < r) ? Bd[a * r + b] : 0.0;
        }
    }
    v4f hi[RT], lo[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) hi[t] = lo[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};

    const int li = lane & 15, lk = lane >> 4;
    const int64_t arow = row0 + li;
    const bool rowok = arow < m;
    const float *Mrow = M + (rowok ? arow : 0);
    for (int64_t j0 = 0; j0 < n; j0 += KC) {
        __syncthreads();
        for (int e = tid; e < RPAD * KC; e += 256) {
            const int k = e / KC, jj = e % KC;
            const int64_t j = j0 + jj;
            Ws[k * WS + jj] = (k < r && j < n) ? W[(int64_t)k * n + j] : 0.0f;
        }
        __syncthreads();
        const int kc = (int)((n - j0 < KC) ? (n - j0) : KC);
        for (int k0 = 0; k0 < kc; k0 += 16) {          // one 16-column accumulator chain
            v4f acc[RT];
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            const int kend = (k0 + 16 < kc) ? k0 + 16 : kc;
            for (int kk = k0; kk < kend; kk += 4) {
                const int64_t j = j0 + kk + lk;
                const float a = (rowok && j < n) ? Mrow[j * ldm] : 0.0f;
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const float b = Ws[(16 * t + li) * WS + kk + lk];
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
                }
            }
#pragma unroll
            for (int t = 0; t < RT; ++t) two_sum_acc(hi[t], lo[t], acc[t]);
        }
    }
    double *Aw = As + wave * 16 * AS;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Aw[(4 * lk + v) * AS + 16 * t + li] = (double)hi[t][v] + (double)lo[t][v];
    __syncthreads();

    if constexpr (MODE == MODE_STORE) {
        for (int e = lane; e < 16 * r; e += 64) {
            const int rr = e & 15, k = e >> 4;
            const int64_t row = row0 + rr;
            if (row < m) Aout[row + (int64_t)k * m] = (float)Aw[rr * AS + k];
        }
    } else {
        const int er = lane >> 2, q = lane & 3;
        const int64_t vrow = row0 + er;
        const bool ok = vrow < m;
        double x[RPAD / 4];
#pragma unroll
        for (int jj = 0; jj < RPAD / 4; ++jj) {
            const int k = 4 * jj + q;
            x[jj] = (ok && k < r) ? (double)V[vrow + (int64_t)k * m] : 0.0;
        }
        row_update<RPAD, MODE>(x, Gs, GS, Aw + er * AS, r, q);
#pragma unroll
        for (int jj = 0; jj < RPAD / 4; ++jj) {
            const int k = 4 * jj + q;
            if (ok && k < r) V[vrow + (int64_t)k * m] = (float)x[jj];
        }
    }
}

// ---------------------------------------------------------------------------
// C-pass partials: block (x = 64-column tile of n, y = chunk of m rows).
// Each wave owns 16 columns; a lane loads 4 consecutive rows of M and V
// (one float4 each) and feeds them to 4 MFMAs, so the k-index of MFMA s maps
// to row i0 + 4*(lane/16) + s.
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(256) void k_cpass_partial(const float *__restrict__ M, int64_t ldm,
                                                       int64_t m, int64_t n,
                                                       const float *__restrict__ V, int r,
                                                       int64_t chunk, double *__restrict__ Cp,
                                                       const int32_t *stop) {
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
    v4f acc[RT], hi[RT], lo[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = hi[t] = lo[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};

    for (int64_t i0 = i_begin; i0 < i_end; i0 += 16) {
        const int64_t ib = i0 + 4 * lg;
        v4f mv, vv[RT];
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
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(mv[s], vv[t][s], acc[t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < RT; ++t) {      // 16 rows per accumulator chain
            two_sum_acc(hi[t], lo[t], acc[t]);
            acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
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
}

// ---------------------------------------------------------------------------
// Reduce the C partials of 16 columns (fixed order) and update those columns
// of W; emit the FP64 partial <C, W_new> for the residual.
// ---------------------------------------------------------------------------
template <int RT, int MODE>
__global__ __launch_bounds__(256) void k_cpass_final(const double *__restrict__ Cp, int chunks,
                                                     int64_t n, int r,
                                                     const double *__restrict__ Dd,
                                                     float *__restrict__ W,
                                                     float *__restrict__ Cout,
                                                     double *__restrict__ rparts,
                                                     const int32_t *stop) {
    constexpr int RPAD = RT * 16, GS = RPAD + 1, CS = RPAD + 1;
    __shared__ double Gs[(MODE == MODE_STORE) ? 1 : RPAD * GS];
    __shared__ double Cs[16 * CS];
    __shared__ double red[4];
    if (stopped(stop)) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t j0 = (int64_t)blockIdx.x * 16;
    if constexpr (MODE != MODE_STORE) {
        for (int e = tid; e < RPAD * RPAD; e += 256) {
            const int a = e / RPAD, b = e % RPAD;
            Gs[a * GS + b] = (a < r && b < r) ? Dd[a * r + b] : 0.0;
        }
    }
    for (int e = tid; e < 16 * RPAD; e += 256) {
        const int jj = e & 15, k = e >> 4;
        const int64_t j = j0 + jj;
        double s = 0.0;
        if (k < r && j < n)
            for (int p = 0; p < chunks; ++p) s += Cp[((int64_t)p * r + k) * n + j];
        Cs[jj * CS + k] = s;
    }
    __syncthreads();
    if constexpr (MODE == MODE_STORE) {
        for (int e = tid; e < 16 * r; e += 256) {
            const int jj = e & 15, k = e >> 4;
            const int64_t j = j0 + jj;
            if (j < n) Cout[(int64_t)k * n + j] = (float)Cs[jj * CS + k];
        }
        return;
    } else {
        double part = 0.0;
        if (tid < 64) {
            const int jj = lane >> 2, q = lane & 3;
            const int64_t j = j0 + jj;
            const bool ok = j < n;
            double x[RPAD / 4];
#pragma unroll
            for (int t = 0; t < RPAD / 4; ++t) {
                const int k = 4 * t + q;
                x[t] = (ok && k < r) ? (double)W[(int64_t)k * n + j] : 0.0;
            }
            row_update<RPAD, MODE>(x, Gs, GS, Cs + jj * CS, r, q);
#pragma unroll
            for (int t = 0; t < RPAD / 4; ++t) {
                const int k = 4 * t + q;
                if (ok && k < r) {
                    const float xf = (float)x[t];
                    W[(int64_t)k * n + j] = xf;
                    part += Cs[jj * CS + k] * (double)xf;
                }
            }
        }
        part = block_sum_f64<256>(part, red);
        if (tid == 0) rparts[blockIdx.x] = part;
    }
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

}  // namespace

int cpass_final_blocks(int64_t n) { return (int)((n + 15) / 16); }

#define NMF_DISPATCH_RT(rpad, MACRO) \
    switch (rpad) {                  \
        case 16: MACRO(1); break;    \
        case 32: MACRO(2); break;    \
        case 48: MACRO(3); break;    \
        case 64: MACRO(4); break;    \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_apass(int rpad, int mode, const float *M, int64_t ldm, int64_t m, int64_t n,
                        const float *W, const double *Bd, float *V, float *Aout, int r,
                        const int32_t *stop, hipStream_t s) {
    const int grid = (int)((m + 63) / 64);
    if (grid == 0) return hipSuccess;
#define L_APASS(RT)                                                                               \
    if (mode == MODE_HALS)                                                                        \
        k_apass<RT, MODE_HALS><<<grid, 256, 0, s>>>(M, ldm, m, n, W, Bd, V, Aout, r, stop);       \
    else if (mode == MODE_MU)                                                                     \
        k_apass<RT, MODE_MU><<<grid, 256, 0, s>>>(M, ldm, m, n, W, Bd, V, Aout, r, stop);         \
    else                                                                                          \
        k_apass<RT, MODE_STORE><<<grid, 256, 0, s>>>(M, ldm, m, n, W, Bd, V, Aout, r, stop);
    NMF_DISPATCH_RT(rpad, L_APASS)
#undef L_APASS
    return hipGetLastError();
}

hipError_t launch_cpass_partial(int rpad, const float *M, int64_t ldm, int64_t m, int64_t n,
                                const float *V, int r, int chunks, int64_t chunk, double *Cp,
                                const int32_t *stop, hipStream_t s) {
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)chunks);
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
#define L_CPART(RT) k_cpass_partial<RT><<<grid, 256, 0, s>>>(M, ldm, m, n, V, r, chunk, Cp, stop);
    NMF_DISPATCH_RT(rpad, L_CPART)
#undef L_CPART
    return hipGetLastError();
}

hipError_t launch_cpass_final(int rpad, int mode, const double *Cp, int chunks, int64_t n, int r,
                              const double *Dd, float *W, float *Cout, double *rparts,
                              const int32_t *stop, hipStream_t s) {
    const int grid = cpass_final_blocks(n);
    if (grid == 0) return hipSuccess;
#define L_CFIN(RT)                                                                              \
    if (mode == MODE_HALS)                                                                      \
        k_cpass_final<RT, MODE_HALS><<<grid, 256, 0, s>>>(Cp, chunks, n, r, Dd, W, Cout, rparts, stop); \
    else if (mode == MODE_MU)                                                                   \
        k_cpass_final<RT, MODE_MU><<<grid, 256, 0, s>>>(Cp, chunks, n, r, Dd, W, Cout, rparts, stop);   \
    else                                                                                        \
        k_cpass_final<RT, MODE_STORE><<<grid, 256, 0, s>>>(Cp, chunks, n, r, Dd, W, Cout, rparts, stop);
    NMF_DISPATCH_RT(rpad, L_CFIN)
#undef L_CFIN
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
