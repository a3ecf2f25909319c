// Multiplicative updates for the generalized Kullback-Leibler divergence
// D(M | V W) = sum M log(M / VW) - M + VW (one of the other objective
// functions of Section 7.1, minimised by the Lee-Seung multiplicative
// updates), on the same hierarchy, transfers and schedule as the Frobenius
// algorithms.  One iteration is five launches:
//
//   k_kl_vpass   per 16-row tile: P = V W on MFMA, Q = M / P (0 where P = 0),
//                A = Q W^T on MFMA, then V <- V o A / (row sums of W)
//   k_kl_wpass   per (row chunk, 64 columns): split-m partials of V^T Q (P and
//                Q again, with the new V) and of the column sums of V
//   k_kl_wfinal  W <- W o (V^T Q) / (column sums of V), its transposed copy,
//                and per-block partial row sums of the new W
//   k_kl_div     per 16-row tile: partial sums of M log(M / P) - M + P (FP64)
//   k_kl_log     D / sum(M_l) logged, the stop test; the row sums of W for
//                the next V pass
//
// Products P, Q W^T and V^T Q run on v_mfma_f32_16x16x4f32 in FP32; the
// update factors and the cross-wave and cross-chunk sums are FP64; each
// divergence term is evaluated in FP32 (kl_term) and the terms added in FP64.  A zero denominator keeps the entry.  Every sum has a fixed order.
//
// MFMA layouts (16x16x4, lane l = 16 lk + li): the A operand is A[li][lk], the
// B operand B[lk][li], the result D[4 lk + v][li].  The V pass forms the
// transposed tile P^T = W^T V^T, so that lane (li, lk) holds P[row li][col
// 4 lk + v]: exactly the A-operand entries of Q W^T for K-step v.  The W pass
// forms P = V W, so that lane (li, lk) holds P[row 4 lk + v][col li]: the
// B-operand entries of V^T Q for K-step v.
#include "device_common.h"
#include "nmf_internal.h"

namespace nmf {

namespace {

constexpr int kKlWaves = 4;

__device__ __forceinline__ float kl_q(float mv, float p) { return p > 0.0f ? mv / p : 0.0f; }

// One divergence term M log(M / P) - M + P = P phi(M / P) with
// phi(x) = x log x - x + 1 >= 0, in FP32.  Near x = 1 the direct form cancels
// (phi ~ (x - 1)^2 / 2), so for |u| < 1/4, u = (M - P) / P, phi is summed as
// its series sum_{k >= 2} (-1)^k u^k / (k (k - 1)) up to k = 12 (truncation
// below 3e-9 relative); elsewhere phi >= 0.028 and the direct form loses at
// most a few units in the last place.  P = 0: +inf where M > 0, 0 where M = 0.
__device__ __forceinline__ float kl_term(float mv, float p) {
    if (!(p > 0.0f)) return mv > 0.0f ? INFINITY : 0.0f;
    const float u = (mv - p) / p;
    float phi;
    if (fabsf(u) < 0.25f) {
        constexpr float c[11] = {1.0f / 2,   -1.0f / 6,   1.0f / 12,  -1.0f / 20,
                                 1.0f / 30,  -1.0f / 42,  1.0f / 56,  -1.0f / 72,
                                 1.0f / 90,  -1.0f / 110, 1.0f / 132};
        float t = c[10];
#pragma unroll
        for (int i = 9; i >= 0; --i) t = fmaf(t, u, c[i]);
        phi = t * u * u;
    } else {
        const float x = mv / p;
        phi = x > 0.0f ? (x * logf(x) - x) + 1.0f : 1.0f;
    }
    return p * phi;
}

// ---------------------------------------------------------------------------
// V pass: block b owns rows 16 b .. 16 b + 15; its four waves split the
// columns into ranges of whole 16-column steps and their partial rows of
// A = Q W^T are added in LDS (FP64, wave order).
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(256) void k_kl_vpass(const float *__restrict__ M, int64_t ldm,
                                                  int64_t m, int64_t n, int r,
                                                  float *__restrict__ V,
                                                  const float *__restrict__ W,
                                                  const float *__restrict__ Wt,
                                                  const double *__restrict__ wsum,
                                                  const int32_t *stop) {
    constexpr int RPAD = 16 * RT, NS = RPAD / 4, AS = RPAD + 1;
    __shared__ float As[kKlWaves][16][AS];
    if (stopped(stop)) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * 16;
    const int64_t rowl = row0 + li;
    const bool rok = rowl < m;
    const int64_t rowc = rok ? rowl : m - 1;
    const auto Vg = to_global(V);
    const auto Wg = to_global(W);
    const auto Mg = to_global(M);
    // B operand of P^T = W^T V^T: V[row li][k = 4 s + lk]
    float vop[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = 4 * s + lk;
        const float v = Vg[rowc + (int64_t)(k < r ? k : 0) * m];
        vop[s] = (rok && k < r) ? v : 0.0f;
    }
    const int64_t per = (n + 16 * kKlWaves - 1) / (16 * kKlWaves) * 16;
    const int64_t c0 = wave * per, c1 = (c0 + per < n) ? c0 + per : n;
    v4f acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t j0 = c0; j0 < c1; j0 += 16) {
        // P^T tile: A operand W^T[col j0 + li][k = 4 s + lk]
        const int64_t ja = j0 + li;
        const bool jaok = ja < c1;
        const int64_t jac = jaok ? ja : c1 - 1;
        // the M entries of this step first: they do not depend on P
        float mv[4];
        gmem<const float> *wtr[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t col = j0 + 4 * lk + v;
            const int64_t cc = col < c1 ? col : c1 - 1;
            mv[v] = Mg[rowc + cc * ldm];
            wtr[v] = to_global(Wt) + cc * RPAD;
        }
        v4f p = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = 4 * s + lk;
            const float w = Wg[(int64_t)(k < r ? k : 0) * n + jac];
            p = __builtin_amdgcn_mfma_f32_16x16x4f32((jaok && k < r) ? w : 0.0f, vop[s], p, 0, 0,
                                                     0);
        }
        // p[v] = P[row li][col j0 + 4 lk + v]; columns past the range and rows
        // past m have P = 0, hence Q = 0
        float q[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) q[v] = kl_q(mv[v], p[v]);
        // A += Q W^T: K-step v takes Q[row li][col j0 + 4 lk + v] and
        // W[16 t + li][the same column] (its row of Wt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float wv[RT];
            load_wt<RT>(wtr[v], li, wv);
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(q[v], wv[t], acc[t], 0, 0, 0);
        }
    }
    // acc[t][v] = A[row 4 lk + v][k = 16 t + li] (this wave's columns)
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) As[wave][4 * lk + v][16 * t + li] = acc[t][v];
    __syncthreads();
    // V <- V o A / (row sums of W): thread (row tid / 16, entries 16 t + tid % 16)
    const int row = tid >> 4, kq = tid & 15;
    const int64_t vr = row0 + row;
    if (vr < m) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + kq;
            if (k < r) {
                double a = 0.0;
#pragma unroll
                for (int w2 = 0; w2 < kKlWaves; ++w2) a += (double)As[w2][row][k];
                const double den = wsum[k];
                if (den > 0.0) {
                    const int64_t idx = vr + (int64_t)k * m;
                    Vg[idx] = (float)((double)Vg[idx] * a / den);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// W pass: block (cx, cy) owns columns 64 cx .. 64 cx + 63 (wave w: 16 of
// them) of row chunk cy.  Each 16-row step stages the V tile in LDS, read in
// the A-operand layout of P = V W and in the transposed layout of V^T Q.
// The first column block of each chunk also sums the chunk's columns of V.
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(256) void k_kl_wpass(const float *__restrict__ M, int64_t ldm,
                                                  int64_t m, int64_t n, int r,
                                                  const float *__restrict__ V,
                                                  const float *__restrict__ W, int ncb,
                                                  int64_t chunk, double *__restrict__ Cp,
                                                  double *__restrict__ vparts,
                                                  const int32_t *stop) {
    constexpr int RPAD = 16 * RT, NS = RPAD / 4, VS = RPAD + 1;
    __shared__ float Vs[16][VS];
    if (stopped(stop)) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int cx = (int)(blockIdx.x % ncb), cy = (int)(blockIdx.x / ncb);
    const int64_t i_begin = (int64_t)cy * chunk;
    const int64_t i_end = (i_begin + chunk < m) ? i_begin + chunk : m;
    const int64_t jl = (int64_t)cx * 64 + wave * 16 + li;
    const bool jok = jl < n;
    const int64_t jc = jok ? jl : n - 1;
    const auto Vg = to_global(V);
    const auto Wg = to_global(W);
    const auto Mg = to_global(M);
    // B operand of P = V W: W[k = 4 s + lk][col jl]
    float wop[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = 4 * s + lk;
        const float w = Wg[(int64_t)(k < r ? k : 0) * n + jc];
        wop[s] = (jok && k < r) ? w : 0.0f;
    }
    v4f acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    double vs = 0.0;
    for (int64_t i0 = i_begin; i0 < i_end; i0 += 16) {
        __syncthreads();   // the previous tile is consumed
        for (int e = tid; e < 16 * RPAD; e += 256) {
            const int rr = e & 15, k = e >> 4;
            const int64_t i = i0 + rr;
            const float v = Vg[(i < i_end ? i : i_end - 1) + (int64_t)(k < r ? k : 0) * m];
            Vs[rr][k] = (i < i_end && k < r) ? v : 0.0f;
        }
        __syncthreads();
        if (cx == 0 && tid < RPAD) {
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) vs += (double)Vs[rr][tid];
        }
        v4f p = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < NS; ++s)
            p = __builtin_amdgcn_mfma_f32_16x16x4f32(Vs[li][4 * s + lk], wop[s], p, 0, 0, 0);
        // p[v] = P[row i0 + 4 lk + v][col jl]; rows past the chunk have P = 0
        float q[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = i0 + 4 * lk + v;
            q[v] = kl_q(Mg[(i < i_end ? i : i_end - 1) + jc * ldm], p[v]);
        }
        // C += V^T Q: K-step v takes V[row i0 + 4 lk + v][k = 16 t + li] and Q[that row][jl]
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(Vs[4 * lk + v][16 * t + li], q[v],
                                                             acc[t], 0, 0, 0);
    }
    // acc[t][v] = (V^T Q)[k = 16 t + 4 lk + v][col jl] over this chunk
    if (jok) {
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = 16 * t + 4 * lk + v;
                if (k < r) to_global(Cp)[((int64_t)cy * r + k) * n + jl] = (double)acc[t][v];
            }
    }
    if (cx == 0 && tid < RPAD) to_global(vparts)[(int64_t)cy * RPAD + tid] = vs;
}

// ---------------------------------------------------------------------------
// W update: block (cb, kg) owns columns 64 cb .. 64 cb + 63 of the four rows
// k = 4 kg .. 4 kg + 3 (thread: row 4 kg + tid / 64, column tid % 64).
// C = sum of the chunk partials and the column sums of V = sum of their
// partials, both in chunk order with the loads issued in batches of 8;
// W <- W o C / vsum (kept where vsum = 0), Wt, and the block's partial row
// sums of the stored new W (column order).  init: no update (start of a
// solve), only Wt and the row sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_kl_wfinal(int64_t n, int r, int rpad, int chunks,
                                                   const double *__restrict__ Cp,
                                                   const double *__restrict__ vparts,
                                                   float *__restrict__ W, float *__restrict__ Wt,
                                                   double *__restrict__ wparts, int init, int ncb,
                                                   const int32_t *stop) {
    constexpr int B = 8;
    __shared__ double vsum[4];
    __shared__ double Wn[4][64];
    if (stopped(stop)) return;
    const int tid = threadIdx.x;
    const int cb = (int)(blockIdx.x % ncb), kg = (int)(blockIdx.x / ncb);
    const int kk = tid >> 6, jj = tid & 63;
    const int k = 4 * kg + kk;
    const int64_t j = (int64_t)cb * 64 + jj;
    const bool live = k < r && j < n;
    // batched, ordered sum of `chunks` values at p, p + stride, ...
    auto ordered_sum = [&](const double *p, int64_t stride) {
        double s = 0.0;
        for (int c0 = 0; c0 < chunks; c0 += B) {
            double v[B];
#pragma unroll
            for (int u = 0; u < B; ++u)
                v[u] = (c0 + u < chunks) ? p[(int64_t)(c0 + u) * stride] : 0.0;
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (c0 + u < chunks) s += v[u];
        }
        return s;
    };
    if (!init && jj == 0) vsum[kk] = k < r ? ordered_sum(vparts + k, rpad) : 0.0;
    double c = 0.0;
    if (!init && live) c = ordered_sum(Cp + (int64_t)k * n + j, (int64_t)r * n);
    __syncthreads();
    const auto Wg = to_global(W);
    float wf = 0.0f;
    if (live) {
        wf = Wg[(int64_t)k * n + j];
        if (!init && vsum[kk] > 0.0) {
            wf = (float)((double)wf * c / vsum[kk]);
            Wg[(int64_t)k * n + j] = wf;
        }
    }
    if (j < n && k < rpad) to_global(Wt)[j * rpad + wt_pos(k, rpad / 16)] = wf;
    Wn[kk][jj] = (double)wf;
    __syncthreads();
    if (jj == 0 && k < rpad) {
        double s = 0.0;
        for (int c2 = 0; c2 < 64; ++c2) s += Wn[kk][c2];
        to_global(wparts)[(int64_t)cb * rpad + k] = s;
    }
}

// Row sums of W from the k_kl_wfinal partials (block order).
__global__ __launch_bounds__(64) void k_kl_wsum(const double *__restrict__ wparts, int nb,
                                                int rpad, double *__restrict__ wsum,
                                                const int32_t *stop) {
    if (stopped(stop)) return;
    const int k = threadIdx.x;
    if (k >= rpad) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += wparts[(int64_t)b * rpad + k];
    wsum[k] = s;
}

// ---------------------------------------------------------------------------
// Divergence partials: the tiles of the V pass (16 rows per block, columns
// split over the waves), sum over the block's entries of the terms of
// kl_term, added in FP64.
// ---------------------------------------------------------------------------
template <int RT>
__global__ __launch_bounds__(256) void k_kl_div(const float *__restrict__ M, int64_t ldm,
                                                int64_t m, int64_t n, int r,
                                                const float *__restrict__ V,
                                                const float *__restrict__ W,
                                                double *__restrict__ dparts, const int32_t *stop) {
    constexpr int RPAD = 16 * RT, NS = RPAD / 4;
    __shared__ double red[kKlWaves];
    if (stopped(stop)) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t rowl = (int64_t)blockIdx.x * 16 + li;
    const bool rok = rowl < m;
    const int64_t rowc = rok ? rowl : m - 1;
    const auto Vg = to_global(V);
    const auto Wg = to_global(W);
    const auto Mg = to_global(M);
    float vop[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = 4 * s + lk;
        const float v = Vg[rowc + (int64_t)(k < r ? k : 0) * m];
        vop[s] = (rok && k < r) ? v : 0.0f;
    }
    const int64_t per = (n + 16 * kKlWaves - 1) / (16 * kKlWaves) * 16;
    const int64_t c0 = wave * per, c1 = (c0 + per < n) ? c0 + per : n;
    double tsum = 0.0;
    for (int64_t j0 = c0; j0 < c1; j0 += 16) {
        const int64_t ja = j0 + li;
        const bool jaok = ja < c1;
        const int64_t jac = jaok ? ja : c1 - 1;
        float mf[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t col = j0 + 4 * lk + v;
            mf[v] = Mg[rowc + (col < c1 ? col : c1 - 1) * ldm];
        }
        v4f p = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = 4 * s + lk;
            const float w = Wg[(int64_t)(k < r ? k : 0) * n + jac];
            p = __builtin_amdgcn_mfma_f32_16x16x4f32((jaok && k < r) ? w : 0.0f, vop[s], p, 0, 0,
                                                     0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t col = j0 + 4 * lk + v;
            if (rok && col < c1) tsum += (double)kl_term(mf[v], p[v]);
        }
    }
    tsum = block_sum_f64<256>(tsum, red);
    if (tid == 0) to_global(dparts)[blockIdx.x] = tsum;
}

// Divergence of the iteration, logged as D / sum(M_depth), the stop test, and
// the row sums of W for the next V pass.
__global__ __launch_bounds__(256) void k_kl_log(const double *__restrict__ dparts, int nd,
                                                const double *__restrict__ wparts, int nw,
                                                int rpad, double *__restrict__ wsum,
                                                const double *__restrict__ msum, int depth,
                                                double *__restrict__ log_rel,
                                                int32_t *__restrict__ log_depth, int log_cap,
                                                DevState *st, int32_t *hstop, double tol) {
    __shared__ double red[4];
    if (st->stop) return;
    const int tid = threadIdx.x;
    if (tid < rpad) {
        double s = 0.0;
        for (int b = 0; b < nw; ++b) s += wparts[(int64_t)b * rpad + tid];
        wsum[tid] = s;
    }
    double s = 0.0;
    for (int i = tid; i < nd; i += 256) s += dparts[i];
    s = block_sum_f64<256>(s, red);
    if (tid == 0) {
        const double tot = msum[depth];
        const double rel = tot > 0.0 ? s / tot : s;
        const int idx = st->log_len;
        if (idx < log_cap) {
            log_rel[idx] = rel;
            log_depth[idx] = depth;
        }
        st->log_len = idx + 1;
        st->last_rel = rel;
        if (!isfinite(s)) {
            st->status = NMF_E_NONFINITE;
            st->stop = 1;
            if (hstop) *hstop = 1;
        } else if (depth == 0 && tol > 0.0 && rel <= tol) {
            st->stopped = 1;
            st->stop = 1;
            if (hstop) *hstop = 1;
        }
    }
}

// sum(M) of an m x n column-major matrix: part p adds the items (column,
// 2048-row chunk) p, p + nparts, ... (FP64), then one block adds the parts.
__global__ __launch_bounds__(256) void k_msum_parts(const float *__restrict__ M, int64_t ldm,
                                                    int64_t m, int64_t n, int nparts,
                                                    double *__restrict__ parts) {
    __shared__ double red[4];
    const int64_t nch = (m + 2047) / 2048;
    double s = 0.0;
    for (int64_t it = blockIdx.x; it < n * nch; it += nparts) {
        const int64_t col = it / nch, r0 = (it % nch) * 2048;
        const int64_t r1 = (r0 + 2048 < m) ? r0 + 2048 : m;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) s += (double)M[i + col * ldm];
    }
    s = block_sum_f64<256>(s, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_msum_final(const double *__restrict__ parts, int nparts,
                                                    double *__restrict__ out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) s += parts[i];
    s = block_sum_f64<256>(s, red);
    if (threadIdx.x == 0) *out = s;
}

}  // namespace

int kl_row_blocks(int64_t m) { return (int)((m + 15) / 16); }
int kl_col_blocks(int64_t n) { return (int)((n + 63) / 64); }

hipError_t launch_kl_vpass(int rpad, const float *M, int64_t ldm, int64_t m, int64_t n, int r,
                           float *V, const float *W, const float *Wt, const double *wsum,
                           const int32_t *stop, hipStream_t s) {
    const int blocks = kl_row_blocks(m);
    switch (rpad) {
        case 16: k_kl_vpass<1><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, Wt, wsum, stop); break;
        case 32: k_kl_vpass<2><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, Wt, wsum, stop); break;
        case 48: k_kl_vpass<3><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, Wt, wsum, stop); break;
        case 64: k_kl_vpass<4><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, Wt, wsum, stop); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_kl_wpass(int rpad, const float *M, int64_t ldm, int64_t m, int64_t n, int r,
                           const float *V, const float *W, int chunks, int64_t chunk, double *Cp,
                           double *vparts, const int32_t *stop, hipStream_t s) {
    const int ncb = kl_col_blocks(n);
    const int blocks = ncb * chunks;
    switch (rpad) {
        case 16: k_kl_wpass<1><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, ncb, chunk, Cp, vparts, stop); break;
        case 32: k_kl_wpass<2><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, ncb, chunk, Cp, vparts, stop); break;
        case 48: k_kl_wpass<3><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, ncb, chunk, Cp, vparts, stop); break;
        case 64: k_kl_wpass<4><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, ncb, chunk, Cp, vparts, stop); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_kl_wfinal(int rpad, int64_t n, int r, int chunks, const double *Cp,
                            const double *vparts, float *W, float *Wt, double *wparts, bool init,
                            const int32_t *stop, hipStream_t s) {
    const int ncb = kl_col_blocks(n);
    k_kl_wfinal<<<ncb * (rpad / 4), 256, 0, s>>>(n, r, rpad, chunks, Cp, vparts, W, Wt, wparts,
                                                 init ? 1 : 0, ncb, stop);
    return hipGetLastError();
}

hipError_t launch_kl_wsum(int rpad, int64_t n, const double *wparts, double *wsum,
                          const int32_t *stop, hipStream_t s) {
    k_kl_wsum<<<1, 64, 0, s>>>(wparts, kl_col_blocks(n), rpad, wsum, stop);
    return hipGetLastError();
}

hipError_t launch_kl_div(int rpad, const float *M, int64_t ldm, int64_t m, int64_t n, int r,
                         const float *V, const float *W, double *dparts, const int32_t *stop,
                         hipStream_t s) {
    const int blocks = kl_row_blocks(m);
    switch (rpad) {
        case 16: k_kl_div<1><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, dparts, stop); break;
        case 32: k_kl_div<2><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, dparts, stop); break;
        case 48: k_kl_div<3><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, dparts, stop); break;
        case 64: k_kl_div<4><<<blocks, 256, 0, s>>>(M, ldm, m, n, r, V, W, dparts, stop); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_kl_log(int64_t m, int64_t n, int rpad, const double *dparts,
                         const double *wparts, double *wsum, const double *msum, int depth,
                         double *log_rel, int32_t *log_depth, int log_cap, DevState *st,
                         int32_t *hstop, double tol, hipStream_t s) {
    k_kl_log<<<1, 256, 0, s>>>(dparts, kl_row_blocks(m), wparts, kl_col_blocks(n), rpad, wsum,
                               msum, depth, log_rel, log_depth, log_cap, st, hstop, tol);
    return hipGetLastError();
}

hipError_t launch_msum(const float *M, int64_t ldm, int64_t m, int64_t n, double *parts,
                       int nparts, double *out, hipStream_t s) {
    k_msum_parts<<<nparts, 256, 0, s>>>(M, ldm, m, n, nparts, parts);
    k_msum_final<<<1, 256, 0, s>>>(parts, nparts, out);
    return hipGetLastError();
}

}  // namespace nmf
