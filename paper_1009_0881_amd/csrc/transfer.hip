// Grid-transfer stencils (Section 4.2) and whole-matrix reductions.
//
// Restriction (eq. restr): coarse node c of a fine axis of length N sits on
// fine node 2c.  Full weighting (FW) uses the 1-D weights 1,2,1 on fine nodes
// 2c-1, 2c, 2c+1; nodes outside the image are dropped and the remaining
// weights are renormalised to sum 1 (the boundary rule "weights adapted
// correspondingly").  The 2-D stencil is the product of the two 1-D ones, so
// interior pixels get (1,2,1)x(1,2,1)/16.  BLOCK2 averages fine nodes 2c, 2c+1.
//
// Prolongation (eq. prol): fine node f takes the mean of the coarse nodes
// rd(f/2) that exist ({f/2} for even f, {(f-1)/2, (f+1)/2} for odd f) per
// axis; BLOCK2 copies coarse node floor(f/2).
//
// One thread per output pixel and image; the taps are recomputed from the
// closed form (no tables), accumulated in FP64 and rounded once to FP32.

#include "device_common.h"
#include "nmf_internal.h"

namespace nmf {

namespace {

// Up to three taps of a 1-D transfer.  Unused taps carry weight 0 and repeat
// a valid index, so every loop has a fixed trip count and the taps stay in
// registers; a zero-weight tap adds +0.0 to a finite nonnegative sum, which
// leaves the result bitwise unchanged.
struct Taps {
    int idx[3];
    double wt[3];
};

__device__ __forceinline__ Taps restrict_taps(int c, int N, int xfer) {
    Taps t;
    if (xfer == NMF_XFER_FW) {
        // weights (1, 2, 1) on fine nodes 2c-1, 2c, 2c+1 that exist, renormalised
        const bool lo = 2 * c - 1 >= 0, hi = 2 * c + 1 < N;
        const double sum = 2.0 + (lo ? 1.0 : 0.0) + (hi ? 1.0 : 0.0);
        int k = 0;
        double w[3] = {0.0, 0.0, 0.0};
        int ix[3] = {2 * c, 2 * c, 2 * c};
        if (lo) { ix[k] = 2 * c - 1; w[k] = 1.0 / sum; ++k; }
        ix[k] = 2 * c; w[k] = 2.0 / sum; ++k;
        if (hi) { ix[k] = 2 * c + 1; w[k] = 1.0 / sum; ++k; }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            t.idx[i] = ix[i];
            t.wt[i] = w[i];
        }
    } else {
        const int f0 = 2 * c;
        const bool two = f0 + 1 < N;
        t.idx[0] = f0;
        t.idx[1] = two ? f0 + 1 : f0;
        t.idx[2] = f0;
        t.wt[0] = two ? 0.5 : 1.0;
        t.wt[1] = two ? 0.5 : 0.0;
        t.wt[2] = 0.0;
    }
    return t;
}

__device__ __forceinline__ Taps prolong_taps(int f, int Nc, int xfer) {
    Taps t;
    if (xfer == NMF_XFER_FW && (f & 1)) {
        const bool two = (f + 1) / 2 < Nc;
        t.idx[0] = (f - 1) / 2;
        t.idx[1] = two ? (f + 1) / 2 : (f - 1) / 2;
        t.wt[0] = two ? 0.5 : 1.0;
        t.wt[1] = two ? 0.5 : 0.0;
    } else {
        t.idx[0] = f / 2;
        t.idx[1] = f / 2;
        t.wt[0] = 1.0;
        t.wt[1] = 0.0;
    }
    t.idx[2] = t.idx[0];
    t.wt[2] = 0.0;
    return t;
}

// One output pixel of a separable transfer: sum_a ty_a sum_b tx_b img[iy_a * rowlen + ix_b],
// accumulated in FP64 in tap order.
__device__ __forceinline__ float stencil(const float *imgp, int rowlen, const Taps &ty,
                                         const Taps &tx) {
    const auto img = to_global(imgp);   // global (not FLAT) loads: the 9 taps stay in flight
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double row = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) row += tx.wt[b] * (double)img[(int64_t)ty.idx[a] * rowlen + tx.idx[b]];
        acc += ty.wt[a] * row;
    }
    return (float)acc;
}

// Columns per thread of k_restrict: 4 for wide matrices (M: fewer threads,
// their loads batched), 1 for the r columns of a factor (more blocks for a
// latency-bound launch).  The per-pixel arithmetic is the same either way.
template <int RC>
__global__ __launch_bounds__(256) void k_restrict(const float *__restrict__ X, int64_t ldx,
                                                  float *__restrict__ Y, int h, int w, int hc,
                                                  int wc, int64_t ncols, int xfer,
                                                  const int32_t *stop) {
    if (stopped(stop)) return;
    // grid: x over coarse pixels, y over groups of RC columns (strided);
    // 32-bit pixel math.  A thread's columns are loaded together (9 taps
    // each), then stored.
    const int mc = hc * wc;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= mc) return;
    const int cy = p / wc, cx = p - cy * wc;
    const Taps ty = restrict_taps(cy, h, xfer);
    const Taps tx = restrict_taps(cx, w, xfer);
    for (int64_t c0 = (int64_t)blockIdx.y * RC; c0 < ncols; c0 += (int64_t)gridDim.y * RC) {
        float out[RC];
#pragma unroll
        for (int u = 0; u < RC; ++u) {
            const int64_t col = c0 + u < ncols ? c0 + u : ncols - 1;
            out[u] = stencil(X + col * ldx, w, ty, tx);
        }
#pragma unroll
        for (int u = 0; u < RC; ++u)
            if (c0 + u < ncols) Y[(c0 + u) * mc + p] = out[u];
    }
}

__global__ __launch_bounds__(256) void k_prolong(const float *__restrict__ Y,
                                                 float *__restrict__ X, int h, int w, int hc,
                                                 int wc, int64_t ncols, int xfer,
                                                 const int32_t *stop) {
    if (stopped(stop)) return;
    // grid: x over fine pixels, y over columns (strided); 32-bit pixel math
    const int mf = h * w, mc = hc * wc;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= mf) return;
    const int y = p / w, x = p - y * w;
    for (int64_t col = blockIdx.y; col < ncols; col += gridDim.y) {
        const Taps ty = prolong_taps(y, hc, xfer);
        const Taps tx = prolong_taps(x, wc, xfer);
        X[col * mf + p] = stencil(Y + col * mc, wc, ty, tx);
    }
}

// 1-D transfer along the second index of a rows x N array (two-sided
// hierarchies: the column index of M, the rows of W).  One output element per
// thread: its up to three taps from the closed form, accumulated in FP64 in
// tap order and rounded once.  The flat index runs over the output with the
// unit-stride index fastest (i_fast: i, else c) so the loads coalesce.
__global__ __launch_bounds__(256) void k_xfer_cols(int restrict_op, int xfer, int64_t rows,
                                                   int64_t N, int64_t Nout,
                                                   const float *__restrict__ X, int64_t xi,
                                                   int64_t xj, float *__restrict__ Y,
                                                   int64_t yi, int64_t yj, int i_fast,
                                                   const int32_t *stop) {
    if (stopped(stop)) return;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= rows * Nout) return;
    const int64_t i = i_fast ? e % rows : e / Nout;
    const int64_t c = i_fast ? e / rows : e % Nout;
    const Taps t = restrict_op ? restrict_taps((int)c, (int)N, xfer)
                               : prolong_taps((int)c, (int)((N + 1) / 2), xfer);
    const auto x = to_global(X);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) acc += t.wt[a] * (double)x[i * xi + (int64_t)t.idx[a] * xj];
    Y[i * yi + c * yj] = (float)acc;
}

// Sum of squares of a column-major matrix in FP64: per-block partials, then a
// single block adds them in index order (deterministic).
// Partial part (of nparts) of ||X||_F^2: work items (column, 2048-row chunk),
// part p takes items p, p + nparts, ...  Full chunks of a 16-byte-aligned
// matrix with ld % 4 == 0 are read as two float4 per thread, four items per
// batch with every load issued before the sums; other items element-wise.
__device__ __forceinline__ double sumsq_part(const float *Xg, int64_t ld, int64_t rows,
                                             int64_t ncols, int part, int nparts) {
    constexpr int64_t CH = 2048, U = 4;
    const auto X = to_global(Xg);
    const int64_t nrc = (rows + CH - 1) / CH, total = ncols * nrc;
    const bool vec = (ld & 3) == 0 && ((uintptr_t)Xg & 15) == 0;
    const int tid = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    auto full = [&](int64_t it) { return it < total && (it % nrc) * CH + CH <= rows; };
    auto sq4 = [&](const v4f &v, double &a) {
#pragma unroll
        for (int e = 0; e < 4; ++e) a += (double)v[e] * (double)v[e];
    };
    int64_t it = part;
    for (; vec && it + (U - 1) * nparts < total; it += U * nparts) {
        bool all = true;
#pragma unroll
        for (int u = 0; u < U; ++u) all = all && full(it + u * nparts);
        if (!all) break;
        v4f a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t iu = it + u * nparts, c = iu / nrc, r0 = (iu - c * nrc) * CH;
            const auto col = X + c * ld + r0;
            a[u] = *(gmem<const v4f> *)(col + 4 * tid);
            b[u] = *(gmem<const v4f> *)(col + 1024 + 4 * tid);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sq4(a[u], acc[u]);
            sq4(b[u], acc[u]);
        }
    }
    for (; it < total; it += nparts) {
        const int64_t c = it / nrc, r0 = (it - c * nrc) * CH;
        const int64_t r1 = r0 + CH < rows ? r0 + CH : rows;
        const auto col = X + c * ld;
        for (int64_t i = r0 + tid; i < r1; i += 256) {
            const double v = col[i];
            acc[0] += v * v;
        }
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

__global__ __launch_bounds__(256) void k_sumsq_partial(const float *__restrict__ X, int64_t ld,
                                                       int64_t rows, int64_t ncols,
                                                       double *__restrict__ parts) {
    __shared__ double scratch[4];
    double acc = sumsq_part(X, ld, rows, ncols, blockIdx.x, gridDim.x);
    acc = block_sum_f64<256>(acc, scratch);
    if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ parts, int nparts,
                                                   double *__restrict__ out) {
    __shared__ double scratch[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += parts[i];
    acc = block_sum_f64<256>(acc, scratch);
    if (threadIdx.x == 0) *out = acc;
}

__global__ __launch_bounds__(256) void k_check_input(const float *__restrict__ M, int64_t ld,
                                                     int64_t m, int64_t n,
                                                     int32_t *__restrict__ flags) {
    const int64_t total = m * n;
    int32_t f = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / m;
        const float v = M[c * ld + (e - c * m)];
        if (!(v >= 0.0f)) f |= (v < 0.0f) ? 1 : 2;   // NaN fails both comparisons
        else if (v == INFINITY) f |= 2;
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_state_reset(DevState *st) {
    if (threadIdx.x == 0) {
        st->stop = 0;
        st->log_len = 0;
        st->status = 0;
        st->stopped = 0;
        st->last_rel = 0.0;
        st->flags = 0;
    }
}

// ---- BF16 operand copies ---------------------------------------------------------

// FP32 -> BF16, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Y (rows_pad x cols_pad, column stride rows_pad) = BF16 of X (rows x cols,
// column stride ldx), zero outside.  Grid: x over rows_pad, y over cols_pad.
__global__ __launch_bounds__(256) void k_to_bf16_cols(const float *__restrict__ X, int64_t ldx,
                                                      int64_t rows, int64_t cols,
                                                      uint16_t *__restrict__ Y, int64_t rows_pad,
                                                      int64_t cols_pad) {
    const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i >= rows_pad) return;
    for (int64_t c = blockIdx.y; c < cols_pad; c += gridDim.y)
        Y[c * rows_pad + i] = (i < rows && c < cols) ? bf16_rne(X[c * ldx + i]) : (uint16_t)0;
}

// K-packed copy for the A-pass: element (i, j) of X (rows x cols, column
// stride ldx) at ((i/16 * G + j/8) * 16 + i%16) * 8 + j%8, G = cols_pad / 8,
// zero outside.  One thread per 8-column group of one row.
__global__ __launch_bounds__(256) void k_pack_bf16(const float *__restrict__ X, int64_t ldx,
                                                   int64_t rows, int64_t cols,
                                                   uint16_t *__restrict__ Y, int64_t rows16,
                                                   int64_t cols_pad) {
    const int64_t G = cols_pad / 8;
    const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;   // (panel, group, row in panel)
    if (e >= rows16 / 16 * G * 16) return;
    const int ii = (int)(e & 15);
    const int64_t pg = e >> 4, p = pg / G, g = pg - p * G;
    const int64_t i = p * 16 + ii;
    uint16_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t j = g * 8 + q;
        v[q] = (i < rows && j < cols) ? bf16_rne(X[j * ldx + i]) : (uint16_t)0;
    }
    uint4 w;
    w.x = v[0] | ((uint32_t)v[1] << 16);
    w.y = v[2] | ((uint32_t)v[3] << 16);
    w.z = v[4] | ((uint32_t)v[5] << 16);
    w.w = v[6] | ((uint32_t)v[7] << 16);
    *reinterpret_cast<uint4 *>(Y + e * 8) = w;
}

// Both BF16 copies of a streaming level in one pass over X: the K-packed
// copy of k_pack_bf16 (Ya: rows16 x cols_pad) and the column-panelled copy
// for the streaming C-pass (Yc: element (i, j) at ((j/16 * S + i/32) * 4 +
// i%32/8) * 128 + j%16 * 8 + i%8, S = rows_pad / 32, columns up to cols
// rounded up to 16), zero outside X.
// Block = 32 x 32 tile (rows_pad and cols_pad are multiples of 32 and cover
// both copies): 8 lanes load a column's 32 rows (128 contiguous bytes, float4
// where aligned), the tile goes through LDS as BF16, then 128 threads write
// its two 1 KB panel-steps of Yc and 128 its eight 256-byte (row panel,
// column group) runs of Ya, 16 bytes each.
__global__ __launch_bounds__(256) void k_pack_bf16_both(const float *__restrict__ X, int64_t ldx,
                                                        int64_t rows, int64_t cols,
                                                        uint16_t *__restrict__ Ya,
                                                        int64_t cols_pad,
                                                        uint16_t *__restrict__ Yc,
                                                        int64_t rows_pad) {
    __shared__ uint16_t T[32 * 32];   // T[c * 32 + r]
    const int64_t ntr = rows_pad / 32;
    const int64_t rt = blockIdx.x % ntr, ct = blockIdx.x / ntr;
    const int64_t i0 = rt * 32, j0 = ct * 32;
    const int t = threadIdx.x;
    {
        const int c = t >> 3, r = (t & 7) * 4;
        const int64_t j = j0 + c, i = i0 + r;
        uint16_t v[4];
        const float *xc = X + j * ldx + i;
        if (j < cols && i + 3 < rows && (ldx & 3) == 0 && ((uintptr_t)xc & 15) == 0) {
            const float4 f = *reinterpret_cast<const float4 *>(xc);
            v[0] = bf16_rne(f.x); v[1] = bf16_rne(f.y); v[2] = bf16_rne(f.z); v[3] = bf16_rne(f.w);
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                v[u] = (j < cols && i + u < rows) ? bf16_rne(xc[u]) : (uint16_t)0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) T[c * 32 + r + u] = v[u];
    }
    __syncthreads();
    uint16_t w[8];
    if (t < 128) {   // Yc: panel pan of the tile, entry e of its 1 KB block
        const int pan = t >> 6, e = t & 63, g = e >> 4, jj = e & 15;
        const int64_t P = ct * 2 + pan;
        if (P * 16 >= cols) return;   // past the panelled columns
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = T[(pan * 16 + jj) * 32 + g * 8 + u];
        const int64_t S = rows_pad / 32;
        uint4 o;
        o.x = w[0] | ((uint32_t)w[1] << 16);
        o.y = w[2] | ((uint32_t)w[3] << 16);
        o.z = w[4] | ((uint32_t)w[5] << 16);
        o.w = w[6] | ((uint32_t)w[7] << 16);
        *reinterpret_cast<uint4 *>(Yc + (P * S + rt) * 512 + e * 8) = o;
    } else {         // Ya: run (row panel pp, column group gg) of the tile, row ii
        const int tt = t - 128, ch = tt >> 4, pp = ch >> 2, gg = ch & 3, ii = tt & 15;
        const int64_t prow = rt * 2 + pp;
        const int64_t rows16 = (rows + 15) / 16 * 16;
        if (prow * 16 >= rows16) return;
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = T[(gg * 8 + q) * 32 + pp * 16 + ii];
        const int64_t G = cols_pad / 8, g8 = ct * 4 + gg;
        uint4 o;
        o.x = w[0] | ((uint32_t)w[1] << 16);
        o.y = w[2] | ((uint32_t)w[3] << 16);
        o.z = w[4] | ((uint32_t)w[5] << 16);
        o.w = w[6] | ((uint32_t)w[7] << 16);
        *reinterpret_cast<uint4 *>(Ya + ((prow * G + g8) * 16 + ii) * 8) = o;
    }
}

// ---- grouped setup kernels (one launch over many problems) ------------------

__global__ __launch_bounds__(256) void k_xfer_many(const XferJob *__restrict__ jobs,
                                                   const int2 *__restrict__ bmap) {
    const int2 jt = bmap[blockIdx.x];
    const XferJob &J = jobs[jt.x];
    if (stopped(J.stop)) return;
    const int hc = (J.h + 1) / 2, wc = (J.w + 1) / 2;
    const bool down = J.kind == 1;
    const int ho = down ? hc : J.h, wo = down ? wc : J.w;
    const int mo = ho * wo;
    const int pt = (mo + 255) / 256;
    const int p = (jt.y % pt) * 256 + threadIdx.x;
    if (p >= mo) return;
    const int64_t c0 = (int64_t)(jt.y / pt) * 16;
    const int y = p / wo, x = p - y * wo;
    const Taps ty = down ? restrict_taps(y, J.h, J.xfer) : prolong_taps(y, hc, J.xfer);
    const Taps tx = down ? restrict_taps(x, J.w, J.xfer) : prolong_taps(x, wc, J.xfer);
    const int rowlen = down ? J.w : wc;
    for (int64_t col = c0; col < c0 + 16 && col < J.ncols; ++col)
        J.Y[col * mo + p] = stencil(J.X + col * J.ldx, rowlen, ty, tx);
}

__global__ __launch_bounds__(256) void k_norm_parts_many(const NormJob *__restrict__ jobs,
                                                         const int2 *__restrict__ bmap) {
    __shared__ double scratch[4];
    const int2 jt = bmap[blockIdx.x];
    const NormJob &J = jobs[jt.x];
    double acc = sumsq_part(J.X, J.ld, J.rows, J.ncols, jt.y, J.nparts);
    acc = block_sum_f64<256>(acc, scratch);
    if (threadIdx.x == 0) J.parts[jt.y] = acc;
}

__global__ __launch_bounds__(256) void k_norm_final_many(const NormJob *__restrict__ jobs) {
    __shared__ double scratch[4];
    const NormJob &J = jobs[blockIdx.x];
    double acc = 0.0;
    for (int i = threadIdx.x; i < J.nparts; i += 256) acc += J.parts[i];
    acc = block_sum_f64<256>(acc, scratch);
    if (threadIdx.x == 0) *J.out = acc;
}

__global__ void k_state_reset_many(DevState *const *__restrict__ sts, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        DevState *st = sts[i];
        st->stop = 0;
        st->log_len = 0;
        st->status = 0;
        st->stopped = 0;
        st->last_rel = 0.0;
        st->flags = 0;
    }
}

__global__ void k_gather_states(DevState *const *__restrict__ sts, int count,
                                DevState *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = *sts[i];
}

inline int grid_for(int64_t total, int cap = 8192) {
    int64_t g = (total + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_restrict(int xfer, int h, int w, int64_t ncols, const float *X, int64_t ldx,
                           float *Y, const int32_t *stop, hipStream_t s) {
    const int hc = (h + 1) / 2, wc = (w + 1) / 2;
    const int mc = hc * wc;
    if (mc == 0 || ncols == 0) return hipSuccess;
    if (ncols <= 64) {
        const dim3 grid((mc + 255) / 256, (unsigned)ncols);
        k_restrict<1><<<grid, 256, 0, s>>>(X, ldx, Y, h, w, hc, wc, ncols, xfer, stop);
    } else {
        const int64_t groups = (ncols + 3) / 4;
        const dim3 grid((mc + 255) / 256, (unsigned)std::min<int64_t>(groups, 65535));
        k_restrict<4><<<grid, 256, 0, s>>>(X, ldx, Y, h, w, hc, wc, ncols, xfer, stop);
    }
    return hipGetLastError();
}

hipError_t launch_prolong(int xfer, int h, int w, int64_t ncols, const float *Y, float *X,
                          const int32_t *stop, hipStream_t s) {
    const int hc = (h + 1) / 2, wc = (w + 1) / 2;
    const int mf = h * w;
    if (mf == 0 || ncols == 0) return hipSuccess;
    const dim3 grid((mf + 255) / 256, (unsigned)std::min<int64_t>(ncols, 65535));
    k_prolong<<<grid, 256, 0, s>>>(Y, X, h, w, hc, wc, ncols, xfer, stop);
    return hipGetLastError();
}

hipError_t launch_xfer_cols(int restrict_op, int xfer, int64_t rows, int64_t N, const float *X,
                            int64_t xi, int64_t xj, float *Y, int64_t yi, int64_t yj,
                            const int32_t *stop, hipStream_t s) {
    const int64_t Nout = restrict_op ? (N + 1) / 2 : N;
    const int64_t total = rows * Nout;
    if (total <= 0) return hipSuccess;
    const int i_fast = xi == 1 ? 1 : 0;
    k_xfer_cols<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(restrict_op, xfer, rows, N, Nout,
                                                                X, xi, xj, Y, yi, yj, i_fast,
                                                                stop);
    return hipGetLastError();
}

hipError_t launch_sumsq(const float *X, int64_t ld, int64_t rows, int64_t ncols, double *parts,
                        int nparts, double *out, hipStream_t s) {
    k_sumsq_partial<<<nparts, 256, 0, s>>>(X, ld, rows, ncols, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sum_parts<<<1, 256, 0, s>>>(parts, nparts, out);
    return hipGetLastError();
}

hipError_t launch_check_input(const float *M, int64_t ld, int64_t m, int64_t n, int32_t *flags,
                              hipStream_t s) {
    k_check_input<<<grid_for(m * n, 4096), 256, 0, s>>>(M, ld, m, n, flags);
    return hipGetLastError();
}

hipError_t launch_xfer_many(const XferJob *jobs, const int2 *bmap, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    k_xfer_many<<<blocks, 256, 0, s>>>(jobs, bmap);
    return hipGetLastError();
}

hipError_t launch_norms_many(const NormJob *jobs, const int2 *bmap, int blocks, int njobs,
                             hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    k_norm_parts_many<<<blocks, 256, 0, s>>>(jobs, bmap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_norm_final_many<<<njobs, 256, 0, s>>>(jobs);
    return hipGetLastError();
}

hipError_t launch_state_reset_many(DevState *const *states, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_state_reset_many<<<(count + 255) / 256, 256, 0, s>>>(states, count);
    return hipGetLastError();
}

hipError_t launch_gather_states(DevState *const *states, int count, DevState *out,
                                hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_gather_states<<<(count + 255) / 256, 256, 0, s>>>(states, count, out);
    return hipGetLastError();
}

hipError_t launch_to_bf16_cols(const float *X, int64_t ldx, int64_t rows, int64_t cols,
                               uint16_t *Y, int64_t rows_pad, int64_t cols_pad, hipStream_t s) {
    if (rows_pad <= 0 || cols_pad <= 0) return hipSuccess;
    const dim3 grid((unsigned)((rows_pad + 255) / 256), (unsigned)std::min<int64_t>(cols_pad, 65535));
    k_to_bf16_cols<<<grid, 256, 0, s>>>(X, ldx, rows, cols, Y, rows_pad, cols_pad);
    return hipGetLastError();
}

hipError_t launch_pack_bf16(const float *X, int64_t ldx, int64_t rows, int64_t cols, uint16_t *Y,
                            int64_t cols_pad, hipStream_t s) {
    const int64_t rows16 = (rows + 15) / 16 * 16;
    const int64_t total = rows16 / 16 * (cols_pad / 8) * 16;
    if (total <= 0) return hipSuccess;
    k_pack_bf16<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(X, ldx, rows, cols, Y, rows16,
                                                                cols_pad);
    return hipGetLastError();
}

hipError_t launch_pack_bf16_both(const float *X, int64_t ldx, int64_t rows, int64_t cols,
                                 uint16_t *Ya, int64_t cols_pad, uint16_t *Yc, int64_t rows_pad,
                                 hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (rows_pad % 32 != 0 || rows_pad < rows || cols_pad % 32 != 0 || cols_pad < cols)
        return hipErrorInvalidValue;
    const int64_t blocks = rows_pad / 32 * (cols_pad / 32);
    k_pack_bf16_both<<<(unsigned)blocks, 256, 0, s>>>(X, ldx, rows, cols, Ya, cols_pad, Yc,
                                                      rows_pad);
    return hipGetLastError();
}

hipError_t launch_state_reset(DevState *st, hipStream_t s) {
    k_state_reset<<<1, 64, 0, s>>>(st);
    return hipGetLastError();
}

}  // namespace nmf
