// FP64 Gram matrices G = X X^T of r vectors (B = W W^T over n, D = V^T V
// over m), the r x r products of Alg. 2 / Alg. 3 and eq. subNNLS.
//
// Products of two FP32 values are exact in FP64, so every partial sum below
// rounds only in the FP64 additions.  Split-length partials per block, then a
// fixed-order reduction, so results are bitwise reproducible and G is
// bitwise symmetric (entries (a,b) and (b,a) sum the same products in the same
// order).

#include "device_common.h"
#include "nmf_internal.h"

namespace nmf {

namespace {

template <int RPAD>
__global__ __launch_bounds__(256) void k_gram_partial(const float *__restrict__ X, int64_t ldx,
                                                      int64_t L, int r, int64_t chunk,
                                                      double *__restrict__ parts,
                                                      const int32_t *stop) {
    constexpr int TB = RPAD / 4;   // threads per side of the 4x4-entry tiling
    constexpr int TT = 64;         // vector positions staged per round
    __shared__ float Xs[TT][RPAD + 1];
    if (stopped(stop)) return;
    const int64_t t_begin = (int64_t)blockIdx.x * chunk;
    const int64_t t_end = (t_begin + chunk < L) ? t_begin + chunk : L;
    const int tid = threadIdx.x;
    const int ta = tid / TB, tb = tid % TB;
    const bool active = tid < TB * TB;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

    for (int64_t t0 = t_begin; t0 < t_end; t0 += TT) {
        __syncthreads();
        for (int e = tid; e < TT * RPAD; e += 256) {
            const int tt = e % TT, a = e / TT;
            const int64_t t = t0 + tt;
            Xs[tt][a] = (a < r && t < t_end) ? X[(int64_t)a * ldx + t] : 0.0f;
        }
        __syncthreads();
        if (active) {
            for (int tt = 0; tt < TT; ++tt) {
                double xa[4], xb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    xa[i] = (double)Xs[tt][4 * ta + i];
                    xb[i] = (double)Xs[tt][4 * tb + i];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(xa[i], xb[j], acc[i][j]);
            }
        }
    }
    if (active) {
        double *out = parts + (int64_t)blockIdx.x * RPAD * RPAD;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) out[(4 * ta + i) * RPAD + 4 * tb + j] = acc[i][j];
    }
}

__global__ __launch_bounds__(256) void k_gram_final(const double *__restrict__ parts, int nparts,
                                                    int rpad, int r, double *__restrict__ Gd,
                                                    float *__restrict__ Gf, const int32_t *stop) {
    if (stopped(stop)) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= r * r) return;
    const int a = e / r, b = e % r;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += parts[(int64_t)p * rpad * rpad + a * rpad + b];
    Gd[e] = s;
    if (Gf) Gf[e] = (float)s;
}

}  // namespace

hipError_t launch_gram(int rpad, int r, int64_t L, const float *X, int64_t ldx, int parts,
                       int64_t chunk, double *gparts, double *Gd, float *Gf, const int32_t *stop,
                       hipStream_t s) {
    switch (rpad) {
        case 16: k_gram_partial<16><<<parts, 256, 0, s>>>(X, ldx, L, r, chunk, gparts, stop); break;
        case 32: k_gram_partial<32><<<parts, 256, 0, s>>>(X, ldx, L, r, chunk, gparts, stop); break;
        case 48: k_gram_partial<48><<<parts, 256, 0, s>>>(X, ldx, L, r, chunk, gparts, stop); break;
        case 64: k_gram_partial<64><<<parts, 256, 0, s>>>(X, ldx, L, r, chunk, gparts, stop); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_gram_final<<<(r * r + 255) / 256, 256, 0, s>>>(gparts, parts, rpad, r, Gd, Gf, stop);
    return hipGetLastError();
}

}  // namespace nmf
