// Multilevel nonnegative tensor factorisation (the extension Section 7.1
// proposes): X (I x J x K, mode 1 the pixels of the image grid) ~ sum_r
// a_r o b_r o c_r, each factor updated in turn by the HALS steps of Alg. 3 on
// its unfolding.
//
// The mode-1 update is the matrix HALS V update with M = X_(1) (I x JK, column
// j + J k) and W = (C kr B)^T (R x JK, the Khatri-Rao product): it runs on the
// regular A-pass.  The C-pass, D reduction and product store of the matrix path
// then give Y = A^T X_(1) (R x JK, FP64) and D = A^T A, from which the other
// two modes need only small contractions:
//   B: a_j[s] = sum_k Y[s, j + J k] C[k, s],  Gram D o (C^T C)
//   C: a_k[s] = sum_j Y[s, j + J k] B[j, s],  Gram D o (B^T B) (new B)
// k_ntf_mode forms a row's vector and updates the row (16 lanes per row, FP64,
// the row_update of the matrix kernels); k_ntf_gram forms the factor Grams and
// the mode-1 Gram (B^T B) o (C^T C) (the Gram of the exact Khatri-Rao product,
// used by the A-pass instead of the Gram of its FP32-rounded copy); k_ntf_kr
// rebuilds (C kr B)^T and its transposed copy for the next A-pass.
// The error uses the Gram form ||X||^2 - 2 <X_(3) (B kr A), C> +
// sum (A^T A o B^T B o C^T C), the middle term from the C update's vectors.
#include "device_common.h"
#include "nmf_internal.h"
#include "sweep_device.h"

namespace nmf {

namespace {

// One block of 256 threads updates 16 rows of a factor F (stored transposed,
// r x L row-major: entry (s, row) at s * L + row).  Row `row`'s vector is
// a[s] = sum_o Y[s, row * sa + o * sb] O[s, o] over the other factor O (r x Lo,
// transposed), and the Gram of the update is D o Go.  rparts (optional): one
// partial per block of sum_rows <a, new row>.
template <int RT>
__global__ __launch_bounds__(256) void k_ntf_mode(const double *__restrict__ Y, int64_t n,
                                                  const double *__restrict__ D,
                                                  const double *__restrict__ Go,
                                                  float *__restrict__ Ft, int64_t L,
                                                  const float *__restrict__ Ot, int64_t Lo,
                                                  int64_t sa, int64_t sb, int r,
                                                  double *__restrict__ rparts,
                                                  const int32_t *stop) {
    constexpr int RPAD = 16 * RT, GS = RPAD + 1;
    __shared__ double Gs[RPAD * GS];
    __shared__ double Gi[RPAD];
    __shared__ double red[4];
    if (stopped(stop)) return;
    const int tid = threadIdx.x;
    for (int e = tid; e < RPAD * RPAD; e += 256) {
        const int a = e / RPAD, b = e % RPAD;
        Gs[a * GS + b] = (a < r && b < r) ? D[a * r + b] * Go[a * r + b] : 0.0;
    }
    if (tid < RPAD) {
        const double g = tid < r ? D[tid * r + tid] * Go[tid * r + tid] : 0.0;
        Gi[tid] = g > 0.0 ? 1.0 / g : 0.0;
    }
    __syncthreads();
    const int p = tid & 15;
    const int64_t row = (int64_t)blockIdx.x * 16 + (tid >> 4);
    const bool ok = row < L;
    double a[RT], x[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int k = 16 * t + p;
        double s = 0.0;
        if (ok && k < r) {
            const double *yk = Y + (int64_t)k * n + row * sa;
            const float *ok_ = Ot + (int64_t)k * Lo;
            for (int64_t o = 0; o < Lo; ++o) s += yk[o * sb] * (double)ok_[o];
        }
        a[t] = s;
        x[t] = (ok && k < r) ? (double)Ft[(int64_t)k * L + row] : 0.0;
    }
    row_update<RT, MODE_HALS>(x, Gs, GS, Gi, a, r, p);
    double part = 0.0;
    if (ok) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + p;
            if (k < r) {
                const float xf = (float)x[t];
                Ft[(int64_t)k * L + row] = xf;
                part += a[t] * (double)xf;
            }
        }
    }
    if (rparts) {
        part = block_sum_f64<256>(part, red);
        if (tid == 0) rparts[blockIdx.x] = part;
    }
}

// G = F F^T (r x r, FP64, exact products of the FP32 entries, summed in index
// order) for a factor stored transposed (r x L row-major); with Hm also
// H = G o Hm.  One block; thread e takes the upper entries e, e + 256, ...
__global__ __launch_bounds__(256) void k_ntf_gram(const float *__restrict__ Ft, int64_t L, int r,
                                                  double *__restrict__ G,
                                                  const double *__restrict__ Hm,
                                                  double *__restrict__ H, const int32_t *stop) {
    if (stopped(stop)) return;
    for (int e = threadIdx.x; e < r * r; e += 256) {
        const int a = e / r, b = e % r;
        if (a > b) continue;
        const float *fa = Ft + (int64_t)a * L, *fb = Ft + (int64_t)b * L;
        double s = 0.0;
        for (int64_t l = 0; l < L; ++l) s += (double)fa[l] * (double)fb[l];
        G[a * r + b] = s;
        G[b * r + a] = s;
        if (Hm) {
            H[a * r + b] = s * Hm[a * r + b];
            H[b * r + a] = s * Hm[b * r + a];
        }
    }
}

// (C kr B)^T: W[s, j + J k] = C[k, s] B[j, s] (r x n row-major, n = J K) and its
// transposed, zero-padded copy Wt (n x rpad, entry s of row idx at wt_pos).
__global__ __launch_bounds__(256) void k_ntf_kr(const float *__restrict__ Bt,
                                                const float *__restrict__ Ct, int64_t J,
                                                int64_t K, int r, int rpad, float *__restrict__ W,
                                                float *__restrict__ Wt, const int32_t *stop) {
    if (stopped(stop)) return;
    const int64_t n = J * K;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n) return;
    const int64_t j = idx % J, k = idx / J;
    for (int s = 0; s < rpad; ++s) {
        const float v = s < r ? Ct[(int64_t)s * K + k] * Bt[(int64_t)s * J + j] : 0.0f;
        if (s < r) W[(int64_t)s * n + idx] = v;
        Wt[idx * rpad + wt_pos(s, rpad / 16)] = v;
    }
}

}  // namespace

int ntf_mode_blocks(int64_t rows) { return (int)((rows + 15) / 16); }

hipError_t launch_ntf_mode(int rpad, const double *Y, int64_t n, const double *D,
                           const double *Go, float *Ft, int64_t L, const float *Ot, int64_t Lo,
                           int64_t sa, int64_t sb, int r, double *rparts, const int32_t *stop,
                           hipStream_t s) {
    const int blocks = ntf_mode_blocks(L);
    switch (rpad) {
        case 16: k_ntf_mode<1><<<blocks, 256, 0, s>>>(Y, n, D, Go, Ft, L, Ot, Lo, sa, sb, r, rparts, stop); break;
        case 32: k_ntf_mode<2><<<blocks, 256, 0, s>>>(Y, n, D, Go, Ft, L, Ot, Lo, sa, sb, r, rparts, stop); break;
        case 48: k_ntf_mode<3><<<blocks, 256, 0, s>>>(Y, n, D, Go, Ft, L, Ot, Lo, sa, sb, r, rparts, stop); break;
        case 64: k_ntf_mode<4><<<blocks, 256, 0, s>>>(Y, n, D, Go, Ft, L, Ot, Lo, sa, sb, r, rparts, stop); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ntf_gram(const float *Ft, int64_t L, int r, double *G, const double *Hm,
                           double *H, const int32_t *stop, hipStream_t s) {
    k_ntf_gram<<<1, 256, 0, s>>>(Ft, L, r, G, Hm, H, stop);
    return hipGetLastError();
}

hipError_t launch_ntf_kr(const float *Bt, const float *Ct, int64_t J, int64_t K, int r, int rpad,
                         float *W, float *Wt, const int32_t *stop, hipStream_t s) {
    const int64_t n = J * K;
    k_ntf_kr<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(Bt, Ct, J, K, r, rpad, W, Wt, stop);
    return hipGetLastError();
}

}  // namespace nmf
