// Exact FP64 nonnegative least squares for ANLS (Alg. 1, Appendix A.2).
//
// The V half-step is m independent problems  min_{x>=0} 0.5 x^T B x - a_i^T x
// (B = W W^T, a_i = row i of M W^T), the W half-step n problems with
// (D = V^T V, c_j = column j of V^T M).  With a positive definite Gram the
// minimiser is unique, so any exact method gives the same point.  Each
// problem is solved by block principal pivoting (the exchange method the
// paper's Section 2.1 footnote points to for ANLS): with the passive set F,
// solve G[F,F] z = b[F] (Cholesky), take the gradient g = G z - b on the
// variables outside F, and call infeasible every passive variable with z < 0
// and every active one with g < -tol; all infeasible variables change sides
// at once while their number keeps falling, for three more rounds after it
// stops falling, and then only the highest-indexed one (the backup rule that
// makes the exchange finite).  No infeasible variable: z is the solution.
// Unlike an active-set method that adds one variable per solve, a whole
// support change costs one solve per round, which keeps the first sweeps
// (random start, all variables passive) short.
//
// One 64-wide wave per problem, lane k owning variable k (r <= 64).  The
// passive set starts from the support of the current factor row (the
// previous ANLS solution), which changes the path but not the result.
// Variables with G_kk = 0 (a zero factor column) take no part and keep their
// value.  Cholesky: lane at passive position p owns row p of the factor in
// wave-private LDS; column values move between lanes with shuffles.

#include "device_common.h"
#include "nmf_internal.h"

namespace nmf {

namespace {

__device__ __forceinline__ double wave_max_f64(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
    return x;
}

__device__ __forceinline__ double wave_min_f64(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, kWave));
    return x;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Solve G[P,P] z = b[P]; lanes in P receive z.  S: wave-private LDS of
// RPAD x (RPAD+1) doubles.  Returns false if a pivot is not positive.
template <int RPAD>
__device__ bool solve_passive(const double *__restrict__ Gs, double *__restrict__ S, uint64_t P,
                              double b, double &z, int lane) {
    constexpr int GS = RPAD + 1;
    const bool inP = (P >> lane) & 1ull;
    const int p = __popcll(P);
    const int pi = inP ? __popcll(P & ((1ull << lane) - 1ull)) : 0;
    double *Srow = S + pi * GS;
    wave_lds_sync();   // earlier readers of S are done
    {
        uint64_t rem = P;
        for (int pk = 0; rem; ++pk) {
            const int k = __ffsll((unsigned long long)rem) - 1;
            rem &= rem - 1ull;
            if (inP && pk <= pi) Srow[pk] = Gs[lane * GS + k];
        }
    }
    double rhs = inP ? b : 0.0;
    uint64_t remc = P;
    for (int c = 0; c < p; ++c) {
        const int lc = __ffsll((unsigned long long)remc) - 1;
        remc &= remc - 1ull;
        const double piv = __shfl(inP ? Srow[c] : 0.0, lc, kWave);
        if (!(piv > 0.0)) return false;
        const double lcc = sqrt(piv);
        double lic = 0.0;
        if (inP && pi > c) {
            lic = Srow[c] / lcc;
            Srow[c] = lic;
            S[c * GS + pi] = lic;        // transposed copy into the unused upper part of row c
        } else if (inP && pi == c) {
            Srow[c] = lcc;
        }
        uint64_t remk = remc;
        for (int k = c + 1; k < p; ++k) {
            const int lk = __ffsll((unsigned long long)remk) - 1;
            remk &= remk - 1ull;
            const double lkc = __shfl(lic, lk, kWave);
            if (inP && pi >= k) Srow[k] -= lic * lkc;
        }
        const double yc = __shfl(rhs, lc, kWave) / lcc;   // forward substitution, merged
        if (inP && pi == c) rhs = yc;
        else if (inP && pi > c) rhs -= lic * yc;
    }
    wave_lds_sync();   // transposed entries written by other lanes
    uint64_t remb = P;
    for (int c = p - 1; c >= 0; --c) {
        const int lc = 63 - __clzll((unsigned long long)remb);
        remb &= ~(1ull << lc);
        const double lcc = __shfl(inP ? Srow[pi] : 0.0, lc, kWave);
        const double zc = __shfl(rhs, lc, kWave) / lcc;
        if (inP && pi == c) rhs = zc;
        else if (inP && pi < c) rhs -= Srow[c] * zc;     // S[pi][c] = L[c][pi]
    }
    z = rhs;
    return true;
}

// Block principal pivoting for one problem; x is the warm start on entry and
// the solution on exit (lane k holds variable k).  Returns false on a
// non-positive pivot, or if the exchange has not ended after 8 RPAD + 16
// rounds (x is then left unchanged).
template <int RPAD>
__device__ bool wave_nnls(const double *__restrict__ Gs, double *__restrict__ S, double b,
                          double &x, int r, int lane) {
    constexpr int GS = RPAD + 1;
    const bool valid = lane < r;
    const bool live = valid && Gs[lane * GS + lane] > 0.0;
    const double tol = 1e-12 * fmax(1.0, wave_max_f64(live ? fabs(b) : 0.0));
    uint64_t F = __ballot(live && x > 0.0 && x < INFINITY);
    int ninf = RPAD + 1, backup = 3;
    for (int round = 0; round < 8 * RPAD + 16; ++round) {
        double z = 0.0;
        if (F != 0ull && !solve_passive<RPAD>(Gs, S, F, b, z, lane)) return false;
        const bool inF = (F >> lane) & 1ull;
        // gradient (G z - b)_k of the variables outside F (z is 0 there)
        double gz = 0.0;
        uint64_t rem = F;
        while (rem) {
            const int l = __ffsll((unsigned long long)rem) - 1;
            rem &= rem - 1ull;
            const double zl = __shfl(z, l, kWave);
            if (valid) gz += Gs[lane * GS + l] * zl;
        }
        const bool bad = live && (inF ? !(z >= 0.0) : (gz - b) < -tol);
        const uint64_t V = __ballot(bad);
        if (V == 0ull) {
            if (inF) x = z;
            else if (live) x = 0.0;
            return true;
        }
        const int nv = __popcll(V);
        if (nv < ninf) {
            ninf = nv;
            backup = 3;
            F ^= V;
        } else if (backup > 0) {
            --backup;
            F ^= V;
        } else {
            F ^= 1ull << (63 - __clzll((unsigned long long)V));
        }
    }
    return false;
}

// COLS = false: problems are rows i of V (x = V[i + k m], rhs = A[i + k m]).
// COLS = true : problems are columns j of W (x = W[k n + j], rhs = C[k n + j]);
//               also emits the FP64 partial <C, W_new> per block.
template <int RPAD, int WAVES, bool COLS>
__global__ __launch_bounds__(WAVES * 64) void k_nnls(const double *__restrict__ Gd,
                                                     const double *__restrict__ Rhs, int64_t count,
                                                     int r, float *__restrict__ X,
                                                     float *__restrict__ Xt,
                                                     double *__restrict__ rparts,
                                                     int32_t *__restrict__ flags,
                                                     const int32_t *stop) {
    constexpr int GS = RPAD + 1;
    __shared__ double Gs[RPAD * GS];
    __shared__ double Ss[WAVES * RPAD * GS];
    __shared__ double red[WAVES];
    if (stopped(stop)) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int e = tid; e < RPAD * RPAD; e += WAVES * 64) {
        const int a = e / RPAD, c = e % RPAD;
        Gs[a * GS + c] = (a < r && c < r) ? Gd[a * r + c] : 0.0;
    }
    __syncthreads();
    double *S = Ss + wave * RPAD * GS;
    double part = 0.0;
    bool failed = false;
    for (int64_t prob = (int64_t)blockIdx.x * WAVES + wave; prob < count;
         prob += (int64_t)gridDim.x * WAVES) {
        const bool ok = lane < r;
        const int64_t idx = COLS ? (int64_t)lane * count + prob : prob + (int64_t)lane * count;
        const double b = ok ? Rhs[idx] : 0.0;
        double x = ok ? (double)X[idx] : 0.0;
        if (!wave_nnls<RPAD>(Gs, S, b, x, r, lane)) failed = true;
        if (ok) {
            const float xf = (float)x;
            X[idx] = xf;
            if (COLS) part += b * (double)xf;
        }
        if (COLS && lane < RPAD) Xt[prob * RPAD + wt_pos(lane, RPAD / 16)] = ok ? (float)x : 0.0f;
    }
    if (failed && lane == 0) atomicOr(flags, 4);
    if constexpr (COLS) {
        part = wave_sum_f64(part);
        __syncthreads();
        if (lane == 0) red[wave] = part;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int i = 0; i < WAVES; ++i) t += red[i];
            rparts[blockIdx.x] = t;
        }
    }
}

template <int RPAD, bool COLS>
hipError_t launch_nnls_t(const double *Gd, const double *Rhs, int64_t count, int r, float *X,
                         float *Xt, double *rparts, int32_t *flags, const int32_t *stop,
                         int blocks, hipStream_t s) {
    constexpr int WAVES = (RPAD >= 64) ? 2 : 4;
    k_nnls<RPAD, WAVES, COLS><<<blocks, WAVES * 64, 0, s>>>(Gd, Rhs, count, r, X, Xt, rparts, flags, stop);
    return hipGetLastError();
}

}  // namespace

int nnls_cols_blocks(int64_t n) {
    int64_t b = (n + 3) / 4;
    return (int)(b > 1024 ? 1024 : (b < 1 ? 1 : b));
}

static hipError_t nnls_dispatch(int rpad, bool cols, const double *Gd, const double *Rhs,
                                int64_t count, int r, float *X, float *Xt, double *rparts,
                                int32_t *flags, const int32_t *stop, int blocks, hipStream_t s) {
    switch (rpad) {
        case 16: return cols ? launch_nnls_t<16, true>(Gd, Rhs, count, r, X, Xt, rparts, flags, stop, blocks, s)
                             : launch_nnls_t<16, false>(Gd, Rhs, count, r, X, Xt, rparts, flags, stop, blocks, s);
        case 32: return cols ? launch_nnls_t<32, true>(Gd, Rhs, count, r, X, Xt, rparts, flags, stop, blocks, s)
                             : launch_nnls_t<32, false>(Gd, Rhs, count, r, X, Xt, rparts, flags, stop, blocks, s);
        case 48: return cols ? launch_nnls_t<48, true>(Gd, Rhs, count, r, X, Xt, rparts, flags, stop, blocks, s)
                             : launch_nnls_t<48, false>(Gd, Rhs, count, r, X, Xt, rparts, flags, stop, blocks, s);
        case 64: return cols ? launch_nnls_t<64, true>(Gd, Rhs, count, r, X, Xt, rparts, flags, stop, blocks, s)
                             : launch_nnls_t<64, false>(Gd, Rhs, count, r, X, Xt, rparts, flags, stop, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_nnls_rows(int rpad, const double *Gd, const double *A, int64_t m, int r,
                            float *V, int32_t *flags, const int32_t *stop, hipStream_t s) {
    int64_t b = (m + 3) / 4;
    const int blocks = (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
    return nnls_dispatch(rpad, false, Gd, A, m, r, V, nullptr, nullptr, flags, stop, blocks, s);
}

hipError_t launch_nnls_cols(int rpad, const double *Gd, const double *C, int64_t n, int r,
                            float *W, float *Wt, double *rparts, int32_t *flags,
                            const int32_t *stop, hipStream_t s) {
    return nnls_dispatch(rpad, true, Gd, C, n, r, W, Wt, rparts, flags, stop, nnls_cols_blocks(n),
                         s);
}

}  // namespace nmf
