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
// value.  The passive systems are solved by a register-resident Cholesky
// (chol_solve), one factor row per lane.

#include "device_common.h"
#include "nmf_internal.h"

namespace nmf {

namespace {

__device__ __forceinline__ double wave_max_f64(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
    return x;
}

// v, as a value the compiler cannot see through (an empty asm taking dep as
// an input): address arithmetic built on it is redone where it is used.
__device__ __forceinline__ int opaque(int v, uint32_t dep) {
    asm volatile("" : "+v"(v) : "s"(dep));
    return v;
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Solve G[F,F] z = b[F] for the passive set F (bit k = variable k); lanes in F
// receive z, the others 0.  Lane i keeps row i of G[F,F] in registers, as an
// RPAD x RPAD matrix whose rows and columns outside F are zero (the steps of
// those variables are skipped, so no compaction is needed), and the
// factorisation is right-looking:
// at step c the pivot lane's diagonal gives L_cc, every lane i > c forms
// L_ic and all lanes apply a_i[k] -= L_ic L_kc for k > c, the column L_.c
// reaching them through a 64-double LDS slot bc (one store per lane, broadcast
// reads).  Because each lane holds its whole symmetric row and the update
// runs over every k > c, the upper part of row i ends as a_i[k] = L_ki L_ii
// (k > i): lane i then holds column i of L as well, and the back substitution
// needs one broadcast per step.  The forward substitution runs with the
// factorisation.  Steps of variables outside F are no-ops and skipped.
// Returns false if a pivot is not positive.
template <int RPAD>
__device__ bool chol_solve(const double *__restrict__ Gs, double *bc, uint64_t F, double b,
                           double &z, int lane_in) {
    constexpr int GS = RPAD + 1;
    // the lane comparisons below are redone at every solve rather than kept
    // (as 64-bit lane masks in scalar registers) across the pivoting rounds
    const int lane = opaque(lane_in, (uint32_t)(F >> 32));
    const bool inF = (F >> lane) & 1ull;
    // Gram row of this lane (the padded lanes read row 0 and discard it); the
    // address is made opaque so the row is re-read from LDS at every solve
    // instead of being held in registers across the pivoting rounds
    const double *Gr = Gs + opaque((lane < RPAD ? lane : 0) * GS, (uint32_t)F);
    double a[RPAD];
#pragma unroll
    for (int k = 0; k < RPAD; ++k) {
        const double g = Gr[k];
        a[k] = (inF && ((F >> k) & 1ull)) ? g : 0.0;
    }
    double y = inF ? b : 0.0;
    double inv_own = 0.0;     // 1 / L_ii of this lane's variable
    bool ok = true;
    static_for<RPAD>([&](auto c_c) {
        constexpr int c = decltype(c_c)::value;
        if (!((F >> c) & 1ull)) return;
        const double piv = readlane_f64(a[c], c);
        ok = ok && piv > 0.0;
        const double inv = 1.0 / sqrt(piv > 0.0 ? piv : 1.0);
        const double l = lane > c ? a[c] * inv : 0.0;
        if (lane == c) inv_own = inv;
        const double yc = readlane_f64(y, c) * inv;
        y = lane == c ? yc : fma(-l, yc, y);
        if constexpr (c + 1 < RPAD) {
            // column c to every lane: reads in groups of CG, each group issued
            // one group ahead of the updates that use it
            bc[lane] = l;
            constexpr int CG = 8, K0 = c + 1, NG = (RPAD - K0 + CG - 1) / CG;
            double buf[2][CG];
            auto rd = [&](auto g_c) {
                constexpr int g = decltype(g_c)::value;
                static_for<CG>([&](auto i_c) {
                    constexpr int k = K0 + CG * g + decltype(i_c)::value;
                    if constexpr (k < RPAD) buf[g & 1][k - K0 - CG * g] = bc[k];
                });
            };
            rd(std::integral_constant<int, 0>{});
            static_for<NG>([&](auto g_c) {
                constexpr int g = decltype(g_c)::value;
                if constexpr (g + 1 < NG) rd(std::integral_constant<int, g + 1>{});
                __builtin_amdgcn_sched_barrier(0);
                static_for<CG>([&](auto i_c) {
                    constexpr int k = K0 + CG * g + decltype(i_c)::value;
                    if constexpr (k < RPAD) a[k] = fma(-l, buf[g & 1][k - K0 - CG * g], a[k]);
                });
                __builtin_amdgcn_sched_barrier(0);
            });
        }
    });
    // back substitution, i descending: z_i = (y_i - acc_i / L_ii) / L_ii with
    // acc_i = sum_{k > i} a_i[k] z_k = L_ii sum_{k > i} L_ki z_k
    double acc = 0.0, zz = 0.0;
    static_for<RPAD>([&](auto j_c) {
        constexpr int i = RPAD - 1 - decltype(j_c)::value;
        if (!((F >> i) & 1ull)) return;
        const double zi = readlane_f64((y - acc * inv_own) * inv_own, i);
        if (lane == i) zz = zi;
        acc = fma(a[i], zi, acc);
    });
    z = inF ? zz : 0.0;
    return ok;
}

// Block principal pivoting for one problem; x is the warm start on entry and
// the solution on exit (lane k holds variable k).  Returns false on a
// non-positive pivot, or if the exchange has not ended after 8 RPAD + 16
// rounds (x is then left unchanged).
template <int RPAD>
__device__ bool wave_nnls(const double *__restrict__ Gs, double *bc, double b, double &x, int r,
                          int lane) {
    constexpr int GS = RPAD + 1;
    const bool valid = lane < r;
    const int lr = lane < RPAD ? lane : 0;
    const bool live = valid && Gs[lr * GS + lr] > 0.0;
    const double tol = 1e-12 * fmax(1.0, wave_max_f64(live ? fabs(b) : 0.0));
    uint64_t F = __ballot(live && x > 0.0 && x < INFINITY);
    int ninf = RPAD + 1, backup = 3;
    for (int round = 0; round < 8 * RPAD + 16; ++round) {
        double z = 0.0;
        if (F != 0ull && !chol_solve<RPAD>(Gs, bc, F, b, z, lane)) return false;
        const bool inF = (F >> lane) & 1ull;
        // gradient (G z - b)_k of the variables outside F (z is 0 there)
        bc[lane] = z;
        const double *Gr = Gs + opaque(lr * GS, (uint32_t)round);
        double gz = 0.0;
        static_for<RPAD / 8>([&](auto q_c) {
            constexpr int l0 = 8 * decltype(q_c)::value;
#pragma unroll
            for (int l = l0; l < l0 + 8; ++l) gz = fma(Gr[l], bc[l], gz);
            __builtin_amdgcn_sched_barrier(0);
        });
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
// Waves per SIMD the register allocation aims for: the factor row takes
// 2 RPAD registers per lane.
template <int RPAD>
constexpr int nnls_occupancy() { return RPAD <= 16 ? 4 : (RPAD <= 32 ? 3 : (RPAD <= 48 ? 2 : 1)); }

template <int RPAD, int WAVES, bool COLS>
__global__ __launch_bounds__(WAVES * 64)
__attribute__((amdgpu_waves_per_eu(nnls_occupancy<RPAD>()))) void k_nnls(const double *__restrict__ Gd,
                                                     const double *__restrict__ Rhs, int64_t count,
                                                     int r, float *__restrict__ X,
                                                     float *__restrict__ Xt,
                                                     double *__restrict__ rparts,
                                                     int32_t *__restrict__ flags,
                                                     const int32_t *stop) {
    constexpr int GS = RPAD + 1;
    __shared__ double Gs[RPAD * GS];
    __shared__ double bcs[WAVES * 64];
    __shared__ double red[WAVES];
    if (stopped(stop)) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int e = tid; e < RPAD * RPAD; e += WAVES * 64) {
        const int a = e / RPAD, c = e % RPAD;
        Gs[a * GS + c] = (a < r && c < r) ? Gd[a * r + c] : 0.0;
    }
    __syncthreads();
    double *bc = bcs + wave * 64;
    double part = 0.0;
    bool failed = false;
    for (int64_t prob = (int64_t)blockIdx.x * WAVES + wave; prob < count;
         prob += (int64_t)gridDim.x * WAVES) {
        const bool ok = lane < r;
        const int64_t idx = COLS ? (int64_t)lane * count + prob : prob + (int64_t)lane * count;
        const double b = ok ? Rhs[idx] : 0.0;
        double x = ok ? (double)X[idx] : 0.0;
        if (!wave_nnls<RPAD>(Gs, bc, b, x, r, lane)) failed = true;
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
    // at most the blocks the chip holds at once (256 CUs, 4 SIMDs each, at the
    // kernel's occupancy); each wave then loops over several rows, and the
    // Gram is staged into LDS once per resident block
    const int occ = rpad <= 16 ? 4 : (rpad <= 32 ? 3 : (rpad <= 48 ? 2 : 1));
    const int waves = rpad >= 64 ? 2 : 4;
    const int64_t cap = (int64_t)256 * 4 * occ / waves;
    const int64_t b = (m + waves - 1) / waves;
    const int blocks = (int)(b > cap ? cap : (b < 1 ? 1 : b));
    return nnls_dispatch(rpad, false, Gd, A, m, r, V, nullptr, nullptr, flags, stop, blocks, s);
}

hipError_t launch_nnls_cols(int rpad, const double *Gd, const double *C, int64_t n, int r,
                            float *W, float *Wt, double *rparts, int32_t *flags,
                            const int32_t *stop, hipStream_t s) {
    return nnls_dispatch(rpad, true, Gd, C, n, r, W, Wt, rparts, flags, stop, nnls_cols_blocks(n),
                         s);
}

}  // namespace nmf
