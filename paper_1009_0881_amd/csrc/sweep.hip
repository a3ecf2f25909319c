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

#include "sweep_device.h"

namespace nmf {

namespace {

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
    // Loads are unconditional from clamped, in-bounds addresses (column j of
    // a step past the wave's range or past n reads column n - 1; a row past m
    // reads row 0) and the operands are masked where they are used: a select
    // right after a load would make the compiler wait for it there, which
    // defeats the double buffering.  Rows past m only feed rows of A that are
    // never stored or used; columns outside the range get M = 0.
    auto load = [&](int64_t s, float (&a)[S][RW], float (&b)[S][RT]) {
#pragma unroll
        for (int u = 0; u < S; ++u) {
            const int64_t j = 4 * (s + u) + lk;
            const int64_t jc = j < n ? j : n - 1;
#pragma unroll
            for (int q = 0; q < RW; ++q) a[u][q] = Mr[q][jc * ldm];
            load_wt<RT>(Wt + jc * RPAD, li, b[u]);
        }
    };
    auto compute = [&](int64_t s, const float (&a)[S][RW], const float (&b)[S][RT]) {
#pragma unroll
        for (int u0 = 0; u0 < S; u0 += 4) {      // 4 steps = 16 products per chain
            v4f acc[RW][RT];
#pragma unroll
            for (int q = 0; q < RW; ++q)
#pragma unroll
                for (int t = 0; t < RT; ++t) acc[q][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int u = u0; u < u0 + 4; ++u) {
                const bool ok = (s + u) < s_end && 4 * (s + u) + lk < n;
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    const float av = ok ? a[u][q] : 0.0f;
#pragma unroll
                    for (int t = 0; t < RT; ++t)
                        acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b[u][t], acc[q][t],
                                                                         0, 0, 0);
                }
            }
#pragma unroll
            for (int q = 0; q < RW; ++q)
#pragma unroll
                for (int t = 0; t < RT; ++t) two_sum_acc(hi[q][t], lo[q][t], acc[q][t]);
        }
    };
    // factor rows of the epilogue (16 lanes per row, rows tid/16 + 16i) and
    // the Gram B: loads issued now from clamped addresses, values masked and
    // stored after the main loop, so their latency overlaps it
    constexpr int EPR = TM / 16;
    double xv[UPD ? EPR : 1][RT];
    float xf[UPD ? EPR : 1][RT];
    GramRegs<RPAD> gregs;
    if constexpr (UPD) {
#pragma unroll
        for (int i = 0; i < EPR; ++i) {
            const int64_t vrow = brow + (tid >> 4) + 16 * i;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + (tid & 15);
                xf[i][t] = Vg[(vrow < m ? vrow : m - 1) + (int64_t)(k < r ? k : 0) * m];
            }
        }
        gram_fetch<RPAD>(J.Bd, r, gregs);
    }
    auto epilogue_inputs = [&]() {
        if constexpr (UPD) {
            gram_put<RPAD>(gregs, r, Gs, GS, Gi);
#pragma unroll
            for (int i = 0; i < EPR; ++i) {
                const int64_t vrow = brow + (tid >> 4) + 16 * i;
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const int k = 16 * t + (tid & 15);
                    xv[i][t] = (vrow < m && k < r) ? (double)xf[i][t] : 0.0;
                }
            }
        }
    };
    double *Aw = As + wave * TMW * AS;
    if constexpr (!BF) {
        load(s_begin, a0, b0);
        // unconditional prefetch of the next batch (clamped addresses; see
        // load); the scheduling barriers keep its loads ahead of the compute
        // of the current batch instead of next to their use
        for (int64_t s = s_begin; s < s_end; s += 2 * S) {
            load(s + S, a1, b1);
            __builtin_amdgcn_sched_barrier(0);
            compute(s, a0, b0);
            if (s + S >= s_end) break;
            load(s + 2 * S, a0, b0);
            __builtin_amdgcn_sched_barrier(0);
            compute(s + S, a1, b1);
        }
        epilogue_inputs();
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
        for (int64_t k0 = k_begin; k0 < k_end; k0 += 2 * SB) {
            if (k0 + SB < k_end) loadb(k0 + SB, ma1, wb1);
            computeb(ma0, wb0);
            if (k0 + SB >= k_end) break;
            if (k0 + 2 * SB < k_end) loadb(k0 + 2 * SB, ma0, wb0);
            computeb(ma1, wb1);
        }
        epilogue_inputs();
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
            if (row >= m) continue;
            if (J.Ad) to_global(J.Ad)[row + (int64_t)k * m] = arow(rr)[k];
            else to_global(J.A)[row + (int64_t)k * m] = (float)arow(rr)[k];
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
// C-pass tile: (x = 64-column tile of n, y = chunk of m rows).  The 4 waves
// form 4/WC column groups of WC 16-column tiles times WC row groups: each
// wave covers its columns over 1/WC of the chunk's rows, so a wave's chain of
// dependent loads is WC times shorter than one wave per column tile over the
// whole chunk, and the WC row-group partials are added in LDS (fixed order).
//
// FP32 operands: a lane loads 4 consecutive rows of M and of the r columns of
// V (float4 each) and feeds them to 4 MFMAs, so the k-index of MFMA s maps to
// row i0 + 4*(lane/16) + s; loads are double buffered SB 16-row steps deep.
// The same V registers feed the FP64 MFMAs of the chunk's partial V^T V.
// BF16 operands (prec = 1): K-steps of 32 rows from the column-major BF16
// copies; V^T V from the same BF16 V operands (products exact in FP32).
// The upper-triangle 16x16 tiles of V^T V are numbered row by row and dealt
// to the (block, column group) slots of the chunk, three per slot fused into
// the main loop; a block whose slots own more (only when n is tiny) forms the
// rest in extra passes over its rows.
// ---------------------------------------------------------------------------
template <int RT, int WC>
constexpr size_t cpass_lds_doubles() {
    // row-group partials of C (per wave: WC tiles x RT x 4 x 64 lanes) and of
    // the fused V^T V tiles (3 x 4 x 64)
    return (size_t)(WC - 1) * 4 * (RT * 4 * 64) + (size_t)(WC - 1) * (4 / WC) * 3 * 4 * 64;
}

template <int RT, int WC, int SB, bool BF>
__device__ __forceinline__ void cpass_tile(const Job &J, int tx, int ty, int ntx, double *smem) {
    constexpr int RPAD = RT * 16, DMAX = 3, NCG = 4 / WC, NPAIR = RT * (RT + 1) / 2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lj = lane & 15, lg = lane >> 4;
    const int cg = wave % NCG, rg = wave / NCG;
    const int64_t m = J.m, n = J.n, ldm = J.ldm;
    const int r = J.r;
    const auto V = to_global(J.V);
    const int64_t jb = (int64_t)tx * 64 + cg * 16 * WC;
    const int64_t i_begin = (int64_t)ty * J.chunk;
    const int64_t i_end = (i_begin + J.chunk < m) ? i_begin + J.chunk : m;
    // chunk is a multiple of 64 (FP32) or 128 (BF16): row groups start on
    // 16-row (FP32) or 32-row (BF16) steps
    const int64_t sub = J.chunk / WC;
    const int64_t ra = i_begin + rg * sub;
    const int64_t rb = (ra + sub < i_end) ? ra + sub : i_end;
    const int slot0 = tx * NCG, nslots = ntx * NCG, slot = slot0 + cg;
    auto tile_pair = [&](int idx, int &ta, int &tb) {
        int fa = 0, fb = 0, q = 0;
#pragma unroll
        for (int a2 = 0; a2 < RT; ++a2)
#pragma unroll
            for (int b2 = a2; b2 < RT; ++b2, ++q)
                if (q == idx) {
                    fa = a2;
                    fb = b2;
                }
        ta = fa;
        tb = fb;
    };
    int dta[DMAX], dtb[DMAX];
    bool dok[DMAX];
#pragma unroll
    for (int d = 0; d < DMAX; ++d) {
        const int idx = slot + nslots * d;
        dok[d] = idx < NPAIR;
        tile_pair(idx, dta[d], dtb[d]);
    }
    gmem<const float> *Mc[WC];
    bool jok[WC];
#pragma unroll
    for (int c = 0; c < WC; ++c) {
        const int64_t j = jb + 16 * c + lj;
        jok[c] = j < n;
        Mc[c] = to_global(J.M) + (jok[c] ? j : 0) * ldm;
    }
    const bool vec = ((ldm & 3) == 0) && ((m & 3) == 0) &&
                     (((uintptr_t)J.M & 15) == 0) && (((uintptr_t)V & 15) == 0);
    v4f hi[WC][RT], lo[WC][RT];
    v4d dacc[DMAX];
#pragma unroll
    for (int c = 0; c < WC; ++c)
#pragma unroll
        for (int t = 0; t < RT; ++t) hi[c][t] = lo[c][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int d = 0; d < DMAX; ++d) dacc[d] = v4d{0.0, 0.0, 0.0, 0.0};

    // FP32: rows ib..ib+3 (ib = i0 + 4 lg) of the wave's M columns and of V.
    // Loads are unconditional from clamped, in-bounds addresses (rows past m
    // read the last rows, columns k >= r of V read column 0) and V is masked
    // where it is used (rows outside [ra, rb), k >= r): a select right after
    // a load would make the compiler wait for it there and defeat the double
    // buffering.  M columns past n were clamped to column 0: they only feed
    // entries of C that are not stored.  VEC: float4 loads (m, ldm multiples
    // of 4 and 16-byte aligned bases), else four scalar loads.
    auto load1 = [&](auto vec_c, int64_t i0, v4f (&mv)[WC], v4f (&vv)[RT]) {
        constexpr bool VEC = decltype(vec_c)::value;
        const int64_t ib = i0 + 4 * lg;
        if constexpr (VEC) {
            const int64_t ibc = ib < m ? ib : m - 4;
#pragma unroll
            for (int c = 0; c < WC; ++c) mv[c] = *(gmem<const v4f> *)(Mc[c] + ibc);
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + lj;
                vv[t] = *(gmem<const v4f> *)(V + ibc + (int64_t)(k < r ? k : 0) * m);
            }
        } else {
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                const int64_t ic = ib + s2 < m ? ib + s2 : m - 1;
#pragma unroll
                for (int c = 0; c < WC; ++c) mv[c][s2] = Mc[c][ic];
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const int k = 16 * t + lj;
                    vv[t][s2] = V[ic + (int64_t)(k < r ? k : 0) * m];
                }
            }
        }
    };
    // V operands of rows ib..ib+3 with rows outside [ra, rb) and k >= r zeroed
    auto mask_v = [&](int64_t ib, const v4f (&vv)[RT], v4f (&vm)[RT]) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const bool kok = 16 * t + lj < r;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) vm[t][s2] = (kok && ib + s2 < rb) ? vv[t][s2] : 0.0f;
        }
    };
    auto dtile_f64 = [&](const v4f (&vv)[RT], const int (&ta)[DMAX], const int (&tb)[DMAX],
                         const bool (&ok)[DMAX]) {
#pragma unroll
        for (int d = 0; d < DMAX; ++d) {
            if (ok[d]) {
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    double va = 0.0, vb = 0.0;
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        if (t == ta[d]) va = (double)vv[t][s2];
                        if (t == tb[d]) vb = (double)vv[t][s2];
                    }
                    dacc[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(va, vb, dacc[d], 0, 0, 0);
                }
            }
        }
    };
    const bf16x8 z8 = {};
    const int64_t mp = J.mpad;
    gmem<const uint16_t> *Vr[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
        Vr[t] = BF ? to_global(J.Vb) + (int64_t)(16 * t + lj) * mp + 8 * lg : nullptr;
    v4f dacc32[DMAX];
#pragma unroll
    for (int d = 0; d < DMAX; ++d) dacc32[d] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    auto dtile_bf16 = [&](const bf16x8 (&b)[RT], const int (&ta)[DMAX], const int (&tb)[DMAX],
                          const bool (&ok)[DMAX]) {
#pragma unroll
        for (int d = 0; d < DMAX; ++d) {
            if (ok[d]) {
                bf16x8 va = z8, vb = z8;
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    if (t == ta[d]) va = b[t];
                    if (t == tb[d]) vb = b[t];
                }
                dacc32[d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, dacc32[d], 0, 0, 0);
            }
        }
    };

    if constexpr (!BF) {
        auto main_loop = [&](auto vec_c) {
            auto load = [&](int64_t i0, v4f (&mv)[SB][WC], v4f (&vv)[SB][RT]) {
#pragma unroll
                for (int u = 0; u < SB; ++u) load1(vec_c, i0 + 16 * u, mv[u], vv[u]);
            };
            auto compute = [&](int64_t i0, const v4f (&mvs)[SB][WC], const v4f (&vvs)[SB][RT]) {
#pragma unroll
                for (int u = 0; u < SB; ++u) {
                    v4f vm[RT];
                    mask_v(i0 + 16 * u + 4 * lg, vvs[u], vm);
                    v4f acc[WC][RT];
#pragma unroll
                    for (int c = 0; c < WC; ++c)
#pragma unroll
                        for (int t = 0; t < RT; ++t) acc[c][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
                        for (int c = 0; c < WC; ++c)
#pragma unroll
                            for (int t = 0; t < RT; ++t)
                                acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                    mvs[u][c][s2], vm[t][s2], acc[c][t], 0, 0, 0);
#pragma unroll
                    for (int c = 0; c < WC; ++c)
#pragma unroll
                        for (int t = 0; t < RT; ++t) two_sum_acc(hi[c][t], lo[c][t], acc[c][t]);
                    dtile_f64(vm, dta, dtb, dok);
                }
            };
            // the next batch is loaded unconditionally (clamped addresses): a
            // conditional prefetch makes the compiler wait for every load at
            // the join; the last one or two batches are loaded for nothing
            v4f m0[SB][WC], m1[SB][WC], v0[SB][RT], v1[SB][RT];
            load(ra, m0, v0);
            for (int64_t i0 = ra; i0 < rb; i0 += 32 * SB) {
                load(i0 + 16 * SB, m1, v1);
                __builtin_amdgcn_sched_barrier(0);
                compute(i0, m0, v0);
                if (i0 + 16 * SB >= rb) break;
                load(i0 + 32 * SB, m0, v0);
                __builtin_amdgcn_sched_barrier(0);
                compute(i0 + 16 * SB, m1, v1);
            }
        };
        if (ra < rb) {
            if (vec) main_loop(std::true_type{});
            else main_loop(std::false_type{});
        }
    } else {
        // rows m..mpad of the copies are zero: K-steps may run past m
        constexpr int KB = 2;
        gmem<const uint16_t> *Mb[WC];
#pragma unroll
        for (int c = 0; c < WC; ++c)
            Mb[c] = to_global(J.Mbc) + (jok[c] ? jb + 16 * c + lj : 0) * mp + 8 * lg;
        v4f acc[WC][RT];
#pragma unroll
        for (int c = 0; c < WC; ++c)
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[c][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        bf16x8 ma0[KB][WC], vb0[KB][RT], ma1[KB][WC], vb1[KB][RT];
        auto loadb = [&](int64_t i0, bf16x8 (&a)[KB][WC], bf16x8 (&b)[KB][RT]) {
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                const int64_t ik = i0 + 32 * u;
                const bool ok = ik < rb;
#pragma unroll
                for (int c = 0; c < WC; ++c)
                    a[u][c] = (ok && jok[c]) ? *(gmem<const bf16x8> *)(Mb[c] + ik) : z8;
#pragma unroll
                for (int t = 0; t < RT; ++t) b[u][t] = ok ? *(gmem<const bf16x8> *)(Vr[t] + ik) : z8;
            }
        };
        auto computeb = [&](const bf16x8 (&a)[KB][WC], const bf16x8 (&b)[KB][RT]) {
#pragma unroll
            for (int u = 0; u < KB; ++u) {
#pragma unroll
                for (int c = 0; c < WC; ++c)
#pragma unroll
                    for (int t = 0; t < RT; ++t)
                        acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][c], b[u][t], acc[c][t],
                                                                            0, 0, 0);
                dtile_bf16(b[u], dta, dtb, dok);
            }
        };
        if (ra < rb) {
            loadb(ra, ma0, vb0);
            for (int64_t i0 = ra; i0 < rb; i0 += 64 * KB) {
                const bool more = i0 + 32 * KB < rb;
                if (more) loadb(i0 + 32 * KB, ma1, vb1);
                computeb(ma0, vb0);
                if (!more) break;
                if (i0 + 64 * KB < rb) loadb(i0 + 64 * KB, ma0, vb0);
                computeb(ma1, vb1);
            }
        }
#pragma unroll
        for (int c = 0; c < WC; ++c)
#pragma unroll
            for (int t = 0; t < RT; ++t) hi[c][t] = acc[c][t];
    }

    // ---- row-group partials -> one sum per output, added in row-group order
    double *redc = smem;                                          // [WC-1][4/WC][WC*RT*4][64]
    double *redd = smem + (size_t)(WC - 1) * 4 * (RT * 4 * 64);   // [WC-1][4/WC][3*4][64]
    const int cslot = (rg - 1) * NCG + cg;
    if (WC > 1 && rg > 0) {
#pragma unroll
        for (int c = 0; c < WC; ++c)
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    redc[((size_t)cslot * WC * RT * 4 + (c * RT + t) * 4 + v) * 64 + lane] =
                        (double)hi[c][t][v] + (double)lo[c][t][v];
    }
    // D partials in the FP64 MFMA layout: dacc[d][v] = D[16 dta + 4v + lg][16 dtb + lj]
    auto d_value = [&](int d, int v) -> double {
        if constexpr (BF) {
            // FP32 MFMA layout D[16 dta + 4 lg + v][16 dtb + lj]: entry (4v + lg)
            // sits in register lg of lane lj + 16 v
            const float x = __shfl(dacc32[d][0], lj + 16 * v, 64);
            const float y = __shfl(dacc32[d][1], lj + 16 * v, 64);
            const float z = __shfl(dacc32[d][2], lj + 16 * v, 64);
            const float w = __shfl(dacc32[d][3], lj + 16 * v, 64);
            return (double)(lg == 0 ? x : lg == 1 ? y : lg == 2 ? z : w);
        } else {
            return dacc[d][v];
        }
    };
    if (WC > 1 && rg > 0) {
        const int dslot = (rg - 1) * NCG + cg;
#pragma unroll
        for (int d = 0; d < DMAX; ++d)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double x = d_value(d, v);
                if (dok[d]) redd[((size_t)dslot * DMAX * 4 + d * 4 + v) * 64 + lane] = x;
            }
    }
    if (WC > 1) __syncthreads();
    if (rg == 0) {
        // hi + lo (+ row groups 1..WC-1) = C[k = 16t + lj][j = jb + 16c + 4*lg + v];
        // FP32 partials in BF16 mode
        const auto out = to_global(J.Cp) + (int64_t)ty * r * n;
        const auto outf = to_global(reinterpret_cast<float *>(J.Cp)) + (int64_t)ty * r * n;
#pragma unroll
        for (int c = 0; c < WC; ++c)
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + lj;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double sum = (double)hi[c][t][v] + (double)lo[c][t][v];
#pragma unroll
                    for (int q = 1; q < WC; ++q)
                        sum += redc[((size_t)((q - 1) * NCG + cg) * WC * RT * 4 + (c * RT + t) * 4 + v) * 64 +
                                    lane];
                    const int64_t jj = jb + 16 * c + 4 * lg + v;
                    if (k < r && jj < n) {
                        if constexpr (BF) outf[jj * r + k] = (float)sum;
                        else out[jj * r + k] = sum;
                    }
                }
            }
        const auto dout = to_global(J.Dp) + (int64_t)ty * RPAD * RPAD;
#pragma unroll
        for (int d = 0; d < DMAX; ++d)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double sum = d_value(d, v);
#pragma unroll
                for (int q = 1; q < WC; ++q)
                    sum += redd[((size_t)((q - 1) * NCG + cg) * DMAX * 4 + d * 4 + v) * 64 + lane];
                if (dok[d]) dout[(16 * dta[d] + 4 * v + lg) * RPAD + 16 * dtb[d] + lj] = sum;
            }
    }

    // ---- V^T V tiles beyond the three fused ones (tiny n only): block-uniform
    // passes over the wave's rows, three tiles per slot each
    for (int g = 1; slot0 + nslots * DMAX * g < NPAIR; ++g) {
        int eta[DMAX], etb[DMAX];
        bool eok[DMAX];
#pragma unroll
        for (int d = 0; d < DMAX; ++d) {
            const int idx = slot + nslots * (DMAX * g + d);
            eok[d] = idx < NPAIR;
            tile_pair(idx, eta[d], etb[d]);
            dacc[d] = v4d{0.0, 0.0, 0.0, 0.0};
            dacc32[d] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        }
        if constexpr (!BF) {
            for (int64_t i0 = ra; i0 < rb; i0 += 16) {
                v4f mv[WC], vv[RT], vm[RT];
                if (vec) load1(std::true_type{}, i0, mv, vv);
                else load1(std::false_type{}, i0, mv, vv);
                mask_v(i0 + 4 * lg, vv, vm);
                dtile_f64(vm, eta, etb, eok);
            }
        } else {
            for (int64_t ik = ra; ik < rb; ik += 32) {
                bf16x8 b[RT];
#pragma unroll
                for (int t = 0; t < RT; ++t) b[t] = *(gmem<const bf16x8> *)(Vr[t] + ik);
                dtile_bf16(b, eta, etb, eok);
            }
        }
        if (WC > 1) __syncthreads();   // previous readers of redd are done
        if (WC > 1 && rg > 0) {
            const int dslot = (rg - 1) * NCG + cg;
#pragma unroll
            for (int d = 0; d < DMAX; ++d)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double x = d_value(d, v);
                    if (eok[d]) redd[((size_t)dslot * DMAX * 4 + d * 4 + v) * 64 + lane] = x;
                }
        }
        if (WC > 1) __syncthreads();
        if (rg == 0) {
            const auto dout = to_global(J.Dp) + (int64_t)ty * RPAD * RPAD;
#pragma unroll
            for (int d = 0; d < DMAX; ++d)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double sum = d_value(d, v);
#pragma unroll
                    for (int q = 1; q < WC; ++q)
                        sum += redd[((size_t)((q - 1) * NCG + cg) * DMAX * 4 + d * 4 + v) * 64 + lane];
                    if (eok[d]) dout[(16 * eta[d] + 4 * v + lg) * RPAD + 16 * etb[d] + lj] = sum;
                }
        }
    }
}

template <int RT, int WC, int SB, bool BF>
__global__ __launch_bounds__(256) void k_cpass(const Job *__restrict__ jobs,
                                               const int2 *__restrict__ bmap) {
    extern __shared__ double smem[];
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
    cpass_tile<RT, WC, SB, BF>(J, tx, ty, J.nCx, smem);
}

// ---------------------------------------------------------------------------
// Upper-triangle 16x16 tile number `idx` (numbered row by row) of an RT x RT
// grid of tiles: (ta, tb) with ta <= tb.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gram_tile_pair(int idx, int rt, int &ta, int &tb) {
    int a = 0;
    while (idx >= rt - a) {
        idx -= rt - a;
        ++a;
    }
    ta = a;
    tb = a + idx;
}

// ---------------------------------------------------------------------------
// D = V^T V from the C-pass partials (upper-triangle 16x16 tiles, row stride
// rpad): one block per upper tile; D[a][b] = sum_p parts[p][a'][b'] with
// (a', b') = (min, max)(a, b), added in index order, written to both halves.
// With J.Cr set, the blocks past the upper tiles sum V^T M over the chunks,
// 256 entries each, in index order from 0 (the W update's own order, so its
// C is the same either way).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(const Job *__restrict__ jobs,
                                                const int2 *__restrict__ bmap) {
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (J.st->stop) return;
    const int r = J.r, rpad = J.rpad;
    const int ntiles = (rpad / 16) * (rpad / 16 + 1) / 2;
    if (jt.y >= ntiles) {
        const int64_t rn = (int64_t)r * J.n;
        const int64_t e = (int64_t)(jt.y - ntiles) * 256 + threadIdx.x;
        if (!J.Cr || e >= rn) return;
        J.Cr[e] = J.prec ? sum_strided<64>(reinterpret_cast<const float *>(J.Cp) + e, rn, J.chunks)
                         : sum_strided<64>(J.Cp + e, rn, J.chunks);
        return;
    }
    int ta, tb;
    gram_tile_pair(jt.y, rpad / 16, ta, tb);
    const int ra = 16 * ta + (threadIdx.x >> 4), rb = 16 * tb + (threadIdx.x & 15);
    const int ua = ra < rb ? ra : rb, ub = ra < rb ? rb : ra;
    if (ra < r && rb < r) {
        const double s = sum_strided<64>(J.Dp + ua * rpad + ub, (int64_t)rpad * rpad, J.chunks);
        J.Dd[ra * r + rb] = s;
        if (ta != tb) J.Dd[rb * r + ra] = s;
    }
}

// ---------------------------------------------------------------------------
// Residual of the iteration from the W-update partials (one block, index
// order): e^2 = ||M_d||^2 + sum of the partials; logs rel_err and sets the
// stop flag.  rs: this thread's share, partials tid, tid + NT, ...
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void log_residual(const Job &J, double rs, double *red) {
    rs = block_sum_f64<NT>(rs, red);
    if (threadIdx.x == 0) {
        DevState *st = J.st;
        const double nm = *J.normM2;
        const double e2 = nm + rs;
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
            if (J.hstop) *J.hstop = 1;
        } else if (J.depth == 0 && J.prec == 0 && J.tol > 0.0 && rel <= J.tol) {
            st->stopped = 1;
            st->stop = 1;
            if (J.hstop) *J.hstop = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// B = W W^T in FP64 from the FP32 W (r x n, row-major): block = (upper tile
// (ta, tb), column segment); its 8 waves split the segment into contiguous
// ranges and run FP64 MFMAs (products of FP32 values are exact), lane (li, lk)
// supplying columns j0 + 4 lk + s of rows 16 ta + li and 16 tb + li to MFMA s;
// the loads of 8 16-column steps go out together, and steps wholly past the
// range are skipped (their operands would be zero).  The wave partials are
// added in LDS in wave order.  One segment (J.gseg = 1): the block writes its
// tile of B, and with with_resid block 0 also logs the iteration's residual.
// Several: the block stores its partial tile and k_gram_sum adds them.
// ---------------------------------------------------------------------------
constexpr int kGramWWaves = 8;

__global__ __launch_bounds__(64 * kGramWWaves) void k_gram_w(const Job *__restrict__ jobs,
                                                             const int2 *__restrict__ bmap,
                                                             int with_resid) {
    constexpr int NW = kGramWWaves, NT = 64 * NW, U = 8;
    __shared__ double part[NW - 1][256];
    __shared__ double red[NW];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (J.st->stop) return;
    const int r = J.r, rpad = J.rpad;
    const int64_t n = J.n;
    const int gseg = J.gseg;
    const int tile = jt.y / gseg, seg = jt.y % gseg;
    int ta, tb;
    gram_tile_pair(tile, rpad / 16, ta, tb);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int ka = 16 * ta + li, kb = 16 * tb + li;
    const auto W = to_global(J.W);
    const gmem<const float> *wa = W + (int64_t)(ka < r ? ka : 0) * n;
    const gmem<const float> *wb = W + (int64_t)(kb < r ? kb : 0) * n;
    const bool va = ka < r, vb = kb < r;
    const bool vec = (n & 3) == 0 && ((uintptr_t)J.W & 15) == 0;
    // residual (block 0, one segment): the W-update partials of the previous kernel
    const bool resid = with_resid && gseg == 1 && jt.y == 0;
    double rs = 0.0;
    if (resid)
        for (int i = tid; i < J.nF; i += NT) rs += to_global(J.rparts)[i];
    // the segment's columns, then columns per wave, multiples of 16
    const int64_t slen = (n + 16 * gseg - 1) / (16 * gseg) * 16;
    const int64_t s0 = seg * slen, s1 = (s0 + slen < n) ? s0 + slen : n;
    const int64_t per = (slen + 16 * NW - 1) / (16 * NW) * 16;
    const int64_t c0 = s0 + wave * per, c1 = (c0 + per < s1) ? c0 + per : s1;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int64_t jg = c0; jg < c1; jg += 16 * U) {
        v4f xa[U], xb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t jb = jg + 16 * u + 4 * lk;
            if (vec && jb + 3 < c1) {
                xa[u] = va ? *(gmem<const v4f> *)(wa + jb) : v4f{0.0f, 0.0f, 0.0f, 0.0f};
                xb[u] = vb ? *(gmem<const v4f> *)(wb + jb) : v4f{0.0f, 0.0f, 0.0f, 0.0f};
            } else {
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    const bool ok = jb + s2 < c1;
                    xa[u][s2] = (va && ok) ? wa[jb + s2] : 0.0f;
                    xb[u][s2] = (vb && ok) ? wb[jb + s2] : 0.0f;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (jg + 16 * u >= c1) break;   // uniform: the rest of the batch is zero
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)xa[u][s2], (double)xb[u][s2], acc,
                                                           0, 0, 0);
        }
    }
    // acc[v] = B[16 ta + 4 v + lk][16 tb + li]
    if (wave > 0)
#pragma unroll
        for (int v = 0; v < 4; ++v) part[wave - 1][v * 64 + lane] = acc[v];
    __syncthreads();
    if (wave == 0) {
        double *pt = J.bparts + ((int64_t)tile * gseg + seg) * 256;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double b = acc[v];
#pragma unroll
            for (int w2 = 0; w2 < NW - 1; ++w2) b += part[w2][v * 64 + lane];
            if (gseg > 1) {
                pt[v * 64 + lane] = b;
                continue;
            }
            const int a1 = 16 * ta + 4 * v + lk, b1 = 16 * tb + li;
            // a diagonal tile keeps exact symmetry: its lower half copies the upper
            if (a1 < r && b1 < r && (ta != tb || a1 <= b1)) {
                J.Bd[a1 * r + b1] = b;
                J.Bd[b1 * r + a1] = b;
            }
        }
    }
    if (resid) log_residual<NT>(J, rs, red);
}

// B from the segment partials of k_gram_w (jobs with J.gseg > 1; others
// return): block = upper tile, thread = tile entry, segments added in order;
// with_resid: block 0 also logs the iteration's residual.
__global__ __launch_bounds__(256) void k_gram_sum(const Job *__restrict__ jobs,
                                                  const int2 *__restrict__ bmap, int with_resid) {
    __shared__ double red[4];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (J.gseg <= 1 || J.st->stop) return;
    const int r = J.r, gseg = J.gseg, tid = threadIdx.x;
    int ta, tb;
    gram_tile_pair(jt.y, J.rpad / 16, ta, tb);
    const bool resid = with_resid && jt.y == 0;
    double rs = 0.0;
    if (resid)
        for (int i = tid; i < J.nF; i += 256) rs += to_global(J.rparts)[i];
    const auto p0 = to_global(J.bparts) + (int64_t)jt.y * gseg * 256 + tid;
    double t[kGramSegMax];
#pragma unroll
    for (int q = 0; q < kGramSegMax; ++q) t[q] = q < gseg ? p0[q * 256] : 0.0;
    double b = 0.0;
#pragma unroll
    for (int q = 0; q < kGramSegMax; ++q)
        if (q < gseg) b += t[q];
    // entry tid = v * 64 + lane of the tile layout: B[16 ta + 4 v + lk][16 tb + li]
    const int v = tid >> 6, lane = tid & 63;
    const int a1 = 16 * ta + 4 * v + (lane >> 4), b1 = 16 * tb + (lane & 15);
    if (a1 < r && b1 < r && (ta != tb || a1 <= b1)) {
        J.Bd[a1 * r + b1] = b;
        J.Bd[b1 * r + a1] = b;
    }
    if (resid) log_residual<256>(J, rs, red);
}

// ---------------------------------------------------------------------------
// W-update tile: CF (4 or 16) columns of W.  The threads reduce the entries
// of those columns of C from the C-pass partials (chunk-major, n x r per
// chunk: the tile's entries are contiguous; fixed order, batched loads), or
// read them from J.Cr where the D-reduction launch has summed them; then
// 16 lanes per column update it (HALS / MU against D) and write W, its
// transposed copy Wt (and the BF16 copy).  Also emits, per 4 columns (one
// wave), the residual partial sum_j (w_j^T D w_j - 2 c_j^T w_j): the first
// term is those columns' share of <D, B> (B = sum_j w_j w_j^T).  Every column
// and every 4-column partial is computed the same way for both CF.
// ---------------------------------------------------------------------------
template <int RT, int MODE, int CF>
__device__ __forceinline__ void cfinal_tile(const Job &J, int tile, double *smem) {
    constexpr int RPAD = RT * 16, GS = RPAD + 1, CS = RPAD + 1;
    constexpr bool UPD = MODE == MODE_HALS || MODE == MODE_MU;
    constexpr bool INIT = MODE == MODE_INIT;     // no C, no update: Wt (and Wb) only
    constexpr int PER = (CF * RPAD + 255) / 256;   // C entries per thread
    static_assert(CF == 4 || CF == 16, "W-update tile width");
    double *Gs = smem;
    double *Gi = Gs + (UPD ? RPAD * GS : 0);
    double *Cs = Gi + (UPD ? RPAD : 0);
    double *red = Cs + (INIT ? 0 : CF * CS);
    const int tid = threadIdx.x;
    const int64_t n = J.n;
    const int r = J.r;
    const int64_t j0 = (int64_t)tile * CF;
    // factor columns of the update: 16 lanes per column, column j0 + tid/16
    // (all waves for CF = 16, wave 0 for CF = 4)
    const bool colt = tid < 16 * CF;
    // The column entries of W and the Gram D are loaded first (clamped
    // addresses) and masked / stored only once the C sums below are done, so
    // all of these loads are in flight together.
    double xw[RT];
    float xwf[RT];
    GramRegs<RPAD> gregs;
    if constexpr (MODE != MODE_STORE) {
        const int64_t j = j0 + (tid >> 4);
        const int64_t jc = j < n ? j : n - 1;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + (tid & 15);
            xwf[t] = to_global(J.W)[(int64_t)(k < r ? k : 0) * n + jc];
        }
    }
    if constexpr (UPD) gram_fetch<RPAD>(J.Dd, r, gregs);
    if constexpr (!INIT) {
        constexpr int B = CF == 4 ? 64 : 16;
        const int64_t str = (int64_t)r * n;
        double cs[PER];
        int64_t off[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i, jj = e / RPAD, k = e % RPAD;
            const int64_t j = j0 + jj;
            off[i] = (jj < CF && k < r && j < n) ? j * r + k : -1;
        }
        bool cok[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) cok[i] = off[i] >= 0;
        if (J.Cr) {   // already summed over the chunks
#pragma unroll
            for (int i = 0; i < PER; ++i) cs[i] = to_global(J.Cr)[cok[i] ? off[i] : 0];
#pragma unroll
            for (int i = 0; i < PER; ++i) cs[i] = cok[i] ? cs[i] : 0.0;
        } else if (J.prec) {
            const float *src[PER];
#pragma unroll
            for (int i = 0; i < PER; ++i)
                src[i] = reinterpret_cast<const float *>(J.Cp) + (cok[i] ? off[i] : 0);
            sum_strided_n<PER, B>(src, cok, str, J.chunks, cs);
        } else {
            const double *src[PER];
#pragma unroll
            for (int i = 0; i < PER; ++i) src[i] = J.Cp + (cok[i] ? off[i] : 0);
            sum_strided_n<PER, B>(src, cok, str, J.chunks, cs);
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i, jj = e / RPAD, k = e % RPAD;
            if (jj < CF) Cs[jj * CS + k] = cs[i];
        }
    }
    if constexpr (UPD) gram_put<RPAD>(gregs, r, Gs, GS, Gi);
    if constexpr (MODE != MODE_STORE) {
        const int64_t j = j0 + (tid >> 4);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int k = 16 * t + (tid & 15);
            xw[t] = (colt && j < n && k < r) ? (double)xwf[t] : 0.0;
        }
    }
    if constexpr (!INIT) __syncthreads();
    if constexpr (MODE == MODE_STORE) {
        for (int e = tid; e < CF * r; e += 256) {
            const int jj = e % CF, k = e / CF;
            const int64_t j = j0 + jj;
            if (j >= n) continue;
            if (J.Cd) to_global(J.Cd)[(int64_t)k * n + j] = Cs[jj * CS + k];
            else to_global(J.C)[(int64_t)k * n + j] = (float)Cs[jj * CS + k];
        }
    } else {
        double part = 0.0;
        if (colt) {
            const int jj = tid >> 4, p = tid & 15;
            const int64_t j = j0 + jj;
            const bool ok = j < n;
            if constexpr (UPD) {
                double cv[RT];
#pragma unroll
                for (int t = 0; t < RT; ++t) cv[t] = Cs[jj * CS + 16 * t + p];
                row_update<RT, MODE>(xw, Gs, GS, Gi, cv, r, p);
            }
            double xs[RT];
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int k = 16 * t + p;
                const float xf = (ok && k < r) ? (float)xw[t] : 0.0f;
                xs[t] = (double)xf;
                if (ok) {
                    to_global(J.Wt)[j * RPAD + wt_pos(k, RT)] = xf;
                    if (J.Wb) to_global(J.Wb)[(int64_t)k * J.npad + j] = bf16_rne(xf);   // BF16 mode
                    if (UPD && k < r) to_global(J.W)[(int64_t)k * n + j] = xf;
                }
            }
            if constexpr (UPD) {
                double dx[RT];
                gram_matvec<RT>(xs, Gs, GS, r, p, dx);
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const int k = 16 * t + p;
                    if (k < r) part += xs[t] * (dx[t] - 2.0 * Cs[jj * CS + k]);
                }
            }
        }
        if constexpr (UPD) {
            // one partial per 4 columns: the 64 lanes of one wave
            if (colt) {
                const double tot = wave_sum_f64(part);
                const int64_t quad = j0 / 4 + (tid >> 6);
                if ((tid & 63) == 0 && quad < J.nF) to_global(J.rparts)[quad] = tot;
            }
        }
    }
}

template <int RT, int MODE, int CF>
__global__ __launch_bounds__(256) void k_cfinal(const Job *__restrict__ jobs,
                                                const int2 *__restrict__ bmap) {
    extern __shared__ double smem[];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (J.st->stop) return;
    cfinal_tile<RT, MODE, CF>(J, jt.y, smem);
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
                                                  DevState *st, int32_t *hstop, double tol) {
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
            if (hstop) *hstop = 1;
        } else if (depth == 0 && tol > 0.0 && rel <= tol) {
            st->stopped = 1;
            st->stop = 1;
            if (hstop) *hstop = 1;
        }
    }
}

}  // namespace


// ---- host side -------------------------------------------------------------

size_t apass_lds_bytes(int rpad, int tm, int mode) {
    const bool upd = mode != MODE_STORE;
    const int rw = tm == 16 ? 1 : 2;
    return sizeof(double) * ((upd ? rpad * (rpad + 1) + rpad : 0) + 4 * 16 * rw * (rpad + 1));
}

size_t cfinal_lds_bytes(int rpad, int mode, int cf) {
    const bool upd = mode == MODE_HALS || mode == MODE_MU;
    const size_t g = upd ? (size_t)rpad * (rpad + 1) + rpad : 0;      // Gram and 1/G_kk
    const size_t c = mode == MODE_INIT ? 0 : (size_t)cf * (rpad + 1);  // C columns
    return sizeof(double) * (g + c + 4);
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

// C-pass configurations: WC column tiles (and row groups) per wave, from the
// plan (1: one wave per column tile over the whole chunk, for throughput; 2
// or 4: shorter per-wave chains, for latency), and SB 16-row steps per FP32
// load batch by rank class and WC (two up to r = 32, and up to r = 48 with at
// most two column tiles per wave: two steps of loads in flight per wave; one
// where the wider operand tiles would not fit the registers).
template <int RT, int WC>
struct CpassCfg {
    static constexpr int SB = RT <= 2 || (RT == 3 && WC <= 2) ? 2 : 1;
};

template <int RT, int WC>
static void cpass_launch(bool bf, const Job *jobs, const int2 *bmap, int blocks, hipStream_t s) {
    constexpr int SB = CpassCfg<RT, WC>::SB;
    const size_t lds = sizeof(double) * cpass_lds_doubles<RT, WC>();
    if (bf) k_cpass<RT, WC, SB, true><<<blocks, 256, lds, s>>>(jobs, bmap);
    else k_cpass<RT, WC, SB, false><<<blocks, 256, lds, s>>>(jobs, bmap);
}

template <int RT>
static void cpass_launch_wc(int wc, bool bf, const Job *jobs, const int2 *bmap, int blocks,
                            hipStream_t s) {
    if (wc == 4) cpass_launch<RT, 4>(bf, jobs, bmap, blocks, s);
    else if (wc == 2) cpass_launch<RT, 2>(bf, jobs, bmap, blocks, s);
    else cpass_launch<RT, 1>(bf, jobs, bmap, blocks, s);
}

hipError_t launch_cpass_jobs(int rpad, int wc, const Job *jobs, const int2 *bmap, int blocks,
                             hipStream_t s, bool bf) {
    if (blocks <= 0) return hipSuccess;
    if (wc != 1 && wc != 2 && wc != 4) return hipErrorInvalidValue;
    switch (rpad) {
        case 16: cpass_launch_wc<1>(wc, bf, jobs, bmap, blocks, s); break;
        case 32: cpass_launch_wc<2>(wc, bf, jobs, bmap, blocks, s); break;
        case 48: cpass_launch_wc<3>(wc, bf, jobs, bmap, blocks, s); break;
        case 64: cpass_launch_wc<4>(wc, bf, jobs, bmap, blocks, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_jobs(const Job *jobs, const int2 *bmap, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    k_reduce<<<blocks, 256, 0, s>>>(jobs, bmap);
    return hipGetLastError();
}

hipError_t launch_gram_w_jobs(int with_resid, const Job *jobs, const int2 *bmap, int blocks,
                              hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    k_gram_w<<<blocks, 64 * kGramWWaves, 0, s>>>(jobs, bmap, with_resid);
    return hipGetLastError();
}

hipError_t launch_gram_sum_jobs(int with_resid, const Job *jobs, const int2 *bmap, int blocks,
                                hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    k_gram_sum<<<blocks, 256, 0, s>>>(jobs, bmap, with_resid);
    return hipGetLastError();
}

template <int RT, int CF>
static void cfinal_launch(int mode, const Job *jobs, const int2 *bmap, int blocks,
                          size_t lds, hipStream_t s) {
    if (mode == MODE_HALS) k_cfinal<RT, MODE_HALS, CF><<<blocks, 256, lds, s>>>(jobs, bmap);
    else if (mode == MODE_MU) k_cfinal<RT, MODE_MU, CF><<<blocks, 256, lds, s>>>(jobs, bmap);
    else if (mode == MODE_INIT) k_cfinal<RT, MODE_INIT, CF><<<blocks, 256, lds, s>>>(jobs, bmap);
    else k_cfinal<RT, MODE_STORE, CF><<<blocks, 256, lds, s>>>(jobs, bmap);
}

template <int RT>
static void cfinal_launch_cf(int mode, int cf, const Job *jobs, const int2 *bmap, int blocks,
                             size_t lds, hipStream_t s) {
    if (cf == 16) cfinal_launch<RT, 16>(mode, jobs, bmap, blocks, lds, s);
    else cfinal_launch<RT, 4>(mode, jobs, bmap, blocks, lds, s);
}

hipError_t launch_cfinal_jobs(int mode, int rpad, int cf, const Job *jobs, const int2 *bmap,
                              int blocks, size_t lds, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (cf != 4 && cf != 16) return hipErrorInvalidValue;
    switch (rpad) {
        case 16: cfinal_launch_cf<1>(mode, cf, jobs, bmap, blocks, lds, s); break;
        case 32: cfinal_launch_cf<2>(mode, cf, jobs, bmap, blocks, lds, s); break;
        case 48: cfinal_launch_cf<3>(mode, cf, jobs, bmap, blocks, lds, s); break;
        case 64: cfinal_launch_cf<4>(mode, cf, jobs, bmap, blocks, lds, s); break;
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
                           int32_t *log_depth, int log_cap, DevState *st, int32_t *hstop,
                           double tol, hipStream_t s) {
    k_residual<<<1, 256, 0, s>>>(rparts, nparts, Dd, Bd, r, normM2, depth, log_rel, log_depth,
                                 log_cap, st, hstop, tol);
    return hipGetLastError();
}

int cpass_final_blocks(int64_t n) { return (int)((n + 3) / 4); }

int cfinal_tile_blocks(int64_t n, int cf) { return (int)((n + cf - 1) / cf); }

int apass_grid_single(int nA) { return 8 * ((nA + 7) / 8); }

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
    set((const void *)k_cfinal<RT, MODE, 4>);
    set((const void *)k_cfinal<RT, MODE, 16>);
    constexpr int S1 = CpassCfg<RT, 1>::SB, S2 = CpassCfg<RT, 2>::SB, S4 = CpassCfg<RT, 4>::SB;
    for (const void *f : {(const void *)k_cpass<RT, 1, S1, false>, (const void *)k_cpass<RT, 1, S1, true>,
                          (const void *)k_cpass<RT, 2, S2, false>, (const void *)k_cpass<RT, 2, S2, true>,
                          (const void *)k_cpass<RT, 4, S4, false>, (const void *)k_cpass<RT, 4, S4, true>})
        set(f);
}

template <int RT>
static void lds_attr_modes(hipError_t &e) {
    lds_attr<RT, MODE_HALS>(e);
    lds_attr<RT, MODE_MU>(e);
    lds_attr<RT, MODE_STORE>(e);
    for (const void *f : {(const void *)k_cfinal<RT, MODE_INIT, 4>,
                          (const void *)k_cfinal<RT, MODE_INIT, 16>}) {
        hipError_t x = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
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
        const hipError_t x = enable_stream_lds();
        return e == hipSuccess ? x : e;
    }();
    return done;
}

}  // namespace nmf
