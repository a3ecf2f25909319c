// Streaming passes for large levels: the A-pass and C-pass of one iteration
// (Alg. 2 / Alg. 3) as long LDS-pipelined loops over the whole of n (A-pass)
// or a long row chunk (C-pass), in BF16 (k_*_stream, m >= kStreamMinRows) or
// FP32 (k_*_s32, m >= kFStreamMinRows).  The Gram, reduction and W-update kernels are those of
// the regular path.

#include "sweep_device.h"

namespace nmf {

namespace {

// ---------------------------------------------------------------------------
// Operand staging through LDS by DMA (global_load_lds_dwordx4): lane l's 16
// bytes at src land at dst + 16 l, dst uniform over the wave.  The copies are
// counted by the wave's vector-memory counter like loads, but the compiler
// places no wait for them: a reader first waits until at most N of the wave's
// vector-memory operations are still in flight, where N counts the copies the
// wave issued after the ones it needs.  Copies complete in issue order, so
// every wait also covers the wave's own earlier loads.
// ---------------------------------------------------------------------------
template <class T>
using lmem = __attribute__((address_space(3))) T;

__device__ __forceinline__ void lds_dma16(gmem<const uint16_t> *src, char *dst) {
    __builtin_amdgcn_global_load_lds((gmem<const void> *)src, (lmem<void> *)dst, 16, 0, 0);
}

// Wait until at most N vector-memory operations of this wave are in flight,
// then meet the other waves of the block (no other counter is waited for).
template <int N>
__device__ __forceinline__ void vm_wait_barrier() {
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

__device__ __forceinline__ bf16x8 lds_bf16x8(const char *p) { return *(const lmem<bf16x8> *)p; }

// Streaming BF16 passes: kStreamStages stages of one 32-wide K-step each, so
// kStreamStages - 1 K-steps are in flight while one is multiplied.  A stage
// holds 4 x 1 KB of the big operand per wave (its four 16-row or 16-column
// panels) and four 1 KB slots of the small one, one copied by each wave.
constexpr int kStreamStages = 4;
constexpr int kStreamStage = 20 * 1024;
constexpr int kStageOps = 5;   // copies one wave issues per stage

// The r x r FP64 Gram Gd (row-major, stride r) into LDS as FP32, zero-padded
// to RPAD x RPAD (stride RPAD), and gi[k] = 1/G_kk (0 when G_kk = 0 or
// k >= r).  Every thread issues all of its loads before its first store, so
// the block waits for one memory latency.
template <int RPAD>
__device__ __forceinline__ void load_gram_f32(const double *__restrict__ Gd, int r, float *Gs,
                                              float *gi) {
    constexpr int PER = (RPAD * RPAD + 255) / 256;
    const auto G = to_global(Gd);
    const int tid = threadIdx.x;
    double v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = tid + 256 * i, a = e / RPAD, b = e % RPAD;
        v[i] = (e < RPAD * RPAD && a < r && b < r) ? G[a * r + b] : 0.0;
    }
    const double d = (tid < r) ? G[tid * r + tid] : 0.0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = tid + 256 * i;
        if (e < RPAD * RPAD) Gs[e] = (float)v[i];
    }
    if (tid < RPAD) gi[tid] = d > 0.0 ? (float)(1.0 / d) : 0.0f;
}

// One factor row held by one lane (x, with arow the lane's row of the
// product in LDS), updated against the RPAD x RPAD Gram G (row-major,
// zero-padded, in LDS; every lane reads the same entry, a broadcast) and
// gi[k] = 1/G_kk (0 when G_kk = 0 or k >= r), in T: FP32 in the BF16 mode,
// FP64 in the FP32 mode.
// HALS (Alg. 3): for k = 1..r in order, x_k <- max(0, (a_k - sum_{l != k}
// x_l G_lk) / G_kk) with the entries l < k already updated; G_kk = 0 keeps x_k.
// MU (Alg. 2): x_k <- x_k a_k / (sum_l x_l G_lk) from the old x; a zero
// denominator keeps x_k.
// Dot products use four interleaved partial sums (entries l = 0, 1, 2, 3 mod
// 4), added as (s0 + s1) + (s2 + s3).  The code is straight-line over all
// RPAD entries and steps: padded entries are zero (x_l = 0, zero Gram rows and
// 1/G_kk = 0), so they change nothing, and a branch per group or step would
// make the compiler wait for every LDS load in flight at each branch.  The
// Gram row of step k is read only once step k - AHEAD is done
// (ordered_after), so its loads overlap the previous steps without all of
// them being hoisted into registers.
template <int RPAD, int MODE, class T>
__device__ __forceinline__ void stream_row_update(T (&x)[RPAD], const T *arow, const T *G,
                                                  const T *gi, int r) {
    typedef double v2d __attribute__((ext_vector_type(2)));
    constexpr int AHEAD = std::is_same<T, float>::value ? 2 : 1;
    auto dot = [&](int k_row, auto skip_c, T dep) -> T {
        constexpr int skip = decltype(skip_c)::value;
        T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
        const T *g = G + ordered_after(k_row * RPAD, dep);
        static_for<RPAD / 4>([&](auto lg_c) {
            constexpr int l = 4 * decltype(lg_c)::value;
            T g0, g1, g2, g3;
            if constexpr (std::is_same<T, float>::value) {
                const v4f gv = *(const lmem<v4f> *)(g + l);
                g0 = gv[0]; g1 = gv[1]; g2 = gv[2]; g3 = gv[3];
            } else {
                const v2d ga = *(const lmem<v2d> *)(g + l);
                const v2d gb = *(const lmem<v2d> *)(g + l + 2);
                g0 = ga[0]; g1 = ga[1]; g2 = gb[0]; g3 = gb[1];
            }
            s0 = (l + 0 == skip) ? s0 : fma_t(x[l + 0], g0, s0);
            s1 = (l + 1 == skip) ? s1 : fma_t(x[l + 1], g1, s1);
            s2 = (l + 2 == skip) ? s2 : fma_t(x[l + 2], g2, s2);
            s3 = (l + 3 == skip) ? s3 : fma_t(x[l + 3], g3, s3);
        });
        return (s0 + s1) + (s2 + s3);
    };
    if constexpr (MODE == MODE_HALS) {
        static_for<RPAD>([&](auto k_c) {
            constexpr int k = decltype(k_c)::value;
            const T num = arow[k] - dot(k, k_c, x[k >= AHEAD ? k - AHEAD : 0]);
            const T gk = gi[k];
            const T c = num * gk;
            x[k] = gk > T(0) ? (c > T(0) ? c : T(0)) : x[k];
        });
    } else {
        T den[RPAD] = {};
        static_for<RPAD>([&](auto k_c) {
            constexpr int k = decltype(k_c)::value;
            den[k] = dot(k, std::integral_constant<int, -1>{}, den[k >= AHEAD ? k - AHEAD : 0]);
        });
#pragma unroll
        for (int k = 0; k < RPAD; ++k)
            if (k < r && den[k] > T(0)) x[k] = x[k] * arow[k] / den[k];
    }
}

// ---------------------------------------------------------------------------
// Streaming passes for large levels in BF16 mode (job.stream = 1).
//
// A-pass: a block of 4 waves owns kStreamARows = 256 rows; each wave owns 64
// rows (four 16-row panels of the K-packed copy of M) over all of n, so every
// W operand feeds four MFMAs and no partial tiles are combined.  M panels and
// W tiles reach LDS by DMA, kStreamStages K-steps deep, one barrier per
// K-step.  Each lane's V row is loaded before the M stream starts (its latency
// hides behind it).  The wave's A rows then go to a wave-private LDS region
// (FP32, aliasing the stages) and lane q updates row q of the wave: V read and
// written with one coalesced access per entry, the r x r arithmetic in FP32
// against the Gram in LDS.  (128-row blocks, two per CU, measured the same:
// the blocks of a CU run in step, so their updates overlap each other, not the
// M stream.)
// ---------------------------------------------------------------------------
constexpr int kStreamAPanels = kStreamARows / 64;                 // 16-row panels per wave
constexpr int kStreamAStage = (4 * kStreamAPanels + 4) * 1024;       // M panels, then 4 W slots
constexpr int kStreamAOps = kStreamAPanels + 1;                      // copies per wave per stage

template <int RT, int MODE>
__device__ __forceinline__ void apass_stream_tile(const Job &J, int tile, double *smem) {
    constexpr int RPAD = RT * 16, AS = RPAD + 1, NST = kStreamStages, PW = kStreamAPanels;
    constexpr int STAGE = kStreamAStage, WSLOT = 4 * PW * 1024, WR = 16 * PW;
    char *pipe = reinterpret_cast<char *>(smem);
    float *Gs = reinterpret_cast<float *>(pipe + NST * STAGE);   // RPAD x RPAD
    float *Gi = Gs + RPAD * RPAD;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m = J.m;
    const int r = J.r;
    const int64_t row0 = (int64_t)tile * kStreamARows + wave * WR;
    // npad is a multiple of 128, so ksteps >= 4 >= NST - 1; panels past m
    // read the last panel (their rows are not written back)
    const int ksteps = (int)(J.npad / 32);
    const int64_t G = J.npad / 8;
    const int64_t lastp = (m - 1) / 16;
    gmem<const uint16_t> *Mp[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) {
        const int64_t pr = row0 / 16 + q;
        Mp[q] = to_global(J.Mbp) + ((pr < lastp ? pr : lastp) * G * 16 + li) * 8 + lk * 128;
    }
    // wave w copies W tile w % RT into W slot w
    gmem<const uint16_t> *Wr =
        to_global(J.Wb) + (int64_t)(16 * (wave % RT) + li) * J.npad + 8 * lk;
    // the V row of the update (lane q: row row0 + q) is loaded before the
    // M stream starts, so its latency hides behind it; these loads are older
    // than every copy, so the copy waits below also cover them
    const int64_t row = row0 + lane;
    const bool live = lane < WR && row < m;
    const auto V = to_global(J.V);
    float x[RPAD];
#pragma unroll
    for (int k = 0; k < RPAD; ++k) x[k] = (live && k < r) ? V[row + (int64_t)k * m] : 0.0f;
    auto issue = [&](int kk) {
        char *st = pipe + (kk % NST) * STAGE;
#pragma unroll
        for (int q = 0; q < PW; ++q)
            lds_dma16(Mp[q] + (int64_t)kk * 512, st + (wave * PW + q) * 1024);
        lds_dma16(Wr + 32 * kk, st + WSLOT + wave * 1024);
    };
    v4f acc[PW][RT];
#pragma unroll
    for (int q = 0; q < PW; ++q)
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[q][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    auto mma = [&](int kk) {
        const char *st = pipe + (kk % NST) * STAGE;
        bf16x8 a[PW], b[RT];
#pragma unroll
        for (int q = 0; q < PW; ++q) a[q] = lds_bf16x8(st + (wave * PW + q) * 1024 + lane * 16);
#pragma unroll
        for (int t = 0; t < RT; ++t) b[t] = lds_bf16x8(st + WSLOT + t * 1024 + lane * 16);
#pragma unroll
        for (int q = 0; q < PW; ++q)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[q], b[t], acc[q][t], 0, 0, 0);
    };
#pragma unroll
    for (int kk = 0; kk < NST - 1; ++kk) issue(kk);
    int kk = 0;
    for (; kk < ksteps - (NST - 1); ++kk) {
        vm_wait_barrier<kStreamAOps * (NST - 2)>();   // stage kk landed, stage kk - 1 read
        issue(kk + NST - 1);
        mma(kk);
    }
    static_for<NST - 1>([&](auto j_c) {               // drain: nothing left to issue
        constexpr int j = decltype(j_c)::value;
        vm_wait_barrier<kStreamAOps * (NST - 2 - j)>();
        mma(kk + j);
    });
    __syncthreads();   // every wave done with the stages
    load_gram_f32<RPAD>(J.Bd, r, Gs, Gi);
    float *Aw = reinterpret_cast<float *>(pipe) + wave * WR * AS;
#pragma unroll
    for (int q = 0; q < PW; ++q)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) Aw[(16 * q + 4 * lk + v) * AS + 16 * t + li] = acc[q][t][v];
    __syncthreads();   // Gram and A rows in LDS
    if (lane >= WR) return;
    stream_row_update<RPAD, MODE, float>(x, Aw + lane * AS, Gs, Gi, r);
    if (live) {
        const auto Vb = to_global(J.Vb);
#pragma unroll
        for (int k = 0; k < RPAD; ++k) {
            if (k < r) V[row + (int64_t)k * m] = x[k];
            Vb[row + (int64_t)k * J.mpad] = bf16_rne(x[k]);
        }
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
// 64 columns (four 16-column panels of the column-panelled copy of M), so
// every V operand feeds four MFMAs.  M panels and V tiles reach LDS by DMA as
// in the A-pass.  The first column block of each chunk also forms the chunk's
// partial D = V^T V from the same V operands (upper-triangle 16x16 tiles
// spread over its waves).
template <int RT>
__device__ __forceinline__ void cpass_stream_tile(const Job &J, int tx, int ty, double *smem) {
    constexpr int RPAD = RT * 16, NST = kStreamStages, DMAX = 3;
    char *pipe = reinterpret_cast<char *>(smem);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lj = lane & 15, lg = lane >> 4;
    const int64_t n = J.n, mp = J.mpad;
    const int r = J.r;
    const int64_t jb = (int64_t)tx * 256 + wave * 64;
    // chunks and mpad are multiples of 128 rows: the chunk is a whole number
    // of >= 4 K-steps and every copy is in bounds (rows past m are zero;
    // panels past the last read the last one and are not stored)
    const int64_t i_begin = (int64_t)ty * J.chunk;
    const int64_t i_stop = (i_begin + J.chunk < mp) ? i_begin + J.chunk : mp;
    const int ksteps = (int)((i_stop - i_begin) / 32);
    const int64_t lastp = (n - 1) / 16;
    gmem<const uint16_t> *Mb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t pc = jb / 16 + c;
        Mb[c] = to_global(J.Mbc) + (pc < lastp ? pc : lastp) * mp * 16 + i_begin * 16 + lane * 8;
    }
    // wave w copies V tile w % RT (rows 16t + lj of Vb) into V slot w
    gmem<const uint16_t> *Vr =
        to_global(J.Vb) + (int64_t)(16 * (wave % RT) + lj) * mp + i_begin + 8 * lg;
    // D tiles (ta <= tb), numbered row by row: wave w takes numbers w + 4d
    constexpr int NPAIR = RT * (RT + 1) / 2;
    int dta[DMAX], dtb[DMAX];
    bool dok[DMAX];
#pragma unroll
    for (int d = 0; d < DMAX; ++d) {
        const int target = wave + 4 * d;
        dok[d] = tx == 0 && target < NPAIR;
        int fa = 0, fb = 0, idx = 0;
#pragma unroll
        for (int ta = 0; ta < RT; ++ta)
#pragma unroll
            for (int tb = ta; tb < RT; ++tb, ++idx)
                if (idx == target) {
                    fa = ta;
                    fb = tb;
                }
        dta[d] = fa;
        dtb[d] = fb;
    }
    auto issue = [&](int kk) {
        char *st = pipe + (kk % NST) * kStreamStage;
#pragma unroll
        for (int c = 0; c < 4; ++c) lds_dma16(Mb[c] + (int64_t)kk * 512, st + (wave * 4 + c) * 1024);
        lds_dma16(Vr + 32 * kk, st + 16384 + wave * 1024);
    };
    v4f acc[4][RT], dacc[DMAX];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[c][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int d = 0; d < DMAX; ++d) dacc[d] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    auto mma = [&](int kk) {
        const char *st = pipe + (kk % NST) * kStreamStage;
        bf16x8 a[4], b[RT];
#pragma unroll
        for (int c = 0; c < 4; ++c) a[c] = lds_bf16x8(st + (wave * 4 + c) * 1024 + lane * 16);
#pragma unroll
        for (int t = 0; t < RT; ++t) b[t] = lds_bf16x8(st + 16384 + t * 1024 + lane * 16);
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b[t], acc[c][t], 0, 0, 0);
#pragma unroll
        for (int d = 0; d < DMAX; ++d) {
            if (dok[d]) {
                const bf16x8 va = lds_bf16x8(st + 16384 + dta[d] * 1024 + lane * 16);
                const bf16x8 vb = lds_bf16x8(st + 16384 + dtb[d] * 1024 + lane * 16);
                dacc[d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, dacc[d], 0, 0, 0);
            }
        }
    };
#pragma unroll
    for (int kk = 0; kk < NST - 1; ++kk) issue(kk);
    int kk = 0;
    for (; kk < ksteps - (NST - 1); ++kk) {
        vm_wait_barrier<kStageOps * (NST - 2)>();   // stage kk landed, stage kk - 1 read
        issue(kk + NST - 1);
        mma(kk);
    }
    static_for<NST - 1>([&](auto j_c) {             // drain: nothing left to issue
        constexpr int j = decltype(j_c)::value;
        vm_wait_barrier<kStageOps * (NST - 2 - j)>();
        mma(kk + j);
    });
    // acc[c][t][v] = C[k = 16t + lj][j = jb + 16c + 4lg + v]; FP32 partials
    const auto out = to_global(reinterpret_cast<float *>(J.Cp)) + (int64_t)ty * r * n;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int k = 16 * t + lj;
        if (k < r) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t j = jb + 16 * c + 4 * lg + v;
                    if (j < n) out[j * r + k] = acc[c][t][v];
                }
        }
    }
    // dacc[d][v] = D[16 dta + 4lg + v][16 dtb + lj]
    const auto dout = to_global(J.Dp) + (int64_t)ty * RPAD * RPAD;
#pragma unroll
    for (int d = 0; d < DMAX; ++d) {
        if (dok[d]) {
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
    extern __shared__ double smem[];
    cpass_stream_tile<RT>(J, tx, ty, smem);
}

// v summed over the 4 lanes of its quad (lanes 4q .. 4q+3), by two DPP
// quad permutations; every lane of the quad gets the same sum.
template <int CTRL>
__device__ __forceinline__ double quad_dpp(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double quad_sum(double v) {
    v += quad_dpp<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    return v + quad_dpp<0x4E>(v);   // quad_perm [2, 3, 0, 1]
}

// HALS (Alg. 3) or MU (Alg. 2) update of one row of V in FP64 by the 4 lanes
// of a quad: lane p holds entries EP p .. EP p + EP - 1 (EP = RPAD / 4) of the
// row in x.  Each Gram dot product sum_l x_l G_kl is split over the quad and
// summed by DPP.  HALS takes k = 0 .. RPAD-1 in turn, x_k <- max(0, x_k +
// (a_k - sum_l x_l G_kl) / G_kk), formed by the lane that owns k; MU forms all
// the sums from the old x, then x_k <- x_k a_k / sum_l x_l G_kl.  Steps with
// 1/G_kk = 0 (k >= r, or G_kk = 0) leave x_k as it is; steps k >= r are
// skipped: each step runs the next one only while k + 1 < r (a nest of
// uniform branches).  Step k reads the lane's part of Gram row k + 2 (with
// a_{k+2} and 1/G_{k+2,k+2}) behind the previous step's sum and holds it two
// steps in registers, so LDS latency stays off the chain of dependent sums;
// without that, each step's reads waited behind its own branch.
template <int RPAD, int MODE>
__device__ __forceinline__ void quad_row_update(double (&x)[RPAD / 4], const double *arow,
                                                const double *G, const double *gi, int p, int r) {
    typedef double v2d __attribute__((ext_vector_type(2)));
    constexpr int EP = RPAD / 4, NV = EP / 2, PD = 2;
    struct Row {
        v2d g[NV];
        double a, gk;
    };
    auto load_row = [&](int k, double dep, Row &dst) {
        const int ko = ordered_after(k, dep);
        const double *g = G + ko * RPAD + EP * p;
#pragma unroll
        for (int v = 0; v < NV; ++v) dst.g[v] = *(const lmem<v2d> *)(g + 2 * v);
        dst.a = arow[ko];
        dst.gk = gi[ko];
    };
    auto dot = [&](const Row &row) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int i = 0; i < EP; i += 4) {
            const v2d ga = row.g[i / 2], gb = row.g[i / 2 + 1];
            s0 = fma_t(x[i], ga[0], s0);
            s1 = fma_t(x[i + 1], ga[1], s1);
            s2 = fma_t(x[i + 2], gb[0], s2);
            s3 = fma_t(x[i + 3], gb[1], s3);
        }
        return quad_sum((s0 + s1) + (s2 + s3));
    };
    if (r <= 0) return;
    Row rows[PD];
#pragma unroll
    for (int i = 0; i < PD; ++i) load_row(i < RPAD ? i : 0, 0.0, rows[i]);
    double dprev = 0.0;
    double den[MODE == MODE_HALS ? 1 : EP];
#pragma unroll
    for (int i = 0; i < (MODE == MODE_HALS ? 1 : EP); ++i) den[i] = 0.0;
    auto step = [&](auto self, auto k_c) -> void {
        constexpr int k = decltype(k_c)::value, ik = k % EP;
        Row rnew;
        if constexpr (k + PD < RPAD) {
            load_row(k + PD, dprev, rnew);
            // keep the reads here, ahead of this step's sum
            __builtin_amdgcn_sched_barrier(0);
        }
        const double d = dot(rows[0]);
        dprev = d;
        if constexpr (MODE == MODE_HALS) {
            const double ak = rows[0].a, gk = rows[0].gk;
            const double c = x[ik] + (ak - d) * gk;
            const double cp = c > 0.0 ? c : 0.0;
            const double nx = gk > 0.0 ? cp : x[ik];
            x[ik] = p == k / EP ? nx : x[ik];
        } else {
            den[ik] = p == k / EP ? d : den[ik];
        }
#pragma unroll
        for (int i = 0; i + 1 < PD; ++i) rows[i] = rows[i + 1];
        if constexpr (k + PD < RPAD) rows[PD - 1] = rnew;
        if constexpr (k + 1 < RPAD) {
            if (k + 1 < r) self(self, std::integral_constant<int, k + 1>{});
        }
    };
    step(step, std::integral_constant<int, 0>{});
    if constexpr (MODE != MODE_HALS) {
#pragma unroll
        for (int i = 0; i < EP; ++i) {
            const int k = EP * p + i;
            if (k < r && den[i] > 0.0) x[i] = x[i] * arow[k] / den[i];
        }
    }
}

// The V update of 16 rows first, first + step, ... of one wave from their rows
// of A in LDS (Aw, stride rpad + 1, FP64): the quad of lanes 4q .. 4q+3 takes
// row first + step q (quad_row_update); MODE_STORE stores A instead.  V (or
// A) is read and written only for rows < m.
template <int RPAD, int MODE>
__device__ __forceinline__ void update_rows(const Job &J, const double *Aw, const double *Gs,
                                            const double *Gi, int64_t first, int step) {
    constexpr int AS = RPAD + 1, EP = RPAD / 4;
    const int lane = threadIdx.x & 63, q = lane >> 2, p = lane & 3;
    const int64_t m = J.m;
    const int r = J.r;
    const auto V = to_global(J.V);
    // lane 4q + p: entries EP p .. EP p + EP - 1 of row first + step q
    const int64_t row = first + (int64_t)step * q;
    const bool live = row < m;
    const double *arow = Aw + q * AS;
    if constexpr (MODE == MODE_STORE) {
        if (live) {
#pragma unroll
            for (int i = 0; i < EP; ++i) {
                const int k = EP * p + i;
                if (k >= r) continue;
                if (J.Ad) to_global(J.Ad)[row + (int64_t)k * m] = arow[k];
                else to_global(J.A)[row + (int64_t)k * m] = (float)arow[k];
            }
        }
    } else {
        // all loads unconditional (clamped row and column), then masked, so
        // that they are in flight together
        const int64_t rc = live ? row : m - 1;
        float xv[EP];
#pragma unroll
        for (int i = 0; i < EP; ++i) {
            const int k = EP * p + i;
            xv[i] = V[rc + (int64_t)(k < r ? k : 0) * m];
        }
        double x[EP];
#pragma unroll
        for (int i = 0; i < EP; ++i) x[i] = (live && EP * p + i < r) ? (double)xv[i] : 0.0;
        quad_row_update<RPAD, MODE>(x, arow, Gs, Gi, p, r);
        if (live) {
#pragma unroll
            for (int i = 0; i < EP; ++i) {
                const int k = EP * p + i;
                if (k < r) V[row + (int64_t)k * m] = (float)x[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Streaming passes for large levels in FP32 mode (job.stream = 1, prec = 0):
// m >= kFStreamMinRows, m and the column stride of M multiples of 4, M 16-byte
// aligned.  FP32 products are MFMA-bound (v_mfma_f32_16x16x4f32), so the
// design keeps the matrix cores busy and M in flight to feed them: both
// passes stage their operands in LDS by DMA, kS32Stages stages of 12 KB (one
// K-step of 16 rows or columns: the 4 waves' 8 KB of M, 4 KB of the small
// operand), kS32Stages - 1 of them in flight while one is multiplied, and
// every wave issues kS32Ops copies per stage in the C-pass (RS + 1 in the
// A-pass).  256 VGPRs, two waves per SIMD.
// ---------------------------------------------------------------------------
constexpr int kS32Stages = 6;
constexpr int kS32Stage = 12 * 1024;
constexpr int kS32Ops = 3;

__device__ __forceinline__ void lds_dma16f(gmem<const float> *src, char *dst) {
    __builtin_amdgcn_global_load_lds((gmem<const void> *)src, (lmem<void> *)dst, 16, 0, 0);
}

__device__ __forceinline__ v4f lds_v4f(const char *p) { return *(const lmem<v4f> *)p; }

// A-pass: a wave owns RW = 16 RS rows (RS = 2, 128-row blocks, from
// m = 65536; RS = 1, 64-row blocks, on smaller levels so that the grid still
// fills the chip); the M columns and the rows of Wt (W transposed, stride
// rpad) reach LDS by DMA, kS32Stages stages of 16 columns (4 K-steps) deep.
// Per stage a wave copies its RW rows x 16 columns as RS 1 KB tiles (lane l:
// column CPD h + l/LPC, rows 4(l%LPC) .. +3; LDS column-major, RW rows per
// column), and 1 KB w % rpad/16 of the stage's 16 x rpad block of Wt (the 4
// slots hold the block contiguously): RS + 1 copies.  Lane (li, lk) then
// reads rows RS li .. RS li + RS - 1 of column 4q + lk (K-step q) and W
// entries 16t + li of that column (adjacent in a row of Wt, wt_pos) and feeds
// RS MFMAs, so MFMA s maps its row index li to row row0 + RS li + s; its
// accumulator v of lane (li', lk') holds A[row0 + RS(4lk' + v) + s][16t + li'].
// Once per stage (16 products per chain) the accumulators are added into FP64
// sums.  Copies past n or m read a clamped column or row; the W operand of
// columns past n is zeroed (only the last kS32Stages - 1 stages can hold
// them) and rows past m are not stored.  The V update (FP64, as in the
// regular kernels) runs one s at a time: the wave's 16 rows of that s go to a
// wave-private LDS slot and the quad of lanes 4q .. 4q+3 updates row
// row0 + RS q + s (quad_row_update).  The Gram and the row slots reuse the
// stage memory.
// ---------------------------------------------------------------------------
template <int RT, int MODE, int RS>
__device__ __forceinline__ void apass_s32_tile(const Job &J, int tile, int part, double *smem) {
    constexpr int RPAD = RT * 16, GS = RPAD, AS = RPAD + 1, NST = kS32Stages;
    constexpr int RW = 16 * RS;      // rows per wave
    constexpr int LPC = RW / 4;      // copy lanes per column (4 rows each)
    constexpr int CPD = 64 / LPC;    // columns per 1 KB copy
    constexpr int WOFF = 4096 * RS;  // Wt slots after the M tiles
    typedef float v2f __attribute__((ext_vector_type(2)));
    char *pipe = reinterpret_cast<char *>(smem);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m = J.m, n = J.n, ldm = J.ldm;
    const int r = J.r;
    const int64_t row0 = (int64_t)tile * 4 * RW + wave * RW;
    // this block's stages kb .. ke-1 (all of n unless the reduction is split)
    const int nstage = (int)((n + 15) / 16);
    const int per = (nstage + J.aks - 1) / J.aks;
    const int kb = part * per;
    const int ke = kb + per < nstage ? kb + per : nstage;
    const int ksteps = ke > kb ? ke - kb : 0;
    const int64_t cend = 16 * (int64_t)ke < n ? 16 * (int64_t)ke : n;   // columns < cend
    // copy sources: lane l takes column CPD h + l/LPC of the stage, rows
    // 4(l%LPC) .. +3
    int64_t rc = row0 + 4 * (lane % LPC);
    rc = rc < m ? rc : m - 4;   // m % 4 == 0
    const auto Mr = to_global(J.M) + rc;
    const int cl = lane / LPC;
    const auto Wt = to_global(J.Wt);
    const int64_t wlast = n * RPAD - 4;   // last 16 bytes of Wt
    const int64_t woff = 256 * (wave % RT) + 4 * lane;
    auto issue = [&](int kk) {
        char *st = pipe + (kk % NST) * kS32Stage;
#pragma unroll
        for (int h = 0; h < RS; ++h) {
            const int64_t j = 16 * (int64_t)(kb + kk) + CPD * h + cl;
            lds_dma16f(Mr + (j < n ? j : n - 1) * ldm, st + wave * 1024 * RS + h * 1024);
        }
        const int64_t e = 16 * (int64_t)(kb + kk) * RPAD + woff;
        lds_dma16f(Wt + (e < wlast ? e : wlast), st + WOFF + wave * 1024);
    };
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
    auto mma = [&](int kk, bool tail) {
        const char *st = pipe + (kk % NST) * kS32Stage;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * q + lk;
            // rows RS li .. RS li + RS - 1 of column c (LDS: RW rows per column)
            const char *ap = st + wave * 1024 * RS + c * 4 * RW + 4 * RS * li;
            float a[RS];
            if constexpr (RS == 2) {
                const v2f x = *(const lmem<v2f> *)ap;
                a[0] = x[0]; a[1] = x[1];
            } else {
                a[0] = *(const lmem<float> *)ap;
            }
            const bool dead = tail && 16 * (int64_t)(kb + kk) + c >= cend;
            // W entries 16t + li of column c: contiguous in the interleaved Wt row
            const char *wp = st + WOFF + (c * RPAD + li * RT) * 4;
            float b[RT];
            if constexpr (RT == 4) {
                const v4f x = *(const lmem<v4f> *)wp;
                b[0] = x[0]; b[1] = x[1]; b[2] = x[2]; b[3] = x[3];
            } else if constexpr (RT == 2) {
                const v2f x = *(const lmem<v2f> *)wp;
                b[0] = x[0]; b[1] = x[1];
            } else {
#pragma unroll
                for (int t = 0; t < RT; ++t) b[t] = *(const lmem<float> *)(wp + 4 * t);
            }
#pragma unroll
            for (int t = 0; t < RT; ++t) b[t] = dead ? 0.0f : b[t];
#pragma unroll
            for (int s2 = 0; s2 < RS; ++s2)
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[s2][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s2], b[t], acc[s2][t], 0, 0, 0);
        }
#pragma unroll
        for (int s2 = 0; s2 < RS; ++s2)
#pragma unroll
            for (int t = 0; t < RT; ++t) {
#pragma unroll
                for (int v = 0; v < 4; ++v) hs[s2][t][v] += (double)acc[s2][t][v];
                acc[s2][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            }
    };
#pragma unroll
    for (int kk = 0; kk < NST - 1; ++kk) issue(kk);
    int kk = 0;
    // stages kk <= ksteps - NST end at or before column 16 (ke - 1) < cend
    for (; kk < ksteps - (NST - 1); ++kk) {
        vm_wait_barrier<(RS + 1) * (NST - 2)>();   // stage kk landed, stage kk - 1 read
        issue(kk + NST - 1);
        mma(kk, false);
    }
    static_for<NST - 1>([&](auto j_c) {   // drain (stages past ksteps are wholly masked)
        constexpr int j = decltype(j_c)::value;
        vm_wait_barrier<(RS + 1) * (NST - 2 - j)>();
        mma(kk + j, true);
    });
    if (J.aks > 1) {
        // split reduction: this part's FP64 rows of A, row i at Cp + (part *
        // nA tm + i) rpad (rows past m too: never stored by the update)
        const auto ap = to_global(J.Cp) + ((int64_t)part * J.nA * J.tm) * RPAD;
#pragma unroll
        for (int s2 = 0; s2 < RS; ++s2)
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    ap[(row0 + RS * (4 * lk + v) + s2) * RPAD + 16 * t + li] = hs[s2][t][v];
        return;
    }
    __syncthreads();   // every wave done with the stages
    double *Gs = smem;
    double *Gi = Gs + RPAD * GS;
    if constexpr (MODE != MODE_STORE) load_gram<RPAD>(J.Bd, r, Gs, GS, Gi);
    double *Aw = Gi + RPAD + wave * 16 * AS;   // 16 rows of this wave (one s)
    __syncthreads();                            // Gram in LDS
    static_for<RS>([&](auto s_c) {
        constexpr int s2 = decltype(s_c)::value;
        __builtin_amdgcn_wave_barrier();
        // hs[s2][t][v] = A[row0 + RS q + s2][16t + li] with q = 4 lk + v
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) Aw[(4 * lk + v) * AS + 16 * t + li] = hs[s2][t][v];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        update_rows<RPAD, MODE>(J, Aw, Gs, Gi, row0 + s2, RS);
    });
}

template <int RT, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_apass_s32(const Job *__restrict__ jobs,
                                                   const int2 *__restrict__ bmap) {
    extern __shared__ double smem[];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (jt.y >= J.nA * J.aks || J.st->stop) return;
    const int tile = jt.y % J.nA, part = jt.y / J.nA;
    if (J.tm == 64)
        apass_s32_tile<RT, MODE, 1>(J, tile, part, smem);
    else
        apass_s32_tile<RT, MODE, 2>(J, tile, part, smem);
}

// Split A-pass, second half (job.aks > 1, 64-row tiles): the aks partial rows
// of A of a tile are added in part order (FP64) into LDS, then each wave
// updates its 16 rows of V as the unsplit A-pass does.
template <int RT, int MODE>
__global__ __launch_bounds__(256) void k_afinal_s32(const Job *__restrict__ jobs,
                                                    const int2 *__restrict__ bmap) {
    constexpr int RPAD = RT * 16, GS = RPAD, AS = RPAD + 1, PER = RPAD / 4;
    extern __shared__ double smem[];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    if (jt.y >= J.nA || J.st->stop) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t rw0 = (int64_t)jt.y * 64 + 16 * wave;   // this wave's 16 rows
    double *Gs = smem;
    double *Gi = Gs + RPAD * GS;
    double *Aw = Gi + RPAD + wave * 16 * AS;
    if constexpr (MODE != MODE_STORE) load_gram<RPAD>(J.Bd, J.r, Gs, GS, Gi);
    // entries e = lane + 64 i of the wave's 16 x RPAD block (row e / RPAD)
    const auto ap = to_global(J.Cp) + rw0 * RPAD;
    const int64_t pstride = (int64_t)J.nA * J.tm * RPAD;
    // parts taken four at a time, (p0 + p1) + (p2 + p3) added to the running
    // sum (fixed order); the four loads of an entry are in flight together,
    // and a part past aks reads part 0 with weight zero
    double a[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) a[i] = 0.0;
    for (int p0 = 0; p0 < J.aks; p0 += 4) {
        double wgt[4];
        int64_t off[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            wgt[u] = p0 + u < J.aks ? 1.0 : 0.0;
            off[u] = (p0 + u < J.aks ? p0 + u : 0) * pstride + lane;
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const double b0 = ap[off[0] + 64 * i], b1 = ap[off[1] + 64 * i];
            const double b2 = ap[off[2] + 64 * i], b3 = ap[off[3] + 64 * i];
            a[i] += (b0 * wgt[0] + b1 * wgt[1]) + (b2 * wgt[2] + b3 * wgt[3]);
        }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = lane + 64 * i;
        Aw[(e / RPAD) * AS + e % RPAD] = a[i];
    }
    __syncthreads();   // Gram and rows of A in LDS
    update_rows<RPAD, MODE>(J, Aw, Gs, Gi, rw0, 1);
}

// (ta, tb) of upper 16x16 tile idx of an RT x RT tile grid, row by row.
__device__ __forceinline__ void upper_tile(int idx, int rt, int &ta, int &tb) {
    int a = 0;
    while (idx >= rt - a) {
        idx -= rt - a;
        ++a;
    }
    ta = a;
    tb = a + idx;
}

// Sum of the 4 waves' FP64-MFMA partials of D tile (ta, tb) (layout
// d[v] = D[4v + lg][lj]) in fixed wave order, stored by wave 0.  dl: 1024
// doubles of LDS; the block must be free to reuse them.
template <int RPAD>
__device__ __forceinline__ void store_d_tile(const v4d &d, double *dl, gmem<double> *dout, int ta,
                                             int tb) {
    const int tid = threadIdx.x, wave = tid >> 6, lj = tid & 15, lg = (tid >> 4) & 3;
#pragma unroll
    for (int v = 0; v < 4; ++v) dl[wave * 256 + (4 * v + lg) * 16 + lj] = d[v];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = (4 * v + lg) * 16 + lj;
            dout[(16 * ta + 4 * v + lg) * RPAD + 16 * tb + lj] =
                ((dl[e] + dl[256 + e]) + dl[512 + e]) + dl[768 + e];
        }
    }
    __syncthreads();
}

// C-pass (FP32): a block of 4 waves owns 128 columns of one row chunk; a wave
// owns 32 columns (two 16-column panels).  Per 16-row K-step lane (lj, g) of
// a wave copies, by DMA, 4 consecutive rows 4g .. 4g+3 of column lj of each
// of its panels, and one wave per rank tile copies the same rows of V; the
// lane reads back its own 16 bytes, which feed 4 MFMAs whose K index g maps
// to row i0 + 4g + s.  Each step's chains (16 products) are added into FP64
// sums.  Copies past the chunk's end read its last 4 rows; the V operand of
// such rows is zeroed (only the last kS32Stages - 1 steps can hold them).
// Rank columns k >= r copy column 0: they feed only C rows and D entries that
// are never stored or read.
//
// The chunk's upper 16x16 tiles of D = V^T V are spread over its column
// blocks.  With FD, block tx forms tile tx from the V operands it already
// reads: per step, wave w takes the FP64 MFMA of rows 4g + w (g = 0..3) of
// the step, so the four waves' partials cover every row once and are added
// in LDS.  Tiles tx + nCx, tx + 2 nCx, ... (only when there are fewer column
// blocks than tiles) take a pass over V alone, the waves taking every fourth
// step.
template <int RT, bool FD>
__device__ __forceinline__ void cpass_s32_tile(const Job &J, int tx, int ty, double *smem) {
    constexpr int RPAD = RT * 16, RN = 2, NT = RT * (RT + 1) / 2, NST = kS32Stages;
    char *pipe = reinterpret_cast<char *>(smem);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lj = lane & 15, lg = lane >> 4;
    const int64_t m = J.m, n = J.n, ldm = J.ldm;
    const int r = J.r;
    const auto V = to_global(J.V);
    const int64_t jb = (int64_t)tx * 128 + wave * 32;
    const int64_t i_begin = (int64_t)ty * J.chunk;
    const int64_t i_end = (i_begin + J.chunk < m) ? i_begin + J.chunk : m;
    const int ksteps = (int)((i_end - i_begin + 15) / 16);
    const int64_t i_last = i_end - 4;   // m % 4 == 0: a whole group of 4 rows
    gmem<const float> *Mc[RN];
#pragma unroll
    for (int c = 0; c < RN; ++c) {
        const int64_t j = jb + 16 * c + lj;
        Mc[c] = to_global(J.M) + (j < n ? j : n - 1) * ldm + 4 * lg;
    }
    const int kv = 16 * (wave % RT) + lj;
    gmem<const float> *Vr = V + (int64_t)(kv < r ? kv : 0) * m + 4 * lg;
    auto issue = [&](int kk) {
        char *st = pipe + (kk % NST) * kS32Stage;
        int64_t i0 = i_begin + 16 * (int64_t)kk;
        i0 = i0 + 4 * lg <= i_last ? i0 : i_last - 4 * lg;   // rows i0 + 4lg .. +3 stay in the chunk
#pragma unroll
        for (int c = 0; c < RN; ++c) lds_dma16f(Mc[c] + i0, st + (wave * RN + c) * 1024);
        lds_dma16f(Vr + i0, st + 8192 + wave * 1024);
    };
    int ta = 0, tb = 0;
    if (FD) upper_tile(tx, RT, ta, tb);
    v4f acc[RN][RT];
    double hs[RN][RT][4];
    v4d dacc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < RN; ++c)
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            acc[c][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int v = 0; v < 4; ++v) hs[c][t][v] = 0.0;
        }
    auto mma = [&](int kk, bool tail) {
        const char *st = pipe + (kk % NST) * kS32Stage;
        v4f a[RN], b[RT];
#pragma unroll
        for (int c = 0; c < RN; ++c) a[c] = lds_v4f(st + (wave * RN + c) * 1024 + lane * 16);
#pragma unroll
        for (int t = 0; t < RT; ++t) b[t] = lds_v4f(st + 8192 + t * 1024 + lane * 16);
        const bool dead = tail && i_begin + 16 * (int64_t)kk + 4 * lg >= i_end;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) b[t][s] = dead ? 0.0f : b[t][s];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < RN; ++c)
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c][s], b[t][s], acc[c][t], 0, 0, 0);
        if constexpr (FD) {   // row 4g + wave of V tiles ta and tb (V slot t holds tile t)
            const char *vw = st + 8192 + lane * 16 + wave * 4;
            const float fa = *(const lmem<float> *)(vw + ta * 1024);
            const float fb = *(const lmem<float> *)(vw + tb * 1024);
            dacc = __builtin_amdgcn_mfma_f64_16x16x4f64(dead ? 0.0 : (double)fa, (double)fb, dacc, 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < RN; ++c)
#pragma unroll
            for (int t = 0; t < RT; ++t) {
#pragma unroll
                for (int v = 0; v < 4; ++v) hs[c][t][v] += (double)acc[c][t][v];
                acc[c][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            }
    };
#pragma unroll
    for (int kk = 0; kk < NST - 1; ++kk) issue(kk);
    int kk = 0;
    // steps kk <= ksteps - NST end at or before row 16 (ksteps - 1) < i_end - i_begin
    for (; kk < ksteps - (NST - 1); ++kk) {
        vm_wait_barrier<kS32Ops * (NST - 2)>();   // stage kk landed, stage kk - 1 read
        issue(kk + NST - 1);
        mma(kk, false);
    }
    static_for<NST - 1>([&](auto j_c) {   // drain (steps past ksteps are wholly masked)
        constexpr int j = decltype(j_c)::value;
        vm_wait_barrier<kS32Ops * (NST - 2 - j)>();
        mma(kk + j, true);
    });
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
                    if (j < n) out[j * r + k] = hs[c][t][v];
                }
        }
    }
    if constexpr (FD) {
        __syncthreads();   // every wave done with the stages
        const auto dout = to_global(J.Dp) + (int64_t)ty * RPAD * RPAD;
        store_d_tile<RPAD>(dacc, smem, dout, ta, tb);
        for (int idx = tx + J.nCx; idx < NT; idx += J.nCx) {
            upper_tile(idx, RT, ta, tb);
            const int ka = 16 * ta + lj, kb = 16 * tb + lj;
            const auto Va = V + (int64_t)(ka < r ? ka : 0) * m;
            const auto Vb = V + (int64_t)(kb < r ? kb : 0) * m;
            v4d d = v4d{0.0, 0.0, 0.0, 0.0};
            for (int st = wave; st < ksteps; st += 4) {
                const int64_t ib = i_begin + 16 * (int64_t)st + 4 * lg;
                const bool ok = ib < i_end;
                const int64_t ic = ok ? ib : i_last;
                v4f xa = *(gmem<const v4f> *)(Va + ic), xb = *(gmem<const v4f> *)(Vb + ic);
                if (!ok) xa = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    d = __builtin_amdgcn_mfma_f64_16x16x4f64((double)xa[s], (double)xb[s], d, 0, 0, 0);
            }
            store_d_tile<RPAD>(d, smem, dout, ta, tb);
        }
    }
}

template <int RT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_cpass_s32(
    const Job *__restrict__ jobs, const int2 *__restrict__ bmap) {
    extern __shared__ double smem[];
    const int2 jt = block_job(bmap);
    const Job &J = jobs[jt.x];
    int tx = jt.y % J.nCx, ty = jt.y / J.nCx;
    if (!bmap) {   // single problem: the column blocks of a chunk run on one XCD
        const int l = (int)(blockIdx.x >> 3);
        ty = (int)(blockIdx.x & 7) + 8 * (l / J.nCx);
        tx = l % J.nCx;
    }
    if (ty >= J.chunks || J.st->stop) return;
    if (tx < RT * (RT + 1) / 2)
        cpass_s32_tile<RT, true>(J, tx, ty, smem);
    else
        cpass_s32_tile<RT, false>(J, tx, ty, smem);
}

}  // namespace

// ---- host side -------------------------------------------------------------

int cpass_stream_grid(int nCx, int chunks) { return 8 * nCx * ((chunks + 7) / 8); }

// The DMA stages, later the FP64 Gram (stride rpad) and 1/G_kk, then 4 waves
// x 16 rows of A (FP64, stride rpad + 1).
size_t apass_s32_lds_bytes(int rpad) {
    const size_t epi = sizeof(double) * ((size_t)rpad * rpad + rpad + 4 * 16 * (size_t)(rpad + 1));
    const size_t pipe = (size_t)kS32Stages * kS32Stage;
    return epi > pipe ? epi : pipe;
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

size_t afinal_s32_lds_bytes(int rpad) {
    return sizeof(double) * ((size_t)rpad * rpad + rpad + 4 * 16 * (size_t)(rpad + 1));
}

hipError_t launch_afinal_s32(int mode, int rpad, const Job *jobs, const int2 *bmap, int blocks,
                             hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (mode != MODE_HALS && mode != MODE_MU) return hipErrorInvalidValue;
    const size_t lds = afinal_s32_lds_bytes(rpad);
    const bool h = mode == MODE_HALS;
    switch (rpad) {
        case 16: h ? k_afinal_s32<1, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_afinal_s32<1, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 32: h ? k_afinal_s32<2, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_afinal_s32<2, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 48: h ? k_afinal_s32<3, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_afinal_s32<3, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 64: h ? k_afinal_s32<4, MODE_HALS><<<blocks, 256, lds, s>>>(jobs, bmap)
                   : k_afinal_s32<4, MODE_MU><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cpass_s32(int rpad, const Job *jobs, const int2 *bmap, int blocks,
                            hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    const size_t lds = (size_t)kS32Stages * kS32Stage;
    switch (rpad) {
        case 16: k_cpass_s32<1><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 32: k_cpass_s32<2><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 48: k_cpass_s32<3><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 64: k_cpass_s32<4><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The DMA stages (later holding the 4 waves' rows of A, FP32, stride
// rpad + 1), then the FP32 Gram and 1/G_kk.
size_t apass_stream_lds_bytes(int rpad) {
    static_assert(4 * 16 * kStreamAPanels * 65 * sizeof(float) <= kStreamStages * kStreamAStage,
                  "A rows must fit in the stages");
    return (size_t)kStreamStages * kStreamAStage + sizeof(float) * ((size_t)rpad * rpad + rpad);
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
    const size_t lds = (size_t)kStreamStages * kStreamStage;
    switch (rpad) {
        case 16: k_cpass_stream<1><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 32: k_cpass_stream<2><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 48: k_cpass_stream<3><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        case 64: k_cpass_stream<4><<<blocks, 256, lds, s>>>(jobs, bmap); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Allow the streaming passes the LDS their DMA stages, Gram and row staging
// take (above the 64 KB default).
template <int RT>
static void stream_lds_attr(hipError_t &e) {
    for (const void *f : {(const void *)k_apass_stream<RT, MODE_HALS>,
                          (const void *)k_apass_stream<RT, MODE_MU>,
                          (const void *)k_cpass_stream<RT>,
                          (const void *)k_apass_s32<RT, MODE_HALS>,
                          (const void *)k_apass_s32<RT, MODE_MU>,
                          (const void *)k_afinal_s32<RT, MODE_HALS>,
                          (const void *)k_afinal_s32<RT, MODE_MU>,
                          (const void *)k_cpass_s32<RT>}) {
        const hipError_t x = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 160 * 1024);
        if (x != hipSuccess && e == hipSuccess) e = x;
    }
}

hipError_t enable_stream_lds() {
    hipError_t e = hipSuccess;
    stream_lds_attr<1>(e);
    stream_lds_attr<2>(e);
    stream_lds_attr<3>(e);
    stream_lds_attr<4>(e);
    return e;
}

}  // namespace nmf
