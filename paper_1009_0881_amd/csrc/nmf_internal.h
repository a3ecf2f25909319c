// Internal declarations of libnmf: plan, workspace layout, device state and
// the kernel launchers.  Host C++ only; the kernels live in *.hip files.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/nmf.h"
#include "job.h"

namespace nmf {

constexpr int kMaxRank = 64;
constexpr int kMaxLevels = 12;
constexpr int kNormParts = 1024;   // max partial sums of ||M_l||^2 (per level)
// BF16 operand copies are padded to multiples of 128 rows and columns (and C-pass
// chunks are multiples of 128 rows), so the streaming loops over 32-wide K-steps
// in batches of two double-buffered pairs need no bounds tests.
constexpr int64_t kBfPad = 128;
inline int64_t bf_pad(int64_t x) { return (x + kBfPad - 1) / kBfPad * kBfPad; }

// Number of partial sums of ||X||^2 for a rows x ncols matrix (work items are
// (column, 2048-row chunk)); every path uses this split, so norms agree bitwise.
inline int norm_parts(int64_t rows, int64_t ncols) {
    const int64_t items = ncols * ((rows + 2047) / 2048);
    return (int)(items < 1 ? 1 : (items > kNormParts ? kNormParts : items));
}

// Device-side control block at the start of every workspace.
struct DevState {
    int32_t stop;        // 1: a stop condition was met; every later kernel returns at once
    int32_t log_len;     // iterations logged so far (index of the next entry)
    int32_t status;      // 0 or an nmf_status error code raised on the device
    int32_t stopped;     // 1: the tolerance was reached
    double last_rel;     // rel_err of the last executed iteration
    int32_t flags;       // input check: bit0 negative entry, bit1 non-finite entry
    int32_t pad[9];
};
static_assert(sizeof(DevState) <= 256, "state block");

struct LevelInfo {
    int32_t h, w;
    int64_t m;
    int64_t n;           // columns at this level (the finest n unless two-sided)
    size_t off_W;        // two-sided: workspace offset of W_l (levels >= 1)
    int32_t gram_w_parts;   // split of the length-n reduction of W W^T (ANLS Gram)
    int64_t gram_w_chunk;
    size_t off_M;        // workspace offset of M_l (levels >= 1)
    size_t off_V;        // workspace offset of V_l (levels >= 1)
    size_t off_Mbp, off_Mbc, off_Vb;   // BF16 mode: copies of M_l (A-pass, C-pass layouts), V_l
    int64_t mpad;        // m rounded up to 32 (column stride of the BF16 copies)
    int32_t atm;         // rows per block of the regular A-pass (16 or 64)
    int32_t gseg;        // B = W W^T: column segments per upper tile (1..kGramSegMax)
    int32_t cp_chunks;   // split of the m-reduction in V^T M
    int64_t cp_chunk;    // rows per chunk (multiple of 16; 32 in BF16 mode)
    bool stream;         // BF16 mode, large level: streaming A/C-pass kernels
    int32_t scp_chunks;  // split of the m-reduction for the streaming C-pass
    int64_t scp_chunk;
    bool fstream;        // large or wide level: FP32 streaming kernels possible (m % 4 == 0)
    int32_t ftm;         // FP32 streaming A-pass rows per block (64 or 128)
    int32_t aks;         // FP32 streaming A-pass: split of the n-reduction (1: none)
    int32_t fcp_chunks;  // split of the m-reduction for the FP32 streaming C-pass
    int64_t fcp_chunk;
    int32_t gram_parts;  // split of the length-m reduction of V^T V
    int64_t gram_chunk;
};

struct Step {            // one schedule entry
    int32_t kind;        // 0 run, 1 restrict V (depth -> depth+1), 2 prolong V (depth+1 -> depth)
    int32_t depth;
    int32_t count;
};

struct Workspace {
    size_t off_state, off_log, off_logdepth, off_norm, off_nparts;
    size_t off_Bd, off_Bf, off_Dd, off_Df;
    size_t off_gparts, off_cparts, off_Cr, off_bparts, off_rparts, off_A, off_C, off_Wb;
    size_t off_Wt, off_Dp, off_jobs;
    size_t off_tmpM;     // two-sided: R_m M_l before the column restriction
    // NMF_KL: row sums of W (rpad), their block partials, the column sums of V
    // per chunk, the divergence partials (16-row blocks of the finest level)
    // and sum(M_l) per level
    size_t off_klw, off_klwp, off_klvp, off_kld, off_klm;
    // NTF: (C kr B)^T (r x n FP32, the W of the jobs) and the Grams B^T B,
    // C^T C (r x r FP64 each; their Hadamard product is Bd); A^T X_(1) is off_C
    size_t off_ntfW, off_ntfG;
    size_t gparts_cap;   // doubles
    size_t rparts_cap;   // doubles
    size_t total;
};

enum KernelKind {
    K_APASS = 0, K_GRAM_V, K_CPART, K_CFINAL, K_GRAM_W, K_RESID, K_NNLS_ROWS, K_NNLS_COLS,
    K_RESTRICT, K_PROLONG, K_SUMSQ, K_KL_DIV, K_NTF, K_NUM_KINDS
};

// Host-mapped stop flags and completion events for tolerance polling: a solve
// takes one flag from the pool (allocated on first use) and returns it; the
// mutex makes concurrent solves on one plan safe.
struct PollPool {
    std::mutex mu;
    std::vector<int32_t *> flags;    // hipHostMalloc(hipHostMallocMapped), idle
    std::vector<hipEvent_t> events;  // timing disabled, idle
};

// Optional HIP-event timing of selected kernel kinds.  A solve takes event
// pairs from the pool, keeps its pending pairs in its own context and returns
// them (with its times added to the totals) when it has synchronised; the
// mutex makes concurrent solves on one plan safe.
struct Profiler {
    uint32_t mask = 0;
    std::mutex mu;                           // guards pool, counts, ms
    std::vector<hipEvent_t> pool;            // idle events, created lazily, reused
    int64_t counts[K_NUM_KINDS] = {};
    double ms[K_NUM_KINDS] = {};
};

struct Plan {
    nmf_desc d;
    Profiler prof;
    PollPool poll;
    std::vector<LevelInfo> lv;
    Workspace ws;
    int rpad;            // r rounded up to a multiple of 16
    int wc, cf;          // tiles: C-pass row groups per tile, W-update columns per tile
    bool grouped;        // NMF_TILE_GROUPED: sized for grouped launches, C-pass chunks
                         // of at least 512 rows
    int num_cu;
    int32_t gram_w_parts;
    int64_t gram_w_chunk;
};

// ratio: iterations per finest-iteration equivalent grow by this factor per
// depth (4: m halved per axis; 8: two-sided).
std::vector<Step> make_schedule(int cycle, int levels, int64_t iters, int ratio = 4);
nmf_status build_plan(const nmf_desc &d, Plan &p, std::string &err);

// ---- launchers (kernels.hip etc.) ------------------------------------------
// All take a stop pointer (may be null): kernels return at once when *stop != 0.
hipError_t launch_restrict(int xfer, int h, int w, int64_t ncols, const float *X, int64_t ldx,
                           float *Y, const int32_t *stop, hipStream_t s);
hipError_t launch_prolong(int xfer, int h, int w, int64_t ncols, const float *Y, float *X,
                          const int32_t *stop, hipStream_t s);
// 1-D transfer (eq. restr / eq. prol of `xfer`) along the second index j of
// a rows x N array X, element (i, j) at X[i * xi + j * xj], into Y (rows x N',
// element (i, c) at Y[i * yi + c * yj]); restrict: N' = ceil(N/2), else N is
// the fine length and Y has N' = N entries per row from N_c = ceil(N/2).
hipError_t launch_xfer_cols(int restrict_op, int xfer, int64_t rows, int64_t N, const float *X,
                            int64_t xi, int64_t xj, float *Y, int64_t yi, int64_t yj,
                            const int32_t *stop, hipStream_t s);
hipError_t launch_sumsq(const float *X, int64_t ld, int64_t rows, int64_t ncols, double *parts,
                        int nparts, double *out, hipStream_t s);
hipError_t launch_check_input(const float *M, int64_t ld, int64_t m, int64_t n, int32_t *flags,
                              hipStream_t s);
hipError_t launch_state_reset(DevState *st, hipStream_t s);
// BF16 operand copies (job.h layouts).  to_bf16_cols: column-major X (rows x
// cols, stride ldx) -> column-major Y (rows_pad x cols_pad), zero padded.
// pack_bf16: the K-packed A-pass layout with cols_pad columns.
hipError_t launch_to_bf16_cols(const float *X, int64_t ldx, int64_t rows, int64_t cols,
                               uint16_t *Y, int64_t rows_pad, int64_t cols_pad, hipStream_t s);
hipError_t launch_pack_bf16(const float *X, int64_t ldx, int64_t rows, int64_t cols, uint16_t *Y,
                            int64_t cols_pad, hipStream_t s);
// pack_bf16_both (streaming levels): the K-packed copy with cols_pad columns
// and the column-panelled C-pass copy (rows_pad rows, columns padded to 16) in
// one pass over X; rows_pad and cols_pad multiples of 32.
hipError_t launch_pack_bf16_both(const float *X, int64_t ldx, int64_t rows, int64_t cols,
                                 uint16_t *Ya, int64_t cols_pad, uint16_t *Yc, int64_t rows_pad,
                                 hipStream_t s);

hipError_t launch_gram(int rpad, int r, int64_t L, const float *X, int64_t ldx, int parts,
                       int64_t chunk, double *gparts, double *Gd, float *Gf, const int32_t *stop,
                       hipStream_t s);

// Job-table sweep kernels (job.h): one launch per phase over the jobs of a
// table; block b works on tile bmap[b].y of job bmap[b].x (bmap null: job 0,
// tile b).  mode: 0 HALS, 1 MU, 2 store the product (ANLS), 3 (W tile kernel
// only) initialise: Wt and the W W^T partials from the current W, no update.
// All jobs of one launch share rpad (and tm for the A-pass).
// bf: BF16 operand copies (job.h) on v_mfma_f32_16x16x32_bf16 (HALS / MU only).
hipError_t launch_apass_jobs(int mode, int rpad, int tm, const Job *jobs, const int2 *bmap,
                             int blocks, size_t lds, hipStream_t s, bool bf = false);
hipError_t launch_cpass_jobs(int rpad, int wc, const Job *jobs, const int2 *bmap, int blocks,
                             hipStream_t s, bool bf = false);
// which = 0: V^T V from the C-pass partials; 1: W W^T and the residual log;
// 2: W W^T only.
// D = V^T V from the C-pass partials, one block per upper tile (gram_tiles).
hipError_t launch_reduce_jobs(const Job *jobs, const int2 *bmap, int blocks, hipStream_t s);
hipError_t launch_cfinal_jobs(int mode, int rpad, int cf, const Job *jobs, const int2 *bmap,
                              int blocks, size_t lds, hipStream_t s);

// Grouped setup kernels for batches (one launch over many problems).
struct XferJob {             // restrict (kind 1) or prolong (kind 2) of ncols images
    const float *X;          // source, column stride ldx
    int64_t ldx;
    float *Y;                // destination, contiguous columns
    int32_t h, w;            // fine grid
    int32_t kind, xfer;
    int64_t ncols;
    const int32_t *stop;     // skip when *stop (may be null)
};
// bmap[b] = (job, tile): tile t covers 256 output pixels (t % pt) of columns
// 16 * (t / pt) .. +15, pt = tiles per column of that job.
hipError_t launch_xfer_many(const XferJob *jobs, const int2 *bmap, int blocks, hipStream_t s);
struct NormJob {             // ||X||_F^2 in FP64 of a rows x ncols matrix
    const float *X;
    int64_t ld, rows, ncols;
    double *parts;           // nparts partial sums
    int32_t nparts;
    double *out;
};
// Two launches: partials (blocks = sum of nparts, bmap as above), then one
// block per job adds its partials in index order.
hipError_t launch_norms_many(const NormJob *jobs, const int2 *bmap, int blocks, int njobs,
                             hipStream_t s);
hipError_t launch_state_reset_many(DevState *const *states, int count, hipStream_t s);
hipError_t launch_gather_states(DevState *const *states, int count, DevState *out,
                                hipStream_t s);
size_t apass_lds_bytes(int rpad, int tm, int mode);
size_t cfinal_lds_bytes(int rpad, int mode, int cf);
int cpass_final_blocks(int64_t n);   // W-update residual partials (one per 4 columns)
int cfinal_tile_blocks(int64_t n, int cf);   // W-update blocks of cf columns
// Upper-triangle 16x16 tiles of an rpad x rpad Gram: blocks of the Gram
// reduction (D) and of the B = W W^T kernel.
inline int gram_tiles(int rpad) { return (rpad / 16) * (rpad / 16 + 1) / 2; }
// Column segments of B = W W^T per upper tile: one below n = 1024 (the blocks
// of one tile then cost less than the hand-over), else one per 256 columns, at
// most kGramSegMax.
constexpr int kGramSegMax = 8;
inline int gram_w_segments(int64_t n) {
    return n < 1024 ? 1 : (int)std::min<int64_t>(kGramSegMax, (n + 255) / 256);
}
// B = W W^T (FP64) from the current W, one block per upper tile.  with_resid:
// block 0 also assembles the residual of the iteration from the W-update
// partials, logs rel_err and sets the stop flag.
hipError_t launch_gram_w_jobs(int with_resid, const Job *jobs, const int2 *bmap, int blocks,
                              hipStream_t s);
// B from the segment partials of launch_gram_w_jobs for jobs with gseg > 1
// (one block per upper tile, blocks = nG per job; jobs with gseg = 1 return).
hipError_t launch_gram_sum_jobs(int with_resid, const Job *jobs, const int2 *bmap, int blocks,
                                hipStream_t s);
// Grids of single-problem (null block map) A-pass / C-pass launches, whose
// blocks are mapped to tiles XCD by XCD.
int apass_grid_single(int nA);
int cpass_grid_single(int nCx, int chunks);
// Streaming BF16 passes (job.stream): A-pass tiles of kStreamARows rows (nA blocks),
// C-pass tiles of 256 columns x one row chunk (XCD-ordered grid).
constexpr int64_t kStreamMinRows = 32768;
// FP32 streaming passes (job.stream with prec = 0): levels with m >= 16384,
// and, in plans whose finest level has m >= 16384, the coarser levels with
// m >= 1024 and n >= 1024 (there the regular A-pass, one block over all of n
// per row tile, is bound by its serial K loop).
constexpr int64_t kFStreamMinRows = 16384;
constexpr int64_t kFStreamWideRows = 1024, kFStreamWideCols = 1024;
constexpr int kStreamARows = 256;   // rows per block of the streaming BF16 A-pass
hipError_t launch_apass_stream(int mode, int rpad, const Job *jobs, const int2 *bmap, int blocks,
                               hipStream_t s);
hipError_t launch_cpass_stream(int rpad, const Job *jobs, const int2 *bmap, int blocks,
                               hipStream_t s);
int cpass_stream_grid(int nCx, int chunks);
// FP32 streaming passes (job.stream with prec 0): A-pass tiles of 128 rows,
// C-pass tiles of 128 columns x one row chunk.  HALS / MU.
hipError_t launch_apass_s32(int mode, int rpad, const Job *jobs, const int2 *bmap, int blocks,
                            hipStream_t s);
hipError_t launch_cpass_s32(int rpad, const Job *jobs, const int2 *bmap, int blocks,
                            hipStream_t s);
size_t apass_s32_lds_bytes(int rpad);
// Second half of a split FP32 streaming A-pass (job.aks > 1): nA blocks.
hipError_t launch_afinal_s32(int mode, int rpad, const Job *jobs, const int2 *bmap, int blocks,
                             hipStream_t s);
size_t apass_stream_lds_bytes(int rpad);
hipError_t launch_make_wt(const float *W, int64_t n, int r, int rpad, float *Wt, hipStream_t s);
// Residual from separately computed Grams (ANLS path): rel_err of
// ||M||^2 - 2 sum(rparts) + <Dd, Bd>, logged at st->log_len.
hipError_t launch_residual(const double *rparts, int nparts, const double *Dd, const double *Bd,
                           int r, const double *normM2, int depth, double *log_rel,
                           int32_t *log_depth, int log_cap, DevState *st, int32_t *hstop,
                           double tol, hipStream_t s);
hipError_t enable_large_lds();
hipError_t enable_stream_lds();   // streaming A-passes (called by enable_large_lds)

// ANLS: exact FP64 NNLS per row of V (G = W W^T, rhs = A rows) or per column
// of W (G = V^T V, rhs = C columns) by block principal pivoting, the passive
// set started from the current factor's support.  A non-positive pivot or an
// exchange that does not end sets bit 2 of *flags (the affected problem keeps
// its previous values).
hipError_t launch_nnls_rows(int rpad, const double *Gd, const double *A, int64_t m, int r,
                            float *V, int32_t *flags, const int32_t *stop, hipStream_t s);
hipError_t launch_nnls_cols(int rpad, const double *Gd, const double *C, int64_t n, int r,
                            float *W, float *Wt, double *rparts, int32_t *flags,
                            const int32_t *stop, hipStream_t s);
int nnls_cols_blocks(int64_t n);

// KL divergence (kl.hip): the kernels of one iteration and the set-up ones.
int kl_row_blocks(int64_t m);
int kl_col_blocks(int64_t n);
hipError_t launch_kl_vpass(int rpad, const float *M, int64_t ldm, int64_t m, int64_t n, int r,
                           float *V, const float *W, const float *Wt, const double *wsum,
                           const int32_t *stop, hipStream_t s);
hipError_t launch_kl_wpass(int rpad, const float *M, int64_t ldm, int64_t m, int64_t n, int r,
                           const float *V, const float *W, int chunks, int64_t chunk, double *Cp,
                           double *vparts, const int32_t *stop, hipStream_t s);
hipError_t launch_kl_wfinal(int rpad, int64_t n, int r, int chunks, const double *Cp,
                            const double *vparts, float *W, float *Wt, double *wparts, bool init,
                            const int32_t *stop, hipStream_t s);
hipError_t launch_kl_wsum(int rpad, int64_t n, const double *wparts, double *wsum,
                          const int32_t *stop, hipStream_t s);
hipError_t launch_kl_div(int rpad, const float *M, int64_t ldm, int64_t m, int64_t n, int r,
                         const float *V, const float *W, double *dparts, const int32_t *stop,
                         hipStream_t s);
hipError_t launch_kl_log(int64_t m, int64_t n, int rpad, const double *dparts,
                         const double *wparts, double *wsum, const double *msum, int depth,
                         double *log_rel, int32_t *log_depth, int log_cap, DevState *st,
                         int32_t *hstop, double tol, hipStream_t s);
hipError_t launch_msum(const float *M, int64_t ldm, int64_t m, int64_t n, double *parts,
                       int nparts, double *out, hipStream_t s);

// NTF (ntf.hip): mode updates of B and C, factor Grams, the Khatri-Rao product.
int ntf_mode_blocks(int64_t rows);
hipError_t launch_ntf_mode(int rpad, const double *Y, int64_t n, const double *D,
                           const double *Go, float *Ft, int64_t L, const float *Ot, int64_t Lo,
                           int64_t sa, int64_t sb, int r, double *rparts, const int32_t *stop,
                           hipStream_t s);
hipError_t launch_ntf_gram(const float *Ft, int64_t L, int r, double *G, const double *Hm,
                           double *H, const int32_t *stop, hipStream_t s);
hipError_t launch_ntf_kr(const float *Bt, const float *Ct, int64_t J, int64_t K, int r, int rpad,
                         float *W, float *Wt, const int32_t *stop, hipStream_t s);

}  // namespace nmf
