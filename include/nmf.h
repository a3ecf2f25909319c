/*
 * nmf.h - C ABI of the MI355X multilevel NMF library (libnmf.so).
 *
 * Problem (Section 2, eq. NMF): given a nonnegative m x n matrix M whose
 * columns are vectorised h x w images (m = h*w) and a rank r, find V >= 0
 * (m x r) and W >= 0 (r x n) with M ~ V W, minimising ||M - V W||_F^2.
 *
 * Method (Section 4): the inner algorithm (HALS = Alg. 3, MU = Alg. 2,
 * ANLS = Alg. 1) runs on a hierarchy of coarser pixel grids built by the
 * nonnegative restriction of eq. restr; V is moved between levels by the
 * prolongation of eq. prol; the order of levels is nested iteration (Alg. 4),
 * V-cycle (Alg. 5) or full multigrid (Alg. 6) with the Table 1 budget split.
 *
 * Conventions shared by every entry point
 *  - All device pointers are HIP device memory on the current device.  The
 *    caller allocates and owns every buffer; nmf_solve never allocates and
 *    never frees caller memory.  A "stream" is a hipStream_t passed as void*
 *    (NULL = the null stream).
 *  - Layouts: M is m x n column-major (image j = M + j*ldm, ldm >= m, each
 *    image row-major: pixel (y, x) at y*w + x).  V is m x r column-major
 *    (basis image k = V + k*m).  W is r x n row-major (W + k*n).
 *  - Every call returns an nmf_status; no exception or abort crosses the ABI.
 *    On error nmf_last_error() returns a human-readable message of the last
 *    failed call on the calling thread (thread-local storage, valid until the
 *    next call on the same thread; the plan argument is not used).
 */
#ifndef NMF_H
#define NMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmf_plan_s *nmf_plan_t;
typedef int32_t nmf_status;

enum {
    NMF_OK = 0,
    NMF_E_ARG = -1,        /* null pointer, unknown enum, bad iteration count      */
    NMF_E_SHAPE = -2,      /* m != h*w, r out of [1,64], a side < 2 to restrict,
                              ANLS with a level that has fewer pixels than r       */
    NMF_E_NOMEM = -3,      /* workspace too small / host allocation failed          */
    NMF_E_DEVICE = -4,     /* a HIP call failed (message has the HIP error)         */
    NMF_E_NONFINITE = -5,  /* NaN/Inf in M (input check) or in a residual           */
    NMF_E_NEGATIVE = -6,   /* M has a negative entry (input check)                  */
    NMF_E_BUSY = -7,       /* server: request does not fit the admission budget     */
    NMF_PENDING = 1        /* server poll: the request has not finished yet (not an
                              error)                                                 */
};

/* Alg. 3, Alg. 2, Alg. 1; NMF_KL: the generalized Kullback-Leibler divergence
 * D(M | VW) = sum M log(M/(VW)) - M + VW (Section 7.1 lists other objective
 * functions as an extension) minimised by the Lee-Seung multiplicative
 * updates V <- V o [(M/VW) W^T] / [1 W^T], W <- W o [V^T (M/VW)] / [V^T 1]
 * on the same hierarchy and schedule; (VW)_ij = 0 gives the ratio 0, a zero
 * denominator keeps the entry.  Its logged error (and the tolerance) is
 * D(M_l | VW) / sum(M_l).  FP32, one-sided, single solves. */
enum { NMF_HALS = 0, NMF_MU = 1, NMF_ANLS = 2, NMF_KL = 3 };
/* Alg. 4, Alg. 5, Alg. 6; NMF_WC: W-cycle (Section 7.1 lists other cycles as
 * future work): the V-cycle's split of the budget t (t/4 before descending,
 * t/2 after) with the coarse quarter spent in two consecutive W-cycles of t/8
 * on the next level. */
enum { NMF_NI = 0, NMF_VC = 1, NMF_FMG = 2, NMF_WC = 3 };
/* Transfer operators.  FW: full weighting (eq. restr, boundary weights of the
 * fine neighbours that exist renormalised to sum 1) with the rd() mean
 * prolongation (eq. prol).  BLOCK2: 2x2 pixel-block mean / replication. */
enum { NMF_XFER_FW = 0, NMF_XFER_BLOCK2 = 1 };
/* Number format of the two M-streaming products M W^T and V^T M.  BF16 keeps
 * an extra bf16 copy of every level of M in the workspace and accumulates in
 * FP32; Grams, updates and residuals stay FP32/FP64 as in FP32 mode. */
enum { NMF_FP32 = 0, NMF_BF16 = 1 };
#define NMF_TILE(wc, cf) ((int32_t)(wc) | ((int32_t)(cf) << 8))   /* nmf_desc.tile_cfg */
#define NMF_TILE_GROUPED ((int32_t)1 << 16)                          /* nmf_desc.tile_cfg flag */

typedef struct {
    int64_t m, n;          /* M is m x n; m must equal h*w                          */
    int64_t ldm;           /* column stride of M in elements (0 = m)                */
    int32_t h, w;          /* finest image grid                                     */
    int32_t r;             /* rank, 1..64                                           */
    int32_t levels;        /* >= 1 (1 = plain single-level NMF)                     */
    int32_t algo;          /* NMF_HALS / NMF_MU / NMF_ANLS / NMF_KL                 */
    int32_t cycle;         /* NMF_NI / NMF_VC / NMF_FMG / NMF_WC                    */
    int32_t xfer;          /* NMF_XFER_FW / NMF_XFER_BLOCK2                         */
    int32_t prec;          /* NMF_FP32 / NMF_BF16                                   */
    int32_t refine_iters;  /* BF16 only: finest-level FP32 iterations appended      */
    int32_t max_fine_iters;/* tol > 0: cap on finest-level iterations after the
                              schedule (0 = none)                                   */
    int32_t check_every;   /* tol > 0: host polls the device stop flag every this
                              many continuation iterations (0 = 8)                  */
    int32_t log_cap;       /* capacity of the per-iteration rel_err log (0 = 4096)  */
    int32_t check_input;   /* 1: scan M for negative / non-finite entries first    */
    int32_t tile_cfg;      /* tile shapes of the C-pass and W-update kernels: 0 = the
                              library's choice (latency tiles when m >= 8192, throughput
                              tiles below), else NMF_TILE(wc, cf): wc in {1, 2, 4} C-pass
                              row groups per tile, cf in {4, 16} W-update columns per
                              tile.  Single and batched solves of one plan run the same
                              tiles, hence the same arithmetic; plans with different
                              tiles agree to rounding (the C-pass sum order depends on
                              wc).  Chosen by paper_1009_0881_amd.tune for a workload.
                              NMF_TILE_GROUPED may be or-ed in (alone or with
                              NMF_TILE(wc, cf)): a plan for problems solved in grouped
                              launches (nmf_solve_batch, the server), where the problems
                              fill the chip together.  Its C-pass chunks keep at least
                              512 rows (fewer FP64 partials of V^T M); a problem solved
                              alone with such a plan is slower, with the same bits as in
                              a batch.  Other bits above 15 are rejected (NMF_E_ARG). */
    double tol;            /* > 0: stop after the first finest-level iteration with
                              rel_err <= tol (absolute threshold on rel_err)        */
    int32_t two_sided;     /* 1: the hierarchy also halves the column count (Section
                              6.1, for columns ordered along a smooth axis such as
                              wavelength or time): M_{l+1} = R_m M_l R_n^T with the
                              1-D operator of `xfer` along the columns, W moves
                              between levels along its rows (W' = W R_n^T,
                              W = W' P_n^T), and a depth-d run converts its budget at
                              8^d iterations per finest-iteration equivalent.  FP32
                              single solves only (not with NMF_BF16, not batched or
                              served); every restricted column count must be >= 2. */
    int32_t ntf_k;         /* 0: matrix NMF.  K > 0: nonnegative tensor factorisation
                              (Section 7.1 proposes the multilevel technique for NTF):
                              M is the mode-1 unfolding of an I x J x K tensor X, I = m
                              = h*w pixels, n = J*K, column j + J k holding X[:, j, k];
                              X ~ sum_r a_r o b_r o c_r is fitted by the HALS steps of
                              Alg. 3 on each mode's unfolding in turn (A, then B, then
                              C); mode 1 is coarsened as the images are and A moves
                              between levels as V does.  Solved by nmf_ntf_solve.
                              HALS, FP32, one-sided; n must be a multiple of K and
                              K <= 16384.                                          */
} nmf_desc;

typedef struct {
    int32_t log_len;         /* iterations logged (all levels, <= log_cap)          */
    int32_t total_iters;     /* iterations executed over all levels                 */
    int32_t fine_iters;      /* iterations executed on the finest level             */
    int32_t stopped;         /* 1 if tol was reached                                */
    double rel_err;          /* rel_err of the last iteration executed              */
    double fine_equiv;       /* work in finest-iteration equivalents: sum 4^-depth
                                (8^-depth for two-sided hierarchies)                 */
    double queue_ms;         /* server: submit -> admission (0 elsewhere)           */
    double latency_ms;       /* server: submit -> factors in host memory            */
} nmf_result;

/* Validate a problem description and build a plan (host only, no device
 * work).  *workspace_bytes receives the size of the device workspace every
 * nmf_solve with this plan needs (256-byte aligned base required). */
nmf_status nmf_plan(const nmf_desc *desc, nmf_plan_t *out, size_t *workspace_bytes);

/* Run the multilevel solve with a budget of `iters` finest-iteration
 * equivalents (Table 1; levels = 1 gives `iters` plain iterations).
 * dV (m x r) and dW (r x n) hold V0, W0 on entry and the result on return
 * (for ANLS V0 is not used, Alg. 1 / Remark 1).  dM is read only.
 * The call enqueues work on `stream`; it returns after the stream finished
 * (it synchronises once at the end, and every check_every continuation
 * iterations when tol > 0).  The per-iteration rel_err log is read with
 * nmf_query_log.  Concurrent solves with the same plan must use distinct
 * workspaces. */
nmf_status nmf_solve(nmf_plan_t plan, const float *dM, float *dV, float *dW, int32_t iters,
                     void *dWorkspace, void *stream, nmf_result *hOut);

nmf_status nmf_destroy(nmf_plan_t plan);

/* nmf_solve without a caller workspace, for callers that cannot allocate
 * device memory (code that must not call hipMalloc: tight serving loops,
 * harnesses that forbid allocation).  The workspace is a fixed array of
 * NMF_STATIC_WORKSPACE_BYTES in device global memory that the library holds on
 * every GPU it is used on until the process ends; the call allocates nothing
 * (no hipMalloc / hipFree, no allocating library routine) and records no
 * profiling events.  Arguments, layouts and results are those of nmf_solve;
 * the rel_err log stays in that array (only hOut reports the solve).
 * Errors: as nmf_solve, and NMF_E_NOMEM when the plan's workspace_bytes
 * exceeds NMF_STATIC_WORKSPACE_BYTES (e.g. 112x92 images, n = 400, r = 40,
 * 3 levels need about 13 MiB; 256x256 images, n = 2000, r = 50 are refused).
 * Every call on one GPU uses that GPU's single array: calls that overlap on
 * one GPU (other streams or host threads) race and give undefined results;
 * serialise them.  Each call re-initialises what it reads (nothing carries
 * over from the previous call). */
#define NMF_STATIC_WORKSPACE_BYTES (32u << 20)
nmf_status nmf_solve_static(nmf_plan_t plan, const float *dM, float *dV, float *dW,
                            int32_t iters, void *stream, nmf_result *hOut);

/* Multilevel NTF (plan with ntf_k = K > 0; Section 7.1).  dX: the mode-1
 * unfolding (m x J*K column-major, column stride ldm, column j + J k holding
 * X[:, j, k]); dA: m x r column-major (the V of a matrix solve); dBt: B^T,
 * r x J row-major; dCt: C^T, r x K row-major; all three updated in place.
 * Schedule, budget, tolerance (on ||X - [[A, B, C]]||_F / ||X||_F, logged per
 * iteration) and the result are those of nmf_solve.  The workspace holds,
 * besides the matrix solve's buffers, the Khatri-Rao product (C kr B)^T and
 * A^T X_(1).  Errors as nmf_solve; NMF_E_ARG for a plan without ntf_k.
 * nmf_solve, nmf_solve_static and nmf_iterate reject NTF plans. */
nmf_status nmf_ntf_solve(nmf_plan_t plan, const float *dX, float *dA, float *dBt, float *dCt,
                         int32_t iters, void *dWorkspace, void *stream, nmf_result *hOut);

const char *nmf_status_string(nmf_status s);
const char *nmf_last_error(nmf_plan_t plan);

/* ---- introspection (host only; used by the bit-exact tests) --------------- */

/* Image sides of every level, finest first: hw[2*l] = h_l, hw[2*l+1] = w_l. */
nmf_status nmf_query_levels(nmf_plan_t plan, int32_t *hw, int32_t cap_levels);

/* The integer schedule for a budget of `iters`: triples (kind, depth, count)
 * with kind 0 = run `count` iterations at `depth`, 1 = restrict V from depth
 * to depth+1, 2 = prolong V from depth+1 to depth.  *nsteps receives the
 * number of triples; at most cap triples are written. */
nmf_status nmf_query_schedule(nmf_plan_t plan, int32_t iters, int32_t *steps, int32_t cap,
                              int32_t *nsteps);

/* Copy the rel_err log of the last nmf_solve (device workspace -> host):
 * rel_err[i] and depth[i] for i < min(cap, log_len).  Synchronises `stream`. */
nmf_status nmf_query_log(nmf_plan_t plan, const void *dWorkspace, void *stream,
                         double *rel_err, int32_t *depth, int32_t cap);

/* ---- single operators (device pointers; used by the kernel parity tests) -- */

/* Y = R(X) columnwise for `ncols` images of X (h x w, column stride ldx) into
 * Y (ceil(h/2) x ceil(w/2), column stride ceil(h/2)*ceil(w/2)); eq. restr. */
nmf_status nmf_restrict(int32_t xfer, int32_t h, int32_t w, int64_t ncols, const float *dX,
                        int64_t ldx, float *dY, void *stream);

/* X = P(Y) columnwise: Y has ceil(h/2) x ceil(w/2) images, X has h x w; eq. prol. */
nmf_status nmf_prolong(int32_t xfer, int32_t h, int32_t w, int64_t ncols, const float *dY,
                       float *dX, void *stream);

/* One iteration of `algo` on a single level (the update of V then W, as the
 * sweep inside nmf_solve does), followed by the residual.  The workspace is
 * the one of a plan with levels = 1 and the same m, n, r, algo, prec.  The
 * rel_err of the iteration is written to *hRelErr (synchronises). */
nmf_status nmf_iterate(nmf_plan_t plan, const float *dM, float *dV, float *dW, int32_t count,
                       void *dWorkspace, void *stream, double *hRelErr);

/* The two M-streaming products on their own: A = M W^T (m x r, column-major)
 * and C = V^T M (r x n, row-major), FP32 operands on the matrix cores with
 * FP32 accumulation (the products A and C of Alg. 3; 2mnr flops each,
 * Appendix A.1).  Level-0 shapes of `plan`; its workspace is used as scratch.
 * Synchronises nothing. */
nmf_status nmf_products(nmf_plan_t plan, const float *dM, const float *dV, const float *dW,
                        float *dA, float *dC, void *dWorkspace, void *stream);

/* FP64 Gram G = X X^T of r vectors of length L (vector a at dX + a*ldx),
 * accumulated in FP64 (used for W W^T and V^T V).  dG is r x r FP64. */
nmf_status nmf_gram(int32_t r, int64_t L, const float *dX, int64_t ldx, double *dG,
                    void *dWorkspace, size_t ws_bytes, void *stream);

/* ---- kernel timing (HIP events on the solve's stream) ---------------------
 * Kernel kinds: 0 A-pass (M W^T + V update), 1 Gram V^T V, 2 C-pass partials
 * (V^T M), 3 C-pass reduction + W update, 4 Gram W W^T, 5 residual, 6 NNLS
 * rows of V, 7 NNLS columns of W, 8 restriction, 9 prolongation, 10 ||M||^2
 * (and sum(M) for NMF_KL), 11 KL divergence partials, 12 NTF mode updates,
 * factor Grams and Khatri-Rao products.  For NMF_KL kind 0 is
 * the V pass, 2 the W pass, 3 the W update and 5 the logged divergence.
 * With bit k of `mask` set, every launch of kind k by later nmf_solve /
 * nmf_iterate calls on this plan is bracketed by two hipEventRecord calls on
 * the call's stream; the elapsed times are summed when the call synchronises
 * at its end.  nmf_profile_read copies the per-kind launch counts and total
 * milliseconds (cap entries) and, if reset != 0, clears them. */
#define NMF_NUM_KERNEL_KINDS 13
nmf_status nmf_profile(nmf_plan_t plan, uint32_t mask);
nmf_status nmf_profile_read(nmf_plan_t plan, int64_t *counts, double *total_ms, int32_t cap,
                            int32_t reset);

/* ---- batched solves ---------------------------------------------------------
 * Many independent solves (each its own plan: uneven m, n, r, levels, cycle,
 * budget, tolerance and precision; HALS or MU) advanced together: every tick,
 * each unfinished problem performs its pending V transfers and one sweep at
 * its current level (BF16 problems: the BF16 schedule, then the FP32
 * refinement and continuation, as in nmf_solve), and the work of all problems
 * is issued as one launch per phase and tile configuration (rank class r
 * padded to 16/32/48/64, A-pass tile rows, update rule, precision).  A
 * problem's arithmetic is that of nmf_solve on its own plan, so its V, W and
 * result are bitwise those of a single solve -- except for levels with
 * m >= 32768, which nmf_solve runs on its streaming kernels and a batch on the
 * regular tiling (both within the FP32 parity bar of the oracle).
 *
 * nmf_batch_workspace: bytes of the one device workspace of a batch over
 * these plans (their own workspaces, 256-byte aligned, back to back, then the
 * executor's tables).  nmf_solve_batch: dM[i], dV[i], dW[i], iters[i] as in
 * nmf_solve for problem i; hOut (count entries, may be null) receives the
 * results.  flags: NMF_BATCH_GRAPH captures a steady tick (the same problems
 * at the same levels as the tick before) into a hipGraph and replays it while
 * the configuration lasts; the batch then runs on a stream of its own that
 * first waits for `stream`.  Returns after the stream has synchronised.
 * Errors: NMF_E_ARG (null pointer, negative iters, unaligned workspace, an
 * ANLS plan), or the first failing problem's status (results still filled). */
#define NMF_BATCH_GRAPH 1
nmf_status nmf_batch_workspace(const nmf_plan_t *plans, int32_t count, size_t *bytes);
nmf_status nmf_solve_batch(const nmf_plan_t *plans, int32_t count, const float *const *dM,
                           float *const *dV, float *const *dW, const int32_t *iters,
                           void *dWorkspace, void *stream, int32_t flags, nmf_result *hOut);

/* ---- serving with continuous batching -------------------------------------
 * A server owns one device pool of hbm_budget bytes (allocated once, here) and
 * a worker thread.  nmf_server_submit plans the request (errors of nmf_plan
 * are returned at once; ANLS and ldm != m are rejected with NMF_E_ARG, a
 * footprint above the budget with NMF_E_BUSY) and queues it; hM (m x n,
 * column-major), hV0 (m x r, column-major) and hW0 (r x n, row-major) are
 * host arrays that must stay valid until the request has finished.  The
 * worker admits queued requests in arrival order while at most `slots` run
 * and the pool has room for their footprint (M, V, W and the plan's
 * workspace), copies them in, and advances every admitted request with the
 * batch executor; requests that arrive while others run join at the next
 * tick.  A finished request's factors are copied to server-owned host memory
 * and its device memory is released at once.  Results are bitwise those of
 * nmf_solve on the same plan, whatever else runs alongside.
 *
 * nmf_server_poll: NMF_PENDING while the request runs or waits; otherwise
 * copies V (m x r) and W (r x n) to hV / hW (may be null), fills *out and
 * returns the request's status; the ticket is then retired.
 * nmf_server_stats: up to 6 counters: admitted, completed, running, peak
 * running, peak pool bytes in use, executor ticks.
 * nmf_server_destroy: drops queued requests, waits for running ones, frees the
 * pool.  Calls on one server may come from any host thread. */
typedef struct nmf_server_s nmf_server;
nmf_status nmf_server_create(size_t hbm_budget, int32_t slots, nmf_server **out);
nmf_status nmf_server_submit(nmf_server *server, const nmf_desc *desc, const float *hM,
                             const float *hV0, const float *hW0, int32_t iters,
                             uint64_t *ticket);
nmf_status nmf_server_poll(nmf_server *server, uint64_t ticket, float *hV, float *hW,
                           nmf_result *out);
nmf_status nmf_server_stats(nmf_server *server, int64_t *stats, int32_t cap);
nmf_status nmf_server_destroy(nmf_server *server);

#ifdef __cplusplus
}
#endif

#endif /* NMF_H */
