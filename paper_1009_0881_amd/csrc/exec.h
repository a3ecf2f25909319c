// Host executor internals shared by the single-solve entry points and the
// batch / serving executor: per-solve device pointers, error and profiling
// helpers, and the building blocks of a solve (level preparation, one sweep).
#pragma once

#include <string>
#include <vector>

#include "nmf_internal.h"

struct nmf_plan_s {
    nmf::Plan p;
};

namespace nmf {

nmf_status fail(nmf_plan_t plan, nmf_status st, const std::string &msg);

#define NMF_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(plan, NMF_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Pointers into one workspace, for one solve.
struct Ctx {
    nmf_plan_t plan;
    const Plan *p;
    hipStream_t s;
    char *ws;
    DevState *st;
    const int32_t *stop;
    double *log_rel;
    int32_t *log_depth;
    double *norm;
    double *nparts;               // norm partials, kNormParts per level
    double *Bd, *Dd, *gparts, *rparts;
    float *Bf, *Df, *Wt;
    double *A, *C;                // ANLS: FP64 products M W^T and V^T M
    double *Cp, *Dp;
    double *Cr;                   // V^T M summed over the chunks (null: KL plans)
    double *bparts;               // partial tiles of B = W W^T (segmented launches)
    // NMF_KL: row sums of W and their block partials, column sums of V per
    // chunk, divergence partials, sum(M_l) per level (null otherwise)
    double *klw = nullptr, *klwp = nullptr, *klvp = nullptr, *kld = nullptr, *klm = nullptr;
    // NTF: B^T (r x J) and C^T (r x K) of the caller and the Grams B^T B,
    // C^T C (their Hadamard product, the mode-1 Gram, lives in Bd; null otherwise)
    float *ntfB = nullptr, *ntfC = nullptr;
    double *ntfGB = nullptr, *ntfGC = nullptr;
    std::vector<const float *> M;
    std::vector<int64_t> ldm;
    std::vector<float *> V;
    std::vector<float *> Wl;      // W of every level (all dW unless two-sided)
    float *W;
    Job *djobs;                   // device copy of `jobs` (workspace)
    std::vector<Job> jobs;        // one job per level, then the FP32 finest-level job
    std::vector<int8_t> depths;   // depth of every executed iteration (host mirror)
    bool prof = true;             // time launches of the kinds in the plan's profile mask
    struct ProfEvent {
        int kind;
        hipEvent_t begin, end;
    };
    std::vector<ProfEvent> prof_pending;   // event pairs recorded by this solve
};

// allow_stream: jobs of large levels may use the streaming kernels (single
// solves); grouped batch launches use the regular tiling.
Ctx make_ctx(nmf_plan_t plan, const float *dM, float *dV, float *dW, void *dws, hipStream_t s,
             bool allow_stream = true);
// BF16 mode: the BF16 operand copies of every level (and padding of the V
// and W copies); nothing in FP32 mode.
nmf_status prepare_bf16(Ctx &c);
// The whole multilevel solve of nmf_solve on a workspace at dWorkspace (256-byte
// aligned, plan->p.ws.total bytes); arguments already validated.  profile:
// honour the plan's profile mask (HIP events); false records no event.
// lookahead: tolerance checks through a host-mapped stop flag with one batch
// of iterations kept queued (pinned host memory and events from the plan's
// pools); false: synchronous checks, nothing allocated.
// NTF plans: dW is ignored (the Khatri-Rao product in the workspace serves as
// W) and dB, dC are B^T and C^T; nullptr for matrix plans.
nmf_status solve_on(nmf_plan_t plan, const float *dM, float *dV, float *dW, int32_t iters,
                    void *dWorkspace, hipStream_t s, nmf_result *hOut, bool profile,
                    bool lookahead, float *dB = nullptr, float *dC = nullptr);
// Fill an nmf_result from the final device state and the host depth log.
nmf_status result_from_state(nmf_plan_t plan, const DevState &hs,
                             const std::vector<int8_t> &depths, nmf_result *out);

}  // namespace nmf
