// Batch / serving executor (batch.cpp): many independent solves advanced in
// lock-step ticks with one grouped launch per phase.
#pragma once

#include <map>
#include <tuple>
#include <vector>

#include "exec.h"

namespace nmf {

// Device area of an executor, after the problems' own workspaces.
struct BatchArea {
    size_t off_stptr;    // DevState* of every slot (for the state gather)
    size_t off_gather;   // gathered DevState copies
    size_t off_arena;    // job tables and block maps, bump-allocated
    size_t arena_cap;
    size_t end;
};

size_t batch_table_bytes(const nmf_plan_t *plans, int count);
BatchArea batch_area_layout(size_t base, int capacity, size_t table_bytes);

class Executor {
public:
    Executor(char *base, const BatchArea &area, int capacity, hipStream_t s, bool graphs);
    ~Executor();
    Executor(const Executor &) = delete;
    Executor &operator=(const Executor &) = delete;

    // Queue a problem (schedule budget `iters`) with its own workspace `dws`;
    // it starts on the next tick.  `id` is the caller's handle.
    nmf_status add(nmf_plan_t plan, const float *dM, float *dV, float *dW, int32_t iters,
                   void *dws, int id);
    // One unit of work for every active problem.
    nmf_status tick();
    nmf_status poll();
    bool all_done() const;
    bool any_done() const;
    bool empty() const { return insts_.empty(); }
    // Results of the finished problems (all problems when only_done is false).
    nmf_status results(std::vector<int> &ids, std::vector<nmf_result> &res,
                       std::vector<nmf_status> &status, bool only_done);
    void remove(int id);
    int64_t ticks() const { return ticks_; }

private:
    struct Inst {
        int id = 0;
        nmf_plan_t plan = nullptr;
        Ctx c;
        std::vector<Step> sched;
        size_t cur = 0;
        int left = -1;        // iterations left in the run step at `cur`
        int stage = 0;        // 0 schedule, 3 FP32 refinement (BF16 mode), 1 fine
                              // iterations after the schedule, 2 done
        int cont_left = 0;
        int since_check = 0;
        int depth = 0;
        int mode = 0;         // 0 HALS, 1 MU
        bool use_tol = false;
        bool bf16 = false;    // BF16 schedule, then FP32 refinement / continuation
        int refine_left = 0;  // stage 3: FP32 refinement iterations left
        bool fp32job = false; // this tick's sweep uses the FP32 finest-level job
    };
    struct G {
        int rpad, tm, mode, wc, cf;
        bool bf;
        const Job *dj;
        const int2 *bA, *bC, *bG, *bF, *bW;   // bW: B = W W^T blocks (nG * gseg per job)
        int nA, nC, nG, nF, nW;
        bool seg;             // some job has gseg > 1: B partials summed by k_gram_sum
    };

    template <class T>
    nmf_status upload(const std::vector<T> &v, const T **out);
    nmf_status sync_reset();
    nmf_status setup_fresh();
    void advance(Inst &I, std::vector<Step> &xfers);
    nmf_status launch_xfers(std::vector<std::pair<Inst *, std::vector<Step>>> &todo);
    nmf_status launch_sweeps(const std::vector<Inst *> &active, bool capture_ok);
    nmf_status gather(std::vector<DevState> &hs);
    int slot_of(int id) const;
    void drop_graph();
    // Look-ahead tolerance checks: at a check the executor queues a gather of
    // the live problems' states into pinned host memory and then waits only
    // for the previous check's gather (issued check_every ticks earlier), so
    // the stream never drains; problems learn of their stop one check late,
    // and the ticks issued meanwhile return at once on the device stop flag.
    struct PendingPoll {
        DevState *h = nullptr;        // pinned host copy of the gathered states
        hipEvent_t ev = nullptr;
        std::vector<int> ids;         // problem ids, in gather order
        std::vector<DevState *> sts;  // their state pointers (the upload source)
        bool live = false;
    };
    nmf_status poll_issue(PendingPoll &pp);
    nmf_status poll_finish(PendingPoll &pp);

    char *base_;
    BatchArea area_;
    int capacity_;
    hipStream_t s_;
    bool use_graph_;
    DevState **dstptr_;
    DevState *dgather_;
    char *arena_;
    size_t arena_off_ = 0;
    int64_t generation_ = 0;
    int64_t ticks_ = 0;
    std::vector<std::vector<char>> staged_;
    std::map<std::vector<int64_t>, G> cache_;
    std::vector<Inst> insts_;
    std::vector<int> fresh_;
    std::vector<int64_t> last_key_, graph_key_;
    hipGraphExec_t gexec_ = nullptr;
    int stable_ticks_ = 0;
    PendingPoll polls_[2];
    int poll_next_ = 0;
};

}  // namespace nmf
