// Batch executor: many independent multilevel solves advanced together on one
// stream.  Every tick, each active problem performs one unit of its own
// schedule (Alg. 4-6 with the Table 1 budgets): its pending V transfers, then
// one sweep at its current level.  Work of all problems is grouped into one
// launch per phase and tile configuration (rank class, A-pass tile rows,
// update rule), over a job table and a block map built on the host.  The
// arithmetic per problem is exactly that of a single solve, so a problem's
// result does not depend on what else is in the batch.
#include <algorithm>
#include <cstring>
#include <map>

#include "batch.h"

namespace nmf {

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tiles of a grouped transfer: 256 output pixels x 16 columns each.
int64_t xfer_tiles(int64_t mout, int64_t ncols) { return cdiv(mout, 256) * cdiv(ncols, 16); }

}  // namespace

size_t batch_table_bytes(const nmf_plan_t *plans, int count) {
    // Upper bound of the device tables one tick (or one setup phase) uploads.
    size_t jobs = 0, blocks = 0, xfers = 0, norms = 0;
    for (int i = 0; i < count; ++i) {
        const Plan &p = plans[i]->p;
        const int64_t n = p.d.n, r = p.d.r;
        const LevelInfo &l0 = p.lv[0];
        const int64_t tm = l0.atm;
        const int64_t nCx = cdiv(n, 64);
        blocks += cdiv(l0.m, tm) + nCx * l0.cp_chunks + gram_tiles(p.rpad) * (1 + l0.gseg) +
                  cpass_final_blocks(n);
        int64_t xt = 0;
        for (size_t l = 1; l < p.lv.size(); ++l)
            xt = std::max<int64_t>(xt, xfer_tiles(p.lv[l].m, n) + xfer_tiles(p.lv[l - 1].m, r));
        blocks += xt + (int64_t)kNormParts * p.lv.size();
        jobs += 1;
        xfers += 1;
        norms += p.lv.size();
    }
    return align256(jobs * sizeof(Job)) + align256(xfers * sizeof(XferJob)) +
           align256(norms * sizeof(NormJob)) + align256(blocks * sizeof(int2)) * 2 + 4096;
}

BatchArea batch_area_layout(size_t base, int capacity, size_t table_bytes) {
    BatchArea a;
    a.off_stptr = base;
    a.off_gather = align256(a.off_stptr + sizeof(DevState *) * capacity);
    a.off_arena = align256(a.off_gather + sizeof(DevState) * capacity);
    a.arena_cap = align256(4 * table_bytes + (1 << 20));
    a.end = a.off_arena + a.arena_cap;
    return a;
}

Executor::Executor(char *base, const BatchArea &area, int capacity, hipStream_t s, bool graphs)
    : base_(base), area_(area), capacity_(capacity), s_(s), use_graph_(graphs) {
    dstptr_ = reinterpret_cast<DevState **>(base + area.off_stptr);
    dgather_ = reinterpret_cast<DevState *>(base + area.off_gather);
    arena_ = base + area.off_arena;
}

Executor::~Executor() {
    // the captured tick or a look-ahead gather may still run
    if (gexec_ || polls_[0].live || polls_[1].live) (void)hipStreamSynchronize(s_);
    drop_graph();
    for (PendingPoll &pp : polls_) {
        if (pp.ev) (void)hipEventDestroy(pp.ev);
        if (pp.h) (void)hipHostFree(pp.h);
    }
}

void Executor::drop_graph() {
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
    graph_key_.clear();
    stable_ticks_ = 0;
}

nmf_status Executor::sync_reset() {
    nmf_plan_t plan = nullptr;
    NMF_HIP(hipStreamSynchronize(s_));
    arena_off_ = 0;
    ++generation_;
    staged_.clear();
    cache_.clear();
    drop_graph();
    return NMF_OK;
}

template <class T>
nmf_status Executor::upload(const std::vector<T> &v, const T **out) {
    nmf_plan_t plan = nullptr;
    const size_t bytes = align256(sizeof(T) * std::max<size_t>(v.size(), 1));
    if (bytes > area_.arena_cap) return fail(nullptr, NMF_E_NOMEM, "batch table exceeds the arena");
    if (arena_off_ + bytes > area_.arena_cap) {
        nmf_status st = sync_reset();
        if (st != NMF_OK) return st;
    }
    char *dst = arena_ + arena_off_;
    arena_off_ += bytes;
    // The host copy stays alive until the next synchronisation of the stream.
    staged_.emplace_back(reinterpret_cast<const char *>(v.data()),
                         reinterpret_cast<const char *>(v.data()) + sizeof(T) * v.size());
    if (!v.empty())
        NMF_HIP(hipMemcpyAsync(dst, staged_.back().data(), sizeof(T) * v.size(),
                               hipMemcpyHostToDevice, s_));
    *out = reinterpret_cast<const T *>(dst);
    return NMF_OK;
}

int Executor::slot_of(int id) const {
    for (size_t i = 0; i < insts_.size(); ++i)
        if (insts_[i].id == id) return (int)i;
    return -1;
}

nmf_status Executor::add(nmf_plan_t plan, const float *dM, float *dV, float *dW, int32_t iters,
                         void *dws, int id) {
    const Plan &p = plan->p;
    if (p.d.algo == NMF_ANLS || p.d.algo == NMF_KL)
        return fail(plan, NMF_E_ARG,
                    "batched solves support HALS and MU (ANLS, KL: use nmf_solve)");
    if (p.d.two_sided)
        return fail(plan, NMF_E_ARG, "two-sided hierarchies run as single solves (nmf_solve)");
    if (p.d.ntf_k > 0)
        return fail(plan, NMF_E_ARG, "NTF plans run as single solves (nmf_ntf_solve)");
    if ((int)insts_.size() >= capacity_) return fail(plan, NMF_E_BUSY, "batch capacity reached");
    Inst I;
    I.id = id;
    I.plan = plan;
    I.c = make_ctx(plan, dM, dV, dW, dws, s_, false);
    I.sched = make_schedule(p.d.cycle, p.d.levels, iters);
    I.use_tol = p.d.tol > 0.0;
    I.mode = p.d.algo == NMF_HALS ? 0 : 1;
    I.bf16 = p.d.prec == NMF_BF16;
    insts_.push_back(std::move(I));
    fresh_.push_back(id);
    return NMF_OK;
}

// Grouped start of every problem added since the last call: state reset,
// restriction of M to every level, ||M_l||^2, Wt and B = W W^T.
nmf_status Executor::setup_fresh() {
    nmf_plan_t plan = nullptr;
    if (fresh_.empty()) return NMF_OK;
    std::vector<Inst *> F;
    for (int id : fresh_) F.push_back(&insts_[slot_of(id)]);
    fresh_.clear();
    nmf_status st;
    // job tables (one per level) of each problem, in its own workspace
    for (Inst *I : F) {
        NMF_HIP(hipMemcpyAsync(I->c.djobs, I->c.jobs.data(), sizeof(Job) * I->c.jobs.size(),
                               hipMemcpyHostToDevice, s_));
    }
    {
        std::vector<DevState *> sts;
        for (Inst *I : F) sts.push_back(I->c.st);
        DevState *const *d;
        if ((st = upload(sts, &d)) != NMF_OK) return st;
        NMF_HIP(launch_state_reset_many(d, (int)sts.size(), s_));
    }
    // M_l = R(M_{l-1}), one grouped launch per level
    int maxL = 0;
    for (Inst *I : F) maxL = std::max<int>(maxL, (int)I->c.p->lv.size());
    for (int l = 1; l < maxL; ++l) {
        std::vector<XferJob> xj;
        std::vector<int2> bm;
        for (Inst *I : F) {
            const Plan &p = *I->c.p;
            if ((int)p.lv.size() <= l) continue;
            XferJob x{};
            x.X = I->c.M[l - 1];
            x.ldx = I->c.ldm[l - 1];
            x.Y = const_cast<float *>(I->c.M[l]);
            x.h = p.lv[l - 1].h;
            x.w = p.lv[l - 1].w;
            x.kind = 1;
            x.xfer = p.d.xfer;
            x.ncols = p.d.n;
            x.stop = nullptr;
            const int64_t t = xfer_tiles(p.lv[l].m, p.d.n);
            for (int64_t k = 0; k < t; ++k) bm.push_back(make_int2((int)xj.size(), (int)k));
            xj.push_back(x);
        }
        const XferJob *dx;
        const int2 *db;
        if ((st = upload(xj, &dx)) != NMF_OK || (st = upload(bm, &db)) != NMF_OK) return st;
        NMF_HIP(launch_xfer_many(dx, db, (int)bm.size(), s_));
    }
    {
        std::vector<NormJob> nj;
        std::vector<int2> bm;
        for (Inst *I : F) {
            const Plan &p = *I->c.p;
            for (size_t l = 0; l < p.lv.size(); ++l) {
                NormJob q{};
                q.X = I->c.M[l];
                q.ld = I->c.ldm[l];
                q.rows = p.lv[l].m;
                q.ncols = p.d.n;
                q.nparts = norm_parts(p.lv[l].m, p.d.n);
                q.parts = I->c.nparts + l * kNormParts;
                q.out = I->c.norm + l;
                for (int k = 0; k < q.nparts; ++k) bm.push_back(make_int2((int)nj.size(), k));
                nj.push_back(q);
            }
        }
        const NormJob *dn;
        const int2 *db;
        if ((st = upload(nj, &dn)) != NMF_OK || (st = upload(bm, &db)) != NMF_OK) return st;
        NMF_HIP(launch_norms_many(dn, db, (int)bm.size(), (int)nj.size(), s_));
    }
    // BF16 problems: operand copies of every level (per problem)
    for (Inst *I : F)
        if (I->bf16 && (st = prepare_bf16(I->c)) != NMF_OK) return st;
    // Wt and B = W W^T: W tile kernel in init mode, then the B-only reduce,
    // grouped by rank class
    std::map<std::pair<int, int>, std::vector<Inst *>> by_rpad;
    for (Inst *I : F) by_rpad[{I->c.p->rpad, I->c.p->cf}].push_back(I);
    for (auto &kv : by_rpad) {
        const int rpad = kv.first.first, cf = kv.first.second;
        std::vector<Job> jobs;
        std::vector<int2> bF, bG;
        for (Inst *I : kv.second) {
            const Job &J = I->c.jobs[0];
            for (int k = 0; k < J.nFb; ++k) bF.push_back(make_int2((int)jobs.size(), k));
            for (int k = 0; k < J.nG * J.gseg; ++k) bG.push_back(make_int2((int)jobs.size(), k));
            jobs.push_back(J);
        }
        std::vector<int2> bT;   // one block per upper tile (k_gram_sum)
        bool seg = false;
        for (size_t j = 0; j < jobs.size(); ++j) {
            for (int k = 0; k < jobs[j].nG; ++k) bT.push_back(make_int2((int)j, k));
            seg = seg || jobs[j].gseg > 1;
        }
        const Job *dj;
        const int2 *dF, *dG, *dT;
        if ((st = upload(jobs, &dj)) != NMF_OK || (st = upload(bF, &dF)) != NMF_OK ||
            (st = upload(bG, &dG)) != NMF_OK || (st = upload(bT, &dT)) != NMF_OK)
            return st;
        NMF_HIP(launch_cfinal_jobs(3, rpad, cf, dj, dF, (int)bF.size(),
                                   cfinal_lds_bytes(rpad, 3, cf), s_));
        NMF_HIP(launch_gram_w_jobs(0, dj, dG, (int)bG.size(), s_));
        if (seg) NMF_HIP(launch_gram_sum_jobs(0, dj, dT, (int)bT.size(), s_));
    }
    return NMF_OK;
}

// Move a problem's cursor over transfer steps (collected in order) to its next
// sweep; after the schedule, BF16 problems run their FP32 refinement, and fine
// iterations continue while a tolerance is set (the order of nmf_solve).
void Executor::advance(Inst &I, std::vector<Step> &xfers) {
    auto after_schedule = [&]() {
        if (I.use_tol && I.c.p->d.max_fine_iters > 0) {
            I.stage = 1;
            I.cont_left = I.c.p->d.max_fine_iters;
        } else {
            I.stage = 2;
        }
    };
    if (I.stage == 3 && I.refine_left <= 0) after_schedule();
    while (I.stage == 0) {
        if (I.cur >= I.sched.size()) {
            if (I.bf16 && I.c.p->d.refine_iters > 0) {
                I.stage = 3;
                I.refine_left = I.c.p->d.refine_iters;
            } else {
                after_schedule();
            }
            break;
        }
        const Step &st = I.sched[I.cur];
        if (st.kind != 0) {
            xfers.push_back(st);
            ++I.cur;
            continue;
        }
        if (I.left < 0) I.left = st.count;
        if (I.left == 0) {
            ++I.cur;
            I.left = -1;
            continue;
        }
        I.depth = st.depth;
        break;
    }
    if (I.stage == 1) {
        if (I.cont_left <= 0) I.stage = 2;
        I.depth = 0;
    }
    if (I.stage == 3) I.depth = 0;
    I.fp32job = I.bf16 && (I.stage == 1 || I.stage == 3);
}

nmf_status Executor::launch_xfers(std::vector<std::pair<Inst *, std::vector<Step>>> &todo) {
    nmf_plan_t plan = nullptr;
    size_t rounds = 0;
    for (auto &t : todo) rounds = std::max(rounds, t.second.size());
    for (size_t k = 0; k < rounds; ++k) {
        std::vector<XferJob> xj;
        std::vector<int2> bm;
        for (auto &t : todo) {
            if (t.second.size() <= k) continue;
            const Inst &I = *t.first;
            const Plan &p = *I.c.p;
            const Step &stp = t.second[k];
            const int d = stp.depth;
            XferJob x{};
            x.h = p.lv[d].h;
            x.w = p.lv[d].w;
            x.kind = stp.kind;
            x.xfer = p.d.xfer;
            x.ncols = p.d.r;
            x.stop = I.c.stop;
            if (stp.kind == 1) {          // V_{d+1} = R(V_d)
                x.X = I.c.V[d];
                x.ldx = p.lv[d].m;
                x.Y = I.c.V[d + 1];
            } else {                      // V_d = P(V_{d+1})
                x.X = I.c.V[d + 1];
                x.ldx = p.lv[d + 1].m;
                x.Y = I.c.V[d];
            }
            const int64_t mo = stp.kind == 1 ? p.lv[d + 1].m : p.lv[d].m;
            const int64_t t2 = xfer_tiles(mo, p.d.r);
            for (int64_t q = 0; q < t2; ++q) bm.push_back(make_int2((int)xj.size(), (int)q));
            xj.push_back(x);
        }
        const XferJob *dx;
        const int2 *db;
        nmf_status st;
        if ((st = upload(xj, &dx)) != NMF_OK || (st = upload(bm, &db)) != NMF_OK) return st;
        NMF_HIP(launch_xfer_many(dx, db, (int)bm.size(), s_));
    }
    return NMF_OK;
}

// Group the tick's sweeps by (rank class, A-pass tile rows, rule) and launch
// the five phases of each group.
nmf_status Executor::launch_sweeps(const std::vector<Inst *> &active, bool capture_ok) {
    nmf_plan_t plan = nullptr;
    std::map<std::tuple<int, int, int, int, int, int>, std::vector<Inst *>> groups;
    auto job_of = [](const Inst *I) -> const Job & {
        return I->fp32job ? I->c.jobs.back() : I->c.jobs[I->depth];
    };
    for (Inst *I : active) {
        const Job &J = job_of(I);
        groups[std::make_tuple(J.rpad, J.tm, I->mode, J.prec, J.wc, J.cf)].push_back(I);
    }
    std::vector<G> gl;
    std::vector<int64_t> key;
    nmf_status st;
    for (auto &kv : groups) {
        G g{};
        g.rpad = std::get<0>(kv.first);
        g.tm = std::get<1>(kv.first);
        g.mode = std::get<2>(kv.first);
        g.bf = std::get<3>(kv.first) == 1;
        g.wc = std::get<4>(kv.first);
        g.cf = std::get<5>(kv.first);
        std::vector<int64_t> gkey{g.rpad, g.tm, g.mode, g.bf ? 1 : 0, g.wc, g.cf};
        for (Inst *I : kv.second) {
            gkey.push_back(I->id);
            gkey.push_back(I->fp32job ? -1 : I->depth);
        }
        key.insert(key.end(), gkey.begin(), gkey.end());
        auto it = cache_.find(gkey);
        if (it != cache_.end()) {
            g = it->second;
        } else {
            std::vector<Job> jobs;
            std::vector<int2> bA, bC, bG, bF, bW;
            for (Inst *I : kv.second) {
                const Job &J = job_of(I);
                const int j = (int)jobs.size();
                for (int k = 0; k < J.nA; ++k) bA.push_back(make_int2(j, k));
                for (int k = 0; k < J.nC; ++k) bC.push_back(make_int2(j, k));
                for (int k = 0; k < J.nG; ++k) bG.push_back(make_int2(j, k));
                for (int k = 0; k < J.nG * J.gseg; ++k) bW.push_back(make_int2(j, k));
                for (int k = 0; k < J.nFb; ++k) bF.push_back(make_int2(j, k));
                jobs.push_back(J);
            }
            if ((st = upload(jobs, &g.dj)) != NMF_OK || (st = upload(bA, &g.bA)) != NMF_OK ||
                (st = upload(bC, &g.bC)) != NMF_OK || (st = upload(bG, &g.bG)) != NMF_OK ||
                (st = upload(bF, &g.bF)) != NMF_OK || (st = upload(bW, &g.bW)) != NMF_OK)
                return st;
            g.nA = (int)bA.size();
            g.nC = (int)bC.size();
            g.nG = (int)bG.size();
            g.nF = (int)bF.size();
            g.nW = (int)bW.size();
            g.seg = false;
            for (const Job &J : jobs) g.seg = g.seg || J.gseg > 1;
            cache_[gkey] = g;
        }
        gl.push_back(g);
    }
    auto launch_all = [&]() -> nmf_status {
        for (const G &g : gl) {
            NMF_HIP(launch_apass_jobs(g.mode, g.rpad, g.tm, g.dj, g.bA, g.nA,
                                      apass_lds_bytes(g.rpad, g.tm, g.mode), s_, g.bf));
            NMF_HIP(launch_cpass_jobs(g.rpad, g.wc, g.dj, g.bC, g.nC, s_, g.bf));
            NMF_HIP(launch_reduce_jobs(g.dj, g.bG, g.nG, s_));
            NMF_HIP(launch_cfinal_jobs(g.mode, g.rpad, g.cf, g.dj, g.bF, g.nF,
                                       cfinal_lds_bytes(g.rpad, g.mode, g.cf), s_));
            NMF_HIP(launch_gram_w_jobs(1, g.dj, g.bW, g.nW, s_));
            if (g.seg) NMF_HIP(launch_gram_sum_jobs(1, g.dj, g.bG, g.nG, s_));
        }
        return NMF_OK;
    };
    if (!use_graph_) return launch_all();
    // hipGraph: a tick configuration seen on two consecutive ticks is captured
    // once and replayed while it lasts.
    key.push_back(generation_);
    if (key == graph_key_ && gexec_) {
        NMF_HIP(hipGraphLaunch(gexec_, s_));
        return NMF_OK;
    }
    if (key != last_key_ || !capture_ok) {
        last_key_ = key;
        return launch_all();
    }
    drop_graph();
    hipGraph_t g = nullptr;
    NMF_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
    st = launch_all();
    hipError_t e = hipStreamEndCapture(s_, &g);
    if (st != NMF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(nullptr, NMF_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        gexec_ = nullptr;
        return fail(nullptr, NMF_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    graph_key_ = key;
    NMF_HIP(hipGraphLaunch(gexec_, s_));
    return NMF_OK;
}

nmf_status Executor::tick() {
    nmf_status st;
    if ((st = setup_fresh()) != NMF_OK) return st;
    std::vector<std::pair<Inst *, std::vector<Step>>> todo;
    std::vector<Inst *> active;
    for (Inst &I : insts_) {
        if (I.stage == 2) continue;
        std::vector<Step> xs;
        advance(I, xs);
        if (!xs.empty()) todo.emplace_back(&I, std::move(xs));
        if (I.stage != 2) active.push_back(&I);
    }
    if (!todo.empty() && (st = launch_xfers(todo)) != NMF_OK) return st;
    if (!active.empty() && (st = launch_sweeps(active, todo.empty())) != NMF_OK) return st;
    bool want_poll = false;
    for (Inst *I : active) {
        I->c.depths.push_back((int8_t)I->depth);
        if (I->stage == 0) {
            if (--I->left == 0) {
                ++I->cur;
                I->left = -1;
            }
        } else if (I->stage == 3) {
            --I->refine_left;
        } else {
            --I->cont_left;
        }
        if (I->use_tol && I->depth == 0 && ++I->since_check >= I->c.p->d.check_every) {
            I->since_check = 0;
            want_poll = true;
        }
    }
    ++ticks_;
    if (want_poll) return poll();
    return NMF_OK;
}

nmf_status Executor::gather(std::vector<DevState> &hs) {
    nmf_plan_t plan = nullptr;
    std::vector<DevState *> sts;
    for (Inst &I : insts_) sts.push_back(I.c.st);
    hs.resize(sts.size());
    if (sts.empty()) return NMF_OK;
    NMF_HIP(hipMemcpyAsync(dstptr_, sts.data(), sizeof(DevState *) * sts.size(),
                           hipMemcpyHostToDevice, s_));
    NMF_HIP(launch_gather_states(dstptr_, (int)sts.size(), dgather_, s_));
    NMF_HIP(hipMemcpyAsync(hs.data(), dgather_, sizeof(DevState) * sts.size(),
                           hipMemcpyDeviceToHost, s_));
    NMF_HIP(hipStreamSynchronize(s_));
    return NMF_OK;
}

// Queue a gather of the live problems' states into pp (pinned host memory).
nmf_status Executor::poll_issue(PendingPoll &pp) {
    nmf_plan_t plan = nullptr;
    if (!pp.h) {
        void *h = nullptr;
        NMF_HIP(hipHostMalloc(&h, sizeof(DevState) * (size_t)std::max(capacity_, 1),
                              hipHostMallocDefault));
        pp.h = static_cast<DevState *>(h);
        NMF_HIP(hipEventCreateWithFlags(&pp.ev, hipEventDisableTiming));
    }
    pp.ids.clear();
    pp.sts.clear();
    for (Inst &I : insts_) {
        if (I.stage == 2) continue;
        pp.ids.push_back(I.id);
        pp.sts.push_back(I.c.st);
    }
    if (pp.sts.empty()) return NMF_OK;
    NMF_HIP(hipMemcpyAsync(dstptr_, pp.sts.data(), sizeof(DevState *) * pp.sts.size(),
                           hipMemcpyHostToDevice, s_));
    NMF_HIP(launch_gather_states(dstptr_, (int)pp.sts.size(), dgather_, s_));
    NMF_HIP(hipMemcpyAsync(pp.h, dgather_, sizeof(DevState) * pp.sts.size(),
                           hipMemcpyDeviceToHost, s_));
    NMF_HIP(hipEventRecord(pp.ev, s_));
    pp.live = true;
    return NMF_OK;
}

// Wait for a queued gather; problems whose stop flag it shows are done.
nmf_status Executor::poll_finish(PendingPoll &pp) {
    nmf_plan_t plan = nullptr;
    if (!pp.live) return NMF_OK;
    NMF_HIP(hipEventSynchronize(pp.ev));
    pp.live = false;
    for (size_t k = 0; k < pp.ids.size(); ++k) {
        const int i = slot_of(pp.ids[k]);
        if (i >= 0 && pp.h[k].stop && insts_[i].stage != 2) insts_[i].stage = 2;
    }
    return NMF_OK;
}

// A tolerance check: queue this check's gather, then act on the previous one.
nmf_status Executor::poll() {
    PendingPoll &now = polls_[poll_next_];
    PendingPoll &prev = polls_[poll_next_ ^ 1];
    nmf_status st = poll_finish(now);   // (only if two checks ago was never read)
    if (st != NMF_OK) return st;
    if ((st = poll_issue(now)) != NMF_OK) return st;
    poll_next_ ^= 1;
    return poll_finish(prev);
}

bool Executor::all_done() const {
    for (const Inst &I : insts_)
        if (I.stage != 2) return false;
    return fresh_.empty();
}

bool Executor::any_done() const {
    for (const Inst &I : insts_)
        if (I.stage == 2) return true;
    return false;
}

nmf_status Executor::results(std::vector<int> &ids, std::vector<nmf_result> &res,
                             std::vector<nmf_status> &status, bool only_done) {
    std::vector<DevState> hs;
    nmf_status st = gather(hs);
    if (st != NMF_OK) return st;
    for (size_t i = 0; i < insts_.size(); ++i) {
        if (only_done && insts_[i].stage != 2) continue;
        nmf_result r;
        status.push_back(result_from_state(insts_[i].plan, hs[i], insts_[i].c.depths, &r));
        ids.push_back(insts_[i].id);
        res.push_back(r);
    }
    return NMF_OK;
}

void Executor::remove(int id) {
    const int k = slot_of(id);
    if (k >= 0) insts_.erase(insts_.begin() + k);
    // cached tables stay valid (they copy jobs, keyed by problem id); the
    // captured tick no longer matches
    drop_graph();
    last_key_.clear();
}

}  // namespace nmf

using namespace nmf;

extern "C" {

nmf_status nmf_batch_workspace(const nmf_plan_t *plans, int32_t count, size_t *bytes) {
    if (!plans || count <= 0 || !bytes) return fail(nullptr, NMF_E_ARG, "bad argument");
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) return fail(nullptr, NMF_E_ARG, "null plan");
        off = align256(off + plans[i]->p.ws.total);
    }
    *bytes = batch_area_layout(off, count, batch_table_bytes(plans, count)).end;
    return NMF_OK;
}

nmf_status nmf_solve_batch(const nmf_plan_t *plans, int32_t count, const float *const *dM,
                           float *const *dV, float *const *dW, const int32_t *iters,
                           void *dWorkspace, void *stream, int32_t flags, nmf_result *hOut) {
    if (!plans || count <= 0 || !dM || !dV || !dW || !iters || !dWorkspace)
        return fail(nullptr, NMF_E_ARG, "null argument");
    if (reinterpret_cast<uintptr_t>(dWorkspace) & 255)
        return fail(nullptr, NMF_E_ARG, "workspace must be 256-byte aligned");
    char *base = static_cast<char *>(dWorkspace);
    std::vector<size_t> offs;
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !dM[i] || !dV[i] || !dW[i] || iters[i] < 0)
            return fail(nullptr, NMF_E_ARG, "null plan / buffer or negative iters in the batch");
        offs.push_back(off);
        off = align256(off + plans[i]->p.ws.total);
    }
    const BatchArea area = batch_area_layout(off, count, batch_table_bytes(plans, count));
    hipStream_t user = static_cast<hipStream_t>(stream);
    const bool graphs = (flags & NMF_BATCH_GRAPH) != 0;
    nmf_plan_t plan = nullptr;
    // Graph capture needs a stream of our own (the legacy default stream
    // cannot be captured); it waits for the caller's stream first.
    hipStream_t s = user;
    hipEvent_t ev = nullptr;
    if (graphs) {
        NMF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        NMF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        NMF_HIP(hipEventRecord(ev, user));
        NMF_HIP(hipStreamWaitEvent(s, ev, 0));
    }
    nmf_status st = NMF_OK;
    {
        Executor ex(base, area, count, s, graphs);
        NMF_HIP(enable_large_lds());
        for (int i = 0; i < count && st == NMF_OK; ++i)
            st = ex.add(plans[i], dM[i], dV[i], dW[i], iters[i], base + offs[i], i);
        while (st == NMF_OK && !ex.all_done()) st = ex.tick();
        std::vector<int> ids;
        std::vector<nmf_result> res;
        std::vector<nmf_status> stats;
        if (st == NMF_OK) st = ex.results(ids, res, stats, false);
        if (st == NMF_OK) {
            for (size_t k = 0; k < ids.size(); ++k) {
                if (hOut) hOut[ids[k]] = res[k];
                if (stats[k] != NMF_OK && st == NMF_OK) st = stats[k];
            }
        }
    }
    if (graphs) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        (void)hipEventDestroy(ev);
    }
    return st;
}

}  // extern "C"
