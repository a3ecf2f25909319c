// Serving loop with continuous batching.  Requests (a plan description and
// host M, V0, W0) queue on submit; a worker thread admits them in arrival
// order while the device pool (allocated once, at creation) has room for
// their footprint (M, V, W and workspace) and a slot is free, and advances
// every admitted solve with the batch executor: requests arriving while
// others run join at the next tick, and a finished request's factors are
// copied back to host memory and its device memory is released at once.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>

#include "batch.h"

namespace nmf {

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit sub-allocator over [0, size) with 256-byte granularity.
class Pool {
public:
    explicit Pool(size_t size) { free_.push_back({0, size}); }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                it->first += bytes;
                it->second -= bytes;
                if (it->second == 0) free_.erase(it);
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        used_ -= bytes;
        auto it = free_.begin();
        while (it != free_.end() && it->first < off) ++it;
        it = free_.insert(it, {off, bytes});
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::list<std::pair<size_t, size_t>> free_;   // (offset, bytes), sorted
    size_t used_ = 0;
};

struct Request {
    uint64_t ticket = 0;
    nmf_plan_t plan = nullptr;
    int32_t iters = 0;
    const float *hM = nullptr, *hV0 = nullptr, *hW0 = nullptr;
    int64_t m = 0, n = 0, r = 0;
    size_t ws_bytes = 0, footprint = 0, off = 0;
    std::vector<float> V, W;       // results, host
    double t_submit = 0, t_admit = 0, t_done = 0;
    nmf_result res{};
    nmf_status status = NMF_OK;
    int state = 0;                 // 0 queued, 1 running, 2 done
};

}  // namespace
}  // namespace nmf

struct nmf_server_s {
    int device = 0;
    size_t budget = 0, area_bytes = 0;
    int slots = 0;
    char *dbase = nullptr;         // executor area, then the request pool
    hipStream_t s = nullptr;
    nmf::BatchArea area{};
    nmf::Pool *pool = nullptr;
    nmf::Executor *ex = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<nmf::Request *> queue;
    std::map<uint64_t, nmf::Request *> reqs;
    uint64_t next_ticket = 1;
    bool shutdown = false;
    nmf_status fatal = NMF_OK;
    std::string fatal_msg;
    int64_t stats[6] = {0, 0, 0, 0, 0, 0};   // admitted, completed, running, peak running,
                                             // peak pool bytes, ticks
    std::thread worker;
};

namespace nmf {
namespace {

// Copy a finished request's factors to host, release its device memory.
nmf_status retire(nmf_server_s *S, Request *R, const nmf_result &res, nmf_status st) {
    nmf_plan_t plan = nullptr;
    char *p = S->dbase + S->area_bytes + R->off;
    const float *dV = reinterpret_cast<const float *>(p + align256(sizeof(float) * R->m * R->n));
    const float *dW = reinterpret_cast<const float *>(reinterpret_cast<const char *>(dV) +
                                                      align256(sizeof(float) * R->m * R->r));
    R->V.resize((size_t)R->m * R->r);
    R->W.resize((size_t)R->r * R->n);
    NMF_HIP(hipMemcpyAsync(R->V.data(), dV, sizeof(float) * R->V.size(), hipMemcpyDeviceToHost,
                           S->s));
    NMF_HIP(hipMemcpyAsync(R->W.data(), dW, sizeof(float) * R->W.size(), hipMemcpyDeviceToHost,
                           S->s));
    NMF_HIP(hipStreamSynchronize(S->s));
    S->ex->remove((int)R->ticket);
    std::lock_guard<std::mutex> lk(S->mu);
    S->pool->release(R->off, R->footprint);
    R->res = res;
    R->status = st;
    R->t_done = now_ms();
    R->res.queue_ms = R->t_admit - R->t_submit;
    R->res.latency_ms = R->t_done - R->t_submit;
    R->state = 2;
    S->stats[1]++;
    S->stats[2]--;
    S->cv.notify_all();
    return NMF_OK;
}

// Admit queued requests in arrival order while a slot and pool room are free.
nmf_status admit(nmf_server_s *S) {
    nmf_plan_t plan = nullptr;
    for (;;) {
        Request *R = nullptr;
        size_t off = 0;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->queue.empty() || S->stats[2] >= S->slots) return NMF_OK;
            R = S->queue.front();
            if (!S->pool->alloc(R->footprint, &off)) return NMF_OK;
            S->queue.pop_front();
            R->off = off;
            R->state = 1;
            R->t_admit = now_ms();
            S->stats[0]++;
            S->stats[2]++;
            S->stats[3] = std::max(S->stats[3], S->stats[2]);
            S->stats[4] = std::max<int64_t>(S->stats[4], (int64_t)S->pool->used());
        }
        char *p = S->dbase + S->area_bytes + off;
        float *dM = reinterpret_cast<float *>(p);
        float *dV = reinterpret_cast<float *>(p + align256(sizeof(float) * R->m * R->n));
        float *dW = reinterpret_cast<float *>(reinterpret_cast<char *>(dV) +
                                              align256(sizeof(float) * R->m * R->r));
        char *dws = reinterpret_cast<char *>(dW) + align256(sizeof(float) * R->r * R->n);
        NMF_HIP(hipMemcpyAsync(dM, R->hM, sizeof(float) * R->m * R->n, hipMemcpyHostToDevice, S->s));
        NMF_HIP(hipMemcpyAsync(dV, R->hV0, sizeof(float) * R->m * R->r, hipMemcpyHostToDevice, S->s));
        NMF_HIP(hipMemcpyAsync(dW, R->hW0, sizeof(float) * R->r * R->n, hipMemcpyHostToDevice, S->s));
        nmf_status st = S->ex->add(R->plan, dM, dV, dW, R->iters, dws, (int)R->ticket);
        if (st != NMF_OK) {
            nmf_result z{};
            if ((st = retire(S, R, z, st)) != NMF_OK) return st;
        }
    }
}

nmf_status collect(nmf_server_s *S) {
    std::vector<int> ids;
    std::vector<nmf_result> res;
    std::vector<nmf_status> sts;
    nmf_status st = S->ex->results(ids, res, sts, true);
    if (st != NMF_OK) return st;
    for (size_t k = 0; k < ids.size(); ++k) {
        Request *R;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            R = S->reqs[(uint64_t)ids[k]];
        }
        if ((st = retire(S, R, res[k], sts[k])) != NMF_OK) return st;
    }
    return NMF_OK;
}

void worker_loop(nmf_server_s *S) {
    (void)hipSetDevice(S->device);
    nmf_status st = NMF_OK;
    while (st == NMF_OK) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait_for(lk, std::chrono::milliseconds(2), [&] {
                return S->shutdown || !S->queue.empty() || S->stats[2] > 0;
            });
            if (S->shutdown && S->queue.empty() && S->stats[2] == 0) break;
        }
        if ((st = admit(S)) != NMF_OK) break;
        if (S->ex->empty()) continue;
        if ((st = S->ex->tick()) != NMF_OK) break;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stats[5] = S->ex->ticks();
        }
        if (S->ex->any_done() && (st = collect(S)) != NMF_OK) break;
    }
    if (st != NMF_OK) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->fatal = st;
        S->fatal_msg = nmf_last_error(nullptr);
        S->cv.notify_all();
    }
}

}  // namespace
}  // namespace nmf

using namespace nmf;

extern "C" {

nmf_status nmf_server_create(size_t hbm_budget, int32_t slots, nmf_server **out) {
    if (!out || slots <= 0 || hbm_budget == 0) return fail(nullptr, NMF_E_ARG, "bad argument");
    nmf_server_s *S = new (std::nothrow) nmf_server_s;
    if (!S) return fail(nullptr, NMF_E_NOMEM, "host allocation failed");
    nmf_plan_t plan = nullptr;
    (void)hipGetDevice(&S->device);
    S->budget = align256(hbm_budget);
    S->slots = slots;
    // executor tables: bounded per slot (job table, block maps, transfers)
    const size_t table = (size_t)slots * (256 << 10) + (16 << 20);
    S->area = batch_area_layout(0, slots, table);
    S->area_bytes = align256(S->area.end);
    hipError_t e = hipMalloc(&S->dbase, S->area_bytes + S->budget);
    if (e != hipSuccess) {
        delete S;
        return fail(nullptr, NMF_E_NOMEM, std::string("hipMalloc of the server pool: ") +
                                              hipGetErrorString(e));
    }
    e = hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(S->dbase);
        delete S;
        return fail(nullptr, NMF_E_DEVICE, "hipStreamCreate failed");
    }
    if (enable_large_lds() != hipSuccess) {
        (void)hipStreamDestroy(S->s);
        (void)hipFree(S->dbase);
        delete S;
        return fail(plan, NMF_E_DEVICE, "kernel attribute setup failed");
    }
    S->pool = new Pool(S->budget);
    S->ex = new Executor(S->dbase, S->area, slots, S->s, false);
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return NMF_OK;
}

nmf_status nmf_server_submit(nmf_server *S, const nmf_desc *desc, const float *hM,
                             const float *hV0, const float *hW0, int32_t iters,
                             uint64_t *ticket) {
    if (!S || !desc || !hM || !hV0 || !hW0 || !ticket || iters < 0)
        return fail(nullptr, NMF_E_ARG, "bad argument");
    if (desc->algo == NMF_ANLS || desc->algo == NMF_KL || desc->ntf_k != 0)
        return fail(nullptr, NMF_E_ARG, "the server runs HALS and MU matrix solves");
    if (desc->ldm != 0 && desc->ldm != desc->m)
        return fail(nullptr, NMF_E_ARG, "server requests take contiguous columns (ldm = m)");
    nmf_plan_t plan = nullptr;
    size_t ws = 0;
    nmf_status st = nmf_plan(desc, &plan, &ws);
    if (st != NMF_OK) return st;
    Request *R = new Request;
    R->plan = plan;
    R->iters = iters;
    R->hM = hM;
    R->hV0 = hV0;
    R->hW0 = hW0;
    R->m = desc->m;
    R->n = desc->n;
    R->r = desc->r;
    R->ws_bytes = ws;
    R->footprint = align256(sizeof(float) * R->m * R->n) + align256(sizeof(float) * R->m * R->r) +
                   align256(sizeof(float) * R->r * R->n) + align256(ws);
    if (R->footprint > S->budget) {
        nmf_destroy(plan);
        delete R;
        return fail(nullptr, NMF_E_BUSY, "request footprint exceeds the server's HBM budget");
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal != NMF_OK) {
        nmf_destroy(plan);
        delete R;
        return fail(nullptr, S->fatal, "server stopped: " + S->fatal_msg);
    }
    R->ticket = S->next_ticket++;
    R->t_submit = now_ms();
    S->reqs[R->ticket] = R;
    S->queue.push_back(R);
    *ticket = R->ticket;
    S->cv.notify_all();
    return NMF_OK;
}

nmf_status nmf_server_poll(nmf_server *S, uint64_t ticket, float *hV, float *hW, nmf_result *out) {
    if (!S) return fail(nullptr, NMF_E_ARG, "null server");
    Request *R = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end()) return fail(nullptr, NMF_E_ARG, "unknown ticket");
        R = it->second;
        if (R->state != 2) {
            if (S->fatal != NMF_OK) return fail(nullptr, S->fatal, "server stopped: " + S->fatal_msg);
            return NMF_PENDING;
        }
        S->reqs.erase(it);
    }
    if (hV) memcpy(hV, R->V.data(), sizeof(float) * R->V.size());
    if (hW) memcpy(hW, R->W.data(), sizeof(float) * R->W.size());
    if (out) *out = R->res;
    const nmf_status st = R->status;
    nmf_destroy(R->plan);
    delete R;
    return st;
}

nmf_status nmf_server_stats(nmf_server *S, int64_t *stats, int32_t cap) {
    if (!S || !stats) return fail(nullptr, NMF_E_ARG, "bad argument");
    std::lock_guard<std::mutex> lk(S->mu);
    for (int i = 0; i < cap && i < 6; ++i) stats[i] = S->stats[i];
    return NMF_OK;
}

nmf_status nmf_server_destroy(nmf_server *S) {
    if (!S) return NMF_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->shutdown = true;
        // queued requests that never started are dropped with their tickets
        for (Request *R : S->queue) {
            S->reqs.erase(R->ticket);
            nmf_destroy(R->plan);
            delete R;
        }
        S->queue.clear();
        S->cv.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    for (auto &kv : S->reqs) {
        nmf_destroy(kv.second->plan);
        delete kv.second;
    }
    delete S->ex;
    delete S->pool;
    (void)hipStreamSynchronize(S->s);
    (void)hipStreamDestroy(S->s);
    (void)hipFree(S->dbase);
    delete S;
    return NMF_OK;
}

}  // extern "C"
