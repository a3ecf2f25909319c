// C ABI of libnmf and the host executor that runs a schedule on a stream.
#include <cstdio>
#include <cstring>
#include <new>

#include "exec.h"

namespace nmf {

namespace {
thread_local std::string g_err;
}  // namespace

nmf_status fail(nmf_plan_t, nmf_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

namespace {

template <class T>
T *at(char *base, size_t off) {
    return reinterpret_cast<T *>(base + off);
}

// ---- optional HIP-event timing of selected kernel kinds -------------------
int prof_begin(Ctx &c, int kind) {
    Profiler &pf = c.plan->p.prof;
    if (!c.prof || !(pf.mask & (1u << kind))) return -1;
    hipEvent_t e[2];
    {
        std::lock_guard<std::mutex> lk(pf.mu);
        for (int i = 0; i < 2; ++i) {
            if (!pf.pool.empty()) {
                e[i] = pf.pool.back();
                pf.pool.pop_back();
            } else if (hipEventCreate(&e[i]) != hipSuccess) {
                if (i) pf.pool.push_back(e[0]);
                return -1;
            }
        }
    }
    if (hipEventRecord(e[0], c.s) != hipSuccess) {
        std::lock_guard<std::mutex> lk(pf.mu);
        pf.pool.push_back(e[0]);
        pf.pool.push_back(e[1]);
        return -1;
    }
    c.prof_pending.push_back(Ctx::ProfEvent{kind, e[0], e[1]});
    return (int)c.prof_pending.size() - 1;
}

void prof_end(Ctx &c, int idx) {
    if (idx >= 0) (void)hipEventRecord(c.prof_pending[idx].end, c.s);
}

// Call only after the stream has been synchronised.
void prof_collect(Ctx &c) {
    if (c.prof_pending.empty()) return;
    Profiler &pf = c.plan->p.prof;
    std::lock_guard<std::mutex> lk(pf.mu);
    for (const Ctx::ProfEvent &e : c.prof_pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e.begin, e.end) == hipSuccess) {
            pf.counts[e.kind]++;
            pf.ms[e.kind] += ms;
        }
        pf.pool.push_back(e.begin);
        pf.pool.push_back(e.end);
    }
    c.prof_pending.clear();
    (void)hipGetLastError();
}

#define NMF_LAUNCH(kind, call)                              \
    do {                                                    \
        const int pi_ = prof_begin(c, (kind));              \
        NMF_HIP(call);                                      \
        prof_end(c, pi_);                                   \
    } while (0)

// Blocks of the D-reduction launch: the upper Gram tiles, then (single
// solves) the blocks that sum V^T M over the chunks.
int reduce_blocks(const Job &J) { return J.nG + (J.Cr ? J.nCr : 0); }

// FP32 streaming tiling of a job when its level qualifies (large, m and the
// column stride of M multiples of 4, M 16-byte aligned).
void set_fp32_stream(Job &J, const LevelInfo &li, const Plan &p) {
    if (!li.fstream || (J.ldm & 3) != 0 || (reinterpret_cast<uintptr_t>(J.M) & 15) != 0) return;
    J.stream = 1;
    J.tm = li.ftm;   // A-pass rows per block (RS = 2 or 1)
    J.nA = (int32_t)((li.m + J.tm - 1) / J.tm);
    J.aks = li.aks;
    J.nCx = (int32_t)((li.n + 127) / 128);
    J.chunks = li.fcp_chunks;
    J.chunk = li.fcp_chunk;
    J.nC = J.nCx * J.chunks;
}

}  // namespace

Ctx make_ctx(nmf_plan_t plan, const float *dM, float *dV, float *dW, void *dws, hipStream_t s,
             bool allow_stream) {
    const Plan &p = plan->p;
    Ctx c;
    c.plan = plan;
    c.p = &p;
    c.s = s;
    c.ws = static_cast<char *>(dws);
    c.st = at<DevState>(c.ws, p.ws.off_state);
    c.stop = &c.st->stop;
    c.log_rel = at<double>(c.ws, p.ws.off_log);
    c.log_depth = at<int32_t>(c.ws, p.ws.off_logdepth);
    c.norm = at<double>(c.ws, p.ws.off_norm);
    c.nparts = at<double>(c.ws, p.ws.off_nparts);
    c.Bd = at<double>(c.ws, p.ws.off_Bd);
    c.Dd = at<double>(c.ws, p.ws.off_Dd);
    c.Bf = at<float>(c.ws, p.ws.off_Bf);
    c.Df = at<float>(c.ws, p.ws.off_Df);
    c.gparts = at<double>(c.ws, p.ws.off_gparts);
    c.rparts = at<double>(c.ws, p.ws.off_rparts);
    c.Cp = at<double>(c.ws, p.ws.off_cparts);
    c.Dp = at<double>(c.ws, p.ws.off_Dp);
    c.Cr = p.ws.off_Cr ? at<double>(c.ws, p.ws.off_Cr) : nullptr;
    c.bparts = at<double>(c.ws, p.ws.off_bparts);
    c.Wt = at<float>(c.ws, p.ws.off_Wt);
    c.A = p.ws.off_A ? at<double>(c.ws, p.ws.off_A) : nullptr;
    c.C = p.ws.off_C ? at<double>(c.ws, p.ws.off_C) : nullptr;
    if (p.d.ntf_k > 0) {
        c.ntfGB = at<double>(c.ws, p.ws.off_ntfG);
        c.ntfGC = c.ntfGB + (size_t)p.d.r * p.d.r;
    }
    if (p.d.algo == NMF_KL) {
        c.klw = at<double>(c.ws, p.ws.off_klw);
        c.klwp = at<double>(c.ws, p.ws.off_klwp);
        c.klvp = at<double>(c.ws, p.ws.off_klvp);
        c.kld = at<double>(c.ws, p.ws.off_kld);
        c.klm = at<double>(c.ws, p.ws.off_klm);
    }
    for (size_t l = 0; l < p.lv.size(); ++l) {
        if (l == 0) {
            c.M.push_back(dM);
            c.ldm.push_back(p.d.ldm);
            c.V.push_back(dV);
            c.Wl.push_back(dW);
        } else {
            c.M.push_back(at<float>(c.ws, p.lv[l].off_M));
            c.ldm.push_back(p.lv[l].m);
            c.V.push_back(at<float>(c.ws, p.lv[l].off_V));
            // W moves between levels only in two-sided hierarchies
            c.Wl.push_back(p.d.two_sided ? at<float>(c.ws, p.lv[l].off_W) : dW);
        }
    }
    c.W = dW;
    c.djobs = at<Job>(c.ws, p.ws.off_jobs);
    for (size_t l = 0; l < p.lv.size(); ++l) {
        const LevelInfo &li = p.lv[l];
        Job J{};
        J.M = c.M[l];
        J.ldm = c.ldm[l];
        J.m = li.m;
        J.n = li.n;
        J.r = p.d.r;
        J.rpad = p.rpad;
        J.tm = li.atm;
        J.chunks = li.cp_chunks;
        J.chunk = li.cp_chunk;
        J.nA = (int32_t)((li.m + J.tm - 1) / J.tm);
        J.nCx = (int32_t)((li.n + 63) / 64);
        J.nC = J.nCx * li.cp_chunks;
        J.nF = cpass_final_blocks(li.n);
        J.wc = p.wc;
        J.cf = p.cf;
        J.nFb = cfinal_tile_blocks(li.n, p.cf);
        J.nG = gram_tiles(p.rpad);
        J.depth = (int32_t)l;
        J.log_cap = p.d.log_cap;
        J.V = c.V[l];
        J.W = c.Wl[l];
        J.Wt = c.Wt;
        J.A = nullptr;
        J.C = nullptr;
        J.Ad = c.A;
        J.Cd = c.C;
        J.Bd = c.Bd;
        J.Dd = c.Dd;
        J.Cp = c.Cp;
        J.Dp = c.Dp;
        // single solves reduce V^T M in the D-reduction launch (more blocks
        // than the W update has); grouped launches keep it in the W update
        J.Cr = allow_stream ? c.Cr : nullptr;
        J.nCr = (int32_t)((li.n * p.d.r + 255) / 256);
        J.gseg = li.gseg;
        J.bparts = c.bparts;
        J.rparts = c.rparts;
        J.normM2 = c.norm + l;
        J.log_rel = c.log_rel;
        J.log_depth = c.log_depth;
        J.st = c.st;
        J.tol = p.d.tol;
        J.prec = 0;
        J.stream = 0;
        J.aks = 1;
        if (p.d.prec == NMF_FP32 && allow_stream) set_fp32_stream(J, li, p);
        if (p.d.prec == NMF_BF16) {
            J.prec = 1;
            if (li.stream && allow_stream) {   // streaming kernels: 256-row / 256-column tiles
                J.stream = 1;
                J.tm = kStreamARows;
                J.nA = (int32_t)((li.m + kStreamARows - 1) / kStreamARows);
                J.nCx = (int32_t)((li.n + 255) / 256);
                J.chunks = li.scp_chunks;
                J.chunk = li.scp_chunk;
                J.nC = J.nCx * J.chunks;
            }
            J.mpad = li.mpad;
            J.npad = bf_pad(p.d.n);
            J.Mbp = at<uint16_t>(c.ws, li.off_Mbp);
            J.Mbc = at<uint16_t>(c.ws, li.off_Mbc);
            J.Vb = at<uint16_t>(c.ws, li.off_Vb);
            J.Wb = at<uint16_t>(c.ws, p.ws.off_Wb);
        }
        c.jobs.push_back(J);
    }
    // entry L: the finest level in FP32 (refinement iterations of BF16 mode)
    Job J0 = c.jobs[0];
    if (J0.stream) {     // the FP32 job uses the regular tiling of level 0
        const LevelInfo &l0 = p.lv[0];
        J0.stream = 0;
        J0.tm = l0.atm;
        J0.nA = (int32_t)((l0.m + J0.tm - 1) / J0.tm);
        J0.nCx = (int32_t)((p.d.n + 63) / 64);
        J0.chunks = l0.cp_chunks;
        J0.chunk = l0.cp_chunk;
        J0.nC = J0.nCx * J0.chunks;
    }
    if (allow_stream) set_fp32_stream(J0, p.lv[0], p);
    J0.prec = 0;
    J0.Mbp = J0.Mbc = nullptr;
    J0.Vb = J0.Wb = nullptr;
    c.jobs.push_back(J0);
    return c;
}

nmf_status result_from_state(nmf_plan_t plan, const DevState &hs,
                             const std::vector<int8_t> &depths, nmf_result *out) {
    if (out) {
        memset(out, 0, sizeof *out);
        const int n = hs.log_len;
        out->log_len = n < plan->p.d.log_cap ? n : plan->p.d.log_cap;
        out->total_iters = n;
        out->stopped = hs.stopped;
        out->rel_err = hs.last_rel;
        const double per_depth = plan->p.d.two_sided ? 0.125 : 0.25;
        for (int i = 0; i < n && i < (int)depths.size(); ++i) {
            if (depths[i] == 0) out->fine_iters++;
            double f = 1.0;
            for (int k = 0; k < depths[i]; ++k) f *= per_depth;
            out->fine_equiv += f;
        }
    }
    if (hs.status != 0)
        return fail(plan, (nmf_status)hs.status, "non-finite residual during the solve");
    if (hs.flags & 4)
        return fail(plan, NMF_E_NONFINITE,
                    "NNLS met a non-positive pivot (collinear or singular Gram) or its "
                    "exchange did not end");
    return NMF_OK;
}

// BF16 mode: operand copies of every M_l (A-pass and C-pass layouts) and the
// zero padding of the V and W copies (their live part is written by the
// kernels that update V and W).
nmf_status prepare_bf16(Ctx &c) {
    nmf_plan_t plan = c.plan;
    const Plan &p = *c.p;
    if (p.d.prec != NMF_BF16) return NMF_OK;
    const Job &J0 = c.jobs[0];
    for (size_t l = 0; l < p.lv.size(); ++l) {
        const Job &J = c.jobs[l];
        if (J.stream) {   // both layouts in one pass over M_l
            NMF_HIP(launch_pack_bf16_both(c.M[l], c.ldm[l], J.m, J.n,
                                          const_cast<uint16_t *>(J.Mbp), J.npad,
                                          const_cast<uint16_t *>(J.Mbc), J.mpad, c.s));
        } else {
            NMF_HIP(launch_pack_bf16(c.M[l], c.ldm[l], J.m, J.n, const_cast<uint16_t *>(J.Mbp),
                                     J.npad, c.s));
            NMF_HIP(launch_to_bf16_cols(c.M[l], c.ldm[l], J.m, J.n,
                                        const_cast<uint16_t *>(J.Mbc), J.mpad, J.n, c.s));
        }
        NMF_HIP(launch_to_bf16_cols(c.V[l], J.m, J.m, J.r, J.Vb, J.mpad, J.rpad, c.s));
    }
    // W (r x n row-major) read as n x r column-major: Wb is rpad x npad row-major
    NMF_HIP(launch_to_bf16_cols(c.W, J0.n, J0.n, J0.r, J0.Wb, J0.npad, J0.rpad, c.s));
    return NMF_OK;
}


namespace {

nmf_status upload_jobs(Ctx &c) {
    nmf_plan_t plan = c.plan;
    NMF_HIP(enable_large_lds());
    NMF_HIP(hipMemcpyAsync(c.djobs, c.jobs.data(), sizeof(Job) * c.jobs.size(),
                           hipMemcpyHostToDevice, c.s));
    return NMF_OK;
}

// B = W W^T of level d's W with the standalone Gram kernels (ANLS).
nmf_status gram_W(Ctx &c, int d) {
    nmf_plan_t plan = c.plan;
    const Plan &p = *c.p;
    const LevelInfo &li = p.lv[d];
    NMF_LAUNCH(K_GRAM_W, launch_gram(p.rpad, p.d.r, li.n, c.Wl[d], li.n, li.gram_w_parts,
                                     li.gram_w_chunk, c.gparts, c.Bd, c.Bf, c.stop, c.s));
    return NMF_OK;
}

// Start of a solve: Wt (transposed, zero-padded W) from the W tile kernel and
// B = W W^T from the B tile kernel.  The batch executor runs the same two
// kernels, so single and batched solves agree bitwise.
// Also after a W transfer of a two-sided hierarchy, for the level it reached.
nmf_status init_w(Ctx &c, int d = 0) {
    nmf_plan_t plan = c.plan;
    const Job &J = c.jobs[d];
    if (c.p->d.ntf_k > 0) {   // B^T B, C^T C, the mode-1 Gram, the Khatri-Rao product
        const int64_t K = c.p->d.ntf_k, Jd = J.n / K;
        NMF_LAUNCH(K_NTF, launch_ntf_gram(c.ntfB, Jd, J.r, c.ntfGB, nullptr, nullptr, c.stop, c.s));
        NMF_LAUNCH(K_NTF, launch_ntf_gram(c.ntfC, K, J.r, c.ntfGC, c.ntfGB, c.Bd, c.stop, c.s));
        NMF_LAUNCH(K_NTF, launch_ntf_kr(c.ntfB, c.ntfC, Jd, K, J.r, J.rpad, c.Wl[d], c.Wt, c.stop,
                                        c.s));
        return NMF_OK;
    }
    if (c.p->d.algo == NMF_KL) {   // Wt and the row sums of W
        NMF_LAUNCH(K_CFINAL, launch_kl_wfinal(J.rpad, J.n, J.r, 0, nullptr, nullptr, c.Wl[d],
                                              c.Wt, c.klwp, true, c.stop, c.s));
        NMF_LAUNCH(K_CFINAL, launch_kl_wsum(J.rpad, J.n, c.klwp, c.klw, c.stop, c.s));
        return NMF_OK;
    }
    NMF_LAUNCH(K_GRAM_W, launch_cfinal_jobs(3, J.rpad, J.cf, c.djobs + d, nullptr, J.nFb,
                                            cfinal_lds_bytes(J.rpad, 3, J.cf), c.s));
    NMF_LAUNCH(K_GRAM_W, launch_gram_w_jobs(0, c.djobs + d, nullptr, J.nG * J.gseg, c.s));
    if (J.gseg > 1)
        NMF_LAUNCH(K_GRAM_W, launch_gram_sum_jobs(0, c.djobs + d, nullptr, J.nG, c.s));
    return NMF_OK;
}

// Two-sided hierarchies: W (r x n_d, row-major) restricted along its rows to
// level d+1 (restrict_op) or prolonged from level d+1 to level d, then the
// reached level's Wt and W W^T.
nmf_status transfer_w(Ctx &c, int d, bool restrict_op) {
    nmf_plan_t plan = c.plan;
    const Plan &p = *c.p;
    const int64_t nf = p.lv[d].n, nc = p.lv[d + 1].n;
    if (restrict_op)
        NMF_LAUNCH(K_RESTRICT, launch_xfer_cols(1, p.d.xfer, p.d.r, nf, c.Wl[d], nf, 1,
                                                c.Wl[d + 1], nc, 1, c.stop, c.s));
    else
        NMF_LAUNCH(K_PROLONG, launch_xfer_cols(0, p.d.xfer, p.d.r, nf, c.Wl[d + 1], nc, 1,
                                               c.Wl[d], nf, 1, c.stop, c.s));
    return init_w(c, restrict_op ? d + 1 : d);
}

// One iteration of the inner algorithm at depth d, then the residual.
// fp32: use the FP32 finest-level job (refinement iterations of BF16 mode).
nmf_status sweep(Ctx &c, int d, bool fp32 = false) {
    nmf_plan_t plan = c.plan;
    const Plan &p = *c.p;
    const int ji = fp32 ? (int)p.lv.size() : d;
    const Job &J = c.jobs[ji];
    const Job *dj = c.djobs + ji;
    if (p.d.ntf_k > 0) {   // NTF: mode 1 on the matrix kernels, then modes 2 and 3
        const int r = p.d.r;
        const int64_t n = J.n, K = p.d.ntf_k, Jd = n / K;
        NMF_LAUNCH(K_APASS, launch_apass_jobs(0, J.rpad, J.tm, dj, nullptr,
                                              apass_grid_single(J.nA),
                                              apass_lds_bytes(J.rpad, J.tm, 0), c.s, false));
        NMF_LAUNCH(K_CPART, launch_cpass_jobs(J.rpad, J.wc, dj, nullptr,
                                              cpass_grid_single(J.nCx, J.chunks), c.s, false));
        NMF_LAUNCH(K_GRAM_V, launch_reduce_jobs(dj, nullptr, reduce_blocks(J), c.s));
        // Y = A^T X_(1) (FP64, J.Cd) by the product-store mode of the W-update kernel
        NMF_LAUNCH(K_CFINAL, launch_cfinal_jobs(2, J.rpad, J.cf, dj, nullptr, J.nFb,
                                                cfinal_lds_bytes(J.rpad, 2, J.cf), c.s));
        // B: rows j, a_j[s] = sum_k Y[s, j + J k] C[k, s], Gram D o C^T C
        NMF_LAUNCH(K_NTF, launch_ntf_mode(J.rpad, c.C, n, c.Dd, c.ntfGC, c.ntfB, Jd, c.ntfC, K,
                                          1, Jd, r, nullptr, c.stop, c.s));
        NMF_LAUNCH(K_NTF, launch_ntf_gram(c.ntfB, Jd, r, c.ntfGB, nullptr, nullptr, c.stop, c.s));
        // C: rows k, a_k[s] = sum_j Y[s, j + J k] B[j, s], Gram D o B^T B; residual partials
        NMF_LAUNCH(K_NTF, launch_ntf_mode(J.rpad, c.C, n, c.Dd, c.ntfGB, c.ntfC, K, c.ntfB, Jd,
                                          Jd, 1, r, c.rparts, c.stop, c.s));
        // C^T C and the mode-1 Gram (B^T B) o (C^T C) of the new B and C (the Gram of
        // their exact Khatri-Rao product, FP64) into Bd: the residual's last term
        // (with D) and the Gram of the next A-pass
        NMF_LAUNCH(K_NTF, launch_ntf_gram(c.ntfC, K, r, c.ntfGC, c.ntfGB, c.Bd, c.stop, c.s));
        NMF_LAUNCH(K_RESID, launch_residual(c.rparts, ntf_mode_blocks(K), c.Dd, c.Bd, r, c.norm,
                                            d, c.log_rel, c.log_depth, p.d.log_cap, c.st,
                                            c.jobs[0].hstop, p.d.tol, c.s));
        // the Khatri-Rao product of the new B and C for the next A-pass
        NMF_LAUNCH(K_NTF, launch_ntf_kr(c.ntfB, c.ntfC, Jd, K, r, J.rpad, J.W, c.Wt, c.stop,
                                        c.s));
        c.depths.push_back((int8_t)d);
        return NMF_OK;
    }
    if (p.d.algo == NMF_KL) {   // KL divergence: V pass, W pass, W update, divergence, log
        const LevelInfo &li = p.lv[d];
        NMF_LAUNCH(K_APASS, launch_kl_vpass(J.rpad, J.M, J.ldm, J.m, J.n, J.r, J.V, J.W, c.Wt,
                                            c.klw, c.stop, c.s));
        NMF_LAUNCH(K_CPART, launch_kl_wpass(J.rpad, J.M, J.ldm, J.m, J.n, J.r, J.V, J.W,
                                            li.cp_chunks, li.cp_chunk, c.Cp, c.klvp, c.stop,
                                            c.s));
        NMF_LAUNCH(K_CFINAL, launch_kl_wfinal(J.rpad, J.n, J.r, li.cp_chunks, c.Cp, c.klvp, J.W,
                                              c.Wt, c.klwp, false, c.stop, c.s));
        NMF_LAUNCH(K_KL_DIV, launch_kl_div(J.rpad, J.M, J.ldm, J.m, J.n, J.r, J.V, J.W, c.kld,
                                           c.stop, c.s));
        NMF_LAUNCH(K_RESID, launch_kl_log(J.m, J.n, J.rpad, c.kld, c.klwp, c.klw, c.klm, d,
                                          c.log_rel, c.log_depth, p.d.log_cap, c.st,
                                          c.jobs[0].hstop, p.d.tol, c.s));
        c.depths.push_back((int8_t)d);
        return NMF_OK;
    }
    const bool bf = J.prec == 1;
    const int r = p.d.r;
    const int64_t n = J.n;
    int32_t *flags = &c.st->flags;
    const int mode = p.d.algo == NMF_HALS ? 0 : (p.d.algo == NMF_MU ? 1 : 2);
    if (J.stream && bf)
        NMF_LAUNCH(K_APASS, launch_apass_stream(mode, J.rpad, dj, nullptr, J.nA, c.s));
    else if (J.stream) {
        NMF_LAUNCH(K_APASS, launch_apass_s32(mode, J.rpad, dj, nullptr, J.nA * J.aks, c.s));
        if (J.aks > 1)
            NMF_LAUNCH(K_APASS, launch_afinal_s32(mode, J.rpad, dj, nullptr, J.nA, c.s));
    }
    else
        NMF_LAUNCH(K_APASS, launch_apass_jobs(mode, J.rpad, J.tm, dj, nullptr,
                                              apass_grid_single(J.nA),
                                              apass_lds_bytes(J.rpad, J.tm, mode), c.s, bf));
    if (mode == 2)
        NMF_LAUNCH(K_NNLS_ROWS, launch_nnls_rows(p.rpad, c.Bd, c.A, J.m, r, J.V, flags, c.stop, c.s));
    if (J.stream && bf)
        NMF_LAUNCH(K_CPART, launch_cpass_stream(J.rpad, dj, nullptr,
                                                cpass_stream_grid(J.nCx, J.chunks), c.s));
    else if (J.stream)
        NMF_LAUNCH(K_CPART, launch_cpass_s32(J.rpad, dj, nullptr,
                                             cpass_stream_grid(J.nCx, J.chunks), c.s));
    else
        NMF_LAUNCH(K_CPART, launch_cpass_jobs(J.rpad, J.wc, dj, nullptr,
                                              cpass_grid_single(J.nCx, J.chunks), c.s, bf));
    NMF_LAUNCH(K_GRAM_V, launch_reduce_jobs(dj, nullptr, reduce_blocks(J), c.s));
    NMF_LAUNCH(K_CFINAL, launch_cfinal_jobs(mode, J.rpad, J.cf, dj, nullptr, J.nFb,
                                            cfinal_lds_bytes(J.rpad, mode, J.cf), c.s));
    if (mode == 2) {
        NMF_LAUNCH(K_NNLS_COLS, launch_nnls_cols(p.rpad, c.Dd, c.C, n, r, J.W, c.Wt, c.rparts,
                                                 flags, c.stop, c.s));
        nmf_status st = gram_W(c, d);
        if (st != NMF_OK) return st;
        NMF_LAUNCH(K_RESID, launch_residual(c.rparts, nnls_cols_blocks(n), c.Dd, c.Bd, r, c.norm,
                                            d, c.log_rel, c.log_depth, p.d.log_cap, c.st,
                                            c.jobs[0].hstop, p.d.tol, c.s));
    } else {
        NMF_LAUNCH(K_GRAM_W, launch_gram_w_jobs(1, dj, nullptr, J.nG * J.gseg, c.s));
        if (J.gseg > 1)
            NMF_LAUNCH(K_GRAM_W, launch_gram_sum_jobs(1, dj, nullptr, J.nG, c.s));
    }
    c.depths.push_back((int8_t)d);
    return NMF_OK;
}

// Restrict M to every level (cached for the whole solve, as in Alg. 6's note)
// and compute ||M_l||_F^2 in FP64.
nmf_status prepare_levels(Ctx &c) {
    nmf_plan_t plan = c.plan;
    const Plan &p = *c.p;
    for (size_t l = 1; l < p.lv.size(); ++l) {
        const LevelInfo &lf = p.lv[l - 1], &lc = p.lv[l];
        float *Ml = const_cast<float *>(c.M[l]);
        if (!p.d.two_sided) {
            NMF_LAUNCH(K_RESTRICT, launch_restrict(p.d.xfer, lf.h, lf.w, lf.n, c.M[l - 1],
                                                   c.ldm[l - 1], Ml, nullptr, c.s));
        } else {
            // R_m M_{l-1} (m_l x n_{l-1}), then along the columns to n_l
            float *tmp = at<float>(c.ws, p.ws.off_tmpM);
            NMF_LAUNCH(K_RESTRICT, launch_restrict(p.d.xfer, lf.h, lf.w, lf.n, c.M[l - 1],
                                                   c.ldm[l - 1], tmp, nullptr, c.s));
            NMF_LAUNCH(K_RESTRICT, launch_xfer_cols(1, p.d.xfer, lc.m, lf.n, tmp, 1, lc.m, Ml,
                                                    1, lc.m, nullptr, c.s));
        }
    }
    for (size_t l = 0; l < p.lv.size(); ++l) {
        NMF_LAUNCH(K_SUMSQ, launch_sumsq(c.M[l], c.ldm[l], p.lv[l].m, p.lv[l].n,
                                         c.nparts + l * kNormParts,
                                         norm_parts(p.lv[l].m, p.lv[l].n), c.norm + l, c.s));
        if (p.d.algo == NMF_KL)   // sum(M_l), the scale of the logged divergence
            NMF_LAUNCH(K_SUMSQ, launch_msum(c.M[l], c.ldm[l], p.lv[l].m, p.lv[l].n,
                                            c.nparts + l * kNormParts,
                                            norm_parts(p.lv[l].m, p.lv[l].n), c.klm + l, c.s));
    }
    return NMF_OK;
}

nmf_status read_state(Ctx &c, DevState &hs) {
    nmf_plan_t plan = c.plan;
    NMF_HIP(hipMemcpyAsync(&hs, c.st, sizeof(DevState), hipMemcpyDeviceToHost, c.s));
    NMF_HIP(hipStreamSynchronize(c.s));
    return NMF_OK;
}

nmf_status check_input(Ctx &c) {
    nmf_plan_t plan = c.plan;
    const Plan &p = *c.p;
    NMF_HIP(launch_check_input(c.M[0], p.d.ldm, p.d.m, p.d.n, &c.st->flags, c.s));
    DevState hs;
    nmf_status st = read_state(c, hs);
    if (st != NMF_OK) return st;
    if (hs.flags & 2) return fail(plan, NMF_E_NONFINITE, "M has a NaN or Inf entry");
    if (hs.flags & 1) return fail(plan, NMF_E_NEGATIVE, "M has a negative entry");
    return NMF_OK;
}

nmf_status finish(Ctx &c, nmf_result *out) {
    nmf_plan_t plan = c.plan;
    DevState hs;
    nmf_status st = read_state(c, hs);
    if (st != NMF_OK) return st;
    prof_collect(c);
    return result_from_state(plan, hs, c.depths, out);
}

}  // namespace
}  // namespace nmf

using namespace nmf;

extern "C" {

const char *nmf_status_string(nmf_status s) {
    switch (s) {
        case NMF_OK: return "ok";
        case NMF_E_ARG: return "invalid argument";
        case NMF_E_SHAPE: return "invalid shape";
        case NMF_E_NOMEM: return "out of memory / workspace too small";
        case NMF_E_DEVICE: return "device (HIP) error";
        case NMF_E_NONFINITE: return "non-finite value";
        case NMF_E_NEGATIVE: return "negative entry in M";
        case NMF_E_BUSY: return "admission budget exceeded";
        default: return "unknown status";
    }
}

const char *nmf_last_error(nmf_plan_t) { return g_err.c_str(); }

nmf_status nmf_plan(const nmf_desc *desc, nmf_plan_t *out, size_t *workspace_bytes) {
    if (!desc || !out) return fail(nullptr, NMF_E_ARG, "null desc or out");
    nmf_plan_t plan = new (std::nothrow) nmf_plan_s;
    if (!plan) return fail(nullptr, NMF_E_NOMEM, "host allocation failed");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
        plan->p.num_cu = cus;
    else
        plan->p.num_cu = 256;
    (void)hipGetLastError();
    std::string err;
    nmf_status st = build_plan(*desc, plan->p, err);
    if (st != NMF_OK) {
        delete plan;
        return fail(nullptr, st, err);
    }
    *out = plan;
    if (workspace_bytes) *workspace_bytes = plan->p.ws.total;
    return NMF_OK;
}

nmf_status nmf_destroy(nmf_plan_t plan) {
    if (plan) {
        {
            std::lock_guard<std::mutex> lk(plan->p.prof.mu);
            for (hipEvent_t e : plan->p.prof.pool) (void)hipEventDestroy(e);
            plan->p.prof.pool.clear();
        }
        std::lock_guard<std::mutex> lk(plan->p.poll.mu);
        for (hipEvent_t e : plan->p.poll.events) (void)hipEventDestroy(e);
        for (int32_t *f : plan->p.poll.flags) (void)hipHostFree(f);
        plan->p.poll.events.clear();
        plan->p.poll.flags.clear();
    }
    delete plan;
    return NMF_OK;
}

nmf_status nmf_query_levels(nmf_plan_t plan, int32_t *hw, int32_t cap_levels) {
    if (!plan || !hw) return fail(plan, NMF_E_ARG, "null argument");
    const auto &lv = plan->p.lv;
    for (size_t l = 0; l < lv.size() && (int32_t)l < cap_levels; ++l) {
        hw[2 * l] = lv[l].h;
        hw[2 * l + 1] = lv[l].w;
    }
    return NMF_OK;
}

nmf_status nmf_query_schedule(nmf_plan_t plan, int32_t iters, int32_t *steps, int32_t cap,
                              int32_t *nsteps) {
    if (!plan || !nsteps || iters < 0) return fail(plan, NMF_E_ARG, "bad argument");
    auto s = make_schedule(plan->p.d.cycle, plan->p.d.levels, iters, plan->p.d.two_sided ? 8 : 4);
    *nsteps = (int32_t)s.size();
    for (size_t i = 0; i < s.size() && (int32_t)i < cap && steps; ++i) {
        steps[3 * i] = s[i].kind;
        steps[3 * i + 1] = s[i].depth;
        steps[3 * i + 2] = s[i].count;
    }
    return NMF_OK;
}

nmf_status nmf_solve(nmf_plan_t plan, const float *dM, float *dV, float *dW, int32_t iters,
                     void *dWorkspace, void *stream, nmf_result *hOut) {
    if (!plan || !dM || !dV || !dW || !dWorkspace)
        return fail(plan, NMF_E_ARG, "null plan or buffer");
    if (iters < 0) return fail(plan, NMF_E_ARG, "iters must be >= 0");
    if (reinterpret_cast<uintptr_t>(dWorkspace) & 255)
        return fail(plan, NMF_E_ARG, "workspace must be 256-byte aligned");
    return solve_on(plan, dM, dV, dW, iters, dWorkspace, static_cast<hipStream_t>(stream), hOut,
                    true, true);
}

nmf_status nmf_ntf_solve(nmf_plan_t plan, const float *dX, float *dA, float *dBt, float *dCt,
                         int32_t iters, void *dWorkspace, void *stream, nmf_result *hOut) {
    if (!plan || !dX || !dA || !dBt || !dCt || !dWorkspace)
        return fail(plan, NMF_E_ARG, "null plan or buffer");
    if (iters < 0) return fail(plan, NMF_E_ARG, "iters must be >= 0");
    if (reinterpret_cast<uintptr_t>(dWorkspace) & 255)
        return fail(plan, NMF_E_ARG, "workspace must be 256-byte aligned");
    if (plan->p.d.ntf_k <= 0) return fail(plan, NMF_E_ARG, "nmf_ntf_solve needs ntf_k > 0");
    return solve_on(plan, dX, dA, nullptr, iters, dWorkspace, static_cast<hipStream_t>(stream),
                    hOut, true, true, dBt, dCt);
}

}  // extern "C"

namespace nmf {

namespace {

// Tolerance checks of a solve.  Synchronous: every check_every counted
// iterations the host reads the device state (the stream drains, then the
// GPU idles until the next launches arrive).  Look-ahead: the stop flag is
// mirrored into host-mapped memory by the kernel that sets it; at each check
// the host records an event and waits only for the event of the previous
// check, so one batch of iterations stays queued while it looks.  Iterations
// issued after the stop return at once (every kernel tests the device flag),
// so both modes compute the same result.
struct Poller {
    Ctx &c;
    bool ahead = false;
    int32_t *hflag = nullptr;    // host side of the mapped flag
    std::vector<hipEvent_t> inflight;
    int since = 0;

    explicit Poller(Ctx &cx) : c(cx) {}
    ~Poller() {
        PollPool &pp = c.plan->p.poll;
        std::lock_guard<std::mutex> lk(pp.mu);
        for (hipEvent_t e : inflight) pp.events.push_back(e);
        if (hflag) pp.flags.push_back(hflag);
    }
    // Take a mapped flag for this solve and point the jobs at it (before the
    // job table is uploaded); stays synchronous if that fails.
    void enable() {
        PollPool &pp = c.plan->p.poll;
        {
            std::lock_guard<std::mutex> lk(pp.mu);
            if (!pp.flags.empty()) {
                hflag = pp.flags.back();
                pp.flags.pop_back();
            }
        }
        if (!hflag) {
            void *h = nullptr;
            if (hipHostMalloc(&h, 256, hipHostMallocMapped) != hipSuccess) {
                (void)hipGetLastError();
                return;
            }
            hflag = static_cast<int32_t *>(h);
        }
        void *dptr = nullptr;
        if (hipHostGetDevicePointer(&dptr, hflag, 0) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        *(volatile int32_t *)hflag = 0;
        for (Job &J : c.jobs) J.hstop = static_cast<int32_t *>(dptr);
        ahead = true;
    }
    nmf_status sync_check(bool &done) {
        DevState hs;
        nmf_status e = read_state(c, hs);
        done = e == NMF_OK && hs.stop != 0;
        return e;
    }
    nmf_status ahead_check(bool &done) {
        nmf_plan_t plan = c.plan;
        PollPool &pp = plan->p.poll;
        hipEvent_t ev = nullptr;
        {
            std::lock_guard<std::mutex> lk(pp.mu);
            if (!pp.events.empty()) {
                ev = pp.events.back();
                pp.events.pop_back();
            }
        }
        if (!ev) NMF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        inflight.push_back(ev);
        NMF_HIP(hipEventRecord(ev, c.s));
        if (inflight.size() > 1) {
            hipEvent_t old = inflight.front();
            inflight.erase(inflight.begin());
            {
                std::lock_guard<std::mutex> lk(pp.mu);
                pp.events.push_back(old);
            }
            NMF_HIP(hipEventSynchronize(old));
        }
        done = *(volatile int32_t *)hflag != 0;
        return NMF_OK;
    }
    // Call after each iteration that counts towards the check interval.
    nmf_status tick(bool &done) {
        if (++since < c.p->d.check_every) return NMF_OK;
        since = 0;
        return now(done);
    }
    nmf_status now(bool &done) { return ahead ? ahead_check(done) : sync_check(done); }
};

}  // namespace

nmf_status solve_on(nmf_plan_t plan, const float *dM, float *dV, float *dW, int32_t iters,
                    void *dWorkspace, hipStream_t s, nmf_result *hOut, bool profile,
                    bool lookahead, float *dB, float *dC) {
    const Plan &p = plan->p;
    const bool ntf = p.d.ntf_k > 0;
    if (ntf != (dB != nullptr && dC != nullptr))
        return fail(plan, NMF_E_ARG, ntf ? "an NTF plan (ntf_k > 0) is solved by nmf_ntf_solve"
                                         : "nmf_ntf_solve needs a plan with ntf_k > 0");
    if (ntf) dW = at<float>(static_cast<char *>(dWorkspace), p.ws.off_ntfW);
    Ctx c = make_ctx(plan, dM, dV, dW, dWorkspace, s);
    c.ntfB = dB;
    c.ntfC = dC;
    c.prof = profile;
    Poller poller(c);
    if (lookahead && p.d.tol > 0.0) poller.enable();
    NMF_HIP(launch_state_reset(c.st, s));
    nmf_status st;
    if (p.d.check_input && (st = check_input(c)) != NMF_OK) return st;
    if ((st = prepare_levels(c)) != NMF_OK) return st;
    if ((st = prepare_bf16(c)) != NMF_OK) return st;
    if ((st = upload_jobs(c)) != NMF_OK) return st;
    if ((st = init_w(c)) != NMF_OK) return st;

    const bool use_tol = p.d.tol > 0.0;
    const bool bf16 = p.d.prec == NMF_BF16;
    bool done = false;
    for (const Step &stp : make_schedule(p.d.cycle, p.d.levels, iters, p.d.two_sided ? 8 : 4)) {
        if (done) break;
        const int d = stp.depth;
        if (stp.kind == 1) {
            NMF_LAUNCH(K_RESTRICT, launch_restrict(p.d.xfer, p.lv[d].h, p.lv[d].w, p.d.r, c.V[d],
                                                   p.lv[d].m, c.V[d + 1], c.stop, s));
            if (p.d.two_sided && (st = transfer_w(c, d, true)) != NMF_OK) return st;
        } else if (stp.kind == 2) {
            NMF_LAUNCH(K_PROLONG, launch_prolong(p.d.xfer, p.lv[d].h, p.lv[d].w, p.d.r, c.V[d + 1],
                                                 c.V[d], c.stop, s));
            if (p.d.two_sided && (st = transfer_w(c, d, false)) != NMF_OK) return st;
        } else {
            for (int i = 0; i < stp.count && !done; ++i) {
                if ((st = sweep(c, d)) != NMF_OK) return st;
                if (use_tol && d == 0 && (st = poller.tick(done)) != NMF_OK) return st;
            }
        }
    }
    // BF16 mode: finish on the finest level in FP32 (the tolerance applies to
    // these iterations only)
    for (int i = 0; bf16 && i < p.d.refine_iters && !done; ++i) {
        if ((st = sweep(c, 0, true)) != NMF_OK) return st;
        if (use_tol && (st = poller.tick(done)) != NMF_OK) return st;
    }
    if (use_tol && !done) {
        if ((st = poller.now(done)) != NMF_OK) return st;
        for (int i = 0; i < p.d.max_fine_iters && !done; ++i) {
            if ((st = sweep(c, 0, bf16)) != NMF_OK) return st;
            if ((st = poller.tick(done)) != NMF_OK) return st;
        }
    }
    return finish(c, hOut);
}

}  // namespace nmf

extern "C" {

nmf_status nmf_query_log(nmf_plan_t plan, const void *dWorkspace, void *stream, double *rel_err,
                         int32_t *depth, int32_t cap) {
    if (!plan || !dWorkspace) return fail(plan, NMF_E_ARG, "null argument");
    const Plan &p = plan->p;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const char *ws = static_cast<const char *>(dWorkspace);
    DevState hs;
    NMF_HIP(hipMemcpyAsync(&hs, ws + p.ws.off_state, sizeof hs, hipMemcpyDeviceToHost, s));
    NMF_HIP(hipStreamSynchronize(s));
    int32_t n = hs.log_len < p.d.log_cap ? hs.log_len : p.d.log_cap;
    if (n > cap) n = cap;
    if (n > 0 && rel_err)
        NMF_HIP(hipMemcpyAsync(rel_err, ws + p.ws.off_log, sizeof(double) * n,
                               hipMemcpyDeviceToHost, s));
    if (n > 0 && depth)
        NMF_HIP(hipMemcpyAsync(depth, ws + p.ws.off_logdepth, sizeof(int32_t) * n,
                               hipMemcpyDeviceToHost, s));
    NMF_HIP(hipStreamSynchronize(s));
    return NMF_OK;
}

nmf_status nmf_iterate(nmf_plan_t plan, const float *dM, float *dV, float *dW, int32_t count,
                       void *dWorkspace, void *stream, double *hRelErr) {
    if (!plan || !dM || !dV || !dW || !dWorkspace || count < 0)
        return fail(plan, NMF_E_ARG, "bad argument");
    if (plan->p.d.ntf_k > 0)
        return fail(plan, NMF_E_ARG, "an NTF plan (ntf_k > 0) is solved by nmf_ntf_solve");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ctx c = make_ctx(plan, dM, dV, dW, dWorkspace, s);
    NMF_HIP(launch_state_reset(c.st, s));
    nmf_status st;
    if ((st = prepare_levels(c)) != NMF_OK) return st;
    if ((st = prepare_bf16(c)) != NMF_OK) return st;
    if ((st = upload_jobs(c)) != NMF_OK) return st;
    if ((st = init_w(c)) != NMF_OK) return st;
    for (int i = 0; i < count; ++i)
        if ((st = sweep(c, 0)) != NMF_OK) return st;
    nmf_result res;
    st = finish(c, &res);
    if (hRelErr) *hRelErr = res.rel_err;
    return st;
}

nmf_status nmf_profile(nmf_plan_t plan, uint32_t mask) {
    if (!plan) return fail(plan, NMF_E_ARG, "null plan");
    plan->p.prof.mask = mask;
    return NMF_OK;
}

nmf_status nmf_profile_read(nmf_plan_t plan, int64_t *counts, double *total_ms, int32_t cap,
                            int32_t reset) {
    if (!plan) return fail(plan, NMF_E_ARG, "null plan");
    Profiler &pf = plan->p.prof;
    std::lock_guard<std::mutex> lk(pf.mu);
    for (int k = 0; k < K_NUM_KINDS && k < cap; ++k) {
        if (counts) counts[k] = pf.counts[k];
        if (total_ms) total_ms[k] = pf.ms[k];
    }
    if (reset) {
        for (int k = 0; k < K_NUM_KINDS; ++k) {
            pf.counts[k] = 0;
            pf.ms[k] = 0.0;
        }
    }
    return NMF_OK;
}

nmf_status nmf_products(nmf_plan_t plan, const float *dM, const float *dV, const float *dW,
                        float *dA, float *dC, void *dWorkspace, void *stream) {
    if (!plan || !dM || !dV || !dW || !dA || !dC || !dWorkspace)
        return fail(plan, NMF_E_ARG, "bad argument");
    const Plan &p = plan->p;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ctx c = make_ctx(plan, dM, const_cast<float *>(dV), const_cast<float *>(dW), dWorkspace, s);
    Job &J = c.jobs[0];
    J.A = dA;
    J.C = dC;
    J.Ad = J.Cd = nullptr;
    J.Cr = nullptr;   // no D-reduction launch here: the W update sums the partials
    NMF_HIP(launch_state_reset(c.st, s));
    NMF_HIP(launch_make_wt(dW, p.d.n, p.d.r, p.rpad, c.Wt, s));
    nmf_status st = upload_jobs(c);
    if (st != NMF_OK) return st;
    NMF_HIP(launch_apass_jobs(2, J.rpad, J.tm, c.djobs, nullptr, apass_grid_single(J.nA),
                              apass_lds_bytes(J.rpad, J.tm, 2), s));
    NMF_HIP(launch_cpass_jobs(J.rpad, J.wc, c.djobs, nullptr, cpass_grid_single(J.nCx, J.chunks),
                              s));
    NMF_HIP(launch_cfinal_jobs(2, J.rpad, J.cf, c.djobs, nullptr, J.nFb,
                               cfinal_lds_bytes(J.rpad, 2, J.cf), s));
    NMF_HIP(hipStreamSynchronize(s));
    return NMF_OK;
}

nmf_status nmf_restrict(int32_t xfer, int32_t h, int32_t w, int64_t ncols, const float *dX,
                        int64_t ldx, float *dY, void *stream) {
    nmf_plan_t plan = nullptr;
    if (!dX || !dY || h < 2 || w < 2 || ncols < 0 || ldx < (int64_t)h * w ||
        (xfer != NMF_XFER_FW && xfer != NMF_XFER_BLOCK2))
        return fail(nullptr, NMF_E_ARG, "bad argument");
    NMF_HIP(launch_restrict(xfer, h, w, ncols, dX, ldx, dY, nullptr,
                            static_cast<hipStream_t>(stream)));
    return NMF_OK;
}

nmf_status nmf_prolong(int32_t xfer, int32_t h, int32_t w, int64_t ncols, const float *dY,
                       float *dX, void *stream) {
    nmf_plan_t plan = nullptr;
    if (!dX || !dY || h < 2 || w < 2 || ncols < 0 ||
        (xfer != NMF_XFER_FW && xfer != NMF_XFER_BLOCK2))
        return fail(nullptr, NMF_E_ARG, "bad argument");
    NMF_HIP(launch_prolong(xfer, h, w, ncols, dY, dX, nullptr, static_cast<hipStream_t>(stream)));
    return NMF_OK;
}

nmf_status nmf_gram(int32_t r, int64_t L, const float *dX, int64_t ldx, double *dG,
                    void *dWorkspace, size_t ws_bytes, void *stream) {
    nmf_plan_t plan = nullptr;
    if (!dX || !dG || !dWorkspace || r < 1 || r > kMaxRank || L < 1 || ldx < L)
        return fail(nullptr, NMF_E_ARG, "bad argument");
    const int rpad = (r + 15) / 16 * 16;
    int64_t parts = (L + 63) / 64;
    if (parts > 256) parts = 256;
    int64_t chunk = ((L + parts - 1) / parts + 63) / 64 * 64;
    parts = (L + chunk - 1) / chunk;
    if ((size_t)parts * rpad * rpad * sizeof(double) > ws_bytes)
        return fail(nullptr, NMF_E_NOMEM, "gram workspace too small");
    NMF_HIP(launch_gram(rpad, r, L, dX, ldx, (int)parts, chunk, static_cast<double *>(dWorkspace),
                        dG, nullptr, nullptr, static_cast<hipStream_t>(stream)));
    return NMF_OK;
}

}  // extern "C"
