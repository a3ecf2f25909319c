// Host check of the planner and the schedule builder, built with
// AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): plans a seeded
// set of valid and invalid problem descriptions and checks that
//   * an invalid description is rejected with a message and a valid one planned,
//   * every workspace region of a plan starts inside the workspace,
//   * the level sizes halve (rounding up) and stay >= 1,
//   * every schedule entry names a depth inside the hierarchy and a count >= 0,
//     and transfers move V one depth at a time.
// Exit status 0 when every check holds; the sanitizers abort on any invalid
// memory access or undefined operation.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "nmf_internal.h"

namespace nmf {
// Launch-size helpers the planner sizes partial buffers with; the real ones
// live beside the kernels.  The same formulas: one block per 4 columns, the
// NNLS column launch capped at 1024 blocks, KL blocks of 16 rows / 64 columns.
int cpass_final_blocks(int64_t n) { return (int)((n + 3) / 4); }
int kl_row_blocks(int64_t m) { return (int)((m + 15) / 16); }
int kl_col_blocks(int64_t n) { return (int)((n + 63) / 64); }
int nnls_cols_blocks(int64_t n) {
    int64_t b = (n + 3) / 4;
    return (int)(b > 1024 ? 1024 : (b < 1 ? 1 : b));
}
}  // namespace nmf

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
uint64_t next() {   // splitmix64
    uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
int64_t pick(int64_t lo, int64_t hi) { return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1)); }

int failures = 0;
void check(bool ok, const char *what, const nmf_desc &d) {
    if (ok) return;
    ++failures;
    std::fprintf(stderr, "FAIL %s: h=%d w=%d n=%lld r=%d levels=%d algo=%d cycle=%d prec=%d two=%d\n",
                 what, d.h, d.w, (long long)d.n, d.r, d.levels, d.algo, d.cycle, d.prec,
                 d.two_sided);
}

}  // namespace

int main() {
    int planned = 0, rejected = 0, schedules = 0;
    for (int trial = 0; trial < 4000; ++trial) {
        nmf_desc d = {};
        d.h = (int32_t)pick(2, 300);
        d.w = (int32_t)pick(2, 300);
        d.m = (int64_t)d.h * d.w;
        d.n = pick(2, 5000);
        d.r = (int32_t)pick(1, 64);
        int deep = 1;   // levels the grid allows: every restricted side >= 2
        for (int s = d.h < d.w ? d.h : d.w; s >= 2 && deep < 12; s = (s + 1) / 2) ++deep;
        d.levels = (int32_t)pick(1, deep - 1 > 1 ? deep - 1 : 1);
        d.algo = (int32_t)pick(0, 3);
        d.cycle = (int32_t)pick(0, 3);
        d.xfer = (int32_t)pick(0, 1);
        d.two_sided = (int32_t)(next() % 4 == 0);
        if (d.algo == NMF_KL) d.two_sided = 0;
        d.prec = (int32_t)(d.algo < NMF_ANLS && !d.two_sided && next() % 3 == 0);
        d.tol = (next() & 1) ? 1e-2 : 0.0;
        d.refine_iters = d.prec ? (int32_t)pick(0, 4) : 0;
        d.tile_cfg = (next() % 4 == 0) ? NMF_TILE(1 << pick(0, 2), pick(0, 1) ? 16 : 4) : 0;
        if (next() % 8 == 0) {   // NTF: n = J K
            d.algo = NMF_HALS;
            d.prec = NMF_FP32;
            d.two_sided = 0;
            d.ntf_k = (int32_t)pick(1, 64);
            d.n = d.ntf_k * pick(1, 80);
        }
        // one field in eight goes out of range
        switch (next() % 16) {
            case 0: d.r = (int32_t)pick(65, 200); break;
            case 1: d.levels = 0; break;
            case 2: d.m += 1; break;
            case 3: d.algo = 7; break;
            case 4: d.cycle = -1; break;
            case 5: d.n = 0; break;
            case 6: d.two_sided = 2; break;
            case 7: d.tol = -1.0; break;
            default: break;
        }
        nmf::Plan p;
        std::string err;
        const nmf_status st = nmf::build_plan(d, p, err);
        if (st != NMF_OK) {
            check(!err.empty(), "rejection without a message", d);
            ++rejected;
            continue;
        }
        ++planned;
        const nmf::Workspace &w = p.ws;
        const size_t offs[] = {w.off_state, w.off_log, w.off_logdepth, w.off_norm, w.off_nparts,
                               w.off_Bd, w.off_Bf, w.off_Dd, w.off_Df, w.off_gparts,
                               w.off_cparts, w.off_rparts, w.off_A, w.off_C, w.off_Wb,
                               w.off_Wt, w.off_Dp, w.off_jobs, w.off_tmpM, w.off_klw,
                               w.off_klwp, w.off_klvp, w.off_kld, w.off_klm, w.off_ntfW,
                               w.off_ntfG};
        for (size_t o : offs) check(o <= w.total, "workspace region past the end", d);
        check((int)p.lv.size() == d.levels, "level count", d);
        for (size_t l = 0; l < p.lv.size(); ++l) {
            const nmf::LevelInfo &li = p.lv[l];
            check(li.h >= 1 && li.w >= 1 && li.m == (int64_t)li.h * li.w, "level shape", d);
            check(li.n >= 1, "level columns", d);
            if (l > 0) {
                const nmf::LevelInfo &up = p.lv[l - 1];
                check(li.h == (up.h + 1) / 2 && li.w == (up.w + 1) / 2, "level halving", d);
                check(li.n == (d.two_sided ? (up.n + 1) / 2 : up.n), "column halving", d);
                check(li.off_M <= w.total && li.off_V <= w.total, "level region past the end", d);
            }
        }
        for (int cyc = 0; cyc < 4; ++cyc) {
            const int64_t iters = pick(0, 64);
            const auto sched = nmf::make_schedule(cyc, d.levels, iters, d.two_sided ? 8 : 4);
            ++schedules;
            int depth = 0;
            for (const nmf::Step &s : sched) {
                check(s.depth >= 0 && s.depth < d.levels && s.count >= 0, "schedule entry", d);
                if (s.kind == 1) {
                    check(s.depth == depth && depth + 1 < d.levels, "restriction step", d);
                    depth = s.depth + 1;
                } else if (s.kind == 2) {
                    check(s.depth + 1 == depth, "prolongation step", d);
                    depth = s.depth;
                } else {
                    check(s.depth == depth, "run at the current depth", d);
                }
            }
            check(depth == 0, "schedule ends on the finest level", d);
        }
    }
    std::printf("planned %d, rejected %d, schedules %d, failures %d\n", planned, rejected,
                schedules, failures);
    return failures == 0 ? 0 : 1;
}
