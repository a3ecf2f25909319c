// Host-side planner: level hierarchy, cycle schedule and workspace layout.
#include <algorithm>
#include <cstdio>
#include <functional>

#include "nmf_internal.h"

namespace nmf {

namespace {

// Exact nonnegative rational (budgets of Alg. 4-6 are T * 3^a / 4^b).
struct Rat {
    int64_t num, den;
};

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a < 0 ? -a : a;
}

Rat mk(int64_t num, int64_t den) {
    const int64_t g = gcd64(num, den);
    return g ? Rat{num / g, den / g} : Rat{0, 1};
}
Rat mul(Rat a, int64_t p, int64_t q) { return mk(a.num * p, a.den * q); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Schedules of the cycles, the budget counted in finest-iteration equivalents:
// Run(d, t) performs floor(t * ratio^d) iterations at depth d (depth 0 =
// finest; ratio 4, or 8 for two-sided hierarchies) and zero-iteration runs
// are dropped.  Every cycle over L > 1 levels with budget t has the same
// shape: a share of t run at the current level, a restriction, one or more
// visits of the next level with shares of t, a prolongation, and a closing
// share, which is a run or (full multigrid) a V-cycle over the same levels.
// The table holds each cycle's shares: nested iteration (Alg. 4) and the
// V-cycle (Alg. 5) give the coarser levels 1/4 of t (Table 1), full
// multigrid (Alg. 6) descends first and closes with a V-cycle of 3t/4, the
// W-cycle spends the coarse quarter in two visits of t/8.
namespace {

struct CycleRule {
    Rat pre;              // run at the current level before descending
    int coarse_cycle;     // cycle used on the next level
    int visits;           // consecutive visits of the next level
    Rat coarse;           // share of t per visit
    bool close_vcycle;    // closing share: V-cycle over the same levels (else a run)
    Rat close;            // closing share of t
};

const CycleRule &cycle_rule(int cycle) {
    static const CycleRule kNI{{0, 1}, NMF_NI, 1, {1, 4}, false, {3, 4}};
    static const CycleRule kVC{{1, 4}, NMF_VC, 1, {1, 4}, false, {1, 2}};
    static const CycleRule kFMG{{0, 1}, NMF_FMG, 1, {1, 4}, true, {3, 4}};
    static const CycleRule kWC{{1, 4}, NMF_WC, 2, {1, 8}, false, {1, 2}};
    switch (cycle) {
        case NMF_VC: return kVC;
        case NMF_FMG: return kFMG;
        case NMF_WC: return kWC;
        default: return kNI;
    }
}

}  // namespace

std::vector<Step> make_schedule(int cycle, int levels, int64_t iters, int ratio) {
    std::vector<Step> out;
    auto run = [&](int d, Rat t) {
        int64_t scale = 1;
        for (int i = 0; i < d; ++i) scale *= ratio;
        const int64_t c = (t.num * scale) / t.den;
        if (c > 0) out.push_back(Step{0, d, (int32_t)c});
    };
    auto share = [](Rat t, Rat f) { return mul(t, f.num, f.den); };
    std::function<void(int, int, Rat, int)> cyc = [&](int cy, int L, Rat t, int d) {
        if (L == 1) return run(d, t);
        const CycleRule &R = cycle_rule(cy);
        if (R.pre.num > 0) run(d, share(t, R.pre));
        out.push_back(Step{1, d, 0});
        for (int v = 0; v < R.visits; ++v) cyc(R.coarse_cycle, L - 1, share(t, R.coarse), d + 1);
        out.push_back(Step{2, d, 0});
        if (R.close_vcycle) cyc(NMF_VC, L, share(t, R.close), d);
        else run(d, share(t, R.close));
    };
    cyc(cycle, levels, Rat{iters, 1}, 0);
    return out;
}

nmf_status build_plan(const nmf_desc &d0, Plan &p, std::string &err) {
    nmf_desc d = d0;
    char buf[256];
    if (d.algo < NMF_HALS || d.algo > NMF_KL || d.cycle < NMF_NI || d.cycle > NMF_WC ||
        d.xfer < NMF_XFER_FW || d.xfer > NMF_XFER_BLOCK2 || d.prec < NMF_FP32 || d.prec > NMF_BF16) {
        err = "unknown algo / cycle / xfer / prec value";
        return NMF_E_ARG;
    }
    if (d.ldm == 0) d.ldm = d.m;
    if (d.check_every <= 0) d.check_every = 8;
    if (d.log_cap <= 0) d.log_cap = 4096;
    if (d.max_fine_iters < 0 || d.refine_iters < 0 || !(d.tol >= 0.0)) {
        err = "negative max_fine_iters / refine_iters / tol";
        return NMF_E_ARG;
    }
    if (d.prec == NMF_BF16 && d.algo == NMF_ANLS) {
        err = "BF16 precision is available for HALS and MU";
        return NMF_E_ARG;
    }
    if (d.ntf_k < 0 || (d.ntf_k > 0 && (d.algo != NMF_HALS || d.prec != NMF_FP32 ||
                                         d.two_sided != 0))) {
        err = "NTF (ntf_k > 0) runs HALS in FP32 on one-sided hierarchies";
        return NMF_E_ARG;
    }
    if (d.ntf_k > 0 && (d.n % d.ntf_k != 0 || d.ntf_k > 16384)) {
        err = "NTF: n must be a multiple of ntf_k = K, and K <= 16384";
        return NMF_E_SHAPE;
    }
    if (d.algo == NMF_KL && (d.prec != NMF_FP32 || d.two_sided != 0)) {
        err = "the KL objective runs in FP32 on one-sided hierarchies";
        return NMF_E_ARG;
    }
    if (d.two_sided != 0 && d.two_sided != 1) {
        err = "two_sided must be 0 or 1";
        return NMF_E_ARG;
    }
    if (d.two_sided && d.prec != NMF_FP32) {
        err = "two-sided hierarchies run in FP32";
        return NMF_E_ARG;
    }
    if (d.h < 1 || d.w < 1 || d.m != (int64_t)d.h * d.w) {
        snprintf(buf, sizeof buf, "m (%lld) must equal h*w (%d*%d)", (long long)d.m, d.h, d.w);
        err = buf;
        return NMF_E_SHAPE;
    }
    if (d.n < 1 || d.ldm < d.m) {
        err = "n must be >= 1 and ldm >= m";
        return NMF_E_SHAPE;
    }
    if (d.r < 1 || d.r > kMaxRank) {
        err = "r must be in [1, 64]";
        return NMF_E_SHAPE;
    }
    if (d.levels < 1 || d.levels > kMaxLevels) {
        err = "levels must be in [1, 12]";
        return NMF_E_SHAPE;
    }
    p.d = d;
    p.rpad = (d.r + 15) / 16 * 16;
    // Tile shapes: latency tiles (row-split C-pass, narrow W-update tiles) for
    // problems large enough to run alone, throughput tiles below.  Wide
    // problems keep 16-column W-update tiles (n = 2000: 125 blocks of 16
    // columns beat 500 of 4; n = 400: 100 blocks of 4 beat 25 of 16).
    const int32_t tiles = d.tile_cfg & 0xffff;
    if ((d.tile_cfg & ~(NMF_TILE_GROUPED | 0xffff)) != 0) {
        err = "tile_cfg: unknown flag bits (only NMF_TILE_GROUPED is defined above bit 15)";
        return NMF_E_ARG;
    }
    p.grouped = (d.tile_cfg & NMF_TILE_GROUPED) != 0;
    if (tiles == 0) {
        const bool big = d.m >= 8192;
        p.wc = big ? (p.rpad <= 32 ? 4 : 2) : 1;
        p.cf = big && d.n < 1536 ? 4 : 16;
    } else {
        p.wc = tiles & 0xff;
        p.cf = (tiles >> 8) & 0xff;
        if ((p.wc != 1 && p.wc != 2 && p.wc != 4) || (p.cf != 4 && p.cf != 16)) {
            err = "tile_cfg must be 0 or NMF_TILE(wc, cf) with wc in {1, 2, 4}, cf in {4, 16} "
                  "(optionally with NMF_TILE_GROUPED)";
            return NMF_E_ARG;
        }
    }
    p.lv.clear();
    int h = d.h, w = d.w;
    int64_t nl = d.n;
    for (int l = 0; l < d.levels; ++l) {
        if (l > 0) {
            if (h < 2 || w < 2) {
                snprintf(buf, sizeof buf, "level %d: cannot restrict a %dx%d grid", l, h, w);
                err = buf;
                return NMF_E_SHAPE;
            }
            if (d.two_sided && nl < 2) {
                snprintf(buf, sizeof buf, "level %d: cannot restrict %lld columns", l,
                         (long long)nl);
                err = buf;
                return NMF_E_SHAPE;
            }
            h = (h + 1) / 2;
            w = (w + 1) / 2;
            if (d.two_sided) nl = (nl + 1) / 2;
        }
        LevelInfo li{};
        li.h = h;
        li.w = w;
        li.m = (int64_t)h * w;
        li.n = nl;
        if (d.algo == NMF_ANLS && li.m < d.r) {
            snprintf(buf, sizeof buf,
                     "ANLS: level %d has %lld pixels < r = %d (singular V^T V)", l,
                     (long long)li.m, d.r);
            err = buf;
            return NMF_E_SHAPE;
        }
        p.lv.push_back(li);
    }
    if (p.num_cu <= 0) p.num_cu = 256;

    // Split of the length-m reductions.  Target about one block per CU for
    // V^T M (deterministic split-m partials) and at most 256 Gram partials.
    // Grouped plans keep chunks of at least 512 rows: in a batch the problems
    // fill the chip, and shorter chunks write FP64 partials that outweigh M
    // (chunks * 8r bytes per column against 4m).  (512-problem batch: 114.9 ms
    // with one block per CU per problem, 107.7 ms with 512-row chunks, 108.3
    // with 256, 111.7 with 1024; 64-row A-pass tiles from m = 1024 on top made
    // it 127.3 ms.  Alone, the 64x64 two-sided solve went from 0.84 to 0.93 ms.)
    size_t max_cp = 0, max_gp = 0, max_ap = 0;
    for (auto &li : p.lv) {
        li.atm = li.m >= 32768 ? 64 : 16;
        li.gseg = gram_w_segments(li.n);
        const int64_t ntiles = (li.n + 63) / 64;
        int64_t chunks = std::max<int64_t>(1, p.num_cu / std::max<int64_t>(1, ntiles));
        chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, (li.m + 63) / 64));
        if (p.grouped) chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, li.m / 512));
        int64_t chunk = (li.m + chunks - 1) / chunks;
        // FP32: whole 16-row steps for each of up to 4 row groups of a C-pass
        // tile; BF16: see kBfPad
        const int64_t q = d.prec == NMF_BF16 ? kBfPad : 64;
        chunk = (chunk + q - 1) / q * q;
        li.cp_chunk = chunk;
        li.cp_chunks = (int32_t)((li.m + chunk - 1) / chunk);
        max_cp = std::max<size_t>(max_cp, (size_t)li.cp_chunks);
        // FP32 streaming C-pass (large levels): about two blocks per CU
        // wide coarse levels stream only in plans whose finest level does
        // (plans that never stream give the same bits alone and in a batch)
        li.fstream = (d.algo == NMF_HALS || d.algo == NMF_MU) && d.ntf_k == 0 && li.m % 4 == 0 &&
                     (li.m >= kFStreamMinRows ||
                      (p.lv[0].m >= kFStreamMinRows && li.m >= kFStreamWideRows &&
                       li.n >= kFStreamWideCols));
        li.ftm = li.m >= 65536 ? 128 : 64;
        li.aks = 1;
        if (li.fstream) {
            // A-pass: split the n-reduction until there are about as many
            // blocks as CUs, into at most 8 parts of at least 4 stages of 16
            // columns
            const int64_t tiles = (li.m + li.ftm - 1) / li.ftm;
            const int64_t stages = (li.n + 15) / 16;
            int64_t ks = (p.num_cu + tiles - 1) / tiles;
            ks = std::min<int64_t>({ks, std::max<int64_t>(1, stages / 4), 8});
            li.aks = li.ftm == 64 ? (int32_t)std::max<int64_t>(1, ks) : 1;   // k_afinal_s32: 64-row tiles
            if (li.aks > 1)
                max_ap = std::max<size_t>(max_ap, (size_t)li.aks * tiles * li.ftm * p.rpad);
            const int64_t ncx = (li.n + 127) / 128;
            int64_t sc = std::max<int64_t>(1, 2 * p.num_cu / ncx);
            sc = std::min<int64_t>(sc, std::max<int64_t>(1, li.m / 64));
            int64_t sch = (li.m + sc - 1) / sc;
            sch = (sch + 63) / 64 * 64;
            li.fcp_chunk = sch;
            li.fcp_chunks = (int32_t)((li.m + sch - 1) / sch);
            max_cp = std::max<size_t>(max_cp, (size_t)li.fcp_chunks);
        }
        // streaming C-pass (large BF16 levels): about one block per CU (at
        // m = 65536, n = 2000 the C-pass took 75 us with 512 blocks of half
        // the rows, 64 us with 256; more DMA stages changed neither)
        li.stream = d.prec == NMF_BF16 && li.m >= kStreamMinRows;
        if (li.stream) {
            const int64_t ncx = (li.n + 255) / 256;
            int64_t sc = std::max<int64_t>(1, p.num_cu / ncx);
            sc = std::min<int64_t>(sc, std::max<int64_t>(1, (li.m + 255) / 256));
            int64_t sch = (li.m + sc - 1) / sc;
            sch = bf_pad(sch);
            li.scp_chunk = sch;
            li.scp_chunks = (int32_t)((li.m + sch - 1) / sch);
            max_cp = std::max<size_t>(max_cp, (size_t)li.scp_chunks);
        }
        int64_t gp = std::min<int64_t>(256, (li.m + 63) / 64);
        int64_t gc = (li.m + gp - 1) / gp;
        gc = (gc + 63) / 64 * 64;
        li.gram_chunk = gc;
        li.gram_parts = (int32_t)((li.m + gc - 1) / gc);
        max_gp = std::max<size_t>(max_gp, (size_t)li.gram_parts);
        gp = std::min<int64_t>(256, (li.n + 63) / 64);
        gc = (li.n + gp - 1) / gp;
        gc = (gc + 63) / 64 * 64;
        li.gram_w_chunk = gc;
        li.gram_w_parts = (int32_t)((li.n + gc - 1) / gc);
        max_gp = std::max<size_t>(max_gp, (size_t)li.gram_w_parts);
    }
    p.gram_w_chunk = p.lv[0].gram_w_chunk;
    p.gram_w_parts = p.lv[0].gram_w_parts;

    Workspace &ws = p.ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t r = d.r, n = d.n, rr = r * r, rp2 = (size_t)p.rpad * p.rpad;
    ws.off_state = take(256);
    ws.off_log = take(sizeof(double) * d.log_cap);
    ws.off_logdepth = take(sizeof(int32_t) * d.log_cap);
    ws.off_norm = take(sizeof(double) * d.levels);
    ws.off_nparts = take(sizeof(double) * kNormParts * d.levels);
    ws.off_Bd = take(sizeof(double) * rr);
    ws.off_Dd = take(sizeof(double) * rr);
    ws.off_Bf = take(sizeof(float) * rr);
    ws.off_Df = take(sizeof(float) * rr);
    if (d.algo == NMF_KL) {
        ws.off_klw = take(sizeof(double) * p.rpad);
        ws.off_klwp = take(sizeof(double) * p.rpad * (size_t)kl_col_blocks(d.n));
        ws.off_klvp = take(sizeof(double) * p.rpad * max_cp);
        ws.off_kld = take(sizeof(double) * (size_t)kl_row_blocks(d.m));
        ws.off_klm = take(sizeof(double) * d.levels);
    } else {
        ws.off_klw = ws.off_klwp = ws.off_klvp = ws.off_kld = ws.off_klm = 0;
    }
    ws.gparts_cap = max_gp * rp2;
    ws.off_gparts = take(sizeof(double) * ws.gparts_cap);
    // C-pass partials; also the split A-pass's partial rows of A (FP32
    // streaming levels with aks > 1), which are used up before the C-pass runs
    ws.off_cparts = take(sizeof(double) * std::max<size_t>(max_cp * r * n, max_ap));
    // V^T M summed over the chunks (single solves of the W-update paths)
    ws.off_Cr = d.algo != NMF_KL ? take(sizeof(double) * r * n) : 0;
    ws.off_bparts = take(sizeof(double) * kGramSegMax * gram_tiles(p.rpad) * 256);
    ws.rparts_cap = std::max<size_t>({(size_t)cpass_final_blocks(d.n),
                                      (size_t)nnls_cols_blocks(d.n), (size_t)1024});
    ws.off_rparts = take(sizeof(double) * ws.rparts_cap);
    if (d.algo == NMF_ANLS) {
        ws.off_A = take(sizeof(double) * (size_t)d.m * r);   // FP64 right-hand sides
        ws.off_C = take(sizeof(double) * r * n);
    } else if (d.ntf_k > 0) {
        ws.off_A = 0;
        ws.off_C = take(sizeof(double) * r * n);             // A^T X_(1)
    } else {
        ws.off_A = ws.off_C = 0;
    }
    if (d.ntf_k > 0) {
        ws.off_ntfW = take(sizeof(float) * r * n);
        ws.off_ntfG = take(sizeof(double) * 3 * rr);
    } else {
        ws.off_ntfW = ws.off_ntfG = 0;
    }
    size_t tmp_elems = 0;
    for (size_t l = 1; l < p.lv.size(); ++l) {
        p.lv[l].off_M = take(sizeof(float) * (size_t)p.lv[l].m * p.lv[l].n);
        p.lv[l].off_V = take(sizeof(float) * (size_t)p.lv[l].m * r);
        if (d.two_sided) {
            p.lv[l].off_W = take(sizeof(float) * r * (size_t)p.lv[l].n);
            tmp_elems = std::max<size_t>(tmp_elems, (size_t)p.lv[l].m * p.lv[l - 1].n);
        }
    }
    ws.off_tmpM = tmp_elems ? take(sizeof(float) * tmp_elems) : 0;
    ws.off_Wt = take(sizeof(float) * n * p.rpad);
    ws.off_Dp = take(sizeof(double) * max_cp * rp2);
    ws.off_jobs = take(sizeof(Job) * (p.lv.size() + 1));   // + FP32 refinement job
    ws.off_Wb = 0;
    const int64_t npad = bf_pad(d.n);
    if (d.prec == NMF_BF16) {
        // BF16 operand copies (job.h): per level M in the A-pass (K-packed) and
        // C-pass (column-major, stride mpad) layouts and V; W once
        for (auto &li : p.lv) {
            li.mpad = bf_pad(li.m);
            li.off_Mbp = take(sizeof(uint16_t) * (size_t)((li.m + 15) / 16 * 16) * npad);
            li.off_Mbc = take(sizeof(uint16_t) * (size_t)li.mpad * (size_t)((n + 15) / 16 * 16));
            li.off_Vb = take(sizeof(uint16_t) * (size_t)li.mpad * p.rpad);
        }
        ws.off_Wb = take(sizeof(uint16_t) * (size_t)p.rpad * npad);
    }
    ws.total = off;
    return NMF_OK;
}

}  // namespace nmf
