#!/usr/bin/env python3
"""Benchmark of the multilevel NMF hot path on one MI355X.

One step = one complete multilevel solve to the accuracy target (restriction
of M to every level, the NMF sweeps at every level, the prolongations, the
per-iteration residual and the tolerance stop) on a synthetic planted-blob
workload whose inputs are already resident in device memory.  The same target
is also reached by plain single-level FP32 NMF on the same GPU.

Prints ONE JSON line.  Workloads (seeded, synthetic):
  orl   (default) 112x92 images, n=400, r=40, 3 levels of full weighting
  small           16x16 images, n=500, r=10, 2 levels of 2x2 block restriction
  large           256x256 images, n=2000, r=50, 4 levels of full weighting
  spectral        64x64 maps x 256 smooth bands, r=12, 3 two-sided levels (the band
                  count halves with the grid); also times the one-sided hierarchy
  batch           512 uneven problems (sides 16-64, n 100-2000, r 5-40), 3 levels,
                  HALS, one batched solve (grouped launches) per step
  serve           Poisson arrivals (default 200 req/s) of problems drawn like
                  `batch`, served with continuous batching; p50/p99 latency
Target: rel_err <= eps_E + tau, eps_E the exact planted-noise level of the
instance (the literal 1e-2 lies below the rank-r error floor of this data).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix
PEAK_BF16_MFMA_TFLOPS = 2500.0  # MI355X dense BF16 matrix
PEAK_FP64_VALU_TFLOPS = 78.6   # MI355X FP64 vector

EXTRA_WORKLOADS = ("batch", "serve", "tensor")

# HBM traffic per launch (bytes) of the sweep kernels, by (workload, precision),
# kernel kind and level size m: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# passes (KiB per dispatch, averaged over the dispatches that ran: launches
# issued past a stop return at once and are left out), scaled by what the
# same counters read for a 256 MiB device-to-device copy (FETCH_SIZE x2.0,
# WRITE_SIZE x1.0).  An entry
# holds while the SHA-256 prefix of the kernel sources its kernels come from
# is `sha`; traffic is null otherwise.
SWEEP_SOURCES = ("sweep.hip", "sweep_device.h", "device_common.h", "job.h")
STREAM_SOURCES = SWEEP_SOURCES + ("stream.hip",)
TRAFFIC = {
    ("orl", "fp32"): {
        "sha": "c9e5231b5947697d",
        "files": SWEEP_SOURCES,
        "apass": {10304: 20994764, 2576: 6151281, 644: 2453004},
        "cpass_partial": {10304: 24911220, 2576: 9514477, 644: 4031221},
    },
}


def kernel_sources_sha(files) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1009_0881_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

WORKLOADS = {
    "orl": dict(spec="CFG_ORL", h=112, w=92, levels=3, xfer="fw"),
    "small": dict(spec="CFG_SMALL", h=16, w=16, levels=2, xfer="block2"),
    # budgets: the fastest V-cycle budgets over 4 levels in a scan of T (FP32:
    # T = 16 leaves too few coarse iterations, T >= 32 too many; BF16 likewise)
    "large": dict(spec="CFG_LARGE", h=256, w=256, levels=4, xfer="fw", budget=22,
                  budget_bf16=20),
    # hyperspectral-like: 64x64 abundance maps x 256 smooth bands, r = 12; the
    # hierarchy halves the band count too (two-sided, Section 6.1)
    # budget: the fastest 3-level two-sided schedule of a scan (VC, T = 1)
    "spectral": dict(spec="CFG_SPECTRAL", h=64, w=64, levels=3, xfer="fw", two_sided=True,
                     budget=1),
}


def level_sides(h, w, levels):
    out = [(h, w)]
    for _ in range(levels - 1):
        h, w = (h + 1) // 2, (w + 1) // 2
        out.append((h, w))
    return out


def parse_tile(text):
    """--tile "wc,cf" -> NMF_TILE value; empty -> 0 (library default)."""
    if not text:
        return 0
    wc, cf = (int(x) for x in text.split(","))
    return wc | (cf << 8)


def tile_desc(tile_cfg):
    return "default" if not tile_cfg else f"wc={tile_cfg & 0xff},cf={tile_cfg >> 8}"


def kernel_bytes_flops(kind, m, n, r, bf=False):
    """Algorithmic HBM bytes and flops of one launch at a level with m pixels.

    Only what the method must move counts: M streamed once per pass (FP32),
    the factors read and written once, the r x r Grams.  Split-reduction
    partials are overhead of this implementation and show up in the measured
    traffic instead.
    """
    b = 2 if bf else 4            # bytes per element of the M / W / V operand copies
    if kind == "apass":           # A = M W^T fused with the V update: read M, W, V; write V
        return (b * m * n + b * r * n + 8 * m * r + (2 * m * r if bf else 0) + 8 * r * r,
                2 * m * n * r + 4 * m * r * r)
    if kind == "cpass_partial":   # C = V^T M and D = V^T V: read M, V; write C
        return (b * m * n + b * m * r + (4 * m * r if bf else 0) + 4 * r * n,
                2 * m * n * r + 2 * m * r * r)
    if kind == "cpass_final":     # W update and W W^T: read C, read/write W
        return 4 * r * n + 8 * r * n + 8 * r * r, 6 * n * r * r
    if kind in ("nnls_rows", "nnls_cols"):
        # one exact solve per problem: a Cholesky of the r x r Gram (r^3 / 3
        # multiply-adds), the two substitutions and the gradient (r^2 each);
        # FP64 right-hand sides in, FP32 factor read and written
        cnt = m if kind == "nnls_rows" else n
        return 8 * cnt * r + 8 * cnt * r + 8 * r * r, cnt * (2 * r ** 3 // 3 + 6 * r * r)
    return 0, 0


def _make_one(a):
    import synth
    spec, s = a
    return spec, synth.make_instance(spec, s)


def _pool_instances(count, seed):
    """Seeded problems of the uneven batch distribution, drawn in worker
    processes (call before the GPU is touched)."""
    import concurrent.futures as cf
    import synth
    specs = synth.batch_specs(count, seed)
    workers = max(1, min(8, len(os.sched_getaffinity(0))))
    out = []
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for k, item in enumerate(ex.map(_make_one, specs, chunksize=8)):
            out.append(item)
            if (k + 1) % 128 == 0:
                print(f"generated {k + 1}/{count} problems", file=sys.stderr, flush=True)
    return out


def bench_batch(args) -> int:
    """512 uneven problems solved as one batch per step (to eps_E + tau)."""
    pool = _pool_instances(args.count, 1000)
    import torch
    import paper_1009_0881_amd as P
    torch.cuda.set_device(0)

    def kwargs(spec, inst):
        return dict(m=spec.m, n=spec.n, h=spec.h, w=spec.w, r=spec.r, levels=3, algo="hals",
                    cycle=args.cycle, xfer="fw", tol=inst.eps_E + args.tau,
                    max_fine_iters=args.max_fine_iters, check_every=4, grouped=True)

    tile_cfg, tuning = parse_tile(args.tile), None
    if args.tune:   # tile autotuner on every 8th problem of the batch
        from paper_1009_0881_amd import tune
        sample = pool[::8]
        tuning = tune.tune_batch([kwargs(sp, it) for sp, it in sample], [it.M for _, it in sample],
                                 [it.V0 for _, it in sample], [it.W0 for _, it in sample],
                                 [args.budget] * len(sample))
        tile_cfg = tuning["tile_cfg"]
    plans, dev = [], []
    for spec, inst in pool:
        plans.append(P.Plan(**kwargs(spec, inst), tile_cfg=tile_cfg))
        dev.append(P.to_device(inst.M, inst.V0, inst.W0))
    V0 = [d[1].clone() for d in dev]
    W0 = [d[2].clone() for d in dev]
    ws = P.batch_workspace(plans)

    def one():
        for i, d in enumerate(dev):
            d[1].copy_(V0[i])
            d[2].copy_(W0[i])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = P.solve_batch(plans, [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev],
                            args.budget, workspace=ws, graph=args.graph)
        return time.perf_counter() - t0, res

    for _ in range(args.warmup):
        one()
    times, res = [], None
    for _ in range(args.steps):
        dt, res = one()
        times.append(dt)
    ms = np.array(times) * 1e3
    # algorithmic HBM bytes of the run: 2 FP32 passes over M_l per iteration
    sides = {}
    tot_bytes = 0
    for (spec, inst), r in zip(pool, res):
        fe = r["fine_equiv"]
        tot_bytes += fe * (8 * spec.m * spec.n)
    ms50 = float(np.percentile(ms, 50))
    ok = all(r["stopped"] for r in res)
    out = {
        "metric": "time to rel. err 1e-2 vs plain FP32 single-level; solves/s + p50/p99 latency",
        "value": round(args.count / (ms50 * 1e-3), 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(float(np.mean(ms)), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch: {args.count} uneven planted-blob problems (sides 16-64, "
                               f"n 100-2000, r 5-40), 3 levels FW, {args.cycle.upper()} HALS FP32, "
                               f"T={args.budget}, each to rel_err <= eps_E+{args.tau:g}, one "
                               f"batched solve per step{' (hipGraph)' if args.graph else ''}"},
        "batch_ms": {"p50": round(ms50, 3), "p99": round(float(np.percentile(ms, 99)), 3)},
        "all_reached_target": bool(ok),
        "iterations_total": int(sum(r["total_iters"] for r in res)),
        "fine_equiv_total": round(float(sum(r["fine_equiv"] for r in res)), 2),
        "algorithmic_hbm_gbs": round(tot_bytes / (ms50 * 1e-3) / 1e9, 1),
        "tile_cfg": tile_desc(tile_cfg),
    }
    if tuning:
        out["tuning_ms"] = {k: round(v, 3) for k, v in tuning["ms"].items()}
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def bench_tensor(args) -> int:
    """Multilevel NTF (mode 1 coarsened) against single-level NTF, both to
    ||X - [[A, B, C]]||_F / ||X||_F <= eps_E + tau, on the video-like planted
    tensor (56x46 pixels x 20 x 20, rank 12)."""
    import torch
    import paper_1009_0881_amd as P
    import synth
    torch.cuda.set_device(0)
    spec = synth.CFG_TENSOR
    inst = synth.make_tensor_instance(spec, args.seed)
    m, n, r, K = spec.m, spec.J * spec.K, spec.r, spec.K
    levels = args.levels or 3
    target = inst.eps_E + args.tau
    Xd = torch.from_numpy(np.ascontiguousarray(inst.X1.T)).cuda()
    A0 = torch.from_numpy(np.ascontiguousarray(inst.A0.T)).cuda()
    B0 = torch.from_numpy(inst.Bt0.copy()).cuda()
    C0 = torch.from_numpy(inst.Ct0.copy()).cuda()
    A, B, C = A0.clone(), B0.clone(), C0.clone()

    def plan(L):
        return P.Plan(m=m, n=n, h=spec.h, w=spec.w, r=r, levels=L, cycle=args.cycle, xfer="fw",
                      tol=target, max_fine_iters=args.max_fine_iters, check_every=args.check_every, ntf_k=K)

    def run(pl, ws, budget):
        A.copy_(A0)
        B.copy_(B0)
        C.copy_(C0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = pl.solve_ntf(Xd, A, B, C, budget, workspace=ws)
        return time.perf_counter() - t0, res

    ml, sl = plan(levels), plan(1)
    wm, wsl = ml.workspace(), sl.workspace()
    for _ in range(args.warmup):
        run(ml, wm, args.budget)
        run(sl, wsl, 0)
    tm, tsl = [], []
    for _ in range(args.steps):
        dt, rm = run(ml, wm, args.budget)
        tm.append(dt)
    for _ in range(args.steps):
        dt, rs = run(sl, wsl, 0)
        tsl.append(dt)
    ml.profile(P.KERNEL_KINDS)
    run(ml, wm, args.budget)
    prof = ml.profile_read(reset=True)
    ml.profile([])
    mm, ms_ = np.array(tm) * 1e3, np.array(tsl) * 1e3
    out = {
        "metric": "time to rel. err 1e-2 vs plain FP32 single-level; solves/s + p50/p99 latency",
        "value": round(1e3 / float(np.mean(mm)), 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(float(np.mean(mm)), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"tensor: {spec.h}x{spec.w} planted-blob images x {spec.J} x "
                               f"{spec.K}, rank {r}, NTF (HALS per mode), {levels} levels (fw) on "
                               f"the image mode, {args.cycle.upper()}, budget T={args.budget}, "
                               f"target rel_err <= eps_E+{args.tau:g}"},
        "time_to_target_ms": {"multilevel_p50": round(float(np.percentile(mm, 50)), 4),
                              "multilevel_p99": round(float(np.percentile(mm, 99)), 4),
                              "single_level_p50": round(float(np.percentile(ms_, 50)), 4)},
        "speedup_vs_single_level": round(float(np.percentile(ms_, 50) / np.percentile(mm, 50)), 3),
        "eps_E": round(inst.eps_E, 6), "target_rel_err": round(target, 6),
        "iterations": {"multilevel_total": rm["total_iters"], "multilevel_fine": rm["fine_iters"],
                       "multilevel_fine_equiv": round(rm["fine_equiv"], 3),
                       "single_level": rs["total_iters"]},
        "all_reached_target": bool(rm["stopped"] and rs["stopped"]),
        "roofline": None, "cpu_baseline": None,
        "kernels": {k: {"launches_per_solve": v[0], "avg_us": round(v[1] / max(1, v[0]) * 1e3, 3),
                        "ms_per_solve": round(v[1], 4)} for k, v in prof.items()},
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args) -> int:
    """Poisson arrivals served with continuous batching; latency arrival -> host result."""
    pool = _pool_instances(128, 5000)
    import torch
    import paper_1009_0881_amd as P
    torch.cuda.set_device(0)
    srv = P.Server(hbm_budget=16 << 30, slots=64)
    rng = np.random.default_rng(7)
    warm = 3.0
    total = warm + args.duration
    gaps = rng.exponential(1.0 / args.rate, size=int(total * args.rate * 1.5) + 16)
    arrivals = np.cumsum(gaps)
    arrivals = arrivals[arrivals < total]
    is_bf16 = rng.random(len(arrivals)) < args.bf16_share
    pending, done = {}, []
    t0 = time.perf_counter()
    k = 0
    try:
        while k < len(arrivals) or pending:
            now = time.perf_counter() - t0
            while k < len(arrivals) and arrivals[k] <= now:
                spec, inst = pool[k % len(pool)]
                prec = dict(prec="bf16", refine_iters=2) if is_bf16[k] else {}
                t = srv.submit(inst.M, inst.V0, inst.W0, args.budget, spec.h, spec.w, spec.r,
                               levels=3, algo="hals", cycle=args.cycle, xfer="fw",
                               tol=inst.eps_E + 2e-2, max_fine_iters=args.max_fine_iters,
                               check_every=4, **prec)
                pending[t] = (arrivals[k], k)
                k += 1
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    arr, idx = pending.pop(t)
                    done.append((arr, time.perf_counter() - t0, r[2], bool(is_bf16[idx])))
            time.sleep(0.0005)
        st = srv.stats()
    finally:
        srv.close()
    meas = [d for d in done if d[0] >= warm]
    lat = np.array([d[2]["latency_ms"] for d in meas])
    lat_host = np.array([(d[1] - d[0]) * 1e3 for d in meas])
    q = np.array([d[2]["queue_ms"] for d in meas])
    span = max(d[1] for d in meas) - min(d[0] for d in meas)
    ok = all(d[2]["stopped"] for d in meas)
    out = {
        "metric": "time to rel. err 1e-2 vs plain FP32 single-level; solves/s + p50/p99 latency",
        "value": round(len(meas) / span, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": len(meas), "warmup": len(done) - len(meas),
        "ms_per_step": round(float(np.mean(lat)), 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": f"serve: Poisson {args.rate:g} req/s for {args.duration:g} s after "
                               f"{warm:g} s warm-up, problems drawn like the 512-problem batch "
                               f"(3 levels FW, {args.cycle.upper()} HALS, T={args.budget}; "
                               f"{100 * args.bf16_share:g}% BF16 with 2 FP32 refinement "
                               f"iterations, the rest FP32), each to rel_err <= eps_E+0.02, "
                               f"64 slots, 16 GiB pool"},
        "bf16_requests": int(sum(1 for d in meas if d[3])),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "host_poll_p50": round(float(np.percentile(lat_host, 50)), 3),
                       "host_poll_p99": round(float(np.percentile(lat_host, 99)), 3)},
        "queue_ms": {"p50": round(float(np.percentile(q, 50)), 3),
                     "p99": round(float(np.percentile(q, 99)), 3)},
        "offered_rate": args.rate, "server": st, "all_reached_target": bool(ok),
    }
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="orl", choices=sorted(WORKLOADS) + list(EXTRA_WORKLOADS))
    ap.add_argument("--count", type=int, default=512, help="batch: problems per batch")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=20.0, help="serve: measured seconds")
    ap.add_argument("--bf16-share", type=float, default=0.3,
                    help="serve: fraction of requests in BF16 with FP32 refinement")
    ap.add_argument("--graph", action="store_true", help="batch: replay steady ticks as hipGraphs")
    ap.add_argument("--tile", default="", help="tile shapes 'wc,cf' (default: the library's)")
    ap.add_argument("--tune", action="store_true",
                    help="batch: pick the tile shapes with the autotuner first")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run 3 device-to-device copies of BYTES bytes (reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--algo", default="hals", choices=["hals", "mu", "anls", "kl"])
    ap.add_argument("--cycle", default=None, choices=["ni", "vc", "fmg", "wc"],
                    help="schedule; default: W-cycle on the 112x92 workload (the fastest to the "
                         "target there among NI / VC / FMG / WC at T = 16, the others are "
                         "reported beside it), nested iteration at T = 8 on the tensor "
                         "workload, V-cycle elsewhere (each the fastest of a scan)")
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--budget", type=int, default=None,
                    help="schedule budget T in finest-iteration equivalents; default 16, "
                         "22 (FP32) or 20 (BF16) for the 256x256 workload")
    ap.add_argument("--tau", type=float, default=1e-2)
    ap.add_argument("--check-every", type=int, default=2,
                    help="single solves: finest-level iterations between host checks of the "
                         "stop flag (look-ahead; fewer iterations queued past the stop than 4)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-fine-iters", type=int, default=20000)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16"],
                    help="multilevel solve precision (bf16: BF16 MFMA passes, then FP32 "
                         "refinement on the finest level)")
    ap.add_argument("--refine", type=int, default=4, help="bf16: FP32 refinement iterations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kl-target", type=float, default=0.02,
                    help="KL objective: target on D(M | VW) / sum(M) (the divergence keeps "
                         "falling far below the planted factors' value, so the target is fixed)")
    ap.add_argument("--no-other-algos", action="store_true",
                    help="orl: skip the time-to-target of the other two algorithms")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.cycle is None:
        args.cycle = {"orl": "wc", "tensor": "ni"}.get(args.workload, "vc")
    if args.budget is None:
        args.budget = 8 if args.workload == "tensor" else 16
        if args.workload in WORKLOADS:
            key = "budget" if args.prec == "fp32" else "budget_bf16"
            args.budget = WORKLOADS[args.workload].get(key, 16)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described, not built", file=sys.stderr)
        return 2

    import torch
    import paper_1009_0881_amd as P
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        import torch
        torch.cuda.set_device(0)
        nb = args.copy_calibration // 4 * 4
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nb, "copies": 3}), flush=True)
        return 0
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "tensor":
        return bench_tensor(args)
    wl = WORKLOADS[args.workload]
    spec = getattr(synth, wl["spec"])
    levels = args.levels or wl["levels"]
    two_sided = bool(wl.get("two_sided"))
    inst = (synth.make_spectral_instance if two_sided else synth.make_instance)(spec, args.seed)
    m, n, r = spec.m, spec.n, spec.r
    target_frob = inst.eps_E + args.tau
    target_kl = args.kl_target
    target = target_kl if args.algo == "kl" else target_frob
    target_desc = (f"D(M|VW)/sum(M) <= {args.kl_target:g}" if args.algo == "kl"
                   else f"rel_err <= eps_E+{args.tau:g}")

    K, Wm = args.steps, args.warmup
    Md, V0d, W0d = P.to_device(inst.M, inst.V0, inst.W0)
    nbuf = K + Wm
    Vs = [V0d.clone() for _ in range(nbuf)]
    Ws = [W0d.clone() for _ in range(nbuf)]

    def make_plan(L, prec="fp32", two=False):
        return P.Plan(m=m, n=n, h=wl["h"], w=wl["w"], r=r, levels=L, algo=args.algo,
                      cycle=args.cycle, xfer=wl["xfer"], tol=target,
                      max_fine_iters=args.max_fine_iters, check_every=args.check_every, prec=prec,
                      refine_iters=args.refine if prec == "bf16" else 0,
                      tile_cfg=parse_tile(args.tile), two_sided=two)

    ml = make_plan(levels, args.prec, two_sided)
    sl = make_plan(1)
    n_sched = sum(c for k, _, c in ml.schedule(args.budget) if k == "run")
    ws_ml, ws_sl = ml.workspace(), sl.workspace()
    stream = torch.cuda.current_stream()

    def run(plan, ws, budget, i):
        Vs[i].copy_(V0d)
        Ws[i].copy_(W0d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.solve(Md, Vs[i], Ws[i], budget, workspace=ws, stream=stream)
        dt = time.perf_counter() - t0
        return dt, res

    # --- warmup; full per-kernel profile on the last warmup solve ------------
    for i in range(Wm):
        run(ml, ws_ml, args.budget, i)
        run(sl, ws_sl, 0, i)
    ml.profile(P.KERNEL_KINDS)
    _, res_prof = run(ml, ws_ml, args.budget, 0)
    prof_all = ml.profile_read(reset=True)
    _, dep_prof = ml.log(ws_ml)
    dep_prof = dep_prof[:res_prof["log_len"]]
    dominant = max(prof_all, key=lambda k: prof_all[k][1])

    # --- timed region: multilevel solves -------------------------------------
    # No events here: an event recorded between two kernels leaves the stream
    # idle for several microseconds, which would be charged to multilevel only.
    ml.profile([])
    torch.cuda.synchronize()
    times, results = [], []
    for i in range(K):
        dt, res = run(ml, ws_ml, args.budget, Wm + i if Wm + i < nbuf else i)
        times.append(dt)
        results.append(res)
    torch.cuda.synchronize()
    rel_log, dep_log = ml.log(ws_ml)
    last = results[-1]
    dep_log = dep_log[:last["log_len"]]

    # --- the same K solves again, events around every launch of the dominant
    # kernel on the solve's stream: its average launch duration ---------------
    ml.profile([dominant])
    ev_times = []
    for i in range(K):
        dt, res = run(ml, ws_ml, args.budget, Wm + i if Wm + i < nbuf else i)
        ev_times.append(dt)
    torch.cuda.synchronize()
    prof_dom = ml.profile_read(reset=True)
    ml.profile([])

    # --- single-level FP32 to the same target --------------------------------
    sl_times, sl_res = [], None
    for i in range(K):
        dt, sl_res = run(sl, ws_sl, 0, i)
        sl_times.append(dt)
    sl_ms_all = np.array(sl_times) * 1e3

    # the other two algorithms of the workload (ORL-shaped: all three), fewer solves
    others = {}
    if args.workload == "orl" and not args.no_other_algos and args.prec == "fp32":
        # each algorithm at the fastest 3-level schedule of a scan over cycles and
        # budgets (MU needs many cheap coarse iterations, KL a nested-iteration start)
        for alg, cyc, bud in (("hals", "vc", 16), ("mu", "vc", 256), ("anls", "ni", 8),
                              ("kl", "ni", 32)):
            if alg == args.algo:
                continue
            tgt = target_kl if alg == "kl" else target_frob
            def plan_for(L):
                return P.Plan(m=m, n=n, h=wl["h"], w=wl["w"], r=r, levels=L, algo=alg, cycle=cyc,
                              xfer=wl["xfer"], tol=tgt, max_fine_iters=args.max_fine_iters,
                              check_every=args.check_every)
            pm, ps = plan_for(levels), plan_for(1)
            wm, wsl = pm.workspace(), ps.workspace()
            tm, tsl = [], []
            for i in range(2 + 5):
                dt, rm = run(pm, wm, bud, i)
                if i >= 2:
                    tm.append(dt)
                dt, rs = run(ps, wsl, 0, i)
                if i >= 2:
                    tsl.append(dt)
            mm, ms_ = float(np.median(tm) * 1e3), float(np.median(tsl) * 1e3)
            others[alg] = {"cycle": cyc, "budget": bud, "target": round(tgt, 6),
                           "multilevel_ms": round(mm, 4),
                           "single_level_ms": round(ms_, 4), "speedup": round(ms_ / mm, 3),
                           "iterations": rm["total_iters"], "fine": rm["fine_iters"],
                           "single_level_iterations": rs["total_iters"],
                           "reached_target": bool(rm["stopped"] and rs["stopped"])}

    # the other cycles of the same algorithm and budget (ORL-shaped workload)
    other_cycles = {}
    if args.workload == "orl" and not args.no_other_algos and args.prec == "fp32":
        for cyc in ("ni", "vc", "fmg", "wc"):
            if cyc == args.cycle:
                continue
            pc = P.Plan(m=m, n=n, h=wl["h"], w=wl["w"], r=r, levels=levels, algo=args.algo,
                        cycle=cyc, xfer=wl["xfer"], tol=target,
                        max_fine_iters=args.max_fine_iters, check_every=args.check_every)
            wc_ = pc.workspace()
            tc = []
            for i in range(2 + 7):
                dt, rc_ = run(pc, wc_, args.budget, i)
                if i >= 2:
                    tc.append(dt)
            mc = float(np.median(tc) * 1e3)
            other_cycles[cyc] = {"ms": round(mc, 4),
                                 "speedup": round(float(np.percentile(sl_ms_all, 50)) / mc, 3),
                                 "iterations": rc_["total_iters"], "fine": rc_["fine_iters"],
                                 "reached_target": bool(rc_["stopped"])}

    # two-sided workload: the one-sided hierarchy on the same data, for comparison
    one_ms = None
    if two_sided:
        ol = make_plan(levels, args.prec, False)
        ws_ol = ol.workspace()
        ot = []
        for i in range(K):
            dt, o_res = run(ol, ws_ol, args.budget, i)
            ot.append(dt)
        one_ms = {"p50": round(float(np.percentile(np.array(ot) * 1e3, 50)), 4),
                  "iterations": o_res["total_iters"], "fine": o_res["fine_iters"],
                  "reached_target": bool(o_res["stopped"])}

    ok = all(res["stopped"] == 1 for res in results) and sl_res["stopped"] == 1
    times_ms = np.array(times) * 1e3
    sl_ms = np.array(sl_times) * 1e3

    # --- roofline of the dominant kernel --------------------------------------
    sides = level_sides(wl["h"], wl["w"], levels)
    ncols = [n]
    for _ in range(levels - 1):
        ncols.append((ncols[-1] + 1) // 2 if two_sided else ncols[-1])
    tot_bytes = tot_flops = 0
    for it, d in enumerate(dep_log):
        b, f = kernel_bytes_flops(dominant, sides[d][0] * sides[d][1], ncols[d], r,
                                  bf=args.prec == "bf16" and it < n_sched)
        tot_bytes += b
        tot_flops += f
    traffic = None
    entry = TRAFFIC.get((args.workload, args.prec))
    tab = entry.get(dominant) if entry else None
    if (tab and kernel_sources_sha(entry["files"]) == entry["sha"] and levels == wl["levels"]
            and args.refine == entry.get("refine", args.refine)):
        ms_ = [sides[d][0] * sides[d][1] for d in dep_log]
        if all(m_ in tab for m_ in ms_):
            traffic = int(sum(tab[m_] for m_ in ms_) / max(1, len(ms_)))
    # achieved = the kernel's algorithmic bytes per solve over its measured time per
    # solve: the same ratio as per launch, and it stays right when a level issues two
    # launches of the kind (split A-pass) and for the launches issued past the stop
    # (they return at once; their time is counted, their bytes are not)
    cnt, ms_tot = prof_dom.get(dominant, (0, 0.0))
    solves = len(results)
    launches_per_solve = cnt / max(1, solves)
    per_launch_bytes = tot_bytes / max(1, len(dep_log))
    t_solve = (ms_tot / max(1, solves)) * 1e-3
    avg_s = (ms_tot / max(1, cnt)) * 1e-3
    alu = dominant in ("nnls_rows", "nnls_cols")
    if alu:     # FP64 vector arithmetic, no matrix cores: one exact solve per problem
        achieved = tot_flops / t_solve / 1e12 if t_solve > 0 else 0.0
        peak, unit = PEAK_FP64_VALU_TFLOPS, "TFLOP/s"
    else:
        achieved = tot_bytes / t_solve / 1e9 if t_solve > 0 else 0.0
        peak, unit = PEAK_HBM_GBS, "GB/s"
    roofline = {
        "kernel": dominant,
        "bound": "alu" if alu else "hbm",
        "achieved": round(achieved, 3 if alu else 1),
        "peak": peak,
        "unit": unit,
        "frac": round(achieved / peak, 4),
        "traffic": traffic,
        "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
        "avg_launch_us": round(avg_s * 1e6, 3),
        "launches_per_solve": launches_per_solve,
        "algorithmic_bytes_per_iteration": int(per_launch_bytes),
        "iterations_per_solve": len(dep_log),
        "mfma_tflops": 0.0 if alu else (round(tot_flops / t_solve / 1e12, 3) if t_solve > 0 else 0.0),
        "mfma_frac": round(tot_flops / t_solve / 1e12 / (PEAK_BF16_MFMA_TFLOPS if args.prec == "bf16"
                                                         else PEAK_FP32_MFMA_TFLOPS), 4)
        if t_solve > 0 and not alu else 0.0,
    }
    kernels = {k: {"launches_per_solve": v[0], "avg_us": round(v[1] / max(1, v[0]) * 1e3, 3),
                   "ms_per_solve": round(v[1], 4)} for k, v in prof_all.items()}

    # --- CPU baseline: the FP64 oracle on a bounded sample --------------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:   # threadpoolctl missing: report the affinity mask
            cores = len(os.sched_getaffinity(0))
        cyc = {"ni": O.NI, "vc": O.VC, "fmg": O.FMG, "wc": O.WC}[args.cycle]
        alg = {"hals": O.HALS, "mu": O.MU, "anls": O.ANLS, "kl": O.KL}[args.algo]
        xf = O.XFER_FW if wl["xfer"] == "fw" else O.XFER_BLOCK2
        t0 = time.perf_counter()
        nsol = 0
        fine_it = 0
        while True:
            ores = O.solve(inst.M, wl["h"], wl["w"], r, levels, alg, cyc, xf, args.budget,
                           inst.V0, inst.W0, tol=target, max_fine_iters=args.max_fine_iters,
                           two_sided=two_sided)
            nsol += 1
            fine_it = ores.fine_iters
            if time.perf_counter() - t0 >= args.cpu_seconds or nsol >= 50:
                break
        el = time.perf_counter() - t0
        cpu = {"value": round(nsol / el, 4), "unit": "solves/s", "cores": int(cores),
               "kind": "oracle",
               "sample": f"{nsol} complete multilevel {args.algo.upper()} solve(s) of this workload "
                         f"to {target_desc} in FP64 numpy ({el:.1f} s, "
                         f"{fine_it} finest-level iterations each); host {platform.processor() or platform.machine()}"}

    ms_step = float(np.mean(times_ms))
    out = {
        "metric": "time to rel. err 1e-2 vs plain FP32 single-level; solves/s + p50/p99 latency",
        "value": round(1e3 / ms_step, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32" if args.prec == "bf16" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {wl['h']}x{wl['w']} planted-blob "
                        f"{'maps x smooth spectra' if two_sided else 'images'}, n={n}, r={r}, "
                        f"{levels} {'two-sided ' if two_sided else ''}levels ({wl['xfer']}), "
                        f"{args.cycle.upper()} {args.algo.upper()} "
                        + ("BF16 GEMMs, FP32 accumulation, " + str(args.refine) + " FP32 refinement "
                           "iterations on the finest level" if args.prec == "bf16" else "FP32")
                        + f", budget T={args.budget}, target {target_desc}",
            "m": m, "n": n, "r": r, "levels": levels, "algo": args.algo, "cycle": args.cycle,
            "seed": args.seed,
        },
        "time_to_target_ms": {"multilevel_p50": round(float(np.percentile(times_ms, 50)), 4),
                              "multilevel_p99": round(float(np.percentile(times_ms, 99)), 4),
                              "single_level_p50": round(float(np.percentile(sl_ms, 50)), 4),
                              "single_level_p99": round(float(np.percentile(sl_ms, 99)), 4)},
        "event_pass_ms_per_solve": round(float(np.percentile(np.array(ev_times) * 1e3, 50)), 4),
        "speedup_vs_single_level": round(float(np.percentile(sl_ms, 50) / np.percentile(times_ms, 50)), 3),
        "target_rel_err": round(target, 6),
        "eps_E": round(inst.eps_E, 6),
        "final_rel_err": {"multilevel": last["rel_err"], "single_level": sl_res["rel_err"]},
        "iterations": {"multilevel_total": last["total_iters"], "multilevel_fine": last["fine_iters"],
                       "multilevel_fine_equiv": round(last["fine_equiv"], 3),
                       "single_level": sl_res["total_iters"]},
        "all_reached_target": bool(ok),
        "one_sided_multilevel_ms": one_ms,
        "other_algorithms": others or None,
        "other_cycles": other_cycles or None,
        "tile_cfg": tile_desc(parse_tile(args.tile)),
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
