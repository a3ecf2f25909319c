"""Serving with continuous batching (nmf_server_*): requests submitted while
others run are admitted as slots and pool memory free up; each result must be
the same alone (nmf_solve) and in the mix -- bitwise, since every request runs
exactly the kernels of a single solve."""
import time

import numpy as np
import pytest

import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1009_0881_amd as P  # noqa: E402

KEYS = ("log_len", "total_iters", "fine_iters", "stopped", "rel_err", "fine_equiv")


def _requests(count, seed):
    specs = synth.batch_specs(count, seed=seed)
    out = []
    for i, (spec, s) in enumerate(specs):
        inst = synth.make_instance(spec, s)
        algo = "mu" if i % 5 == 3 else "hals"
        tau = 2e-2 if i % 3 else 0.0
        desc = dict(levels=3, algo=algo, cycle="vc" if i % 2 else "ni", xfer="fw",
                    tol=inst.eps_E + tau if tau else 0.0,
                    max_fine_iters=300 if tau else 0, check_every=4)
        if i % 10 in (2, 5, 8):          # 30% BF16 with FP32 refinement
            desc.update(prec="bf16", refine_iters=2)
        out.append((spec, inst, desc, 8))
    return out


def _alone(spec, inst, desc, T):
    pl = P.Plan(m=spec.m, n=spec.n, h=spec.h, w=spec.w, r=spec.r, **desc)
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    res = pl.solve(Md, Vd, Wd, T)
    torch.cuda.synchronize()
    return Vd.cpu().numpy().T, Wd.cpu().numpy(), res


def _drain(srv, tickets, timeout_s=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            r = srv.poll(t)
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout_s, "server did not finish in time"
        time.sleep(0.001)
    return out


def _footprint(spec, desc):
    pl = P.Plan(m=spec.m, n=spec.n, h=spec.h, w=spec.w, r=spec.r, **desc)
    a = lambda b: (b + 255) // 256 * 256
    return (a(4 * spec.m * spec.n) + a(4 * spec.m * spec.r) + a(4 * spec.r * spec.n)
            + a(pl.workspace_bytes))


def test_server_alone_vs_mix_bitwise():
    reqs = _requests(10, seed=7000)
    srv = P.Server(hbm_budget=2 << 30, slots=4)
    try:
        tickets = []
        for (spec, inst, desc, T) in reqs:      # staggered arrivals
            tickets.append(srv.submit(inst.M, inst.V0, inst.W0, T, spec.h, spec.w, spec.r, **desc))
            time.sleep(0.002)
        got = _drain(srv, tickets)
        st = srv.stats()
        say("server stats", st)
        assert st["completed"] == len(reqs) and st["peak_running"] <= 4
        for k, (spec, inst, desc, T) in enumerate(reqs):
            V, W, res = got[tickets[k]]
            aV, aW, ares = _alone(spec, inst, desc, T)
            say(f"  request {k}: {spec.h}x{spec.w} n={spec.n} r={spec.r} {desc['algo']} "
                f"iters {res['total_iters']} rel {res['rel_err']:.6g} queue {res['queue_ms']:.2f} ms "
                f"latency {res['latency_ms']:.2f} ms")
            assert all(res[key] == ares[key] for key in KEYS), (res, ares)
            assert np.array_equal(V, aV) and np.array_equal(W, aW)
    finally:
        srv.close()


def test_server_admission_by_footprint():
    # six requests of one shape: a budget of 2.2 footprints runs at most two
    spec = synth.BlobSpec(h=48, w=48, n=1500, r=30, k_lo=3, k_hi=8, sig_lo=3.0, sig_hi=12.0)
    desc = dict(levels=3, algo="hals", cycle="vc", xfer="fw")
    reqs = [(spec, synth.make_instance(spec, 7100 + i), desc, 8) for i in range(6)]
    fp = _footprint(spec, desc)
    budget = int(2.2 * fp)
    srv = P.Server(hbm_budget=budget, slots=8)
    try:
        tickets = [srv.submit(i.M, i.V0, i.W0, T, s.h, s.w, s.r, **d) for s, i, d, T in reqs]
        _drain(srv, tickets)
        st = srv.stats()
        say("admission by footprint: budget", budget, "max footprint", fp, "stats", st)
        assert st["completed"] == 6
        assert st["peak_running"] <= 2
        assert st["peak_pool_bytes"] <= budget
    finally:
        srv.close()


def test_server_rejects_oversized_and_anls():
    spec, inst, desc, T = _requests(1, seed=7200)[0]
    srv = P.Server(hbm_budget=_footprint(spec, desc) // 2, slots=2)
    try:
        with pytest.raises(P.NmfError) as e:
            srv.submit(inst.M, inst.V0, inst.W0, T, spec.h, spec.w, spec.r, **desc)
        assert e.value.status == -7
        d2 = dict(desc, algo="anls")
        with pytest.raises(P.NmfError) as e2:
            srv.submit(inst.M, inst.V0, inst.W0, T, spec.h, spec.w, spec.r, **d2)
        assert e2.value.status == -1
    finally:
        srv.close()
