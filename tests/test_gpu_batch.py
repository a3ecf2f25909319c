"""Batched solves (nmf_solve_batch): one grouped launch per phase over many
uneven problems.  Each problem's arithmetic is that of a single solve, so the
batch must reproduce nmf_solve bitwise; the single path itself is pinned to the
FP64 oracle elsewhere, and a direct oracle check is repeated here."""
import numpy as np
import pytest

import synth
from gpu_util import TOL_FACTOR, TOL_REL_ERR, frob_rel, oracle_solve, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1009_0881_amd as P  # noqa: E402

# (h, w, n, r, levels, algo, cycle, xfer, T, tau) -- uneven shapes, every rank
# class, 1-3 levels, all cycles, both rules, with and without a tolerance.
MIX = [
    (16, 16, 120, 5, 2, "hals", "ni", "block2", 12, 0.0),
    (32, 32, 300, 17, 3, "hals", "vc", "fw", 16, 0.0),
    (24, 20, 257, 33, 2, "mu", "fmg", "fw", 8, 0.0),
    (48, 48, 640, 40, 3, "hals", "ni", "fw", 16, 1e-2),
    (16, 16, 100, 12, 1, "mu", "ni", "fw", 10, 0.0),
    (20, 28, 411, 40, 3, "hals", "fmg", "fw", 8, 2e-2),
    (64, 64, 200, 9, 3, "hals", "vc", "fw", 8, 1e-2),
    (32, 32, 320, 24, 3, "hals-bf16", "vc", "fw", 8, 1e-2),   # BF16 + FP32 refinement
    (24, 24, 150, 12, 2, "mu-bf16", "ni", "fw", 10, 0.0),
]


def _instances(mix, seed0=300):
    out = []
    for i, (h, w, n, r, L, algo, cyc, xf, T, tau) in enumerate(mix):
        spec = synth.BlobSpec(h=h, w=w, n=n, r=r, k_lo=3, k_hi=8, sig_lo=1.0 * h / 16,
                              sig_hi=4.0 * h / 16)
        inst = synth.make_instance(spec, seed0 + i)
        tol = inst.eps_E + tau if tau > 0 else 0.0
        out.append(dict(inst=inst, h=h, w=w, n=n, r=r, L=L, algo=algo, cyc=cyc, xf=xf, T=T,
                        tol=tol))
    return out


def _plan(d):
    algo, _, prec = d["algo"].partition("-")
    return P.Plan(m=d["h"] * d["w"], n=d["n"], h=d["h"], w=d["w"], r=d["r"], levels=d["L"],
                  algo=algo, cycle=d["cyc"], xfer=d["xf"], tol=d["tol"],
                  max_fine_iters=200 if d["tol"] > 0 else 0, check_every=4,
                  prec=prec or "fp32", refine_iters=3 if prec else 0,
                  grouped=d.get("grouped", False))


def _run_single(d):
    pl = _plan(d)
    Md, Vd, Wd = P.to_device(d["inst"].M, d["inst"].V0, d["inst"].W0)
    res = pl.solve(Md, Vd, Wd, d["T"])
    torch.cuda.synchronize()
    return res, Vd, Wd


def _run_batch(ds, graph=False):
    plans = [_plan(d) for d in ds]
    dev = [P.to_device(d["inst"].M, d["inst"].V0, d["inst"].W0) for d in ds]
    res = P.solve_batch(plans, [x[0] for x in dev], [x[1] for x in dev], [x[2] for x in dev],
                        [d["T"] for d in ds], graph=graph)
    torch.cuda.synchronize()
    return res, [x[1] for x in dev], [x[2] for x in dev]


KEYS = ("log_len", "total_iters", "fine_iters", "stopped", "rel_err", "fine_equiv")


def _same(r1, r2):
    return all(r1[k] == r2[k] for k in KEYS)


def test_batch_equals_single_bitwise():
    ds = _instances(MIX)
    say("batch of", len(ds), "mixed problems vs single solves")
    bres, bV, bW = _run_batch(ds)
    for i, d in enumerate(ds):
        sres, sV, sW = _run_single(d)
        say(f"  problem {i}: {d['h']}x{d['w']} n={d['n']} r={d['r']} L={d['L']} {d['algo']} "
            f"{d['cyc']} iters {sres['total_iters']}/{bres[i]['total_iters']} "
            f"rel {sres['rel_err']:.6g}/{bres[i]['rel_err']:.6g} stopped {bres[i]['stopped']}")
        assert _same(sres, bres[i]), (sres, bres[i])
        assert torch.equal(sV, bV[i]) and torch.equal(sW, bW[i])
    assert any(r["stopped"] for r in bres)


def test_batch_graph_equals_eager():
    ds = _instances(MIX[:4] + MIX[:3], seed0=400)
    say("graph-captured batch vs eager batch,", len(ds), "problems")
    e_res, eV, eW = _run_batch(ds, graph=False)
    g_res, gV, gW = _run_batch(ds, graph=True)
    for i in range(len(ds)):
        assert _same(e_res[i], g_res[i]), (e_res[i], g_res[i])
        assert torch.equal(eV[i], gV[i]) and torch.equal(eW[i], gW[i])
    # and a second run of the same batch with graphs reproduces it
    g2, gV2, gW2 = _run_batch(ds, graph=True)
    for i in range(len(ds)):
        assert _same(g_res[i], g2[i])
        assert torch.equal(gV[i], gV2[i]) and torch.equal(gW[i], gW2[i])


def test_batch_vs_oracle():
    mix = [(16, 16, 150, 6, 2, "hals", "ni", "block2", 20, 0.0),
           (20, 24, 180, 18, 2, "mu", "vc", "fw", 16, 0.0),
           (28, 23, 200, 40, 3, "hals", "vc", "fw", 16, 0.0)]
    ds = _instances(mix, seed0=500)
    bres, bV, bW = _run_batch(ds)
    for i, d in enumerate(ds):
        ores, orel, _ = oracle_solve(d["inst"].M, d["inst"].V0, d["inst"].W0, d["h"], d["w"],
                                     d["r"], d["L"], d["algo"], d["cyc"], d["xf"], d["T"])
        V, W = P.factors_to_host(bV[i], bW[i])
        dV, dW = frob_rel(V, ores.V), frob_rel(W, ores.W)
        drel = abs(bres[i]["rel_err"] - orel[-1])
        say(f"  problem {i} vs oracle: |d rel_err| {drel:.3g} V {dV:.3g} W {dW:.3g}")
        assert bres[i]["total_iters"] == len(orel)
        assert drel <= TOL_REL_ERR
        assert dV <= TOL_FACTOR and dW <= TOL_FACTOR


def test_batch_sampled_from_uneven_distribution():
    """32 problems drawn from the uneven batch distribution (sides 16-64,
    n 100-2000, r 5-40), 3 levels each; three of them re-run alone."""
    specs = synth.batch_specs(32, seed=1000)
    ds = []
    for spec, seed in specs:
        inst = synth.make_instance(spec, seed)
        ds.append(dict(inst=inst, h=spec.h, w=spec.w, n=spec.n, r=spec.r, L=3, algo="hals",
                       cyc="vc", xf="fw", T=8, tol=inst.eps_E + 1e-2))
    say("uneven batch of 32 (tol eps_E + 1e-2)")
    bres, bV, bW = _run_batch(ds)
    assert all(r["total_iters"] > 0 for r in bres)
    for i in (0, 13, 31):
        sres, sV, sW = _run_single(ds[i])
        assert _same(sres, bres[i])
        assert torch.equal(sV, bV[i]) and torch.equal(sW, bW[i])
    say("  stopped", sum(r["stopped"] for r in bres), "of 32")


def test_grouped_plans_batch_equals_single_and_oracle():
    """Plans with NMF_TILE_GROUPED (C-pass chunks of at least 512 rows): the
    batch still reproduces single solves of the same plans bitwise, and the
    factors stay at the oracle parity bar."""
    mix = [MIX[1], MIX[3], MIX[6], MIX[7],
           (40, 36, 300, 20, 3, "hals", "vc", "fw", 16, 0.0),
           (64, 48, 500, 33, 3, "mu", "ni", "fw", 12, 0.0)]
    ds = _instances(mix, seed0=700)
    for d in ds:
        d["grouped"] = True
    say("grouped plans: batch of", len(ds), "vs single solves and the oracle")
    bres, bV, bW = _run_batch(ds)
    for i, d in enumerate(ds):
        sres, sV, sW = _run_single(d)
        assert _same(sres, bres[i]), (sres, bres[i])
        assert torch.equal(sV, bV[i]) and torch.equal(sW, bW[i])
    for i in (0, 4, 5):   # FP32 problems without a tolerance
        d = ds[i]
        ores, orel, _ = oracle_solve(d["inst"].M, d["inst"].V0, d["inst"].W0, d["h"], d["w"],
                                     d["r"], d["L"], d["algo"], d["cyc"], d["xf"], d["T"])
        V, W = P.factors_to_host(bV[i], bW[i])
        dV, dW = frob_rel(V, ores.V), frob_rel(W, ores.W)
        drel = abs(bres[i]["rel_err"] - orel[-1])
        say(f"  problem {i} vs oracle: |d rel_err| {drel:.3g} V {dV:.3g} W {dW:.3g}")
        assert bres[i]["total_iters"] == len(orel)
        assert drel <= TOL_REL_ERR
        assert dV <= TOL_FACTOR and dW <= TOL_FACTOR


def test_batch_rejects_anls():
    d = _instances(MIX[:1])[0]
    d["algo"] = "anls"
    with pytest.raises(P.NmfError) as e:
        _run_batch([d])
    assert e.value.status == -1
