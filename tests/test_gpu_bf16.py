"""BF16 precision mode: A- and C-pass products on BF16 operand copies
(v_mfma_f32_16x16x32_bf16, FP32 accumulation), FP32 refinement on the finest
level.  BF16 follows a different trajectory from FP32, so no parity is
claimed; the tests check that it tracks FP32 closely for every rank class and
tile shape (a layout error would not), that the refined solve stops at its
tolerance with an exact residual, and report the error against the FP64
oracle at equal schedules."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import frob_rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1009_0881_amd as P  # noqa: E402


def _iterate(inst, spec, prec, iters, algo="hals"):
    pl = P.Plan(m=spec.m, n=spec.n, h=spec.h, w=spec.w, r=spec.r, algo=algo, prec=prec)
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    ws = pl.workspace()
    rel = pl.iterate(Md, Vd, Wd, iters, workspace=ws)
    V, W = P.factors_to_host(Vd, Wd)
    return rel, V, W


def _direct_rel(M, V, W):
    M = M.astype(np.float64)
    return float(np.linalg.norm(M - V @ W) / np.linalg.norm(M))


@pytest.mark.parametrize("h,w,n,r,algo", [
    (16, 16, 300, 10, "hals"),     # rank class 16
    (32, 32, 257, 20, "hals"),     # 32
    (28, 23, 400, 40, "mu"),       # 48
    (40, 40, 500, 50, "hals"),     # 64
    (192, 192, 120, 24, "hals"),   # m >= 32768: streaming passes, rank class 32
    (182, 182, 130, 40, "hals"),   # streaming, rank class 48
    (184, 184, 150, 50, "mu"),     # streaming, rank class 64
])
def test_bf16_tracks_fp32(h, w, n, r, algo):
    """One iteration from the same start: BF16 factors within the operand
    rounding of FP32 (a wrong operand layout in any rank tile fails this);
    after 20 iterations, rel_err close (trajectories may separate on
    ill-conditioned problems, so only loosely), and the logged rel_err within
    the BF16 Gram-form error of the direct FP64 residual."""
    spec = synth.BlobSpec(h=h, w=w, n=n, r=r, k_lo=3, k_hi=8, sig_lo=h / 16, sig_hi=4 * h / 16)
    inst = synth.make_instance(spec, 11)
    _, V32, W32 = _iterate(inst, spec, "fp32", 1, algo)
    _, V16, W16 = _iterate(inst, spec, "bf16", 1, algo)
    e1v, e1w = frob_rel(V16, V32), frob_rel(W16, W32)
    r32, _, _ = _iterate(inst, spec, "fp32", 20, algo)
    r16, V16b, W16b = _iterate(inst, spec, "bf16", 20, algo)
    d16 = _direct_rel(inst.M, V16b, W16b)
    say(f"  {h}x{w} n={n} r={r} {algo}: 1 it: V {e1v:.3g} W {e1w:.3g}; 20 its: rel fp32 {r32:.6f} "
        f"bf16 {r16:.6f} (direct {d16:.6f})")
    assert (V16b >= 0).all() and (W16b >= 0).all()
    assert e1v <= 2e-2 and e1w <= 2e-2
    assert abs(r16 - r32) <= 0.08 * r32
    # the logged rel_err of a BF16 iteration comes from the Gram form with the
    # BF16 product C (error ~ u_bf16 ||M||^2 / sqrt(m) ~ 1e-4 ||M||^2); the
    # tolerance is therefore only tested on FP32 iterations
    assert abs(d16 ** 2 - r16 ** 2) <= 2e-4


def test_bf16_refined_solve_reaches_target_with_exact_residual():
    spec = synth.CFG_ORL
    inst = synth.make_instance(spec, 0)
    tol = inst.eps_E + 1e-2
    pl = P.Plan(m=spec.m, n=spec.n, h=spec.h, w=spec.w, r=spec.r, levels=3, algo="hals",
                cycle="vc", prec="bf16", refine_iters=3, tol=tol, max_fine_iters=500,
                check_every=1)
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    res = pl.solve(Md, Vd, Wd, 16)
    V, W = P.factors_to_host(Vd, Wd)
    d = _direct_rel(inst.M, V, W)
    say(f"  bf16 VC T=16 + refine: iters {res['total_iters']} fine {res['fine_iters']} "
        f"rel {res['rel_err']:.6f} direct {d:.6f} tol {tol:.6f}")
    assert res["stopped"] == 1 and res["rel_err"] <= tol
    assert abs(d - res["rel_err"]) <= 1e-5


def test_bf16_error_vs_oracle_equal_schedule():
    """Equal schedule (NI, T=24, 2 levels) plus 5 FP32 refinement iterations on
    the GPU; the oracle runs the same schedule and 5 more fine iterations in FP64."""
    spec = synth.BlobSpec(h=32, w=32, n=300, r=16, k_lo=3, k_hi=8, sig_lo=2, sig_hi=8)
    inst = synth.make_instance(spec, 21)
    pl = P.Plan(m=spec.m, n=spec.n, h=32, w=32, r=16, levels=2, algo="hals", cycle="ni",
                prec="bf16", refine_iters=5)
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    res = pl.solve(Md, Vd, Wd, 24)
    V, W = P.factors_to_host(Vd, Wd)
    ores = O.solve(inst.M, 32, 32, 16, 2, O.HALS, O.NI, O.XFER_FW, 24, inst.V0, inst.W0)
    Vo, Wo = ores.V, ores.W
    for _ in range(5):
        Vo, Wo = O.iteration(O.HALS, inst.M.astype(np.float64), Vo, Wo)
    ro = _direct_rel(inst.M, Vo, Wo)
    say(f"  bf16+refine rel {res['rel_err']:.6f} vs FP64 oracle {ro:.6f} (diff {res['rel_err'] - ro:+.2e}); "
        f"V {frob_rel(V, Vo):.3g} W {frob_rel(W, Wo):.3g}")
    assert res["total_iters"] == len(ores.log) + 5
    assert abs(res["rel_err"] - ro) <= 0.02 * ro


def test_bf16_rejects_anls():
    with pytest.raises(P.NmfError) as e:
        P.Plan(m=256, n=100, h=16, w=16, r=8, algo="anls", prec="bf16")
    assert e.value.status == -1
