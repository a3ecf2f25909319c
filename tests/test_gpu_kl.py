"""GPU parity of the KL-divergence solves (multiplicative updates of the
generalized Kullback-Leibler divergence, Section 7.1's other objective
functions) against the FP64 oracle.

Bars.  The logged value is D(M_l | VW) / sum(M_l).  The GPU forms P = VW on
FP32 matrix cores (relative error at most about r 2^-24 per entry) and sums
the terms M log(M/P) - M + P in FP64; the derivative of a term in P is
1 - M/P, so the logged value moves by at most max|1 - M/P| * r 2^-24, below
1e-6 for these fits (|1 - M/P| < 1, r <= 64): the bar is 1e-6 absolute on
every logged value over the first 50 iterations.  Factors: 1e-4
Frobenius-relative, the bar of the Frobenius algorithms (MU-type updates
carry the FP32 product rounding forward without amplifying it)."""
import numpy as np
import pytest

import oracle as O
import paper_1009_0881_amd as P
import synth
from gpu_util import TOL_FACTOR, frob_rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_KL = 1e-6


def _both(M, V0, W0, h, w, r, levels, cycle, xfer, T, tol=0.0, max_fine=0):
    m, n = M.shape
    pl = P.Plan(m=m, n=n, h=h, w=w, r=r, levels=levels, algo="kl", cycle=cycle, xfer=xfer,
                tol=tol, max_fine_iters=max_fine)
    Md, Vd, Wd = P.to_device(M, V0, W0)
    res = pl.solve(Md, Vd, Wd, T)
    rel, dep = pl.log(res["_workspace"])
    k = res["log_len"]
    V, W = P.factors_to_host(Vd, Wd)
    ores = O.solve(M, h, w, r, levels, O.KL, P.CYCLES[cycle], P.XFERS[xfer], T, V0, W0,
                   tol=tol, max_fine_iters=max_fine)
    orel = np.array([e for _, e in ores.log])
    odep = np.array([d for d, _ in ores.log], dtype=np.int32)
    return res, rel[:k], dep[:k], V, W, ores, orel, odep


def _check(tag, out, factor_bar=TOL_FACTOR):
    res, rel, dep, V, W, ores, orel, odep = out
    k = min(50, len(orel))
    d = float(np.max(np.abs(rel[:k] - orel[:k]))) if k else 0.0
    dv, dw = frob_rel(V, ores.V), frob_rel(W, ores.W)
    say(f"  {tag}: iters {len(rel)}/{len(orel)} max|d log| {d:.2e} (log {orel[-1]:.4e}) "
        f"V {dv:.2e} W {dw:.2e}")
    assert len(rel) == len(orel)
    np.testing.assert_array_equal(dep, odep)
    assert d <= TOL_KL
    assert dv <= factor_bar and dw <= factor_bar


@pytest.mark.parametrize("cycle", ["ni", "vc", "fmg", "wc"])
def test_small_config_kl(cycle):
    inst = synth.make_instance(synth.CFG_SMALL, 0)      # 16x16, n = 500, r = 10
    _check(f"small kl {cycle}", _both(inst.M, inst.V0, inst.W0, 16, 16, 10, 2, cycle,
                                      "block2", 16))


@pytest.mark.parametrize("cycle", ["vc", "fmg"])
def test_orl_shape_kl_three_levels(cycle):
    inst = synth.make_instance(synth.CFG_ORL, 0)        # 112x92, n = 400, r = 40
    _check(f"orl kl {cycle}", _both(inst.M, inst.V0, inst.W0, 112, 92, 40, 3, cycle, "fw", 16))


def test_orl_shape_kl_single_level_50_iterations():
    inst = synth.make_instance(synth.CFG_ORL, 0)
    _check("orl kl L=1 50 it", _both(inst.M, inst.V0, inst.W0, 112, 92, 40, 1, "ni", "fw", 50))


@pytest.mark.parametrize("h,w,n,r", [(5, 7, 37, 1), (9, 9, 130, 17), (13, 11, 200, 33),
                                     (16, 16, 80, 64), (20, 28, 65, 48)])
def test_kl_rank_classes_and_ragged_shapes(h, w, n, r):
    """Every rank class (16, 32, 48, 64 after padding), ragged tiles in both
    dimensions, two levels of full weighting."""
    rng = np.random.default_rng(h * 1000 + n)
    V = rng.uniform(0.1, 1.0, size=(h * w, r))
    Wt = rng.uniform(0.1, 1.0, size=(r, n))
    M = (V @ Wt * rng.uniform(0.5, 1.5, size=(h * w, n))).astype(np.float32)
    V0 = rng.uniform(0.1, 1.0, size=(h * w, r)).astype(np.float32)
    W0 = rng.uniform(0.1, 1.0, size=(r, n)).astype(np.float32)
    levels = 2 if min(h, w) >= 4 else 1
    _check(f"kl {h}x{w} n={n} r={r}", _both(M, V0, W0, h, w, r, levels, "vc", "fw", 8))


def test_kl_tolerance_stop():
    inst = synth.make_instance(synth.CFG_SMALL, 0)
    base = O.solve(inst.M, 16, 16, 10, 2, O.KL, O.NI, O.XFER_BLOCK2, 16, inst.V0, inst.W0,
                   tol=1e-12, max_fine_iters=60)
    fine = [e for d, e in base.log if d == 0]
    tol = 0.5 * (fine[30] + fine[31])
    assert fine[30] - fine[31] > 4 * TOL_KL
    out = _both(inst.M, inst.V0, inst.W0, 16, 16, 10, 2, "ni", "block2", 16, tol=tol,
                max_fine=100)
    assert out[0]["stopped"] == 1 and out[5].stopped
    _check("kl tol stop", out)


def test_kl_zero_row_and_column_keep_entries():
    """A zero row of W (its row sum is 0) keeps that column of V, and a zero
    column of V keeps that row of W, at every level (R17, as R7)."""
    inst = synth.make_instance(synth.CFG_SMALL, 0)
    V0 = inst.V0.copy()
    W0 = inst.W0.copy()
    W0[3, :] = 0.0
    V0[:, 6] = 0.0
    out = _both(inst.M, V0, W0, 16, 16, 10, 2, "vc", "block2", 8)
    _check("kl zero row/column", out)
    V, W = out[3], out[4]
    assert np.all(W[3, :] == 0.0) and np.all(V[:, 6] == 0.0)
