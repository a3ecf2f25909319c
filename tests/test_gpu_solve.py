"""GPU parity of whole multilevel solves (trajectory of rel_err and final
factors) against the FP64 oracle on the small and the ORL-shaped workloads."""
import numpy as np
import pytest

import oracle as O
import paper_1009_0881_amd as P
import synth
from gpu_util import TOL_FACTOR, TOL_REL_ERR, frob_rel, gpu_solve, oracle_solve, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def check(tag, g, o):
    res, rel, dep, V, W = g
    ores, orel, odep = o
    k = min(50, len(orel))
    say(tag, "iters", len(rel), len(orel), "max|d rel| (first 50)",
        float(np.max(np.abs(rel[:k] - orel[:k]))), "V", frob_rel(V, ores.V), "W", frob_rel(W, ores.W))
    assert len(rel) == len(orel)
    np.testing.assert_array_equal(dep, odep)
    assert np.max(np.abs(rel[:k] - orel[:k])) <= TOL_REL_ERR
    return res, ores


def test_small_config_first_50_iterations():
    # 16x16 images, n=500, r=10, 2 levels of 2x2 block restriction, NI, T=200:
    # the first 50 iterations all run on the 8x8 level.
    inst = synth.make_instance(synth.CFG_SMALL, 0)
    args = (inst.M, inst.V0, inst.W0, 16, 16, 10, 2, "hals", "ni", "block2", 200)
    g = gpu_solve(*args)
    o = oracle_solve(*args)
    res, ores = check("cfg-small T=200", g, o)
    assert res["total_iters"] == 350 and res["fine_iters"] == 150
    assert frob_rel(g[3], ores.V) <= 10 * TOL_FACTOR     # after all 350 iterations


@pytest.mark.parametrize("algo", ["hals", "mu", "anls"])
@pytest.mark.parametrize("cycle", ["ni", "vc", "fmg", "wc"])
def test_small_config_full_schedule(algo, cycle):
    inst = synth.make_instance(synth.CFG_SMALL, 0)
    T = 16 if algo != "anls" else 8
    args = (inst.M, inst.V0, inst.W0, 16, 16, 10, 2, algo, cycle, "block2", T)
    g = gpu_solve(*args)
    o = oracle_solve(*args)
    _, ores = check(f"cfg-small {algo} {cycle}", g, o)
    assert frob_rel(g[3], ores.V) <= TOL_FACTOR
    assert frob_rel(g[4], ores.W) <= TOL_FACTOR


@pytest.mark.parametrize("algo", ["hals", "mu"])
@pytest.mark.parametrize("cycle", ["ni", "vc", "fmg", "wc"])
def test_orl_shape_three_levels(algo, cycle):
    inst = synth.make_instance(synth.CFG_ORL, 0)
    args = (inst.M, inst.V0, inst.W0, 112, 92, 40, 3, algo, cycle, "fw", 16)
    g = gpu_solve(*args)
    o = oracle_solve(*args)
    _, ores = check(f"orl {algo} {cycle}", g, o)
    assert frob_rel(g[3], ores.V) <= TOL_FACTOR
    assert frob_rel(g[4], ores.W) <= TOL_FACTOR


def test_orl_shape_single_level_50_iterations():
    inst = synth.make_instance(synth.CFG_ORL, 0)
    args = (inst.M, inst.V0, inst.W0, 112, 92, 40, 1, "hals", "ni", "fw", 50)
    g = gpu_solve(*args)
    o = oracle_solve(*args)
    _, ores = check("orl hals L=1 50 it", g, o)
    assert frob_rel(g[3], ores.V) <= TOL_FACTOR
    assert frob_rel(g[4], ores.W) <= TOL_FACTOR


@pytest.mark.parametrize("level", [1, 2])
def test_orl_per_level_restart(level):
    # Start a level from the oracle's own state there (FP32-rounded) and run 50
    # iterations: every level's kernels are checked without accumulated drift.
    inst = synth.make_instance(synth.CFG_ORL, 0)
    sides = O.level_sides(112, 92, 3)
    Ml = inst.M.astype(np.float64)
    for d in range(level):
        Ml = O.restrict_images(Ml, *sides[d], O.XFER_FW)
    seen = {}

    def cb(d, V, W, e):
        if d == level:
            seen["V"], seen["W"] = V.copy(), W.copy()

    O.solve(inst.M, 112, 92, 40, 3, O.HALS, O.NI, O.XFER_FW, 16, inst.V0, inst.W0, callback=cb)
    M32 = Ml.astype(np.float32)
    V32 = seen["V"].astype(np.float32)
    W32 = seen["W"].astype(np.float32)
    h, w = sides[level]
    g = gpu_solve(M32, V32, W32, h, w, 40, 1, "hals", "ni", "fw", 50)
    o = oracle_solve(M32, V32, W32, h, w, 40, 1, "hals", "ni", "fw", 50)
    _, ores = check(f"orl restart level {level}", g, o)
    assert frob_rel(g[3], ores.V) <= TOL_FACTOR
    assert frob_rel(g[4], ores.W) <= TOL_FACTOR


def test_tolerance_stop_iteration_matches_oracle():
    inst = synth.make_instance(synth.CFG_SMALL, 0)
    base = oracle_solve(inst.M, inst.V0, inst.W0, 16, 16, 10, 2, "hals", "ni", "block2", 16,
                        tol=1e-12, max_fine=60)
    fine = [e for d, e in base[0].log if d == 0]
    # a threshold half-way between two consecutive fine-level values
    tol = 0.5 * (fine[30] + fine[31])
    assert fine[30] - fine[31] > 4 * TOL_REL_ERR
    args = (inst.M, inst.V0, inst.W0, 16, 16, 10, 2, "hals", "ni", "block2", 16)
    g = gpu_solve(*args, tol=tol, max_fine=100)
    o = oracle_solve(*args, tol=tol, max_fine=100)
    assert g[0]["stopped"] == 1 and o[0].stopped
    check("tol stop", g, o)


def test_solve_rejects_bad_input_values():
    M, V, W = synth.uniform_pair(64, 10, 3, seed=1)
    M[5, 3] = -1.0
    pl = P.Plan(m=64, n=10, h=8, w=8, r=3, check_input=True)
    with pytest.raises(P.NmfError) as e:
        pl.solve(*P.to_device(M, V, W), 4)
    assert e.value.status == -6
    M[5, 3] = np.nan
    with pytest.raises(P.NmfError) as e:
        pl.solve(*P.to_device(M, V, W), 4)
    assert e.value.status == -5


def test_zero_iterations():
    # levels = 1: nothing runs; levels = 2: V only goes down and back up (P R V0)
    M, V, W = synth.uniform_pair(64, 10, 3, seed=2)
    for levels in (1, 2):
        pl = P.Plan(m=64, n=10, h=8, w=8, r=3, levels=levels)
        Md, Vd, Wd = P.to_device(M, V, W)
        res = pl.solve(Md, Vd, Wd, 0)
        assert res["total_iters"] == 0
        Vh, Wh = P.factors_to_host(Vd, Wd)
        ores = O.solve(M, 8, 8, 3, levels, O.HALS, O.NI, O.XFER_FW, 0, V, W)
        np.testing.assert_allclose(Vh, ores.V, rtol=2 ** -22, atol=1e-30)
        np.testing.assert_array_equal(Wh, W.astype(np.float64))


@pytest.mark.parametrize("algo", ["hals", "mu"])
def test_one_step_from_oracle_states(algo):
    # One GPU iteration from the oracle's own state (FP32-rounded) at several
    # points of the small workload's coarse-level trajectory must equal one
    # oracle iteration from the same state to FP32 accuracy.
    inst = synth.make_instance(synth.CFG_SMALL, 0)
    Mc = O.restrict_images(inst.M.astype(np.float64), 16, 16, O.XFER_BLOCK2).astype(np.float32)
    Vc = O.restrict_images(inst.V0.astype(np.float64), 16, 16, O.XFER_BLOCK2).astype(np.float32)
    states = {}

    def cb(d, V, W, e):
        states[len(states)] = (V.astype(np.float32), W.astype(np.float32))

    O.solve(Mc, 8, 8, 10, 1, P.ALGOS[algo], O.NI, O.XFER_FW, 45, Vc, inst.W0, callback=cb)
    worst = 0.0
    for t in (0, 5, 10, 20, 30, 40, 44):
        V32, W32 = states[t]
        g = gpu_solve(Mc, V32, W32, 8, 8, 10, 1, algo, "ni", "fw", 1)
        o = oracle_solve(Mc, V32, W32, 8, 8, 10, 1, algo, "ni", "fw", 1)
        dv, dw = frob_rel(g[3], o[0].V), frob_rel(g[4], o[0].W)
        de = abs(g[1][0] - o[1][0])
        say(f"  step from state {t}: |d rel| {de:.2e} V {dv:.2e} W {dw:.2e}")
        worst = max(worst, dv, dw)
        assert de <= 1e-6
    assert worst <= 1e-5


@pytest.mark.timeout(600)
def test_orl_shape_anls_three_levels():
    """ANLS on the ORL-shaped workload (112x92, n = 400, r = 40, 3 levels, full
    weighting, NI, T = 8: 8 iterations at 28x23, 6 at 56x46, 6 at 112x92).
    The oracle's Python active-set loop makes this the slowest parity test
    (about a minute of CPU).  Same bar as HALS and MU: per-iteration rel_err
    within 1e-5, factors within 1e-4."""
    inst = synth.make_instance(synth.CFG_ORL, 0)
    args = (inst.M, inst.V0, inst.W0, 112, 92, 40, 3, "anls", "ni", "fw", 8)
    g = gpu_solve(*args)
    o = oracle_solve(*args)
    _, ores = check("orl anls ni", g, o)
    say("  cond(V^T V) %.3e  cond(W W^T) %.3e" % (np.linalg.cond(ores.V.T @ ores.V),
                                                  np.linalg.cond(ores.W @ ores.W.T)))
    assert frob_rel(g[3], ores.V) <= TOL_FACTOR
    assert frob_rel(g[4], ores.W) <= TOL_FACTOR
