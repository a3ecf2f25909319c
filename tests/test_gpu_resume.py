"""A solve split in two equals one solve.  The state a solve carries between
iterations on the finest level is (V, W): the Grams and products are rebuilt
from them at the start of every solve by the same kernels that update them.
So T1 iterations, then T2 more from the factors the first call returned, give
bit for bit the factors and the rel_err log of one call of T1 + T2
iterations; and a multilevel schedule followed by a single-level call of T2
iterations equals the multilevel call that continues T2 iterations on the
finest level."""
import numpy as np
import pytest

import paper_1009_0881_amd as P
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(pl, M, V, W, T):
    Md, Vd, Wd = P.to_device(M, V, W)
    res = pl.solve(Md, Vd, Wd, T)
    rel, dep = pl.log(res["_workspace"])
    k = res["log_len"]
    Vh, Wh = P.factors_to_host(Vd, Wd)
    return res, rel[:k].copy(), dep[:k].copy(), Vh, Wh


@pytest.mark.parametrize("algo", ["hals", "mu", "anls"])
def test_single_level_split_equals_one_solve(algo):
    inst = synth.make_instance(synth.CFG_SMALL, 0)       # 16x16 images, n = 500, r = 10
    T1, T2 = 7, 9
    pl = P.Plan(m=256, n=500, h=16, w=16, r=10, levels=1, algo=algo)
    _, rel_all, _, V_all, W_all = _run(pl, inst.M, inst.V0, inst.W0, T1 + T2)
    _, rel1, _, V1, W1 = _run(pl, inst.M, inst.V0, inst.W0, T1)
    _, rel2, _, V2, W2 = _run(pl, inst.M, np.asfortranarray(V1.astype(np.float32)),
                              W1.astype(np.float32), T2)
    say(f"  {algo}: {len(rel1)} + {len(rel2)} iterations vs {len(rel_all)}")
    np.testing.assert_array_equal(V2, V_all)
    np.testing.assert_array_equal(W2, W_all)
    np.testing.assert_array_equal(np.concatenate([rel1, rel2]), rel_all)


def test_multilevel_then_finest_level_continuation():
    inst = synth.make_instance(synth.CFG_ORL, 0)         # 112x92 images, n = 400, r = 40
    kw = dict(m=10304, n=400, h=112, w=92, r=40, cycle="vc")
    T, T2 = 8, 6
    # one call: the V-cycle schedule, then exactly T2 continuation iterations on
    # the finest level (a target no iteration reaches, capped at T2)
    ml_cont = P.Plan(levels=3, tol=1e-9, max_fine_iters=T2, check_every=2, **kw)
    res_all, rel_all, dep_all, V_all, W_all = _run(ml_cont, inst.M, inst.V0, inst.W0, T)
    ml = P.Plan(levels=3, **kw)
    _, rel1, dep1, V1, W1 = _run(ml, inst.M, inst.V0, inst.W0, T)
    sl = P.Plan(levels=1, **kw)
    _, rel2, _, V2, W2 = _run(sl, inst.M, np.asfortranarray(V1.astype(np.float32)),
                              W1.astype(np.float32), T2)
    say(f"  multilevel {len(rel1)} + single-level {len(rel2)} vs {len(rel_all)} "
        f"(stopped {res_all['stopped']})")
    assert res_all["stopped"] == 0
    np.testing.assert_array_equal(V2, V_all)
    np.testing.assert_array_equal(W2, W_all)
    np.testing.assert_array_equal(np.concatenate([rel1, rel2]), rel_all)
    np.testing.assert_array_equal(dep_all[len(rel1):], 0)
