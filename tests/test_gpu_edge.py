"""GPU parity with the FP64 oracle on the degenerate cases of the method:
readings R6 (HALS with a zero Gram diagonal B_kk = 0 or D_kk = 0: the column
of V / row of W keeps its value), R7 (MU with a zero denominator: the entry
keeps its value; entries that start at zero stay zero, Alg. 2) and plans whose
coarsest level has fewer pixels than the rank (m_l < r: HALS and MU stay
well defined there).  Same parity bar as the other whole-solve tests."""
import numpy as np
import pytest

import synth
from gpu_util import TOL_FACTOR, TOL_REL_ERR, frob_rel, gpu_solve, oracle_solve, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _compare(tag, args, **kw):
    res, rel, dep, V, W = gpu_solve(*args, **kw)
    ores, orel, odep = oracle_solve(*args, **kw)
    k = min(50, len(orel))
    d = float(np.max(np.abs(rel[:k] - orel[:k]))) if k else 0.0
    dv, dw = frob_rel(V, ores.V), frob_rel(W, ores.W)
    say(f"  {tag}: iters {len(rel)}/{len(orel)} max|d rel| {d:.2e} V {dv:.2e} W {dw:.2e}")
    assert len(rel) == len(orel)
    np.testing.assert_array_equal(dep, odep)
    assert d <= TOL_REL_ERR
    assert dv <= TOL_FACTOR and dw <= TOL_FACTOR
    return V, W, ores


@pytest.mark.parametrize("levels,cycle", [(1, "ni"), (3, "vc")])
def test_hals_zero_gram_diagonal_keeps_factor(levels, cycle):
    """Row 3 of W0 and column 3 of V0 are zero: B_33 = 0 at every V half-step
    and D_33 = 0 at every W half-step, so both stay zero through restriction,
    prolongation and every sweep (R6); column 7 of V0 alone is zero, which the
    first V half-step refills (B_77 > 0)."""
    spec = synth.BlobSpec(h=32, w=28, n=150, r=12, k_lo=2, k_hi=6, sig_lo=1.5, sig_hi=6)
    inst = synth.make_instance(spec, 31)
    V0, W0 = inst.V0.copy(), inst.W0.copy()
    W0[3, :] = 0.0
    V0[:, 3] = 0.0
    V0[:, 7] = 0.0
    args = (inst.M, V0, W0, 32, 28, 12, levels, "hals", cycle, "fw", 16)
    V, W, ores = _compare(f"hals R6 L={levels}", args)
    assert not V[:, 3].any() and not W[3, :].any()
    assert V[:, 7].any()


@pytest.mark.parametrize("levels,cycle", [(1, "ni"), (2, "ni"), (3, "fmg")])
def test_mu_zero_denominators_and_zero_entries(levels, cycle):
    """MU: row 5 of W0 is zero, so every denominator (V B)_ik of column 5 is
    zero and V[:, 5] keeps its value (R7) while W[5, :] stays zero; a block of
    zero entries in V0 and in W0 stays zero (Alg. 2 multiplies by the old
    entry)."""
    spec = synth.BlobSpec(h=24, w=20, n=120, r=9, k_lo=2, k_hi=5, sig_lo=1.5, sig_hi=5)
    inst = synth.make_instance(spec, 32)
    V0, W0 = inst.V0.copy(), inst.W0.copy()
    W0[5, :] = 0.0
    V0[40:60, 2] = 0.0
    W0[1, 10:30] = 0.0
    args = (inst.M, V0, W0, 24, 20, 9, levels, "mu", cycle, "fw", 16)
    V, W, ores = _compare(f"mu R7 L={levels}", args)
    assert not W[5, :].any() and not W[1, 10:30].any()
    if levels == 1:
        # single level: no transfer mixes the zero block with its neighbours
        assert not V[40:60, 2].any()
        np.testing.assert_allclose(V[:, 5], V0[:, 5].astype(np.float64), rtol=0, atol=0)
    else:
        np.testing.assert_allclose(V[:, 5], ores.V[:, 5], rtol=1e-6, atol=1e-30)


@pytest.mark.parametrize("algo", ["hals", "mu"])
@pytest.mark.parametrize("cycle", ["ni", "vc", "fmg"])
def test_coarsest_level_smaller_than_rank(algo, cycle):
    """16x16 images, 3 levels (16x16 -> 8x8 -> 4x4): the coarsest level has
    m = 16 pixels for r = 20, so V^T V is singular there; HALS and MU remain
    well defined (zero-Gram-diagonal columns keep their value) and the GPU
    must follow the oracle's trajectory."""
    spec = synth.BlobSpec(h=16, w=16, n=100, r=20, k_lo=3, k_hi=8, sig_lo=1, sig_hi=4)
    inst = synth.make_instance(spec, 33)
    args = (inst.M, inst.V0, inst.W0, 16, 16, 20, 3, algo, cycle, "fw", 16)
    _compare(f"m_l < r {algo} {cycle}", args)
