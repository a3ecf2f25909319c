"""GPU parity of two-sided multilevel solves (Section 6.1: the hierarchy also
halves the column count, for columns ordered along a smooth axis) against
the FP64 oracle: per-iteration rel_err within 1e-5 and factors within 1e-4,
the level sequence bit-exact."""
import numpy as np
import pytest

import oracle as O
import paper_1009_0881_amd as P
import synth
from gpu_util import TOL_FACTOR, TOL_REL_ERR, frob_rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve_both(inst, h, w, r, levels, algo, cycle, xfer, T, tol=0.0, max_fine=0):
    m, n = inst.M.shape
    pl = P.Plan(m=m, n=n, h=h, w=w, r=r, levels=levels, algo=algo, cycle=cycle, xfer=xfer,
                tol=tol, max_fine_iters=max_fine, two_sided=True)
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    res = pl.solve(Md, Vd, Wd, T)
    rel, dep = pl.log(res["_workspace"])
    k = res["log_len"]
    V, W = P.factors_to_host(Vd, Wd)
    ores = O.solve(inst.M, h, w, r, levels, P.ALGOS[algo], P.CYCLES[cycle], P.XFERS[xfer], T,
                   inst.V0, inst.W0, tol=tol, max_fine_iters=max_fine, two_sided=True)
    orel = np.array([e for _, e in ores.log])
    odep = np.array([d for d, _ in ores.log], dtype=np.int32)
    return res, rel[:k], dep[:k], V, W, ores, orel, odep


def _check(tag, out):
    res, rel, dep, V, W, ores, orel, odep = out
    k = min(50, len(orel))
    d = float(np.max(np.abs(rel[:k] - orel[:k])))
    dv, dw = frob_rel(V, ores.V), frob_rel(W, ores.W)
    say(f"  {tag}: iters {len(rel)}/{len(orel)} max|d rel| {d:.2e} V {dv:.2e} W {dw:.2e} "
        f"fine_equiv {res['fine_equiv']:.3f}/{ores.fine_equiv:.3f}")
    assert len(rel) == len(orel)
    np.testing.assert_array_equal(dep, odep)
    assert d <= TOL_REL_ERR
    assert dv <= TOL_FACTOR and dw <= TOL_FACTOR
    assert abs(res["fine_equiv"] - ores.fine_equiv) < 1e-12


@pytest.mark.parametrize("algo", ["hals", "mu", "anls"])
@pytest.mark.parametrize("cycle", ["ni", "vc", "fmg", "wc"])
def test_spectral_two_sided_matches_oracle(algo, cycle):
    """32x32 abundance maps, 96 smooth bands, r = 8, 3 levels (96 -> 48 -> 24
    columns), full weighting on both sides."""
    spec = synth.SpectralSpec(h=32, w=32, n=96, r=8, sig_lo=2.0, sig_hi=6.0, bw_lo=4.0,
                              bw_hi=16.0)
    inst = synth.make_spectral_instance(spec, 1)
    T = 8 if algo != "anls" else 4
    _check(f"spectral {algo} {cycle}", _solve_both(inst, 32, 32, 8, 3, algo, cycle, "fw", T))


@pytest.mark.parametrize("xfer", ["fw", "block2"])
def test_two_sided_odd_column_counts(xfer):
    """Odd counts at every level (37 -> 19 -> 10 columns; 13x11 -> 7x6 -> 4x3
    pixels), HALS, V-cycle."""
    spec = synth.SpectralSpec(h=13, w=11, n=37, r=5, sig_lo=1.5, sig_hi=4.0, bw_lo=3.0,
                              bw_hi=8.0)
    inst = synth.make_spectral_instance(spec, 2)
    _check(f"odd {xfer}", _solve_both(inst, 13, 11, 5, 3, "hals", "vc", xfer, 8))


def test_two_sided_tolerance_stop():
    """Stops at the first finest-level iteration under the target, like the
    oracle (the continuation runs on the finest level only)."""
    spec = synth.CFG_SPECTRAL
    inst = synth.make_spectral_instance(spec, 0)
    out = _solve_both(inst, spec.h, spec.w, spec.r, 3, "hals", "vc", "fw", 8,
                      tol=inst.eps_E + 1e-2, max_fine=300)
    assert out[0]["stopped"] == 1 and out[5].stopped
    _check("spectral 64x64 n=256 to eps_E+0.01", out)


def test_two_sided_streaming_levels():
    """128x128 maps, 2200 bands, r = 20: the finest level (16384 x 2200) and the
    wide second level (4096 x 1100) run the FP32 streaming kernels with their
    own column counts; the third (1024 x 550) the regular ones."""
    spec = synth.SpectralSpec(h=128, w=128, n=2200, r=20, sig_lo=4.0, sig_hi=16.0, bw_lo=40.0,
                              bw_hi=160.0)
    inst = synth.make_spectral_instance(spec, 3)
    _check("streaming two-sided", _solve_both(inst, 128, 128, 20, 3, "hals", "vc", "fw", 8))


def test_two_sided_exact_block_factorisation_kept():
    """M = (P_m V') (W' P_n^T) with 2x2-block operators: the factors stay an
    exact fit through every level (a wrong W transfer breaks this).  Checked on
    the final factors directly in FP64; the logged Gram-form rel_err of an
    exact fit only reads its cancellation floor (e^2 is a difference of terms
    of size ||M||^2 that carry FP32 product rounding, so it reads up to about
    sqrt(1e-7) = 3e-4)."""
    rng = np.random.default_rng(3)
    h, w, n, r = 16, 16, 48, 4
    Vc = rng.uniform(0.5, 1.0, size=(64, r))
    Wc = rng.uniform(0.5, 1.0, size=(r, 24))
    V0 = O.prolong_images(Vc, h, w, O.XFER_BLOCK2).astype(np.float32)
    W0 = O.prolong_cols(Wc, n, O.XFER_BLOCK2).astype(np.float32)
    M = (V0.astype(np.float64) @ W0.astype(np.float64)).astype(np.float32)
    pl = P.Plan(m=h * w, n=n, h=h, w=w, r=r, levels=2, cycle="vc", xfer="block2",
                two_sided=True)
    Md, Vd, Wd = P.to_device(np.asfortranarray(M), np.asfortranarray(V0), W0)
    res = pl.solve(Md, Vd, Wd, 8)
    rel, dep = pl.log(res["_workspace"])
    k = res["log_len"]
    V, W = P.factors_to_host(Vd, Wd)
    M64 = M.astype(np.float64)
    direct = float(np.linalg.norm(M64 - V @ W) / np.linalg.norm(M64))
    say(f"  exact block factorisation: direct rel_err {direct:.2e}; logged max "
        f"{rel[:k].max():.2e} over {k} iterations")
    assert set(dep[:k].tolist()) == {0, 1}
    assert direct < 1e-5
    assert rel[:k].max() < 5e-4
