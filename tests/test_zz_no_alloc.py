"""nmf_solve_static (the entry point that allocates nothing) against nmf_solve.

Both run the same kernels on the same inputs; the static entry point uses the
library's fixed device array as its workspace.  Its results must equal
nmf_solve's bit for bit, on two calls in a row, the second with a smaller
problem (the array keeps the first call's contents)."""
import numpy as np
import pytest

import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1009_0881_amd as P  # noqa: E402


def _pair(spec, seed, levels, algo, cycle, xfer, T, **kw):
    inst = synth.make_instance(spec, seed)
    pl = P.Plan(m=spec.m, n=spec.n, h=spec.h, w=spec.w, r=spec.r, levels=levels, algo=algo,
                cycle=cycle, xfer=xfer, **kw)
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    ref = pl.solve(Md, Vd, Wd, T)
    Vr, Wr = P.factors_to_host(Vd, Wd)
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    res = pl.solve_static(Md, Vd, Wd, T)
    Vs, Ws = P.factors_to_host(Vd, Wd)
    return ref, res, (Vr, Wr), (Vs, Ws)


def _same(tag, ref, res, fr, fs):
    say(f"  {tag}: iterations {res['total_iters']} rel_err {res['rel_err']:.9f} "
        f"(nmf_solve {ref['rel_err']:.9f})")
    for k in ("log_len", "total_iters", "fine_iters", "stopped", "rel_err", "fine_equiv"):
        assert res[k] == ref[k], k
    np.testing.assert_array_equal(fs[0], fr[0])
    np.testing.assert_array_equal(fs[1], fr[1])


def test_static_solve_equals_solve_twice_second_smaller():
    # first: the 112x92 workload (3 levels, V-cycle, HALS, stop at a tolerance)
    spec1 = synth.CFG_ORL
    tol = synth.make_instance(spec1, 0).eps_E + 1e-2
    a = _pair(spec1, 0, 3, "hals", "vc", "fw", 16, tol=tol, max_fine_iters=200)
    _same("112x92 hals vc", *a)
    assert a[1]["stopped"] == 1
    # second, smaller: 16x16 images, 2 levels of block restriction, MU, NI
    b = _pair(synth.CFG_SMALL, 0, 2, "mu", "ni", "block2", 24)
    _same("16x16 mu ni", *b)


def test_static_solve_anls_then_smaller_hals():
    spec = synth.BlobSpec(h=28, w=23, n=120, r=12, k_lo=1, k_hi=5, sig_lo=1.0, sig_hi=6.0)
    a = _pair(spec, 4, 2, "anls", "ni", "fw", 8)
    _same("28x23 anls", *a)
    b = _pair(synth.BlobSpec(h=8, w=8, n=30, r=3, k_lo=1, k_hi=3, sig_lo=1, sig_hi=2), 5, 1,
              "hals", "ni", "fw", 10)
    _same("8x8 hals", *b)


def test_static_solve_rejects_a_plan_above_its_limit():
    spec = synth.CFG_LARGE
    pl = P.Plan(m=spec.m, n=spec.n, h=spec.h, w=spec.w, r=spec.r, levels=4)
    assert pl.workspace_bytes > P.STATIC_WORKSPACE_BYTES
    M = torch.zeros((spec.n, spec.m), dtype=torch.float32, device="cuda")
    V = torch.zeros((spec.r, spec.m), dtype=torch.float32, device="cuda")
    W = torch.zeros((spec.r, spec.n), dtype=torch.float32, device="cuda")
    with pytest.raises(P.NmfError) as e:
        pl.solve_static(M, V, W, 4)
    assert e.value.status == -3
