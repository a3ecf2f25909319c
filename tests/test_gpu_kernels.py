"""GPU parity of the single operators (transfer stencils, FP64 Grams, the two
M-streaming MFMA products, one iteration) against the FP64 oracle / numpy."""
import numpy as np
import pytest

import oracle as O
import paper_1009_0881_amd as P
import synth
from gpu_util import TOL_FACTOR, TOL_REL_ERR, frob_rel, gpu_solve, oracle_solve, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(3, 3), (4, 5), (9, 17), (16, 16), (23, 28), (56, 46), (112, 92)]


@pytest.mark.parametrize("xfer", ["fw", "block2"])
@pytest.mark.parametrize("hw", SHAPES[:5])
def test_restrict_and_prolong_impulse_responses_are_bitexact(xfer, hw):
    h, w = hw
    say("impulse", xfer, hw)
    m = h * w
    X = torch.eye(m, dtype=torch.float32, device="cuda")      # image i = impulse at pixel i
    Y = P.restrict(X, h, w, xfer).cpu().numpy()                # (m, mc): response of pixel i
    R = O.restrict_matrix(h, w, P.XFERS[xfer])
    np.testing.assert_array_equal(Y.T, R.astype(np.float32))
    mc = R.shape[0]
    Yc = torch.eye(mc, dtype=torch.float32, device="cuda")
    Xf = P.prolong(Yc, h, w, xfer).cpu().numpy()               # (mc, m)
    Pm = O.prolong_matrix(h, w, P.XFERS[xfer])
    np.testing.assert_array_equal(Xf.T, Pm.astype(np.float32))


@pytest.mark.parametrize("xfer", ["fw", "block2"])
@pytest.mark.parametrize("hw", SHAPES)
def test_restrict_and_prolong_random_images(xfer, hw):
    h, w = hw
    say("random transfer", xfer, hw)
    rng = np.random.default_rng(h * 1000 + w)
    X = rng.uniform(size=(h * w, 37)).astype(np.float32)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    got = P.restrict(Xd, h, w, xfer).cpu().numpy().T.astype(np.float64)
    want = O.restrict_images(X.astype(np.float64), h, w, P.XFERS[xfer])
    np.testing.assert_allclose(got, want, rtol=2 ** -23, atol=0)
    Yc = rng.uniform(size=(want.shape[0], 11)).astype(np.float32)
    got = P.prolong(torch.from_numpy(np.ascontiguousarray(Yc.T)).cuda(), h, w, xfer)
    want = O.prolong_images(Yc.astype(np.float64), h, w, P.XFERS[xfer])
    np.testing.assert_allclose(got.cpu().numpy().T.astype(np.float64), want, rtol=2 ** -23, atol=0)


@pytest.mark.parametrize("hw,ncols", [((64, 64), 37), ((31, 40), 5), ((256, 256), 9),
                                      ((130, 132), 3)])
def test_restrict_fw_larger_images(hw, ncols):
    """Full-weighting restriction of larger and ragged images (up to the 256x256 grid),
    odd column counts included.  Same bar as above against the oracle."""
    h, w = hw
    say("restrict fw", hw, ncols)
    rng = np.random.default_rng(h * 7 + w + ncols)
    X = rng.uniform(size=(h * w, ncols)).astype(np.float32)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    got = P.restrict(Xd, h, w, "fw").cpu().numpy().T.astype(np.float64)
    want = O.restrict_images(X.astype(np.float64), h, w, P.XFERS["fw"])
    np.testing.assert_allclose(got, want, rtol=2 ** -23, atol=0)


@pytest.mark.parametrize("r,L", [(1, 5), (10, 500), (17, 1000), (40, 10304), (50, 2000),
                                 (64, 333), (33, 65536)])
def test_gram_fp64(r, L):
    say("gram", r, L)
    X = np.random.default_rng(r + L).uniform(size=(r, L)).astype(np.float32)
    G = P.gram(torch.from_numpy(X).cuda()).cpu().numpy()
    X64 = X.astype(np.float64)
    want = X64 @ X64.T
    np.testing.assert_allclose(G, want, rtol=1e-13)
    np.testing.assert_array_equal(G, G.T)


PROD_SHAPES = [  # (h, w, n, r): tiles, ragged tails, odd m (scalar path), r = 1 and 64
    (16, 16, 500, 10), (5, 7, 37, 3), (9, 9, 130, 17), (8, 8, 20, 1), (32, 32, 100, 64),
    (112, 92, 400, 40), (28, 23, 400, 40), (64, 64, 1999, 50), (3, 3, 5, 2),
]


@pytest.mark.parametrize("h,w,n,r", PROD_SHAPES)
def test_products_match_fp64(h, w, n, r):
    say("products", h, w, n, r)
    m = h * w
    M, V, W = synth.uniform_pair(m, n, r, seed=m + n + r)
    pl = P.Plan(m=m, n=n, h=h, w=w, r=r)
    Md, Vd, Wd = P.to_device(M, V, W)
    A, C = pl.products(Md, Vd, Wd)
    A = A.cpu().numpy().T.astype(np.float64)
    C = C.cpu().numpy().astype(np.float64)
    M64, V64, W64 = M.astype(np.float64), V.astype(np.float64), W.astype(np.float64)
    Aw = M64 @ W64.T
    Cw = V64.T @ M64
    # FP32 accumulation over n (resp. m) terms of positive products
    assert np.max(np.abs(A - Aw) / Aw) < 4e-6 * max(1.0, np.log2(n))
    assert np.max(np.abs(C - Cw) / Cw) < 4e-6 * max(1.0, np.log2(m))


ITER_SHAPES = [(16, 16, 500, 10), (5, 7, 37, 3), (9, 9, 130, 17), (8, 8, 20, 1),
               (32, 32, 100, 64), (112, 92, 400, 40)]


@pytest.mark.parametrize("algo", ["hals", "mu"])
@pytest.mark.parametrize("h,w,n,r", ITER_SHAPES)
def test_single_level_iterations_match_oracle(algo, h, w, n, r):
    say("iterate", algo, h, w, n, r)
    spec = synth.BlobSpec(h=h, w=w, n=n, r=r, k_lo=1, k_hi=max(1, min(5, r)),
                          sig_lo=1.0, sig_hi=max(1.5, h / 4))
    inst = synth.make_instance(spec, seed=3)
    iters = 50
    pl = P.Plan(m=h * w, n=n, h=h, w=w, r=r, algo=algo)
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    res = pl.solve(Md, Vd, Wd, iters)
    rel, _ = pl.log(res["_workspace"])
    V, W = P.factors_to_host(Vd, Wd)
    ores = O.solve(inst.M, h, w, r, 1, P.ALGOS[algo], O.NI, O.XFER_FW, iters, inst.V0, inst.W0)
    orel = ores.rel_errs
    assert res["log_len"] == iters
    d = np.max(np.abs(rel[:iters] - orel))
    say("  max |d rel_err|", d, "V", frob_rel(V, ores.V), "W", frob_rel(W, ores.W))
    assert d <= TOL_REL_ERR
    assert frob_rel(V, ores.V) <= TOL_FACTOR
    assert frob_rel(W, ores.W) <= TOL_FACTOR


@pytest.mark.parametrize("algo", ["hals", "mu"])
@pytest.mark.parametrize("h,w,n,r", [(184, 184, 70, 10), (184, 184, 66, 20), (182, 184, 61, 40),
                                     (184, 184, 64, 50), (182, 186, 300, 50),
                                     (184, 184, 1300, 50), (128, 130, 90, 30),
                                     (258, 262, 90, 50)])
def test_streaming_fp32_iterations_match_oracle(algo, h, w, n, r):
    """Levels with m >= 16384 use the FP32 streaming A- and C-pass kernels
    (every rank class here); same parity bar as the regular kernels.  The
    A-pass takes 64-row blocks below m = 65536 (m = 16640 and 33852 .. 33856
    here) and 128-row blocks from there (m = 67596, ending in a partial
    block).  The
    C-pass's D tiles ride on column blocks 0 .. nCx-1 and the rest take passes
    over V alone: n <= 128 (one column block, all extra), n = 300 (three
    blocks, mixed, with m = 33852 ending in a partial 16-row step) and
    n = 1300 (eleven blocks: every tile fused, the last block partly past
    n)."""
    say("streaming fp32", algo, h, w, n, r)
    spec = synth.BlobSpec(h=h, w=w, n=n, r=r, k_lo=1, k_hi=max(1, min(5, r)),
                          sig_lo=2.0, sig_hi=max(2.5, h / 4))
    inst = synth.make_instance(spec, seed=5)
    iters = 12
    pl = P.Plan(m=h * w, n=n, h=h, w=w, r=r, algo=algo)
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    res = pl.solve(Md, Vd, Wd, iters)
    rel, _ = pl.log(res["_workspace"])
    V, W = P.factors_to_host(Vd, Wd)
    ores = O.solve(inst.M, h, w, r, 1, P.ALGOS[algo], O.NI, O.XFER_FW, iters, inst.V0, inst.W0)
    orel = ores.rel_errs
    assert res["log_len"] == iters
    d = np.max(np.abs(rel[:iters] - orel))
    say("  max |d rel_err|", d, "V", frob_rel(V, ores.V), "W", frob_rel(W, ores.W))
    assert d <= TOL_REL_ERR
    assert frob_rel(V, ores.V) <= TOL_FACTOR
    assert frob_rel(W, ores.W) <= TOL_FACTOR


@pytest.mark.parametrize("algo", ["hals", "mu"])
@pytest.mark.parametrize("h,w,n,r", [(128, 128, 1100, 20), (128, 130, 1030, 50)])
def test_streaming_fp32_multilevel_matches_oracle(algo, h, w, n, r):
    """A plan whose finest level streams (m >= 16384) also streams its wide
    coarse levels (m >= 1024, n >= 1024), splitting the A-pass's n-reduction
    over several blocks per 64-row tile and adding the parts in a second
    kernel: m = 4096 (4 parts) and 1024 (8 parts of 9 stages of 16 columns,
    the last one short) here, m = 4160 and 1056 in the second case.  Three
    levels, V-cycle, full weighting; same parity bar as the other solves."""
    say("streaming fp32 multilevel", algo, h, w, n, r)
    spec = synth.BlobSpec(h=h, w=w, n=n, r=r, k_lo=1, k_hi=max(1, min(5, r)),
                          sig_lo=2.0, sig_hi=max(2.5, h / 4))
    inst = synth.make_instance(spec, seed=6)
    T = 8
    res, rel, dep, V, W = gpu_solve(inst.M, inst.V0, inst.W0, h, w, r, 3, algo, "vc", "fw", T)
    ores, orel, odep = oracle_solve(inst.M, inst.V0, inst.W0, h, w, r, 3, algo, "vc", "fw", T)
    k = min(len(rel), 50)
    d = float(np.max(np.abs(rel[:k] - orel[:k])))
    say("  max |d rel_err|", d, "V", frob_rel(V, ores.V), "W", frob_rel(W, ores.W))
    assert len(rel) == len(orel) and np.array_equal(dep, odep)
    assert d <= TOL_REL_ERR
    assert frob_rel(V, ores.V) <= TOL_FACTOR
    assert frob_rel(W, ores.W) <= TOL_FACTOR


@pytest.mark.parametrize("h,w,n,r", [(16, 16, 500, 10), (5, 7, 37, 3), (9, 9, 130, 17),
                                     (8, 8, 20, 1), (16, 16, 80, 64), (28, 23, 120, 40)])
def test_anls_iterations_match_oracle(h, w, n, r):
    """ANLS parity at the full bar (rel_err within 1e-5, factors within 1e-4).
    Each half-step is an exact NNLS solve on FP64 right-hand sides that carry
    only the rounding of the FP32 matrix-core products, so the unique solution
    moves by about cond(V^T V) times that error: the three cases with cond above
    1e5 (1.7e5, 3.8e8 and 7.8e5 here) drift by up to 9.7e-5 in W (the 64-rank
    one), inside the bar.  cond is printed for every case."""
    say("anls", h, w, n, r)
    spec = synth.BlobSpec(h=h, w=w, n=n, r=r, k_lo=1, k_hi=max(1, min(5, r)),
                          sig_lo=1.0, sig_hi=max(1.5, h / 4))
    inst = synth.make_instance(spec, seed=4)
    iters = 8
    pl = P.Plan(m=h * w, n=n, h=h, w=w, r=r, algo="anls")
    Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
    res = pl.solve(Md, Vd, Wd, iters)
    rel, _ = pl.log(res["_workspace"])
    V, W = P.factors_to_host(Vd, Wd)
    ores = O.solve(inst.M, h, w, r, 1, O.ANLS, O.NI, O.XFER_FW, iters, inst.V0, inst.W0)
    d = np.max(np.abs(rel[:iters] - ores.rel_errs))
    cond = np.linalg.cond(ores.V.T @ ores.V)
    say("  max |d rel_err|", d, "V", frob_rel(V, ores.V), "W", frob_rel(W, ores.W),
        "cond(V^T V) %.2e" % cond)
    assert d <= TOL_REL_ERR
    assert (V >= 0).all() and (W >= 0).all()
    assert frob_rel(V, ores.V) <= TOL_FACTOR
    assert frob_rel(W, ores.W) <= TOL_FACTOR
