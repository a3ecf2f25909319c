"""Tile configurations (nmf_desc.tile_cfg = NMF_TILE(wc, cf)).

Every configuration runs the same iteration.  The W-update tile width cf
changes no arithmetic (each column and each 4-column residual partial is
computed the same way), so results are bitwise equal across cf; the C-pass
row groups wc change the order of the chunk sums only, so every wc meets the
parity bar against the FP64 oracle.  A batch with explicit tiles reproduces
single solves of the same plans bitwise, and the tuner returns one of its
candidates with a timing for each."""
import numpy as np
import pytest

import synth
from gpu_util import TOL_FACTOR, TOL_REL_ERR, frob_rel, gpu_solve, oracle_solve, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1009_0881_amd as P  # noqa: E402
from paper_1009_0881_amd import tune  # noqa: E402


def _instance(h, w, n, r, seed):
    spec = synth.BlobSpec(h=h, w=w, n=n, r=r, k_lo=3, k_hi=8, sig_lo=1.0 * h / 16,
                          sig_hi=4.0 * h / 16)
    return synth.make_instance(spec, seed)


@pytest.mark.parametrize("wc", [1, 2, 4])
@pytest.mark.parametrize("algo,r", [("hals", 20), ("mu", 40)])
def test_w_update_width_is_bitwise_invariant(wc, algo, r):
    h = w = 96                                   # m = 9216: several C-pass chunks
    inst = _instance(h, w, 300, r, 610 + wc)
    out = {}
    for cf in (4, 16):
        res, rel, _, V, W = gpu_solve(inst.M, inst.V0, inst.W0, h, w, r, 2, algo, "vc", "fw", 8,
                                      tile_cfg=(wc, cf))
        out[cf] = (rel, V, W, res["rel_err"])
    say(f"wc={wc} {algo} r={r}: rel_err {out[4][3]:.8g} / {out[16][3]:.8g}")
    assert np.array_equal(out[4][0], out[16][0])
    assert np.array_equal(out[4][1], out[16][1]) and np.array_equal(out[4][2], out[16][2])


@pytest.mark.parametrize("wc,cf", tune.CANDIDATES)
def test_every_tile_configuration_matches_oracle(wc, cf):
    h = w = 40
    r, n, T = 24, 220, 12
    inst = _instance(h, w, n, r, 640)
    res, rel, dep, V, W = gpu_solve(inst.M, inst.V0, inst.W0, h, w, r, 2, "hals", "vc", "fw", T,
                                    tile_cfg=(wc, cf))
    ores, orel, odep = oracle_solve(inst.M, inst.V0, inst.W0, h, w, r, 2, "hals", "vc", "fw", T)
    k = min(len(rel), 50)
    d_rel = float(np.max(np.abs(rel[:k] - orel[:k])))
    dV, dW = frob_rel(V, ores.V), frob_rel(W, ores.W)
    say(f"tiles ({wc},{cf}): max |d rel_err| {d_rel:.3g}, V {dV:.3g}, W {dW:.3g}")
    assert len(rel) == len(orel) and np.array_equal(dep, odep)
    assert d_rel <= TOL_REL_ERR
    assert dV <= TOL_FACTOR and dW <= TOL_FACTOR


def test_batch_with_explicit_tiles_equals_single():
    shapes = [(32, 32, 300, 17, (4, 4)), (24, 20, 257, 33, (2, 16)), (48, 48, 640, 40, (1, 4))]
    ds = []
    for i, (h, w, n, r, tc) in enumerate(shapes):
        inst = _instance(h, w, n, r, 660 + i)
        ds.append((P.Plan(m=h * w, n=n, h=h, w=w, r=r, levels=3, algo="hals", cycle="vc",
                          xfer="fw", tile_cfg=tc), inst))
    dev = [P.to_device(inst.M, inst.V0, inst.W0) for _, inst in ds]
    bres = P.solve_batch([pl for pl, _ in ds], [d[0] for d in dev], [d[1] for d in dev],
                         [d[2] for d in dev], [8] * len(ds))
    torch.cuda.synchronize()
    for i, (pl, inst) in enumerate(ds):
        Md, Vd, Wd = P.to_device(inst.M, inst.V0, inst.W0)
        sres = pl.solve(Md, Vd, Wd, 8)
        torch.cuda.synchronize()
        keys = ("log_len", "total_iters", "rel_err", "fine_equiv")
        assert all(sres[k] == bres[i][k] for k in keys), (sres, bres[i])
        assert torch.equal(Vd, dev[i][1]) and torch.equal(Wd, dev[i][2])


def test_tuner_returns_a_candidate(tmp_path):
    h = w = 32
    inst = _instance(h, w, 200, 12, 680)
    kw = dict(m=h * w, n=200, h=h, w=w, r=12, levels=2, algo="hals", cycle="vc", xfer="fw")
    res = tune.tune_solve(kw, inst.M, inst.V0, inst.W0, 4, repeats=1)
    say("tuner:", res)
    assert tuple(res["best"]) in tune.CANDIDATES
    assert set(res["ms"]) == {f"{a},{b}" for a, b in tune.CANDIDATES}
    path = str(tmp_path / "tiles.json")
    tune.save_result(path, tune.shape_key(kw), res)
    assert tune.choose(kw, "solve", path) == res["tile_cfg"]
