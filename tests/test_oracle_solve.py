"""Pins for the oracle's whole multilevel solve and for the input generator."""
import numpy as np
import pytest

import oracle as O
import synth


def small_instance(seed=0, h=8, w=8, n=40, r=4):
    spec = synth.BlobSpec(h=h, w=w, n=n, r=r, k_lo=1, k_hi=3, sig_lo=1.0, sig_hi=2.0)
    return synth.make_instance(spec, seed)


@pytest.mark.parametrize("algo", [O.HALS, O.MU])
def test_single_level_solve_is_repeated_iteration(algo):
    inst = small_instance()
    res = O.solve(inst.M, 8, 8, 4, 1, algo, O.NI, O.XFER_FW, 5, inst.V0, inst.W0)
    M = inst.M.astype(np.float64)
    V, W = inst.V0.astype(np.float64), inst.W0.astype(np.float64)
    for _ in range(5):
        V, W = O.iteration(algo, M, V, W)
    np.testing.assert_allclose(res.V, V, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(res.W, W, rtol=1e-12, atol=1e-14)
    assert [d for d, _ in res.log] == [0] * 5


@pytest.mark.parametrize("cycle", [O.NI, O.VC, O.FMG])
@pytest.mark.parametrize("algo", [O.HALS, O.MU, O.ANLS])
def test_multilevel_log_matches_schedule_and_bound_holds(cycle, algo):
    inst = small_instance(seed=1, h=16, w=12, n=30, r=3)
    L, T = 3, 32
    res = O.solve(inst.M, 16, 12, 3, L, algo, cycle, O.XFER_FW, T, inst.V0, inst.W0,
                  check_bound=True)
    tot = O.level_iteration_totals(O.schedule(cycle, L, T), L)
    got = [sum(1 for d, _ in res.log if d == k) for k in range(L)]
    assert got == tot
    assert res.bound_checks, "no prolongation happened"
    for lhs, rhs in res.bound_checks:          # Section 4.1, step 4
        assert lhs <= rhs * (1 + 1e-12)
    assert (res.V >= 0).all() and (res.W >= 0).all()


def test_tolerance_stops_on_the_fine_level():
    inst = small_instance(seed=2)
    full = O.solve(inst.M, 8, 8, 4, 2, O.HALS, O.NI, O.XFER_BLOCK2, 8, inst.V0, inst.W0)
    tol = full.log[-1][1] + 0.02
    res = O.solve(inst.M, 8, 8, 4, 2, O.HALS, O.NI, O.XFER_BLOCK2, 8, inst.V0, inst.W0,
                  tol=tol, max_fine_iters=50)
    assert res.stopped
    assert res.log[-1][0] == 0 and res.log[-1][1] <= tol
    assert all(not (d == 0 and e <= tol) for d, e in res.log[:-1])


def test_tolerance_continuation_runs_past_the_schedule():
    inst = small_instance(seed=3)
    res = O.solve(inst.M, 8, 8, 4, 1, O.HALS, O.NI, O.XFER_FW, 2, inst.V0, inst.W0,
                  tol=1e-9, max_fine_iters=7)
    assert not res.stopped and len(res.log) == 2 + 7


def test_generator_is_deterministic_and_well_formed():
    a = synth.make_instance(synth.CFG_SMALL, 0)
    b = synth.make_instance(synth.CFG_SMALL, 0)
    c = synth.make_instance(synth.CFG_SMALL, 1)
    assert a.M.dtype == np.float32 and a.M.shape == (256, 500) and a.M.flags.f_contiguous
    assert a.V0.shape == (256, 10) and a.W0.shape == (10, 500)
    np.testing.assert_array_equal(a.M, b.M)
    np.testing.assert_array_equal(a.W0, b.W0)
    assert not np.array_equal(a.M, c.M)
    assert (a.M >= 0).all() and (a.V0 >= 0).all() and (a.W0 >= 0).all()
    M64 = a.M.astype(np.float64)
    assert a.eps_E == pytest.approx(np.linalg.norm(M64 - a.Vstar @ a.Wstar) / np.linalg.norm(M64))
    # every column mixes between 3 and 8 atoms
    nnz = (a.Wstar > 0).sum(axis=0)
    assert nnz.min() >= 3 and nnz.max() <= 8


def test_planted_data_is_smooth_and_reachable():
    inst = synth.make_instance(synth.CFG_SMALL, 0)
    sM = O.smoothness(inst.M, 16, 16, O.XFER_BLOCK2)
    assert 0.01 < sM < 0.3
    floor = O.eckart_young_floor(inst.M, 10)
    assert floor <= inst.eps_E * (1 + 1e-9)       # planted rank-r product reaches eps_E
