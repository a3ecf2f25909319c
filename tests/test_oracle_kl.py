"""Pins of the oracle's Kullback-Leibler objective (reading R17: Section 7.1's
other objective functions, minimised by the Lee-Seung multiplicative
updates).  Each check is fixed by mathematics, not by retyping the oracle:
  * the divergence equals the sum of scipy.special.kl_div (its elementwise
    definition x log(x/y) - x + y), including 0 log 0 = 0;
  * after the V update the row sums of V W equal those of M, and after the W
    update the column sums do (the updates' normalising denominators make
    this exact);
  * the divergence does not increase over either half-update (Lee and Seung's
    auxiliary-function argument);
  * an exact positive factorisation is a fixed point;
  * the V update is the gradient step V - (V / (1 W^T)) o grad_V D, with the
    gradient taken by central differences of the divergence;
  * zero rows of W / columns of V keep the matching factor entries (R17, as R7).
"""
import numpy as np
import pytest
from scipy.special import kl_div

import oracle as O


def _pos(rng, m, n, r, lo=0.1):
    V = rng.uniform(lo, 1.0, size=(m, r))
    W = rng.uniform(lo, 1.0, size=(r, n))
    M = rng.uniform(0.0, 1.0, size=(m, n)) * (V @ W) * 2.0
    return M, V, W


def test_divergence_is_scipy_kl_div_sum():
    rng = np.random.default_rng(0)
    M, V, W = _pos(rng, 13, 9, 4)
    M[2, 3] = 0.0                       # 0 log 0 = 0: the term is (VW)_23
    M[5, :] = 0.0
    ref = float(np.sum(kl_div(M, V @ W)))
    assert O.kl_divergence(M, V, W) == pytest.approx(ref, rel=1e-13)
    assert O.rel_kl(M, V, W) == pytest.approx(ref / M.sum(), rel=1e-13)
    # closed form of one term: D(2 | 1) = 2 log 2 - 1
    assert O.kl_divergence(np.array([[2.0]]), np.array([[1.0]]), np.array([[1.0]])) == \
        pytest.approx(2 * np.log(2) - 1, rel=1e-15)
    # zero fit where M > 0: infinite
    assert O.kl_divergence(np.array([[1.0]]), np.array([[0.0]]), np.array([[1.0]])) == np.inf


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_half_updates_match_margins(seed):
    rng = np.random.default_rng(seed)
    M, V, W = _pos(rng, 20, 15, 5)
    V1 = O.kl_update_V(M, V, W)
    np.testing.assert_allclose((V1 @ W).sum(axis=1), M.sum(axis=1), rtol=1e-12)
    W1 = O.kl_update_W(M, V1, W)
    np.testing.assert_allclose((V1 @ W1).sum(axis=0), M.sum(axis=0), rtol=1e-12)


def test_divergence_nonincreasing():
    rng = np.random.default_rng(4)
    M, V, W = _pos(rng, 30, 25, 6)
    prev = O.kl_divergence(M, V, W)
    for _ in range(40):
        V = O.kl_update_V(M, V, W)
        d1 = O.kl_divergence(M, V, W)
        W = O.kl_update_W(M, V, W)
        d2 = O.kl_divergence(M, V, W)
        assert d1 <= prev * (1 + 1e-14) and d2 <= d1 * (1 + 1e-14)
        prev = d2
    assert prev < O.kl_divergence(*_pos(np.random.default_rng(4), 30, 25, 6)) * 0.9


def test_exact_factorisation_is_fixed_point():
    rng = np.random.default_rng(5)
    V = rng.uniform(0.2, 1.0, size=(12, 3))
    W = rng.uniform(0.2, 1.0, size=(3, 8))
    M = V @ W
    V1, W1 = O.kl_iteration(M, V, W)
    np.testing.assert_allclose(V1, V, rtol=1e-13)
    np.testing.assert_allclose(W1, W, rtol=1e-13)
    assert abs(O.kl_divergence(M, V1, W1)) < 1e-12


def test_update_is_scaled_gradient_step():
    rng = np.random.default_rng(6)
    M, V, W = _pos(rng, 7, 6, 3)
    h = 1e-6
    G = np.zeros_like(V)
    for i in range(V.shape[0]):
        for k in range(V.shape[1]):
            Vp, Vm = V.copy(), V.copy()
            Vp[i, k] += h
            Vm[i, k] -= h
            G[i, k] = (O.kl_divergence(M, Vp, W) - O.kl_divergence(M, Vm, W)) / (2 * h)
    step = V - V / W.sum(axis=1)[None, :] * G
    np.testing.assert_allclose(O.kl_update_V(M, V, W), step, rtol=1e-7, atol=1e-9)
    # and for W: W - (W / (V^T 1)) o grad_W D
    GW = np.zeros_like(W)
    for k in range(W.shape[0]):
        for j in range(W.shape[1]):
            Wp, Wm = W.copy(), W.copy()
            Wp[k, j] += h
            Wm[k, j] -= h
            GW[k, j] = (O.kl_divergence(M, V, Wp) - O.kl_divergence(M, V, Wm)) / (2 * h)
    stepW = W - W / V.sum(axis=0)[:, None] * GW
    np.testing.assert_allclose(O.kl_update_W(M, V, W), stepW, rtol=1e-7, atol=1e-9)


def test_zero_rows_and_columns_keep_entries():
    rng = np.random.default_rng(7)
    M, V, W = _pos(rng, 10, 8, 4)
    W[2, :] = 0.0                       # sum_j W_2j = 0: column 2 of V kept
    V[:, 1] = 0.0                       # sum_i V_i1 = 0: row 1 of W kept
    V1 = O.kl_update_V(M, V, W)
    np.testing.assert_array_equal(V1[:, 2], V[:, 2])
    W1 = O.kl_update_W(M, V1, W)
    np.testing.assert_array_equal(W1[1, :], W[1, :])
    assert np.all(np.isfinite(V1)) and np.all(np.isfinite(W1))


def test_multilevel_solve_logs_relative_divergence():
    """The KL solve runs at every level of the hierarchy, logs a nonnegative
    relative divergence, and its last entry is D(M | V W) / sum(M) of the
    returned factors."""
    import synth
    inst = synth.make_instance(synth.CFG_SMALL, 0)
    seen = []

    def cb(d, V, W, e):
        seen.append((d, e, V.shape[0]))

    res = O.solve(inst.M, 16, 16, 10, 2, O.KL, O.NI, O.XFER_BLOCK2, 8, inst.V0, inst.W0,
                  callback=cb)
    assert {d for d, _, _ in seen} == {0, 1}
    assert all(mm == (64 if d == 1 else 256) for d, _, mm in seen)
    # the last logged value is the divergence of the returned factors
    assert res.log[-1][1] == pytest.approx(O.rel_kl(inst.M, res.V, res.W), rel=1e-12)
    # each logged coarse value is a relative divergence of the coarse matrix
    assert all(e >= 0 for _, e, _ in seen)
