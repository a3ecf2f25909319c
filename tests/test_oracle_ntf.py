"""Pins of the oracle's nonnegative tensor factorisation (reading R18:
Section 7.1's multilevel NTF), each fixed by something other than the
oracle's own formulas:
  * the unfoldings and Khatri-Rao products agree with the CP tensor built by
    einsum (X_(1) = A (C kr B)^T and the other two), and element by element
    with the index convention X_(1)[i, j + J k] = X[i, j, k];
  * the Gram of a Khatri-Rao product is the Hadamard product of the Grams;
  * for rank 1 the A update is the closed-form least-squares vector
    X x_2 b x_3 c / (|b|^2 |c|^2);
  * an exact positive CP tensor is a fixed point of the iteration;
  * the objective does not increase over any of the three mode updates;
  * the coarse tensor is the restriction of every frontal slice's image.
"""
import numpy as np
import pytest

import oracle as O


def _rand(rng, I, J, K, R, lo=0.1):
    return (rng.uniform(lo, 1, (I, R)), rng.uniform(lo, 1, (J, R)), rng.uniform(lo, 1, (K, R)))


def test_unfoldings_match_cp_tensor():
    rng = np.random.default_rng(0)
    I, J, K, R = 6, 5, 4, 3
    A, B, C = _rand(rng, I, J, K, R)
    X = O.cp_tensor(A, B, C)
    np.testing.assert_allclose(O.unfold(X, 1), A @ O.khatri_rao(C, B).T, rtol=1e-13)
    np.testing.assert_allclose(O.unfold(X, 2), B @ O.khatri_rao(C, A).T, rtol=1e-13)
    np.testing.assert_allclose(O.unfold(X, 3), C @ O.khatri_rao(B, A).T, rtol=1e-13)
    X1 = O.unfold(X, 1)
    for _ in range(50):
        i, j, k = rng.integers(I), rng.integers(J), rng.integers(K)
        assert X1[i, j + J * k] == X[i, j, k]
        assert O.khatri_rao(C, B)[j + J * k, 1] == C[k, 1] * B[j, 1]
    np.testing.assert_array_equal(O.fold1(X1, J, K), X)


def test_khatri_rao_gram_is_hadamard_of_grams():
    rng = np.random.default_rng(1)
    B = rng.uniform(size=(7, 4))
    C = rng.uniform(size=(5, 4))
    KR = O.khatri_rao(C, B)
    np.testing.assert_allclose(KR.T @ KR, (C.T @ C) * (B.T @ B), rtol=1e-13)


def test_rank_one_update_is_closed_form():
    rng = np.random.default_rng(2)
    X = rng.uniform(0.1, 1.0, size=(8, 6, 5))
    A, B, C = _rand(rng, 8, 6, 5, 1)
    A1, _, _ = O.ntf_iteration(X, A, B, C)
    b, c = B[:, 0], C[:, 0]
    ref = np.einsum("ijk,j,k->i", X, b, c) / ((b @ b) * (c @ c))
    np.testing.assert_allclose(A1[:, 0], ref, rtol=1e-13)


def test_exact_cp_tensor_is_fixed_point():
    rng = np.random.default_rng(3)
    A, B, C = _rand(rng, 9, 7, 6, 3, lo=0.3)
    X = O.cp_tensor(A, B, C)
    A1, B1, C1 = O.ntf_iteration(X, A, B, C)
    for P, Q in ((A1, A), (B1, B), (C1, C)):
        np.testing.assert_allclose(P, Q, rtol=1e-11)
    assert O.ntf_rel_err(X, A1, B1, C1) < 1e-12


def test_objective_nonincreasing_per_mode():
    rng = np.random.default_rng(4)
    X = rng.uniform(0.0, 1.0, size=(12, 9, 8))
    A, B, C = _rand(rng, 12, 9, 8, 4)
    f = lambda A_, B_, C_: float(np.sum((X - O.cp_tensor(A_, B_, C_)) ** 2))
    prev = f(A, B, C)
    for _ in range(15):
        A = O.hals_update_V(O.unfold(X, 1), A, O.khatri_rao(C, B).T)
        f1 = f(A, B, C)
        B = O.hals_update_V(O.unfold(X, 2), B, O.khatri_rao(C, A).T)
        f2 = f(A, B, C)
        C = O.hals_update_V(O.unfold(X, 3), C, O.khatri_rao(B, A).T)
        f3 = f(A, B, C)
        assert f1 <= prev * (1 + 1e-12) and f2 <= f1 * (1 + 1e-12) and f3 <= f2 * (1 + 1e-12)
        prev = f3


def test_multilevel_solve_restricts_every_slice():
    rng = np.random.default_rng(5)
    h, w, J, K, R = 8, 6, 5, 4, 3
    X = rng.uniform(0.0, 1.0, size=(h * w, J, K))
    A0, B0, C0 = _rand(rng, h * w, J, K, R)
    seen = {}

    def cb(d, A, B, C, e):
        seen.setdefault(d, A.shape)

    res = O.solve_ntf(X, h, w, R, 2, O.VC, O.XFER_FW, 8, A0, B0, C0, callback=cb)
    assert seen == {0: (48, 3), 1: (12, 3)}
    assert res.log[-1][1] == pytest.approx(O.ntf_rel_err(X, res.A, res.B, res.C), rel=1e-12)
    # the coarse tensor: every frontal slice's image restricted on its own
    Xc = O.fold1(O.restrict_images(O.unfold(X, 1), h, w, O.XFER_FW), J, K)
    for j in range(J):
        for k in range(K):
            np.testing.assert_allclose(
                Xc[:, j, k], O.restrict_images(X[:, j, k][:, None], h, w, O.XFER_FW)[:, 0],
                rtol=1e-14)
