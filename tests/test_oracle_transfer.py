"""Pins for the oracle's levels and transfer operators (Section 4.2)."""
import numpy as np
import pytest

import oracle as O
from conftest import load_golden

SIDES = [2, 3, 4, 5, 8, 9, 16, 17, 23, 28, 46, 56, 92, 112]


def test_fw_restriction_equals_printed_3x3_example():
    R = O.restrict_matrix(3, 3, O.XFER_FW)
    want = load_golden("fw_restrict_3x3_to_2x2.txt")
    assert R.shape == (4, 9)
    np.testing.assert_array_equal(np.rint(R * 9), want)
    np.testing.assert_allclose(R * 9, want, rtol=0, atol=1e-13)


def test_fw_prolongation_equals_printed_2x2_example():
    P = O.prolong_matrix(3, 3, O.XFER_FW)
    want = load_golden("fw_prolong_2x2_to_3x3_transposed.txt")
    assert P.shape == (9, 4)
    np.testing.assert_allclose(P.T * 4, want, rtol=0, atol=1e-13)


def test_fw_interior_weights_are_eq_restr():
    # On a (2^a+1) grid, an interior coarse pixel uses weights
    # (1,2,1) x (1,2,1) / 16 centred on fine pixel (2i, 2j) (eq. restr).
    h = w = 9
    R = O.restrict_matrix(h, w, O.XFER_FW)
    hc, wc = 5, 5
    stencil = np.outer([1, 2, 1], [1, 2, 1]) / 16.0
    for ci in range(1, hc - 1):
        for cj in range(1, wc - 1):
            row = R[ci * wc + cj].reshape(h, w)
            want = np.zeros((h, w))
            want[2 * ci - 1:2 * ci + 2, 2 * cj - 1:2 * cj + 2] = stencil
            np.testing.assert_allclose(row, want, atol=1e-15)


def test_prolongation_rd_rule():
    # eq. prol: fine (i, j) is the mean of coarse rd(i/2) x rd(j/2).
    h, w = 9, 7
    P = O.prolong_matrix(h, w, O.XFER_FW)
    hc, wc = 5, 4

    def rd(k, nc):
        s = [k // 2] if k % 2 == 0 else [(k - 1) // 2, (k + 1) // 2]
        return [c for c in s if c < nc]

    for i in range(h):
        for j in range(w):
            nb = [(a, b) for a in rd(i, hc) for b in rd(j, wc)]
            want = np.zeros(hc * wc)
            for a, b in nb:
                want[a * wc + b] = 1.0 / len(nb)
            np.testing.assert_allclose(P[i * w + j], want, atol=1e-15)


@pytest.mark.parametrize("xfer", [O.XFER_FW, O.XFER_BLOCK2])
@pytest.mark.parametrize("N", SIDES)
def test_1d_operators_nonnegative_and_averaging(xfer, N):
    R, P = O.transfer_1d(N, xfer)
    assert R.shape == ((N + 1) // 2, N) and P.shape == (N, (N + 1) // 2)
    assert (R >= 0).all() and (P >= 0).all()          # Section 4.1 condition
    np.testing.assert_allclose(R.sum(axis=1), 1.0, atol=1e-15)   # weighted average
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-15)   # mean of neighbours


@pytest.mark.parametrize("N", [3, 5, 9, 17, 33])
def test_fw_second_order_on_odd_grids(N):
    # Full weighting is exact for linear data at interior nodes, and the
    # prolongation (linear interpolation) reproduces coarse linear data exactly.
    R, P = O.transfer_1d(N, O.XFER_FW)
    f = 0.3 + 1.7 * np.arange(N)
    rf = R @ f
    coarse_pos = 2 * np.arange(R.shape[0])
    np.testing.assert_allclose(rf[1:-1], 0.3 + 1.7 * coarse_pos[1:-1], atol=1e-12)
    g = -2.0 + 0.5 * coarse_pos
    np.testing.assert_allclose(P @ g, -2.0 + 0.5 * np.arange(N), atol=1e-12)


@pytest.mark.parametrize("N", [2, 4, 8, 16, 92])
def test_block2_identities(N):
    R, P = O.transfer_1d(N, O.XFER_BLOCK2)
    np.testing.assert_allclose(R @ P, np.eye(R.shape[0]), atol=1e-15)
    x = np.random.default_rng(0).uniform(size=N)
    assert abs(2 * (R @ x).sum() - x.sum()) < 1e-12   # column mass (per axis)


def test_block2_2d_mass():
    h, w = 16, 16
    R = O.restrict_matrix(h, w, O.XFER_BLOCK2)
    x = np.random.default_rng(1).uniform(size=h * w)
    assert abs(4 * (R @ x).sum() - x.sum()) < 1e-12


@pytest.mark.parametrize("xfer", [O.XFER_FW, O.XFER_BLOCK2])
@pytest.mark.parametrize("hw", [(3, 3), (4, 5), (9, 17), (16, 16), (23, 28)])
def test_separable_application_equals_kronecker(xfer, hw):
    h, w = hw
    X = np.random.default_rng(2).uniform(size=(h * w, 7))
    np.testing.assert_allclose(O.restrict_images(X, h, w, xfer),
                               O.restrict_matrix(h, w, xfer) @ X, atol=1e-13)
    Y = np.random.default_rng(3).uniform(size=(((h + 1) // 2) * ((w + 1) // 2), 5))
    np.testing.assert_allclose(O.prolong_images(Y, h, w, xfer),
                               O.prolong_matrix(h, w, xfer) @ Y, atol=1e-13)


def test_restriction_preserves_nonnegativity_of_images():
    X = np.abs(np.random.default_rng(4).normal(size=(112 * 92, 3)))
    assert (O.restrict_images(X, 112, 92, O.XFER_FW) >= 0).all()
    Y = np.abs(np.random.default_rng(5).normal(size=(56 * 46, 3)))
    assert (O.prolong_images(Y, 112, 92, O.XFER_FW) >= 0).all()


def test_level_sides():
    # (2^a+1) x (2^b+1) -> (2^(a-1)+1) x (2^(b-1)+1)  (Section 4.2, Fig. 2)
    assert O.level_sides(17, 33, 3) == [(17, 33), (9, 17), (5, 9)]
    assert O.level_sides(112, 92, 3) == [(112, 92), (56, 46), (28, 23)]
    assert O.level_sides(256, 256, 4) == [(256, 256), (128, 128), (64, 64), (32, 32)]
    assert O.level_sides(16, 16, 2) == [(16, 16), (8, 8)]
    with pytest.raises(ValueError):
        O.level_sides(2, 1, 2)
    with pytest.raises(ValueError):
        O.level_sides(4, 4, 0)


def test_smoothness_of_smooth_and_rough_data():
    h = w = 33
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    smooth = np.exp(-((yy - 16.0) ** 2 + (xx - 12.0) ** 2) / 200.0).reshape(-1, 1)
    rough = np.random.default_rng(6).uniform(size=(h * w, 1))
    assert O.smoothness(smooth, h, w, O.XFER_FW) < 0.02
    assert O.smoothness(rough, h, w, O.XFER_FW) > 0.1
