"""Pins for the oracle's two-sided hierarchy (Section 6.1: the multilevel
strategy generalised to the column index, for columns ordered along a smooth
axis such as wavelength or time)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def test_column_restriction_weights_written_out():
    # eq. restr's 1-D weights along the column index: interior (1,2,1)/4,
    # boundary rows renormalised over the fine neighbours that exist (R2)
    a, b, c, d, e = 1.0, 2.0, 4.0, 8.0, 16.0
    X = np.array([[a, b, c, d, e]])
    want = [(2 * a + b) / 3, (b + 2 * c + d) / 4, (d + 2 * e) / 3]
    np.testing.assert_allclose(O.restrict_cols(X, O.XFER_FW), [want], rtol=1e-15)
    # even count: the last coarse node has neighbours 2c-1, 2c only
    X = np.array([[a, b, c, d]])
    np.testing.assert_allclose(O.restrict_cols(X, O.XFER_FW), [[(2 * a + b) / 3, (b + 2 * c + d) / 4]],
                               rtol=1e-15)
    # BLOCK2: pair means
    np.testing.assert_allclose(O.restrict_cols(np.array([[a, b, c, d, e]]), O.XFER_BLOCK2),
                               [[(a + b) / 2, (c + d) / 2, e]], rtol=1e-15)


def test_column_prolongation_weights_written_out():
    # eq. prol along the column index: even f copies coarse f/2, odd f averages
    # the coarse neighbours (f-1)/2, (f+1)/2 that exist (R3)
    Y = np.array([[1.0, 3.0, 7.0]])
    np.testing.assert_allclose(O.prolong_cols(Y, 5, O.XFER_FW), [[1.0, 2.0, 3.0, 5.0, 7.0]])
    np.testing.assert_allclose(O.prolong_cols(Y, 6, O.XFER_FW), [[1.0, 2.0, 3.0, 5.0, 7.0, 7.0]])


@pytest.mark.parametrize("n", [2, 3, 7, 64, 65])
@pytest.mark.parametrize("xfer", [O.XFER_FW, O.XFER_BLOCK2])
def test_column_transfers_preserve_constants_and_sign(n, xfer):
    rng = np.random.default_rng(n)
    ones = np.ones((3, n))
    np.testing.assert_allclose(O.restrict_cols(ones, xfer), 1.0, rtol=1e-15)
    np.testing.assert_allclose(O.prolong_cols(np.ones((3, (n + 1) // 2)), n, xfer), 1.0, rtol=1e-15)
    X = rng.uniform(size=(4, n))
    assert (O.restrict_cols(X, xfer) >= 0).all() and (O.prolong_cols(X[:, :(n + 1) // 2], n, xfer) >= 0).all()


def test_level_column_counts():
    assert O.level_ns(400, 4) == [400, 200, 100, 50]
    assert O.level_ns(33, 3) == [33, 17, 9]
    with pytest.raises(ValueError):
        O.level_ns(1, 2)


def test_schedule_with_two_sided_cost_ratio():
    # the Table 1 time split is unchanged; a depth-d run converts its budget at
    # 8^d iterations per fine-iteration equivalent (m/4 and n/2 per level)
    T = 16
    ni = O.schedule(O.NI, 2, T, 8)
    assert ni == [("restrict", 0, 0), ("run", 1, 2 * T), ("prolong", 0, 0), ("run", 0, 3 * T // 4)]
    for L in (2, 3, 4):
        tot_ni = O.level_iteration_totals(O.schedule(O.NI, L, 64, 8), L)
        tot_vc = O.level_iteration_totals(O.schedule(O.VC, L, 64, 8), L)
        assert tot_ni == tot_vc
        want = [int(Fraction(3, 4) * 64 * Fraction(8, 4) ** d) for d in range(L - 1)]
        want.append(int(64 * Fraction(8, 4) ** (L - 1)))
        assert tot_ni == want


def test_two_sided_block_exact_factorisation_is_kept():
    # M = (P_m V') (W' P_n^T) with BLOCK2 operators (R P = I on both sides):
    # every coarse level holds the restricted exact factors, so rel_err stays
    # at rounding level through restriction, coarse sweeps and prolongation.
    # A wrong W transfer (or none) breaks this.
    rng = np.random.default_rng(3)
    h, w, n, r = 8, 8, 24, 3
    Vc = rng.uniform(0.5, 1.0, size=(16, r))
    Wc = rng.uniform(0.5, 1.0, size=(r, 12))
    V0 = O.prolong_images(Vc, h, w, O.XFER_BLOCK2)
    W0 = O.prolong_cols(Wc, n, O.XFER_BLOCK2)
    M = V0 @ W0
    for algo in (O.HALS, O.MU, O.ANLS):
        res = O.solve(M, h, w, r, 2, algo, O.VC, O.XFER_BLOCK2, 8, V0, W0, two_sided=True)
        assert max(e for _, e in res.log) < 1e-10, algo
        assert {d for d, _ in res.log} == {0, 1}


@pytest.mark.parametrize("algo", [O.HALS, O.MU, O.ANLS])
@pytest.mark.parametrize("xfer", [O.XFER_FW, O.XFER_BLOCK2])
def test_two_sided_prolongation_bound_holds(algo, xfer):
    rng = np.random.default_rng(11)
    h, w, n, r = 12, 10, 30, 4
    # smooth along both axes: products of smooth images and smooth spectra
    yy, xx = np.mgrid[0:h, 0:w]
    imgs = np.stack([np.exp(-((yy - rng.uniform(0, h)) ** 2 + (xx - rng.uniform(0, w)) ** 2) / 8.0).ravel()
                     for _ in range(r)], axis=1)
    t = np.arange(n)
    spec = np.stack([np.exp(-(t - rng.uniform(0, n)) ** 2 / 40.0) for _ in range(r)])
    M = imgs @ spec + 0.01 * rng.uniform(size=(h * w, n))
    V0, W0 = rng.uniform(size=(h * w, r)), rng.uniform(size=(r, n))
    res = O.solve(M, h, w, r, 3, algo, O.FMG, xfer, 8, V0, W0, two_sided=True, check_bound=True)
    assert len(res.bound_checks) >= 2
    for lhs, rhs in res.bound_checks:
        assert lhs <= rhs * (1 + 1e-12)


def test_two_sided_levels_hold_the_restricted_data():
    # the coarse matrices are R_m M R_n^T, the Kronecker operator written out
    rng = np.random.default_rng(5)
    h, w, n = 6, 5, 9
    M = rng.uniform(size=(h * w, n))
    Rm = O.restrict_matrix(h, w, O.XFER_FW)
    Rn, _ = O.transfer_1d(n, O.XFER_FW)
    seen = {}

    def cb(d, V, W, e):
        seen.setdefault(d, (V.shape, W.shape))

    O.solve(M, h, w, 2, 2, O.HALS, O.NI, O.XFER_FW, 4, rng.uniform(size=(h * w, 2)),
            rng.uniform(size=(2, n)), two_sided=True, callback=cb)
    assert seen[1] == ((9, 2), (2, 5)) and seen[0] == ((30, 2), (2, 9))
    np.testing.assert_allclose(O.restrict_cols(O.restrict_images(M, h, w, O.XFER_FW), O.XFER_FW),
                               Rm @ M @ Rn.T, rtol=1e-13)
