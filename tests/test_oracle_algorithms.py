"""Pins for the oracle's inner NMF algorithms (Alg. 1-3, Appendix A)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.optimize as so

import oracle as O


def rand_problem(m, n, r, seed):
    rng = np.random.default_rng(seed)
    M = rng.uniform(size=(m, n))
    V = rng.uniform(size=(m, r))
    W = rng.uniform(size=(r, n))
    return M, V, W


# --------------------------------------------------------------------- HALS

@pytest.mark.parametrize("seed", range(6))
def test_hals_each_column_step_is_the_bruteforce_minimiser(seed):
    # Each V[:,k] (resp. W[k,:]) update is the exact minimiser of the objective
    # over that column (row) with the others fixed (Section 2.3).  The brute
    # force: a bounded least-squares solver on the one-column problem.
    M, V, W = rand_problem(5, 6, 3, seed)
    state = {"V": V.copy(), "W": W.copy()}

    def hook_v(which, k, Vnew):
        Vprev = state["V"]
        assert W[k, :].any()
        rest = M - np.delete(Vprev, k, axis=1) @ np.delete(W, k, axis=0)
        A = np.kron(W[k, :][:, None], np.eye(M.shape[0]))      # vec(v w_k^T) = (w_k (x) I) v
        sol = so.lsq_linear(A, rest.reshape(-1, order="F"), bounds=(0, np.inf),
                            tol=1e-14, method="bvls").x
        np.testing.assert_allclose(Vnew[:, k], sol, atol=1e-9)
        # the other columns are untouched by this step
        np.testing.assert_array_equal(np.delete(Vnew, k, 1), np.delete(Vprev, k, 1))
        state["V"] = Vnew.copy()

    Vn = O.hals_update_V(M, V, W, hook=hook_v)

    def hook_w(which, k, Wnew):
        Wprev = state["W"]
        if not Vn[:, k].any():
            # D_kk = 0: every row is a minimiser; the oracle keeps it (reading R6)
            np.testing.assert_array_equal(Wnew[k, :], Wprev[k, :])
            state["W"] = Wnew.copy()
            return
        rest = M - np.delete(Vn, k, axis=1) @ np.delete(Wprev, k, axis=0)
        A = np.kron(np.eye(M.shape[1]), Vn[:, k][:, None])     # vec(v_k w^T) = (I (x) v_k) w
        sol = so.lsq_linear(A, rest.reshape(-1, order="F"), bounds=(0, np.inf),
                            tol=1e-14, method="bvls").x
        np.testing.assert_allclose(Wnew[k, :], sol, atol=1e-9)
        state["W"] = Wnew.copy()

    O.hals_update_W(M, Vn, W, hook=hook_w)


def test_hals_objective_nonincreasing_after_every_column_update():
    M, V, W = rand_problem(12, 9, 4, 7)
    vals = [O.objective(M, V, W)]
    cur = {"W": W}
    Vn = O.hals_update_V(M, V, W, hook=lambda _, k, Vk: vals.append(O.objective(M, Vk, W)))
    O.hals_update_W(M, Vn, W, hook=lambda _, k, Wk: vals.append(O.objective(M, Vn, Wk)))
    assert len(vals) == 1 + 2 * 4
    assert all(b <= a * (1 + 1e-13) for a, b in zip(vals, vals[1:]))


def test_hals_zero_row_of_W_leaves_V_column_unchanged():
    M, V, W = rand_problem(6, 5, 3, 1)
    W[1, :] = 0.0
    Vn = O.hals_update_V(M, V, W)
    np.testing.assert_array_equal(Vn[:, 1], V[:, 1])


# ----------------------------------------------------------------------- MU

@pytest.mark.parametrize("seed", range(4))
def test_mu_each_half_step_is_nonincreasing(seed):
    M, V, W = rand_problem(15, 11, 4, seed)
    for _ in range(20):
        f0 = O.objective(M, V, W)
        V = O.mu_update_V(M, V, W)
        f1 = O.objective(M, V, W)
        W = O.mu_update_W(M, V, W)
        f2 = O.objective(M, V, W)
        assert f1 <= f0 * (1 + 1e-13) and f2 <= f1 * (1 + 1e-13)


def test_mu_zero_entries_stay_zero_and_scalar_case():
    M, V, W = rand_problem(8, 7, 3, 3)
    V[2, 1] = 0.0
    W[0, 4] = 0.0
    V2, W2 = O.mu_iteration(M, V, W)
    assert V2[2, 1] == 0.0 and W2[0, 4] == 0.0
    # 1x1x1: V <- V * (M W) / (V W W) = M / W exactly
    v = O.mu_update_V(np.array([[6.0]]), np.array([[5.0]]), np.array([[2.0]]))
    assert v[0, 0] == 3.0


# --------------------------------------------------------------------- ANLS

def enumerate_nnls(G, b):
    """Exhaustive search over all 2^r passive sets with a KKT check."""
    r = len(b)
    best = None
    for mask in itertools.product([False, True], repeat=r):
        idx = [i for i in range(r) if mask[i]]
        x = np.zeros(r)
        if idx:
            x[idx] = np.linalg.solve(G[np.ix_(idx, idx)], b[idx])
        g = G @ x - b
        if (x >= -1e-12).all() and all(abs(g[i]) < 1e-9 for i in idx) and \
                all(g[i] >= -1e-9 for i in range(r) if i not in idx):
            assert best is None or np.allclose(best, x, atol=1e-9), "KKT point not unique"
            best = x
    return best


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", range(10))
def test_nnls_equals_exhaustive_enumeration(r, seed):
    rng = np.random.default_rng(100 * r + seed)
    X = rng.normal(size=(r + 3, r))
    y = rng.normal(size=r + 3)
    G, b = X.T @ X, X.T @ y
    np.testing.assert_allclose(O.nnls_gram(G, b), enumerate_nnls(G, b), atol=1e-9)


@pytest.mark.parametrize("r", [5, 10, 20, 40])
def test_nnls_equals_scipy_nnls(r):
    rng = np.random.default_rng(r)
    for _ in range(5):
        X = np.abs(rng.normal(size=(3 * r, r)))
        y = rng.normal(size=3 * r) + 0.3
        ref, _ = so.nnls(X, y)
        got = O.nnls_gram(X.T @ X, X.T @ y)
        np.testing.assert_allclose(got, ref, atol=1e-8 * max(1, np.abs(ref).max()))


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", range(10))
def test_bpp_equals_exhaustive_enumeration(r, seed):
    # block principal pivoting (Section 2.1 footnote) reaches the unique
    # minimiser from an empty, a full and a random starting support
    rng = np.random.default_rng(500 + 100 * r + seed)
    X = rng.normal(size=(r + 3, r))
    y = rng.normal(size=r + 3)
    G, b = X.T @ X, X.T @ y
    want = enumerate_nnls(G, b)
    for start in (None, np.ones(r), rng.uniform(size=r) * (rng.uniform(size=r) > 0.5)):
        np.testing.assert_allclose(O.nnls_bpp(G, b, start), want, atol=1e-9)


@pytest.mark.parametrize("r", [5, 10, 20, 40, 64])
def test_bpp_equals_active_set_and_scipy(r):
    rng = np.random.default_rng(70 + r)
    for _ in range(5):
        X = np.abs(rng.normal(size=(3 * r, r)))
        y = rng.normal(size=3 * r) + 0.3
        ref, _ = so.nnls(X, y)
        G, b = X.T @ X, X.T @ y
        for start in (None, np.ones(r)):
            got = O.nnls_bpp(G, b, start)
            np.testing.assert_allclose(got, ref, atol=1e-8 * max(1, np.abs(ref).max()))
            np.testing.assert_allclose(got, O.nnls_gram(G, b), atol=1e-9 * max(1, np.abs(ref).max()))


def test_bpp_backup_rule_ends_a_cycling_exchange():
    # From the empty passive set, exchanging every infeasible variable at each
    # round cycles on this positive definite instance ({} -> {0,2} -> {1,2} ->
    # {} ...; found by a random search); the backup rule (single exchanges
    # once the count stops falling) ends it at the minimiser (0, 0, 0.2418).
    G = np.array([[2.8233, -1.9276, 4.3994], [-1.9276, 2.6995, -4.3377],
                  [4.3994, -4.3377, 8.3432]])
    b = np.array([0.2136, -1.6076, 2.0171])

    def full_exchange_round(passive):
        idx = np.flatnonzero(passive)
        z = np.zeros(3)
        z[idx] = np.linalg.solve(G[np.ix_(idx, idx)], b[idx]) if idx.size else 0.0
        bad = np.where(passive, z < 0, G[:, idx] @ z[idx] - b < -1e-12)
        return passive ^ bad

    p = np.zeros(3, dtype=bool)
    seen = [tuple(p)]
    for _ in range(3):
        p = full_exchange_round(p)
        seen.append(tuple(p))
    assert seen[3] == seen[0] and len(set(seen[:3])) == 3      # a 3-cycle
    want = enumerate_nnls(G, b)
    np.testing.assert_allclose(want, [0.0, 0.0, 2.0171 / 8.3432], atol=1e-12)
    np.testing.assert_allclose(O.nnls_bpp(G, b), want, atol=1e-12)


def test_bpp_zero_diagonal_variable_keeps_value():
    X = np.random.default_rng(0).uniform(size=(6, 3))
    X[:, 1] = 0.0
    y = np.random.default_rng(1).uniform(size=6)
    x = O.nnls_bpp(X.T @ X, X.T @ y, np.array([9.0, 7.0, 9.0]))
    assert x[1] == 7.0
    ref, _ = so.nnls(X[:, [0, 2]], y)
    np.testing.assert_allclose(x[[0, 2]], ref, atol=1e-10)


def test_anls_half_steps_are_exact_minimisers():
    M, V, W = rand_problem(20, 15, 5, 11)
    Vn = O.anls_update_V(M, V, W)
    for i in range(M.shape[0]):
        ref, _ = so.nnls(W.T, M[i, :])
        np.testing.assert_allclose(Vn[i], ref, atol=1e-9)
    Wn = O.anls_update_W(M, Vn, W)
    for j in range(M.shape[1]):
        ref, _ = so.nnls(Vn, M[:, j])
        np.testing.assert_allclose(Wn[:, j], ref, atol=1e-9)


def test_anls_ignores_initial_V():
    M, V, W = rand_problem(10, 8, 3, 5)
    a = O.anls_iteration(M, V, W)
    b = O.anls_iteration(M, np.zeros_like(V), W)
    np.testing.assert_allclose(a[0], b[0], atol=1e-13)
    np.testing.assert_allclose(a[1], b[1], atol=1e-13)


def test_nnls_zero_diagonal_variable_keeps_value():
    X = np.random.default_rng(0).uniform(size=(6, 3))
    X[:, 1] = 0.0
    y = np.random.default_rng(1).uniform(size=6)
    x = O.nnls_gram(X.T @ X, X.T @ y, x_keep=np.array([9.0, 7.0, 9.0]))
    assert x[1] == 7.0
    ref, _ = so.nnls(X[:, [0, 2]], y)
    np.testing.assert_allclose(x[[0, 2]], ref, atol=1e-10)


# -------------------------------------------------------------- all three

@pytest.mark.parametrize("algo", [O.HALS, O.MU, O.ANLS])
def test_exact_positive_factorisation_is_a_fixed_point(algo):
    rng = np.random.default_rng(42)
    Vs = rng.uniform(0.5, 1.5, size=(9, 3))
    Ws = rng.uniform(0.5, 1.5, size=(3, 7))
    M = Vs @ Ws
    V, W = O.iteration(algo, M, Vs, Ws)
    np.testing.assert_allclose(V, Vs, rtol=1e-9)
    np.testing.assert_allclose(W, Ws, rtol=1e-9)


@pytest.mark.parametrize("algo", [O.HALS, O.MU, O.ANLS])
def test_monotone_and_above_eckart_young(algo):
    M, V, W = rand_problem(30, 20, 4, 9)
    floor = O.eckart_young_floor(M, 4)
    prev = O.rel_err(M, V, W)
    for _ in range(15):
        V, W = O.iteration(algo, M, V, W)
        e = O.rel_err(M, V, W)
        assert e <= prev * (1 + 1e-12)
        assert e >= floor * (1 - 1e-12)
        assert (V >= 0).all() and (W >= 0).all()
        prev = e


def test_gram_form_residual_equals_direct_residual_exactly():
    # eq. subNNLS summed over columns, checked in exact rational arithmetic.
    rng = np.random.default_rng(3)
    M = rng.integers(0, 9, size=(5, 4)).astype(object)
    V = rng.integers(0, 5, size=(5, 2)).astype(object)
    W = rng.integers(0, 5, size=(2, 4)).astype(object)
    F = np.vectorize(Fraction)
    M, V, W = F(M), F(V), F(W)
    direct = np.sum((M - V.dot(W)) ** 2)
    normM2 = np.sum(M * M)
    got = O.gram_form_residual2(normM2, V.T.dot(M), W, V.T.dot(V), W.dot(W.T))
    assert got == direct


def test_rel_err_definition():
    M = np.array([[3.0, 0.0], [0.0, 4.0]])
    V = np.array([[1.0], [0.0]])
    W = np.array([[3.0, 0.0]])
    assert O.rel_err(M, V, W) == pytest.approx(4.0 / 5.0, abs=1e-15)


# ----------------------------------------------- bfloat16 product operands

def test_bf16_round_closed_forms():
    # 8 significant bits, ties to even (255 has exactly 8, 257 = 256 + 1 needs 9
    # and ties down to the even 256): 1 + 2^-8 lies half-way between 1 and
    # 1 + 2^-7 (mantissa 0 is even), 1 + 3*2^-8 half-way between 1 + 2^-7 and
    # 1 + 2^-6 (mantissa 2 is even); anything above a tie rounds up
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -3.0, 0.0,
                  255.0, 257.0, 2.0 ** -100, 0.1])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -3.0, 0.0, 255.0, 256.0, 2.0 ** -100,
                     0.10009765625])
    np.testing.assert_array_equal(O.bf16_round(x), want)


def test_bf16_round_equals_bit_rounding_of_float32():
    # independent route on FP32 inputs: keep the top 16 bits of the IEEE single
    # pattern after adding 0x7FFF plus the lowest kept bit (round to nearest even)
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    ref = (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(O.bf16_round(x.astype(np.float64)), ref)


@pytest.mark.parametrize("algo", [O.HALS, O.MU])
def test_bf16_iteration_reduces_to_the_plain_iteration(algo):
    # With M, V and W already bfloat16 values, the V half-step equals Alg. 3 /
    # Alg. 2 exactly; the W half-step equals the plain one applied to the
    # bfloat16-rounded new V.  A rounded Gram W W^T, a rounded update or a
    # product formed from the wrong operand breaks one of the two equalities.
    M, V, W = (O.bf16_round(a) for a in rand_problem(7, 6, 3, 11))
    V1, W1 = O.iteration_bf16(algo, M, V, W)
    Vp = (O.hals_update_V if algo == O.HALS else O.mu_update_V)(M, V, W)
    np.testing.assert_array_equal(V1, Vp)
    assert not np.array_equal(O.bf16_round(V1), V1)
    Wp = (O.hals_update_W if algo == O.HALS else O.mu_update_W)(M, O.bf16_round(V1), W)
    np.testing.assert_array_equal(W1, Wp)


def test_bf16_solve_refines_in_full_precision():
    # the scheduled iterations use the rounded products, the refinement the
    # plain ones; the log has both, and the tolerance only ends refinement steps
    M, V, W = rand_problem(64, 20, 3, 5)
    a = O.solve(M.astype(np.float32), 8, 8, 3, 2, O.HALS, O.NI, O.XFER_FW, 4, V, W,
                bf16_products=True, refine_iters=2)
    b = O.solve(M.astype(np.float32), 8, 8, 3, 2, O.HALS, O.NI, O.XFER_FW, 4, V, W)
    assert len(a.log) == len(b.log) + 2
    assert [d for d, _ in a.log[-2:]] == [0, 0]
    assert a.log[0][1] != b.log[0][1]
