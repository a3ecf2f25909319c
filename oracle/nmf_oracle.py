"""Plain, slow, FP64 reference implementation of multilevel NMF.

TEST INFRASTRUCTURE ONLY.  This module is the correctness oracle for the HIP
library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it.  It shares no code, tables or helpers with the
GPU path.

Paper: N. Gillis and F. Glineur, "A Multilevel Approach for Nonnegative Matrix
Factorization" (arXiv:1009.0881).  Every function cites the passage it follows.
Everything is numpy float64; inputs are the generator's FP32 arrays widened
exactly.  Library primitives (matmul, solve, svd, norm) serve as single steps;
there is no blocking, fusion or reordering beyond what the paper states.

Readings of passages where the paper is silent (each one also listed in the
design notes):
  R1  levels: h_{l+1} = ceil(h_l / 2); coarse node c sits on fine node 2c.
      Reduces to the paper's (2^a+1) -> (2^(a-1)+1) grid (Section 4.2, Fig. 2).
  R2  full weighting at a boundary: keep the 1-D weights (1,2,1) of the fine
      neighbours that exist and renormalise each row to sum 1 ("weights adapted
      correspondingly", eq. restr).  Reproduces the printed 3x3 -> 2x2 R.
  R3  prolongation at an even-side edge: the mean over the coarse neighbours
      rd(i/2) that exist (eq. prol).  Reproduces the printed P^T.
  R4  BLOCK2 (2x2 pixel-block restriction, not in the paper): restriction is
      the block mean, prolongation replicates.
  R5  schedule: the time budget T of Alg. 4-6 is counted in fine-iteration
      equivalents with the paper's cost model m' ~ m/4 (Section 4.3, Table 1);
      Run(d, t) performs floor(t * 4^d) iterations at depth d.
  R6  HALS with B_kk = 0 (resp. D_kk = 0): that column of V (row of W) is left
      unchanged (every value minimises its one-column problem).
  R7  MU with a zero denominator: that entry is left unchanged (it is then 0).
  R8  ANLS: NNLS by the Lawson-Hanson active-set method on the Gram form
      (Appendix A.2); variables whose Gram diagonal is 0 keep their value.
  R9  error: e = ||M_l - V W||_F (not squared) and rel_err = e / ||M_l||_F,
      evaluated after every full iteration at the current level.
  R10 stopping: with tol > 0 the solve ends after the first finest-level
      iteration whose rel_err <= tol; after the schedule, finest-level
      iterations continue until then or until max_fine_iters more iterations.
  R13 W-cycle (Section 7.1 names other cycles as future work): the V-cycle's
      time split with the coarse quarter spent in two consecutive W-cycles
      of one eighth each at the next level.
  R17 KL objective (Section 7.1 names other objective functions): the
      generalized Kullback-Leibler divergence D(M | VW) = sum M log(M/(VW))
      - M + VW (0 log 0 = 0), minimised by the multiplicative updates of Lee
      and Seung: V <- V o [(M / VW) W^T] / [1 W^T], then W <- W o [V^T (M /
      VW)] / [V^T 1].  The hierarchy, transfers and schedule are unchanged;
      the logged error of an iteration is D(M_l | VW) / sum(M_l).  Where
      (VW)_ij = 0 the ratio M_ij / (VW)_ij is taken as 0; a zero denominator
      (a zero row of W or column of V) leaves the entry unchanged, as R7.
  R18 NTF (Section 7.1: multilevel techniques for nonnegative tensor
      factorisation): a 3-way tensor X (I x J x K) whose mode 1 is the pixel
      index of an h x w grid, approximated by sum_r a_r o b_r o c_r with
      A (I x R), B (J x R), C (K x R) >= 0.  One iteration updates A, then B,
      then C, each by the HALS steps of Alg. 3 on that mode's unfolding
      (X_(1) = A (C kr B)^T, X_(2) = B (C kr A)^T, X_(3) = C (B kr A)^T, kr
      the Khatri-Rao product, column (j, k) of X_(1) at j + J k).  Mode 1 is
      coarsened as the images are (X_(1) restricted by rows, A transferred as
      V); B and C stay on every level.  The error is ||X - [[A, B, C]]||_F /
      ||X||_F after each iteration; schedule, budget and stopping as R5, R10.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

HALS, MU, ANLS, KL = 0, 1, 2, 3
NI, VC, FMG, WC = 0, 1, 2, 3
XFER_FW, XFER_BLOCK2 = 0, 1

ALGO_NAMES = {HALS: "hals", MU: "mu", ANLS: "anls", KL: "kl"}
CYCLE_NAMES = {NI: "ni", VC: "vc", FMG: "fmg", WC: "wc"}

__all__ = [
    "HALS", "MU", "ANLS", "KL", "NI", "VC", "FMG", "WC", "XFER_FW", "XFER_BLOCK2",
    "level_sides", "transfer_1d", "restrict_matrix", "prolong_matrix",
    "restrict_images", "prolong_images", "smoothness", "level_ns", "restrict_cols",
    "prolong_cols", "prolongation_bound_two_sided",
    "schedule", "level_iteration_totals",
    "hals_update_V", "hals_update_W", "hals_iteration",
    "mu_update_V", "mu_update_W", "mu_iteration",
    "nnls_gram", "nnls_bpp", "anls_update_V", "anls_update_W", "anls_iteration",
    "kl_ratio", "kl_divergence", "rel_kl", "kl_update_V", "kl_update_W", "kl_iteration",
    "khatri_rao", "unfold", "fold1", "cp_tensor", "ntf_iteration", "ntf_rel_err", "solve_ntf",
    "NtfResult",
    "iteration", "bf16_round", "hals_update_V_bf16", "hals_update_W_bf16",
    "mu_iteration_bf16", "iteration_bf16", "rel_err", "objective", "gram_form_residual2",
    "eckart_young_floor", "prolongation_bound", "solve", "SolveResult",
]


# ---------------------------------------------------------------------------
# Levels and transfer operators (Section 4.2: Fig. 2, eq. restr, eq. prol)
# ---------------------------------------------------------------------------

def level_sides(h: int, w: int, levels: int) -> List[Tuple[int, int]]:
    """Image sides per level, finest first (reading R1).

    Section 4.2 keeps one grid point out of two in each direction.  A side
    smaller than 2 cannot be restricted further and is rejected.
    """
    if levels < 1:
        raise ValueError("levels must be >= 1")
    sides = [(h, w)]
    for _ in range(levels - 1):
        ph, pw = sides[-1]
        if ph < 2 or pw < 2:
            raise ValueError("cannot restrict a side smaller than 2")
        sides.append(((ph + 1) // 2, (pw + 1) // 2))
    return sides


def transfer_1d(N: int, xfer: int) -> Tuple[np.ndarray, np.ndarray]:
    """1-D restriction R1 (N' x N) and prolongation P1 (N x N'), N' = ceil(N/2).

    FW (eq. restr read per axis): coarse node c averages fine nodes 2c-1, 2c,
    2c+1 with weights 1, 2, 1; missing nodes are dropped and the row is
    renormalised (reading R2).  Prolongation (eq. prol): fine node f takes the
    mean of the coarse nodes rd(f/2) = {f/2} (f even) or {(f-1)/2, (f+1)/2}
    (f odd) that exist (reading R3).

    BLOCK2 (reading R4): coarse c is the mean of fine {2c, 2c+1} that exist;
    fine f copies coarse floor(f/2).
    """
    Nc = (N + 1) // 2
    R = np.zeros((Nc, N))
    P = np.zeros((N, Nc))
    if xfer == XFER_FW:
        for c in range(Nc):
            for delta, wgt in ((-1, 1.0), (0, 2.0), (1, 1.0)):
                f = 2 * c + delta
                if 0 <= f < N:
                    R[c, f] = wgt
            R[c, :] /= R[c, :].sum()
        for f in range(N):
            if f % 2 == 0:
                nb = [f // 2]
            else:
                nb = [(f - 1) // 2, (f + 1) // 2]
            nb = [c for c in nb if 0 <= c < Nc]
            for c in nb:
                P[f, c] = 1.0 / len(nb)
    elif xfer == XFER_BLOCK2:
        for c in range(Nc):
            fs = [f for f in (2 * c, 2 * c + 1) if f < N]
            for f in fs:
                R[c, f] = 1.0 / len(fs)
        for f in range(N):
            P[f, f // 2] = 1.0
    else:
        raise ValueError("unknown transfer operator")
    return R, P


def restrict_matrix(h: int, w: int, xfer: int) -> np.ndarray:
    """Dense 2-D restriction R = R_h (x) R_w for row-major vectorised h x w
    images (pixel (y, x) -> y*w + x); Section 4.2 allows either vectorisation
    order.  Dense: only for small images (tests)."""
    Rh, _ = transfer_1d(h, xfer)
    Rw, _ = transfer_1d(w, xfer)
    return np.kron(Rh, Rw)


def prolong_matrix(h: int, w: int, xfer: int) -> np.ndarray:
    """Dense 2-D prolongation P = P_h (x) P_w from the ceil(h/2) x ceil(w/2)
    grid to the h x w grid (Section 4.2, eq. prol)."""
    _, Ph = transfer_1d(h, xfer)
    _, Pw = transfer_1d(w, xfer)
    return np.kron(Ph, Pw)


def restrict_images(X: np.ndarray, h: int, w: int, xfer: int) -> np.ndarray:
    """R(X) applied columnwise (Section 4.1): each column of X is a row-major
    h x w image.  Uses the separable form R_h X_img R_w^T, which equals the
    Kronecker operator applied to the vectorised image."""
    Rh, _ = transfer_1d(h, xfer)
    Rw, _ = transfer_1d(w, xfer)
    ncol = X.shape[1]
    imgs = np.asarray(X, dtype=np.float64).T.reshape(ncol, h, w)
    out = np.einsum("ay,nyx,bx->nab", Rh, imgs, Rw, optimize=True)
    return out.reshape(ncol, -1).T.copy()


def prolong_images(Y: np.ndarray, h: int, w: int, xfer: int) -> np.ndarray:
    """P(Y) applied columnwise from the coarse grid of an h x w image."""
    _, Ph = transfer_1d(h, xfer)
    _, Pw = transfer_1d(w, xfer)
    hc, wc = Ph.shape[1], Pw.shape[1]
    ncol = Y.shape[1]
    imgs = np.asarray(Y, dtype=np.float64).T.reshape(ncol, hc, wc)
    out = np.einsum("ya,nab,xb->nyx", Ph, imgs, Pw, optimize=True)
    return out.reshape(ncol, -1).T.copy()


def level_ns(n: int, levels: int) -> List[int]:
    """Column counts per level of a two-sided hierarchy, finest first:
    n_{l+1} = ceil(n_l / 2) (reading R1 applied to the column index)."""
    ns = [n]
    for _ in range(levels - 1):
        if ns[-1] < 2:
            raise ValueError("cannot restrict fewer than 2 columns")
        ns.append((ns[-1] + 1) // 2)
    return ns


def restrict_cols(X: np.ndarray, xfer: int) -> np.ndarray:
    """X R_n^T: the 1-D operator of eq. restr applied along the column index
    (Section 6.1's generalisation to n, for columns ordered along a smooth
    axis: wavelength, time).  X is k x n; the result k x ceil(n/2)."""
    R, _ = transfer_1d(X.shape[1], xfer)
    return np.asarray(X, dtype=np.float64) @ R.T


def prolong_cols(Y: np.ndarray, n: int, xfer: int) -> np.ndarray:
    """Y P_n^T: the 1-D prolongation of eq. prol along the column index, back
    to n columns."""
    _, P = transfer_1d(n, xfer)
    return np.asarray(Y, dtype=np.float64) @ P.T


def smoothness(M: np.ndarray, h: int, w: int, xfer: int) -> float:
    """s_M = ||M - P(R(M))||_F / ||M||_F (Section 4.1)."""
    M = np.asarray(M, dtype=np.float64)
    back = prolong_images(restrict_images(M, h, w, xfer), h, w, xfer)
    return float(np.linalg.norm(M - back) / np.linalg.norm(M))


# ---------------------------------------------------------------------------
# Multigrid cycles (Alg. 4 NI, Alg. 5 VC, Alg. 6 FMG; Table 1 budget)
# ---------------------------------------------------------------------------

def schedule(cycle: int, levels: int, T, ratio: int = 4) -> List[Tuple[str, int, int]]:
    """Flat list of steps ("restrict", d, 0), ("prolong", d, 0) or
    ("run", d, count) for a budget of T fine-iteration equivalents.

    restrict d   : V at depth d -> depth d+1
    prolong d    : V at depth d+1 -> depth d
    run d count  : ``count`` iterations of the NMF algorithm at depth d

    Depth 0 is the finest level.  Budgets are exact rationals; Run(d, t)
    performs floor(t * ratio^d) iterations (reading R5): ratio = 4 is the
    paper's m' ~ m/4 cost model; a two-sided hierarchy also halves n, so a
    coarse iteration costs about 1/8 (ratio = 8).  Zero-iteration runs are
    dropped.
    """
    steps: List[Tuple[str, int, int]] = []
    T = Fraction(T)

    def run(d: int, t: Fraction) -> None:
        count = math.floor(t * ratio ** d)
        if count > 0:
            steps.append(("run", d, int(count)))

    def ni(L: int, t: Fraction, d: int) -> None:          # Alg. 4
        if L == 1:
            run(d, t)
            return
        steps.append(("restrict", d, 0))
        ni(L - 1, t / 4, d + 1)
        steps.append(("prolong", d, 0))
        run(d, 3 * t / 4)

    def vc(L: int, t: Fraction, d: int) -> None:          # Alg. 5
        if L == 1:
            run(d, t)
            return
        run(d, t / 4)
        steps.append(("restrict", d, 0))
        vc(L - 1, t / 4, d + 1)
        steps.append(("prolong", d, 0))
        run(d, t / 2)

    def fmg(L: int, t: Fraction, d: int) -> None:         # Alg. 6
        if L == 1:
            run(d, t)
            return
        steps.append(("restrict", d, 0))
        fmg(L - 1, t / 4, d + 1)
        steps.append(("prolong", d, 0))
        vc(L, 3 * t / 4, d)

    def wc(L: int, t: Fraction, d: int) -> None:
        # W-cycle (Section 7.1 lists other cycles as future work; reading R13):
        # the V-cycle's split of t (1/4 before, 1/2 after, 1/4 to the coarser
        # levels) with the coarse share spent in two consecutive W-cycles of
        # t/8 each at the next level
        if L == 1:
            run(d, t)
            return
        run(d, t / 4)
        steps.append(("restrict", d, 0))
        wc(L - 1, t / 8, d + 1)
        wc(L - 1, t / 8, d + 1)
        steps.append(("prolong", d, 0))
        run(d, t / 2)

    {NI: ni, VC: vc, FMG: fmg, WC: wc}[cycle](levels, T, 0)
    return steps


def level_iteration_totals(steps: Sequence[Tuple[str, int, int]], levels: int) -> List[int]:
    tot = [0] * levels
    for kind, d, c in steps:
        if kind == "run":
            tot[d] += c
    return tot


# ---------------------------------------------------------------------------
# Inner NMF algorithms (Section 2: Alg. 1 ANLS, Alg. 2 MU, Alg. 3 HALS)
# ---------------------------------------------------------------------------

def hals_update_V(M: np.ndarray, V: np.ndarray, W: np.ndarray, hook=None) -> np.ndarray:
    """First half of Alg. 3: A = M W^T, B = W W^T, then for k = 1..r in order
    V[:,k] <- max(0, (A[:,k] - sum_{l != k} V[:,l] B[l,k]) / B[k,k]),
    using already-updated columns (Gauss-Seidel).  B[k,k] = 0: unchanged (R6)."""
    V = np.array(V, dtype=np.float64, copy=True)
    A = M @ W.T
    B = W @ W.T
    r = V.shape[1]
    for k in range(r):
        if B[k, k] > 0:
            others = [l for l in range(r) if l != k]
            s = V[:, others] @ B[others, k]
            V[:, k] = np.maximum(0.0, (A[:, k] - s) / B[k, k])
        if hook is not None:
            hook("V", k, V)
    return V


def hals_update_W(M: np.ndarray, V: np.ndarray, W: np.ndarray, hook=None) -> np.ndarray:
    """Second half of Alg. 3: C = V^T M, D = V^T V, then for k = 1..r
    W[k,:] <- max(0, (C[k,:] - sum_{l != k} D[k,l] W[l,:]) / D[k,k])."""
    W = np.array(W, dtype=np.float64, copy=True)
    C = V.T @ M
    D = V.T @ V
    r = W.shape[0]
    for k in range(r):
        if D[k, k] > 0:
            others = [l for l in range(r) if l != k]
            s = D[k, others] @ W[others, :]
            W[k, :] = np.maximum(0.0, (C[k, :] - s) / D[k, k])
        if hook is not None:
            hook("W", k, W)
    return W


def hals_iteration(M, V, W):
    V = hals_update_V(M, V, W)
    W = hals_update_W(M, V, W)
    return V, W


def mu_update_V(M: np.ndarray, V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Alg. 2, first line: V <- V o [M W^T] / [V (W W^T)] (Hadamard ops).
    Zero denominator: entry unchanged (R7)."""
    num = M @ W.T
    den = V @ (W @ W.T)
    out = np.array(V, dtype=np.float64, copy=True)
    ok = den > 0
    out[ok] = V[ok] * num[ok] / den[ok]
    return out


def mu_update_W(M: np.ndarray, V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Alg. 2, second line: W <- W o [V^T M] / [(V^T V) W]."""
    num = V.T @ M
    den = (V.T @ V) @ W
    out = np.array(W, dtype=np.float64, copy=True)
    ok = den > 0
    out[ok] = W[ok] * num[ok] / den[ok]
    return out


def mu_iteration(M, V, W):
    V = mu_update_V(M, V, W)
    W = mu_update_W(M, V, W)
    return V, W


def nnls_gram(G: np.ndarray, b: np.ndarray, x_keep: Optional[np.ndarray] = None,
              tol_scale: float = 1e-12) -> np.ndarray:
    """min_{x >= 0} 0.5 x^T G x - b^T x by the Lawson-Hanson active-set method
    (Appendix A.2, steps 0-3).

    Start with every variable active (at zero).  Repeatedly move into the
    passive set the active variable with the largest positive negative-gradient
    b - G x (lowest index on ties), solve the unconstrained problem on the
    passive set from the normal equations, and whenever a passive variable of
    that solution is nonpositive, step from x towards it only as far as
    feasibility allows and return the variables that reached zero to the active
    set.  Stop when no active variable has a positive negative-gradient above
    tol = tol_scale * max(1, max|b|).

    Variables with G[k,k] == 0 take no part and keep ``x_keep[k]`` (R8): for a
    Gram matrix G = X^T X this means column k of X is zero, so row/column k of
    G and b[k] vanish and the variable does not affect the objective.
    """
    r = b.shape[0]
    live = np.array([G[k, k] > 0 for k in range(r)], dtype=bool)
    x = np.zeros(r)
    if x_keep is not None:
        x[~live] = np.asarray(x_keep, dtype=np.float64)[~live]
    tol = tol_scale * max(1.0, float(np.max(np.abs(b))) if r else 1.0)
    passive = np.zeros(r, dtype=bool)
    blocked = np.zeros(r, dtype=bool)   # entered and was immediately rejected
    for _outer in range(10 * r + 10):
        grad_neg = b - G @ x
        cand = live & ~passive & ~blocked & (grad_neg > tol)
        if not cand.any():
            break
        j = int(np.argmax(np.where(cand, grad_neg, -np.inf)))
        passive[j] = True
        first = True
        while True:
            idx = np.flatnonzero(passive)
            z = np.zeros(r)
            z[~live] = x[~live]
            z[idx] = np.linalg.solve(G[np.ix_(idx, idx)], b[idx])
            if np.all(z[idx] > 0):
                x = z
                blocked[:] = False
                break
            if first and z[j] <= 0:
                # rounding made the entering variable infeasible: reject it
                passive[j] = False
                blocked[j] = True
                break
            first = False
            bad = idx[z[idx] <= 0]
            ratios = x[bad] / (x[bad] - z[bad])
            alpha = float(np.min(ratios))
            x = x + alpha * (z - x)
            leave = passive & (x <= 0)
            leave[bad[int(np.argmin(ratios))]] = True
            x[leave] = 0.0
            passive &= ~leave
            blocked[:] = False
            if not passive.any():
                break
    return x


def nnls_bpp(G: np.ndarray, b: np.ndarray, x_start: Optional[np.ndarray] = None,
             tol_scale: float = 1e-12, max_rounds: Optional[int] = None) -> np.ndarray:
    """min_{x >= 0} 0.5 x^T G x - b^T x by block principal pivoting, the
    exchange method that Section 2.1's footnote points to for the ANLS
    subproblems (Judice and Pires; Kim and Park for NMF).

    Keep a passive set F (free variables) and its complement (variables at
    zero).  Each round solves G[F,F] z = b[F], sets z = 0 outside F, and
    marks as infeasible every passive variable with z < 0 and every other one
    whose gradient (G z - b) is below -tol.  While the number of infeasible
    variables keeps falling, all of them change sides; once it stops falling,
    three more rounds exchange all of them, and after that only the infeasible
    variable with the highest index changes sides until the count falls again.
    No infeasible variable: z is the minimiser.  F starts as the support of
    x_start (all zero: empty).  Variables with G[k,k] == 0 keep x_start[k]
    and take no part (R8).  The minimiser is unique for a positive definite
    G, so the result equals nnls_gram's up to rounding.
    """
    r = b.shape[0]
    live = np.array([G[k, k] > 0 for k in range(r)], dtype=bool)
    x0 = np.zeros(r) if x_start is None else np.asarray(x_start, dtype=np.float64)
    tol = tol_scale * max(1.0, float(np.max(np.abs(b[live]))) if live.any() else 1.0)
    passive = live & (x0 > 0)
    ninf, backup = r + 1, 3
    for _ in range(max_rounds if max_rounds is not None else 8 * r + 16):
        z = np.zeros(r)
        idx = np.flatnonzero(passive)
        if idx.size:
            z[idx] = np.linalg.solve(G[np.ix_(idx, idx)], b[idx])
        grad = G[:, idx] @ z[idx] - b
        bad = live & np.where(passive, z < 0, grad < -tol)
        if not bad.any():
            out = np.where(live, z, x0)
            return out
        nv = int(bad.sum())
        if nv < ninf:
            ninf, backup = nv, 3
            passive ^= bad
        elif backup > 0:
            backup -= 1
            passive ^= bad
        else:
            j = int(np.flatnonzero(bad)[-1])
            passive[j] = ~passive[j]
    raise RuntimeError("block principal pivoting did not terminate")


def anls_update_V(M: np.ndarray, V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Alg. 1, first line: V <- argmin_{V >= 0} ||M - V W||_F^2, i.e. m
    independent NNLS problems V[i,:] (W W^T) = M[i,:] W^T (Appendix A.2)."""
    B = W @ W.T
    A = M @ W.T
    out = np.empty_like(np.asarray(V, dtype=np.float64))
    for i in range(M.shape[0]):
        out[i, :] = nnls_gram(B, A[i, :], x_keep=np.asarray(V[i, :], dtype=np.float64))
    return out


def anls_update_W(M: np.ndarray, V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Alg. 1, second line: W <- argmin_{W >= 0} ||M - V W||_F^2, column-wise
    on the Gram form (V^T V, V^T M[:,j]) (eq. subNNLS)."""
    D = V.T @ V
    C = V.T @ M
    out = np.empty_like(np.asarray(W, dtype=np.float64))
    for j in range(M.shape[1]):
        out[:, j] = nnls_gram(D, C[:, j], x_keep=np.asarray(W[:, j], dtype=np.float64))
    return out


def anls_iteration(M, V, W):
    V = anls_update_V(M, V, W)
    W = anls_update_W(M, V, W)
    return V, W


# ---------------------------------------------------------------------------
# Kullback-Leibler objective (Section 7.1's other objective functions; R17)
# ---------------------------------------------------------------------------

def kl_ratio(M: np.ndarray, P: np.ndarray) -> np.ndarray:
    """M / P entrywise, 0 where P = 0 (R17)."""
    Q = np.zeros_like(P)
    ok = P > 0
    Q[ok] = M[ok] / P[ok]
    return Q


def kl_divergence(M, V, W) -> float:
    """D(M | V W) = sum_ij M_ij log(M_ij / (VW)_ij) - M_ij + (VW)_ij, with
    0 log 0 = 0 (R17); +inf where M_ij > 0 = (VW)_ij."""
    M = np.asarray(M, dtype=np.float64)
    P = V @ W
    t = P - M
    pos = M > 0
    with np.errstate(divide="ignore"):
        t[pos] += M[pos] * np.log(M[pos] / P[pos])
    return float(np.sum(t))


def rel_kl(M, V, W) -> float:
    """The logged error of the KL objective: D(M | V W) / sum(M) (R17)."""
    return kl_divergence(M, V, W) / float(np.sum(np.asarray(M, dtype=np.float64)))


def kl_update_V(M: np.ndarray, V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """V <- V o [(M / VW) W^T] / [1 W^T]: the denominator of column k is
    sum_j W_kj; zero denominators keep the entry (R17)."""
    Q = kl_ratio(M, V @ W)
    num = Q @ W.T
    den = W.sum(axis=1)
    out = np.array(V, dtype=np.float64, copy=True)
    ok = den > 0
    out[:, ok] = V[:, ok] * num[:, ok] / den[ok]
    return out


def kl_update_W(M: np.ndarray, V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """W <- W o [V^T (M / VW)] / [V^T 1]: the denominator of row k is
    sum_i V_ik; zero denominators keep the entry (R17)."""
    Q = kl_ratio(M, V @ W)
    num = V.T @ Q
    den = V.sum(axis=0)
    out = np.array(W, dtype=np.float64, copy=True)
    ok = den > 0
    out[ok, :] = W[ok, :] * num[ok, :] / den[ok, None]
    return out


def kl_iteration(M, V, W):
    V = kl_update_V(M, V, W)
    W = kl_update_W(M, V, W)
    return V, W


def iteration(algo: int, M, V, W):
    return {HALS: hals_iteration, MU: mu_iteration, ANLS: anls_iteration,
            KL: kl_iteration}[algo](M, V, W)


# ---------------------------------------------------------------------------
# Nonnegative tensor factorisation (Section 7.1; reading R18)
# ---------------------------------------------------------------------------

def khatri_rao(C: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Column-wise Kronecker product C kr B: row j + J k, column r holds
    C[k, r] B[j, r] (the row order of the mode-1 unfolding's columns)."""
    K, R = C.shape
    J = B.shape[0]
    return (C[:, None, :] * B[None, :, :]).reshape(K * J, R)


def unfold(X: np.ndarray, mode: int) -> np.ndarray:
    """Mode-n unfolding of a 3-way tensor: X_(1)[i, j + J k], X_(2)[j, i + I k],
    X_(3)[k, i + I j] (the first remaining index fastest)."""
    I, J, K = X.shape
    if mode == 1:
        return X.transpose(0, 2, 1).reshape(I, K * J)
    if mode == 2:
        return X.transpose(1, 2, 0).reshape(J, K * I)
    return X.transpose(2, 1, 0).reshape(K, J * I)


def fold1(X1: np.ndarray, J: int, K: int) -> np.ndarray:
    """Inverse of unfold(., 1): the tensor from its mode-1 unfolding."""
    I = X1.shape[0]
    return X1.reshape(I, K, J).transpose(0, 2, 1)


def cp_tensor(A: np.ndarray, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """[[A, B, C]] = sum_r a_r o b_r o c_r."""
    return np.einsum("ir,jr,kr->ijk", A, B, C)


def ntf_iteration(X: np.ndarray, A, B, C):
    """One HALS-NTF iteration (R18): each factor in turn takes the HALS steps
    of Alg. 3 on its unfolding, with the Khatri-Rao product of the other two
    (already updated ones included) as the fixed factor."""
    A = hals_update_V(unfold(X, 1), A, khatri_rao(C, B).T)
    B = hals_update_V(unfold(X, 2), B, khatri_rao(C, A).T)
    C = hals_update_V(unfold(X, 3), C, khatri_rao(B, A).T)
    return A, B, C


def ntf_rel_err(X: np.ndarray, A, B, C) -> float:
    """||X - [[A, B, C]]||_F / ||X||_F, evaluated directly."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.linalg.norm(X - cp_tensor(A, B, C)) / np.linalg.norm(X))


class NtfResult:
    def __init__(self):
        self.A = self.B = self.C = None
        self.log: List[Tuple[int, float]] = []
        self.stopped = False
        self.fine_iters = 0
        self.total_iters = 0
        self.fine_equiv = 0.0


def solve_ntf(X, h: int, w: int, r: int, levels: int, cycle: int, xfer: int, T, A0, B0, C0,
              tol: float = 0.0, max_fine_iters: int = 0, callback=None) -> NtfResult:
    """Multilevel HALS-NTF (R18): the hierarchy, schedule and stopping of
    solve() with the tensor's mode 1 (the h x w grid) coarsened; A moves
    between levels as V does, B and C are shared by all levels."""
    X = np.asarray(X, dtype=np.float64)
    I, J, K = X.shape
    assert I == h * w
    sides = level_sides(h, w, levels)
    Xs = [X]
    for d in range(levels - 1):
        hd, wd = sides[d]
        Xs.append(fold1(restrict_images(unfold(Xs[-1], 1), hd, wd, xfer), J, K))
    A = np.asarray(A0, dtype=np.float64).copy()
    B = np.asarray(B0, dtype=np.float64).copy()
    C = np.asarray(C0, dtype=np.float64).copy()
    res = NtfResult()
    depth = 0

    def one(d):
        nonlocal A, B, C
        A, B, C = ntf_iteration(Xs[d], A, B, C)
        e = ntf_rel_err(Xs[d], A, B, C)
        res.log.append((d, e))
        res.total_iters += 1
        res.fine_equiv += 4.0 ** (-d)
        if d == 0:
            res.fine_iters += 1
        if callback is not None:
            callback(d, A, B, C, e)
        return e

    for kind, d, count in schedule(cycle, levels, T):
        if kind == "restrict":
            assert depth == d
            A = restrict_images(A, *sides[d], xfer)
            depth = d + 1
        elif kind == "prolong":
            assert depth == d + 1
            A = prolong_images(A, *sides[d], xfer)
            depth = d
        else:
            assert depth == d
            for _ in range(count):
                if one(d) <= tol and tol > 0 and d == 0:
                    res.stopped = True
                    break
        if res.stopped:
            break
    assert res.stopped or depth == 0
    if tol > 0 and not res.stopped:
        for _ in range(max_fine_iters):
            if one(0) <= tol:
                res.stopped = True
                break
    res.A, res.B, res.C = A, B, C
    return res


# ---------------------------------------------------------------------------
# Reduced-precision products (the library's BF16 mode; the paper fixes no
# precision, so this is the definition that mode follows, not a paper passage)
# ---------------------------------------------------------------------------

def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 value (8 significant bits, ties to even),
    for normal-range inputs: with x = f 2^e, 0.5 <= |f| < 1, keep round(f 2^8)."""
    x = np.asarray(x, dtype=np.float64)
    f, e = np.frexp(x)
    return np.ldexp(np.round(f * 256.0) / 256.0, e)


def hals_update_V_bf16(M, V, W, Mb=None):
    """Alg. 3's V half with the product A = M W^T formed from bfloat16-rounded
    M and W (exact products, FP64 sums); B = W W^T and the update unchanged.
    Mb: bf16_round(M) when the caller has it already."""
    V = np.array(V, dtype=np.float64, copy=True)
    A = (bf16_round(M) if Mb is None else Mb) @ bf16_round(W).T
    B = W @ W.T
    r = V.shape[1]
    for k in range(r):
        if B[k, k] > 0:
            others = [l for l in range(r) if l != k]
            V[:, k] = np.maximum(0.0, (A[:, k] - V[:, others] @ B[others, k]) / B[k, k])
    return V


def hals_update_W_bf16(M, V, W, Mb=None):
    """Alg. 3's W half with C = V^T M and D = V^T V formed from bfloat16-rounded
    V and M (exact products, FP64 sums)."""
    W = np.array(W, dtype=np.float64, copy=True)
    Vb = bf16_round(V)
    C = Vb.T @ (bf16_round(M) if Mb is None else Mb)
    D = Vb.T @ Vb
    r = W.shape[0]
    for k in range(r):
        if D[k, k] > 0:
            others = [l for l in range(r) if l != k]
            W[k, :] = np.maximum(0.0, (C[k, :] - D[k, others] @ W[others, :]) / D[k, k])
    return W


def mu_iteration_bf16(M, V, W, Mb=None):
    """Alg. 2 with the two M products formed from bfloat16-rounded operands:
    V <- V o [bf(M) bf(W)^T] / [V (W W^T)], then
    W <- W o [bf(V)^T bf(M)] / [(bf(V)^T bf(V)) W]; zero denominators keep the entry."""
    if Mb is None:
        Mb = bf16_round(M)
    num = Mb @ bf16_round(W).T
    den = V @ (W @ W.T)
    Vn = np.array(V, dtype=np.float64, copy=True)
    ok = den > 0
    Vn[ok] = V[ok] * num[ok] / den[ok]
    Vb = bf16_round(Vn)
    num = Vb.T @ Mb
    den = (Vb.T @ Vb) @ W
    Wn = np.array(W, dtype=np.float64, copy=True)
    ok = den > 0
    Wn[ok] = W[ok] * num[ok] / den[ok]
    return Vn, Wn


def iteration_bf16(algo: int, M, V, W, Mb=None):
    """One iteration of HALS or MU with bfloat16 operands in the two M products
    (Mb: bf16_round(M), if already formed)."""
    if Mb is None:
        Mb = bf16_round(M)
    if algo == HALS:
        V = hals_update_V_bf16(M, V, W, Mb)
        return V, hals_update_W_bf16(M, V, W, Mb)
    if algo == MU:
        return mu_iteration_bf16(M, V, W, Mb)
    raise ValueError("bfloat16 products: HALS and MU only")


# ---------------------------------------------------------------------------
# Objective and diagnostics (eq. NMF, eq. subNNLS, Section 4.1 bound)
# ---------------------------------------------------------------------------

def objective(M, V, W) -> float:
    """||M - V W||_F^2 (eq. NMF)."""
    return float(np.sum((np.asarray(M, dtype=np.float64) - V @ W) ** 2))


def rel_err(M, V, W) -> float:
    """||M - V W||_F / ||M||_F, evaluated directly (reading R9)."""
    M = np.asarray(M, dtype=np.float64)
    return float(np.linalg.norm(M - V @ W) / np.linalg.norm(M))


def gram_form_residual2(normM2, C, W, D, B):
    """||M - V W||_F^2 written through Gram products (eq. subNNLS summed over
    columns): ||M||^2 - 2 <V^T M, W> + <V^T V, W W^T>.  Works for numpy floats,
    and for object arrays of Fractions (exact pins)."""
    return normM2 - 2 * np.sum(C * W) + np.sum(D * B)


def eckart_young_floor(M, r: int) -> float:
    """Lower bound on rel_err for any rank-r product: sqrt(sum_{i>r} s_i^2)/||M||."""
    s = np.linalg.svd(np.asarray(M, dtype=np.float64), compute_uv=False)
    return float(np.sqrt(np.sum(s[r:] ** 2)) / np.sqrt(np.sum(s ** 2)))


def prolongation_bound(M, h, w, xfer, Vc, W) -> Tuple[float, float]:
    """Section 4.1, step 4: ||M - P(V') W|| <= s_M ||M|| + ||P||_F ||R(M) - V' W||.
    Returns (lhs, rhs)."""
    M = np.asarray(M, dtype=np.float64)
    Pm = prolong_matrix(h, w, xfer)
    lhs = float(np.linalg.norm(M - prolong_images(Vc, h, w, xfer) @ W))
    sM = smoothness(M, h, w, xfer)
    Rm = restrict_images(M, h, w, xfer)
    rhs = sM * float(np.linalg.norm(M)) + float(np.linalg.norm(Pm)) * float(np.linalg.norm(Rm - Vc @ W))
    return lhs, rhs


def prolongation_bound_two_sided(M, h, w, xfer, Vc, Wc) -> Tuple[float, float]:
    """Section 4.1's step-4 bound with both sides coarsened: writing
    M' = R_m M R_n^T, M - P_m V' W' P_n^T = (M - P_m M' P_n^T)
    + P_m (M' - V' W') P_n^T, so
    ||M - P_m V' W' P_n^T|| <= ||M - P_m M' P_n^T|| + ||P_m||_F ||M' - V'W'|| ||P_n||_F.
    Returns (lhs, rhs)."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[1]
    _, Pn = transfer_1d(n, xfer)
    Pm = prolong_matrix(h, w, xfer)
    Mc = restrict_cols(restrict_images(M, h, w, xfer), xfer)
    back = prolong_cols(prolong_images(Mc, h, w, xfer), n, xfer)
    lhs = float(np.linalg.norm(M - prolong_cols(prolong_images(Vc, h, w, xfer) @ Wc, n, xfer)))
    rhs = (float(np.linalg.norm(M - back))
           + float(np.linalg.norm(Pm)) * float(np.linalg.norm(Mc - Vc @ Wc)) * float(np.linalg.norm(Pn)))
    return lhs, rhs


# ---------------------------------------------------------------------------
# Whole multilevel solve
# ---------------------------------------------------------------------------

class SolveResult:
    def __init__(self):
        self.V: Optional[np.ndarray] = None
        self.W: Optional[np.ndarray] = None
        self.log: List[Tuple[int, float]] = []   # (depth, rel_err) per iteration
        self.stopped = False
        self.fine_iters = 0
        self.total_iters = 0
        self.fine_equiv = 0.0
        self.bound_checks: List[Tuple[float, float]] = []

    @property
    def rel_errs(self) -> np.ndarray:
        return np.array([e for _, e in self.log])


def solve(M, h: int, w: int, r: int, levels: int, algo: int, cycle: int, xfer: int,
          T, V0, W0, tol: float = 0.0, max_fine_iters: int = 0,
          check_bound: bool = False, callback=None, bf16_products: bool = False,
          refine_iters: int = 0, two_sided: bool = False) -> SolveResult:
    """Multilevel NMF (Section 4.1 steps 1-5 applied recursively by Alg. 4/5/6).

    The restrictions of M are computed once per level and kept (Alg. 6 note).
    W is passed between levels unchanged (only m is coarsened).  For ANLS the
    V iterate is not an input of the algorithm (Alg. 1, Remark 1), so its
    transfers do not influence the result.

    bf16_products: the scheduled iterations use iteration_bf16 (the library's
    BF16 mode), then `refine_iters` full-precision finest-level iterations
    follow; the tolerance applies to those only, as in that mode.

    two_sided: the hierarchy also coarsens the column index (Section 6.1's
    generalisation for columns ordered along a smooth axis): M_{l+1} =
    R_m M_l R_n^T, W moves between levels as V does but along its rows
    (W' = W R_n^T, W = W' P_n^T), and the budget uses ratio 8 (schedule).
    """
    M = np.asarray(M, dtype=np.float64)
    sides = level_sides(h, w, levels)
    ns = level_ns(M.shape[1], levels) if two_sided else [M.shape[1]] * levels
    Ms = [M]
    for d in range(levels - 1):
        hd, wd = sides[d]
        Mc = restrict_images(Ms[-1], hd, wd, xfer)
        Ms.append(restrict_cols(Mc, xfer) if two_sided else Mc)
    V = np.asarray(V0, dtype=np.float64).copy()
    W = np.asarray(W0, dtype=np.float64).copy()
    res = SolveResult()
    depth = 0

    Mbs = [bf16_round(Ml) for Ml in Ms] if bf16_products else None

    def one(d, low=False):
        nonlocal V, W
        V, W = iteration_bf16(algo, Ms[d], V, W, Mbs[d]) if low else iteration(algo, Ms[d], V, W)
        e = rel_kl(Ms[d], V, W) if algo == KL else rel_err(Ms[d], V, W)
        res.log.append((d, e))
        res.total_iters += 1
        res.fine_equiv += (8.0 if two_sided else 4.0) ** (-d)
        if d == 0:
            res.fine_iters += 1
        if callback is not None:
            callback(d, V, W, e)
        return e

    for kind, d, count in schedule(cycle, levels, T, 8 if two_sided else 4):
        if kind == "restrict":
            assert depth == d
            hd, wd = sides[d]
            V = restrict_images(V, hd, wd, xfer)
            if two_sided:
                W = restrict_cols(W, xfer)
            depth = d + 1
        elif kind == "prolong":
            assert depth == d + 1
            hd, wd = sides[d]
            if check_bound:
                res.bound_checks.append(
                    prolongation_bound_two_sided(Ms[d], hd, wd, xfer, V, W) if two_sided
                    else prolongation_bound(Ms[d], hd, wd, xfer, V, W))
            V = prolong_images(V, hd, wd, xfer)
            if two_sided:
                W = prolong_cols(W, ns[d], xfer)
            depth = d
        else:
            assert depth == d
            for _ in range(count):
                e = one(d, bf16_products)
                if tol > 0 and d == 0 and e <= tol and not bf16_products:
                    res.stopped = True
                    break
        if res.stopped:
            break
    assert res.stopped or depth == 0
    for _ in range(refine_iters if bf16_products and not res.stopped else 0):
        if one(0) <= tol and tol > 0:
            res.stopped = True
            break
    if tol > 0 and not res.stopped:
        for _ in range(max_fine_iters):
            if one(0) <= tol:
                res.stopped = True
                break
    res.V, res.W = V, W
    return res
