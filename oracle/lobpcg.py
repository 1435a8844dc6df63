"""LOBPCG for the lowest J eigenpairs of one element (FP64, dense NumPy).

The paper solves each local eigenproblem with LOBPCG (Knyazev 2001) and lists
its ingredients (Sec. II.B, "Generation of the ALB functions"): one
application of H per iteration, products Phi^T Psi of N_g x J blocks (twelve
per iteration), products Phi C with small C (seven per iteration), a
Rayleigh-Ritz diagonalisation of size O(J) done sequentially, and a
preconditioner applied column by column.  It gives no further detail, so the
variant below is a reading; its steps are, per iteration:

  a. residual R = HX - X diag(theta), r_i = ||R_i||_2; stop when max_i r_i <= tol
  b. W = K(R) (Teter, with the band kinetic energy of x_i)
  c. W <- W - [X P]([X P]^T W); W <- W T_W with T_W from a diagonally scaled
     Cholesky of W^T W (CholQR); eigenvalue-based SVQB when that Cholesky breaks
  d. HW = H W
  e. S = [X P W], HS = [HX HP HW];  Hh = sym(S^T HS), M = sym(S^T S)
     -- the twelve J x J Gram blocks of the paper are the upper block triangles
  f. Rayleigh-Ritz: lowest J of Hh c = theta M c (Cholesky of M; if M is not
     numerically SPD, reduce to the eigenvectors of M above 1e-10 max)
  g. X <- S C, HX <- HS C; the new search direction is the part of
     S [0; C_P; C_W] that is M-orthogonal to C, normalised through a Cholesky of
     its M-Gram (P is dropped for one iteration if that Cholesky breaks):
     P <- S D, HP <- HS D

Initial step: X <- X0 T (CholQR), HX = H X, Rayleigh-Ritz on X alone.
Final step (once converged or out of iterations): HX is recomputed from
scratch, Rayleigh-Ritz on X alone, FP64 residuals reported.

Guard columns (optional, not in the paper): with n_check < J the block
carries J - n_check extra columns that take part in every step but not in
the stopping test of a. (nor in `converged`): the wanted n_check states then
converge at the rate set by the gap to state J + 1.

The oracle computes in this order with no blocking or fusion beyond
NumPy/LAPACK calls on whole blocks.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

CHOL_TOL = 1e-10  # smallest admissible Cholesky pivot of a unit-diagonal Gram


class Breakdown(RuntimeError):
    """The initial block has (numerically) dependent columns."""


@dataclasses.dataclass
class Result:
    theta: np.ndarray
    X: np.ndarray
    resid: np.ndarray
    iters: int
    converged: bool
    history: list
    n_chol_fallback: int = 0
    n_rr_fallback: int = 0
    n_p_drop: int = 0


def scaled_cholqr(Y: np.ndarray):
    """T with Y T orthonormal: Y D^-1 = Q R, T = D^-1 R^-1.  None on breakdown."""
    d = np.linalg.norm(Y, axis=0)
    if not np.all(d > 0.0):
        return None
    G = (Y.T @ Y) / np.outer(d, d)
    G = 0.5 * (G + G.T)
    try:
        L = np.linalg.cholesky(G)
    except np.linalg.LinAlgError:
        return None
    if np.min(np.diag(L)) ** 2 <= CHOL_TOL:
        return None
    Rinv = sla.solve_triangular(L.T, np.eye(Y.shape[1]), lower=False)
    return Rinv / d[:, None]


def svqb(Y: np.ndarray):
    """Eigenvalue-based orthonormalisation (Stathopoulos-Wu SVQB), clamped."""
    d = np.linalg.norm(Y, axis=0)
    d = np.where(d > 0.0, d, 1.0)
    G = (Y.T @ Y) / np.outer(d, d)
    G = 0.5 * (G + G.T)
    lam, U = np.linalg.eigh(G)
    lam = np.maximum(lam, CHOL_TOL * max(lam.max(), 1e-300))
    return (U / np.sqrt(lam)[None, :]) / d[:, None]


def rayleigh_ritz(S, HS, J, stats):
    Hh = S.T @ HS
    Hh = 0.5 * (Hh + Hh.T)
    M = S.T @ S
    M = 0.5 * (M + M.T)
    try:
        dm = np.sqrt(np.diag(M))
        L = np.linalg.cholesky(M / np.outer(dm, dm))
        if np.min(np.diag(L)) ** 2 <= CHOL_TOL:
            raise np.linalg.LinAlgError
        theta, C = sla.eigh(Hh, M, subset_by_index=[0, J - 1])
    except np.linalg.LinAlgError:
        stats.n_rr_fallback += 1
        lam, V = np.linalg.eigh(M)
        keep = lam > CHOL_TOL * lam.max()
        if keep.sum() < J:
            raise Breakdown("Rayleigh-Ritz basis has fewer than J independent vectors")
        T = V[:, keep] / np.sqrt(lam[keep])[None, :]
        A = T.T @ Hh @ T
        A = 0.5 * (A + A.T)
        theta, Y = np.linalg.eigh(A)
        theta, C = theta[:J], T @ Y[:, :J]
    return theta, C, M


def next_direction(C, M, J):
    """D such that S D spans the M-orthogonal complement of S C inside
    S [0; C_P; C_W], with (S D)^T (S D) = I.  None if it breaks down."""
    E = C.copy()
    E[:J, :] = 0.0
    D = E - C @ (C.T @ (M @ E))
    G = D.T @ M @ D
    G = 0.5 * (G + G.T)
    dg = np.sqrt(np.maximum(np.diag(G), 0.0))
    if not np.all(dg > 0.0):
        return None
    try:
        L = np.linalg.cholesky(G / np.outer(dg, dg))
    except np.linalg.LinAlgError:
        return None
    if np.min(np.diag(L)) ** 2 <= CHOL_TOL:
        return None
    Rinv = sla.solve_triangular(L.T, np.eye(J), lower=False) / dg[:, None]
    return D @ Rinv


def lobpcg(apply_h, precond, X0, tol, max_iter, n_check=None) -> Result:
    X0 = np.asarray(X0, dtype=np.float64)
    N, J = X0.shape
    nc = J if n_check is None else int(n_check)
    if not 1 <= nc <= J:
        raise ValueError("n_check must be in 1..J")
    stats = Result(None, None, None, 0, False, [])
    T = scaled_cholqr(X0)
    if T is None:
        raise Breakdown("initial block is rank deficient")
    X = X0 @ T
    HX = apply_h(X)
    theta, C, _ = rayleigh_ritz(X, HX, J, stats)
    X, HX = X @ C, HX @ C
    P = HP = None
    it = 0
    while True:
        R = HX - X * theta[None, :]
        r = np.linalg.norm(R, axis=0)
        stats.history.append(float(r[:nc].max()))
        if r[:nc].max() <= tol or it >= max_iter:
            break
        W = precond(R, X)
        B = X if P is None else np.hstack([X, P])
        W = W - B @ (B.T @ W)
        T = scaled_cholqr(W)
        if T is None:
            stats.n_chol_fallback += 1
            T = svqb(W)
        W = W @ T
        HW = apply_h(W)
        if P is None:
            S, HS = np.hstack([X, W]), np.hstack([HX, HW])
        else:
            S, HS = np.hstack([X, P, W]), np.hstack([HX, HP, HW])
        theta, C, M = rayleigh_ritz(S, HS, J, stats)
        D = next_direction(C, M, J)
        X, HX = S @ C, HS @ C
        if D is None:
            stats.n_p_drop += 1
            P = HP = None
        else:
            P, HP = S @ D, HS @ D
        it += 1
    # final FP64 check: fresh H X, Rayleigh-Ritz on X, residuals
    HX = apply_h(X)
    theta, C, _ = rayleigh_ritz(X, HX, J, stats)
    X, HX = X @ C, HX @ C
    r = np.linalg.norm(HX - X * theta[None, :], axis=0)
    stats.theta, stats.X, stats.resid, stats.iters = theta, X, r, it
    stats.converged = bool(r[:nc].max() <= tol)
    return stats
