"""Restriction of the local eigenvectors to the element, then SVD truncation.

Sec. II.A (after Eq. localproblem) and Sec. II.B (end of "Generation of the
ALB functions"): the eigenvectors computed on Q_K are restricted to E_K,
orthonormalised (the restricted vectors are not orthonormal) and set to zero
outside E_K; the ALBs are orthonormal on E_K (Eq. orthonormal).  Here the
orthonormalisation keeps the n_alb leading left singular vectors of the
restricted block, which spans the same space when n_alb = J and otherwise
truncates by singular value.

Conventions: ALBs are returned in the psi normalisation dV sum phi^2 = 1, in
descending sigma, with the largest-magnitude entry of each made positive.
Rows are the box points in x-fastest order.
"""
from __future__ import annotations

import numpy as np


def box_rows(grid, lo, hi) -> np.ndarray:
    n1, n2, _ = grid
    i = np.arange(lo[0], hi[0])
    j = np.arange(lo[1], hi[1])
    k = np.arange(lo[2], hi[2])
    return (k[:, None, None] * (n1 * n2) + j[None, :, None] * n1 + i[None, None, :]).reshape(-1)


def canonical_sign(A: np.ndarray) -> np.ndarray:
    piv = np.argmax(np.abs(A), axis=0)
    s = np.sign(A[piv, np.arange(A.shape[1])])
    s[s == 0] = 1.0
    return A * s[None, :]


def restrict_svd(X: np.ndarray, grid, lo, hi, dv: float, n_alb: int):
    """X: unit eigenvectors on Q (N_g x J).  Returns (albs, sigma)."""
    rows = box_rows(grid, lo, hi)
    U, s, _ = np.linalg.svd(X[rows, :], full_matrices=False)
    A = canonical_sign(U[:, :n_alb])
    return A / np.sqrt(dv), s[:n_alb]
