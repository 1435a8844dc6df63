"""Lowest eigenpairs of the explicit operator by dense diagonalisation.

This is the plain definition of what the local eigenproblem of Sec. II.A
(Eq. localproblem) asks for: the J_K smallest eigenvalues of H and their
eigenvectors, with no iteration.  LAPACK's symmetric eigensolver through
scipy is the library primitive.  Feasible up to N_g ~ 1.4e4 (24^3 grid).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def lowest(H: np.ndarray, k: int):
    """(w, U): the k smallest eigenvalues (ascending) and unit eigenvectors."""
    w, U = sla.eigh(H, subset_by_index=[0, k - 1], driver="evr")
    return w, U
