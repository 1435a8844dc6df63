"""Teter preconditioner (FP64), as cited for LOBPCG in Sec. II.B.

The paper accelerates LOBPCG with the preconditioner of Payne, Teter, Allan
et al. (Rev. Mod. Phys. 64, 1045 (1992)), applied column by column with no
communication.  That preconditioner is diagonal in G:

    K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4),
    x    = (|G|^2/2) / T_i,

with T_i the kinetic energy of band i.  Reading taken here: T_i is the
kinetic energy of the current unit Ritz vector x_i,
T_i = sum_G |G|^2/2 |x^_i(G)|^2 / N_g (Parseval for the unnormalised DFT),
floored at the smallest nonzero planewave energy (2 pi / L_max)^2 / 2 so that a
constant vector (T = 0) is safe.  The correction for column i is
w_i = F^-1 K F r_i.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .hamiltonian import FFT_WORKERS, kinetic_diagonal


def teter_k(x):
    x = np.asarray(x, dtype=np.float64)
    num = 27.0 + x * (18.0 + x * (12.0 + x * 8.0))
    return num / (num + 16.0 * x ** 4)


def band_kinetic(X: np.ndarray, grid, box) -> np.ndarray:
    """T_i = x_i^T (-1/2 Laplacian) x_i, evaluated in G space."""
    n1, n2, n3 = grid
    m = X.shape[1]
    t = kinetic_diagonal(grid, box)
    Xh = sfft.fftn(X.T.reshape(m, n3, n2, n1), axes=(1, 2, 3), workers=FFT_WORKERS)
    ng = n1 * n2 * n3
    return np.einsum("abcd,bcd->a", np.abs(Xh) ** 2, t) / ng


def kinetic_floor(box) -> float:
    return 0.5 * (2.0 * np.pi / max(box)) ** 2


def precondition(R: np.ndarray, X: np.ndarray, grid, box) -> np.ndarray:
    n1, n2, n3 = grid
    m = R.shape[1]
    t = kinetic_diagonal(grid, box)
    T = np.maximum(band_kinetic(X, grid, box), kinetic_floor(box))
    K = teter_k(t[None] / T[:, None, None, None])
    Rh = sfft.fftn(R.T.reshape(m, n3, n2, n1), axes=(1, 2, 3), workers=FFT_WORKERS)
    W = sfft.ifftn(K * Rh, axes=(1, 2, 3), workers=FFT_WORKERS).real
    return np.asfortranarray(W.reshape(m, n1 * n2 * n3).T)
