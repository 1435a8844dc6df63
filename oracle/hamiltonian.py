"""The discrete local Kohn-Sham operator of one extended element (FP64).

Sec. II.A, Eq. localproblem: H = -1/2 Laplacian + V_eff^Q + V_nl^Q on Q_K,
with eigenfunctions normalised by the integral over Q_K.  Sec. II.B (grid
rule Eq. Ngecut and "Generation of the ALB functions"): the eigenproblem is
discretised with planewaves, the orbitals are N_g real-space values, and the
Laplacian is applied by FFT.  Gamma point only (Sec. II.A), so everything is
real.  The nonlocal term is the Kleinman-Bylander form of Eq. DGvar:
V_nl = sum_p gamma_p |b_p><b_p|.

Basis: the oracle works with unit vectors u = sqrt(dV) * psi, in which the
operator is the real symmetric N_g x N_g matrix

    H = F^-1 diag(|G|^2/2) F + diag(V) + sum_p gamma_p beta_p beta_p^T,
    beta_p = sqrt(dV) * b_p   (so beta_p^T u = dV sum b_p psi = <b_p, psi>).

Planewave set (reading of the paper): every frequency of the FFT box, no
spherical cutoff; G_d = 2 pi m_d / L_d with m_d = k for k <= n_d/2 and k - n_d
otherwise, so the Nyquist bin of an even axis carries (pi n_d / L_d)^2 / 2.

Layout: a column is a flat array of N_g values, x fastest
(flat = i + n1*(j + n2*k)), i.e. a C-order array of shape (n3, n2, n1).
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

# threads of the FFT library (the BLAS pool is set by OMP_NUM_THREADS)
FFT_WORKERS = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
import scipy.sparse as sp


def frequencies(n: int) -> np.ndarray:
    """Integer frequencies m of an n-point periodic axis (Nyquist as +n/2)."""
    k = np.arange(n)
    return np.where(k <= n // 2, k, k - n)


def kinetic_diagonal(grid, box) -> np.ndarray:
    """|G|^2/2 on the FFT box, shape (n3, n2, n1)."""
    n1, n2, n3 = grid
    g1 = 2.0 * np.pi * frequencies(n1) / box[0]
    g2 = 2.0 * np.pi * frequencies(n2) / box[1]
    g3 = 2.0 * np.pi * frequencies(n3) / box[2]
    return 0.5 * (g3[:, None, None] ** 2 + g2[None, :, None] ** 2 + g1[None, None, :] ** 2)


def projector_matrix(kb, ng: int, dv: float) -> sp.csc_matrix:
    """B = [beta_1 .. beta_P] as an N_g x P sparse matrix, beta_p = sqrt(dV) b_p."""
    n_proj = kb.gamma.shape[0]
    return sp.csc_matrix((np.sqrt(dv) * kb.val, kb.idx.astype(np.int64), kb.ptr),
                         shape=(ng, n_proj))


class Operator:
    """H of one element acting on unit-basis columns."""

    def __init__(self, grid, box, V, kb):
        self.grid = tuple(int(n) for n in grid)
        self.box = tuple(float(b) for b in box)
        self.ng = int(np.prod(self.grid))
        self.dv = float(np.prod(self.box)) / self.ng
        self.V = np.asarray(V, dtype=np.float64).reshape(self.ng)
        self.t = kinetic_diagonal(self.grid, self.box)
        self.B = projector_matrix(kb, self.ng, self.dv)
        self.gamma = np.asarray(kb.gamma, dtype=np.float64)

    def kinetic(self, U: np.ndarray) -> np.ndarray:
        """F^-1 diag(|G|^2/2) F applied column by column."""
        n1, n2, n3 = self.grid
        m = U.shape[1]
        A = U.T.reshape(m, n3, n2, n1)
        out = sfft.ifftn(self.t[None] * sfft.fftn(A, axes=(1, 2, 3), workers=FFT_WORKERS), axes=(1, 2, 3), workers=FFT_WORKERS)
        return np.asfortranarray(out.real.reshape(m, self.ng).T)

    def nonlocal_(self, U: np.ndarray) -> np.ndarray:
        """sum_p gamma_p beta_p (beta_p^T U)."""
        if self.gamma.size == 0:
            return np.zeros_like(U)
        proj = self.B.T @ U
        return self.B @ (self.gamma[:, None] * proj)

    def apply(self, U: np.ndarray) -> np.ndarray:
        U = np.asarray(U, dtype=np.float64)
        single = U.ndim == 1
        if single:
            U = U[:, None]
        HU = self.kinetic(U) + self.V[:, None] * U + self.nonlocal_(U)
        return HU[:, 0] if single else HU

    def dense(self) -> np.ndarray:
        """The explicit N_g x N_g matrix (small grids only)."""
        n1, n2, n3 = self.grid
        ng = self.ng
        # kinetic block via the FFT of identity columns, in chunks
        H = np.empty((ng, ng))
        step = 512
        for c0 in range(0, ng, step):
            c1 = min(ng, c0 + step)
            E = np.zeros((ng, c1 - c0))
            E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
            H[:, c0:c1] = self.kinetic(E)
        H[np.diag_indices(ng)] += self.V
        if self.gamma.size:
            Bd = self.B.toarray()
            H += (Bd * self.gamma[None, :]) @ Bd.T
        return H
