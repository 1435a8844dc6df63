"""Element-local DG quantities from the ALBs (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Density (Sec. II.A, Eq. newdensity): ALBs of different elements do not
  overlap, so rho on element E_K needs only the diagonal density-matrix block:
  rho_K(x) = sum_{j,j'} phi_{K,j}(x) P_{K,j;K,j'} phi_{K,j'}(x).
* Nonlocal DG term (Sec. II.A, Eq. DGHamiltonian, the Kleinman-Bylander
  bracket with K = K'): H_K[j][j'] = sum_p gamma_p <phi_j, b_p> <b_p, phi_j'>
  with <f, g> = dV sum over the element box (reading: the element's uniform
  grid stands in for the paper's quadrature grid).
"""
from __future__ import annotations

import numpy as np

from .alb import box_rows


def density(albs, P):
    """albs: N_E x n_alb; P: n_alb x n_alb -> rho (N_E)."""
    return np.einsum("xj,jk,xk->x", albs, P, albs)


def nonlocal_block(albs, kb, grid, lo, hi, dv):
    """albs: N_E x n_alb on the element box; kb: the element's projectors
    (CSR over the extended grid) -> n_alb x n_alb."""
    rows = box_rows(grid, lo, hi)                 # flat grid index of each box row
    pos = -np.ones(int(np.prod(grid)), dtype=np.int64)
    pos[rows] = np.arange(rows.shape[0])
    n_proj = kb.gamma.shape[0]
    B = np.zeros((n_proj, albs.shape[1]))
    for p in range(n_proj):
        idx = kb.idx[kb.ptr[p]:kb.ptr[p + 1]].astype(np.int64)
        val = kb.val[kb.ptr[p]:kb.ptr[p + 1]]
        r = pos[idx]
        keep = r >= 0
        B[p] = dv * (val[keep] @ albs[r[keep]])
    return B.T @ (kb.gamma[:, None] * B)
