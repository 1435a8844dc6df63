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


# ---------------------------------------------------------------------------
# Volume terms of the diagonal DG block (Sec. II.A, Eq. DGHamiltonian, first
# group; Sec. III "Construction of the DG Hamiltonian"):
#   A_K[j][j'] = 1/2 <grad phi_j, grad phi_j'>_E + <phi_j, V_eff phi_j'>_E
# with every integral a Gauss quadrature on the element's Legendre-Gauss-
# Lobatto grid (per direction twice the uniform points of the element, as in
# the accuracy study of Sec. IV), grad Phi from LGL differentiation matrices.
#
# Readings (the paper does not spell these out):
# * phi on the LGL grid: the eigenvectors on Q_K are trigonometric
#   polynomials of the periodic box, so they are evaluated at the LGL points
#   by Fourier interpolation (the even-n Nyquist mode as a cosine) and the
#   ALBs follow as phi = psi_E T with the same T that maps the restricted
#   eigenvectors to the ALBs on the uniform grid: T = dV psi_E^T phi sigma^-2
#   (a zero column where sigma = 0).
# * V_eff at the LGL points: Fourier interpolation of V on Q_K.
# * E_K along axis d is [lo_d h_d, hi_d h_d] with grid point i at i h_d.
# ---------------------------------------------------------------------------

def lgl(m):
    """Nodes (ascending) and weights of the m-point Legendre-Gauss-Lobatto
    rule on [-1, 1].  Interior nodes: eigenvalues of the Jacobi matrix of the
    Jacobi polynomials P^(1,1) (Golub-Welsch); weights 2 / (N (N+1) P_N(x)^2)
    with N = m - 1."""
    N = m - 1
    k = np.arange(1, N - 1, dtype=np.float64)
    b = np.sqrt(k * (k + 2) / ((2 * k + 1) * (2 * k + 3)))
    J = np.diag(b, 1) + np.diag(b, -1)
    inner = np.linalg.eigvalsh(J) if N >= 2 else np.zeros(0)
    x = np.concatenate(([-1.0], inner, [1.0]))
    c = np.zeros(N + 1)
    c[N] = 1.0
    w = 2.0 / (N * (N + 1) * np.polynomial.legendre.legval(x, c) ** 2)
    return x, w


def diff_matrix(x):
    """Derivative matrix of the polynomial interpolant on nodes x, from the
    barycentric weights (Berrut and Trefethen 2004): D[i][j] =
    (l_j / l_i) / (x_i - x_j), D[i][i] = -sum_{j != i} D[i][j]."""
    d = x[:, None] - x[None, :]
    np.fill_diagonal(d, 1.0)
    lam = 1.0 / np.prod(d, axis=1)
    D = (lam[None, :] / lam[:, None]) / d
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, -D.sum(axis=1))
    return D


def fourier_matrix(n, L, pts):
    """Rows: evaluation at pts of the trigonometric interpolant of n samples
    at i L / n, acting on numpy FFT coefficients (divided by n inside)."""
    k = np.fft.fftfreq(n, 1.0 / n)
    E = np.exp(2j * np.pi * np.outer(pts, k) / L) / n
    if n % 2 == 0:
        E[:, n // 2] = np.cos(np.pi * n * pts / L) / n
    return E


def fourier_eval(F, grid, box, pts):
    """F: (Ng, c) samples on the periodic grid (flat x-fastest); pts: three
    point lists -> values on their tensor grid, (m3, m2, m1, c)."""
    n1, n2, n3 = grid
    A = np.fft.fftn(F.reshape(n3, n2, n1, -1), axes=(0, 1, 2))
    A = np.einsum("ix,zyxc->zyic", fourier_matrix(n1, box[0], pts[0]), A)
    A = np.einsum("jy,zyic->zjic", fourier_matrix(n2, box[1], pts[1]), A)
    A = np.einsum("kz,zjic->kjic", fourier_matrix(n3, box[2], pts[2]), A)
    return A.real


def lgl_grid(grid, box, lo, hi, ratio=2):
    """Per axis: LGL points on [lo h, hi h], weights and derivative matrix,
    ratio * (hi - lo) points."""
    out = []
    for d in range(3):
        h = box[d] / grid[d]
        ell = (hi[d] - lo[d]) * h
        r, w = lgl(ratio * (hi[d] - lo[d]))
        out.append((lo[d] * h + 0.5 * (r + 1.0) * ell, 0.5 * ell * w,
                    (2.0 / ell) * diff_matrix(r)))
    return out


def volume_block(psi, albs, sigma, V, grid, box, lo, hi, ratio=2):
    """psi: Ng x J eigenvectors on Q_K (dV sum psi^2 = 1); albs: N_E x n_alb
    and sigma: n_alb from their restriction (oracle.alb.restrict_svd);
    V: Ng -> n_alb x n_alb volume terms of the diagonal DG block."""
    dv = float(np.prod(box)) / float(np.prod(grid))
    rows = box_rows(grid, lo, hi)
    inv = np.zeros_like(sigma)                # a zero singular value gives a zero column
    inv[sigma > 0] = 1.0 / sigma[sigma > 0] ** 2
    T = dv * (psi[rows].T @ albs) * inv[None, :]            # psi_E T = albs
    ax = lgl_grid(grid, box, lo, hi, ratio)
    pts = [a[0] for a in ax]
    Phi = np.einsum("zyxj,jk->zyxk", fourier_eval(psi, grid, box, pts), T)
    VL = fourier_eval(V.reshape(-1, 1), grid, box, pts)[..., 0]
    W = ax[2][1][:, None, None] * ax[1][1][None, :, None] * ax[0][1][None, None, :]
    A = np.einsum("zyxj,zyx,zyxk->jk", Phi, W * VL, Phi)
    grads = (np.einsum("ix,zyxk->zyik", ax[0][2], Phi),
             np.einsum("jy,zyxk->zjxk", ax[1][2], Phi),
             np.einsum("kz,zyxc->kyxc", ax[2][2], Phi))
    for G in grads:
        A += 0.5 * np.einsum("zyxj,zyx,zyxk->jk", G, W, G)
    return A
