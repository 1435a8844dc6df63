"""Pins of the element-local DG quantities (density from the diagonal
density-matrix blocks, nonlocal Kleinman-Bylander block)."""
import numpy as np

import synth
from oracle import dgblocks
from oracle.alb import box_rows


def test_density_closed_forms():
    rng = np.random.default_rng(0)
    ne, n, dv = 200, 7, 0.3
    Q, _ = np.linalg.qr(rng.standard_normal((ne, n)))
    phi = Q / np.sqrt(dv)                                     # dV phi^T phi = I
    assert np.allclose(dgblocks.density(phi, np.eye(n)), np.sum(phi ** 2, axis=1))
    c = rng.standard_normal(n)
    assert np.allclose(dgblocks.density(phi, np.outer(c, c)), (phi @ c) ** 2)
    A = rng.standard_normal((n, n))
    P = A + A.T
    rho = dgblocks.density(phi, P)
    assert abs(dv * rho.sum() - np.trace(P)) < 1e-10 * np.abs(P).sum()
    brute = np.array([sum(phi[x, j] * P[j, k] * phi[x, k] for j in range(n) for k in range(n))
                      for x in range(5)])
    assert np.allclose(rho[:5], brute)


def test_nonlocal_block_single_projector_closed_form():
    el = synth.single_element(seed=3, grid=(12, 12, 12), n_states=6, n_atoms=1)
    kb = el.kb
    rows = box_rows(el.grid, el.elem_lo, el.elem_hi)
    dv = el.dv
    # projector 0 restricted to the box
    bfull = np.zeros(el.ng)
    bfull[kb.idx[kb.ptr[0]:kb.ptr[1]]] = kb.val[kb.ptr[0]:kb.ptr[1]]
    bE = bfull[rows]
    nrm2 = dv * np.sum(bE ** 2)
    assert nrm2 > 0
    rng = np.random.default_rng(1)
    M = np.column_stack([bE, rng.standard_normal((rows.shape[0], 3))])
    Q, _ = np.linalg.qr(M)
    phi = Q / np.sqrt(dv)
    phi[:, 0] *= np.sign(phi[:, 0] @ bE)
    one = type(kb)(gamma=kb.gamma[:1], ptr=kb.ptr[:2], idx=kb.idx[:kb.ptr[1]], val=kb.val[:kb.ptr[1]])
    H = dgblocks.nonlocal_block(phi, one, el.grid, el.elem_lo, el.elem_hi, dv)
    assert abs(H[0, 0] - kb.gamma[0] * nrm2) < 1e-12 * abs(kb.gamma[0] * nrm2)
    assert np.abs(H[1:, 1:]).max() < 1e-12 and np.abs(H[0, 1:]).max() < 1e-12


def test_nonlocal_block_dense_definition():
    el = synth.single_element(seed=4, grid=(12, 12, 12), n_states=6, n_atoms=3)
    kb, dv = el.kb, el.dv
    rows = box_rows(el.grid, el.elem_lo, el.elem_hi)
    rng = np.random.default_rng(2)
    phi = rng.standard_normal((rows.shape[0], 4))
    # dense V_nl = sum_p gamma_p b_p b_p^T on the full grid, then dV^2 phi^T V phi on the box
    Vnl = np.zeros((el.ng, el.ng))
    for p in range(kb.gamma.shape[0]):
        b = np.zeros(el.ng)
        b[kb.idx[kb.ptr[p]:kb.ptr[p + 1]]] = kb.val[kb.ptr[p]:kb.ptr[p + 1]]
        Vnl += kb.gamma[p] * np.outer(b, b)
    ref = dv * dv * phi.T @ Vnl[np.ix_(rows, rows)] @ phi
    H = dgblocks.nonlocal_block(phi, kb, el.grid, el.elem_lo, el.elem_hi, dv)
    assert np.abs(H - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(H - H.T).max() < 1e-14 * np.abs(H).max()
