"""Pins of the element-local DG quantities (density from the diagonal
density-matrix blocks, nonlocal Kleinman-Bylander block, volume terms of the
diagonal block on the LGL grid)."""
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


# ---- volume terms on the LGL grid ---------------------------------------

def test_lgl_closed_forms():
    """Nodes and weights of the 2- to 5-point Lobatto rules (textbook values)."""
    table = {2: ([-1, 1], [1, 1]),
             3: ([-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
             4: ([-1, -5 ** -0.5, 5 ** -0.5, 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
             5: ([-1, -(3 / 7) ** 0.5, 0, (3 / 7) ** 0.5, 1],
                 [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10])}
    for m, (xs, ws) in table.items():
        x, w = dgblocks.lgl(m)
        assert np.allclose(x, xs, atol=1e-15) and np.allclose(w, ws, atol=1e-15)


def test_lgl_degree_of_exactness():
    """An m-point Lobatto rule integrates x^k exactly up to k = 2m - 3 and no
    further (a Gauss rule would reach 2m - 1)."""
    for m in (6, 16, 40):
        x, w = dgblocks.lgl(m)
        for k in range(2 * m - 2):
            exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
            assert abs(w @ x ** k - exact) < 1e-13, (m, k)
    x, w = dgblocks.lgl(6)
    assert abs(w @ x ** 10 - 2.0 / 11) > 1e-4


def test_diff_matrix_exact_on_polynomials():
    rng = np.random.default_rng(4)
    for m in (5, 16, 40):
        x, _ = dgblocks.lgl(m)
        D = dgblocks.diff_matrix(x)
        c = rng.standard_normal(m)                       # degree m - 1
        p = np.polynomial.Polynomial(c)
        assert np.allclose(D @ p(x), p.deriv()(x), atol=1e-10 * np.abs(c).sum() * m * m)
        N = m - 1                                        # corner entries at the LGL nodes
        assert abs(D[0, 0] + N * (N + 1) / 4) < 1e-9 and abs(D[N, N] - N * (N + 1) / 4) < 1e-9


def _trig(kind, k, L):
    w = 2 * np.pi * k / L
    if kind == "c":
        return (lambda x: np.cos(w * x)), (lambda x: -w * np.sin(w * x))
    return (lambda x: np.sin(w * x)), (lambda x: w * np.cos(w * x))


def test_fourier_eval_reproduces_trig_polynomials():
    """Samples of a band-limited function (with an even-n Nyquist cosine) are
    interpolated exactly, at grid points and between them."""
    rng = np.random.default_rng(5)
    grid, box = (8, 10, 6), (3.0, 4.0, 2.5)
    terms = [(rng.standard_normal(), [("c", 1), ("s", 2), ("c", 0)]),
             (rng.standard_normal(), [("s", 3), ("c", 4), ("s", 2)]),
             (rng.standard_normal(), [("c", 4), ("c", 5), ("c", 3)])]      # Nyquist on every axis

    def f(x, y, z):
        return sum(a * _trig(*s[0], box[0])[0](x) * _trig(*s[1], box[1])[0](y) *
                   _trig(*s[2], box[2])[0](z) for a, s in terms)
    ax = [np.arange(grid[d]) * box[d] / grid[d] for d in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    F = f(X, Y, Z).reshape(-1, 1)
    pts = [rng.uniform(0, box[d], 5) for d in range(3)]
    Z, Y, X = np.meshgrid(pts[2], pts[1], pts[0], indexing="ij")
    got = dgblocks.fourier_eval(F, grid, box, pts)[..., 0]
    assert np.allclose(got, f(X, Y, Z), atol=1e-12)
    assert np.allclose(dgblocks.fourier_eval(F, grid, box, ax)[..., 0].reshape(-1), F[:, 0], atol=1e-12)


def test_volume_block_analytic():
    """Band-limited separable eigenvector stand-ins: the volume terms equal
    T^T A_psi T with A_psi's entries integrated adaptively one axis at a time
    (scipy.integrate.quad) and T solved by least squares from psi_E T = phi."""
    import warnings
    from scipy.integrate import IntegrationWarning, quad
    from oracle.alb import restrict_svd
    grid, box = (24, 24, 30), (10.0, 9.0, 12.5)
    lo, hi = (8, 8, 10), (16, 16, 20)
    cols = [[("c", 1), ("c", 0), ("s", 1)],
            [("s", 2), ("c", 1), ("c", 0)],
            [("c", 0), ("s", 1), ("c", 2)]]
    vterms = [(0.7, [("c", 0), ("c", 0), ("c", 0)]),
              (-1.3, [("c", 1), ("c", 0), ("c", 0)]),
              (0.4, [("c", 0), ("s", 2), ("c", 1)])]
    ax = [np.arange(grid[d]) * box[d] / grid[d] for d in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    P3 = (X, Y, Z)

    def sample(spec):
        out = np.ones_like(X)
        for d in range(3):
            out = out * _trig(*spec[d], box[d])[0](P3[d])
        return out.reshape(-1)
    psi = np.column_stack([sample(c) for c in cols])
    V = sum(a * sample(s) for a, s in vterms)
    dv = float(np.prod(box)) / float(np.prod(grid))
    rows = box_rows(grid, lo, hi)
    for n_alb in (3, 2):
        albs, sigma = restrict_svd(np.sqrt(dv) * psi, grid, lo, hi, dv, n_alb)
        A = dgblocks.volume_block(psi, albs, sigma, V, grid, box, lo, hi)
        T = np.linalg.lstsq(psi[rows], albs, rcond=None)[0]

        def integral(d, g):
            h = box[d] / grid[d]
            with warnings.catch_warnings():      # near-zero integrals hit the absolute floor
                warnings.simplefilter("ignore", IntegrationWarning)
                return quad(g, lo[d] * h, hi[d] * h, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
        J = len(cols)
        Apsi = np.zeros((J, J))
        for i in range(J):
            for j in range(J):
                for d in range(3):                       # kinetic
                    t = 0.5
                    for e in range(3):
                        fi, dfi = _trig(*cols[i][e], box[e])
                        fj, dfj = _trig(*cols[j][e], box[e])
                        t *= integral(e, (lambda x, a=dfi, b=dfj: a(x) * b(x)) if e == d else
                                      (lambda x, a=fi, b=fj: a(x) * b(x)))
                    Apsi[i, j] += t
                for a, s in vterms:                      # potential
                    t = a
                    for e in range(3):
                        fi, fj, v = (_trig(*cols[i][e], box[e])[0], _trig(*cols[j][e], box[e])[0],
                                     _trig(*s[e], box[e])[0])
                        t *= integral(e, lambda x, a=fi, b=fj, c=v: a(x) * b(x) * c(x))
                    Apsi[i, j] += t
        ref = T.T @ Apsi @ T
        assert np.allclose(A, ref, rtol=0, atol=1e-9 * np.abs(ref).max()), np.abs(A - ref).max()


def test_volume_block_invariants():
    """On a solved element: symmetric; the kinetic part (V = 0) is positive
    semidefinite; a constant V adds c times the LGL overlap matrix, which is
    symmetric positive definite and independent of c."""
    from oracle import dense
    from oracle.hamiltonian import Operator
    from oracle.alb import restrict_svd
    el = synth.single_element(seed=2, grid=(12, 12, 12), n_states=8, n_atoms=2)
    H = Operator(el.grid, el.box, el.V, el.kb).dense()
    w, X = dense.lowest(H, el.n_states)
    albs, sigma = restrict_svd(X, el.grid, el.elem_lo, el.elem_hi, el.dv, el.n_alb)
    psi = X / np.sqrt(el.dv)
    A = dgblocks.volume_block(psi, albs, sigma, el.V, el.grid, el.box, el.elem_lo, el.elem_hi)
    assert np.allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    K = dgblocks.volume_block(psi, albs, sigma, np.zeros(el.ng), el.grid, el.box,
                              el.elem_lo, el.elem_hi)
    assert np.linalg.eigvalsh(K).min() > -1e-10 * np.abs(K).max()
    c = 0.37
    A2 = dgblocks.volume_block(psi, albs, sigma, np.full(el.ng, c), el.grid, el.box,
                               el.elem_lo, el.elem_hi)
    S = (A2 - K) / c
    assert np.allclose(S, S.T, atol=1e-12)
    assert np.linalg.eigvalsh(S).min() > 0
    A3 = dgblocks.volume_block(psi, albs, sigma, np.full(el.ng, -2.0), el.grid, el.box,
                               el.elem_lo, el.elem_hi)
    assert np.allclose(A3 - K, -2.0 * S, atol=1e-10 * np.abs(S).max())
