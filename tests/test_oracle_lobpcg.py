"""Pins of the oracle LOBPCG (Sec. II.B) against brute force, closed forms and
an independent Krylov library."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as ssl

import synth
from oracle import dense, lobpcg as lob, teter
from oracle.hamiltonian import Operator
from oracle.solve import solve_element
from tests._pins import fourier_d2, free_electron_levels

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "one_element_dense.json")


def _run(el, tol, max_iter=400, X0=None):
    op = Operator(el.grid, el.box, el.V, el.kb)
    pre = lambda R, X: teter.precondition(R, X, op.grid, op.box)  # noqa: E731
    return op, lob.lobpcg(op.apply, pre, el.X0 if X0 is None else X0, tol, max_iter)


def test_small_grid_vs_dense_eigh():
    el = synth.single_element(seed=2, grid=(12, 12, 12), n_states=10, n_atoms=3)
    op, res = _run(el, 1e-9)
    assert res.converged
    H = op.dense()
    w, U = dense.lowest(H, 14)
    J = 10
    assert np.abs(res.theta - w[:J]).max() < 1e-10
    # orthonormality and residual reported honestly
    assert np.abs(res.X.T @ res.X - np.eye(J)).max() < 1e-12
    r = np.linalg.norm(H @ res.X - res.X * res.theta, axis=0)
    assert np.allclose(r, res.resid, atol=1e-12)
    # variational bound (Cauchy interlacing) and residual bound
    assert np.all(res.theta >= w[:J] - 1e-12)
    assert np.all(np.abs(res.theta - w[:J]) <= res.resid + 1e-13)
    # subspace: largest principal angle, where the cut has a gap
    if w[J] - w[J - 1] > 1e-4:
        s = np.linalg.svd(U[:, :J].T @ res.X, compute_uv=False)
        assert np.sqrt(max(0.0, 1 - s.min() ** 2)) < 1e-7


def test_free_electron_closed_form():
    el = synth.single_element(seed=0, grid=(16, 16, 16), n_states=19, wells=False, kb=False)
    _, res = _run(el, 1e-9)
    ref = free_electron_levels(el.grid, el.box, 19)
    assert res.converged
    assert np.abs(res.theta - ref).max() < 1e-12


def test_separable_spectrum_36x36x60():
    """Exact reference from three 1D closed-form operators; dense 3D is infeasible."""
    grid = (36, 36, 60)
    box = tuple(n * synth.H_SPACING for n in grid)
    xs = [np.arange(n) * (L / n) for n, L in zip(grid, box)]
    vs = [-1.5 * np.exp(-((x - L / 3) ** 2) / (2 * 0.8 ** 2)) for x, L in zip(xs, box)]
    V = (vs[2][:, None, None] + vs[1][None, :, None] + vs[0][None, None, :]).reshape(-1)
    ev = [np.linalg.eigvalsh(-0.5 * fourier_d2(n, L) + np.diag(v))
          for n, L, v in zip(grid, box, vs)]
    sums = np.sort((ev[2][:, None, None] + ev[1][None, :, None] + ev[0][None, None, :]).ravel())
    J = 12
    el = synth.Element(grid=grid, box=box, V=V,
                       kb=synth.KB(np.zeros(0), np.zeros(1, np.int64), np.zeros(0, np.int32),
                                   np.zeros(0)),
                       X0=synth.initial_guess(int(np.prod(grid)), J, 9, 0, 0), n_states=J,
                       elem_lo=(0, 0, 0), elem_hi=grid, n_alb=J, atoms=np.zeros((0, 5)))
    _, res = _run(el, 1e-8)
    assert res.converged
    # compare values below the largest cut with a gap
    assert np.abs(res.theta - sums[:J]).max() < 1e-11


def test_one_element_workload_vs_stored_dense():
    """Full one-element workload (24^3, 32 states) against the dense LAPACK
    eigenvalues written by tests/golden/make_golden.py."""
    gold = json.load(open(GOLDEN))
    el = synth.single_element(seed=0)
    _, res = _run(el, 1e-8)
    w = np.asarray(gold["seeds"]["0"])
    assert res.converged
    assert np.abs(res.theta - w[:32]).max() < 1e-10
    assert np.all(res.theta >= w[:32] - 1e-12)


def test_guard_columns_same_states_fewer_iterations():
    """8 guard columns on the one-element workload (block of 40, the lowest
    32 tested): the 32 eigenvalues equal the stored dense ones and bound them
    from above, in fewer iterations than the block of 32; the guard Ritz
    values still bound eigenvalues 33..40 from above."""
    gold = json.load(open(GOLDEN))
    w = np.asarray(gold["seeds"]["0"])
    el = synth.single_element(seed=0)
    op = Operator(el.grid, el.box, el.V, el.kb)
    pre = lambda R, X: teter.precondition(R, X, op.grid, op.box)  # noqa: E731
    X0 = np.hstack([el.X0, synth.guard_columns(el.ng, 8, (0, el.n_states))])
    res = lob.lobpcg(op.apply, pre, X0, 1e-8, 400, n_check=32)
    plain = lob.lobpcg(op.apply, pre, el.X0, 1e-8, 400)
    assert res.converged and plain.converged
    assert res.resid[:32].max() <= 1e-8
    assert np.abs(res.theta[:32] - w[:32]).max() < 1e-10
    assert np.all(res.theta[:32] >= w[:32] - 1e-12)
    if len(w) >= 40:
        assert np.all(res.theta[32:] >= w[32:40] - 1e-12)
    assert res.iters < plain.iters
    with pytest.raises(ValueError):
        lob.lobpcg(op.apply, pre, X0, 1e-8, 1, n_check=41)


def test_vs_arpack_on_slab_geometry():
    """An independent library (ARPACK through scipy) on a LinearOperator."""
    grid = (24, 24, 36)
    box = tuple(n * synth.H_SPACING for n in grid)
    el = synth.slab_batch(1, grid=grid, n_states=12, n_atoms=6)[0]
    op, res = _run(el, 1e-9)
    A = ssl.LinearOperator((op.ng, op.ng), matvec=lambda v: op.apply(v.ravel()), dtype=float)
    w = np.sort(ssl.eigsh(A, k=12, which="SA", tol=1e-13, maxiter=20000,
                          v0=np.ones(op.ng))[0])
    assert res.converged
    assert np.abs(res.theta - w).max() < 1e-10


def test_rank_deficient_initial_guess_breaks_down():
    el = synth.single_element(seed=0, grid=(12, 12, 12), n_states=6, n_atoms=2)
    X0 = el.X0.copy()
    X0[:, 3] = X0[:, 1]
    with pytest.raises(lob.Breakdown):
        _run(el, 1e-8, X0=X0)


def test_iteration_cap_reports_not_converged():
    el = synth.single_element(seed=0, grid=(12, 12, 12), n_states=6, n_atoms=2)
    _, res = _run(el, 1e-10, max_iter=2)
    assert res.iters == 2 and not res.converged
    assert res.resid.max() > 1e-10


def test_warm_start_converges_immediately():
    el = synth.single_element(seed=4, grid=(12, 12, 12), n_states=6, n_atoms=2)
    _, res = _run(el, 1e-9)
    _, res2 = _run(el, 1e-8, X0=res.X)
    assert res2.iters == 0 and res2.converged
    assert np.abs(res2.theta - res.theta).max() < 1e-12


def test_solve_element_normalisation():
    el = synth.single_element(seed=2, grid=(12, 12, 12), n_states=8, n_atoms=3)
    out = solve_element(el, tol=1e-9)
    dv = el.dv
    psi = out["eigvecs"]
    assert np.abs(dv * psi.T @ psi - np.eye(8)).max() < 1e-12
    phi = out["albs"]
    assert np.abs(dv * phi.T @ phi - np.eye(el.n_alb)).max() < 1e-12


# ---------------------------------------------------------------------------
# Fallback branches of the oracle's LOBPCG (Sec. II.B; Knyazev's method as
# cited there): SVQB orthonormalisation, the rank-deficient Rayleigh-Ritz
# reduction and the next search direction (with its P-drop case), each
# pinned by linear algebra that does not go through the oracle.

def _scaled(Y):
    return Y / np.linalg.norm(Y, axis=0)[None, :]


def test_svqb_orthonormalises_a_well_conditioned_block():
    rng = np.random.default_rng(11)
    Y = rng.standard_normal((300, 12)) * np.logspace(-3, 3, 12)[None, :]
    T = lob.svqb(Y)
    Q = Y @ T
    assert np.abs(Q.T @ Q - np.eye(12)).max() < 1e-12
    # span preserved (principal angles from an SVD-based library routine)
    import scipy.linalg as sla
    assert sla.subspace_angles(Y, Q).max() < 1e-10


def test_svqb_nearly_dependent_block_clamps_only_the_small_directions():
    """Two columns 1e-6 apart (after scaling): the scaled CholQR refuses the
    block, SVQB returns mutually orthogonal columns whose squared norms are
    min(1, s_i^2 / (1e-10 s_max^2)), s_i the singular values of the
    column-scaled block (from an SVD, not the oracle's eigh)."""
    rng = np.random.default_rng(12)
    Y = rng.standard_normal((400, 10)) * np.linspace(0.5, 20.0, 10)[None, :]
    Y[:, 7] = 3.0 * (Y[:, 2] + 1e-6 * np.linalg.norm(Y[:, 2]) / 20.0 * rng.standard_normal(400))
    assert lob.scaled_cholqr(Y) is None
    T = lob.svqb(Y)
    G = (Y @ T).T @ (Y @ T)
    s = np.linalg.svd(_scaled(Y), compute_uv=False)
    lam = np.sort(s ** 2)
    expect = np.minimum(1.0, lam / (lob.CHOL_TOL * lam.max()))
    assert expect[0] < 0.1   # the small direction really is clamped
    assert np.abs(np.diag(G) - expect).max() < 1e-5
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-9
    import scipy.linalg as sla
    assert sla.subspace_angles(Y, Y @ T).max() < 1e-8


def _sym_problem(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    H = A + A.T
    w, U = np.linalg.eigh(H)
    return rng, H, w, U


def test_rayleigh_ritz_full_rank_nonorthonormal_basis():
    rng, H, w, U = _sym_problem(60, 13)
    J = 6
    S = U[:, :J + 3] @ rng.standard_normal((J + 3, J + 3))
    st = lob.Result(None, None, None, 0, False, [])
    theta, C, M = lob.rayleigh_ritz(S, H @ S, J, st)
    X = S @ C
    assert st.n_rr_fallback == 0
    assert np.abs(theta - w[:J]).max() < 1e-11
    assert np.abs(X.T @ X - np.eye(J)).max() < 1e-11
    assert np.abs(H @ X - X * theta[None, :]).max() < 1e-10


def test_rayleigh_ritz_rank_deficient_basis_takes_the_reduction():
    """A basis with a duplicated column: M is singular, the oracle reduces to
    the eigenvectors of M, and still returns the exact lowest pairs of H on
    the span (which holds the J + 3 lowest eigenvectors)."""
    rng, H, w, U = _sym_problem(60, 14)
    J = 6
    A = U[:, :J + 3] @ rng.standard_normal((J + 3, J + 3))
    S = np.hstack([A, A[:, [1]]])
    st = lob.Result(None, None, None, 0, False, [])
    theta, C, M = lob.rayleigh_ritz(S, H @ S, J, st)
    X = S @ C
    assert st.n_rr_fallback == 1
    assert np.abs(theta - w[:J]).max() < 1e-11
    assert np.abs(X.T @ X - np.eye(J)).max() < 1e-10
    assert np.abs(H @ X - X * theta[None, :]).max() < 1e-9
    # fewer than J independent columns: breakdown
    S2 = np.hstack([A[:, :J - 1], A[:, [0]]])
    with pytest.raises(lob.Breakdown):
        lob.rayleigh_ritz(S2, H @ S2, J, st)


def test_next_direction_is_the_orthogonal_complement():
    """D spans the part of S [0; C_P; C_W] orthogonal to S C, with
    (S D)^T (S D) = I: checked by orthogonality, normalisation and a rank
    count of the combined span against [C, E]."""
    rng, H, w, U = _sym_problem(90, 15)
    J = 5
    S = rng.standard_normal((90, 3 * J))
    st = lob.Result(None, None, None, 0, False, [])
    theta, C, M = lob.rayleigh_ritz(S, H @ S, J, st)
    D = lob.next_direction(C, M, J)
    assert D is not None
    X, P = S @ C, S @ D
    assert np.abs(P.T @ P - np.eye(J)).max() < 1e-10
    assert np.abs(X.T @ P).max() < 1e-10
    E = C.copy()
    E[:J] = 0.0
    # D lies in span[C, E] and together with C spans all of it
    B = np.hstack([C, E])
    coef = np.linalg.lstsq(B, D, rcond=None)[0]
    assert np.abs(B @ coef - D).max() < 1e-10
    assert np.linalg.matrix_rank(np.hstack([C, D]), tol=1e-8) == np.linalg.matrix_rank(B, tol=1e-8)


def test_next_direction_drops_p_when_ritz_vectors_stay_in_x():
    """When the Ritz vectors have no P or W component (C = [I; 0; 0]) there
    is no new direction: the oracle returns None (P is dropped)."""
    J = 4
    C = np.zeros((3 * J, J))
    C[:J] = np.eye(J)
    assert lob.next_direction(C, np.eye(3 * J), J) is None


def test_lobpcg_without_p_still_reaches_the_dense_eigenvalues(monkeypatch):
    """Every iteration takes the P-drop path (next_direction forced to None):
    the method degenerates to a block preconditioned steepest descent and
    must still converge to the dense eigenvalues."""
    el = synth.single_element(seed=2, grid=(12, 12, 12), n_states=6, n_atoms=3)
    monkeypatch.setattr(lob, "next_direction", lambda C, M, J: None)
    op, res = _run(el, 1e-9, max_iter=800)
    assert res.converged and res.n_p_drop == res.iters > 0
    w, _ = dense.lowest(op.dense(), 8)
    assert np.abs(res.theta - w[:6]).max() < 1e-10


def test_lobpcg_with_svqb_for_every_w_reaches_the_dense_eigenvalues(monkeypatch):
    """Every W orthonormalisation takes the SVQB branch (the CholQR of W
    forced to fail; the initial block keeps its CholQR)."""
    el = synth.single_element(seed=2, grid=(12, 12, 12), n_states=6, n_atoms=3)
    real = lob.scaled_cholqr
    calls = {"n": 0}

    def first_only(Y):
        calls["n"] += 1
        return real(Y) if calls["n"] == 1 else None

    monkeypatch.setattr(lob, "scaled_cholqr", first_only)
    op, res = _run(el, 1e-9)
    assert res.converged and res.n_chol_fallback == res.iters > 0
    w, _ = dense.lowest(op.dense(), 8)
    assert np.abs(res.theta - w[:6]).max() < 1e-10
