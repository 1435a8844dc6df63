"""Pins of the oracle's discrete operator (Eq. localproblem, planewave
discretisation of Sec. II.B, KB term of Eq. DGvar)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle.hamiltonian import Operator
from oracle import dense
from tests._pins import fourier_d2, free_electron_levels, kron_sum


def _empty_kb():
    return synth.KB(np.zeros(0), np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))


def test_free_electron_dense_matches_closed_form():
    grid, box = (12, 10, 8), (5.0, 4.2, 3.7)
    op = Operator(grid, box, np.zeros(960), _empty_kb())
    w = np.linalg.eigvalsh(op.dense())
    ref = free_electron_levels(grid, box, 960)
    assert np.abs(w - ref).max() < 1e-11


def test_kinetic_matches_trefethen_kronecker_sum_entrywise():
    grid, box = (8, 6, 5), (3.1, 2.7, 2.2)
    rng = np.random.default_rng(7)
    v1, v2, v3 = (rng.uniform(-1, 1, n) for n in grid)
    V = (v3[:, None, None] + v2[None, :, None] + v1[None, None, :]).reshape(-1)
    op = Operator(grid, box, V, _empty_kb())
    A = [-0.5 * fourier_d2(n, L) + np.diag(v) for n, L, v in zip(grid, box, (v1, v2, v3))]
    ref = kron_sum(*A)
    assert np.abs(op.dense() - ref).max() < 1e-12 * np.abs(ref).max()


def test_separable_spectrum_large_grid_dense_1d():
    """Separable V = v(x)+v(y)+v(z): lowest eigenvalues are the smallest sums
    of three 1D spectra (1D matrices from the closed form, not the FFT)."""
    grid, box = (12, 12, 16), (5.0, 5.0, 6.6)
    xs = [np.arange(n) * (L / n) for n, L in zip(grid, box)]
    vs = [-2.0 * np.exp(-((x - L / 2) ** 2) / (2 * 0.7 ** 2)) for x, L in zip(xs, box)]
    V = (vs[2][:, None, None] + vs[1][None, :, None] + vs[0][None, None, :]).reshape(-1)
    op = Operator(grid, box, V, _empty_kb())
    ev = [np.linalg.eigvalsh(-0.5 * fourier_d2(n, L) + np.diag(v))
          for n, L, v in zip(grid, box, vs)]
    sums = np.sort((ev[2][:, None, None] + ev[1][None, :, None] + ev[0][None, None, :]).ravel())
    w, _ = dense.lowest(op.dense(), 20)
    assert np.abs(w - sums[:20]).max() < 1e-11


def test_constant_shift():
    el = synth.single_element(seed=3, grid=(10, 10, 10), n_states=8)
    op0 = Operator(el.grid, el.box, el.V, el.kb)
    op1 = Operator(el.grid, el.box, el.V + 0.37, el.kb)
    w0 = np.linalg.eigvalsh(op0.dense())[:12]
    w1 = np.linalg.eigvalsh(op1.dense())[:12]
    assert np.abs(w1 - w0 - 0.37).max() < 1e-12


def _secular_roots(t_levels, weights, gamma, lo, hi, count):
    """Roots of 1 + gamma sum_t w_t/(t - lam) = 0 by bisection on each interval
    between distinct levels (textbook rank-one update of a diagonal)."""
    f = lambda lam: 1.0 + gamma * np.sum(weights / (t_levels - lam))  # noqa: E731
    edges = np.concatenate([[lo], t_levels, [hi]])
    roots = []
    for a, b in zip(edges[:-1], edges[1:]):
        a1, b1 = a + 1e-13 * max(1, abs(a)), b - 1e-13 * max(1, abs(b))
        if a1 >= b1 or np.sign(f(a1)) == np.sign(f(b1)):
            continue
        for _ in range(200):
            m = 0.5 * (a1 + b1)
            if np.sign(f(m)) == np.sign(f(a1)):
                a1 = m
            else:
                b1 = m
        roots.append(0.5 * (a1 + b1))
        if len(roots) >= count:
            break
    return np.asarray(roots)


@pytest.mark.parametrize("gamma", [-0.8, 0.6])
def test_kb_rank_one_secular_equation(gamma):
    grid = (10, 10, 10)
    box = tuple(n * synth.H_SPACING for n in grid)
    atoms = np.array([[1.3, 2.2, 0.7, 0.0, 0.8]])
    kb = synth.gaussian_kb(grid, box, atoms, np.array([[gamma, 0, 0, 0]]))
    kb = synth.KB(kb.gamma[:1], kb.ptr[:2], kb.idx[:kb.ptr[1]], kb.val[:kb.ptr[1]])
    ng = 1000
    dv = np.prod(box) / ng
    op = Operator(grid, box, np.zeros(ng), kb)
    w = np.linalg.eigvalsh(op.dense())
    # projector in the unit basis and its planewave weights, grouped by level
    beta = np.zeros(ng)
    beta[kb.idx] = np.sqrt(dv) * kb.val
    bh = np.fft.fftn(beta.reshape(10, 10, 10))
    m = np.where(np.arange(10) <= 5, np.arange(10), np.arange(10) - 10)
    t = 0.5 * (2 * np.pi / box[0]) ** 2 * (m[:, None, None] ** 2 + m[None, :, None] ** 2 +
                                           m[None, None, :] ** 2)
    tk = np.round(t.ravel(), 12)
    levels = np.unique(tk)
    wts = np.array([np.sum(np.abs(bh.ravel()[tk == lv]) ** 2) / ng for lv in levels])
    assert abs(wts.sum() - 1.0) < 1e-12      # beta is a unit vector
    roots = _secular_roots(levels, wts, gamma, levels[0] - 10.0, levels[-1] + 10.0, 40)
    # every secular root is an eigenvalue, and the remaining low eigenvalues are
    # unperturbed levels
    for r in roots[:6]:
        assert np.min(np.abs(w - r)) < 1e-10
    low = w[w < levels[3]]
    for x in low:
        assert min(np.min(np.abs(roots - x)), np.min(np.abs(levels - x))) < 1e-10


def test_hermiticity():
    el = synth.single_element(seed=1)
    op = Operator(el.grid, el.box, el.V, el.kb)
    rng = np.random.default_rng(11)
    u, v = rng.standard_normal(op.ng), rng.standard_normal(op.ng)
    hnorm = op.t.max() + np.abs(el.V).max() + np.abs(el.kb.gamma).sum()
    assert abs(u @ op.apply(v) - v @ op.apply(u)) <= 1e-13 * np.linalg.norm(u) * \
        np.linalg.norm(v) * hnorm


def test_translation_by_grid_steps_and_axis_permutation():
    # narrow wells (w = 0.5 bohr) so that images beyond the 27 summed ones and
    # the projector cut-off (4w < L/2) are below rounding on this small box
    grid = (10, 10, 10)
    el = synth.single_element(seed=5, grid=grid, n_states=8, n_atoms=3)
    el.atoms[:, 4] = 0.5
    h = synth.H_SPACING
    L = np.asarray(el.box)

    def spectrum(atoms):
        box = el.box
        V = synth.gaussian_wells(grid, box, atoms)
        gam = np.random.default_rng(0).uniform(-1, 1, (len(atoms), 4))
        kb = synth.gaussian_kb(grid, box, atoms, gam)
        return np.linalg.eigvalsh(Operator(grid, box, V, kb).dense())[:15], gam

    w0, _ = spectrum(el.atoms)
    sh = el.atoms.copy()
    sh[:, :3] = np.mod(sh[:, :3] + np.array([2 * h, -3 * h, 5 * h]), L)
    w1, _ = spectrum(sh)
    assert np.abs(w1 - w0).max() < 1e-11
    # permuting the axes of a cube permutes p_x/p_y/p_z among themselves; use
    # s-only couplings so the projector set maps onto itself
    at = el.atoms.copy()
    box = el.box
    gam = np.zeros((len(at), 4))
    gam[:, 0] = [0.5, -0.3, 0.2]

    def spec2(atoms):
        V = synth.gaussian_wells(grid, box, atoms)
        kb = synth.gaussian_kb(grid, box, atoms, gam)
        return np.linalg.eigvalsh(Operator(grid, box, V, kb).dense())[:15]

    perm = at.copy()
    perm[:, [0, 1, 2]] = at[:, [2, 0, 1]]
    assert np.abs(spec2(perm) - spec2(at)).max() < 1e-11
