"""Pins of restriction + SVD truncation (Sec. II.A after Eq. localproblem;
Sec. II.B end of "Generation of the ALB functions"; Eq. orthonormal)."""
import numpy as np

from oracle import alb


def _orthonormal(n, k, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    return q


def test_box_rows_order():
    rows = alb.box_rows((4, 3, 2), (1, 0, 1), (3, 2, 2))
    assert rows.tolist() == [13, 14, 17, 18]


def test_whole_box_gives_unit_sigma_and_same_span():
    grid = (6, 5, 4)
    X = _orthonormal(120, 7, 0)
    A, s = alb.restrict_svd(X, grid, (0, 0, 0), grid, 0.25, 7)
    assert np.allclose(s, 1.0, atol=1e-13)
    Au = A * np.sqrt(0.25)
    assert np.abs(Au.T @ Au - np.eye(7)).max() < 1e-13
    sv = np.linalg.svd(X.T @ Au, compute_uv=False)
    assert np.allclose(sv, 1.0, atol=1e-12)


def test_sigma_against_gram_eigenvalues_and_rotation_invariance():
    grid = (8, 8, 8)
    X = _orthonormal(512, 10, 1)
    lo, hi = (2, 1, 3), (6, 7, 8)
    rows = alb.box_rows(grid, lo, hi)
    A, s = alb.restrict_svd(X, grid, lo, hi, 1.0, 10)
    lam = np.sort(np.linalg.eigvalsh(X[rows].T @ X[rows]))[::-1]
    assert np.allclose(s ** 2, lam, atol=1e-13)
    assert abs(np.sum(s ** 2) - np.sum(X[rows] ** 2)) < 1e-12
    Q = _orthonormal(10, 10, 2)
    A2, s2 = alb.restrict_svd(X @ Q, grid, lo, hi, 1.0, 4)
    assert np.allclose(s2, s[:4], atol=1e-13)
    assert np.abs(np.abs(A2) - np.abs(A[:, :4])).max() < 1e-10
    # sign convention: the largest-magnitude entry of each ALB is positive
    piv = np.argmax(np.abs(A2), axis=0)
    assert np.all(A2[piv, np.arange(4)] > 0)
    # the truncated ALBs span the leading left singular space
    U = np.linalg.svd(X[rows], full_matrices=False)[0][:, :4]
    sv = np.linalg.svd(U.T @ A2, compute_uv=False)
    assert np.allclose(sv, 1.0, atol=1e-10)
