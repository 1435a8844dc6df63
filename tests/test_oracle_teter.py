"""Pins of the Teter preconditioner (Sec. II.B cites Payne, Teter, Allan et al.)."""
import numpy as np

from oracle import teter
import synth


def test_teter_function_limits_and_shape():
    assert teter.teter_k(0.0) == 1.0
    x = np.linspace(0, 50, 5001)
    k = teter.teter_k(x)
    assert np.all(k > 0) and np.all(k <= 1.0)
    assert np.all(np.diff(k) < 0)
    # high-x tail K(x) ~ 1/(2x)
    assert abs(teter.teter_k(1e6) * 2e6 - 1.0) < 1e-5
    assert abs(teter.teter_k(100.0) * 200.0 - 1.0101) < 1e-4


def test_band_kinetic_of_plane_waves():
    grid, box = (12, 10, 8), (5.0, 4.0, 3.5)
    n1, n2, n3 = grid
    x = np.arange(n1) * box[0] / n1
    y = np.arange(n2) * box[1] / n2
    z = np.arange(n3) * box[2] / n3
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    cols, expect = [], []
    for m in [(1, 0, 0), (2, 3, 1), (0, 0, 0), (-3, 1, 2)]:
        G = 2 * np.pi * np.array(m) / np.array(box)
        c = np.cos(G[0] * X + G[1] * Y + G[2] * Z).ravel()
        cols.append(c / np.linalg.norm(c))
        expect.append(0.5 * G @ G)
    T = teter.band_kinetic(np.column_stack(cols), grid, box)
    assert np.allclose(T, expect, rtol=1e-13, atol=1e-13)


def test_precondition_is_diagonal_in_g():
    """A plane-wave residual is an eigenvector of the preconditioner with
    eigenvalue K(|G|^2/2 / T)."""
    grid, box = (12, 12, 12), (5.0, 5.0, 5.0)
    n = 12
    x = np.arange(n) * 5.0 / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    G = 2 * np.pi * np.array([2, 1, 0]) / 5.0
    r = np.sin(G[0] * X + G[1] * Y).ravel()
    G0 = 2 * np.pi * np.array([1, 0, 0]) / 5.0
    xv = np.cos(G0[0] * X).ravel()
    xv /= np.linalg.norm(xv)
    T = 0.5 * G0 @ G0
    w = teter.precondition(r[:, None], xv[:, None], grid, box)[:, 0]
    assert np.allclose(w, teter.teter_k(0.5 * G @ G / T) * r, atol=1e-13)
    # floor: a constant vector has T = 0 and uses the smallest planewave energy
    c = np.ones(n ** 3) / np.sqrt(n ** 3)
    w2 = teter.precondition(r[:, None], c[:, None], grid, box)[:, 0]
    assert np.allclose(w2, teter.teter_k(0.5 * G @ G / teter.kinetic_floor(box)) * r, atol=1e-13)
