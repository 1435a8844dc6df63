"""Independent closed forms used to pin the oracle (no oracle code here)."""
import numpy as np


def fourier_d2(n: int, L: float) -> np.ndarray:
    """Second-derivative matrix of the periodic trigonometric interpolant on n
    equispaced points of a period-L interval (Trefethen, Spectral Methods in
    MATLAB, ch. 3), written out entry by entry."""
    h = 2.0 * np.pi / n
    D = np.empty((n, n))
    for a in range(n):
        for b in range(n):
            if a == b:
                D[a, b] = -np.pi ** 2 / (3 * h * h) + (-1.0 / 6.0 if n % 2 == 0 else 1.0 / 12.0)
            else:
                x = (a - b) * h / 2.0
                s = (-1.0) ** (a - b)
                D[a, b] = -s / (2 * np.sin(x) ** 2) if n % 2 == 0 else \
                    -s * np.cos(x) / (2 * np.sin(x) ** 2)
    return D * (2.0 * np.pi / L) ** 2


def free_electron_levels(grid, box, count):
    """The `count` smallest values of |G|^2/2 over all integer triples of the box,
    with multiplicity (closed form of the V = 0 spectrum)."""
    vals = []
    rngs = [range(-(n // 2) + (1 if n % 2 == 0 else 0), n // 2 + 1) for n in grid]
    for m1 in rngs[0]:
        for m2 in rngs[1]:
            for m3 in rngs[2]:
                vals.append(2 * np.pi ** 2 * ((m1 / box[0]) ** 2 + (m2 / box[1]) ** 2 +
                                              (m3 / box[2]) ** 2))
    return np.sort(np.asarray(vals))[:count]


def kron_sum(A1, A2, A3):
    """Kronecker sum for x-fastest flattening (flat = i + n1*(j + n2*k))."""
    I1, I2, I3 = (np.eye(A.shape[0]) for A in (A1, A2, A3))
    return (np.kron(np.kron(I3, I2), A1) + np.kron(np.kron(I3, A2), I1) +
            np.kron(np.kron(A3, I2), I1))
