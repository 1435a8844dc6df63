"""Learned diagonal preconditioner and its training objective (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not in the paper.  The paper applies the Teter preconditioner (Sec. II.B,
citing Payne, Teter, Allan et al.) column by column; this module defines a
learned refinement of it and the data it is trained on:

* Shells.  The Teter factor K(x), x = (|G|^2/2) / T_i, depends on G only
  through |G|^2, so a refinement that keeps that property is a table over the
  distinct values of |G|^2 on the FFT box ("shells").  Shell s has kinetic
  energy t_s; shells are ascending and equal values (up to 1e-12 relative)
  are one shell.
* Model.  K_i(G) = K_Teter(t / T_i) * exp(f(u)), f = FMAX tanh(z(u) / FMAX),
  where z is a multilayer perceptron 3 -> 64 -> 64 -> 1 with SiLU activations
  and u = ((log max(x, XMIN), theta_i, Vbar) - mu) / sd: the Teter ratio x of
  the shell, the Ritz value theta_i of the band and the mean local potential
  of the element, standardised with constants mu, sd fixed before training.
  The bound keeps the learned factor within exp(+-FMAX) of Teter's, so the
  preconditioned residuals cannot collapse onto a few shells.  With the last
  layer zero, f = 0 and the preconditioner is exactly Teter's.  The
  weights are kept in FP32 and rounded to bfloat16 (round to nearest, ties to
  even) for every evaluation; gradients are taken with respect to the rounded
  values and applied to the FP32 copy.
* Target.  For band i at some iteration with unit Ritz vectors X and residual
  r_i, the ideal correction is e_i = (I - X X^T) x~_i, where x~_i is x_i
  projected on the converged eigenvectors of its cluster (eigenvalues of the
  converged solve within CLUSTER_TOL of each other), which fixes the sign and
  the rotation inside degenerate clusters.  LOBPCG only uses the span of the
  preconditioned residuals, so the loss of one sample is scale invariant:
  L_i = 1 - cos^2(K_i o r^_i, e^_i) over the spectrum.  Because K_i is
  constant on a shell, it only needs the per-shell sums
  a_s = sum_{G in s} Re(conj(r^(G)) e^(G)) and b_s = sum_{G in s} |r^(G)|^2
  and e2 = sum_G |e^(G)|^2 (unnormalised DFT):
  L_i = 1 - (sum_s K_s a_s)^2 / ((sum_s K_s^2 b_s) e2).
* Training uses Adam (Kingma and Ba, 2015) on the mean loss of a minibatch.
* Teter fallback: a band whose residual has not fallen below 0.9 times its
  value three iterations earlier uses the Teter factor for the rest of the
  solve.

Parameter vector (NTOT values, FP32 at the C ABI):
  W1 [64][3] (row = hidden unit), b1 [64], W2 [64][64] (row = output unit),
  b2 [64], w3 [64], b3, then mu [3] and sd [3] (not trained).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .hamiltonian import FFT_WORKERS, kinetic_diagonal
from .teter import band_kinetic, kinetic_floor, teter_k

H = 64
NW = 3 * H + H + H * H + H + H + 1          # 4481 trained parameters
NTOT = NW + 6                                # + mu[3], sd[3]
XMIN = 1e-3
FMAX = 2.0
CLUSTER_TOL = 1e-6
STALL_FACTOR = 0.9
STALL_LAG = 3

_OFF = {}
_o = 0
for _name, _size in (("W1", 3 * H), ("b1", H), ("W2", H * H), ("b2", H), ("w3", H), ("b3", 1),
                     ("mu", 3), ("sd", 3)):
    _OFF[_name] = (_o, _o + _size)
    _o += _size
assert _o == NTOT


def part(w, name):
    a, b = _OFF[name]
    return w[a:b]


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    The input is first taken to FP32; bfloat16 keeps the top 16 bits of the
    FP32 encoding (8 exponent bits, 7 stored mantissa bits)."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (a >> np.uint64(16)) & np.uint64(1)
    r = ((a + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- shells
def shells(grid, box):
    """(shell_of, t_shell): shell index of every grid frequency (flat, x
    fastest) and the ascending distinct values of |G|^2/2."""
    t = kinetic_diagonal(grid, box).ravel()
    order = np.argsort(t, kind="stable")
    ts = t[order]
    new = np.empty(ts.shape, dtype=bool)
    new[0] = True
    new[1:] = (ts[1:] - ts[:-1]) > 1e-12 * np.maximum(1.0, ts[1:])
    sid = np.cumsum(new) - 1
    shell_of = np.empty_like(sid)
    shell_of[order] = sid
    return shell_of.astype(np.int64), ts[new]


# ---------------------------------------------------------------- pairs
def clusters(theta, tol=CLUSTER_TOL):
    """Cluster id of each (ascending) eigenvalue: consecutive values closer
    than tol share a cluster."""
    theta = np.asarray(theta)
    c = np.zeros(theta.shape[0], dtype=np.int64)
    for i in range(1, theta.shape[0]):
        c[i] = c[i - 1] + (1 if theta[i] - theta[i - 1] > tol else 0)
    return c


def correction(X, Xstar, theta_star, tol=CLUSTER_TOL):
    """E (N_g x J): column i is (I - X X^T) x~_i with x~_i the projection of
    x_i on the converged eigenvectors of its cluster."""
    c = clusters(theta_star, tol)
    G = Xstar.T @ X                                   # G[j, i] = x*_j . x_i
    G = np.where(c[:, None] == c[None, :], G, 0.0)
    Xt = Xstar @ G
    return Xt - X @ (X.T @ Xt)


def pair_sums(R, E, grid, shell_of, nsh):
    """Per column i: a[i, s], b[i, s] (shell sums over the unnormalised DFT)
    and e2[i]."""
    n1, n2, n3 = grid
    m = R.shape[1]
    Rh = sfft.fftn(R.T.reshape(m, n3, n2, n1), axes=(1, 2, 3), workers=FFT_WORKERS).reshape(m, -1)
    Eh = sfft.fftn(E.T.reshape(m, n3, n2, n1), axes=(1, 2, 3), workers=FFT_WORKERS).reshape(m, -1)
    a = np.zeros((m, nsh))
    b = np.zeros((m, nsh))
    for i in range(m):
        a[i] = np.bincount(shell_of, weights=(np.conj(Rh[i]) * Eh[i]).real, minlength=nsh)
        b[i] = np.bincount(shell_of, weights=np.abs(Rh[i]) ** 2, minlength=nsh)
    e2 = np.sum(np.abs(Eh) ** 2, axis=1)
    return a, b, e2


# ---------------------------------------------------------------- model
def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def features(t_shell, T, theta, vbar):
    """Raw inputs (log x, theta, Vbar) of every (band, shell): (J, nsh, 3)."""
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    x = np.asarray(t_shell)[None, :] / T[:, None]
    F = np.empty(x.shape + (3,))
    F[..., 0] = np.log(np.maximum(x, XMIN))
    F[..., 1] = theta[:, None]
    F[..., 2] = vbar
    return F


def effective(w, bf16=True):
    """Parameters as evaluated: trained ones rounded to bfloat16, mu/sd FP32."""
    w = np.asarray(w, dtype=np.float64)
    out = np.array(np.asarray(w, dtype=np.float32), dtype=np.float64)
    if bf16:
        out[:NW] = round_bf16(w[:NW])
    return out


def forward(w, F, bf16=True):
    """f for raw features F (..., 3); returns f and the activations."""
    p = effective(w, bf16)
    W1 = part(p, "W1").reshape(H, 3)
    W2 = part(p, "W2").reshape(H, H)
    U = (F - part(p, "mu")) / part(p, "sd")
    Z1 = U @ W1.T + part(p, "b1")
    H1 = silu(Z1)
    Z2 = H1 @ W2.T + part(p, "b2")
    H2 = silu(Z2)
    z = H2 @ part(p, "w3") + part(p, "b3")[0]
    f = FMAX * np.tanh(z / FMAX)
    return f, (p, U, Z1, H1, Z2, H2, z)


def gain_table(w, t_shell, T, theta, vbar, fallback=None, bf16=True):
    """exp(f) for every (band, shell); bands flagged in `fallback` get 1."""
    f, _ = forward(w, features(t_shell, T, theta, vbar), bf16)
    g = np.exp(f)
    if fallback is not None:
        g[np.asarray(fallback, dtype=bool)] = 1.0
    return g


def sample_loss(K, a, b, e2):
    s1 = np.sum(K * a)
    s2 = np.sum(K * K * b)
    return 1.0 - s1 * s1 / (s2 * e2)


def loss_and_grad(w, samples, bf16=True):
    """Mean loss over samples and its gradient with respect to the NW trained
    parameters.  A sample is a dict with t (nsh), a (nsh), b (nsh), theta, T,
    vbar, e2."""
    grad = np.zeros(NW)
    total = 0.0
    n = len(samples)
    for smp in samples:
        F = features(smp["t"], smp["T"], smp["theta"], smp["vbar"])[0]
        f, (p, U, Z1, H1, Z2, H2, z) = forward(w, F, bf16)
        x = np.asarray(smp["t"]) / smp["T"]
        K = teter_k(x) * np.exp(f)
        a, b, e2 = np.asarray(smp["a"]), np.asarray(smp["b"]), smp["e2"]
        s1 = np.sum(K * a)
        s2 = np.sum(K * K * b)
        total += 1.0 - s1 * s1 / (s2 * e2)
        dK = (-2.0 * s1 / (s2 * e2)) * a + (s1 * s1 / (s2 * s2 * e2)) * 2.0 * K * b
        df = dK * K / n * (1.0 - np.tanh(z / FMAX) ** 2)     # with respect to z
        W2 = part(p, "W2").reshape(H, H)
        w3 = part(p, "w3")
        g_w3 = H2.T @ df
        g_b3 = np.sum(df)
        dZ2 = (df[:, None] * w3[None, :]) * dsilu(Z2)
        g_W2 = dZ2.T @ H1
        g_b2 = dZ2.sum(axis=0)
        dZ1 = (dZ2 @ W2) * dsilu(Z1)
        g_W1 = dZ1.T @ U
        g_b1 = dZ1.sum(axis=0)
        grad += np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return total / n, grad


def adam_step(w, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on the trained parameters (t counts from 1)."""
    w = np.array(w, dtype=np.float64)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    w[:NW] = w[:NW] - lr * mh / (np.sqrt(vh) + eps)
    return w, m, v


def normalisation(samples):
    """mu, sd of the raw features over every (sample, shell) row (population
    standard deviation; 1 where it is below 1e-6 of the root mean square)."""
    rows = np.concatenate([features(s["t"], s["T"], s["theta"], s["vbar"])[0] for s in samples])
    mu = rows.mean(axis=0)
    sd = rows.std(axis=0)
    # an input that is constant over the data (up to rounding) is left unscaled
    rms = np.sqrt(np.mean(rows * rows, axis=0))
    sd = np.where(sd > 1e-6 * rms, sd, 1.0)
    return mu, sd


# ---------------------------------------------------------------- preconditioner
def precondition(R, X, grid, box, gain, shell_of):
    """W_i = F^-1 (K_Teter(t / T_i) * gain[i, shell(G)]) F R_i."""
    n1, n2, n3 = grid
    m = R.shape[1]
    t = kinetic_diagonal(grid, box)
    T = np.maximum(band_kinetic(X, grid, box), kinetic_floor(box))
    K = teter_k(t[None] / T[:, None, None, None])
    K = K * np.asarray(gain)[:, shell_of].reshape(m, n3, n2, n1)
    Rh = sfft.fftn(R.T.reshape(m, n3, n2, n1), axes=(1, 2, 3), workers=FFT_WORKERS)
    W = sfft.ifftn(K * Rh, axes=(1, 2, 3), workers=FFT_WORKERS).real
    return np.asfortranarray(W.reshape(m, n1 * n2 * n3).T)


class LearnedPreconditioner:
    """Callable (R, X) -> W for the oracle's LOBPCG: learned factor with the
    Teter fallback for stalled bands.  Ritz values are recomputed from X as
    diag(X^T H X) through `apply_h`."""

    def __init__(self, w, op, vbar):
        self.w = w
        self.op = op
        self.vbar = vbar
        self.shell_of, self.t_shell = shells(op.grid, op.box)
        self.hist = []
        self.fallback = None

    def __call__(self, R, X):
        r = np.linalg.norm(R, axis=0)
        if self.fallback is None:
            self.fallback = np.zeros(r.shape[0], dtype=bool)
        self.hist.append(r)
        if len(self.hist) > STALL_LAG:
            self.fallback |= r > STALL_FACTOR * self.hist[-1 - STALL_LAG]
        theta = np.einsum("ij,ij->j", X, self.op.apply(X))
        T = np.maximum(band_kinetic(X, self.op.grid, self.op.box), kinetic_floor(self.op.box))
        g = gain_table(self.w, self.t_shell, T, theta, self.vbar, self.fallback)
        return precondition(R, X, self.op.grid, self.op.box, g, self.shell_of)
