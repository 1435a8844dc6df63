"""Pins of the learned preconditioner's oracle: bfloat16 rounding, shells,
per-shell spectral sums, the correction target, the loss and its gradient,
Adam, and the reduction to the Teter preconditioner."""
import numpy as np
import pytest

from oracle import learned, teter, lobpcg
from oracle.hamiltonian import Operator
import synth


def test_bf16_rounding_ieee_cases():
    r = learned.round_bf16
    assert r(1.0) == 1.0
    assert r(1.0 + 2.0 ** -8) == 1.0                      # tie -> even (mantissa 0)
    assert r(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie -> even (mantissa 2)
    assert r(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7   # above the tie
    assert r(-1.5) == -1.5
    assert r(2.0 ** -130) == 2.0 ** -130                  # subnormal, exact in bf16
    x = np.random.default_rng(0).standard_normal(1000)
    y = r(x)
    assert np.all(np.abs(y - x) <= 2.0 ** -8 * np.abs(x) + 1e-45)


def _int_key_shells(grid, box_int):
    """Brute force with integers: box edges given as integers, shell key =
    sum_d m_d^2 * prod_{d' != d} L_{d'}^2 (proportional to |G|^2)."""
    keys = set()
    L = box_int
    rngs = [range(-(n // 2) + (1 if n % 2 == 0 else 0), n // 2 + 1) for n in grid]
    for m1 in rngs[0]:
        for m2 in rngs[1]:
            for m3 in rngs[2]:
                keys.add(m1 * m1 * L[1] ** 2 * L[2] ** 2 + m2 * m2 * L[0] ** 2 * L[2] ** 2 +
                         m3 * m3 * L[0] ** 2 * L[1] ** 2)
    return sorted(keys)


@pytest.mark.parametrize("grid,box", [((24, 24, 24), (10, 10, 10)), ((36, 36, 60), (15, 15, 25)),
                                      ((12, 10, 9), (5, 4, 3))])
def test_shells_match_integer_brute_force(grid, box):
    shell_of, t = learned.shells(grid, tuple(float(b) for b in box))
    keys = _int_key_shells(grid, box)
    assert t.shape[0] == len(keys)
    L2 = float(box[0] ** 2 * box[1] ** 2 * box[2] ** 2)
    expect = 2 * np.pi ** 2 * np.asarray(keys, dtype=np.float64) / L2
    assert np.allclose(t, expect, rtol=1e-13, atol=1e-14)
    assert np.all(np.diff(t) > 0)
    assert np.bincount(shell_of).sum() == np.prod(grid)
    assert np.all(np.bincount(shell_of) > 0)


def test_pair_sums_brute_force_dft():
    grid, box = (4, 3, 5), (2.0, 1.5, 2.5)
    n1, n2, n3 = grid
    ng = n1 * n2 * n3
    rng = np.random.default_rng(1)
    R = rng.standard_normal((ng, 3))
    E = rng.standard_normal((ng, 3))
    shell_of, t = learned.shells(grid, box)
    a, b, e2 = learned.pair_sums(R, E, grid, shell_of, t.shape[0])
    # explicit DFT: F[g, x] = exp(-2 pi i (m.x)) over flat indices, x fastest
    idx = np.arange(ng)
    i, j, k = idx % n1, (idx // n1) % n2, idx // (n1 * n2)
    ph = (np.outer(i, i) / n1 + np.outer(j, j) / n2 + np.outer(k, k) / n3)
    F = np.exp(-2j * np.pi * ph)
    a_bf = np.zeros_like(a)
    b_bf = np.zeros_like(b)
    for c in range(3):
        rh, eh = F @ R[:, c], F @ E[:, c]
        for g in range(ng):
            a_bf[c, shell_of[g]] += (np.conj(rh[g]) * eh[g]).real
            b_bf[c, shell_of[g]] += abs(rh[g]) ** 2
        assert abs(e2[c] - np.sum(np.abs(eh) ** 2)) < 1e-10 * e2[c]
    assert np.allclose(a, a_bf, atol=1e-10)
    assert np.allclose(b, b_bf, atol=1e-10)
    # Parseval
    assert np.allclose(a.sum(axis=1), ng * np.einsum("ij,ij->j", R, E))
    assert np.allclose(b.sum(axis=1), ng * np.einsum("ij,ij->j", R, R))


def test_correction_orthogonal_and_zero_at_convergence():
    rng = np.random.default_rng(2)
    ng, J = 200, 6
    Xs, _ = np.linalg.qr(rng.standard_normal((ng, J)))
    theta = np.array([-1.0, 0.5, 0.5, 0.5 + 1e-8, 2.0, 3.0])   # one 3-fold cluster
    X, _ = np.linalg.qr(Xs + 0.1 * rng.standard_normal((ng, J)))
    E = learned.correction(X, Xs, theta)
    assert np.abs(X.T @ E).max() < 1e-13
    # rotation inside the cluster and sign flips: already converged -> E = 0
    Q = np.eye(J)
    Q[1:4, 1:4], _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Q[0, 0] = -1.0
    E0 = learned.correction(Xs @ Q, Xs, theta)
    assert np.abs(E0).max() < 1e-13
    assert list(learned.clusters(theta)) == [0, 1, 1, 1, 2, 3]


def _samples(rng, grid, box, n=3):
    """Training samples from real vectors (so that the sums are consistent)."""
    ng = int(np.prod(grid))
    shell_of, t = learned.shells(grid, box)
    R = rng.standard_normal((ng, n))
    E = rng.standard_normal((ng, n))
    a, b, e2 = learned.pair_sums(R, E, grid, shell_of, t.shape[0])
    out = []
    for i in range(n):
        out.append(dict(t=t, a=a[i], b=b[i], e2=e2[i], theta=rng.uniform(-2, 1),
                        T=rng.uniform(0.3, 3.0), vbar=-0.4))
    return out


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    grid, box = (6, 5, 4), (3.0, 2.5, 2.0)
    smp = _samples(rng, grid, box)
    w = synth.mlp_init(seed=1, last_layer=0.3).astype(np.float64)
    w[learned._OFF["mu"][0]:learned._OFF["mu"][1]] = [0.5, -0.5, -0.4]
    w[learned._OFF["sd"][0]:learned._OFF["sd"][1]] = [2.0, 1.0, 0.1]
    w[learned._OFF["b1"][0]:learned._OFF["b1"][1]] = rng.uniform(-0.2, 0.2, 64)
    w[learned._OFF["b3"][0]] = 0.1
    L0, g = learned.loss_and_grad(w, smp, bf16=False)
    assert 0.0 < L0 < 1.0
    h = 1e-6
    idx = np.concatenate([rng.choice(learned.NW, 60, replace=False),
                          [learned.NW - 1, 0, 200, 4420]])
    for k in idx:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        # float64 evaluation (the FP32 cast of `effective` is bypassed)
        fd = (_loss64(wp, smp) - _loss64(wm, smp)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g).max()), (k, fd, g[k])


def _loss64(w, smp):
    orig = learned.effective
    learned.effective = lambda ww, bf16=True: np.asarray(ww, dtype=np.float64)
    try:
        return learned.loss_and_grad(w, smp, bf16=False)[0]
    finally:
        learned.effective = orig


def test_loss_zero_for_ideal_factor_and_scale_invariant():
    rng = np.random.default_rng(4)
    grid, box = (6, 6, 6), (3.0, 3.0, 3.0)
    n1, n2, n3 = grid
    ng = 216
    shell_of, t = learned.shells(grid, box)
    w = synth.mlp_init(seed=2, last_layer=0.5).astype(np.float64)
    T, theta, vbar = 0.8, -0.3, -0.2
    f, _ = learned.forward(w, learned.features(t, T, theta, vbar)[0])
    K = teter.teter_k(t / T) * np.exp(f)
    r = rng.standard_normal(ng)
    Kg = K[shell_of].reshape(n3, n2, n1)
    e = np.fft.ifftn(Kg * np.fft.fftn(r.reshape(n3, n2, n1))).real.ravel() * 3.7
    a, b, e2 = learned.pair_sums(r[:, None], e[:, None], grid, shell_of, t.shape[0])
    smp = [dict(t=t, a=a[0], b=b[0], e2=e2[0], theta=theta, T=T, vbar=vbar)]
    L, _ = learned.loss_and_grad(w, smp)
    assert abs(L) < 1e-12
    # a constant factor on K leaves the loss unchanged
    smp2 = _samples(rng, grid, box, 2)[0]
    Kr = rng.uniform(0.1, 2.0, t.shape[0])
    l1 = learned.sample_loss(Kr, smp2["a"], smp2["b"], smp2["e2"])
    l2 = learned.sample_loss(3.7 * Kr, smp2["a"], smp2["b"], smp2["e2"])
    assert 0.0 <= l1 <= 1.0 and abs(l1 - l2) < 1e-12
    # the network's factor stays within exp(+-FMAX) of Teter's
    wbig = w.copy()
    wbig[learned._OFF["b3"][0]] = 50.0
    fb, _ = learned.forward(wbig, learned.features(t, T, theta, vbar)[0])
    assert np.all(np.abs(fb) <= learned.FMAX)


def test_adam_first_step_is_signed_lr():
    w = np.zeros(learned.NTOT)
    g = np.random.default_rng(5).standard_normal(learned.NW)
    w1, m, v = learned.adam_step(w, g, np.zeros(learned.NW), np.zeros(learned.NW), 1, lr=1e-3)
    assert np.allclose(w1[:learned.NW], -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.all(w1[learned.NW:] == 0)


def test_zero_output_layer_is_teter():
    el = synth.single_element(seed=3, grid=(12, 12, 12), n_states=6, n_atoms=3)
    op = Operator(el.grid, el.box, el.V, el.kb)
    rng = np.random.default_rng(6)
    X, _ = np.linalg.qr(rng.standard_normal((op.ng, 6)))
    R = rng.standard_normal((op.ng, 6))
    w = synth.mlp_init(seed=4, last_layer=0.0)
    shell_of, t = learned.shells(el.grid, el.box)
    T = np.maximum(teter.band_kinetic(X, el.grid, el.box), teter.kinetic_floor(el.box))
    g = learned.gain_table(w, t, T, np.zeros(6), 0.0)
    assert np.all(g == 1.0)
    W1 = learned.precondition(R, X, el.grid, el.box, g, shell_of)
    W0 = teter.precondition(R, X, el.grid, el.box)
    assert np.abs(W1 - W0).max() < 1e-14
    # the whole LOBPCG with the learned callable and a zero output layer
    pre = learned.LearnedPreconditioner(w, op, float(el.V.mean()))
    r1 = lobpcg.lobpcg(op.apply, pre, el.X0, 1e-8, 200)
    r0 = lobpcg.lobpcg(op.apply, lambda R_, X_: teter.precondition(R_, X_, op.grid, op.box),
                       el.X0, 1e-8, 200)
    assert r1.iters == r0.iters
    assert np.abs(r1.theta - r0.theta).max() < 1e-12


def test_stall_rule_flags_bands():
    class Op:
        grid, box = (4, 4, 4), (2.0, 2.0, 2.0)

        def apply(self, X):
            return X
    pre = learned.LearnedPreconditioner(synth.mlp_init(0), Op(), 0.0)
    X = np.linalg.qr(np.random.default_rng(7).standard_normal((64, 2)))[0]
    seq = [(1.0, 1.0), (0.5, 0.99), (0.2, 0.98), (0.1, 0.97), (0.05, 0.89)]
    for k, (ra, rb) in enumerate(seq):
        R = np.zeros((64, 2))
        R[0, 0], R[1, 1] = ra, rb
        pre(R, X)
        if k < 3:
            assert not pre.fallback.any()
    # band 1: 0.97 > 0.9 * 1.0 at k = 3 -> fallback, kept afterwards
    assert list(pre.fallback) == [False, True]


def test_normalisation_hand_computed_rows():
    """Four (band, shell) rows written out by hand: band 1 has T = 2 and shells
    t = 2, 2e, 2e^2 (x = 1, e, e^2, so log x = 0, 1, 2) with theta = 0.5; band
    2 has T = 1 and one shell t = 1e-4 (x below the 1e-3 floor, so
    log x = log 1e-3) with theta = 2.5; Vbar = -1 everywhere.  Population mean
    and standard deviation per column from the standard library; the constant
    Vbar column gets sd = 1."""
    import math
    import statistics
    e = math.e
    samples = [dict(t=np.array([2.0, 2.0 * e, 2.0 * e * e]), T=2.0, theta=0.5, vbar=-1.0),
               dict(t=np.array([1e-4]), T=1.0, theta=2.5, vbar=-1.0)]
    mu, sd = learned.normalisation(samples)
    c0 = [0.0, 1.0, 2.0, math.log(1e-3)]
    c1 = [0.5, 0.5, 0.5, 2.5]
    assert abs(mu[0] - statistics.fmean(c0)) < 1e-14
    assert abs(sd[0] - statistics.pstdev(c0)) < 1e-14
    assert abs(mu[1] - 1.0) < 1e-15 and abs(sd[1] - math.sqrt(3.0) / 2.0) < 1e-15
    assert mu[2] == -1.0 and sd[2] == 1.0
