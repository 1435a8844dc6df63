"""GPU LOBPCG + ALB parity against the oracle (through the C ABI)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle.solve import solve_element

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "one_element_dense.json")


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _solve(els, dev, tol, max_iter=500, X0s=None, expect_ok=True):
    import torch
    from paper_1506_08147_amd import ALB
    h = ALB([e.grid for e in els], [e.box for e in els], [e.n_states for e in els], tol=tol,
            max_iter=max_iter, elem_lo=[e.elem_lo for e in els], elem_hi=[e.elem_hi for e in els],
            n_alb=[e.n_alb for e in els])
    V = torch.cat([torch.from_numpy(e.V) for e in els]).to(dev)
    X0s = X0s if X0s is not None else [e.X0 for e in els]
    X0 = torch.cat([torch.from_numpy(np.ascontiguousarray(x.T)).reshape(-1) for x in X0s]).to(dev)
    out = h.solve(V, ALB.kb_batch([e.kb for e in els], dev), X0)
    res = [h.split(out, i) for i in range(len(els))]
    res = [{k: v.cpu().numpy() for k, v in r.items()} for r in res]
    stats = out["stats"]
    h.close()
    return res, stats, out["status"]


def _span_err(A, B):
    """sin of the largest principal angle between the column spans of A, B
    (orthonormal in the same inner product)."""
    s = np.linalg.svd(A.T @ B, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))


def test_small_element_matches_oracle(dev):
    el = synth.single_element(seed=2, grid=(12, 12, 12), n_states=10, n_atoms=3)
    (r,), (st,), status = _solve([el], dev, 1e-9)
    ref = solve_element(el, tol=1e-9)
    print("iters gpu", st["iters"], "oracle", ref["iters"])
    assert status == 0 and st["converged"]
    assert np.abs(r["eigvals"] - ref["eigvals"]).max() < 1e-10
    dv = el.dv
    psi = r["eigvecs"]
    assert np.abs(dv * psi.T @ psi - np.eye(10)).max() < 1e-12
    assert abs(st["iters"] - ref["iters"]) <= 2


def test_one_element_workload_vs_dense_and_oracle(dev):
    """24^3, 32 states, 8 wells: dense LAPACK eigenvalues (stored) and the oracle."""
    gold = json.load(open(GOLDEN))
    el = synth.single_element(seed=0)
    (r,), (st,), status = _solve([el], dev, 1e-8)
    w = np.asarray(gold["seeds"]["0"])
    assert st["converged"]
    assert np.abs(r["eigvals"] - w[:32]).max() < 1e-10
    ref = solve_element(el, tol=1e-8)
    print("iters gpu", st["iters"], "oracle", ref["iters"])
    assert abs(st["iters"] - ref["iters"]) <= 3
    # eigenvectors: span of the lowest 32 (gap w[32]-w[31] checked by the golden)
    dv = el.dv
    X = r["eigvecs"] * np.sqrt(dv)
    assert _span_err(X, ref["X"]) < 1e-6
    # ALBs: singular values and span against the oracle's SVD truncation
    assert np.abs(r["sigma"] - ref["sigma"]).max() < 1e-8
    A = r["albs"] * np.sqrt(dv)
    B = ref["albs"] * np.sqrt(dv)
    assert np.abs(A.T @ A - np.eye(el.n_alb)).max() < 1e-11
    assert _span_err(A, B) < 1e-6


def test_batch_equals_single_solves(dev):
    els = [synth.single_element(seed=s, grid=g, n_states=J, n_atoms=3)
           for s, g, J in [(11, (12, 12, 12), 6), (12, (16, 12, 20), 9), (13, (10, 15, 12), 5)]]
    rb, sb, _ = _solve(els, dev, 1e-9)
    for i, el in enumerate(els):
        (r1,), (s1,), _ = _solve([el], dev, 1e-9)
        assert np.array_equal(rb[i]["eigvals"], r1["eigvals"])
        assert sb[i]["iters"] == s1["iters"]
        ref = solve_element(el, tol=1e-9)
        assert np.abs(rb[i]["eigvals"] - ref["eigvals"]).max() < 1e-10


def test_iteration_cap_reports_not_converged(dev):
    el = synth.single_element(seed=0, grid=(12, 12, 12), n_states=6, n_atoms=2)
    (r,), (st,), status = _solve([el], dev, 1e-10, max_iter=2)
    assert status == 1 and not st["converged"] and st["iters"] == 2


def test_rank_deficient_initial_guess(dev):
    from paper_1506_08147_amd import DGDFTError
    el = synth.single_element(seed=0, grid=(12, 12, 12), n_states=6, n_atoms=2)
    X0 = el.X0.copy()
    X0[:, 3] = X0[:, 1]
    with pytest.raises(DGDFTError) as ei:
        _solve([el], dev, 1e-8, X0s=[X0])
    assert ei.value.code == -5


def test_nonfinite_potential_rejected(dev):
    from paper_1506_08147_amd import DGDFTError
    el = synth.single_element(seed=0, grid=(12, 12, 12), n_states=6, n_atoms=2)
    el.V = el.V.copy()
    el.V[17] = np.nan
    with pytest.raises(DGDFTError) as ei:
        _solve([el], dev, 1e-8)
    assert ei.value.code == -1


def test_projector_change_rebuilds_the_layout(dev):
    """One handle solving two elements of the same grid in turn (different
    atoms, so different projectors and potential), then the first again: each
    solve equals a fresh handle's solve bit for bit (the projector layout is
    kept only while the arrays are bitwise unchanged)."""
    import torch
    from paper_1506_08147_amd import ALB
    a = synth.single_element(seed=5, grid=(12, 12, 12), n_states=6, n_atoms=3)
    b = synth.single_element(seed=6, grid=(12, 12, 12), n_states=6, n_atoms=2)

    def handle():
        return ALB([a.grid], [a.box], [a.n_states], tol=1e-9, elem_lo=[a.elem_lo],
                   elem_hi=[a.elem_hi], n_alb=[a.n_alb])

    def inputs(el):
        return (torch.from_numpy(el.V).to(dev), ALB.kb_batch([el.kb], dev),
                torch.from_numpy(np.ascontiguousarray(a.X0.T)).reshape(-1).to(dev))

    h = handle()
    runs = [h.solve(*inputs(el))["eigvals"].cpu().numpy() for el in (a, b, a)]
    h.close()
    for el, got in zip((a, b, a), runs):
        f = handle()
        ref = f.solve(*inputs(el))["eigvals"].cpu().numpy()
        f.close()
        assert np.array_equal(got, ref)
    assert not np.allclose(runs[0], runs[1])
