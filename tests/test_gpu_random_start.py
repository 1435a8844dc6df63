"""The start block the library draws when it is given none (X0 = NULL):
against the oracle's own implementation of the same counter-based generator
(Philox4x32-10 + Box-Muller, written separately from its published
definition), and a solve from it against the oracle's solve from its copy."""
import numpy as np
import pytest

import synth
from oracle import random_start as rs
from oracle.solve import solve_element

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def test_start_block_matches_oracle_generator(dev):
    """Three elements, one with an odd N_g (15 x 9 x 5), seed above 2^32 so
    both key words are used; the uniforms are exact on both sides, the
    deviates agree to the last bits of log, sqrt, cos and sin."""
    from paper_1506_08147_amd import ALB
    grids = [(12, 12, 12), (15, 9, 5), (10, 8, 6)]
    J = [7, 4, 9]
    h = ALB(grids, [tuple(0.4 * n for n in g) for g in grids], J)
    seed = (3 << 32) + 12345
    X0 = h.initial_guess(seed, dev).cpu().numpy()
    off = 0
    for e, (g, j) in enumerate(zip(grids, J)):
        ng = int(np.prod(g))
        got = X0[off:off + ng * j].reshape(j, ng).T
        ref = rs.start_block(ng, j, e, seed)
        print(f"element {e}: max |dx| {np.abs(got - ref).max():.2e}", flush=True)
        assert np.abs(got - ref).max() < 1e-13
        off += ng * j
    assert off == X0.size
    h.close()


def test_solve_without_initial_guess_matches_oracle(dev):
    import torch
    from paper_1506_08147_amd import ALB
    el = synth.single_element(seed=2, grid=(12, 12, 12), n_states=10, n_atoms=3)
    seed = 777
    h = ALB([el.grid], [el.box], [el.n_states], tol=1e-9, max_iter=500, elem_lo=[el.elem_lo],
            elem_hi=[el.elem_hi], n_alb=[el.n_alb], seed=seed)
    V = torch.from_numpy(el.V).to(dev)
    out = h.solve(V, ALB.kb_batch([el.kb], dev), None, device=dev)
    st = out["stats"][0]
    ref = solve_element(el, tol=1e-9, X0=rs.start_block(el.ng, el.n_states, 0, seed))
    ev = out["eigvals"].cpu().numpy()
    print("iters gpu", st["iters"], "oracle", ref["iters"], "phases", st["ms_by_phase"], flush=True)
    assert st["converged"] and ref["converged"]
    assert np.abs(ev - ref["eigvals"]).max() < 1e-10
    assert abs(st["iters"] - ref["iters"]) <= 2
    assert all(v >= 0.0 for v in st["ms_by_phase"].values())
    assert st["ms_by_phase"]["iterations"] > 0.0
    h.close()
