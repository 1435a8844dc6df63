"""Element-local DG quantities on the GPU against the oracle (through the C
ABI): density from diagonal density-matrix blocks and the nonlocal block."""
import numpy as np
import pytest

import synth
from oracle import dgblocks

pytestmark = pytest.mark.gpu


def test_density_and_nonlocal_block_match_oracle():
    import torch
    from paper_1506_08147_amd import ALB
    dev = torch.device("cuda:0")
    els = [synth.single_element(seed=s, grid=g, n_states=J, n_atoms=4)
           for s, g, J in [(31, (16, 16, 16), 10), (32, (18, 16, 20), 12)]]
    h = ALB([e.grid for e in els], [e.box for e in els], [e.n_states for e in els], tol=1e-8,
            elem_lo=[e.elem_lo for e in els], elem_hi=[e.elem_hi for e in els],
            n_alb=[e.n_alb for e in els])
    V = torch.cat([torch.from_numpy(e.V) for e in els]).to(dev)
    X0 = torch.cat([torch.from_numpy(np.ascontiguousarray(e.X0.T)).reshape(-1) for e in els]).to(dev)
    out = h.solve(V, ALB.kb_batch([e.kb for e in els], dev), X0)
    assert out["status"] == 0
    rng = np.random.default_rng(0)
    Ps = []
    for e in els:
        A = rng.standard_normal((e.n_alb, e.n_alb))
        Ps.append(A @ A.T / e.n_alb)
    Pt = torch.cat([torch.from_numpy(np.asfortranarray(P).ravel(order="F")) for P in Ps]).to(dev)
    rho = h.density(out["albs"], Pt).cpu().numpy()
    Hnl = h.nonlocal_block(out["albs"]).cpu().numpy()
    oa = on = 0
    for i, e in enumerate(els):
        phi = h.split(out, i)["albs"].cpu().numpy()
        ne, n = phi.shape
        ref = dgblocks.density(phi, Ps[i])
        assert np.abs(rho[oa:oa + ne] - ref).max() < 1e-12 * np.abs(ref).max()
        # electron count: dV sum rho = tr(P) for orthonormal ALBs
        assert abs(e.dv * rho[oa:oa + ne].sum() - np.trace(Ps[i])) < 1e-9 * np.trace(Ps[i])
        Hr = dgblocks.nonlocal_block(phi, e.kb, e.grid, e.elem_lo, e.elem_hi, e.dv)
        Hg = Hnl[on:on + n * n].reshape(n, n, order="F")
        assert np.abs(Hg - Hr).max() < 1e-12 * max(np.abs(Hr).max(), 1e-300)
        oa += ne
        on += n * n
    h.close()
