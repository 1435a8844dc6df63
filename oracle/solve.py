"""One element end to end: LOBPCG on the local problem, then the ALBs.

Outputs follow the normalisation of Eq. localproblem (integral over Q_K of
psi_j psi_j' = delta, i.e. dV sum psi^2 = 1) for the eigenvectors and of
Eq. orthonormal for the ALBs (dV sum over E_K of phi^2 = 1).
"""
from __future__ import annotations

import numpy as np

from . import alb, lobpcg as lob, teter
from .hamiltonian import Operator


def solve_element(el, tol=1e-8, max_iter=500, X0=None):
    op = Operator(el.grid, el.box, el.V, el.kb)
    pre = lambda R, X: teter.precondition(R, X, op.grid, op.box)  # noqa: E731
    res = lob.lobpcg(op.apply, pre, el.X0 if X0 is None else X0, tol, max_iter)
    albs, sigma = alb.restrict_svd(res.X, op.grid, el.elem_lo, el.elem_hi, op.dv, el.n_alb)
    return {
        "eigvals": res.theta,
        "eigvecs": res.X / np.sqrt(op.dv),
        "X": res.X,
        "albs": albs,
        "sigma": sigma,
        "resid": res.resid,
        "iters": res.iters,
        "converged": res.converged,
        "history": res.history,
        "result": res,
        "op": op,
    }
