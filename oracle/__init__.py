"""Plain FP64 CPU oracle for DGDFT's adaptive-local-basis (ALB) generation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP path (no kernels, headers, helpers, tables or pre/post-processing); the
only thing both sides see is the seeded input from ``synth``.

What it computes (Hu, Lin, Yang, "DGDFT: a massively parallel method for
large scale density functional theory calculations", Sec. II.A):

* the local Kohn-Sham operator of one extended element Q_K (Eq. localproblem)
  discretised by planewaves on the periodic box of Q_K, with the nonlocal
  pseudopotential in Kleinman-Bylander form (the gamma*|<b,psi>|^2 term of
  Eq. DGvar) -- ``hamiltonian``;
* its lowest J_K eigenpairs, by dense diagonalisation (definition) and by
  Teter-preconditioned LOBPCG (the method of Sec. II.B, "Generation of the
  ALB functions") -- ``dense``, ``teter``, ``lobpcg``;
* restriction of the eigenvectors from Q_K to the element E_K followed by
  orthonormalisation, done as an SVD truncation -- ``alb``;
* a learned refinement of the Teter preconditioner (not in the paper): the
  network, its training loss and gradient, Adam, the per-shell spectral sums
  of residual/correction pairs and the Teter fallback -- ``learned``;
* element-local DG quantities from the ALBs: the density from diagonal
  density-matrix blocks (Eq. newdensity), the Kleinman-Bylander block of
  Eq. DGHamiltonian and its volume terms (kinetic and V_eff) by Gauss-Lobatto
  quadrature with differentiation matrices (Sec. III, construction of the DG
  Hamiltonian) -- ``dgblocks``.

Pins: every function is checked in ``tests/test_oracle_*.py`` against closed
forms, textbook special cases, independent libraries or brute force.  The
results with no such pin are the LOBPCG iteration count, which depends on
the path taken, and what a trained network gains over Teter's factor:
**parity unpinned** (iteration counts are only compared between runs with
identical settings).
"""
from . import hamiltonian, dense, teter, lobpcg, alb, solve, learned, dgblocks, random_start  # noqa: F401
