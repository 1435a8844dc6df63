"""Seeded synthetic inputs for the ALB-generation step (local problem on an
extended element).

The paper treats the restricted effective potential V_eff^Q and the
Kleinman-Bylander projectors b_{I,l}, gamma_{I,l} of an extended element as
given inputs of the local eigenproblem (Sec. II.A, Eq. localproblem, and the
KB form inside Eq. DGvar).  This module only *produces* such inputs: Gaussian
wells for V, Gaussian s/p projectors for the KB term, seeded random initial
guesses and element boxes.  It contains none of the method's arithmetic (no
operator, no FFT, no eigensolver) and is the only code shared between the CPU
oracle and the GPU path, and only as input.

Units: Hartree atomic units (bohr, Ha).  Grids are flattened x-fastest,
flat = i + n1*(j + n2*k).  Block matrices are column-major (Fortran order).
"""
from __future__ import annotations

import dataclasses
from concurrent.futures import ThreadPoolExecutor

import numpy as np

H_SPACING = 10.0 / 24.0  # grid spacing of every workload (bohr)


@dataclasses.dataclass
class KB:
    """Kleinman-Bylander projectors of one element in CSR-by-projector form.

    gamma[p]            coupling constant of projector p (Ha)
    ptr[p]:ptr[p+1]     range of projector p in idx/val
    idx[k]              flat grid index (int32, ascending within a projector)
    val[k]              b_p sampled on the grid, continuum-normalised so that
                        dV * sum_k val[k]**2 == 1 (units bohr^-3/2)
    """
    gamma: np.ndarray
    ptr: np.ndarray
    idx: np.ndarray
    val: np.ndarray

    @property
    def n_proj(self) -> int:
        return int(self.gamma.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.idx.shape[0])


@dataclasses.dataclass
class Element:
    grid: tuple          # (n1, n2, n3)
    box: tuple           # (L1, L2, L3) bohr
    V: np.ndarray        # (Ng,) Ha, flat x-fastest
    kb: KB
    X0: np.ndarray       # (Ng, J) Fortran order, N(0,1)
    n_states: int
    elem_lo: tuple       # restriction box, half-open, grid indices
    elem_hi: tuple
    n_alb: int
    atoms: np.ndarray    # (n_atoms, 5): x, y, z, depth, width

    @property
    def ng(self) -> int:
        return int(np.prod(self.grid))

    @property
    def dv(self) -> float:
        return float(np.prod(self.box)) / self.ng


def _axis_offsets(n, L, a):
    """Minimum-image signed offsets x_i - a along one periodic axis."""
    d = np.arange(n) * (L / n) - a
    return d - L * np.round(d / L)


def gaussian_wells(grid, box, atoms):
    """V(r) = -sum_a D_a sum_{27 periodic images} exp(-|r-R_a-nL|^2 / (2 w_a^2)).

    The Gaussian factorises over the axes, so the 27-image sum is the product
    of three 1D sums over images n_d in {-1, 0, 1}."""
    n1, n2, n3 = grid
    V = np.zeros((n3, n2, n1))
    for (ax, ay, az, depth, width) in atoms:
        fac = []
        for n, L, a in ((n1, box[0], ax), (n2, box[1], ay), (n3, box[2], az)):
            x = np.arange(n) * (L / n) - a
            fac.append(sum(np.exp(-((x - s * L) ** 2) / (2.0 * width * width))
                           for s in (-1, 0, 1)))
        V -= depth * fac[2][:, None, None] * fac[1][None, :, None] * fac[0][None, None, :]
    return V.reshape(-1)


def gaussian_kb(grid, box, atoms, gammas, rcut_factor=4.0):
    """Four projectors per atom (s, p_x, p_y, p_z), Gaussian of the well width,
    support cut at r_c = rcut_factor*w (minimum-image distance), each normalised
    to dV*sum b^2 = 1.  All four share one support (sorted flat indices)."""
    n1, n2, n3 = grid
    dv = float(np.prod(box)) / int(np.prod(grid))
    ptr = [0]
    idx_all, val_all, gam_all = [], [], []
    for a, (ax, ay, az, _depth, width) in enumerate(atoms):
        dx = _axis_offsets(n1, box[0], ax)
        dy = _axis_offsets(n2, box[1], ay)
        dz = _axis_offsets(n3, box[2], az)
        d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        mask = (d2 < (rcut_factor * width) ** 2).reshape(-1)
        sel = np.flatnonzero(mask)
        k, rem = np.divmod(sel, n1 * n2)
        j, i = np.divmod(rem, n1)
        ddx, ddy, ddz = dx[i], dy[j], dz[k]
        g = np.exp(-(ddx * ddx + ddy * ddy + ddz * ddz) / (2.0 * width * width))
        comps = (g, ddx / width * g, ddy / width * g, ddz / width * g)
        for l, b in enumerate(comps):
            nrm = np.sqrt(dv * np.sum(b * b))
            idx_all.append(sel.astype(np.int32))
            val_all.append(b / nrm)
            gam_all.append(gammas[a, l])
            ptr.append(ptr[-1] + sel.size)
    return KB(gamma=np.asarray(gam_all, dtype=np.float64),
              ptr=np.asarray(ptr, dtype=np.int64),
              idx=np.concatenate(idx_all) if idx_all else np.zeros(0, np.int32),
              val=np.concatenate(val_all) if val_all else np.zeros(0))


def initial_guess(ng, n_states, cfg, elem, seed):
    rng = np.random.default_rng([cfg, elem, seed, 1])
    return np.asfortranarray(rng.standard_normal((n_states, ng)).T)


def guard_columns(ng, n_guard, key):
    """Seeded N(0,1) start columns for guard vectors (ng x n_guard, Fortran
    order); key: tuple of ints naming the element."""
    rng = np.random.default_rng([9, *key])
    return np.asfortranarray(rng.standard_normal((n_guard, ng)).T)


def _fill_x0(elems, cfg, seed, elements):
    ids = list(range(len(elems))) if elements is None else list(elements)

    def one(k):
        el = elems[k]
        el.X0 = initial_guess(el.ng, el.n_states, cfg, ids[k], seed)

    with ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(one, range(len(elems))))


def central_box(grid):
    """Central floor(n/3) points per axis (restriction box of the uneven batch)."""
    lo, hi = [], []
    for n in grid:
        m = n // 3
        o = (n - m) // 2
        lo.append(o)
        hi.append(o + m)
    return tuple(lo), tuple(hi)


def _element(cfg, elem, seed, grid, box, n_atoms, zrange, n_states, lo, hi, n_alb,
             rng, wells=True, kb=True, with_x0=True):
    L = np.asarray(box)
    pos = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * L
    if zrange is not None:
        pos[:, 2] = rng.uniform(zrange[0], zrange[1], size=n_atoms)
    depth = rng.uniform(1.0, 3.0, size=n_atoms)
    width = rng.uniform(0.5, 1.0, size=n_atoms)
    gammas = rng.uniform(-1.0, 1.0, size=(n_atoms, 4))
    atoms = np.column_stack([pos, depth, width])
    ng = int(np.prod(grid))
    V = gaussian_wells(grid, box, atoms) if wells else np.zeros(ng)
    if kb:
        kbs = gaussian_kb(grid, box, atoms, gammas)
    else:
        kbs = KB(np.zeros(0), np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    X0 = initial_guess(ng, n_states, cfg, elem, seed) if with_x0 else None
    return Element(grid=tuple(grid), box=tuple(float(b) for b in box), V=V, kb=kbs,
                   X0=X0, n_states=n_states, elem_lo=tuple(lo), elem_hi=tuple(hi),
                   n_alb=n_alb, atoms=atoms)


def single_element(seed=0, grid=(24, 24, 24), n_states=32, n_atoms=8, wells=True,
                   kb=True, cfg=1):
    """One extended element: cubic periodic box, Gaussian wells (depth U[1,3] Ha,
    width U[0.5,1] bohr) at uniform positions, 4 Gaussian KB projectors per
    atom with gamma U[-1,1], seeded N(0,1) initial guess.  At the default
    grid this is the one-element workload (10 bohr cube, 24^3, 32 states)."""
    rng = np.random.default_rng([cfg, 0, seed, 0])
    box = tuple(n * H_SPACING for n in grid)
    lo, hi = central_box(grid)
    return _element(cfg, 0, seed, grid, box, n_atoms, None, n_states, lo, hi,
                    n_states // 2, rng, wells=wells, kb=kb)


def slab_batch(n_elem=64, seed=0, grid=(36, 36, 60), n_states=128, n_atoms=20,
               elements=None):
    """Extended elements of a synthetic 2D slab: 36x36x60 grid at h=10/24 bohr
    (15x15x25 bohr, vacuum along z), ~20 atoms in a 6-bohr layer centred in z,
    128 states; element = central 12x12 columns in-plane, full z; 64 ALBs."""
    box = tuple(n * H_SPACING for n in grid)
    zc = box[2] / 2.0
    m1, m2 = grid[0] // 3, grid[1] // 3
    lo = (m1, m2, 0)
    hi = (2 * m1, 2 * m2, grid[2])
    out = []
    for e in (range(n_elem) if elements is None else elements):
        rng = np.random.default_rng([2, e, seed, 0])
        out.append(_element(2, e, seed, grid, box, n_atoms, (zc - 3.0, zc + 3.0),
                            n_states, lo, hi, n_states // 2, rng, with_x0=False))
    _fill_x0(out, 2, seed, elements)
    return out


EDGES = (24, 32, 36, 48)


def uneven_batch(n_elem=200, seed=0, elements=None, edges=EDGES, j_range=(64, 256),
                 atom_range=(5, 30)):
    """Uneven batch: per element, each grid edge drawn from {24,32,36,48},
    states from U{64..256}, atoms from U{5..30}; h = 10/24 bohr; restriction
    box = central floor(n/3) points per axis; n_alb = floor(J/2)."""
    out = []
    for e in (range(n_elem) if elements is None else elements):
        rng = np.random.default_rng([4, e, seed, 0])
        grid = tuple(int(v) for v in rng.choice(edges, size=3))
        J = int(rng.integers(j_range[0], j_range[1] + 1))
        na = int(rng.integers(atom_range[0], atom_range[1] + 1))
        box = tuple(n * H_SPACING for n in grid)
        lo, hi = central_box(grid)
        out.append(_element(4, e, seed, grid, box, na, None, J, lo, hi, J // 2, rng,
                            with_x0=False))
    _fill_x0(out, 4, seed, elements)
    return out


# ---------------------------------------------------------------- MLP inputs
MLP_HIDDEN = 64
MLP_NW = 3 * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + 3 * MLP_HIDDEN + 1   # 4481
MLP_NTOT = MLP_NW + 6


def mlp_init(seed=0, last_layer=0.0):
    """Seeded initial parameters of the learned preconditioner's network, FP32,
    in the order W1 [64][3], b1, W2 [64][64], b2, w3, b3, mu [3], sd [3]:
    hidden weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases 0, output layer
    U(-last_layer, last_layer) (0: the network starts as the identity factor),
    mu = 0, sd = 1."""
    h = MLP_HIDDEN
    rng = np.random.default_rng([5, 0, seed, 2])
    w = np.zeros(MLP_NTOT, dtype=np.float32)
    o = 0
    w[o:o + 3 * h] = rng.uniform(-1, 1, 3 * h) / np.sqrt(3.0); o += 3 * h
    o += h
    w[o:o + h * h] = rng.uniform(-1, 1, h * h) / np.sqrt(h); o += h * h
    o += h
    w[o:o + h] = rng.uniform(-1, 1, h) * last_layer; o += h
    o += 1
    w[o + 3:o + 6] = 1.0
    return w


# ---------------------------------------------------------------- SCF-like updates
def perturbed_potential(el, step, amp=0.02, modes=6):
    """V of element `el` plus a smooth seeded perturbation standing in for the
    change of the effective potential between two SCF steps: `modes` random
    low-frequency cosines (|m_d| <= 2), total amplitude `amp` Ha."""
    rng = np.random.default_rng([6, 0, step, int(el.grid[0] * 10000 + el.grid[1] * 100 + el.grid[2])])
    n1, n2, n3 = el.grid
    x = np.arange(n1) / n1
    y = np.arange(n2) / n2
    z = np.arange(n3) / n3
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    dV = np.zeros((n3, n2, n1))
    for _ in range(modes):
        m = rng.integers(-2, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        dV += np.cos(2 * np.pi * (m[0] * X + m[1] * Y + m[2] * Z) + ph)
    dV *= amp / modes
    return el.V + dV.ravel()
