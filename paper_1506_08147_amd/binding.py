"""ctypes binding of libdgdft_alb.so (argument marshalling only).

Device buffers are torch tensors on the current HIP device; their data_ptr()
and torch's current stream are handed to the C ABI.  Names follow the C
entry points (dgdft_alb_create -> ALB(...), dgdft_alb_solve -> ALB.solve, ...).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgdft_alb.so")

EXPORTS = (
    "dgdft_alb_create", "dgdft_alb_destroy", "dgdft_alb_sizes", "dgdft_alb_set_potential",
    "dgdft_alb_solve", "dgdft_alb_apply_h", "dgdft_alb_precondition", "dgdft_small_syev",
    "dgdft_gemm_batched", "dgdft_alb_last_error", "dgdft_strerror", "dgdft_alb_profile",
    "dgdft_alb_kernel_stats", "dgdft_kernel_class_name", "dgdft_small_gemm_batched",
    "dgdft_alb_set_mlp", "dgdft_alb_shells", "dgdft_alb_log_capacity", "dgdft_alb_log_pairs",
    "dgdft_mlp_train", "dgdft_mlp_grad", "dgdft_mlp_eval", "dgdft_alb_get_tuning",
    "dgdft_alb_density", "dgdft_alb_nonlocal_block", "dgdft_alb_dg_volume",
    "dgdft_alb_orthonormalise", "dgdft_alb_rayleigh_ritz", "dgdft_small_syev_noalloc",
    "dgdft_alb_initial_guess", "dgdft_alb_set_tuning",
)
MLP_NW = 4481
MLP_NTOT = 4487
KCLASS = ("dg_gram", "dg_gram_reduce", "dg_update", "dg_fft_xy_fwd", "dg_fft_z", "dg_fft_xy_inv",
          "dg_kb_project", "dg_resid", "dg_rr_*", "dg_cholqr", "other", "dg_sgemm", "dg_bgemm")

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "ENOMEM",
          -4: "EHIP", -5: "EBREAKDOWN"}
PRECOND = {"teter": 0, "learned": 1, "none": 2}


class LibraryMissing(ImportError):
    pass


class DGDFTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("precond", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("poll_every", C.c_int32),
                ("elem_lo", C.POINTER(C.c_int32)), ("elem_hi", C.POINTER(C.c_int32)),
                ("n_alb", C.POINTER(C.c_int32)), ("mlp_weights", C.c_void_p),
                ("graph_iters", C.c_int32), ("tune", C.c_int32), ("n_guard", C.c_int32),
                ("n_streams", C.c_int32), ("seed", C.c_uint64)]


class KB(C.Structure):
    _fields_ = [("n_proj", C.POINTER(C.c_int32)), ("gamma", C.c_void_p), ("ptr", C.c_void_p),
                ("idx", C.c_void_p), ("val", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("max_res", C.c_double),
                ("n_chol_fallback", C.c_int32), ("n_rr_fallback", C.c_int32),
                ("n_p_drop", C.c_int32), ("n_ql_fail", C.c_int32),
                ("n_teter_fallback", C.c_int32), ("graph_launches", C.c_int32),
                ("n_rr_cholesky", C.c_int32), ("n_rr_series", C.c_int32),
                ("ms_by_phase", C.c_double * 5)]
PHASES = ("potential", "start", "iterations", "final_check", "albs")


class Pairs(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("n_elem", C.c_int32), ("shell_off", C.c_void_p),
                ("t_shell", C.c_void_p), ("s_elem", C.c_void_p), ("s_row", C.c_void_p),
                ("s_feat", C.c_void_p), ("a", C.c_void_p), ("b", C.c_void_p)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("seed", C.c_uint64), ("set_norm", C.c_int32)]


_lib = None


def load_library():
    """Load the in-tree library; raise LibraryMissing if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    lib.dgdft_alb_create.argtypes = [P(vp), P(i32), P(dbl), i32, P(i32), P(Opts)]
    lib.dgdft_alb_create.restype = i32
    lib.dgdft_alb_destroy.argtypes = [vp]
    lib.dgdft_alb_destroy.restype = None
    lib.dgdft_alb_sizes.argtypes = [vp, i32, P(i64), P(i64), P(i32), P(i32), P(i64)]
    lib.dgdft_alb_sizes.restype = i32
    lib.dgdft_alb_set_potential.argtypes = [vp, vp, P(KB), vp]
    lib.dgdft_alb_set_potential.restype = i32
    lib.dgdft_alb_solve.argtypes = [vp, vp, P(KB), vp, vp, vp, vp, vp, P(Stats), vp]
    lib.dgdft_alb_solve.restype = i32
    lib.dgdft_alb_apply_h.argtypes = [vp, i32, vp, vp, i32, vp]
    lib.dgdft_alb_apply_h.restype = i32
    lib.dgdft_alb_precondition.argtypes = [vp, i32, vp, vp, vp, i32, vp]
    lib.dgdft_alb_precondition.restype = i32
    lib.dgdft_small_syev.argtypes = [i32, i32, i32, vp, vp, vp, i32, vp]
    lib.dgdft_small_syev.restype = i32
    lib.dgdft_small_syev_noalloc.argtypes = [i32, i32, i32, vp, vp, vp, i32, vp]
    lib.dgdft_small_syev_noalloc.restype = i32
    lib.dgdft_gemm_batched.argtypes = [i32, i32, i64, i32, i32, dbl, vp, vp, dbl, vp, vp]
    lib.dgdft_gemm_batched.restype = i32
    lib.dgdft_alb_last_error.argtypes = [vp]
    lib.dgdft_alb_last_error.restype = C.c_char_p
    lib.dgdft_strerror.argtypes = [i32]
    lib.dgdft_strerror.restype = C.c_char_p
    lib.dgdft_alb_profile.argtypes = [vp, i32]
    lib.dgdft_alb_profile.restype = i32
    lib.dgdft_alb_kernel_stats.argtypes = [vp, i32, P(i64), P(dbl), P(dbl), P(dbl)]
    lib.dgdft_alb_kernel_stats.restype = i32
    lib.dgdft_small_gemm_batched.argtypes = [i32, i32, i32, i32, i32, i32, i32, i32, dbl, vp, vp,
                                             dbl, vp, vp]
    lib.dgdft_small_gemm_batched.restype = i32
    lib.dgdft_kernel_class_name.argtypes = [i32]
    lib.dgdft_kernel_class_name.restype = C.c_char_p
    lib.dgdft_alb_set_mlp.argtypes = [vp, vp]
    lib.dgdft_alb_set_mlp.restype = i32
    lib.dgdft_alb_shells.argtypes = [vp, i32, P(C.c_int32), P(dbl)]
    lib.dgdft_alb_shells.restype = i32
    lib.dgdft_alb_log_capacity.argtypes = [vp, i32, P(i64), P(i64)]
    lib.dgdft_alb_log_capacity.restype = i32
    lib.dgdft_alb_log_pairs.argtypes = [vp, vp, P(KB), vp, i32, vp, vp, vp, vp, vp, P(C.c_int32), vp]
    lib.dgdft_alb_log_pairs.restype = i32
    lib.dgdft_mlp_train.argtypes = [P(Pairs), P(i64), i64, P(TrainOpts), vp, P(dbl), vp]
    lib.dgdft_mlp_train.restype = i32
    lib.dgdft_mlp_grad.argtypes = [P(Pairs), P(i64), i64, vp, P(dbl), vp, vp]
    lib.dgdft_mlp_grad.restype = i32
    lib.dgdft_mlp_eval.argtypes = [vp, i64, vp, vp, vp]
    lib.dgdft_mlp_eval.restype = i32
    lib.dgdft_alb_get_tuning.argtypes = [vp, i32, P(C.c_int32)]
    lib.dgdft_alb_get_tuning.restype = i32
    lib.dgdft_alb_set_tuning.argtypes = [vp, i32, i32]
    lib.dgdft_alb_set_tuning.restype = i32
    lib.dgdft_alb_density.argtypes = [vp, vp, vp, vp, vp]
    lib.dgdft_alb_density.restype = i32
    lib.dgdft_alb_nonlocal_block.argtypes = [vp, vp, vp, vp]
    lib.dgdft_alb_nonlocal_block.restype = i32
    lib.dgdft_alb_dg_volume.argtypes = [vp, vp, vp, vp, i32, vp, vp]
    lib.dgdft_alb_dg_volume.restype = i32
    lib.dgdft_alb_initial_guess.argtypes = [vp, C.c_uint64, vp, vp]
    lib.dgdft_alb_initial_guess.restype = i32
    lib.dgdft_alb_orthonormalise.argtypes = [vp, i32, vp, vp, i32, P(i32), vp]
    lib.dgdft_alb_orthonormalise.restype = i32
    lib.dgdft_alb_rayleigh_ritz.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, P(i32), vp]
    lib.dgdft_alb_rayleigh_ritz.restype = i32
    _lib = lib
    return lib


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


class ALB:
    """Handle over dgdft_alb_create for a batch of extended elements.

    grids: (n_elem, 3) ints; boxes: (n_elem, 3) bohr; n_states: (n_elem,).
    n_guard: the last n_guard of every element's n_states columns are guard
    columns (iterated, not held to tol, left out of the ALBs).
    n_streams: element groups iterating on their own HIP streams (1 or 2;
    0 = the library default, 2).
    """

    def __init__(self, grids, boxes, n_states, tol=1e-8, max_iter=500, elem_lo=None,
                 elem_hi=None, n_alb=None, precond="teter", mlp_weights=None, graph_iters=0,
                 tune=False, precision="fp64", n_guard=0, n_streams=0, seed=0):
        import torch  # noqa: F401  (device memory and streams)
        self.lib = load_library()
        self.grids = np.ascontiguousarray(grids, dtype=np.int32).reshape(-1, 3)
        self.n_elem = self.grids.shape[0]
        boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        self._keep = []
        o = Opts()
        o.precision = {"fp64": 0, "mixed": 1}[precision]
        o.precond = PRECOND[precond]
        o.tol = tol
        o.max_iter = max_iter
        o.poll_every = 1
        o.graph_iters = int(graph_iters)
        o.tune = 1 if tune else 0
        o.n_guard = int(n_guard)
        o.n_streams = int(n_streams)
        o.seed = int(seed)
        self.n_guard = int(n_guard)
        if mlp_weights is not None:
            self._mlp = mlp_weights
            o.mlp_weights = mlp_weights.data_ptr()
        if elem_lo is not None:
            lo, plo = _i32(np.asarray(elem_lo).reshape(-1))
            hi, phi = _i32(np.asarray(elem_hi).reshape(-1))
            self._keep += [lo, hi]
            o.elem_lo, o.elem_hi = plo, phi
        if n_alb is not None:
            na, pna = _i32(n_alb)
            self._keep.append(na)
            o.n_alb = pna
        g, pg = _i32(self.grids.reshape(-1))
        ns, pns = _i32(n_states)
        h = C.c_void_p()
        rc = self.lib.dgdft_alb_create(C.byref(h), pg, boxes.ctypes.data_as(C.POINTER(C.c_double)),
                                       self.n_elem, pns, C.byref(o))
        if rc != 0:
            raise DGDFTError(rc, self.lib.dgdft_alb_last_error(None).decode())
        self.h = h
        self.sizes = [self._sizes(e) for e in range(self.n_elem)]

    # ---------------------------------------------------------------- ABI
    def _check(self, rc, allow=(0,)):
        if rc not in allow:
            raise DGDFTError(rc, self.lib.dgdft_alb_last_error(self.h).decode())
        return rc

    def _sizes(self, e):
        ng, ne = C.c_int64(), C.c_int64()
        J, na = C.c_int32(), C.c_int32()
        off = (C.c_int64 * 4)()
        self._check(self.lib.dgdft_alb_sizes(self.h, e, C.byref(ng), C.byref(ne), C.byref(J),
                                             C.byref(na), off))
        return dict(ng=ng.value, ne=ne.value, J=J.value, n_alb=na.value, off_ng=off[0],
                    off_ngj=off[1], off_j=off[2], off_alb=off[3])

    def totals(self):
        s = self.sizes
        return (sum(x["ng"] for x in s), sum(x["ng"] * x["J"] for x in s),
                sum(x["J"] for x in s), sum(x["ne"] * x["n_alb"] for x in s),
                sum(x["n_alb"] for x in s))

    @staticmethod
    def kb_batch(kbs, device):
        """Concatenate per-element CSR projector tables into the batch form."""
        import torch
        n_proj = np.array([k.gamma.shape[0] for k in kbs], dtype=np.int32)
        gam = np.concatenate([k.gamma for k in kbs]) if len(kbs) else np.zeros(0)
        ptrs, idxs, vals = [np.zeros(1, np.int64)], [], []
        base = 0
        for k in kbs:
            ptrs.append(np.asarray(k.ptr[1:], dtype=np.int64) + base)
            base += int(k.ptr[-1])
            idxs.append(np.asarray(k.idx, dtype=np.int32))
            vals.append(np.asarray(k.val, dtype=np.float64))
        t = dict(
            n_proj=n_proj,
            gamma=torch.from_numpy(np.ascontiguousarray(gam, dtype=np.float64)).to(device),
            ptr=torch.from_numpy(np.concatenate(ptrs)).to(device),
            idx=torch.from_numpy(np.concatenate(idxs) if idxs else np.zeros(0, np.int32)).to(device),
            val=torch.from_numpy(np.concatenate(vals) if vals else np.zeros(0)).to(device),
        )
        return t

    def _kb_struct(self, kbt):
        k = KB()
        if kbt is None:
            return None
        npj, p = _i32(kbt["n_proj"])
        self._kbkeep = (npj, kbt)
        k.n_proj = p
        k.gamma = kbt["gamma"].data_ptr() if kbt["gamma"].numel() else None
        k.ptr = kbt["ptr"].data_ptr()
        k.idx = kbt["idx"].data_ptr() if kbt["idx"].numel() else None
        k.val = kbt["val"].data_ptr() if kbt["val"].numel() else None
        return k

    def set_potential(self, V, kbt):
        k = self._kb_struct(kbt)
        self._check(self.lib.dgdft_alb_set_potential(self.h, _ptr(V), C.byref(k) if k else None,
                                                     _stream()))

    def initial_guess(self, seed, device):
        """The start block the solver draws for X0 = None (device [sum N_g*J])."""
        import torch
        X0 = torch.empty(self.totals()[1], dtype=torch.float64, device=device)
        self._check(self.lib.dgdft_alb_initial_guess(self.h, int(seed), _ptr(X0), _stream()))
        return X0

    def solve(self, V, kbt, X0, want_vecs=True, want_albs=True, device=None):
        """X0 = None: the library draws the start block (seed of the handle)."""
        import torch
        sng, sngj, sj, salb, snalb = self.totals()
        dev = X0.device if X0 is not None else (device or torch.device("cuda", torch.cuda.current_device()))
        vals = torch.empty(sj, dtype=torch.float64, device=dev)
        vecs = torch.empty(sngj, dtype=torch.float64, device=dev) if want_vecs else None
        albs = torch.empty(salb, dtype=torch.float64, device=dev) if want_albs else None
        sig = torch.empty(max(snalb, 1), dtype=torch.float64, device=dev)
        st = (Stats * self.n_elem)()
        k = self._kb_struct(kbt) if V is not None else None
        rc = self.lib.dgdft_alb_solve(self.h, _ptr(V), C.byref(k) if k else None, _ptr(X0),
                                      _ptr(vals), _ptr(vecs), _ptr(albs), _ptr(sig), st, _stream())
        self._check(rc, allow=(0, 1))
        stats = [dict(iters=s.iters, converged=bool(s.converged), max_res=s.max_res,
                      n_chol_fallback=s.n_chol_fallback, n_rr_fallback=s.n_rr_fallback,
                      n_p_drop=s.n_p_drop, n_ql_fail=s.n_ql_fail,
                      n_teter_fallback=s.n_teter_fallback,
                      graph_launches=s.graph_launches, n_rr_cholesky=s.n_rr_cholesky,
                      n_rr_series=s.n_rr_series,
                      ms_by_phase=dict(zip(PHASES, list(s.ms_by_phase)))) for s in st]
        return dict(status=rc, eigvals=vals, eigvecs=vecs, albs=albs, sigma=sig[:snalb],
                    stats=stats)

    def density(self, albs, P):
        """rho on every element box (device [sum N_E]) from ALBs and the
        diagonal density-matrix blocks P (device [sum n_alb^2])."""
        import torch
        rho = torch.empty(sum(x["ne"] for x in self.sizes), dtype=torch.float64, device=albs.device)
        self._check(self.lib.dgdft_alb_density(self.h, _ptr(albs), _ptr(P), _ptr(rho), _stream()))
        return rho

    def nonlocal_block(self, albs):
        """KB term of the DG Hamiltonian per element (device [sum n_alb^2])."""
        import torch
        out = torch.empty(sum(x["n_alb"] ** 2 for x in self.sizes), dtype=torch.float64,
                          device=albs.device)
        self._check(self.lib.dgdft_alb_nonlocal_block(self.h, _ptr(albs), _ptr(out), _stream()))
        return out

    def dg_volume(self, eigvecs, albs, sigma, lgl_ratio=2):
        """Volume terms (kinetic + V) of the diagonal DG block per element on
        its LGL grid (device [sum n_alb^2]); inputs as solve() returns them."""
        import torch
        out = torch.empty(sum(x["n_alb"] ** 2 for x in self.sizes), dtype=torch.float64,
                          device=albs.device)
        self._check(self.lib.dgdft_alb_dg_volume(self.h, _ptr(eigvecs), _ptr(albs), _ptr(sigma),
                                                 int(lgl_ratio), _ptr(out), _stream()))
        return out

    def get_tuning(self, e):
        """Tuned split-K chunk count of element e's Gram products (0: default)."""
        v = C.c_int32()
        self._check(self.lib.dgdft_alb_get_tuning(self.h, e, C.byref(v)))
        return v.value

    def set_tuning(self, e, gram_split):
        """Cached tuning: element e's split-K chunk count (0: default rule)."""
        self._check(self.lib.dgdft_alb_set_tuning(self.h, e, int(gram_split)))

    def set_mlp(self, weights):
        """Network of the learned preconditioner (device FP32 tensor [MLP_NTOT])."""
        self._mlp = weights
        self._check(self.lib.dgdft_alb_set_mlp(self.h, _ptr(weights)))

    def shells(self, e):
        """Ascending |G|^2/2 shell values of element e (numpy)."""
        n = C.c_int32()
        self._check(self.lib.dgdft_alb_shells(self.h, e, C.byref(n), None))
        t = np.zeros(n.value)
        self._check(self.lib.dgdft_alb_shells(self.h, e, C.byref(n),
                                              t.ctypes.data_as(C.POINTER(C.c_double))))
        return t

    def log_pairs(self, V, kbt, X0, max_log):
        """Training pairs from two solves (see dgdft_alb_log_pairs): a dict of
        device tensors in the dgdft_pairs layout plus n_logged (numpy)."""
        import torch
        dev = X0.device
        ns, nr = C.c_int64(), C.c_int64()
        self._check(self.lib.dgdft_alb_log_capacity(self.h, max_log, C.byref(ns), C.byref(nr)))
        ns, nr = ns.value, nr.value
        out = dict(s_elem=torch.empty(ns, dtype=torch.int32, device=dev),
                   s_row=torch.empty(ns, dtype=torch.int64, device=dev),
                   s_feat=torch.empty(4 * ns, dtype=torch.float64, device=dev),
                   a=torch.empty(max(nr, 1), dtype=torch.float64, device=dev),
                   b=torch.empty(max(nr, 1), dtype=torch.float64, device=dev))
        nl = np.zeros(self.n_elem, dtype=np.int32)
        k = self._kb_struct(kbt) if V is not None else None
        rc = self.lib.dgdft_alb_log_pairs(self.h, _ptr(V), C.byref(k) if k else None, _ptr(X0),
                                          max_log, _ptr(out["s_elem"]), _ptr(out["s_row"]),
                                          _ptr(out["s_feat"]), _ptr(out["a"]), _ptr(out["b"]),
                                          nl.ctypes.data_as(C.POINTER(C.c_int32)), _stream())
        self._check(rc)
        tsh = [self.shells(e) for e in range(self.n_elem)]
        off = np.zeros(self.n_elem + 1, dtype=np.int64)
        off[1:] = np.cumsum([t.shape[0] for t in tsh])
        out["shell_off"] = torch.from_numpy(off).to(dev)
        out["t_shell"] = torch.from_numpy(np.concatenate(tsh)).to(dev)
        out["n_samples"] = ns
        out["n_elem"] = self.n_elem
        out["n_logged"] = nl
        return out

    def split(self, out, e):
        """Per-element views (eigvals, eigvecs (Ng x J), albs (NE x n_alb), sigma)."""
        s = self.sizes[e]
        J, ng, ne, na = s["J"], s["ng"], s["ne"], s["n_alb"]
        off_nalb = sum(x["n_alb"] for x in self.sizes[:e])
        r = dict(eigvals=out["eigvals"][s["off_j"]:s["off_j"] + J])
        if out["eigvecs"] is not None:
            r["eigvecs"] = out["eigvecs"][s["off_ngj"]:s["off_ngj"] + ng * J].view(J, ng).T
        if out["albs"] is not None:
            r["albs"] = out["albs"][s["off_alb"]:s["off_alb"] + ne * na].view(na, ne).T
        r["sigma"] = out["sigma"][off_nalb:off_nalb + na]
        return r

    def apply_h(self, e, X):
        """X: (ncols, Ng) contiguous device tensor (column-major Ng x ncols)."""
        import torch
        HX = torch.empty_like(X)
        self._check(self.lib.dgdft_alb_apply_h(self.h, e, _ptr(X), _ptr(HX), X.shape[0], _stream()))
        return HX

    def precondition(self, e, R, X):
        import torch
        W = torch.empty_like(R)
        self._check(self.lib.dgdft_alb_precondition(self.h, e, _ptr(R), _ptr(X), _ptr(W),
                                                    R.shape[0], _stream()))
        return W

    def orthonormalise(self, e, G, init=False):
        """T (J x J) with Y T orthonormal for the Gram G = Y^T Y (device
        float64, J x J); returns (T, flags) with flags as in the header."""
        import torch
        Gc = G.t().contiguous()   # column-major
        T = torch.empty_like(Gc)
        fl = np.zeros(6, dtype=np.int32)
        self._check(self.lib.dgdft_alb_orthonormalise(
            self.h, e, _ptr(Gc), _ptr(T), int(bool(init)),
            fl.ctypes.data_as(C.POINTER(C.c_int32)), _stream()))
        return T.t(), fl

    def rayleigh_ritz(self, e, kb, Hh, M):
        """(theta, C, D, flags) of the Rayleigh-Ritz step on n x n matrices
        Hh = S^T H S, M = S^T S (device float64, n = kb J); C, D are n x J
        (D is None for kb = 1)."""
        import torch
        J = self.sizes[e]["J"]
        n = kb * J
        Hc, Mc = Hh.t().contiguous(), M.t().contiguous()
        th = torch.empty(J, dtype=torch.float64, device=Hh.device)
        Cm = torch.empty(J, n, dtype=torch.float64, device=Hh.device)
        Dm = torch.empty(J, n, dtype=torch.float64, device=Hh.device) if kb > 1 else None
        fl = np.zeros(6, dtype=np.int32)
        self._check(self.lib.dgdft_alb_rayleigh_ritz(
            self.h, e, int(kb), _ptr(Hc), _ptr(Mc), _ptr(th), _ptr(Cm), _ptr(Dm),
            fl.ctypes.data_as(C.POINTER(C.c_int32)), _stream()))
        return th, Cm.t(), (Dm.t() if Dm is not None else None), fl

    def profile(self, enable=True):
        """Enable per-kernel HIP-event timing and reset the counters."""
        self._check(self.lib.dgdft_alb_profile(self.h, int(enable)))

    def kernel_stats(self):
        out = {}
        for k in range(len(KCLASS)):
            n, ms, fl, by = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
            self._check(self.lib.dgdft_alb_kernel_stats(self.h, k, C.byref(n), C.byref(ms),
                                                        C.byref(fl), C.byref(by)))
            out[self.lib.dgdft_kernel_class_name(k).decode()] = dict(
                launches=n.value, ms=ms.value, flops=fl.value, bytes=by.value)
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.dgdft_alb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def small_syev(A, k, method=0):
    """A: (count, n, n) device float64 (upper triangle read, column-major per
    matrix); returns w (count, n) ascending and Z (count, k, n) (columns)."""
    import torch
    lib = load_library()
    count, n, _ = A.shape
    A = A.contiguous()
    w = torch.empty(count, n, dtype=torch.float64, device=A.device)
    Z = torch.empty(count, k, n, dtype=torch.float64, device=A.device)
    rc = lib.dgdft_small_syev(count, n, k, _ptr(A), _ptr(w), _ptr(Z), int(method), _stream())
    if rc != 0:
        raise DGDFTError(rc, lib.dgdft_alb_last_error(None).decode())
    return w, Z


def small_syev_noalloc(A, k, method=0, w=None, Z=None):
    """dgdft_small_syev_noalloc: as small_syev, with the library's static
    workspace (no device allocation inside the call).  Output tensors may be
    passed in (w: (count, n), Z: (count, k, n)) so that nothing is allocated
    here either; raises DGDFTError (EINVAL) when the batch exceeds the
    workspace."""
    import torch
    lib = load_library()
    count, n, _ = A.shape
    if w is None:
        w = torch.empty(count, n, dtype=torch.float64, device=A.device)
    if Z is None:
        Z = torch.empty(count, k, n, dtype=torch.float64, device=A.device)
    rc = lib.dgdft_small_syev_noalloc(count, n, k, _ptr(A), _ptr(w), _ptr(Z), int(method), _stream())
    if rc != 0:
        raise DGDFTError(rc, lib.dgdft_alb_last_error(None).decode())
    return w, Z


def small_gemm_batched(ta, tb, J, kb, dm, dn, dk, A, B, C, alpha=1.0, beta=0.0):
    """The Rayleigh-Ritz small-matrix product kernel: per problem
    C = alpha op(A) op(B) + beta C, dims coded 0 -> kb*J, 1 -> J.  A, B, C:
    (count, cols, rows) device tensors (column-major per problem).  Returns C'."""
    lib = load_library()
    Ac, Bc, Cc = A.contiguous(), B.contiguous(), C.clone().contiguous()
    rc = lib.dgdft_small_gemm_batched(int(ta), int(tb), A.shape[0], int(J), int(kb), int(dm),
                                      int(dn), int(dk), float(alpha), _ptr(Ac), _ptr(Bc),
                                      float(beta), _ptr(Cc), _stream())
    if rc != 0:
        raise DGDFTError(rc, lib.dgdft_alb_last_error(None).decode())
    return Cc


def gemm_batched(trans, A, B, alpha=1.0, beta=0.0, Cin=None, fp32=False):
    """Column-major batched products on the library's MFMA kernels.
    A: (count, m, K) device tensor = column-major K x m per problem.
    trans=1: B (count, n, K) -> C (count, n, m) = column-major (A^T B) m x n.
    trans=0: B (count, n, m) (column-major m x n) -> C (count, n, K) = alpha A B + beta C.
    fp32: the mixed form's FP32 kernels (FP64 storage)."""
    import torch
    lib = load_library()
    count, m, K = A.shape
    n = B.shape[1]
    if trans:
        Cout = torch.empty(count, n, m, dtype=torch.float64, device=A.device)
    else:
        Cout = (Cin.clone() if Cin is not None else
                torch.zeros(count, n, K, dtype=torch.float64, device=A.device))
    Ac, Bc = A.contiguous(), B.contiguous()
    rc = lib.dgdft_gemm_batched(int(trans) | (2 if fp32 else 0), count, K, m, n, alpha, _ptr(Ac),
                                _ptr(Bc), beta,
                                _ptr(Cout), _stream())
    if rc != 0:
        raise DGDFTError(rc, lib.dgdft_alb_last_error(None).decode())
    return Cout


def _pairs_struct(d):
    p = Pairs()
    p.n_samples = int(d["n_samples"])
    p.n_elem = int(d["n_elem"])
    for f in ("shell_off", "t_shell", "s_elem", "s_row", "s_feat", "a", "b"):
        setattr(p, f, d[f].data_ptr())
    return p


def _index(index):
    if index is None:
        return None, None, 0
    idx = np.ascontiguousarray(index, dtype=np.int64)
    return idx, idx.ctypes.data_as(C.POINTER(C.c_int64)), idx.shape[0]


def mlp_train(pairs, weights, index=None, epochs=10, batch=256, lr=1e-3, seed=0, set_norm=True,
              beta1=0.9, beta2=0.999, eps=1e-8):
    """Train the learned preconditioner's network in place on the GPU
    (dgdft_mlp_train); returns the mean loss of each epoch."""
    lib = load_library()
    p = _pairs_struct(pairs)
    keep, ip, n = _index(index)
    o = TrainOpts(epochs=epochs, batch=batch, lr=lr, beta1=beta1, beta2=beta2, eps=eps, seed=seed,
                  set_norm=1 if set_norm else 0)
    hist = np.zeros(epochs)
    rc = lib.dgdft_mlp_train(C.byref(p), ip, n, C.byref(o), _ptr(weights),
                             hist.ctypes.data_as(C.POINTER(C.c_double)), _stream())
    if rc != 0:
        raise DGDFTError(rc, lib.dgdft_alb_last_error(None).decode())
    return hist


def mlp_grad(pairs, weights, index=None):
    """(mean loss, gradient tensor [MLP_NW] FP64) at the given weights."""
    import torch
    lib = load_library()
    p = _pairs_struct(pairs)
    keep, ip, n = _index(index)
    g = torch.empty(MLP_NW, dtype=torch.float64, device=weights.device)
    loss = C.c_double()
    rc = lib.dgdft_mlp_grad(C.byref(p), ip, n, _ptr(weights), C.byref(loss), _ptr(g), _stream())
    if rc != 0:
        raise DGDFTError(rc, lib.dgdft_alb_last_error(None).decode())
    return loss.value, g


def mlp_eval(feat, weights):
    """f for raw input rows feat (device [n, 3]: x = t/T, theta, Vbar)."""
    import torch
    lib = load_library()
    feat = feat.contiguous()
    f = torch.empty(feat.shape[0], dtype=torch.float64, device=feat.device)
    rc = lib.dgdft_mlp_eval(_ptr(feat), feat.shape[0], _ptr(weights), _ptr(f), _stream())
    if rc != 0:
        raise DGDFTError(rc, lib.dgdft_alb_last_error(None).decode())
    return f
