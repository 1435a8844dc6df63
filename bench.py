#!/usr/bin/env python3
"""Benchmark of ALB generation on one MI355X.

A step is one whole pass of the method over one batch of extended elements:
loading the potentials, LOBPCG from the seeded initial guesses to the
residual tolerance, the final FP64 check, and restriction + SVD truncation to
ALBs (all through the C ABI).  The metric is converged element eigensolves
per second.

Default workload: the uneven batch of 200 extended elements (grid edges drawn
from {24, 32, 36, 48} per axis at h = 10/24 bohr, 64-256 states, 5-30
Gaussian-well atoms with 4 KB projectors each), residual 1e-6, 16 guard
columns, restriction to the central third per axis and floor(J/2) ALBs.
The 64-element slab (36x36x60, 128 states, 64 ALBs) and the one-element
workload (24^3, 32 states) are measured beside it under "forms".  Inputs are
resident in HBM before the timed region starts.

Roofline of the dominant product class, from the algorithmic work of the
method per element and LOBPCG iteration: the twelve J x J blocks of the
Gram products are 24 N_g J^2 flops and the seven update products 14 N_g J^2
(the paper's operation count per iteration, Sec. II.B), with J the block
width (states plus guard columns) and the iteration counts the solver
reports; divided by the class's kernel time measured with HIP events on its
launch stream over the timed region.

Prints one JSON line (rank 0).  One GPU only.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "converged element eigensolves/s at residual 1e-6: plain FP64 vs mixed+learned"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# algorithmic flops per element and LOBPCG iteration, in units of N_g J^2
ALG_UNITS = {"dg_gram": 24.0, "dg_update": 14.0}
# HBM bytes per launch of a product class from the FETCH_SIZE / WRITE_SIZE
# counter runs of the default command, calibrated on a 1 GiB copy (see
# profiles/): (kernel class, workload, guard columns, streams) -> bytes.  Valid
# only for the kernel build that was measured; removed when the kernel changes.
MEASURED_TRAFFIC = {("dg_gram", "uneven_edges_24-48_J64-256", 16, 1): 105.643e9,
                    ("dg_update", "uneven_edges_24-48_J64-256", 16, 1): 85.412e9}
# guard columns per element when --guard is not given: 16 on the slab (block
# of 144 columns, the tile width of the 144-wide GEMM kernels) and on the
# uneven batch, 8 on the one-element workload (32 states)
DEFAULT_GUARD = {"slab": 16, "uneven": 16, "one": 8}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name, n_elem):
    import synth
    if name == "slab":
        els = synth.slab_batch(n_elem or 64)
        desc = dict(workload="slab_36x36x60_J128", elements=len(els), grid=[36, 36, 60],
                    n_states=128, atoms_per_element=20, n_alb=64, element_box=[12, 12, 60])
    elif name == "one":
        els = [synth.single_element(seed=s) for s in range(n_elem or 1)]
        desc = dict(workload="cube_24^3_J32", elements=len(els), grid=[24, 24, 24], n_states=32,
                    atoms_per_element=8, n_alb=16)
    else:
        els = synth.uneven_batch(n_elem or 200)
        desc = dict(workload="uneven_edges_24-48_J64-256", elements=len(els),
                    grid_edges=[24, 32, 36, 48], n_states=[64, 256], atoms_per_element=[5, 30],
                    element_box="central third per axis", n_alb="floor(J/2)")
    return els, desc


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(el, tol, n_guard):
    """The oracle on one element of the same workload: its LOBPCG with the
    same start block as the GPU (the element's n_states columns plus n_guard
    guard columns, stopping test on the n_states wanted residuals) run to the
    tolerance, then the restriction + SVD truncation; one converged element
    per that time, with all host threads on the one element."""
    import numpy as np
    from oracle import alb, lobpcg as lob, teter
    from oracle.hamiltonian import FFT_WORKERS, Operator
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        blas = 1
    op = Operator(el.grid, el.box, el.V, el.kb)
    pre = lambda R, X: teter.precondition(R, X, op.grid, op.box)  # noqa: E731

    import synth
    X0 = el.X0
    if n_guard:
        X0 = np.hstack([el.X0, synth.guard_columns(el.ng, n_guard, (0, el.n_states))])
    t = time.perf_counter()
    res = lob.lobpcg(op.apply, pre, X0, tol, 500, n_check=el.n_states)
    t_solve = time.perf_counter() - t
    alb.restrict_svd(res.X[:, :el.n_states], op.grid, el.elem_lo, el.elem_hi, op.dv, el.n_alb)
    est = time.perf_counter() - t
    return dict(value=1.0 / est, unit="elements/s", cores=int(max(FFT_WORKERS, blas)),
                kind="oracle", cpu_model=cpu_model(), host_threads=os.cpu_count(),
                sample=(f"element 0 of the workload (grid {list(el.grid)}, {el.n_states} states "
                        f"+ {n_guard} guard columns): oracle LOBPCG to residual {tol:g} "
                        f"({res.iters} iterations, converged={res.converged}, {t_solve:.1f} s) "
                        f"+ ALB step: {est:.1f} s per converged element, one element at a time "
                        f"with all threads on it (per-element rate; no concurrent elements)"))


def start_block(els, n_guard, dev):
    """X0 of the batch on the device: each element's seeded start columns,
    then n_guard seeded guard columns."""
    import numpy as np
    import torch
    import synth
    parts = []
    for k, e in enumerate(els):
        parts.append(torch.from_numpy(np.ascontiguousarray(e.X0.T)).reshape(-1))
        if n_guard:
            G = synth.guard_columns(e.ng, n_guard, (k, e.n_states))
            parts.append(torch.from_numpy(np.ascontiguousarray(G.T)).reshape(-1))
    return torch.cat(parts).to(dev)


def make_handle(args, els, guard=None, **kw):
    from paper_1506_08147_amd import ALB
    g = args.guard if guard is None else guard
    kw.setdefault("n_streams", args.streams)
    return ALB([e.grid for e in els], [e.box for e in els], [e.n_states + g for e in els],
               elem_lo=[e.elem_lo for e in els], elem_hi=[e.elem_hi for e in els],
               n_alb=[e.n_alb for e in els], n_guard=g, **kw)


def resident_inputs(els, guard, dev):
    import torch
    from paper_1506_08147_amd import ALB
    V = torch.cat([torch.from_numpy(e.V) for e in els]).to(dev)
    return V, ALB.kb_batch([e.kb for e in els], dev), start_block(els, guard, dev)


def warm_mode(args, h, els, desc, V, kbt, out):
    """SCF-like ALB updates: each step perturbs every element's potential
    (smooth seeded change of 0.02 Ha), then runs 3 LOBPCG iterations from the
    previous eigenvectors and the restriction + SVD truncation."""
    import numpy as np
    import torch
    import synth
    dev = V.device
    Vs = [torch.cat([torch.from_numpy(synth.perturbed_potential(e, s + 1)) for e in els]).to(dev)
          for s in range(args.warm)]
    h3 = make_handle(args, els, tol=1e-14, max_iter=3)
    X = out["eigvecs"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.warm):
        o = h3.solve(Vs[s], kbt, X)
        X = o["eigvecs"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = [st["max_res"] for st in o["stats"]]
    h3.close()
    h.close()
    n = len(els)
    line = dict(metric="ALB element updates/s (3 warm-start LOBPCG iterations + ALBs per SCF step)",
                value=round(n * args.warm / el, 3), unit="element updates/s", n_gpus=1,
                steps=args.warm, warmup=0, ms_per_step=round(1e3 * el / args.warm, 2),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
                data="synthetic", config=dict(desc, precision="fp64", preconditioner="teter",
                                              warm_iterations=3, dV_amplitude=0.02,
                                              guard_columns=args.guard),
                residual_after_step=dict(max=float(max(res)), median=float(np.median(res))),
                paper_context="1,185 element updates/s: 1,600 elements in 1.35 s on 12,800 CPU "
                              "cores (P3500 phosphorene, 80 ALBs per element); different "
                              "hardware and workload")
    print(json.dumps(line), flush=True)


def algorithmic_units(els, guard, stats):
    """sum over elements of iterations * N_g * J^2 (J = block width) of one solve."""
    return sum(float(st["iters"]) * e.ng * float(e.n_states + guard) ** 2
               for e, st in zip(els, stats))


def algorithmic_flops(k, v, units_per_step, steps):
    """The method's flops for product class k over the timed region: the
    paper's count (ALG_UNITS per N_g J^2 and iteration), or the flops the
    kernels executed where that is less (the Gram products form the carried
    [X P] blocks and the W columns of S^T S in small space), so that the
    rate never counts work that was not done."""
    return min(ALG_UNITS[k] * units_per_step * steps, v["flops"])


def roofline(ks, units_per_step, steps):
    """Dominant product class by kernel time in the timed region, with its
    algorithmic flops per launch over the class's average HIP-event launch
    time."""
    dom = max(ALG_UNITS, key=lambda k: ks[k]["ms"])
    d = ks[dom]
    launches = max(d["launches"], 1)
    alg = algorithmic_flops(dom, d, units_per_step, steps)
    ach = alg / (d["ms"] * 1e-3) / 1e12
    paper = ALG_UNITS[dom] * units_per_step * steps
    return dict(bound="mfma", achieved=round(ach, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                frac=round(ach / PEAK_FP64_TFLOPS, 4), traffic=None, kernel=dom,
                launches=d["launches"], avg_launch_ms=round(d["ms"] / launches, 4),
                algorithmic_flops_per_launch=alg / launches,
                algorithmic_count=("paper: " if alg == paper else "executed (below the paper's "
                                   f"{ALG_UNITS[dom]:g} N_g J^2): ") +
                f"{alg / max(units_per_step * steps, 1):.2f} N_g J^2 per element-iteration",
                executed_flops_per_launch=d["flops"] / launches)


def kernel_table(ks, units_per_step, steps):
    out = {}
    for k, v in ks.items():
        if not v["launches"]:
            continue
        r = dict(ms_per_step=round(v["ms"] / steps, 3), launches=v["launches"])
        if v["ms"] and v["flops"]:
            r["executed_tflops"] = round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 3)
        if v["ms"] and k in ALG_UNITS:
            r["algorithmic_tflops"] = round(
                algorithmic_flops(k, v, units_per_step, steps) / (v["ms"] * 1e-3) / 1e12, 3)
        if v["ms"] and v["bytes"]:
            r["gbs"] = round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
        out[k] = r
    return out


def time_solves(h, V, kbt, X0, steps):
    """1 warm-up solve, then `steps` timed solves; (elements/s, s per step, last output)."""
    import torch
    out = h.solve(V, kbt, X0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_conv = 0
    for _ in range(steps):
        out = h.solve(V, kbt, X0)
        n_conv += sum(1 for st in out["stats"] if st["converged"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return n_conv / el, el / steps, out


def form_summary(value, s_step, out, **kw):
    import numpy as np
    st = out["stats"]
    return dict(value=round(value, 4), ms_per_step=round(1e3 * s_step, 2),
                iterations_mean=float(np.mean([s["iters"] for s in st])),
                converged=f"{sum(1 for s in st if s['converged'])}/{len(st)}",
                teter_fallback_bands=int(sum(s["n_teter_fallback"] for s in st)), **kw)


def train_network(dev, guard=8):
    """Network of the learned preconditioner: pairs logged by the solver on
    one-element workloads (seeds 100-115, 24^3, 32 states + `guard` guard
    columns, the block layout the learned form runs with, residual 1e-8,
    first 40 iterations), the wanted bands only, 30 epochs of Adam on the
    GPU."""
    import numpy as np
    import torch
    import synth
    from paper_1506_08147_amd import ALB, mlp_train
    t = time.perf_counter()
    els = [synth.single_element(seed=s) for s in range(100, 116)]
    h = ALB([e.grid for e in els], [e.box for e in els], [e.n_states + guard for e in els], tol=1e-8,
            elem_lo=[e.elem_lo for e in els], elem_hi=[e.elem_hi for e in els],
            n_alb=[e.n_alb for e in els], n_guard=guard)
    V, kbt, X0 = resident_inputs(els, guard, dev)
    max_log = 40
    P = h.log_pairs(V, kbt, X0, max_log)
    h.close()
    # samples are laid out [element][logged iteration][band of the block]
    idx, base = [], 0
    for e, nl in enumerate(P["n_logged"]):
        jb = els[e].n_states + guard
        for it in range(int(nl)):
            idx += [base + it * jb + b for b in range(els[e].n_states)]
        base += max_log * jb
    w = torch.from_numpy(synth.mlp_init(seed=0, last_layer=0.0)).to(dev)
    hist = mlp_train(P, w, index=np.asarray(idx), epochs=30, batch=256, lr=2e-3, seed=1)
    el = time.perf_counter() - t
    log(f"network trained in {el:.1f} s: loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    return w, dict(samples=len(idx), epochs=30, guard_columns=guard, loss_first=round(float(hist[0]), 5),
                   loss_last=round(float(hist[-1]), 5), seconds=round(el, 1))


def mixed_vs_oracle(args, dev, seeds=(1000, 1001, 1002, 1003)):
    """The mixed form on one-element workloads (24^3, 32 states, residual 1e-6)
    against the FP64 oracle: per element the largest eigenvalue difference
    and the sine of the largest principal angle between the GPU's and the
    oracle's eigenvectors (states below the largest cut with a gap >= 1e-4
    Ha)."""
    import numpy as np
    import synth
    from oracle.solve import solve_element
    els = [synth.single_element(seed=s) for s in seeds]
    h = make_handle(args, els, guard=0, tol=1e-6, max_iter=1000, precision="mixed")
    V, kbt, X0 = resident_inputs(els, 0, dev)
    out = h.solve(V, kbt, X0)
    rows = []
    for i, el in enumerate(els):
        r = h.split(out, i)
        ref = solve_element(el, tol=1e-6)
        lam_g = r["eigvals"].cpu().numpy()
        Xg = r["eigvecs"].cpu().numpy() * np.sqrt(el.dv)
        Xo = ref["eigvecs"] * np.sqrt(el.dv)
        gaps = np.diff(ref["eigvals"])
        cut = int(np.nonzero(gaps >= 1e-4)[0].max()) + 1 if np.any(gaps >= 1e-4) else el.n_states
        s = np.linalg.svd(Xo[:, :cut].T @ Xg[:, :cut], compute_uv=False)
        rows.append(dict(seed=int(seeds[i]),
                         max_abs_dlambda_ha=float(np.abs(lam_g - ref["eigvals"]).max()),
                         sin_max_angle=float(np.sqrt(max(0.0, 1.0 - s.min() ** 2))),
                         angle_states=cut, gpu_iters=out["stats"][i]["iters"],
                         oracle_iters=int(ref["iters"])))
    h.close()
    return dict(workload="cube_24^3_J32", tol=1e-6, reference="FP64 oracle", elements=rows)


def learned_eval(args, dev, w, seeds=range(1000, 1016), guard=8):
    """The learned preconditioner against Teter's on the one-element
    workloads of the evaluation seeds (24^3, 32 states + 8 guard columns,
    mixed precision, residual 1e-6): per seed the iterations of each and
    the wall time of a solve of the 16 elements together."""
    import numpy as np
    import synth
    els = [synth.single_element(seed=s) for s in seeds]
    V, kbt, X0 = resident_inputs(els, guard, dev)
    out = {}
    for name, kw in (("teter", {}), ("learned", dict(precond="learned", mlp_weights=w))):
        h = make_handle(args, els, guard=guard, tol=1e-6, max_iter=1000, precision="mixed", **kw)
        v, s_step, o = time_solves(h, V, kbt, X0, 1)
        h.close()
        out[name] = dict(iterations=[int(st["iters"]) for st in o["stats"]],
                         converged=int(sum(1 for st in o["stats"] if st["converged"])),
                         seconds=round(s_step, 3),
                         teter_fallback_bands=int(sum(st["n_teter_fallback"] for st in o["stats"])))
    it_t, it_l = np.array(out["teter"]["iterations"]), np.array(out["learned"]["iterations"])
    out["seeds"] = list(seeds)
    out["guard_columns"] = guard
    out["learned_fewer"] = int((it_l < it_t).sum())
    out["learned_more"] = int((it_l > it_t).sum())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uneven", choices=["uneven", "slab", "one"])
    ap.add_argument("--elements", type=int, default=None)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--streams", type=int, default=1, choices=[1, 2],
                    help="element groups on their own HIP streams (1: kernel durations are not "
                         "shared with a second group, so HIP events and rocprofv3 agree)")
    ap.add_argument("--guard", type=int, default=None,
                    help="guard columns per element: the block holds n_states + G columns, "
                         "convergence and ALBs use the first n_states (default: 16 on the "
                         "slab and the uneven batch, 8 on the one-element workload)")
    ap.add_argument("--graph", type=int, default=0,
                    help="LOBPCG iterations per captured HIP graph launch (0: eager)")
    ap.add_argument("--tune", type=int, default=0, help="1: autotune at create")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--precond", default="teter", choices=["teter", "learned"],
                    help="preconditioner of the timed form (learned: the network trained as "
                         "for the mixed + learned form)")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="1: one 1 GiB device copy before the timed region, whose hardware "
                         "counters calibrate FETCH_SIZE / WRITE_SIZE in profiler runs")
    ap.add_argument("--forms", type=int, default=1,
                    help="1: also time the mixed and the mixed + learned-preconditioner forms "
                         "of the workload, the slab and the one-element mixed form against the "
                         "oracle, and report them under 'forms'")
    ap.add_argument("--form-steps", type=int, default=1,
                    help="timed solves per form (after one warm-up solve)")
    ap.add_argument("--dg-blocks", type=int, default=1,
                    help="1: time the element-local DG quantities from the last step's ALBs")
    ap.add_argument("--warm", type=int, default=0,
                    help="S > 0: warm-start mode instead: after one converged solve, S timed "
                         "SCF-like steps (perturbed V, 3 LOBPCG iterations from the previous "
                         "eigenvectors, ALBs); reports element updates per second")
    args = ap.parse_args()
    if args.guard is None:
        args.guard = DEFAULT_GUARD.get(args.workload, 0)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the "
              "extended elements would be split across GPUs, each solving its share with no "
              "communication). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.warm > 0 and args.warmup < 1:
        args.warmup = 1   # the converged solve the warm steps start from
    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    t = time.perf_counter()
    els, desc = workload(args.workload, args.elements)
    log(f"inputs generated: {len(els)} elements in {time.perf_counter() - t:.1f} s")
    V, kbt, X0 = resident_inputs(els, args.guard, dev)
    extra = {}
    if args.precond == "learned":
        # the network the mixed + learned form uses (trained before timing)
        w_main, _ = train_network(dev)
        extra = dict(precond="learned", mlp_weights=w_main)
    h = make_handle(args, els, tol=args.tol, max_iter=1000, graph_iters=args.graph,
                    tune=bool(args.tune), precision=args.precision, **extra)
    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    torch.cuda.synchronize()
    for w in range(args.warmup):
        t = time.perf_counter()
        out = h.solve(V, kbt, X0)
        log(f"warmup {w}: {time.perf_counter() - t:.2f} s")
    if args.warm > 0:
        warm_mode(args, h, els, desc, V, kbt, out)
        return
    h.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_conv = 0
    for s in range(args.steps):
        out = h.solve(V, kbt, X0)
        n_conv += sum(1 for st in out["stats"] if st["converged"])
        log(f"step {s}: done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ks = h.kernel_stats()
    h.profile(False)
    stats = out["stats"]
    iters = [st["iters"] for st in stats]
    ms_step = 1e3 * elapsed / args.steps
    units = algorithmic_units(els, args.guard, stats)

    roof = roofline(ks, units, args.steps)
    roof["traffic"] = MEASURED_TRAFFIC.get((roof["kernel"], desc["workload"], args.guard,
                                            args.streams))
    kernels = kernel_table(ks, units, args.steps)
    dgb = None
    if args.dg_blocks:
        dgb = dg_blocks(h, els, out, dev)
    h.close()
    forms = None
    if args.forms:
        forms = dict(fp64_plain=dict(value=round(n_conv / elapsed, 4), ms_per_step=round(ms_step, 2),
                                     iterations_mean=float(np.mean(iters)), streams=args.streams))
        if args.streams == 1:
            # the same solve on two element groups (two streams): one group's
            # small dense Rayleigh-Ritz steps overlap the other's products;
            # per-kernel event times then share the GPU, so the roofline is
            # taken from the one-stream run above
            h2 = make_handle(args, els, tol=args.tol, max_iter=1000, n_streams=2)
            v, s_step, o = time_solves(h2, V, kbt, X0, args.form_steps)
            h2.close()
            forms["fp64_two_streams"] = form_summary(v, s_step, o, precision="fp64",
                                                     preconditioner="teter", streams=2)
            log(f"form fp64 two streams: {v:.3f} elements/s")
        hm = make_handle(args, els, tol=args.tol, max_iter=1000, precision="mixed")
        v, s_step, o = time_solves(hm, V, kbt, X0, args.form_steps)
        hm.close()
        forms["mixed"] = form_summary(v, s_step, o, precision="mixed", preconditioner="teter")
        log(f"form mixed/teter: {v:.3f} elements/s")
        w, training = train_network(dev)
        hl = make_handle(args, els, tol=args.tol, max_iter=1000, precision="mixed",
                         precond="learned", mlp_weights=w)
        v, s_step, o = time_solves(hl, V, kbt, X0, args.form_steps)
        hl.close()
        forms["mixed_learned"] = form_summary(v, s_step, o, precision="mixed",
                                              preconditioner="learned", training=training)
        log(f"form mixed/learned: {v:.3f} elements/s")
        forms["learned_vs_teter_one_element"] = learned_eval(args, dev, w)
        log("learned vs Teter on the evaluation seeds: fewer iterations on "
            f"{forms['learned_vs_teter_one_element']['learned_fewer']} of 16")
        forms["ratio_mixed_learned_over_fp64"] = round(
            forms["mixed_learned"]["value"] / forms["fp64_plain"]["value"], 3)
        if args.workload != "slab":
            sels, sdesc = workload("slab", None)
            sg = DEFAULT_GUARD["slab"]
            sV, skb, sX0 = resident_inputs(sels, sg, dev)
            hs = make_handle(args, sels, guard=sg, tol=args.tol, max_iter=1000)
            v, s_step, o = time_solves(hs, sV, skb, sX0, args.form_steps)
            hs.close()
            del sV, skb, sX0
            forms["slab_fp64"] = form_summary(v, s_step, o, precision="fp64",
                                              preconditioner="teter", workload=sdesc["workload"],
                                              elements=len(sels), guard_columns=sg)
            log(f"form slab fp64: {v:.3f} elements/s")
        forms["mixed_one_element_vs_oracle"] = mixed_vs_oracle(args, dev)
    line = dict(metric=METRIC, value=round(n_conv / elapsed, 4), unit="elements/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_step, 2),
                higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f64" if args.precision == "fp64" else "f64+f32",
                data="synthetic", config=dict(desc, tol=args.tol, precision=args.precision,
                                              preconditioner=args.precond, graph_iters=args.graph,
                                              tuned=bool(args.tune), guard_columns=args.guard,
                                              streams=args.streams),
                roofline=roof, kernels=kernels,
                iterations=dict(mean=float(np.mean(iters)), min=int(min(iters)), max=int(max(iters))),
                converged=f"{sum(1 for st in stats if st['converged'])}/{len(stats)}",
                rr_reductions=dict(cholesky=int(sum(st["n_rr_cholesky"] for st in stats)),
                                   series=int(sum(st["n_rr_series"] for st in stats))))
    if dgb is not None:
        line["dg_blocks"] = dgb
    if forms is not None:
        line["forms"] = forms
    if args.cpu_baseline:
        log("timing the oracle sample on the host")
        line["cpu_baseline"] = cpu_baseline(els[0], args.tol, args.guard)
    print(json.dumps(line), flush=True)


def dg_blocks(h, els, out, dev):
    """Element-local DG quantities from the last step's ALBs: density from
    P = 2 I, the nonlocal block and the volume terms on the LGL grid (twice
    the uniform points per axis), each timed once after an untimed call."""
    import torch
    nal = [e.n_alb for e in els]
    Pd = torch.cat([torch.eye(n, dtype=torch.float64).reshape(-1) * 2.0 for n in nal]).to(dev)
    h.density(out["albs"], Pd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rho = h.density(out["albs"], Pd)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    h.nonlocal_block(out["albs"])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    h.dg_volume(out["eigvecs"], out["albs"], out["sigma"])
    torch.cuda.synchronize()
    h.profile(True)
    t4 = time.perf_counter()
    vol = h.dg_volume(out["eigvecs"], out["albs"], out["sigma"])
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    bg = h.kernel_stats()["dg_bgemm"]
    h.profile(False)
    bg_tf = bg["flops"] / (bg["ms"] * 1e-3) / 1e12 if bg["ms"] else 0.0
    sym = max(float((v.reshape(n, n) - v.reshape(n, n).T).abs().max())
              for v, n in zip(torch.split(vol, [n * n for n in nal]), nal))
    return dict(density_ms=round(1e3 * (t2 - t1), 3), nonlocal_block_ms=round(1e3 * (t3 - t2), 3),
                electrons_check=round(sum(
                    e.dv * float(r.sum()) for e, r in zip(els, torch.split(rho, [x["ne"] for x in h.sizes])))
                    / (2.0 * sum(nal)), 12),
                volume_ms_with_events=round(1e3 * (t5 - t4), 3),
                volume_bgemm=dict(launches=bg["launches"], ms=round(bg["ms"], 3),
                                  gflop=round(bg["flops"] / 1e9, 2), tflops=round(bg_tf, 2),
                                  frac_fp64_peak=round(bg_tf / PEAK_FP64_TFLOPS, 4)),
                volume_asymmetry=sym)


if __name__ == "__main__":
    main()
