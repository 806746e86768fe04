#!/usr/bin/env python3
"""Benchmark of the hex8 finite-strain Hill-48 residual + tangent + CSR pass.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (synthetic, seeded): the 100x100x100 hex8 cube (1,000,000 elements,
1,030,301 nodes, 3,090,903 dofs, 8,000,000 Gauss points, nnz 245,438,109),
per-element Hill-48 F,G,H from smooth random fields, 30% of the Gauss points
yielding at the trial state, x = 0 face constrained.  A step is one
fem_residual_tangent call in FP64, the paper's precision (element kernel with
return map / residual / element tangent, residual assembly with Dirichlet
rows and the FP64 residual norm, tangent assembly into the CSR values),
inputs resident in HBM.  Prints ONE JSON line.

Also reported (same JSON line, "extras"): the FP32-mixed pass on the same
cube with its own roofline, the 4x4x4 and 40x40x4 configurations, the
parameter VJP on the 200x200x2 voided specimen, the batched 64-specimen
forward + VJP (graph against separate calls, in each precision, with tuned
launch shapes), per-kernel rooflines (live HIP-event timing of each kernel on
its launch stream), model variants, the linear solve, and the CPU oracle on
bounded samples (median of 5, all host threads and one thread).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Published MI355X vector peaks: FP64 78.6 TFLOP/s (256 CUs x 4 SIMDs x 16
# lanes x 2 flop x 2.4 GHz), FP32 157.3 TFLOP/s (packed FMA; the library is
# built without packed FP32 instructions, so 78.6 is what its FP32 code can
# reach).
FP64_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
FP32_PEAK_TFLOPS = 2 * FP64_PEAK_TFLOPS

# Counter figures of the element and assembly kernels, taken with rocprofv3 on
# the 100^3 cube (profiles/): counted VALU flops per Gauss point
# (SQ_INSTS_VALU_FLOPS_FP32/_FP64/_FP32_TRANS/_FP64_TRANS x 64 lanes / 8e6)
# and HBM bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors of
# a plain 1 GiB copy).  They hold for the kernel sources whose hash is "sha";
# once the sources differ they are reported as null.
PROFILED = {
    "sha": "8739b213676c8139",
    "fp64": {"flop_per_gp": 9155.2,
             "traffic": {"fwd_kernel": 6.051e9, "assemble_tangent": 6.759e9, "assemble_residual": 3.660e8}},
    "mixed": {"flop_per_gp": 7516.4,
              "traffic": {"fwd_kernel": 3.757e9, "assemble_tangent": 3.475e9, "assemble_residual": 3.660e8}},
}
KERNEL_SOURCES = ("paper_2606_17390_amd/csrc/forward.hip", "paper_2606_17390_amd/csrc/fem_device.h",
                  "paper_2606_17390_amd/csrc/barlat.h")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled(prec, what, kernel=None):
    """A counter figure of PROFILED if it was taken on the current sources."""
    if PROFILED["sha"] is None or PROFILED["sha"] != kernel_source_sha():
        return None
    v = PROFILED[prec][what]
    return v.get(kernel) if kernel is not None else v


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(p, nnz, prec_mixed, per_elem_cols):
    """Bytes an ideal residual + tangent + assembly pass moves through HBM,
    each input and output array once: X, d, conn, h_n, per-element
    parameters, elem_rank, row_ptr, R, K values and h_{n+1} (no element
    scratch).  On the 100^3 cube: 382 B per Gauss point in FP64, 259 in
    FP32-mixed (K values in FP32)."""
    ne, nn = p.n_elems, p.n_nodes
    ngp = 8 * ne
    kb = 4 if prec_mixed else 8
    b = 0
    b += nn * 24          # X
    b += nn * 24          # d
    b += ne * 32          # conn
    b += ngp * 56         # hist_n
    b += ne * 8 * per_elem_cols  # per-element parameters
    b += ne * 64          # elem_rank
    b += (3 * nn + 1) * 4  # row_ptr
    b += 3 * nn * 8       # R
    b += nnz * kb         # K values
    b += ngp * 56         # hist_np1
    return b


def design_bytes(p, nnz, prec_mixed, per_elem_cols, bc_row_nnz):
    """Bytes each kernel of this design's pass reads and writes once, element
    scratch (R^e, K^e) included: the design's traffic floor, not the method's
    algorithmic bytes."""
    ne, nn = p.n_elems, p.n_nodes
    ngp = 8 * ne
    kb = 4 if prec_mixed else 8
    fwd = nn * 48 + ne * 32 + ngp * 56 + ne * 8 * per_elem_cols + ngp * 56 + ne * 24 * 8 + ne * 576 * kb
    asm_k = (ne * 576 * kb + ne * 64 + ne * 8 * 4 + (nn + 1) * 4 + (3 * nn + 1) * 4 + 3 * nn
             + nnz * kb + bc_row_nnz * 4)
    asm_r = ne * 24 * 8 + ne * 8 * 4 + (nn + 1) * 4 + 3 * nn + 3 * nn * 8
    return {"fwd_kernel": fwd, "assemble_tangent": asm_k, "assemble_residual": asm_r}


def time_passes(fn, steps, warmup, torch, kernels, fem):
    """Event-timed steps; returns (ms per step, wall ms per step, {kernel id: average launch ms})."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    for k in kernels:
        fem.timing_read(k)  # drop launches of the warm-up
    fem.timing_enable(bool(kernels))  # per-launch events only where kernel times are read
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fem.timing_enable(False)
    avg = {}
    for k in kernels:
        kms, nl = fem.timing_read(k)
        avg[k] = kms / nl if nl else None
    return e0.elapsed_time(e1) / steps, wall / steps * 1e3, avg


def _cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def _median_time(fn, reps):
    import statistics
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), ts


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _sub_mesh(p, n):
    """The first n elements of a problem, its nodes renumbered."""
    import numpy as np
    conn = p.conn[:n]
    used = np.unique(conn)
    remap = -np.ones(p.n_nodes, dtype=np.int64)
    remap[used] = np.arange(used.size)
    prm = p.prm[:n] if p.prm.ndim == 2 else p.prm
    return used, remap[conn].astype(np.int32), prm, np.ascontiguousarray(p.hist_n[:, :8 * n])


def cpu_baseline(p, n_sample, n_sample_1t, reps=5):
    """The CPU oracle (FP64 residual + tangent + CSR, OpenMP over elements) on
    the first n_sample elements of the cube with every host thread, and on
    the first n_sample_1t elements with one thread; median of `reps` runs
    each.  The oracle is timed as it stands (it is the checker, not tuned)."""
    import oracle
    cores = _cores()
    res = {}
    for key, n, nt in (("all", n_sample, cores), ("one", n_sample_1t, 1)):
        used, sc, prm, hist = _sub_mesh(p, n)
        rp, ci, _ = oracle.csr_pattern(sc, used.size, with_rank=False)
        X, d = p.X[used], p.d[used]
        res[key] = _median_time(lambda: oracle.residual_tangent(X, sc, rp, ci, prm, d, hist, n_threads=nt), reps)
    t_all, ts_all = res["all"]
    t_one, ts_one = res["one"]
    return dict(value=8 * n_sample / t_all, unit="GP/s", cores=cores, kind="oracle",
                sample=f"first {n_sample} elements ({8 * n_sample} Gauss points) of the 100^3 cube, FP64 "
                       f"residual+tangent+CSR, median of {reps} runs: {t_all:.3f} s wall",
                runs_s=ts_all,
                single_thread=dict(value=8 * n_sample_1t / t_one, unit="GP/s", cores=1,
                                   sample=f"first {n_sample_1t} elements, median of {reps} runs: {t_one:.3f} s",
                                   runs_s=ts_one),
                cpu_model=_cpu_model())


def cpu_baseline_vjp(pv, n_sample_1t, reps=5):
    """The CPU oracle's parameter VJP (forward-mode App. D, OpenMP over
    elements) on the whole voided specimen with every host thread, and on its
    first n_sample_1t elements with one thread; median of `reps` runs each."""
    import oracle
    cores = _cores()
    t_all, ts_all = _median_time(lambda: oracle.residual_vjp(pv.X, pv.conn, pv.prm, pv.d, pv.hist_n, pv.lam,
                                                             n_threads=cores), reps)
    used, sc, prm, h1 = _sub_mesh(pv, n_sample_1t)
    X, d, lam = pv.X[used], pv.d[used], pv.lam[used]
    t_one, ts_one = _median_time(lambda: oracle.residual_vjp(X, sc, prm, d, h1, lam, n_threads=1), reps)
    return dict(vjp_per_s=1.0 / t_all, gp_vjp_per_s=8 * pv.n_elems / t_all, cores=cores, kind="oracle",
                sample=f"200x200x2 voided specimen ({pv.n_elems} elements), median of {reps} runs: {t_all:.3f} s",
                runs_s=ts_all,
                single_thread=dict(gp_vjp_per_s=8 * n_sample_1t / t_one, cores=1,
                                   sample=f"first {n_sample_1t} elements, median of {reps} runs: {t_one:.3f} s",
                                   runs_s=ts_one))


# The paper's forward benchmarks on these meshes, one H100, wall time in
# seconds, and what it says of the run.
PAPER_FORWARD_S = {
    (100, 100, 100): (2030.0, "2030 s on one H100 (3598 s on A100), 31 increments, 111 Newton iterations"),
    (250, 150, 120): (3.06 * 3600, "3.06 h on one H100, 122 Newton iterations"),
}


def elastic_solve(csr, torch, fem, synth):
    """The linear-elastic solve of App. F on the 100^3 unit cube (3,090,903
    dofs): the elastic tangent of the undeformed unit-cube forward problem
    (the same pattern as the benchmark cube) and the right-hand side of its
    first load increment, by CG and BiCGSTAB with the node-block preconditioner
    and with the aggregation multigrid's V-cycle, and by FGMRES with its
    K-cycle (numeric set-up inside each timed solve, the hierarchy built in
    the warm-up) to relative residuals 1e-6 and 1e-8 (seconds, iterations)."""
    p = synth.unit_cube_forward(100)
    mesh = fem.Mesh(p.X, p.conn)
    params = fem.Params(p.prm, p.n_elems, hardening="voce")
    bc = torch.as_tensor(p.bc_mask).cuda()
    d = torch.as_tensor(p.meta["bc_at"](1e-3)).cuda()
    h0 = torch.zeros((7, 8 * p.n_elems), dtype=torch.float64, device="cuda")
    # K of the undeformed cube (elastic everywhere); b = -R at the first increment's start
    out = fem.residual_tangent(mesh, csr, params, torch.zeros_like(d), h0, bc_mask=bc, prec=fem.FP64_K32)
    b = -fem.residual_tangent(mesh, csr, params, d, h0, bc_mask=bc, prec=fem.FP64, want_K=False).R
    res = {"dofs": 3 * p.n_nodes, "context": "paper App. F, same mesh, linear elastic, one H100: AMGX BiCGSTAB "
                                             "1.96 s, JAX BiCGSTAB 11.21 s (tolerance not stated)"}
    for pc, tag in ((fem.PC_BLOCK_JACOBI, ""), (fem.PC_AMG, "_amg")):
        for method in ("cg", "bicgstab") + (("fgmres",) if pc == fem.PC_AMG else ()):
            solver = fem.Solver(csr, method=method, precond=pc, bc_mask=bc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solver.solve(out.K, b, rtol=1e-2, check=False)  # warm-up (and the multigrid hierarchy)
            torch.cuda.synchronize()
            if pc == fem.PC_AMG:
                res[f"{method}{tag}_setup_s"] = time.perf_counter() - t0
            for rtol in (1e-6, 1e-8):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, its, rr = solver.solve(out.K, b, rtol=rtol, max_iter=50000, check=False)
                torch.cuda.synchronize()
                res[f"{method}{tag}_{rtol:.0e}"] = dict(seconds=time.perf_counter() - t0, iterations=its, rel_res=rr)
            del solver
    log("elastic solve: " + ", ".join(f"{k} {v['seconds']:.3f} s / {v['iterations']} it"
                                      for k, v in res.items() if isinstance(v, dict)))
    return res


def gradient_benchmark(torch, fem, synth):
    """One iteration of the inverse problem of Sec. 3.2 on the tensile-specimen
    stand-in (5,250 hex8, 45 degree orientation, ten unequal load steps):
    the forward run at the current parameters (damped Newton per step to
    1e-11 relative, FP64, linearised starts, Eisenstat-Walker tolerances)
    with its checkpoints, the objective J = w sum ||u^n - u_gt^n||^2 against
    a forward run at the reference parameters, and dJ/dtheta for the seven
    differentiated parameters (F, G, H, N, sig0, Q, b) by the time-history
    adjoint of Alg. 1.  `value` times forward + objective + adjoint."""
    import numpy as np

    from paper_2606_17390_amd import adjoint
    p = synth.tensile_specimen()
    mesh = fem.Mesh(p.X, p.conn)
    csr = fem.csr_pattern(mesh)
    bc = torch.as_tensor(p.bc_mask).cuda()
    steps = [torch.as_tensor(p.meta["bc_at"](t)).cuda() for t in p.meta["steps"]]
    h0 = torch.zeros((7, 8 * p.n_elems), dtype=torch.float64, device="cuda")
    ref = fem.Params(p.prm, p.n_elems, hardening="voce", orient=p.orient)
    prm0 = p.prm.copy()
    prm0[2:5] *= 1.05  # F, G, H
    prm0[7] *= 1.05    # N
    prm0[8:11] *= (0.95, 1.1, 0.9)  # sig0, Q, b
    cur = fem.Params(prm0, p.n_elems, hardening="voce", orient=p.orient)
    solver = fem.Solver(csr, method="cg")  # symmetric tangent (no F-bar): CG for K and K^T
    log("gradient benchmark: reference forward run")
    gt = adjoint.forward(mesh, csr, ref, bc, steps, h0, solver=solver, forcing="ew", tangent_start=True)
    w = 1.0
    adjoint.gradient(mesh, csr, cur, bc, gt, gt.d, w, solver=solver)  # warm-up of every kernel (zero cotangent)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ck = adjoint.forward(mesh, csr, cur, bc, steps, h0, solver=solver, forcing="ew", tangent_start=True)
    J = adjoint.objective(ck, gt.d, w)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    grad, _, _ = adjoint.gradient(mesh, csr, cur, bc, ck, gt.d, w, solver=solver)
    g = grad.cpu().numpy()
    t2 = time.perf_counter()
    # outside the timed region: central difference of J in Q (slot 9, gradient entry FEM_G_Q = 5)
    hq = 1e-4 * prm0[9]
    jq = []
    for sgn in (1.0, -1.0):
        pq = prm0.copy()
        pq[9] += sgn * hq
        prq = fem.Params(pq, p.n_elems, hardening="voce", orient=p.orient)
        jq.append(adjoint.objective(adjoint.forward(mesh, csr, prq, bc, steps, h0, solver=solver, forcing="ew",
                                                    tangent_start=True), gt.d, w))
    fd_q = (jq[0] - jq[1]) / (2.0 * hq)
    return {
        "metric": "inverse-iteration gradient wall time (forward + time-history adjoint)",
        "value": t2 - t0,
        "unit": "s",
        "n_gpus": 1,
        "steps": len(steps),
        "warmup": 1,
        "ms_per_step": (t2 - t0) * 1e3 / len(steps),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"tensile-specimen stand-in: {p.n_elems} hex8, {3 * p.n_nodes} dofs, 45 degree "
                               "orientation, 10 unequal load steps to 0.5 mm, Hill-48 + Voce, 7 parameters"},
        "forward_s": t1 - t0,
        "adjoint_s": t2 - t1,
        "newton_iterations": int(sum(ck.iterations)),
        "objective": J,
        "gradient": [float(v) for v in g],
        "gradient_finite": bool(np.all(np.isfinite(g))),
        "fd_check_Q": {"adjoint": float(g[5]), "central_difference": fd_q,
                       "rel_diff": abs(float(g[5]) - fd_q) / abs(fd_q)},
        "context": ("paper Sec. 3.2, its tensile specimen (5,250 hex8, 25,083 dofs, 10 steps, 6 parameters): "
                    "234 s by the JAX adjoint, 2,166 s by central differences; GPU not stated; the specimen's "
                    "shape differs from this stand-in"),
    }


def forward_benchmark(spec, torch, fem, synth, fbar=True, precond="amg", krylov="auto"):
    """The unit-cube forward simulation of the performance study, Sec. 3.1.3 (Hill-48
    from the r-values, Voce, x = 0 clamped, x = 1 moved by t (0.2, 0.1) mm)
    through the adaptive load path: FP64 residual and history, float tangent
    for the Krylov solve preconditioned by the aggregation multigrid (or the
    3x3 node-block Jacobi) with Eisenstat-Walker tolerances, convergence at
    1e-6 of the reaction norm.  The element is the
    F-bar hex8 of Sec. 2.2.4 (the paper's; unsymmetric tangent: BiCGSTAB) or
    the plain hex8 (symmetric tangent: CG)."""
    from paper_2606_17390_amd import loadpath
    dims = tuple(int(v) for v in spec.lower().split("x"))
    if len(dims) == 1:
        dims = dims * 3
    log(f"forward benchmark: unit cube {dims}")
    p = synth.unit_cube_forward(*dims)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh = fem.Mesh(p.X, p.conn)
    csr = fem.csr_pattern(mesh)
    params = fem.Params(p.prm, p.n_elems, hardening="voce", fbar=fbar)
    bc = torch.as_tensor(p.bc_mask).cuda()
    u1 = torch.as_tensor(p.meta["bc_at"](1.0)).cuda()
    h0 = torch.zeros((7, 8 * p.n_elems), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    pc = fem.PC_AMG if precond == "amg" else fem.PC_BLOCK_JACOBI
    res = loadpath.solve(mesh, csr, params, bc, u1, h0, log=lambda m: log(m), precond=pc, krylov=krylov)
    if krylov == "auto":
        krylov = fem.default_krylov(pc, fbar)
    n_it = max(res["newton_iterations"], 1)
    alpha = res["hist"][6]
    paper = PAPER_FORWARD_S.get(dims)
    return {
        "metric": "forward simulation wall time (unit-cube load path to t = 1)",
        "value": res["seconds"],
        "unit": "s",
        "n_gpus": 1,
        "steps": len(res["steps"]),
        "warmup": 0,
        "ms_per_step": res["seconds"] * 1e3 / max(len(res["steps"]), 1),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": res["seconds"] / paper[0] if paper else None,
        "dtype": "f64 (tangent f32 in the solve)",
        "data": "synthetic",
        "config": {"workload": f"unit cube {dims[0]}x{dims[1]}x{dims[2]} {'F-bar ' if fbar else ''}hex8, "
                               f"{3 * p.n_nodes} dofs, Hill-48 "
                               "r = (1.5449, 1.0666, 1, 1.0307, 1, 1), Voce sigma0 138 Q 410 b 3.8, E 219 GPa, "
                               "nu 0.3; dt0 1e-3, dt_min 1e-5, dt_max 5e-2",
                   "nnz": csr.nnz, "element": "fbar" if fbar else "plain",
                   "krylov": krylov,
                   "preconditioner": ("3x3 node-block Jacobi" if precond != "amg" else
                                      "aggregation multigrid K-cycle" if krylov == "fgmres" else
                                      "aggregation multigrid V(1,1)")},
        "increments": len(res["steps"]),
        "failed_increments": len(res["failed"]),
        "newton_iterations": res["newton_iterations"],
        "linear_iterations": res["linear_iterations"],
        "linear_solve_s": res["linear_seconds"],
        "s_per_newton_iteration": res["seconds"] / n_it,
        "setup_s": setup_s,
        "final_plastic_fraction": float((alpha > 0).double().mean().cpu()),
        "final_alpha_max": float(alpha.max().cpu()),
        "context": (f"paper, same workload: {paper[1]}, AMGX BiCGSTAB; the paper's Newton tolerance is not stated"
                    if paper else None),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the linear solve, model variants, adjoint step, batched and forward-simulation extras")
    ap.add_argument("--only", choices=("fp64", "mixed", "barlat"), default=None,
                    help="time only this pass on the cube and print its timing (for profiler runs); barlat: "
                         "the FP64 pass with the Barlat Yld2004-18p function (published AA6111 fit)")
    ap.add_argument("--no-forward", action="store_true",
                    help="skip the paper's forward simulation (about 40 s) among the extras")
    ap.add_argument("--cpu-sample", type=int, default=100000,
                    help="elements of the cube in the all-threads CPU oracle sample")
    ap.add_argument("--cpu-sample-1t", type=int, default=8000,
                    help="elements of the cube in the one-thread CPU oracle sample")
    ap.add_argument("--cpu-sample-vjp-1t", type=int, default=6000,
                    help="elements of the voided specimen in the one-thread CPU oracle VJP sample")
    ap.add_argument("--forward-benchmark", nargs="?", const="100x100x100", default=None, metavar="NXxNYxNZ",
                    help="instead of the pass benchmark: the paper's unit-cube forward simulation (adaptive load "
                         "path, Newton + BiCGSTAB) on an NX x NY x NZ mesh, one JSON line with its wall time")
    ap.add_argument("--elastic-solve", action="store_true",
                    help="instead of the pass benchmark: only the linear-elastic solves of App. F on the 100^3 cube "
                         "(the elastic_solve extra), one JSON line")
    ap.add_argument("--gradient-benchmark", action="store_true",
                    help="instead of the pass benchmark: one inverse-iteration gradient (forward + time-history "
                         "adjoint) on the tensile-specimen stand-in, one JSON line with its wall time")
    ap.add_argument("--element", choices=("fbar", "plain"), default="fbar",
                    help="element of --forward-benchmark: the paper's F-bar hex8 (BiCGSTAB) or the plain hex8 (CG)")
    ap.add_argument("--krylov", choices=("auto", "fgmres", "gmres", "bicgstab", "cg"), default="auto",
                    help="Krylov method of --forward-benchmark (auto: FGMRES with the multigrid K-cycle; with "
                         "block Jacobi BiCGSTAB for F-bar, CG for the plain element)")
    ap.add_argument("--precond", choices=("amg", "bj"), default="amg",
                    help="preconditioner of --forward-benchmark: aggregation multigrid or 3x3 node-block Jacobi")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU; sharding the path over GPUs (z-slab row ownership, "
              "one-plane halo) is described, not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_17390_amd import fem, synth

    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 4, "copy_probe_bytes_written": dst.numel() * 4}))
        return
    if args.gradient_benchmark:
        print(json.dumps(gradient_benchmark(torch, fem, synth)), flush=True)
        return
    if args.elastic_solve:
        p = synth.unit_cube_forward(100)
        csr = fem.csr_pattern(fem.Mesh(p.X, p.conn))
        print(json.dumps({"elastic_solve": elastic_solve(csr, torch, fem, synth)}), flush=True)
        return
    if args.forward_benchmark:
        print(json.dumps(forward_benchmark(args.forward_benchmark, torch, fem, synth, args.element == "fbar",
                                           args.precond, args.krylov)), flush=True)
        return
    log("generating the 100^3 cube")
    p = synth.large_cube()
    mesh = fem.Mesh(p.X, p.conn)
    params = fem.Params(p.prm, p.n_elems)
    d = torch.as_tensor(p.d).cuda()
    h = torch.as_tensor(p.hist_n).cuda()
    bc = torch.as_tensor(p.bc_mask).cuda()
    csr = fem.csr_pattern(mesh)
    # the pattern is built once per mesh (two library calls with one nnz read-back)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        fem.csr_pattern(mesh, out=csr)  # rebuilt into the same buffers
    torch.cuda.synchronize()
    ms_pattern = (time.perf_counter() - t0) / 3 * 1e3
    per_elem_cols = bin(params.per_elem_mask).count("1")
    n_gp = 8 * p.n_elems
    log(f"nnz {csr.nnz}, per-element parameter columns {per_elem_cols}")
    bc_np = p.bc_mask.astype(bool)
    rp = csr.row_ptr.cpu().numpy()
    bc_rows = np.nonzero(bc_np)[0]
    bc_row_nnz = int((rp[bc_rows + 1] - rp[bc_rows]).sum())
    KS = (fem.KERNEL_FORWARD, fem.KERNEL_ASSEMBLE_K, fem.KERNEL_ASSEMBLE_R)
    KNAMES = {fem.KERNEL_FORWARD: "fwd_kernel", fem.KERNEL_ASSEMBLE_K: "assemble_tangent",
              fem.KERNEL_ASSEMBLE_R: "assemble_residual"}
    if args.only:
        prec = fem.FP32_MIXED if args.only == "mixed" else fem.FP64
        prm_o = params
        if args.only == "barlat":
            pb = synth.with_model(p, 11, barlat=synth.BARLAT_AA6111)
            prm_o = fem.Params(pb.prm, pb.n_elems, barlat=synth.BARLAT_AA6111)
        oo = fem.Forward(mesh, csr, prec)
        ms_o, _, kt_o = time_passes(
            lambda: fem.residual_tangent(mesh, csr, prm_o, d, h, bc_mask=bc, prec=prec, out=oo),
            args.steps, args.warmup, torch, KS, fem)
        print(json.dumps({"only": args.only, "ms_per_pass": ms_o, "steps": args.steps,
                          "kernel_ms": {KNAMES[k]: kt_o[k] for k in KS}}), flush=True)
        return

    def pass_record(prec_name, ms, kt):
        """Roofline record of one pass: the pass's algorithmic bytes (382 or 259
        B per Gauss point) over the dominant kernel's launch time against HBM,
        the counted VALU flops over the same time against the published peak
        of the kernel's type, and per-kernel design bytes."""
        mixed = prec_name == "mixed"
        alg = algorithmic_bytes(p, csr.nnz, mixed, per_elem_cols)
        kb = design_bytes(p, csr.nnz, mixed, per_elem_cols, bc_row_nnz)
        kms = {KNAMES[k]: kt[k] for k in KS}
        dom = max(kms, key=lambda k: kms[k])
        fl = profiled(prec_name, "flop_per_gp")
        peak_alu = FP32_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS
        alu = None
        if fl and dom == "fwd_kernel":
            ach_f = fl * n_gp / (kms[dom] * 1e-3) / 1e12
            alu = dict(achieved=ach_f, peak=peak_alu, unit="TFLOP/s", frac=ach_f / peak_alu, flop_per_gp=fl)
        ach = alg / (kms[dom] * 1e6)
        roof = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=profiled(prec_name, "traffic", dom),
                    bytes_per_gp=alg / n_gp, n_gp=n_gp, kernel_ms=kms[dom],
                    pass_ms=ms, pass_frac=alg / (ms * 1e6) / HBM_PEAK_GBS, alu=alu,
                    binding=("alu" if alu and alu["frac"] > ach / HBM_PEAK_GBS else "hbm"))
        kernels = {}
        for name, ms_k in kms.items():
            kernels[name] = dict(kernel_ms=ms_k, design_bytes=kb[name], design_GBps=kb[name] / (ms_k * 1e6),
                                 traffic=profiled(prec_name, "traffic", name))
        return roof, kernels

    # ---- headline: FP64 residual + tangent + CSR pass
    out_d = fem.Forward(mesh, csr, fem.FP64)
    ms_d, _, kt_d = time_passes(
        lambda: fem.residual_tangent(mesh, csr, params, d, h, bc_mask=bc, prec=fem.FP64, out=out_d),
        args.steps, args.warmup, torch, KS, fem)
    plastic = float((out_d.hist[6] != h[6]).double().mean().cpu())
    diag_d = out_d.diag.cpu().tolist()
    log(f"fp64: {ms_d:.3f} ms/pass, element kernel {kt_d[fem.KERNEL_FORWARD]:.3f} ms, tangent assembly "
        f"{kt_d[fem.KERNEL_ASSEMBLE_K]:.3f} ms, residual assembly {kt_d[fem.KERNEL_ASSEMBLE_R]:.3f} ms, "
        f"plastic {plastic:.4f}, diag {diag_d}")
    roof_d, kern_d = pass_record("fp64", ms_d, kt_d)
    extras = {"csr_pattern_ms": ms_pattern, "kernels_fp64": kern_d, "kernel_source_sha": kernel_source_sha(),
              "counters_source_sha": PROFILED["sha"]}

    # ---- FP32-mixed pass on the same cube
    out_m = fem.Forward(mesh, csr, fem.FP32_MIXED)
    ms_m, _, kt_m = time_passes(
        lambda: fem.residual_tangent(mesh, csr, params, d, h, bc_mask=bc, prec=fem.FP32_MIXED, out=out_m),
        args.steps, args.warmup, torch, KS, fem)
    roof_m, kern_m = pass_record("mixed", ms_m, kt_m)
    torch.cuda.synchronize()
    km = out_m.K.double()
    err_k = float(((km - out_d.K).abs().max() / out_d.K.abs().max()).cpu())
    err_r = float(((out_m.R - out_d.R).abs().max() / out_d.R.abs().max()).cpu())
    del km
    log(f"mixed: {ms_m:.3f} ms/pass, element kernel {kt_m[fem.KERNEL_FORWARD]:.3f} ms, tangent assembly "
        f"{kt_m[fem.KERNEL_ASSEMBLE_K]:.3f} ms; mixed vs fp64 K {err_k:.2e} R {err_r:.2e}")
    extras["mixed"] = dict(gp_updates_per_s=n_gp / (ms_m * 1e-3), ms_per_pass=ms_m, dtype="f32+f64",
                           speedup_vs_fp64=ms_d / ms_m, roofline=roof_m, kernels=kern_m,
                           diag=out_m.diag.cpu().tolist(), rel_err_vs_fp64=dict(K=err_k, R=err_r))
    del out_d
    torch.cuda.empty_cache()

    # ---- the small configurations: 4x4x4 unit cube and the 40x40x4 sheet slab
    small = {}
    for cname, pc in (("tiny_cube_4x4x4", synth.tiny_cube()), ("sheet_slab_40x40x4", synth.sheet_slab())):
        mc = fem.Mesh(pc.X, pc.conn)
        cc = fem.csr_pattern(mc)
        prc = fem.Params(pc.prm, pc.n_elems)
        dc, hc = torch.as_tensor(pc.d).cuda(), torch.as_tensor(pc.hist_n).cuda()
        bcc, lc = torch.as_tensor(pc.bc_mask).cuda(), torch.as_tensor(pc.lam).cuda()
        row = dict(n_elems=pc.n_elems, dofs=3 * pc.n_nodes, nnz=cc.nnz)
        for pn, pr in (("fp64", fem.FP64), ("mixed", fem.FP32_MIXED)):
            oc = fem.Forward(mc, cc, pr)
            ms_c, _, _ = time_passes(lambda: fem.residual_tangent(mc, cc, prc, dc, hc, bc_mask=bcc, prec=pr, out=oc),
                                     max(args.steps, 20), 5, torch, (), fem)
            vo = fem.Vjp(mc)
            ms_v, _, _ = time_passes(lambda: fem.residual_vjp(mc, prc, dc, hc, lc, prec=pr, out=vo),
                                     max(args.steps, 20), 5, torch, (), fem)
            row[pn] = dict(ms_per_pass=ms_c, gp_updates_per_s=8 * pc.n_elems / (ms_c * 1e-3), ms_per_vjp=ms_v,
                           vjp_per_s=1e3 / ms_v)
        small[cname] = row
        log(f"{cname}: fp64 {row['fp64']['ms_per_pass']:.3f} ms, mixed {row['mixed']['ms_per_pass']:.3f} ms per pass")
    extras["small_configs"] = small

    if not args.no_extras:
        # ---- linear solve of a Newton iteration on the same system (FP32 K)
        solver = fem.Solver(csr)
        xv = torch.ones(csr.n_rows, dtype=torch.float64, device="cuda")
        yv = torch.empty_like(xv)
        for _ in range(3):
            fem.csr_spmv(csr, out_m.K, xv, yv)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fem.csr_spmv(csr, out_m.K, xv, yv)
        e1.record()
        torch.cuda.synchronize()
        ms_spmv = e0.elapsed_time(e1) / 10
        # FP32 values, the column list once per node (shared by its 3 rows), row_ptr, x and y once
        spmv_bytes = csr.nnz * 4 + csr.nnz // 3 * 4 + (csr.n_rows + 1) * 4 + 2 * csr.n_rows * 8
        rhs = -out_m.R
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, its, res = solver.solve(out_m.K, rhs, rtol=0.0, max_iter=64, check=False)
        torch.cuda.synchronize()
        ms_it = (time.perf_counter() - t0) * 1e3 / max(its, 1)
        extras["linear_solve"] = dict(spmv_ms=ms_spmv, spmv_GBps=spmv_bytes / (ms_spmv * 1e6),
                                      spmv_hbm_frac=spmv_bytes / (ms_spmv * 1e6) / HBM_PEAK_GBS,
                                      bicgstab_ms_per_iteration=ms_it, bicgstab_rel_res_after_64=res)
        log(f"spmv {ms_spmv:.3f} ms ({spmv_bytes / (ms_spmv * 1e6):.0f} GB/s), bicgstab {ms_it:.3f} ms/iteration")
        del solver, xv, yv, rhs
        extras["elastic_solve"] = elastic_solve(csr, torch, fem, synth)

        # ---- model variants on the same cube (FP32-mixed): Voce hardening, one
        # orientation per element (in-plane angles), the F-bar element, all
        # three, and the Barlat yield function (FP64 element kernel)
        variants = {}
        for vname, hard, fbar, orient, bar in (("voce", "voce", False, None, None),
                                               ("orient_per_elem", "swift", False, "per_element", None),
                                               ("fbar", "swift", True, None, None),
                                               ("fbar_voce_orient", "voce", True, "per_element", None),
                                               ("barlat_aa6111", "swift", False, None, synth.BARLAT_AA6111)):
            pm = synth.with_model(p, 11, hard, fbar, orient, barlat=bar)
            vparams = fem.Params(pm.prm, pm.n_elems, hardening=hard, fbar=fbar, orient=pm.orient, barlat=bar)
            ms_v, _, kt_v = time_passes(
                lambda: fem.residual_tangent(mesh, csr, vparams, d, h, bc_mask=bc, prec=fem.FP32_MIXED, out=out_m),
                max(args.steps // 2, 3), 2, torch, KS, fem)
            variants[vname] = dict(ms_per_pass=ms_v, gp_updates_per_s=n_gp / (ms_v * 1e-3),
                                   fwd_kernel_ms=kt_v[fem.KERNEL_FORWARD],
                                   plastic_fraction=float((out_m.hist[6] != h[6]).double().mean().cpu()))
            log(f"mixed {vname}: {ms_v:.3f} ms/pass, element kernel {kt_v[fem.KERNEL_FORWARD]:.3f} ms")
            del vparams, pm
        extras["mixed_model_variants"] = variants
        torch.cuda.empty_cache()

        # ---- one step of the time-history adjoint on the same cube (FP64):
        # the local-adjoint kernel for (lambda, mu), and K^T for the adjoint solve
        gen = torch.Generator(device="cuda").manual_seed(5)
        lam_c = torch.randn((p.n_nodes, 3), dtype=torch.float64, device="cuda", generator=gen)
        mu_c = torch.randn((7, n_gp), dtype=torch.float64, device="cuda", generator=gen)
        adj = fem.HistoryAdjoint(mesh)

        def timed(fn, reps=5):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        ms_adj = timed(lambda: fem.history_adjoint(mesh, csr, params, d, h, lam=lam_c, mu=mu_c, out=adj))
        ms_adj_mu = timed(lambda: fem.history_adjoint(mesh, csr, params, d, h, lam=None, mu=mu_c, out=adj,
                                                      want_hbar=False))
        KT = torch.empty_like(out_m.K)
        ms_tr = timed(lambda: fem.csr_transpose(csr, out_m.K, bc_mask=bc, out=KT))
        extras["history_adjoint_step"] = dict(
            ms_lambda_mu=ms_adj, gp_per_s=n_gp / (ms_adj * 1e-3), ms_mu_ubar=ms_adj_mu, ms_transpose_f32=ms_tr,
            transpose_GBps=(2 * csr.nnz * 4 + csr.nnz // 3 * 4) / (ms_tr * 1e6))
        log(f"history adjoint step: {ms_adj:.3f} ms (lambda, mu -> g, hbar), {ms_adj_mu:.3f} ms (mu -> ubar), "
            f"K^T {ms_tr:.3f} ms")
        del lam_c, mu_c, adj, KT
        torch.cuda.empty_cache()

    # ---- VJP on the voided specimen
    pv = synth.void_specimen()
    mv = fem.Mesh(pv.X, pv.conn)
    pv_params = fem.Params(pv.prm, pv.n_elems)
    dv = torch.as_tensor(pv.d).cuda()
    hv = torch.as_tensor(pv.hist_n).cuda()
    lv = torch.as_tensor(pv.lam).cuda()
    vj = {}
    for name, prec in (("fp64", fem.FP64), ("mixed", fem.FP32_MIXED)):
        vo = fem.Vjp(mv)
        ms_v, _, kt_v = time_passes(
            lambda: fem.residual_vjp(mv, pv_params, dv, hv, lv, prec=prec, out=vo),
            args.steps, args.warmup, torch, (fem.KERNEL_VJP,), fem)
        kms_v = kt_v[fem.KERNEL_VJP]
        vj[name] = dict(vjp_per_s=1e3 / ms_v, gp_vjp_per_s=8 * pv.n_elems / (ms_v * 1e-3), ms_per_vjp=ms_v,
                        kernel_ms=kms_v)
        log(f"vjp {name}: {ms_v:.3f} ms")
    extras["vjp_void_specimen"] = dict(n_elems=pv.n_elems, **vj)

    if not args.no_extras:
        extras["batched_64"] = batched_benchmark(args, torch, fem, synth)
        if not args.no_forward:
            # the paper's forward simulation of Sec. 3.1.3 end to end (F-bar element), after the timed pass
            try:
                fw = forward_benchmark("100x100x100", torch, fem, synth, True)
                extras["forward_simulation"] = {k: fw[k] for k in (
                    "metric", "value", "unit", "config", "increments", "failed_increments", "newton_iterations",
                    "linear_iterations", "linear_solve_s", "vs_baseline", "context")}
            except RuntimeError as err:
                extras["forward_simulation"] = {"error": str(err)}

    if not args.no_cpu_baseline:
        log("cpu baseline")
        result_cpu = cpu_baseline(p, args.cpu_sample, args.cpu_sample_1t)
        result_cpu["vjp"] = cpu_baseline_vjp(pv, args.cpu_sample_vjp_1t)
        log(f"cpu baseline: {result_cpu['value']:.3e} GP/s on {result_cpu['cores']} threads, "
            f"{result_cpu['single_thread']['value']:.3e} GP/s on one")
    else:
        result_cpu = None
    result = {
        "metric": "Gauss-point updates/s (residual + tangent + CSR assembly), FP64",
        "value": n_gp / (ms_d * 1e-3),
        "unit": "GP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_d,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "large_cube 100x100x100 hex8, 1e6 elements, 3,090,903 dofs, 8e6 Gauss points, "
                               "per-element Hill-48 fields, 30% plastic at trial, x=0 face constrained",
                   "n_elems": p.n_elems, "nnz": csr.nnz, "plastic_fraction": plastic, "diag": diag_d},
        "roofline": roof_d,
        "cpu_baseline": result_cpu,
        "extras": extras,
    }
    print(json.dumps(result), flush=True)


def batched_benchmark(args, torch, fem, synth):
    """64 uneven specimens, forward + VJP: one graph replay of the batched
    calls against 64 separate eager calls per specimen, in FP64 and in
    FP32-mixed (like for like), after the autotuner has picked the element
    kernels' launch shapes for the batched workload in each precision."""
    from paper_2606_17390_amd import tune
    specs = synth.batch64()
    mb = synth.concat(specs)
    bmesh = fem.Mesh(mb.X, mb.conn)
    bcsr = fem.csr_pattern(bmesh)
    bparams = fem.Params(mb.meta["spec_prm"], mb.n_elems, per_spec=True)
    batch = fem.Batch(mb.meta["elem_off"])
    bd = torch.as_tensor(mb.d).cuda()
    bh = torch.as_tensor(mb.hist_n).cuda()
    bl = torch.as_tensor(mb.lam).cuda()
    bbc = torch.as_tensor(mb.bc_mask).cuda()
    sep = []
    for s in specs:
        ms_ = fem.Mesh(s.X, s.conn)
        sep.append((ms_, fem.csr_pattern(ms_), fem.Params(s.prm, s.n_elems), torch.as_tensor(s.d).cuda(),
                    torch.as_tensor(s.hist_n).cuda(), torch.as_tensor(s.lam).cuda(),
                    torch.as_tensor(s.bc_mask).cuda()))
    res = dict(n_spec=len(specs), n_elems=mb.n_elems)
    st = torch.cuda.Stream()
    for pname, prec in (("fp64", fem.FP64), ("mixed", fem.FP32_MIXED)):
        tf = tune.tune_forward(bmesh, bcsr, bparams, bd, bh, prec=prec, bc_mask=bbc, batch=batch, use_cache=False)
        tv = tune.tune_vjp(bmesh, bparams, bd, bh, bl, prec=prec, batch=batch, use_cache=False)
        tuned = dict(forward=dict(block=tf[1], waves_per_cu=tf[2], xcd_remap=tf[3], kernel_ms=tf[0]),
                     vjp=dict(block=tv[1], waves_per_cu=tv[2], xcd_remap=tv[3], kernel_ms=tv[0]))
        bo = fem.Forward(bmesh, bcsr, prec)
        bvo = fem.Vjp(bmesh, batch.n_spec)
        g = fem.Graph()
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            with g.capture(st):
                fem.residual_tangent(bmesh, bcsr, bparams, bd, bh, bc_mask=bbc, prec=prec, out=bo, batch=batch,
                                     stream=st)
                fem.residual_vjp(bmesh, bparams, bd, bh, bl, prec=prec, out=bvo, batch=batch, stream=st)
            for _ in range(3):
                g.replay(st)
            st.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(args.steps):
                g.replay(st)
            e1.record(st)
            st.synchronize()
        ms_g = e0.elapsed_time(e1) / args.steps
        sep_out = [(fem.Forward(a[0], a[1], prec), fem.Vjp(a[0])) for a in sep]

        def run_sep():
            for (ms_, cs, pr, dd, hh, ll, bb), (fo, vo) in zip(sep, sep_out):
                fem.residual_tangent(ms_, cs, pr, dd, hh, bc_mask=bb, prec=prec, out=fo)
                fem.residual_vjp(ms_, pr, dd, hh, ll, prec=prec, out=vo)
        ms_sep, _, _ = time_passes(run_sep, max(args.steps // 4, 3), 2, torch, (), fem)
        res[pname] = dict(ms_graph_fwd_vjp=ms_g, ms_64_separate_calls=ms_sep, graph_speedup=ms_sep / ms_g,
                          specimen_fwd_vjp_per_s=len(specs) / (ms_g * 1e-3),
                          gp_updates_per_s=8 * mb.n_elems / (ms_g * 1e-3), tuned_launch=tuned)
        log(f"batched {pname}: graph {ms_g:.3f} ms vs 64 separate calls {ms_sep:.3f} ms; tuned forward "
            f"{tf[1:]} vjp {tv[1:]}")
        del bo, bvo, g, sep_out
        fem.set_launch(fem.KERNEL_FORWARD, prec)
        fem.set_launch(fem.KERNEL_VJP, prec)
    res["mixed_vs_fp64_graph_speedup"] = res["fp64"]["ms_graph_fwd_vjp"] / res["mixed"]["ms_graph_fwd_vjp"]
    return res


if __name__ == "__main__":
    main()
