"""Quasi-static load path on the GPU: load factor t from 0 to t_end in
adaptive increments, each solved by the damped Newton iteration of newton.py
(Sec. 2.2.4: R(d; h_n) = 0 with the history of the last converged increment),
with the automatic stepping of Sec. 2.2.5:

* prescribed values t u1 on the constrained dofs (a load proportional to t);
* the Newton start of an increment is the linear extrapolation of the two
  last converged solutions; before two exist, the solution of the problem
  linearised about the converged state with the boundary increment
  (tangent_start; else the converged solution with the boundary increment);
* a failed increment (no convergence in max_it iterations, a residual that
  has not halved over the last stall_window iterations, a non-finite
  residual) is retried with dt times `cutback`, down to dt_min; after
  `grow_after` converged increments in a row dt grows by `grow`, up to
  dt_max;
* convergence: ||R|| <= ftol f_ref, f_ref the largest norm of the reactions
  (the unconstrained residual on the constrained dofs) met so far, or of the
  first increment's starting residual before any reaction exists;
* linear solves (krylov="auto") by flexible GMRES with the multigrid
  K-cycle, or with block Jacobi by conjugate gradients where the tangent is
  symmetric (every model but F-bar; BiCGSTAB for F-bar, and where CG meets a
  direction of non-positive curvature), to the Eisenstat-Walker tolerance of
  newton.py (floor lin_rtol) unless forcing is None (then lin_rtol
  throughout); the linear
  step of the tangent start, or without it the first solve of an increment
  with no extrapolated start, goes to first_eta, since that direction
  carries the whole boundary increment; preconditioner: the aggregation
  multigrid (precond=fem.PC_AMG: hierarchy built at the first solve,
  numeric set-up for every tangent) or fem.PC_BLOCK_JACOBI.

The performance study of Sec. 3.1.3 uses dt0 1e-3, dt_min 1e-5, dt_max 5e-2.

    res = loadpath.solve(mesh, csr, params, bc_mask, u1, hist0)
"""
import time

import torch

from . import fem, newton


def _sync(dev):
    if dev.type == "cuda":
        torch.cuda.synchronize(dev)


def reaction_norm(mesh, csr, params, d, hist, bc, prec=fem.FP64):
    """Norm of the internal force on the constrained dofs (flat bool mask bc)."""
    r = fem.residual_tangent(mesh, csr, params, d, hist, bc_mask=None, prec=prec, want_K=False, want_hist=False)
    return float(r.R[bc].norm().cpu())


def linearised_start(mesh, csr, params, d, h, trial, bc_mask, prec, out, solver, rtol, max_iter):
    """Moves `trial` (the converged solution d with the boundary increment on
    the constrained dofs) to the solution of the problem linearised about the
    converged state (d, h): K_n du = -(R_n + K_n delta) on the free dofs,
    delta = trial - d, solved to rtol.  Starting Newton from the boundary
    increment alone lets the elements along the moved boundary take the whole
    increment and yield.  `out` (a Forward of this pattern) is overwritten.
    Returns the linear iterations and the norm of the right-hand side (the
    force scale of the increment)."""
    bc = bc_mask.bool().view(-1)
    fem.residual_tangent(mesh, csr, params, d, h, bc_mask=bc_mask, prec=prec, out=out)
    rhs = fem.csr_spmv(csr, out.K, (trial - d).view(-1))
    rhs.add_(out.R).neg_()
    rhs[bc] = 0.0
    du, its, _ = solver.solve(out.K, rhs, rtol=rtol, max_iter=max_iter, check=False)
    trial.view(-1).add_(du)
    return its, float(rhs.norm().cpu())


def solve(mesh, csr, params, bc_mask, u1, hist0, prec=fem.FP64_K32, dt0=1e-3, dt_min=1e-5, dt_max=5e-2, grow=2.0,
          grow_after=1, cutback=0.5, ftol=1e-6, max_it=30, stall_window=5, stall_ratio=0.5, lin_rtol=1e-6,
          lin_max_iter=20000, t_end=1.0, max_steps=10000, log=None, precond=fem.PC_AMG, forcing="ew",
          first_eta=1e-4, eta_max=0.1, krylov="auto", line_search=True, tangent_start=True):
    """Returns a dict with the final displacement and history, the accepted
    increments [(t, dt, Newton iterations, linear iterations)], the failed
    increments, the total Newton and linear iterations, the wall time and
    the part of it spent in linear solves."""
    dev = hist0.device
    bc = bc_mask.bool().view(-1)
    out = fem.Forward(mesh, csr, prec)
    if krylov == "auto":
        krylov = fem.default_krylov(precond, params.model & fem.MODEL_FBAR)
    solver = fem.Solver(csr, dev, precond=precond, method=krylov, bc_mask=bc_mask)
    d = torch.zeros((mesh.n_nodes, 3), dtype=torch.float64, device=dev)
    d_prev, dt_prev = None, None
    h = hist0.clone()
    u1f = u1.reshape(-1)
    t, dt = 0.0, dt0
    f_ref = 0.0
    steps, failed, newton_its, lin_its, streak, lin_s = [], [], 0, 0, 0, 0.0
    _sync(dev)
    t0 = time.perf_counter()
    while t < t_end * (1 - 1e-12) and len(steps) < max_steps:
        dt = min(dt, t_end - t)
        trial = d.clone()
        if d_prev is not None:
            trial.add_(d - d_prev, alpha=dt / dt_prev)
        trial.view(-1)[bc] = (t + dt) * u1f[bc]
        trace = []
        if d_prev is None and tangent_start:
            t_lin = time.perf_counter()
            lin_its += linearised_start(mesh, csr, params, d, h, trial, bc_mask, prec, out, solver, first_eta,
                                        lin_max_iter)[0]
            lin_s += time.perf_counter() - t_lin
        try:
            h_new, its, norms = newton.solve_step(mesh, csr, params, trial, h, bc_mask, prec=prec,
                                                  tol=ftol if f_ref == 0.0 else 0.0, atol=ftol * f_ref,
                                                  max_it=max_it, lin_rtol=lin_rtol, lin_max_iter=lin_max_iter,
                                                  solver=solver, out=out, trace=trace, forcing=forcing,
                                                  eta0=None if d_prev is not None or tangent_start else first_eta,
                                                  line_search=line_search, stall_window=stall_window,
                                                  stall_ratio=stall_ratio, eta_max=eta_max)
        except RuntimeError as err:
            failed.append((t, dt, str(err)))
            if log:
                log(f"increment t={t:.5f} dt={dt:.2e} failed: {err} | linear "
                    + " ".join(f"{x[0]}@{x[4]:.0e}" for x in trace)
                    + " | steps " + " ".join(f"{x[2]:g}" for x in trace))
            dt *= cutback
            streak = 0
            if dt < dt_min:
                raise RuntimeError(f"load path: increment below {dt_min:g} at t = {t:.5f}") from err
            continue
        finally:
            lin_its += sum(x[0] for x in trace)
            lin_s += sum(x[3] for x in trace)
        d_prev, dt_prev = d, dt
        d, h = trial, h_new
        t += dt
        newton_its += its
        f_reac = reaction_norm(mesh, csr, params, d, h_new, bc)
        f_ref = max(f_ref, f_reac)
        steps.append((t, dt, its, sum(x[0] for x in trace)))
        if log:
            log(f"t={t:.5f} dt={dt:.2e} Newton {its} reaction {f_reac:.3e} ||R|| "
                + " ".join(f"{r:.1e}" for r in norms)
                + " | linear " + " ".join(f"{x[0]}@{x[4]:.0e}" for x in trace)
                + " | steps " + " ".join(f"{x[2]:g}" for x in trace))
        streak += 1
        if streak >= grow_after:
            dt = min(dt * grow, dt_max)
            streak = 0
    _sync(dev)
    return dict(d=d, hist=h, steps=steps, failed=failed, newton_iterations=newton_its, linear_iterations=lin_its,
                linear_seconds=lin_s, seconds=time.perf_counter() - t0)
