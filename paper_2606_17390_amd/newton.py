"""Global Newton iteration of one load step on the GPU (Sec. 2.2.4): find d
with R(d; h_n) = 0 for the history h_n of the last converged step, solving
K du = -R with fem_solve at every iteration.  Constrained dofs carry their
prescribed values in d before the call; their rows of R are zero and of K
identity rows (App. E), so du vanishes there.

    from paper_2606_17390_amd import fem, newton
    hist_np1, its, norms = newton.solve_step(mesh, csr, params, d, hist_n, bc_mask)

The Newton step is damped by backtracking on ||R|| (halving the step until
||R|| decreases by the factor 1 - 1e-4 t): full steps from a poor start can
wander (the F-bar element shows it on a load step that starts from the
previous solution).  Every trial point is evaluated with its tangent, so an
accepted full step costs no extra pass.  The linear solve may stop short of
lin_rtol (stagnation of BiCGSTAB at its attainable accuracy): an inexact
direction only slows Newton down, so any finite solve with a relative
residual below 1e-3 is used.

With forcing="ew" the linear tolerance follows the Eisenstat-Walker rule
(their choice 2, gamma 0.9, exponent 2): eta_k = 0.9 (||R_k|| /
||R_k-1||)^2, safeguarded by 0.9 eta_k-1^2 when that exceeds 0.1, capped at
eta_max, and never tighter than lin_rtol or than half the distance to the
Newton target: the early, far-from-converged iterations get loose solves.
The first iteration uses eta0 (default eta_max).  forcing="const" keeps
eta_max throughout (the same floors): Newton then contracts by about eta_max
per iteration, for solves that stop at the cheap first decades.

Every step runs in the library (residual, tangent, assembly, linear solve);
this module only sequences the calls and reads the residual norm back.
"""
import math
import time

from . import fem


def solve_step(mesh, csr, params, d, hist_n, bc_mask, prec=fem.FP64, tol=1e-10, max_it=30, lin_rtol=1e-10,
               lin_max_iter=5000, solver=None, out=None, stream=None, line_search=True, max_backtracks=8, atol=0.0,
               trace=None, forcing=None, eta_max=0.1, eta0=None, stall_window=0, stall_ratio=0.5):
    """Newton iteration on d (device [n_nodes][3], updated in place) until
    ||R|| <= max(tol ||R_0||, atol); with stall_window > 0 it also gives up
    once ||R|| has not fallen by the factor stall_ratio over that many
    iterations.  Returns (hist_np1, iterations, list of
    ||R||).  Raises RuntimeError if the tolerance is not reached in max_it
    iterations, a linear solve fails or ||R|| is not finite.  solver: a
    fem.Solver of the pattern (default flexible GMRES preconditioned by the
    aggregation multigrid's K-cycle, built for bc_mask).  A list passed
    as trace receives one (linear iterations, linear relative residual, step
    length, seconds in the linear solve, linear tolerance) tuple per Newton
    iteration."""
    if out is None:
        out = fem.Forward(mesh, csr, prec)
    if solver is None:
        solver = fem.Solver(csr, d.device, precond=fem.PC_AMG, method="fgmres", bc_mask=bc_mask)
    flat = d.view(-1)

    def evaluate():
        fem.residual_tangent(mesh, csr, params, d, hist_n, bc_mask=bc_mask, prec=prec, out=out, stream=stream)
        return float(out.rnorm2.sqrt().cpu())

    norms = []
    rn = evaluate()
    for it in range(max_it + 1):
        norms.append(rn)
        if not math.isfinite(rn):
            raise RuntimeError(f"Newton: ||R|| is not finite at iteration {it}")
        if rn == 0.0 or rn <= max(tol * norms[0], atol):
            return out.hist.clone(), it, norms
        if it == max_it:
            break
        if stall_window and it >= stall_window and rn > stall_ratio * norms[-1 - stall_window]:
            raise RuntimeError(f"Newton: stalled at ||R|| = {rn:.3e} after {it} iterations (start {norms[0]:.3e}; "
                               + " ".join(f"{r:.1e}" for r in norms) + ")")
        rt = lin_rtol
        if forcing in ("ew", "const"):
            if it == 0:
                eta = eta_max if eta0 is None else eta0
            elif forcing == "const":
                eta = eta_max
            else:
                e = 0.9 * (rn / norms[-2]) ** 2
                if 0.9 * eta * eta > 0.1:
                    e = max(e, 0.9 * eta * eta)
                eta = min(eta_max, e)
            rt = max(lin_rtol, min(eta_max, max(eta, 0.5 * max(tol * norms[0], atol) / rn)))
        elif forcing is not None:
            raise ValueError(f"forcing must be None, 'ew' or 'const', not {forcing!r}")
        t_lin = time.perf_counter()
        du, lin_its, res = solver.solve(out.K, -out.R, rtol=rt, max_iter=lin_max_iter, stream=stream, check=False)
        if not (res <= max(1e-3, rt)) and solver.method == fem.KRYLOV["cg"]:
            # CG stops on a direction of non-positive curvature: BiCGSTAB instead
            du, its2, res = solver.solve(out.K, -out.R, rtol=rt, max_iter=lin_max_iter, stream=stream, check=False,
                                         method="bicgstab")
            lin_its += its2
        t_lin = time.perf_counter() - t_lin
        if not (res <= max(1e-3, rt)):
            raise RuntimeError(f"Newton: linear solve reached only a relative residual of {res:.3e}")
        base = flat.clone()
        t = 1.0
        for k in range(max_backtracks + 1):
            flat.copy_(base)
            flat.add_(du, alpha=t)
            rn_new = evaluate()
            if not line_search or rn_new < (1.0 - 1e-4 * t) * rn or k == max_backtracks:
                break
            t *= 0.5
        if trace is not None:
            trace.append((lin_its, res, t, t_lin, rt))
        rn = rn_new
    raise RuntimeError(f"Newton: ||R|| = {norms[-1]:.3e} after {max_it} iterations (start {norms[0]:.3e}; "
                       + " ".join(f"{r:.1e}" for r in norms) + ")")
