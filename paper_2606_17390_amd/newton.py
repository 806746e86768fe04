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

Every step runs in the library (residual, tangent, assembly, linear solve);
this module only sequences the calls and reads the residual norm back.
"""
import math

from . import fem


def solve_step(mesh, csr, params, d, hist_n, bc_mask, prec=fem.FP64, tol=1e-10, max_it=30, lin_rtol=1e-10,
               lin_max_iter=5000, solver=None, out=None, stream=None, line_search=True, max_backtracks=8, atol=0.0,
               trace=None):
    """Newton iteration on d (device [n_nodes][3], updated in place) until
    ||R|| <= max(tol ||R_0||, atol).  Returns (hist_np1, iterations, list of
    ||R||).  Raises RuntimeError if the tolerance is not reached in max_it
    iterations, a linear solve fails or ||R|| is not finite.  A list passed
    as trace receives one (linear iterations, linear relative residual, step
    length) tuple per Newton iteration."""
    if out is None:
        out = fem.Forward(mesh, csr, prec)
    if solver is None:
        solver = fem.Solver(csr, d.device)
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
        du, lin_its, res = solver.solve(out.K, -out.R, rtol=lin_rtol, max_iter=lin_max_iter, stream=stream, check=False)
        if not (res <= 1e-3):
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
            trace.append((lin_its, res, t))
        rn = rn_new
    raise RuntimeError(f"Newton: ||R|| = {norms[-1]:.3e} after {max_it} iterations (start {norms[0]:.3e})")
