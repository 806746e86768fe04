"""Global Newton iteration of one load step on the GPU (Sec. 2.2.4): find d
with R(d; h_n) = 0 for the history h_n of the last converged step, solving
K du = -R with fem_solve at every iteration.  Constrained dofs carry their
prescribed values in d before the call; their rows of R are zero and of K
identity rows (App. E), so du vanishes there.

    from paper_2606_17390_amd import fem, newton
    hist_np1, its, norms = newton.solve_step(mesh, csr, params, d, hist_n, bc_mask)

Every step runs in the library (residual, tangent, assembly, linear solve);
this module only sequences the calls and reads the residual norm back.
"""
from . import fem


def solve_step(mesh, csr, params, d, hist_n, bc_mask, prec=fem.FP64, tol=1e-10, max_it=30, lin_rtol=1e-12,
               lin_max_iter=20000, solver=None, out=None, stream=None):
    """Newton iteration on d (device [n_nodes][3], updated in place) until
    ||R|| <= tol ||R_0||.  Returns (hist_np1, iterations, list of ||R||).
    Raises RuntimeError if the tolerance is not reached in max_it iterations."""
    if out is None:
        out = fem.Forward(mesh, csr, prec)
    if solver is None:
        solver = fem.Solver(csr, d.device)
    norms = []
    flat = d.view(-1)
    for it in range(max_it + 1):
        fem.residual_tangent(mesh, csr, params, d, hist_n, bc_mask=bc_mask, prec=prec, out=out, stream=stream)
        rn = float(out.rnorm2.sqrt().cpu())
        norms.append(rn)
        if rn == 0.0 or rn <= tol * norms[0]:
            return out.hist.clone(), it, norms
        if it == max_it:
            break
        du, _, _ = solver.solve(out.K, -out.R, rtol=lin_rtol, max_iter=lin_max_iter, stream=stream)
        flat.add_(du)
    raise RuntimeError(f"Newton: ||R|| = {norms[-1]:.3e} after {max_it} iterations (start {norms[0]:.3e})")
