"""Time-history adjoint on the GPU (Sec. 2.3, Eqs. (Lagrangian)-(dR_u), Alg. 1).

The forward pass solves every load step with the damped Newton driver and
keeps the checkpoints H[n] = (u^n, h^n) in device memory.  The backward pass
runs from the last step with mu^{N_T} = 0:

    ubar   = mu^n^T dH^n/du^n                          (fem_history_adjoint)
    K^n^T lambda^n = -(2 w (u^n - u_gt^n) + ubar)      (fem_solve; fem_csr_transpose for F-bar)
    g     += lambda^n^T dR^n/dtheta + mu^n^T dH^n/dtheta
    mu^{n-1} = lambda^n^T dR^n/dh^{n-1} + mu^n^T dH^n/dh^{n-1}

for the objective J = w sum_n ||u^n - u_gt^n||^2 of Eq. (J).  Constrained
dofs are prescribed: their rows of K^T are identity rows and their
right-hand side is zero, so lambda vanishes there.  The system is then the
free-free block K_ff^T lambda_f = b_f, and for a symmetric tangent (every
element but F-bar) K_ff^T = K_ff: the assembled K itself is solved (its
constrained rows are identity rows too) and no transpose is formed.  Every
step runs in the library; this module sequences the calls.

    ck = adjoint.forward(mesh, csr, params, bc_mask, bc_steps, hist0)
    J, grad = adjoint.objective(ck, u_gt, w), adjoint.gradient(mesh, csr, params, bc_mask, ck, u_gt, w)[0]
"""
import torch

from . import fem, loadpath, newton


class Checkpoints:
    """u^n and h^n of every load step (device tensors); h[0] is the initial history."""

    def __init__(self, hist0):
        self.d = []
        self.h = [hist0.clone()]
        self.iterations = []


def forward(mesh, csr, params, bc_mask, bc_steps, hist0, prec=fem.FP64, tol=1e-11, max_it=40, solver=None,
            lin_rtol=1e-10, lin_max_iter=20000, forcing=None, tangent_start=False):
    """Solve the load steps; bc_steps[n] (device [n_nodes, 3]) holds the prescribed
    values of the constrained dofs at step n.  forcing="ew": Eisenstat-Walker
    linear tolerances (floor lin_rtol); tangent_start: each step starts from
    the problem linearised about the previous converged state
    (loadpath.linearised_start, solved to 1e-4) instead of the previous
    solution with the new boundary values.  The default solver is flexible
    GMRES with the aggregation multigrid's K-cycle (also for gradient)."""
    ck = Checkpoints(hist0)
    out = fem.Forward(mesh, csr, prec)
    solver = solver or fem.Solver(csr, hist0.device, precond=fem.PC_AMG, method="fgmres", bc_mask=bc_mask)
    d = torch.zeros((mesh.n_nodes, 3), dtype=torch.float64, device=hist0.device)
    bc = bc_mask.bool().view(-1)
    for ub in bc_steps:
        d_prev = d.clone() if tangent_start else None
        d.view(-1)[bc] = ub.reshape(-1)[bc]
        rtol, atol = tol, 0.0
        if tangent_start:
            # the tolerance is taken relative to the increment's force scale,
            # not to the (already small) residual of the linearised start
            _, f_inc = loadpath.linearised_start(mesh, csr, params, d_prev, ck.h[-1], d, bc_mask, prec, out, solver,
                                                 1e-4, lin_max_iter)
            rtol, atol = 0.0, tol * f_inc
        hist, its, _ = newton.solve_step(mesh, csr, params, d, ck.h[-1], bc_mask, prec=prec, tol=rtol, atol=atol,
                                         max_it=max_it, solver=solver, out=out, lin_rtol=lin_rtol,
                                         lin_max_iter=lin_max_iter, forcing=forcing)
        ck.d.append(d.clone())
        ck.h.append(hist)
        ck.iterations.append(its)
    return ck


def objective(ck, u_gt, w):
    return float(sum(w * torch.sum((d - g) ** 2) for d, g in zip(ck.d, u_gt)))


def gradient(mesh, csr, params, bc_mask, ck, u_gt, w, lin_rtol=1e-12, lin_max_iter=20000, solver=None):
    """dJ/dtheta [7] (sum over elements; per-element parameters: the element
    gradients are summed per step into g_elem_total) and the multipliers lambda^n."""
    dev = ck.h[0].device
    solver = solver or fem.Solver(csr, dev, precond=fem.PC_AMG, method="fgmres", bc_mask=bc_mask)
    fwd = fem.Forward(mesh, csr, fem.FP64)
    adj = fem.HistoryAdjoint(mesh)
    bc = bc_mask.bool().view(-1)
    mu = torch.zeros_like(ck.h[0])
    grad = torch.zeros(fem.NGRAD, dtype=torch.float64, device=dev)
    g_elem = torch.zeros((fem.NGRAD, mesh.n_elems), dtype=torch.float64, device=dev)
    KT = None
    symmetric = (params.model & fem.MODEL_FBAR) == 0
    lams = [None] * len(ck.d)
    for n in range(len(ck.d) - 1, -1, -1):
        d, h_prev = ck.d[n], ck.h[n]
        fem.history_adjoint(mesh, csr, params, d, h_prev, lam=None, mu=mu, out=adj, want_hbar=False)
        rhs = -(2.0 * w * (d - u_gt[n]) + adj.ubar).reshape(-1)
        rhs[bc] = 0.0
        fem.residual_tangent(mesh, csr, params, d, h_prev, bc_mask=bc_mask, prec=fem.FP64, out=fwd)
        if symmetric:
            KT = fwd.K  # K_ff^T = K_ff
        else:
            KT = fem.csr_transpose(csr, fwd.K, bc_mask=bc_mask, out=KT)
        lam, _, res = solver.solve(KT, rhs, rtol=lin_rtol, max_iter=lin_max_iter, check=False)
        if not (res <= 1e-8):
            raise RuntimeError(f"adjoint solve of step {n + 1}: relative residual {res:.3e}")
        lam = lam.view(-1, 3).clone()
        lams[n] = lam
        fem.history_adjoint(mesh, csr, params, d, h_prev, lam=lam, mu=mu, out=adj, want_ubar=False)
        grad += adj.g_uniform
        g_elem += adj.g_elem
        mu = adj.hbar.clone()
    return grad, lams, g_elem
