"""Time-history adjoint on the CPU (dense; small problems only).

TEST INFRASTRUCTURE ONLY (see the package docstring).  It follows the
discrete adjoint of Sec. 2.3 (Eqs. (Lagrangian) ... (dR_u), Alg. 1) for the
time-discrete forward problem in which the history h^n of every Gauss point
is produced by the local update H^n(u^n, h^{n-1}, theta) of the converged
step (the internal variables are embedded in the constitutive update).
With multipliers lambda^n for R^n = 0 and mu^n for h^n = H^n:

  K^n^T lambda^n = -[dJ^n/du^n + (dH^n/du^n)^T mu^n]          (adjoint solve)
  mu^{n-1}      = (dR^n/dh^{n-1})^T lambda^n + (dH^n/dh^{n-1})^T mu^n
  dJ/dtheta     = sum_n lambda^n^T dR^n/dtheta + mu^n^T dH^n/dtheta

backward from n = N_T with mu^{N_T} = 0.  Constrained dofs are prescribed
(not unknowns): the adjoint solve uses the free-free block and lambda is
zero on constrained dofs.  The objective is Eq. (J):
J = w sum_n ||u^n - u_gt^n||^2.

Every element quantity comes from the oracle (oracle_element,
oracle_element_adjoint); assembly and solves are dense numpy.
"""
import numpy as np

from . import csr_pattern, element_adjoint, expand_orient, expand_params, residual_tangent

__all__ = ["simulate", "objective", "adjoint_gradient"]


def _dense(K, rp, ci, n):
    A = np.zeros((n, n))
    for r in range(n):
        A[r, ci[rp[r]:rp[r + 1]]] = K[rp[r]:rp[r + 1]]
    return A


def simulate(X, conn, prm, bc_mask, bc_steps, hist0, model=0, orient=None, tol=1e-12, max_it=50):
    """Forward pass: for each load step n, prescribed values bc_steps[n] ([n_nodes, 3];
    read on constrained dofs) and a damped Newton iteration (backtracking on ||R||)
    from the previous solution.  Returns (list of d^n, list of h^n), h^0 = hist0."""
    X = np.asarray(X, dtype=np.float64)
    nn = X.shape[0]
    rp, ci, _ = csr_pattern(conn, nn, with_rank=False)
    bc = np.asarray(bc_mask, dtype=bool)
    d = np.zeros((nn, 3))
    ds, hs = [], [np.array(hist0, dtype=np.float64)]
    for ub in bc_steps:
        d = d.copy()
        d.reshape(-1)[bc] = np.asarray(ub).reshape(-1)[bc]
        h_prev = hs[-1]

        def ev(dd):
            R, K, hn, _, _ = residual_tangent(X, conn, rp, ci, prm, dd, h_prev, bc_mask=bc_mask, model=model,
                                              orient=orient)
            return R, K, hn

        R, K, hn = ev(d)
        r0 = np.linalg.norm(R)
        for _ in range(max_it):
            rn = np.linalg.norm(R)
            if rn <= tol * max(r0, 1e-300):
                break
            du = np.linalg.solve(_dense(K, rp, ci, 3 * nn), -R).reshape(nn, 3)
            t = 1.0
            for _ls in range(12):
                R2, K2, hn2 = ev(d + t * du)
                if np.linalg.norm(R2) < (1 - 1e-4 * t) * rn:
                    break
                t *= 0.5
            d, R, K, hn = d + t * du, R2, K2, hn2
        else:
            raise RuntimeError(f"oracle Newton did not converge: {np.linalg.norm(R):.3e}")
        ds.append(d)
        hs.append(hn)
    return ds, hs


def objective(ds, u_gt, w):
    return float(w * sum(np.sum((d - g) ** 2) for d, g in zip(ds, u_gt)))


def adjoint_gradient(X, conn, prm, bc_mask, ds, hs, u_gt, w, model=0, orient=None):
    """dJ/dtheta [7] (uniform parameters) and the multipliers lambda^n [n_nodes, 3]
    for the forward solution (ds, hs) of simulate()."""
    X = np.asarray(X, dtype=np.float64)
    conn = np.asarray(conn)
    nn, ne = X.shape[0], conn.shape[0]
    prm_e = expand_params(prm, ne)
    ori = expand_orient(orient, ne)
    rp, ci, _ = csr_pattern(conn, nn, with_rank=False)
    bc = np.asarray(bc_mask, dtype=bool)
    free = ~bc
    grad = np.zeros(7)
    mu = np.zeros((ne, 8, 7))
    lams = [None] * len(ds)
    for n in range(len(ds) - 1, -1, -1):
        d, h_prev = ds[n], hs[n]
        # (dH^n/du^n)^T mu^n, assembled
        ubar = np.zeros(3 * nn)
        for e in range(ne):
            he = h_prev[:, 8 * e:8 * e + 8].T
            th = None if ori is None else ori[e]
            _, _, ub = element_adjoint(X[conn[e]], d[conn[e]], he, prm_e[e], None, mu[e], model, th)
            np.add.at(ubar, (3 * conn[e][:, None] + np.arange(3)).ravel(), ub)
        rhs = -(2.0 * w * (d - u_gt[n]).reshape(-1) + ubar)
        _, K, _, _, _ = residual_tangent(X, conn, rp, ci, prm, d, h_prev, bc_mask=None, model=model, orient=orient)
        A = _dense(K, rp, ci, 3 * nn)
        lam = np.zeros(3 * nn)
        lam[free] = np.linalg.solve(A[np.ix_(free, free)].T, rhs[free])
        lams[n] = lam.reshape(nn, 3)
        mu_prev = np.zeros_like(mu)
        for e in range(ne):
            he = h_prev[:, 8 * e:8 * e + 8].T
            th = None if ori is None else ori[e]
            tb, hb, _ = element_adjoint(X[conn[e]], d[conn[e]], he, prm_e[e], lam.reshape(nn, 3)[conn[e]], mu[e],
                                        model, th)
            grad += tb
            mu_prev[e] = hb
        mu = mu_prev
    return grad, lams
