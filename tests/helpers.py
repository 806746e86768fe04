"""Shared test helpers: run the HIP path and the oracle on the same seeded
inputs and compare them with the metrics stated in the design notes."""
import numpy as np

import oracle

# tolerances
TOL_FP64 = 1e-10   # FP64 path vs FP64 oracle (normwise relative)
TOL_MIXED = 1e-5   # FP32-mixed path vs FP64 (normwise relative)


def rel_inf(a, b, scale=None):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    s = np.abs(b).max() if scale is None else scale
    if s == 0:
        return float(np.abs(a - b).max()) if a.size else 0.0
    return float(np.abs(a - b).max() / s) if a.size else 0.0


def hist_rel(a, b):
    """History error: the six eps^p rows against their common |eps^p|_inf,
    alpha against |alpha|_inf (a row of pure rounding noise has no scale of
    its own)."""
    a, b = np.asarray(a), np.asarray(b)
    se = max(np.abs(b[:6]).max(), 1e-300)
    sa = max(np.abs(b[6]).max(), 1e-300)
    return max(float(np.abs(a[:6] - b[:6]).max() / se), float(np.abs(a[6] - b[6]).max() / sa))


def oracle_model(p):
    """Model flags and per-element orientation of a synth.Problem for the oracle
    (the Barlat coefficients, if any, are installed in the oracle)."""
    flags = (oracle.MODEL_VOCE if p.hardening == "voce" else 0) | (oracle.MODEL_FBAR if p.fbar else 0)
    if p.barlat is not None:
        oracle.set_barlat(p.barlat)
        flags |= oracle.MODEL_BARLAT
    return flags, p.orient


def residual_scale(p):
    """|| sum_e |R^e| ||_inf : assembled absolute element contributions (robust
    to cancellation near equilibrium)."""
    acc = np.zeros(3 * p.n_nodes)
    prm = oracle.expand_params(p.prm, p.n_elems)
    model, orient = oracle_model(p)
    ori = oracle.expand_orient(orient, p.n_elems)
    for e in range(p.n_elems):
        he = p.hist_n[:, 8 * e:8 * e + 8].T
        Re, _, _, _ = oracle.element(p.X[p.conn[e]], p.d[p.conn[e]], he, prm[e], want_K=False, model=model,
                                     Theta=None if ori is None else ori[e])
        dofs = (3 * p.conn[e][:, None] + np.arange(3)).ravel()
        np.add.at(acc, dofs, np.abs(Re))
    return float(acc.max())


def oracle_forward(p, bc=True, want_K=True):
    rp, ci, rank = oracle.csr_pattern(p.conn, p.n_nodes)
    model, orient = oracle_model(p)
    R, K, hn, rn, diag = oracle.residual_tangent(p.X, p.conn, rp, ci, p.prm, p.d, p.hist_n,
                                                 bc_mask=p.bc_mask if bc else None, want_K=want_K,
                                                 model=model, orient=orient)
    return dict(row_ptr=rp, col_idx=ci, rank=rank, R=R, K=K, hist=hn, rnorm2=rn, diag=diag)


def gpu_problem(p, fem, device="cuda"):
    """Device copies of a synth.Problem for the binding."""
    import torch
    mesh = fem.Mesh(p.X, p.conn, device)
    params = fem.Params(p.prm, p.n_elems, device, hardening=p.hardening, fbar=p.fbar, orient=p.orient,
                        barlat=p.barlat)
    d = torch.as_tensor(np.ascontiguousarray(p.d, dtype=np.float64)).to(device)
    h = torch.as_tensor(np.ascontiguousarray(p.hist_n, dtype=np.float64)).to(device)
    bc = torch.as_tensor(np.ascontiguousarray(p.bc_mask, dtype=np.uint8)).to(device) if p.bc_mask is not None else None
    lam = torch.as_tensor(np.ascontiguousarray(p.lam, dtype=np.float64)).to(device) if p.lam is not None else None
    return mesh, params, d, h, bc, lam


def gpu_forward(p, fem, prec, bc=True, want_K=True, csr=None):
    import torch
    mesh, params, d, h, bcm, _ = gpu_problem(p, fem)
    if csr is None:
        csr = fem.csr_pattern(mesh)
    out = fem.residual_tangent(mesh, csr, params, d, h, bc_mask=bcm if bc else None, prec=prec, want_K=want_K)
    torch.cuda.synchronize()
    return dict(csr=csr, R=out.R.cpu().numpy(), K=out.K.double().cpu().numpy() if out.K is not None else None,
                hist=out.hist.cpu().numpy(), rnorm2=float(out.rnorm2.cpu()[0]), diag=out.diag.cpu().numpy())
