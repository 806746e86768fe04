"""The time-history adjoint on the GPU (through the C ABI) against the oracle:
the transposed tangent against scipy, one adjoint step (g, hbar, ubar for
random lambda and mu) element by element for every model option, and dJ/dtheta
of a multi-step load history (forward Newton, backward sweep) against the
oracle's dense adjoint, FP64."""
import sys

import numpy as np
import pytest

import oracle
from helpers import gpu_problem, oracle_model
from oracle import adjoint as oadj
from paper_2606_17390_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fem():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2606_17390_amd import fem as F
    F.lib()
    return F


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec_name", ["FP64", "FP32_MIXED"])
def test_transpose_matches_scipy(fem, prec_name):
    import scipy.sparse as sp
    p = synth.small_slab(81, 5, 4, 3)
    mesh, params, d, h, bc, _ = gpu_problem(p, fem)
    csr = fem.csr_pattern(mesh)
    out = fem.residual_tangent(mesh, csr, params, d, h, bc_mask=bc, prec=getattr(fem, prec_name))
    KT = fem.csr_transpose(csr, out.K, bc_mask=bc)
    torch.cuda.synchronize()
    say("transpose", prec_name, csr.nnz)
    rp, ci = csr.row_ptr.cpu().numpy(), csr.col_idx.cpu().numpy()
    n = csr.n_rows
    A = sp.csr_matrix((out.K.double().cpu().numpy(), ci, rp), shape=(n, n)).toarray()
    B = sp.csr_matrix((KT.double().cpu().numpy(), ci, rp), shape=(n, n)).toarray()
    ref = A.T.copy()
    m = p.bc_mask.astype(bool)
    ref[m] = 0.0
    ref[m, np.nonzero(m)[0]] = 1.0
    assert np.array_equal(B, ref)  # a permutation of the values: bit-exact


MODELS = {"plain": ("swift", False, None), "voce_orient_pe": ("voce", False, "per_element"),
          "fbar": ("swift", True, None), "fbar_voce_orient": ("voce", True, "uniform")}


@pytest.mark.parametrize("name", list(MODELS))
def test_adjoint_step_matches_oracle(fem, name):
    hard, fbar, orient = MODELS[name]
    p = synth.with_model(synth.small_slab(82, 5, 3, 2, strain=0.02), 13, hard, fbar, orient)
    rng = np.random.default_rng(83)
    mu = rng.standard_normal((7, 8 * p.n_elems)) * np.array([1e3] * 6 + [1e2])[:, None]
    say("adjoint step", name, p.n_elems)
    model, ori = oracle_model(p)
    ori_e = oracle.expand_orient(ori, p.n_elems)
    prm_e = oracle.expand_params(p.prm, p.n_elems)
    ge = np.zeros((7, p.n_elems))
    hb = np.zeros((7, 8 * p.n_elems))
    ub = np.zeros((p.n_nodes, 3))
    for e in range(p.n_elems):
        c = p.conn[e]
        th = None if ori_e is None else ori_e[e]
        he = p.hist_n[:, 8 * e:8 * e + 8].T
        tb, hbe, _ = oracle.element_adjoint(p.X[c], p.d[c], he, prm_e[e], p.lam[c], mu[:, 8 * e:8 * e + 8].T,
                                            model, th)
        _, _, ube = oracle.element_adjoint(p.X[c], p.d[c], he, prm_e[e], None, mu[:, 8 * e:8 * e + 8].T, model, th)
        ge[:, e] = tb
        hb[:, 8 * e:8 * e + 8] = hbe.T
        np.add.at(ub, c, ube.reshape(8, 3))
    mesh, params, d, h, _, lam = gpu_problem(p, fem)
    csr = fem.csr_pattern(mesh)
    mu_t = torch.as_tensor(mu).cuda()
    a = fem.history_adjoint(mesh, csr, params, d, h, lam=lam, mu=mu_t, want_ubar=False)
    torch.cuda.synchronize()
    g_elem, g_u, hbar = a.g_elem.cpu().numpy(), a.g_uniform.cpu().numpy(), a.hbar.cpu().numpy()
    b = fem.history_adjoint(mesh, csr, params, d, h, lam=None, mu=mu_t, want_hbar=False)
    torch.cuda.synchronize()
    ubar = b.ubar.cpu().numpy()
    assert (p.hist_n[6] != 0).any()
    tol = 1e-10
    assert np.abs(g_elem - ge).max() <= tol * np.abs(ge).max()
    assert np.abs(g_u - ge.sum(axis=1)).max() <= tol * np.abs(ge).max() * p.n_elems
    for rows in (slice(0, 6), slice(6, 7)):
        assert np.abs(hbar[rows] - hb[rows]).max() <= tol * np.abs(hb[rows]).max(), rows
    assert np.abs(ubar - ub).max() <= tol * np.abs(ub).max()


@pytest.mark.parametrize("variant,start", [("plain", "previous"), ("voce_orient", "previous"),
                                           ("fbar", "previous"), ("voce_orient", "linearised")])
def test_time_history_gradient_matches_oracle(fem, variant, start):
    """start "linearised": the forward run starts each step from the problem
    linearised about the previous state, with Eisenstat-Walker tolerances
    (the settings of the gradient benchmark); the converged states and the
    gradient are the same."""
    from paper_2606_17390_amd import adjoint
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from test_oracle_adjoint import load_history
    X, conn, bc, steps, hist0 = load_history(73)
    rng = np.random.default_rng(74)
    if variant == "voce_orient":
        prm, hard, fbar, orient = synth.voce_params(F=0.3, G=0.6, H=0.45, N=1.7), "voce", False, synth.random_rotation(rng)
    elif variant == "fbar":
        prm, hard, fbar, orient = synth.params(F=0.3, G=0.6, H=0.45, N=1.7), "swift", True, None
    else:
        prm, hard, fbar, orient = synth.params(F=0.3, G=0.6, H=0.45, N=1.7), "swift", False, None
    model = (oracle.MODEL_VOCE if hard == "voce" else 0) | (oracle.MODEL_FBAR if fbar else 0)
    ds, hs = oadj.simulate(X, conn, prm, bc, steps, hist0, model=model, orient=orient)
    u_gt = [dd * 0.97 + 1e-4 * rng.standard_normal(dd.shape) for dd in ds]
    w = 10.0
    g_ref, lam_ref = oadj.adjoint_gradient(X, conn, prm, bc, ds, hs, u_gt, w, model=model, orient=orient)
    say("time-history gradient", variant)
    mesh = fem.Mesh(X, conn)
    csr = fem.csr_pattern(mesh)
    params = fem.Params(prm, conn.shape[0], hardening=hard, fbar=fbar, orient=orient)
    bct = torch.as_tensor(bc).cuda()
    kw = dict(forcing="ew", tangent_start=True) if start == "linearised" else {}
    ck = adjoint.forward(mesh, csr, params, bct, [torch.as_tensor(s).cuda() for s in steps],
                         torch.as_tensor(hist0).cuda(), tol=1e-12, **kw)
    for n in range(len(ds)):
        assert np.abs(ck.d[n].cpu().numpy() - ds[n]).max() <= 1e-10 * np.abs(ds[n]).max()
    ugt = [torch.as_tensor(u).cuda() for u in u_gt]
    g, lams, _ = adjoint.gradient(mesh, csr, params, bct, ck, ugt, w)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    say("gradient", g, "oracle", g_ref)
    assert np.abs(g - g_ref).max() <= 1e-7 * np.abs(g_ref).max()
    for n in range(len(ds)):
        assert np.abs(lams[n].cpu().numpy() - lam_ref[n]).max() <= 1e-7 * np.abs(lam_ref[n]).max()
