"""Pins of the oracle's time-history adjoint (CPU only).

* The Jacobian of the local update (App. D forward mode) against central
  differences of the material point in eps (through F = exp(eps)), in the
  history h_n and in theta, with Voce hardening and an orientation.
* The element adjoint's parameter part with lambda alone equals the
  parameter VJP (forward-mode, one solve per parameter).
* dJ/dtheta of a multi-step load history (Eq. J, Alg. 1 with the history
  multipliers) against central differences of J(theta) through the whole
  forward simulation, for the plain element, Voce with an orientation, and
  F-bar."""
import numpy as np
import pytest

import oracle
from oracle import adjoint
from paper_2606_17390_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore")
VOCE, FBAR = oracle.MODEL_VOCE, oracle.MODEL_FBAR
W = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])


def expm_sym(eps):
    w, Q = np.linalg.eigh(eps)
    return Q @ np.diag(np.exp(w)) @ Q.T


def mandel_to_sym(v):
    return np.array([[v[0], v[5] / np.sqrt(2), v[4] / np.sqrt(2)], [v[5] / np.sqrt(2), v[1], v[3] / np.sqrt(2)],
                     [v[4] / np.sqrt(2), v[3] / np.sqrt(2), v[2]]])


def sym_to_mandel(M):
    return np.array([M[0, 0], M[1, 1], M[2, 2], np.sqrt(2) * M[1, 2], np.sqrt(2) * M[0, 2], np.sqrt(2) * M[0, 1]])


@pytest.mark.parametrize("model,use_theta,plastic", [(0, False, True), (VOCE, True, True), (0, False, False)])
def test_local_jacobian_matches_fd(model, use_theta, plastic):
    rng = np.random.default_rng(71)
    prm = (synth.voce_params if model & VOCE else synth.params)(F=0.3, G=0.6, H=0.45, L=1.3, M=1.6, N=1.4)
    Th = synth.random_rotation(rng) if use_theta else None
    D = rng.standard_normal((3, 3))
    eps = 0.5 * (D + D.T) * (0.01 if plastic else 1e-5)
    h = np.array([3e-4, -1e-4, -2e-4, 1e-4, -5e-5, 8e-5, 0.03])
    if not plastic:
        h[:6] = 0.0
    em = sym_to_mandel(eps)

    def z_of(em_, h_, prm_):
        mp = oracle.material_point(expm_sym(mandel_to_sym(em_)), h_, prm_, model=model, Theta=Th)
        return np.concatenate([sym_to_mandel(mp["T"]), mp["hist"]]), mp["plastic"]

    Jz, rc = oracle.local_jacobian(expm_sym(eps), h, prm, model=model, Theta=Th)
    assert rc == 0
    assert z_of(em, h, prm)[1] == plastic
    Jfd = np.zeros((13, 20))
    for k in range(20):
        if k < 6:
            st = 1e-8
            a, b = em.copy(), em.copy()
            a[k] += st
            b[k] -= st
            Jfd[:, k] = (z_of(a, h, prm)[0] - z_of(b, h, prm)[0]) / (2 * st)
        elif k < 13:
            st = 1e-8 if k < 12 else 1e-6
            a, b = h.copy(), h.copy()
            a[k - 6] += st
            b[k - 6] -= st
            Jfd[:, k] = (z_of(em, a, prm)[0] - z_of(em, b, prm)[0]) / (2 * st)
        else:
            col = synth.GRAD_PARAM_INDEX[k - 13]
            st = 1e-6 * abs(prm[col])
            a, b = prm.copy(), prm.copy()
            a[col] += st
            b[col] -= st
            Jfd[:, k] = (z_of(em, h, a)[0] - z_of(em, h, b)[0]) / (2 * st)
    # rows scaled separately: stresses (MPa) and history (strain)
    for rows in (slice(0, 6), slice(6, 13)):
        s = np.abs(Jfd[rows]).max(axis=0) + 1e-300
        err = np.abs(Jz[rows] - Jfd[rows]).max(axis=0)
        assert np.all(err <= 2e-5 * np.maximum(s, 1e-3 * np.abs(Jfd[rows]).max())), (rows, err / s)


def test_element_adjoint_parameter_part_equals_vjp():
    p = synth.with_model(synth.small_slab(72, 3, 2, 2, strain=0.01), 3, "voce", False, "uniform")
    gu, ge, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam, model=VOCE, orient=p.orient)
    th = p.orient.reshape(9)
    tot = np.zeros(7)
    for e in range(p.n_elems):
        tb, _, ub = oracle.element_adjoint(p.X[p.conn[e]], p.d[p.conn[e]], p.hist_n[:, 8 * e:8 * e + 8].T, p.prm,
                                           p.lam[p.conn[e]], None, VOCE, th)
        assert np.all(ub == 0.0)
        assert np.abs(tb - ge[:, e]).max() <= 1e-10 * np.abs(ge).max()
        tot += tb
    assert np.abs(tot - gu).max() <= 1e-10 * np.abs(gu).max()


def load_history(seed, n_steps=4):
    """2x2x2 jittered block, x = 0 clamped, the x = 2 face pulled and sheared."""
    rng = np.random.default_rng(seed)
    X0, conn = synth.hex_grid(2, 2, 2)
    X = synth.jitter_nodes(X0, 1.0, 0.05, rng)
    nn = X.shape[0]
    bc = np.zeros((nn, 3), dtype=bool)
    left, right = np.isclose(X0[:, 0], 0.0), np.isclose(X0[:, 0], 2.0)
    bc[left] = True
    bc[right] = True
    steps = []
    for n in range(1, n_steps + 1):
        u = np.zeros((nn, 3))
        u[right, 0] = 0.012 * n
        u[right, 1] = 0.006 * n * (X[right, 2] - 1.0)
        steps.append(u)
    hist0 = np.zeros((7, 8 * conn.shape[0]))
    hist0[6] = 0.01
    return X, conn, bc.ravel().astype(np.uint8), steps, hist0


@pytest.mark.parametrize("variant", ["plain", "voce_orient", "fbar"])
def test_time_history_adjoint_matches_fd(variant):
    X, conn, bc, steps, hist0 = load_history(73)
    rng = np.random.default_rng(74)
    if variant == "voce_orient":
        prm, model, orient = synth.voce_params(F=0.3, G=0.6, H=0.45, N=1.7), VOCE, synth.random_rotation(rng)
    elif variant == "fbar":
        prm, model, orient = synth.params(F=0.3, G=0.6, H=0.45, N=1.7), FBAR, None
    else:
        prm, model, orient = synth.params(F=0.3, G=0.6, H=0.45, N=1.7), 0, None
    ds, hs = adjoint.simulate(X, conn, prm, bc, steps, hist0, model=model, orient=orient)
    assert (hs[-1][6] > hist0[6]).any()  # plastic flow develops
    u_gt = [d * 0.97 + 1e-4 * rng.standard_normal(d.shape) for d in ds]
    w = 10.0
    grad, _ = adjoint.adjoint_gradient(X, conn, prm, bc, ds, hs, u_gt, w, model=model, orient=orient)

    def J(pr):
        d2, _ = adjoint.simulate(X, conn, pr, bc, steps, hist0, model=model, orient=orient, tol=1e-13)
        return adjoint.objective(d2, u_gt, w)

    # fourth-order central differences with step 1e-3 |theta_k| (truncation
    # O(h^4)); small steps are limited by the Newton tolerance of the forward
    # runs (~1e-13 relative in J) in the smallest components
    def shifted(col, x):
        q = prm.copy()
        q[col] += x
        return J(q)

    for k, col in enumerate(synth.GRAD_PARAM_INDEX):
        st = 1e-3 * abs(prm[col])
        fd = (-shifted(col, 2 * st) + 8 * shifted(col, st) - 8 * shifted(col, -st) + shifted(col, -2 * st)) / (12 * st)
        assert abs(grad[k] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(grad).max()), (variant, k, grad[k], fd)
