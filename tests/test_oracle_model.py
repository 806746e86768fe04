"""Pins of the oracle's model options (CPU only): Voce hardening (Eq. Hard),
the orientation Theta of the Hill tensor (App. A) and the F-bar element
(Sec. 2.2.4).

* Voce: the single-step uniaxial solution of a generic Hill material, from
  the scalar equation eps11 = sigma_y(a)/(s E) + s a (s = sqrt(G + H)).
* Theta: equivariance (Theta with strain eps equals the identity with strain
  Theta^T eps Theta, rotated back), the quarter turn about z that swaps F<->G
  and L<->M, and an off-axis uniaxial solution built from the textbook Hill
  gradient in the material frame (no fourth-order rotation involved).
* Tangents: A = dP/dF against central differences of P(F) with Voce and
  Theta; K^e against central differences of R^e with F-bar.
* F-bar: equals the plain element under a homogeneous deformation (F-bar
  leaves a uniform J unchanged), the patch test, objectivity.
* VJP: central differences of lambda^T R(theta) for every model option."""
import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_2606_17390_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore")
VOCE, FBAR = oracle.MODEL_VOCE, oracle.MODEL_FBAR


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def voce(prm, a):
    return prm[8] + prm[9] * (1.0 - np.exp(-prm[10] * a))


def expm_sym(eps):
    w, Q = np.linalg.eigh(eps)
    return Q @ np.diag(np.exp(w)) @ Q.T


def hist_of(ep, alpha):
    return np.array([ep[0, 0], ep[1, 1], ep[2, 2], ep[1, 2], ep[0, 2], ep[0, 1], alpha])


def sym_of(h):
    return np.array([[h[0], h[5], h[4]], [h[5], h[1], h[3]], [h[4], h[3], h[2]]])


def random_state(rng):
    F = np.eye(3) + 0.03 * rng.standard_normal((3, 3))
    D = rng.standard_normal((3, 3))
    D = 0.5 * (D + D.T)
    D -= np.trace(D) / 3 * np.eye(3)
    D *= 2e-3 / np.linalg.norm(D)
    return F, hist_of(D, 0.02)


@pytest.mark.parametrize("eps11", [0.004, 0.02, 0.15])
def test_voce_uniaxial_single_step(eps11):
    prm = synth.voce_params(F=0.3, G=0.55, H=0.4, L=1.3, M=1.6, N=1.4)
    E, nu, G, H = prm[0], prm[1], prm[3], prm[4]
    s = np.sqrt(G + H)
    a = brentq(lambda x: voce(prm, x) / (s * E) + s * x - eps11, 0.0, 1.0, xtol=1e-16, rtol=1e-15)
    sig = voce(prm, a) / s
    e22 = -nu * sig / E - a * H / s
    e33 = -nu * sig / E - a * G / s
    F = np.diag(np.exp([eps11, e22, e33]))
    mp = oracle.material_point(F, np.zeros(7), prm, model=VOCE)
    assert mp["plastic"] and mp["converged"]
    assert rel(mp["T"], np.diag([sig, 0.0, 0.0])) <= 1e-10
    assert abs(mp["hist"][6] - a) <= 1e-10 * a
    assert rel(mp["hist"][:3], [s * a, -H / s * a, -G / s * a]) <= 1e-9


def test_orientation_equivariance():
    rng = np.random.default_rng(41)
    prm = synth.params(F=0.3, G=0.65, H=0.45, L=1.25, M=1.7, N=1.45)
    for model in (0, VOCE):
        p = prm if model == 0 else synth.voce_params(F=0.3, G=0.65, H=0.45, L=1.25, M=1.7, N=1.45)
        for _ in range(4):
            Th = synth.random_rotation(rng)
            F, h = random_state(rng)
            a = oracle.material_point(F, h, p, model=model, Theta=Th)
            hr = hist_of(Th.T @ sym_of(h) @ Th, h[6])
            b = oracle.material_point(F @ Th, hr, p, model=model)
            assert a["plastic"] and b["plastic"]
            assert rel(Th.T @ a["T"] @ Th, b["T"]) <= 1e-11
            assert rel(Th.T @ a["S"] @ Th, b["S"]) <= 1e-11
            assert rel(a["P"] @ Th, b["P"]) <= 1e-11
            assert rel(Th.T @ sym_of(a["hist"]) @ Th, sym_of(b["hist"])) <= 1e-10
            assert abs(a["hist"][6] - b["hist"][6]) <= 1e-12
            # A'_aAbB = A_aCbD Theta_CA Theta_DB
            assert rel(np.einsum("aCbD,CA,DB->aAbB", a["A"], Th, Th), b["A"]) <= 1e-10


def test_quarter_turn_swaps_hill_parameters():
    """Theta = 90 degrees about z maps material axis 1 to global y and 2 to -x:
    in global terms F and G, and L and M, trade places."""
    rng = np.random.default_rng(42)
    prm = synth.params(F=0.3, G=0.65, H=0.45, L=1.25, M=1.7, N=1.45)
    swapped = synth.params(F=0.65, G=0.3, H=0.45, L=1.7, M=1.25, N=1.45)
    Th = synth.rotation_z(np.pi / 2)
    for _ in range(4):
        F, h = random_state(rng)
        a = oracle.material_point(F, h, prm, Theta=Th)
        b = oracle.material_point(F, h, swapped)
        assert a["plastic"]
        for k in ("T", "S", "P", "hist", "A"):
            assert rel(a[k], b[k]) <= 1e-11, k


def hill_gradient(prm, T):
    """phi and d phi/dT of the textbook Hill-48 function (material frame)."""
    Fh, Gh, Hh, Lh, Mh, Nh = prm[2:8]
    phi = np.sqrt(Fh * (T[1, 1] - T[2, 2]) ** 2 + Gh * (T[2, 2] - T[0, 0]) ** 2 + Hh * (T[0, 0] - T[1, 1]) ** 2
                  + 2 * Lh * T[1, 2] ** 2 + 2 * Mh * T[0, 2] ** 2 + 2 * Nh * T[0, 1] ** 2)
    N = np.zeros((3, 3))
    N[0, 0] = -Gh * (T[2, 2] - T[0, 0]) + Hh * (T[0, 0] - T[1, 1])
    N[1, 1] = Fh * (T[1, 1] - T[2, 2]) - Hh * (T[0, 0] - T[1, 1])
    N[2, 2] = -Fh * (T[1, 1] - T[2, 2]) + Gh * (T[2, 2] - T[0, 0])
    N[1, 2] = N[2, 1] = Lh * T[1, 2]
    N[0, 2] = N[2, 0] = Mh * T[0, 2]
    N[0, 1] = N[1, 0] = Nh * T[0, 1]
    return phi, N / phi


@pytest.mark.parametrize("psi_deg", [22.5, 45.0, 70.0])
def test_off_axis_uniaxial_single_step(psi_deg):
    """Uniaxial stress sigma along global x of a material rotated by psi about
    z (Voce hardening), one step from the virgin state: eps = E^-1 T + a N with
    N the Hill gradient at T, phi(T) = sigma_y(a)."""
    prm = synth.voce_params(F=0.3, G=0.55, H=0.4, L=1.3, M=1.6, N=1.9)
    E, nu = prm[0], prm[1]
    Th = synth.rotation_z(np.radians(psi_deg))
    n = np.array([1.0, 0.0, 0.0])
    Tl = Th.T @ np.outer(n, n) @ Th
    s_psi, Nl = hill_gradient(prm, Tl)
    N = Th @ Nl @ Th.T
    a = 0.03
    sig = voce(prm, a) / s_psi
    T = sig * np.outer(n, n)
    eps = (1 + nu) / E * T - nu / E * np.trace(T) * np.eye(3) + a * N
    mp = oracle.material_point(expm_sym(eps), np.zeros(7), prm, model=VOCE, Theta=Th)
    assert mp["plastic"] and mp["converged"]
    assert rel(mp["T"], T) <= 1e-10
    assert abs(mp["hist"][6] - a) <= 1e-10 * a
    assert rel(sym_of(mp["hist"]), a * N) <= 1e-9


def test_nominal_tangent_matches_fd_with_voce_and_orientation():
    rng = np.random.default_rng(43)
    prm = synth.voce_params(F=0.3, G=0.65, H=0.45, L=1.25, M=1.7, N=1.45)
    Th = synth.random_rotation(rng)
    F, h = random_state(rng)
    a = oracle.material_point(F, h, prm, model=VOCE, Theta=Th)
    assert a["plastic"]
    hstep = 1e-7
    Afd = np.zeros((3, 3, 3, 3))
    for b in range(3):
        for B in range(3):
            Fp, Fm = F.copy(), F.copy()
            Fp[b, B] += hstep
            Fm[b, B] -= hstep
            Afd[:, :, b, B] = (oracle.material_point(Fp, h, prm, model=VOCE, Theta=Th)["P"]
                               - oracle.material_point(Fm, h, prm, model=VOCE, Theta=Th)["P"]) / (2 * hstep)
    assert rel(a["A"], Afd) <= 1e-6
    assert rel(a["Cep"], a["Cep_implicit"]) <= 1e-11


def jittered_element(rng, jit=0.15):
    X0 = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]],
                  dtype=float)
    return X0 * np.array([1.2, 0.9, 1.1]) + jit * rng.uniform(-1, 1, (8, 3))


def element_hist(rng, mag=3e-4):
    h = np.zeros((8, 7))
    for g in range(8):
        D = rng.standard_normal((3, 3))
        D = 0.5 * (D + D.T)
        D -= np.trace(D) / 3 * np.eye(3)
        D *= mag / np.linalg.norm(D)
        h[g] = hist_of(D, rng.uniform(0, 0.1))
    return h


@pytest.mark.parametrize("model,use_theta,scale", [(FBAR, False, 1e-4), (FBAR, False, 0.03),
                                                   (FBAR | VOCE, True, 0.03), (VOCE, True, 0.03)])
def test_element_tangent_matches_fd(model, use_theta, scale):
    rng = np.random.default_rng(44)
    Xe = jittered_element(rng)
    de = scale * rng.standard_normal((8, 3))
    he = element_hist(rng)
    prm = (synth.voce_params if model & VOCE else synth.params)(F=0.3, G=0.65, H=0.5, L=1.3, M=1.6, N=1.4)
    Th = synth.random_rotation(rng) if use_theta else None
    R, K, hn, diag = oracle.element(Xe, de, he, prm, model=model, Theta=Th)
    if scale > 1e-3:
        assert np.any(hn[:, 6] != he[:, 6])  # plastic somewhere
    h = 1e-7 * max(1.0, np.abs(de).max())
    Kfd = np.zeros((24, 24))
    for j in range(24):
        dp, dm = de.copy().ravel(), de.copy().ravel()
        dp[j] += h
        dm[j] -= h
        Kfd[:, j] = (oracle.element(Xe, dp, he, prm, False, model, Th)[0]
                     - oracle.element(Xe, dm, he, prm, False, model, Th)[0]) / (2 * h)
    assert rel(K, Kfd) <= 2e-6
    if model & FBAR:
        # the F-bar tangent is not symmetric
        assert np.abs(K - K.T).max() > 1e-6 * np.abs(K).max()


def test_fbar_equals_plain_element_under_homogeneous_deformation():
    rng = np.random.default_rng(45)
    Xe = jittered_element(rng)
    F0 = np.array([[1.03, 0.01, -0.004], [0.006, 0.985, 0.002], [-0.003, 0.004, 0.99]])
    de = Xe @ (F0 - np.eye(3)).T
    he = np.tile(hist_of(np.diag([2e-4, -1e-4, -1e-4]), 0.02), (8, 1))
    prm = synth.params(F=0.3, G=0.65, H=0.5)
    R0, K0, h0, _ = oracle.element(Xe, de, he, prm)
    R1, K1, h1, _ = oracle.element(Xe, de, he, prm, model=FBAR)
    assert rel(R1, R0) <= 1e-13 and rel(h1, h0) <= 1e-13
    assert np.abs(K1 - K0).max() > 1e-6 * np.abs(K0).max()  # the tangents differ


def test_fbar_patch_test_and_objectivity():
    rng = np.random.default_rng(46)
    nx, ny, nz = 4, 3, 3
    X0, conn = synth.hex_grid(nx, ny, nz)
    X = synth.jitter_nodes(X0, 1.0, 0.15, rng)
    F0 = np.array([[1.012, 0.004, -0.002], [0.003, 0.995, 0.001], [-0.001, 0.002, 0.996]])
    d = X @ (F0 - np.eye(3)).T
    prm = synth.voce_params(F=0.35, G=0.6, H=0.45)
    ne = conn.shape[0]
    hist = np.tile(np.array([4e-4, -1e-4, -3e-4, 1e-4, -5e-5, 2e-4, 0.02])[:, None], (1, 8 * ne))
    Th = synth.random_rotation(rng)
    rp, ci, _ = oracle.csr_pattern(conn, X.shape[0], with_rank=False)
    model = FBAR | VOCE
    R, K, hn, _, _ = oracle.residual_tangent(X, conn, rp, ci, prm, d, hist, model=model, orient=Th)
    mp = oracle.material_point(F0, hist[:, 0], prm, model=VOCE, Theta=Th)
    assert mp["plastic"]
    interior = ~(np.isclose(X0, X0.min(0)) | np.isclose(X0, X0.max(0))).any(axis=1)
    assert np.abs(R.reshape(-1, 3)[interior]).max() <= 1e-12 * np.abs(mp["P"]).max()
    assert rel(hn, np.tile(mp["hist"][:, None], (1, 8 * ne))) <= 1e-12
    # objectivity: x' = Q x on a non-homogeneous field
    d2 = d + 0.004 * rng.standard_normal(d.shape)
    R2, K2, h2, _, _ = oracle.residual_tangent(X, conn, rp, ci, prm, d2, hist, model=model, orient=Th)
    Q = synth.random_rotation(rng)
    dq = (X + d2) @ Q.T - X
    R3, K3, h3, _, _ = oracle.residual_tangent(X, conn, rp, ci, prm, dq, hist, model=model, orient=Th)
    assert rel(R3.reshape(-1, 3), R2.reshape(-1, 3) @ Q.T) <= 1e-9
    assert rel(h3, h2) <= 1e-9


def lamR(p, prm, rp, ci, model, orient):
    R, _, _, _, _ = oracle.residual_tangent(p.X, p.conn, rp, ci, prm, p.d, p.hist_n, want_K=False,
                                            model=model, orient=orient)
    return float(np.dot(p.lam.ravel(), R))


@pytest.mark.parametrize("model,orient", [(VOCE, None), (FBAR, None), (0, "uniform"),
                                          (VOCE | FBAR, "per_element")])
def test_vjp_matches_central_fd(model, orient):
    base = synth.small_slab(33, 3, 3, 2, strain=0.01)
    p = synth.with_model(base, 7, "voce" if model & VOCE else "swift", bool(model & FBAR), orient)
    rp, ci, _ = oracle.csr_pattern(p.conn, p.n_nodes, with_rank=False)
    gu, ge, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam, model=model, orient=p.orient)
    assert np.any(gu != 0.0)
    # step 1e-5 |theta_k|: at 1e-6 the stopping tolerance of the local Newton
    # (about 1e-12 relative) shows in the quotient of the smallest components
    for k, col in enumerate(synth.GRAD_PARAM_INDEX):
        h = 1e-5 * abs(p.prm[col])
        pp, pm = p.prm.copy(), p.prm.copy()
        pp[col] += h
        pm[col] -= h
        fd = (lamR(p, pp, rp, ci, model, p.orient) - lamR(p, pm, rp, ci, model, p.orient)) / (2 * h)
        assert abs(gu[k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gu).max()), (k, gu[k], fd)
