"""Pins of the oracle's Barlat Yld2004-18p yield function (Eq. Phi_barlat,
App. A) and its return map (CPU only).

* Reductions stated in App. A: all 18 coefficients 1 with m = 2 or m = 4 is
  von Mises (phi = sigma_vm for any stress; the material point equals Hill-48
  at F = G = H = 1/2, L = M = N = 3/2); C' = C'' with m = 2 is Hill-48 with the
  parameters of the quadratic form (3/2) |dev(C' : P : T)|^2, derived here
  independently.
* The published AA6111-T4 fit (tests/golden/barlat_yld2004_aa6111.json, the
  paper's verification table) gives a uniaxial yield stress along the first
  axis of sigma0 within 1e-3 (the normalisation of the paper's pi-plane
  figure).
* N = dphi/dT against central differences of phi (m = 8, with orientation).
* dP/dF (through the Hessian of phi in the tangent) against central
  differences of P(F), and K^e against central differences of R^e, m = 8."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2606_17390_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore")
BARLAT, VOCE = oracle.MODEL_BARLAT, oracle.MODEL_VOCE
HERE = os.path.dirname(os.path.abspath(__file__))
KEYS = ("c12", "c13", "c21", "c23", "c31", "c32", "c44", "c55", "c66")


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def published():
    with open(os.path.join(HERE, "golden", "barlat_yld2004_aa6111.json")) as f:
        g = json.load(f)
    return np.array([g["c_prime"][k] for k in KEYS] + [g["c_double_prime"][k] for k in KEYS] + [g["m"]]), g


def sym(rng, scale=100.0):
    A = rng.standard_normal((3, 3))
    return scale * 0.5 * (A + A.T)


def vm(T):
    s = T - np.trace(T) / 3 * np.eye(3)
    return np.sqrt(1.5 * np.sum(s * s))


@pytest.mark.parametrize("m", [2.0, 4.0])
def test_unit_coefficients_are_von_mises(m):
    oracle.set_barlat(np.r_[np.ones(18), m])
    rng = np.random.default_rng(91)
    prm = synth.params()
    for _ in range(5):
        T = sym(rng)
        phi, _ = oracle.effective_stress(T, prm, BARLAT)
        assert abs(phi - vm(T)) <= 1e-12 * vm(T)
    # the whole material point: Barlat = Hill-48 at its von Mises parameters
    F = np.eye(3) + 0.02 * rng.standard_normal((3, 3))
    h = np.array([2e-4, -1e-4, -1e-4, 5e-5, 0.0, 1e-4, 0.01])
    a = oracle.material_point(F, h, prm, model=BARLAT)
    b = oracle.material_point(F, h, prm)
    assert a["plastic"] and b["plastic"]
    for k in ("T", "hist", "A"):
        assert rel(a[k], b[k]) <= 1e-9, k


def test_order_eight_is_not_von_mises():
    oracle.set_barlat(np.r_[np.ones(18), 8.0])
    rng = np.random.default_rng(92)
    T = sym(rng)
    phi, _ = oracle.effective_stress(T, synth.params(), BARLAT)
    assert abs(phi - vm(T)) > 1e-4 * vm(T)


def hill_equivalent(c9):
    """(F, G, H, L, M, N) of phi^2 = (3/2)|dev(C' : P : T)|^2 (Mandel algebra)."""
    C = np.zeros((6, 6))
    C[0, 1], C[0, 2], C[1, 0], C[1, 2], C[2, 0], C[2, 1] = [-c for c in c9[:6]]
    C[3, 3], C[4, 4], C[5, 5] = c9[6:9]
    P = np.zeros((6, 6))
    P[:3, :3] = (3 * np.eye(3) - 1) / 3
    P[3:, 3:] = np.eye(3)
    Hq = 1.5 * (C @ P).T @ P @ (C @ P)  # P is also the deviatoric projector in Mandel
    return dict(F=-Hq[1, 2], G=-Hq[0, 2], H=-Hq[0, 1], L=Hq[3, 3], M=Hq[4, 4], N=Hq[5, 5]), Hq


def test_equal_transforms_with_m2_are_hill():
    c9 = np.array([0.9, 1.1, 0.85, 1.05, 1.2, 0.95, 1.1, 0.9, 1.25])
    oracle.set_barlat(np.r_[c9, c9, 2.0])
    hp, Hq = hill_equivalent(c9)
    assert np.allclose(Hq[:3, 3:], 0.0) and np.allclose(Hq[:3, :3].sum(axis=1), 0.0)
    prm_b = synth.params()
    prm_h = synth.params(**hp)
    rng = np.random.default_rng(93)
    for _ in range(3):
        T = sym(rng)
        assert abs(oracle.effective_stress(T, prm_b, BARLAT)[0] - oracle.effective_stress(T, prm_h)[0]) <= 1e-12 * vm(T)
    F = np.eye(3) + 0.02 * rng.standard_normal((3, 3))
    h = np.array([2e-4, -1e-4, -1e-4, 5e-5, 0.0, 1e-4, 0.01])
    a = oracle.material_point(F, h, prm_b, model=BARLAT)
    b = oracle.material_point(F, h, prm_h)
    assert a["plastic"]
    for k in ("T", "hist", "A"):
        assert rel(a[k], b[k]) <= 1e-9, k


def test_published_fit_is_normalised_to_sigma0():
    coef, g = published()
    oracle.set_barlat(coef)
    phi, _ = oracle.effective_stress(np.diag([1.0, 0.0, 0.0]), synth.params(E=g["E"], nu=g["nu"]), BARLAT)
    assert abs(1.0 / phi - g["sigma0"]) <= 1e-3


def test_gradient_matches_fd():
    coef, _ = published()
    oracle.set_barlat(coef)
    rng = np.random.default_rng(94)
    prm = synth.params()
    for Th in (None, synth.random_rotation(rng)):
        T = sym(rng)
        phi, N = oracle.effective_stress(T, prm, BARLAT, Th)
        Nfd = np.zeros((3, 3))
        h = 1e-6 * np.abs(T).max()
        for i in range(3):
            for j in range(i, 3):
                E = np.zeros((3, 3))
                E[i, j] = E[j, i] = h if i != j else h
                d = (oracle.effective_stress(T + E, prm, BARLAT, Th)[0]
                     - oracle.effective_stress(T - E, prm, BARLAT, Th)[0]) / (2 * h)
                # dphi = N : dT, dT symmetric: off-diagonal perturbation counts N_ij twice
                Nfd[i, j] = Nfd[j, i] = d if i == j else d / 2
        assert rel(N, Nfd) <= 1e-7


def test_nominal_tangent_and_element_tangent_match_fd():
    coef, _ = published()
    oracle.set_barlat(coef)
    rng = np.random.default_rng(95)
    prm = synth.voce_params(sig0=200.0, Q=100.0, b=15.0)
    Th = synth.rotation_z(0.3)
    F = np.eye(3) + 0.02 * rng.standard_normal((3, 3))
    h = np.array([2e-4, -1e-4, -1e-4, 5e-5, 0.0, 1e-4, 0.01])
    model = BARLAT | VOCE
    a = oracle.material_point(F, h, prm, model=model, Theta=Th)
    assert a["plastic"] and a["converged"]
    st = 1e-7
    Afd = np.zeros((3, 3, 3, 3))
    for b in range(3):
        for B in range(3):
            Fp, Fm = F.copy(), F.copy()
            Fp[b, B] += st
            Fm[b, B] -= st
            Afd[:, :, b, B] = (oracle.material_point(Fp, h, prm, model=model, Theta=Th)["P"]
                               - oracle.material_point(Fm, h, prm, model=model, Theta=Th)["P"]) / (2 * st)
    assert rel(a["A"], Afd) <= 1e-6
    assert rel(a["Cep"], a["Cep_implicit"]) <= 1e-10
    # element level
    X0 = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)
    Xe = X0 + 0.1 * rng.uniform(-1, 1, (8, 3))
    de = 0.02 * rng.standard_normal((8, 3))
    he = np.tile(h, (8, 1))
    R, K, hn, _ = oracle.element(Xe, de, he, prm, model=model, Theta=Th)
    assert np.any(hn[:, 6] != he[:, 6])
    Kfd = np.zeros((24, 24))
    hs = 1e-7
    for j in range(24):
        dp, dm = de.copy().ravel(), de.copy().ravel()
        dp[j] += hs
        dm[j] -= hs
        Kfd[:, j] = (oracle.element(Xe, dp, he, prm, False, model, Th)[0]
                     - oracle.element(Xe, dm, he, prm, False, model, Th)[0]) / (2 * hs)
    assert rel(K, Kfd) <= 2e-6
