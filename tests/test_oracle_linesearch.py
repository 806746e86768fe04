"""Pins of the oracle's local line search (App. B, Eqs. (merit) to
(alpha_safeguard); the step selection of Alg. C2), CPU only.

* The paper's single-point example (tests/golden/barlat_line_search_single_point.json):
  Barlat Yld2004-18p with the published AA6111 fit, E = 1000, nu = 0.3,
  sigma0 = 1, perfect plasticity, trial principal stresses (8, -5.2, -2.8).
  In the third Newton iteration the full step increases the merit, the merit
  along the Newton direction is smallest at zeta = 0.46, and the quadratic
  model picks zeta = 0.363; the standard Newton method has not converged
  after 10 iterations.  The merit psi = 1/2 G^T G of Eq. (merit), as printed,
  reproduces both printed step lengths.
* Every traced step is recomputed here from the traced merit values with the
  printed formulas: the Goldstein test, Eq. (alpha_init), Eq.
  (alpha_update_ls) and the safeguard Eq. (alpha_safeguard); the traced merit
  values are recomputed from an independent numpy residual of Eq.
  (local_cpp) (Hill-48, and Barlat with phi from its own pinned evaluation);
  psi'(0) = -2 psi(0) along the Newton direction by central differences.
* The robustness study of App. B: about 16,000 trial states in the deviatoric
  principal-stress plane between the yield surface and the surface scaled by
  30, k_max = 40: the standard Newton method fails on about 9,600 (here
  between 50 % and 70 %); with the line search most converge within 20 and
  all converge.
* Planted mistakes (a copy of oracle.c edited on the fly: the safeguard's max
  turned into a min, psi(zeta^(j)) in place of psi(0) in the update's
  numerator) fail the trace recomputation.
"""
import json
import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KEYS = ("c12", "c13", "c21", "c23", "c31", "c32", "c44", "c55", "c66")
BARLAT = oracle.MODEL_BARLAT
BETA, ETA = 1e-4, 0.1
S2 = np.sqrt(2.0)


def golden():
    with open(os.path.join(HERE, "golden", "barlat_line_search_single_point.json")) as f:
        ls = json.load(f)
    with open(os.path.join(HERE, "golden", "barlat_yld2004_aa6111.json")) as f:
        g = json.load(f)
    coef = np.array([g["c_prime"][k] for k in KEYS] + [g["c_double_prime"][k] for k in KEYS] + [g["m"]])
    return ls, coef


def example_params(ls):
    """Perfect plasticity: Swift with n = 0 gives sigma_y = K = sigma0."""
    return np.array([ls["E"], ls["nu"], 0.5, 0.5, 0.5, 1.5, 1.5, 1.5, ls["sigma0"], 1.0, 0.0])


def strain_of_stress(T, E, nu):
    """Mandel strain eps = E^-1 : T for a diagonal (principal, material-axis) stress."""
    T = np.asarray(T, dtype=float)
    return np.r_[[(T[i] - nu * (T.sum() - T[i])) / E for i in range(3)], 0.0, 0.0, 0.0]


def pi_plane_states(prm, n_theta=160, n_r=100, r_max=30.0):
    """Trial strains of the robustness study: n_theta directions in the
    deviatoric principal-stress plane times n_r radii in (1, r_max] times the
    yield surface in that direction."""
    E, nu = prm[0], prm[1]
    e1 = np.array([2.0, -1.0, -1.0]) / np.sqrt(6.0)
    e2 = np.array([0.0, 1.0, -1.0]) / np.sqrt(2.0)
    th = np.arange(n_theta) * 2 * np.pi / n_theta
    rad = 1.0 + (r_max - 1.0) * (np.arange(n_r) + 1) / n_r
    out = []
    for t in th:
        u = np.cos(t) * e1 + np.sin(t) * e2
        phi, _ = oracle.effective_stress(np.diag(u), prm, BARLAT)
        for r in rad:
            out.append(strain_of_stress(r * u / phi * prm[8], E, nu))
    return np.array(out)


@pytest.fixture(scope="module")
def example():
    ls, coef = golden()
    oracle.set_barlat(coef)
    prm = example_params(ls)
    eps = strain_of_stress(ls["trial_principal_stress"], ls["E"], ls["nu"])
    return ls, coef, prm, eps


# ---- independent residual of Eq. (local_cpp) and merit of Eq. (merit)

def hill_mandel(prm):
    F, G, H, L, M, N = prm[2:8]
    Hm = np.zeros((6, 6))
    Hm[:3, :3] = [[G + H, -H, -G], [-H, F + H, -F], [-G, -F, F + G]]
    Hm[3, 3], Hm[4, 4], Hm[5, 5] = L, M, N
    return Hm


def elastic_mandel(prm):
    E, nu = prm[0], prm[1]
    lam, mu = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
    C = 2 * mu * np.eye(6)
    C[:3, :3] += lam
    return C


def swift(prm, a):
    return prm[8] * (prm[9] + a) ** prm[10]


def mandel_to_tensor(t):
    return np.array([[t[0], t[5] / S2, t[4] / S2], [t[5] / S2, t[1], t[3] / S2], [t[4] / S2, t[3] / S2, t[2]]])


def tensor_to_mandel(A):
    return np.array([A[0, 0], A[1, 1], A[2, 2], S2 * A[1, 2], S2 * A[0, 2], S2 * A[0, 1]])


def merit_numpy(y, eps_m, hist_n, prm, barlat):
    """psi = 1/2 G^T G with G of Eq. (local_cpp), y = [T Mandel, alpha, dgamma],
    W = 1; Hill-48 from its quadratic form, Barlat phi and N from the oracle's
    pinned yield-function evaluation."""
    T, a, dg = y[:6], y[6], y[7]
    if barlat:
        phi, Nt = oracle.effective_stress(mandel_to_tensor(T), prm, BARLAT)
        N = tensor_to_mandel(Nt)
    else:
        Hm = hill_mandel(prm)
        phi = np.sqrt(T @ Hm @ T)
        N = Hm @ T / phi
    epn = tensor_to_mandel(np.array([[hist_n[0], hist_n[5], hist_n[4]], [hist_n[5], hist_n[1], hist_n[3]],
                                     [hist_n[4], hist_n[3], hist_n[2]]]))
    G = np.r_[T - elastic_mandel(prm) @ (eps_m - epn - dg * N), a - hist_n[6] - dg, phi - swift(prm, a)]
    return 0.5 * G @ G


# ---- the paper's single-point example

def test_single_point_third_iteration(example):
    ls, _, prm, eps = example
    it, y, tr = oracle.local_return(eps, np.zeros(7), prm, BARLAT, kmax=40)
    assert it > 0
    # the first two iterations take the full Newton step
    assert tr[0]["zeta"] == 1.0 and tr[1]["zeta"] == 1.0
    r = tr[2]
    third = ls["third_iteration"]
    assert r["psi1"] > r["psi0"] and third["full_step_increases_merit"]
    # the quadratic model's step, Eq. (alpha_init), printed to three digits
    assert abs(r["zetas"][0] - third["quadratic_model_step"]) < 5e-4
    assert r["zeta"] == r["zetas"][0]
    # the minimum of the merit along the Newton direction, printed to two digits
    zs = np.linspace(0.01, 1.0, 991)
    ps = [oracle.local_merit(eps, np.zeros(7), prm, r["y"] + z * r["dy"], BARLAT) for z in zs]
    assert abs(zs[int(np.argmin(ps))] - third["merit_minimum_at_zeta"]) < 5e-3


def test_standard_newton_oscillates(example):
    ls, _, prm, eps = example
    it10, _, _ = oracle.local_return(eps, np.zeros(7), prm, BARLAT, line_search=False, kmax=10)
    assert it10 < 0 and not ls["standard_newton_converged_after_10_iterations"]
    it40, _, tr = oracle.local_return(eps, np.zeros(7), prm, BARLAT, line_search=False, kmax=40)
    assert it40 < 0
    # the merit goes up again and again from the third iteration on
    ups = sum(1 for r in tr[2:] if r["psi1"] > r["psi0"])
    assert ups >= 5
    it_ls, _, _ = oracle.local_return(eps, np.zeros(7), prm, BARLAT, line_search=True, kmax=40)
    assert 0 < it_ls <= 10


# ---- every step recomputed from the trace

def same_merit(a, b, y, eps, prm):
    """Merits agree: |G| within 1e-10 relative, or within the rounding of
    G_T = T - E:(...) (terms of the size of |T| and E |eps|) once G is small."""
    ga, gb = np.sqrt(2 * a), np.sqrt(2 * b)
    scale = np.abs(y[:6]).max() + prm[0] * np.abs(eps).max() + prm[8]
    return abs(ga - gb) <= 1e-10 * gb + 1e-12 * scale


def check_trace(tr, eps, hist, prm, barlat):
    """Recompute each traced step length from the traced merit values with the
    printed formulas; returns the number of line-search updates checked."""
    n_upd = 0
    for r in tr:
        psi0, psi1 = r["psi0"], r["psi1"]
        assert same_merit(psi0, merit_numpy(r["y"], eps, hist, prm, barlat), r["y"], eps, prm)
        zs, ps = r["zetas"], r["psis"]
        if psi1 < (1.0 - 2.0 * BETA) * psi0:  # Goldstein at the full step
            assert len(zs) == 0 and r["zeta"] == 1.0
            continue
        assert len(zs) >= 1
        assert zs[0] == psi0 / (psi0 + psi1)  # Eq. (alpha_init)
        for j in range(len(zs)):
            ok = ps[j] < (1.0 - 2.0 * BETA * zs[j]) * psi0
            if j < len(zs) - 1:
                assert not ok  # every rejected candidate fails the Goldstein test
                # Eq. (alpha_update_ls) then Eq. (alpha_safeguard)
                assert zs[j + 1] == max(ETA * zs[j], psi0 / (psi0 + ps[j]))
                n_upd += 1
            else:
                assert ok or len(zs) == oracle.TRACE_JMAX2
        assert r["zeta"] == zs[-1]
        for j in (0, len(zs) - 1):
            yt = r["y"] + zs[j] * r["dy"]
            assert same_merit(ps[j], merit_numpy(yt, eps, hist, prm, barlat), yt, eps, prm)
    return n_upd


def robustness_sample(prm):
    """A spread of the study's states (every 8th direction at three radii) and
    states whose line search runs the update loop of Eq. (alpha_update_ls)
    (directions 28, 74, 108 and 154 of 160 at large radii)."""
    allp = pi_plane_states(prm)
    idx = [a * 100 + b for a in range(0, 160, 8) for b in (20, 60, 95)]
    idx += [2860, 2890, 7490, 10860, 10890, 15490]
    return allp[idx]


def test_trace_recomputed_barlat(example):
    _, _, prm, eps = example
    states = np.vstack([eps[None, :], robustness_sample(prm)])
    n_upd = 0
    n_ls = 0
    for e in states:
        it, _, tr = oracle.local_return(e, np.zeros(7), prm, BARLAT, kmax=40)
        n_upd += check_trace(tr, e, np.zeros(7), prm, True)
        n_ls += sum(1 for r in tr if len(r["zetas"]))
    # the sample exercises both the initial candidate and the update loop
    assert n_ls > 20 and n_upd > 20


def test_trace_recomputed_hill_with_hardening():
    """Hill-48 with Swift hardening far outside the yield surface."""
    prm = np.array([200000.0, 0.3, 0.25, 0.7, 0.4, 1.5, 1.5, 1.5, 500.0, 0.01, 0.2])
    rng = np.random.default_rng(17)
    n_ls = 0
    for _ in range(30):
        # deviatoric strain up to about 20 times the yield strain (a large
        # hydrostatic part would only add rounding of cancelling stress terms)
        A = rng.standard_normal((3, 3))
        A = A + A.T
        A -= np.trace(A) / 3 * np.eye(3)
        eps = tensor_to_mandel(0.02 * A)
        hist = np.r_[0.002 * rng.standard_normal(6), 0.0]
        hist[2] = -hist[0] - hist[1]
        it, _, tr = oracle.local_return(eps, hist, prm, 0)
        assert it >= 0
        check_trace(tr, eps, hist, prm, False)
        n_ls += sum(1 for r in tr if len(r["zetas"]))
    assert n_ls >= 0  # Hill-48 mostly takes full steps; every step is still checked


def test_newton_direction_slope(example):
    """psi'(0) = -2 psi(0) along the Newton direction (App. B): pins the
    analytic Jacobian of Eq. (local_cpp) and the direction solve."""
    _, _, prm, eps = example
    for e in np.vstack([eps[None, :], robustness_sample(prm)[::7]]):
        _, _, tr = oracle.local_return(e, np.zeros(7), prm, BARLAT, kmax=40)
        for r in tr[:4]:
            h = 1e-6
            fp = oracle.local_merit(e, np.zeros(7), prm, r["y"] + h * r["dy"], BARLAT)
            fm = oracle.local_merit(e, np.zeros(7), prm, r["y"] - h * r["dy"], BARLAT)
            slope = (fp - fm) / (2 * h)
            assert abs(slope + 2 * r["psi0"]) <= 1e-6 * 2 * r["psi0"]


# ---- the robustness study

def test_robustness_study(example):
    ls, _, prm, _ = example
    study = ls["robustness_study"]
    pts = pi_plane_states(prm, r_max=study["outer_surface_scale"])
    assert len(pts) == study["n_states"]
    kmax = study["k_max"]
    plain = oracle.local_return_batch(pts, np.zeros(7), prm, BARLAT, line_search=False, kmax=kmax)
    with_ls = oracle.local_return_batch(pts, np.zeros(7), prm, BARLAT, line_search=True, kmax=kmax)
    long_ls = oracle.local_return_batch(pts, np.zeros(7), prm, BARLAT, line_search=True, kmax=100)
    n = len(pts)
    fail_plain = int((plain < 0).sum())
    fail_ls = int((with_ls < 0).sum())
    within20 = int(((with_ls >= 0) & (with_ls <= study["line_search_most_within_iterations"])).sum())
    print(f"standard Newton: {fail_plain} of {n} not converged in {kmax}; line search: {fail_ls} not converged "
          f"in {kmax}, {within20} within 20, all within {int(long_ls.max())}")
    # paper: about 9,600 of about 16,000 fail without the line search
    assert 0.5 * n <= fail_plain <= 0.7 * n
    assert abs(fail_plain - study["standard_newton_failures"]) <= 0.05 * n
    # with it: all converge, most within 20 iterations
    assert (long_ls >= 0).all()
    assert fail_ls <= 0.01 * n
    assert within20 >= 0.8 * n


# ---- planted mistakes fail the recomputation

MUTATIONS = {
    "safeguard_min": ("zn = fmax(LS_ETA * zs[jj], zn);", "zn = fmin(LS_ETA * zs[jj], zn);"),
    "update_numerator": ("double zn = psi0 / (psi0 + ps[jj]);", "double zn = ps[jj] / (psi0 + ps[jj]);"),
}

CHILD = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[2])
import oracle, test_oracle_linesearch as t
ls, coef = t.golden()
oracle.set_barlat(coef)
prm = t.example_params(ls)
try:
    for e in t.robustness_sample(prm):
        _, _, tr = oracle.local_return(e, np.zeros(7), prm, oracle.MODEL_BARLAT, kmax=40)
        t.check_trace(tr, e, np.zeros(7), prm, True)
except AssertionError:
    print("CAUGHT")
    sys.exit(0)
print("MISSED")
"""


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1
    with tempfile.TemporaryDirectory() as d:
        for f in ("oracle.c", "oracle.h"):
            shutil.copy(os.path.join(ROOT, "oracle", f), d)
        with open(os.path.join(d, "oracle.c"), "w") as f:
            f.write(src.replace(old, new))
        lib = os.path.join(d, "liboracle_mut.so")
        subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", os.path.join(d, "oracle.c"),
                               "-o", lib, "-lm"])
        env = dict(os.environ, ORACLE_LIB=lib)
        out = subprocess.run([sys.executable, "-c", CHILD, ROOT, HERE], env=env, capture_output=True, text=True,
                             timeout=300)
    assert "CAUGHT" in out.stdout, out.stdout + out.stderr
