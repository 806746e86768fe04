"""Parity of the Barlat Yld2004-18p forward path (through the C ABI) with the
oracle: R, K, history and diag for the published AA6111 coefficients (m = 8),
alone and with Voce hardening, one orientation per element and the F-bar
element, FP64 within 1e-10 and FP32-mixed (FP64 local update, K in FP32)
within 1e-5; the App. A reduction (unit coefficients, m = 2) equals the
Hill-48 kernel at its von Mises parameters; the VJP rejects Barlat."""
import sys

import numpy as np
import pytest

from helpers import TOL_FP64, TOL_MIXED, gpu_forward, gpu_problem, hist_rel, oracle_forward, rel_inf, residual_scale
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


# (hardening, F-bar, orientation, strain): strain 0.004 leaves about a third
# of the Gauss points elastic, 0.03 none
CASES = {"barlat": ("swift", False, None, 0.03), "barlat_voce_orient_pe": ("voce", False, "per_element", 0.03),
         "barlat_fbar_mixed_state": ("swift", True, None, 0.004)}


@pytest.mark.parametrize("name", list(CASES))
def test_barlat_forward_matches_oracle(fem, name):
    hard, fbar, orient, strain = CASES[name]
    p = synth.with_model(synth.small_slab(101, 5, 4, 2, strain=strain), 14, hard, fbar, orient,
                         barlat=synth.BARLAT_AA6111)
    say("barlat forward", name, p.n_elems)
    o = oracle_forward(p)
    assert (o["hist"][6] != p.hist_n[6]).any()
    assert o["diag"][0] == 0
    sR = residual_scale(p)
    g = gpu_forward(p, fem, fem.FP64)
    assert rel_inf(g["R"], o["R"], sR) <= TOL_FP64
    assert rel_inf(g["K"], o["K"]) <= TOL_FP64
    assert hist_rel(g["hist"], o["hist"]) <= TOL_FP64
    assert np.array_equal(g["diag"], o["diag"])
    m = gpu_forward(p, fem, fem.FP32_MIXED, csr=g["csr"])
    assert rel_inf(m["R"], o["R"], sR) <= TOL_MIXED
    assert rel_inf(m["K"], o["K"]) <= TOL_MIXED
    assert hist_rel(m["hist"], o["hist"]) <= TOL_MIXED


def test_unit_coefficients_reduce_to_von_mises(fem):
    base = synth.small_slab(102, 4, 3, 2, strain=0.03)
    base.prm[2:8] = [0.5, 0.5, 0.5, 1.5, 1.5, 1.5]
    p = synth.with_model(base, 15, barlat=np.r_[np.ones(18), 2.0])
    a = gpu_forward(base, fem, fem.FP64)
    b = gpu_forward(p, fem, fem.FP64, csr=a["csr"])
    assert (a["hist"][6] != base.hist_n[6]).any()
    assert rel_inf(b["K"], a["K"]) <= 1e-9
    assert rel_inf(b["R"], a["R"]) <= 1e-9
    assert hist_rel(b["hist"], a["hist"]) <= 1e-9


def test_vjp_rejects_barlat(fem):
    p = synth.with_model(synth.small_slab(103, 2, 2, 1), 16, barlat=synth.BARLAT_AA6111)
    mesh, params, d, h, bc, lam = gpu_problem(p, fem)
    with pytest.raises(fem.FemError) as ei:
        fem.residual_vjp(mesh, params, d, h, lam, prec=fem.FP64)
    assert ei.value.code == fem.FEM_EINVAL


def robustness_problem(n_theta=160, n_r=100):
    """Trial states of App. B's robustness study (Barlat Yld2004-18p with the
    verification table's fit, E = 1000, nu = 0.3, sigma0 = 1, perfect
    plasticity, trial stresses in the deviatoric principal-stress plane between
    the yield surface and 30 times it), one state per element: disjoint unit
    cubes, each deformed homogeneously with principal stretches exp(eps_i)
    along the material axes, so that the log strain of every Gauss point is
    the state's trial strain."""
    from test_oracle_linesearch import BARLAT, example_params, golden, pi_plane_states
    import oracle
    ls, coef = golden()
    oracle.set_barlat(coef)
    prm = example_params(ls)
    eps = pi_plane_states(prm, n_theta=n_theta, n_r=n_r, r_max=ls["robustness_study"]["outer_surface_scale"])
    n = eps.shape[0]
    Xc, cc = synth.hex_grid(1, 1, 1, 1.0, 1.0, 1.0)
    X = np.concatenate([Xc + np.array([2.0 * i, 0.0, 0.0]) for i in range(n)])
    conn = np.concatenate([cc + 8 * i for i in range(n)]).astype(np.int32)
    d = np.zeros_like(X)
    for i in range(n):
        Fd = np.exp(eps[i, :3]) - 1.0
        xi = X[8 * i:8 * i + 8]
        d[8 * i:8 * i + 8] = (xi - xi.mean(axis=0)) * Fd
    p = synth.Problem("barlat_robustness", X, conn, d, np.zeros((7, 8 * n)), prm, None, None,
                      barlat=np.asarray(coef, dtype=np.float64))
    assert BARLAT == oracle.MODEL_BARLAT
    return p


def test_barlat_return_map_over_the_robustness_states(fem):
    """The GPU closest-point iteration (radial start on the current yield
    surface, Newton on (T, dgamma), line search of App. B on the merit of
    Eq. (merit)) over the robustness study's 16,000 trial states (160
    directions x 100 radii), up to 30 times the yield surface: every Gauss
    point converges (diag zero) to the oracle's state (Alg. C2 from the
    trial state): history within 1e-10, residual within 1e-9 (both sides
    may stop on a stalled decrease of the scaled local residual below 1e-9,
    the stop rule of the local iteration, at different iterates inside that
    band; over the 384,000 residual entries the largest difference is about
    1.2e-10 of the largest entry)."""
    p = robustness_problem()
    say("barlat robustness states", p.n_elems)
    o = oracle_forward(p, bc=False, want_K=False)
    assert list(o["diag"]) == [0, 0, 0, 0]
    assert (o["hist"][6] > 0).all()  # every state is plastic
    g = gpu_forward(p, fem, fem.FP64, bc=False, want_K=False)
    assert list(g["diag"]) == [0, 0, 0, 0]
    assert hist_rel(g["hist"], o["hist"]) <= TOL_FP64
    assert rel_inf(g["R"], o["R"]) <= 1e-9
