"""Parity of the HIP path (through the C ABI) with the oracle for the model
options: Voce hardening, a material orientation (one rotation, or one per
element) and the F-bar element, in the forward call (R, K, history, diag)
and the parameter VJP, FP64 within 1e-10 and FP32-mixed within 1e-5."""
import sys

import numpy as np
import pytest

import oracle
from helpers import (TOL_FP64, TOL_MIXED, gpu_forward, gpu_problem, hist_rel, oracle_forward, oracle_model,
                     rel_inf, residual_scale)
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


# (hardening, fbar, orient) on a uniform and a per-element slab
MODELS = {
    "voce": ("voce", False, None),
    "orient": ("swift", False, "uniform"),
    "voce_orient_pe": ("voce", False, "per_element"),
    "fbar": ("swift", True, None),
    "fbar_voce_orient": ("voce", True, "uniform"),
}


def problem(name, per_element):
    hard, fbar, orient = MODELS[name]
    base = synth.small_slab(61 if per_element else 62, 7, 4, 3, per_element=per_element)
    return synth.with_model(base, 8, hard, fbar, orient)


@pytest.mark.parametrize("per_element", [False, True])
@pytest.mark.parametrize("name", list(MODELS))
def test_forward_matches_oracle(fem, name, per_element):
    p = problem(name, per_element)
    say("model forward", p.name, p.n_elems)
    o = oracle_forward(p)
    assert (o["hist"][6] != p.hist_n[6]).any()  # some Gauss points yield
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
    assert np.array_equal(o["hist"][6] != p.hist_n[6], m["hist"][6] != p.hist_n[6])


@pytest.mark.parametrize("per_element", [False, True])
@pytest.mark.parametrize("name", list(MODELS))
def test_vjp_matches_oracle(fem, name, per_element):
    p = problem(name, per_element)
    say("model vjp", p.name, p.n_elems)
    model, orient = oracle_model(p)
    gu, ge, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam, model=model, orient=orient)
    assert np.any(ge != 0.0)
    mesh, params, d, h, _, lam = gpu_problem(p, fem)
    for prec, tol in ((fem.FP64, TOL_FP64), (fem.FP32_MIXED, TOL_MIXED)):
        v = fem.residual_vjp(mesh, params, d, h, lam, prec=prec)
        torch.cuda.synchronize()
        hu, he = v.g_uniform[0].cpu().numpy(), v.g_elem.cpu().numpy()
        assert np.abs(hu - gu).max() <= tol * np.abs(gu).max(), prec
        assert np.abs(he - ge).max() <= tol * np.abs(ge).max(), prec


def test_identity_orientation_equals_no_orientation(fem):
    """Theta = I (per element) runs the orientation kernel and must give the
    plain kernel's results to rounding."""
    base = synth.small_slab(63, 5, 4, 2)
    p = synth.with_model(base, 9, "swift", False, np.tile(np.eye(3).ravel(), (base.n_elems, 1)))
    a = gpu_forward(base, fem, fem.FP64)
    b = gpu_forward(p, fem, fem.FP64, csr=a["csr"])
    assert rel_inf(b["K"], a["K"]) <= 1e-13
    assert rel_inf(b["R"], a["R"]) <= 1e-12
    assert hist_rel(b["hist"], a["hist"]) <= 1e-13


def test_unknown_model_flags_are_rejected(fem):
    p = synth.small_slab(64, 2, 2, 1)
    mesh, params, d, h, bc, lam = gpu_problem(p, fem)
    params.model = 8
    with pytest.raises(fem.FemError) as ei:
        fem.residual_tangent(mesh, fem.csr_pattern(mesh), params, d, h, prec=fem.FP64)
    assert ei.value.code == fem.FEM_EINVAL
    with pytest.raises(fem.FemError):
        fem.residual_vjp(mesh, params, d, h, lam, prec=fem.FP64)
