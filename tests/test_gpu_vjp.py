"""Parity of the HIP parameter VJP (through the C ABI) with the oracle's
forward-mode implicit differentiation, central finite differences of the HIP
residual, and the torch.autograd.Function wrapper."""
import sys

import numpy as np
import pytest

import oracle
from helpers import TOL_FP64, TOL_MIXED, gpu_problem
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


VCASES = {
    "ragged_uniform": lambda: synth.small_slab(51, 9, 4, 2, strain=0.01),
    "ragged_per_elem": lambda: synth.small_slab(52, 11, 3, 3, per_element=True, strain=0.01),
    "sheet_slab": lambda: synth.sheet_slab(),
}


def gpu_vjp(p, fem, prec):
    mesh, params, d, h, bc, lam = gpu_problem(p, fem)
    v = fem.residual_vjp(mesh, params, d, h, lam, prec=prec)
    torch.cuda.synchronize()
    return v.g_uniform[0].cpu().numpy(), v.g_elem.cpu().numpy(), v.diag.cpu().numpy()


@pytest.mark.parametrize("name", list(VCASES))
def test_vjp_fp64_matches_oracle(fem, name):
    p = VCASES[name]()
    say("vjp fp64", name, p.n_elems)
    gu, ge, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam)
    hu, he, hd = gpu_vjp(p, fem, fem.FP64)
    assert np.abs(hu - gu).max() <= TOL_FP64 * np.abs(gu).max()
    assert np.abs(he - ge).max() <= TOL_FP64 * np.abs(ge).max()
    # elastic elements are exactly zero on both sides
    assert np.array_equal(ge == 0.0, he == 0.0)


@pytest.mark.parametrize("name", ["ragged_per_elem", "sheet_slab"])
def test_vjp_mixed_within_1e5(fem, name):
    p = VCASES[name]()
    gu, ge, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam)
    hu, he, _ = gpu_vjp(p, fem, fem.FP32_MIXED)
    assert np.abs(hu - gu).max() <= TOL_MIXED * np.abs(gu).max()
    assert np.abs(he - ge).max() <= TOL_MIXED * np.abs(ge).max()


def test_vjp_void_specimen(fem):
    p = synth.void_specimen()
    say("vjp void", p.n_elems)
    gu, ge, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam)
    hu, he, _ = gpu_vjp(p, fem, fem.FP64)
    assert np.abs(hu - gu).max() <= TOL_FP64 * np.abs(gu).max()
    assert np.abs(he - ge).max() <= TOL_FP64 * np.abs(ge).max()


def test_vjp_matches_fd_of_hip_residual(fem):
    """Central FD (h = 1e-6 |theta_k|) of lam^T R(theta) computed by the HIP
    forward pass, against the HIP VJP."""
    p = VCASES["ragged_uniform"]()
    mesh, params, d, h, bc, lam = gpu_problem(p, fem)
    hu, _, _ = gpu_vjp(p, fem, fem.FP64)

    def lamR(prm):
        pr = fem.Params(prm, p.n_elems)
        out = fem.residual_tangent(mesh, None, pr, d, h, prec=fem.FP64, want_K=False, want_hist=False)
        return float(torch.dot(out.R, lam.reshape(-1)).cpu())

    for k, col in enumerate(synth.GRAD_PARAM_INDEX):
        step = 1e-6 * abs(p.prm[col])
        pp, pm = p.prm.copy(), p.prm.copy()
        pp[col] += step
        pm[col] -= step
        fd = (lamR(pp) - lamR(pm)) / (2 * step)
        assert abs(hu[k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(hu).max())


def test_all_elastic_vjp_is_zero(fem):
    p = synth.small_slab(53, 4, 3, 2, strain=1e-7, alpha_max=0.0)
    p.hist_n[:] = 0.0
    hu, he, _ = gpu_vjp(p, fem, fem.FP64)
    assert np.all(hu == 0.0) and np.all(he == 0.0)


def test_autograd_function(fem):
    p = VCASES["ragged_uniform"]()
    mesh, params, d, h, bc, lam = gpu_problem(p, fem)
    base = torch.as_tensor(p.prm)
    theta = torch.tensor([p.prm[c] for c in synth.GRAD_PARAM_INDEX], dtype=torch.float64, requires_grad=True)
    R = fem.ResidualFn.apply(theta, base, mesh, d, h, fem.FP64)
    (R * lam.reshape(-1)).sum().backward()
    gu, _, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam)
    assert np.abs(theta.grad.numpy() - gu).max() <= TOL_FP64 * np.abs(gu).max()
    # per-element parameters
    the = torch.tensor(np.tile(theta.detach().numpy()[:, None], (1, p.n_elems)), requires_grad=True)
    R2 = fem.ResidualFn.apply(the, base, mesh, d, h, fem.FP64)
    (R2 * lam.reshape(-1)).sum().backward()
    _, ge, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam)
    assert np.abs(the.grad.cpu().numpy() - ge).max() <= TOL_FP64 * np.abs(ge).max()
