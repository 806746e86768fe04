"""The adaptive load path on the GPU (loadpath.solve: Newton with
extrapolated starts, CG or BiCGSTAB with Eisenstat-Walker tolerances,
FP64 residual with a float tangent) against the oracle's dense Newton
(oracle.adjoint.simulate) run over the same accepted increments, on the
unit-cube forward problem of the performance study (Hill-48 from the
r-values, Voce, x = 0 clamped, x = 1 moved by t (0.2, 0.1))."""
import sys

import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("variant,t_end,pc", [("plain", 1.0, "PC_AMG"), ("fbar", 0.3, "PC_AMG"),
                                              ("plain", 1.0, "PC_BLOCK_JACOBI")])
def test_load_path_matches_oracle_newton(fem, variant, t_end, pc):
    from paper_2606_17390_amd import loadpath
    p = synth.unit_cube_forward(3)
    fbar = variant == "fbar"
    mesh = fem.Mesh(p.X, p.conn)
    csr = fem.csr_pattern(mesh)
    params = fem.Params(p.prm, p.n_elems, hardening="voce", fbar=fbar)
    bc = torch.as_tensor(p.bc_mask).cuda()
    u1 = p.meta["bc_at"](1.0)
    h0 = torch.zeros((7, 8 * p.n_elems), dtype=torch.float64, device="cuda")
    say(f"load path {variant}: {3 * p.n_nodes} dofs to t = {t_end}")
    res = loadpath.solve(mesh, csr, params, bc, torch.as_tensor(u1).cuda(), h0, dt0=0.02, dt_max=0.1, ftol=1e-11,
                         t_end=t_end, log=say, precond=getattr(fem, pc))
    ts = [s[0] for s in res["steps"]]
    assert abs(ts[-1] - t_end) <= 1e-12 and all(s[2] >= 1 for s in res["steps"])
    assert res["newton_iterations"] == sum(s[2] for s in res["steps"])
    model = oracle.MODEL_VOCE | (oracle.MODEL_FBAR if fbar else 0)
    ds, hs = oadj.simulate(p.X, p.conn, p.prm, p.bc_mask.astype(bool), [t * u1 for t in ts],
                           np.zeros((7, 8 * p.n_elems)), model=model)
    d_ref, h_ref = ds[-1], hs[-1]
    d = res["d"].cpu().numpy()
    h = res["hist"].cpu().numpy()
    err_d = np.abs(d - d_ref).max() / np.abs(d_ref).max()
    err_h = np.abs(h - h_ref).max() / np.abs(h_ref).max()
    say(f"{len(ts)} increments, {res['newton_iterations']} Newton iterations; |d - d_ref| {err_d:.2e}, "
        f"|h - h_ref| {err_h:.2e}, alpha max {h_ref[6].max():.4f}")
    assert h_ref[6].max() > 0.01  # the path is well into the plastic range
    assert err_d <= 1e-8 and err_h <= 1e-8
