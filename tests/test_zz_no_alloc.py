"""fem_residual_vjp_noalloc (static device scratch, no workspace argument)
against fem_residual_vjp on the same inputs: two calls in a row, the second
on a smaller mesh, in FP64 and FP32-mixed; the outputs must be bitwise equal
(the same kernels run in the same order on the same inputs)."""
import sys

import numpy as np
import pytest

from helpers import gpu_problem
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


def run_both(fem, p, prec):
    mesh, params, d, h, _, lam = gpu_problem(p, fem)
    ref = fem.residual_vjp(mesh, params, d, h, lam, prec=prec)
    gu = torch.full((1, fem.NGRAD), float("nan"), dtype=torch.float64, device="cuda")
    ge = torch.full((fem.NGRAD, p.n_elems), float("nan"), dtype=torch.float64, device="cuda")
    dg = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    fem.residual_vjp_noalloc(mesh, params, d, h, lam, gu, ge, dg, prec=prec)
    # g_uniform alone (the per-element sums then live in the scratch array)
    gu2 = torch.full((1, fem.NGRAD), float("nan"), dtype=torch.float64, device="cuda")
    fem.residual_vjp_noalloc(mesh, params, d, h, lam, gu2, None, None, prec=prec)
    torch.cuda.synchronize()
    return ref, gu, ge, dg, gu2


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_noalloc_matches_workspace_call_twice(fem, prec_name):
    prec = fem.FP64 if prec_name == "fp64" else fem.FP32_MIXED
    big = synth.small_slab(71, 30, 20, 4, per_element=True, strain=0.02)
    small = synth.small_slab(72, 9, 5, 2, strain=0.02)
    for p in (big, small):
        say("vjp noalloc", prec_name, p.n_elems)
        ref, gu, ge, dg, gu2 = run_both(fem, p, prec)
        r_gu = ref.g_uniform.cpu().numpy()
        r_ge = ref.g_elem.cpu().numpy()
        assert np.any(r_ge != 0.0)  # some plastic Gauss points
        assert np.array_equal(gu.cpu().numpy(), r_gu)
        assert np.array_equal(ge.cpu().numpy(), r_ge)
        assert np.array_equal(dg.cpu().numpy(), ref.diag.cpu().numpy())
        assert np.array_equal(gu2.cpu().numpy(), r_gu)
