"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: CSR pattern and elem_rank bit-exact; FP64 residual, tangent and history
within 1e-10 (normwise relative); FP32-mixed within 1e-5 of FP64."""
import sys

import numpy as np
import pytest

import oracle
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


CASES = {
    "tiny_cube": lambda: synth.tiny_cube(step=5),
    "single": lambda: synth.small_slab(41, 1, 1, 1),
    "ragged_7x3x2": lambda: synth.small_slab(42, 7, 3, 2, per_element=True),
    "ragged_13x5x3": lambda: synth.small_slab(43, 13, 5, 3),
    "sheet_slab": lambda: synth.sheet_slab(),
}


@pytest.mark.parametrize("name", list(CASES))
def test_pattern_bit_exact(fem, name):
    p = CASES[name]()
    say("pattern", name, p.n_elems)
    mesh, *_ = gpu_problem(p, fem)
    csr = fem.csr_pattern(mesh)
    rp, ci, rank = oracle.csr_pattern(p.conn, p.n_nodes)
    assert csr.nnz == len(ci)
    assert np.array_equal(csr.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(csr.col_idx.cpu().numpy(), ci)
    assert np.array_equal(csr.elem_rank.cpu().numpy(), rank)


def test_pattern_void_specimen_bit_exact(fem):
    p = synth.void_specimen()
    say("pattern void", p.n_elems)
    mesh, *_ = gpu_problem(p, fem)
    csr = fem.csr_pattern(mesh)
    rp, ci, rank = oracle.csr_pattern(p.conn, p.n_nodes)
    assert np.array_equal(csr.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(csr.col_idx.cpu().numpy(), ci)
    assert np.array_equal(csr.elem_rank.cpu().numpy(), rank)


def test_pattern_incidence_and_rebuild_in_place(fem):
    """The node -> element incidence (entries 8 e + i, ascending per node) is
    the one read off the connectivity, and a rebuild into the buffers of an
    existing pattern reproduces every array bit for bit."""
    p = synth.void_specimen()
    mesh, *_ = gpu_problem(p, fem)
    csr = fem.csr_pattern(mesh)
    flat = p.conn.ravel().astype(np.int64)
    order = np.argsort(flat, kind="stable")  # entries 8 e + i grouped by node, ascending
    ptr = np.concatenate([[0], np.cumsum(np.bincount(flat, minlength=p.n_nodes))])
    assert np.array_equal(csr.node_elem_ptr.cpu().numpy(), ptr)
    assert np.array_equal(csr.node_elem.cpu().numpy(), order)
    before = [t.cpu().numpy().copy() for t in (csr.row_ptr, csr.col_idx, csr.elem_rank, csr.node_elem_ptr,
                                                csr.node_elem)]
    for t in (csr.col_idx, csr.elem_rank, csr.node_elem):
        t.fill_(0)
    again = fem.csr_pattern(mesh, out=csr)
    assert again.col_idx.data_ptr() == csr.col_idx.data_ptr()
    after = [t.cpu().numpy() for t in (again.row_ptr, again.col_idx, again.elem_rank, again.node_elem_ptr,
                                       again.node_elem)]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)


def test_pattern_rejects_bad_meshes(fem):
    X, conn = synth.hex_grid(2, 1, 1)
    mesh = fem.Mesh(np.vstack([X, [[9.0, 9.0, 9.0]]]), conn)  # orphan node
    with pytest.raises(fem.FemError) as ei:
        fem.csr_pattern(mesh)
    assert ei.value.code == fem.FEM_EMESH
    bad = conn.copy()
    bad[1, 3] = 1000
    with pytest.raises(fem.FemError) as ei:
        fem.csr_pattern(fem.Mesh(X, bad))
    assert ei.value.code == fem.FEM_EMESH


@pytest.mark.parametrize("name", list(CASES))
def test_forward_fp64_matches_oracle(fem, name):
    p = CASES[name]()
    say("fp64 forward", name, p.n_elems)
    o = oracle_forward(p)
    g = gpu_forward(p, fem, fem.FP64)
    sR = residual_scale(p)
    assert rel_inf(g["R"], o["R"], sR) <= TOL_FP64
    assert rel_inf(g["K"], o["K"]) <= TOL_FP64
    assert hist_rel(g["hist"], o["hist"]) <= TOL_FP64
    assert abs(g["rnorm2"] - o["rnorm2"][1]) <= 1e-10 * o["rnorm2"][1]
    assert np.array_equal(g["diag"], o["diag"])


@pytest.mark.parametrize("name", ["ragged_13x5x3", "sheet_slab"])
def test_forward_mixed_within_1e5(fem, name):
    p = CASES[name]()
    say("mixed forward", name, p.n_elems)
    o = oracle_forward(p)
    g = gpu_forward(p, fem, fem.FP32_MIXED)
    sR = residual_scale(p)
    assert rel_inf(g["R"], o["R"], sR) <= TOL_MIXED
    assert rel_inf(g["K"], o["K"]) <= TOL_MIXED
    assert hist_rel(g["hist"], o["hist"]) <= TOL_MIXED
    # the elastic/plastic decision of every Gauss point equals the FP64 one
    plastic_o = o["hist"][6] != p.hist_n[6]
    plastic_g = g["hist"][6] != p.hist_n[6]
    assert np.array_equal(plastic_o, plastic_g)


def test_void_specimen_fp64_and_mixed(fem):
    p = synth.void_specimen()
    say("void forward", p.n_elems)
    o = oracle_forward(p)
    g = gpu_forward(p, fem, fem.FP64)
    s = np.abs(o["R"]).max()
    assert rel_inf(g["R"], o["R"], s) <= TOL_FP64
    assert rel_inf(g["K"], o["K"]) <= TOL_FP64
    assert hist_rel(g["hist"], o["hist"]) <= TOL_FP64
    gm = gpu_forward(p, fem, fem.FP32_MIXED, csr=g["csr"])
    assert rel_inf(gm["R"], o["R"], s) <= TOL_MIXED
    assert rel_inf(gm["K"], o["K"]) <= TOL_MIXED


def test_residual_only_and_no_bc(fem):
    p = CASES["ragged_7x3x2"]()
    o = oracle_forward(p, bc=False, want_K=False)
    g = gpu_forward(p, fem, fem.FP64, bc=False, want_K=False)
    assert rel_inf(g["R"], o["R"]) <= TOL_FP64
    assert abs(g["rnorm2"] - o["rnorm2"][1]) <= 1e-10 * o["rnorm2"][1]


@pytest.mark.parametrize("prec_name", ["FP64", "FP32_MIXED"])
@pytest.mark.parametrize("bc", [True, False])
def test_residual_same_with_and_without_tangent(fem, prec_name, bc):
    """R and ||R||^2 are assembled by the tangent kernel when K is requested
    and by the residual kernel otherwise: the two are bitwise equal."""
    p = CASES["ragged_13x5x3"]()
    prec = getattr(fem, prec_name)
    say(f"residual with/without K: {prec_name} bc={bc}")
    full = gpu_forward(p, fem, prec, bc=bc, want_K=True)
    ronly = gpu_forward(p, fem, prec, bc=bc, want_K=False)
    assert np.array_equal(full["R"], ronly["R"])
    assert full["rnorm2"] == ronly["rnorm2"]


def test_empty_mesh(fem):
    X = np.zeros((0, 3))
    conn = np.zeros((0, 8), dtype=np.int32)
    mesh = fem.Mesh(X, conn)
    csr = fem.csr_pattern(mesh)
    assert csr.nnz == 0
    params = fem.Params(synth.params(), 0)
    d = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    h = torch.zeros((7, 0), dtype=torch.float64, device="cuda")
    out = fem.residual_tangent(mesh, csr, params, d, h, prec=fem.FP64)
    torch.cuda.synchronize()
    assert float(out.rnorm2.cpu()[0]) == 0.0
    v = fem.residual_vjp(mesh, params, d, h, d, prec=fem.FP64)
    torch.cuda.synchronize()
    assert np.all(v.g_uniform.cpu().numpy() == 0.0)


@pytest.mark.parametrize("block", [64, 128, 256])
@pytest.mark.parametrize("remap", [0, 1])
def test_launch_configurations_agree(fem, block, remap):
    p = CASES["ragged_13x5x3"]()
    o = oracle_forward(p)
    try:
        fem.set_launch(fem.KERNEL_FORWARD, fem.FP64, block=block, waves_per_cu=4, xcd_remap=remap)
        g = gpu_forward(p, fem, fem.FP64)
    finally:
        fem.set_launch(fem.KERNEL_FORWARD, fem.FP64)
    assert rel_inf(g["K"], o["K"]) <= TOL_FP64
    assert rel_inf(g["R"], o["R"]) <= TOL_FP64


def test_invalid_arguments(fem):
    p = CASES["single"]()
    mesh, params, d, h, bc, lam = gpu_problem(p, fem)
    csr = fem.csr_pattern(mesh)
    out = fem.Forward(mesh, csr, fem.FP64)
    out.prec = 7
    with pytest.raises(fem.FemError) as ei:
        fem.residual_tangent(mesh, csr, params, d, h, out=out)
    assert ei.value.code == fem.FEM_EINVAL
    with pytest.raises(ValueError):
        fem._prec("fp16")
    out = fem.Forward(mesh, csr, fem.FP64)
    out.ws_bytes = 8
    with pytest.raises(fem.FemError) as ei:
        fem.residual_tangent(mesh, csr, params, d, h, out=out)
    assert ei.value.code == fem.FEM_ENOMEM
