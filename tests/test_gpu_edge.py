"""Edge cases of the HIP path against the oracle (through the C ABI):

* nodes with more than 8 incident elements (duplicated elements; the
  assembly then takes its incident elements in several chunks of 8),
* an inverted element (detJ0 < 0 at its 8 Gauss points) and a displacement
  that turns det F negative (finite values, counted in diag),
* a non-finite displacement at one node (counted per Gauss point; every other
  row unaffected)."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
from helpers import TOL_FP64, TOL_MIXED, gpu_forward, gpu_problem, hist_rel, oracle_forward, rel_inf
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


def with_repeats(p, node, times):
    """p with every element around `node` repeated `times` more times (the
    node then has 8 (times + 1) incident elements)."""
    sel = np.nonzero((p.conn == node).any(axis=1))[0]
    conn = np.concatenate([p.conn] + [p.conn[sel]] * times).astype(np.int32)
    cols = (8 * sel[:, None] + np.arange(8)).ravel()
    hist = np.concatenate([p.hist_n] + [p.hist_n[:, cols]] * times, axis=1)
    prm = np.concatenate([p.prm] + [p.prm[sel]] * times) if p.per_element else p.prm
    return dataclasses.replace(p, conn=conn, hist_n=np.ascontiguousarray(hist), prm=prm)


def interior_node(p):
    nx, ny, nz = p.meta["nx"], p.meta["ny"], p.meta["nz"]
    return (nz // 2) * (ny + 1) * (nx + 1) + (ny // 2) * (nx + 1) + nx // 2


def test_more_than_8_elements_per_node(fem):
    base = synth.small_slab(46, 4, 3, 3, per_element=True)
    p = with_repeats(base, interior_node(base), 2)  # one node with 24 elements, neighbours with 10..20
    counts = np.bincount(p.conn.ravel(), minlength=p.n_nodes)
    assert counts.max() == 24 and (counts > 8).sum() > 8
    say(f"repeats: {p.n_elems} elements, max incidence {counts.max()}")
    o = oracle_forward(p)
    g = gpu_forward(p, fem, fem.FP64)
    assert np.array_equal(np.asarray(g["csr"].row_ptr.cpu()), o["row_ptr"])
    assert np.array_equal(np.asarray(g["csr"].col_idx.cpu()), o["col_idx"])
    assert rel_inf(g["K"], o["K"]) <= TOL_FP64
    assert rel_inf(g["R"], o["R"]) <= TOL_FP64
    assert hist_rel(g["hist"], o["hist"]) <= TOL_FP64
    m = gpu_forward(p, fem, fem.FP32_MIXED)
    assert rel_inf(m["K"], o["K"]) <= TOL_MIXED
    assert rel_inf(m["R"], o["R"]) <= TOL_MIXED
    # residual-only path (its own multi-chunk gather) and the VJP
    r = gpu_forward(p, fem, fem.FP64, want_K=False)
    assert np.array_equal(r["R"], g["R"])
    mesh, params, d, h, _, lam = gpu_problem(p, fem)
    v = fem.residual_vjp(mesh, params, d, h, lam, prec=fem.FP64)
    torch.cuda.synchronize()
    gu, ge, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam)
    assert rel_inf(v.g_elem.cpu().numpy(), ge) <= TOL_FP64
    assert rel_inf(v.g_uniform.cpu().numpy()[0], gu) <= TOL_FP64


def test_inverted_element_and_negative_det_f_are_counted(fem):
    p = synth.small_slab(47, 3, 3, 2)
    conn = p.conn.copy()
    conn[4] = conn[4][[4, 5, 6, 7, 0, 1, 2, 3]]  # mirrored: detJ0 < 0 at its 8 Gauss points
    d = p.d.copy()
    # push one node through its neighbours: det F < 0 at some Gauss points
    n = interior_node(p)
    d[n] += 2.5 * (p.X[n - 1] - p.X[n])
    prm = p.prm.copy()
    prm[8] = 1e12  # Swift K: elastic everywhere, so the strain this large has one answer
    q = dataclasses.replace(p, conn=conn, d=d, prm=prm)
    o = oracle_forward(q)
    assert o["diag"][0] == 0 and o["diag"][1] == 8 and o["diag"][2] > 0 and o["diag"][3] == 0
    say(f"inverted/negative det F: oracle diag {o['diag'].tolist()}")
    g = gpu_forward(q, fem, fem.FP64)
    assert g["diag"][1] == o["diag"][1] and g["diag"][2] == o["diag"][2] and g["diag"][3] == 0
    assert rel_inf(g["K"], o["K"]) <= TOL_FP64
    assert rel_inf(g["R"], o["R"]) <= TOL_FP64


@pytest.mark.parametrize("prec_name", ["FP64", "FP32_MIXED"])
def test_non_finite_displacement_is_counted_and_contained(fem, prec_name):
    p = synth.small_slab(49, 3, 3, 2)
    n = interior_node(p)
    d = p.d.copy()
    d[n] = np.nan
    q = dataclasses.replace(p, d=d)
    o = oracle_forward(q)
    assert o["diag"][3] == 64
    say(f"non-finite displacement: {prec_name}")
    g = gpu_forward(q, fem, getattr(fem, prec_name))
    assert g["diag"][3] == 64
    # rows of nodes that share no element with n are finite and match
    touched = np.unique(q.conn[(q.conn == n).any(axis=1)])
    keep = np.setdiff1d(np.arange(q.n_nodes), touched)
    rows = (3 * keep[:, None] + np.arange(3)).ravel()
    assert np.isnan(g["R"][(3 * touched[:, None] + np.arange(3)).ravel()]).any()
    assert np.all(np.isfinite(g["R"][rows]))
    tol = TOL_FP64 if prec_name == "FP64" else TOL_MIXED
    assert rel_inf(g["R"][rows], o["R"][rows]) <= tol


EXTREME_F = {
    "stretch": np.diag([3.0, 0.2, 1.0]),
    "stretch_shear": np.array([[3.0, 0.8, 0.0], [0.0, 0.2, 0.1], [0.3, 0.0, 1.0]]),
}


def extreme_problem(kind, hardening):
    """A 2x1x1 slab deformed homogeneously by an extreme increment (stretches 3
    and 0.2 in one step, hydrostatic stress near -8.5e4 MPa) from a plastic
    history alpha_n = 1.5 (with a small random plastic strain), so that the
    local Newton (Alg. C2) runs far from its start at every Gauss point."""
    p = synth.small_slab(83, 2, 1, 1)
    if hardening != "swift":
        p = synth.with_model(p, 84, hardening)
    F0 = EXTREME_F[kind]
    Xc = p.X.mean(axis=0)
    d = (p.X - Xc) @ (F0 - np.eye(3)).T
    rng = np.random.default_rng(85)
    h = np.zeros((7, 8 * p.n_elems))
    h[:3] = rng.uniform(-1e-3, 1e-3, (3, 8 * p.n_elems))
    h[:3] -= h[:3].mean(axis=0)  # plastic strain is deviatoric
    h[6] = 1.5
    return dataclasses.replace(p, d=d, hist_n=h, bc_mask=None)


@pytest.mark.parametrize("kind", list(EXTREME_F))
@pytest.mark.parametrize("hardening", ["swift", "voce"])
def test_extreme_increment_matches_oracle(fem, kind, hardening):
    """R, K, history and the diagnostic counters of an extreme increment
    against the oracle: both local solvers converge (diag zero) to the same
    state, in FP64 within 1e-10 and in the mixed form within 1e-5."""
    p = extreme_problem(kind, hardening)
    say("extreme increment", kind, hardening)
    o = oracle_forward(p, bc=False)
    assert list(o["diag"]) == [0, 0, 0, 0]
    assert (o["hist"][6] > 2.5).all()  # far into the plastic range
    g = gpu_forward(p, fem, fem.FP64, bc=False)
    assert list(g["diag"]) == list(o["diag"])
    assert rel_inf(g["R"], o["R"]) <= TOL_FP64
    assert rel_inf(g["K"], o["K"]) <= TOL_FP64
    assert hist_rel(g["hist"], o["hist"]) <= TOL_FP64
    m = gpu_forward(p, fem, fem.FP32_MIXED, bc=False)
    assert list(m["diag"]) == list(o["diag"])
    assert rel_inf(m["R"], o["R"]) <= TOL_MIXED
    assert rel_inf(m["K"], o["K"]) <= TOL_MIXED
    assert hist_rel(m["hist"], o["hist"]) <= TOL_MIXED
