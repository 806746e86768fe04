"""Host-side logic of bench.py (no GPU): the algorithmic bytes per Gauss
point of the pass, recounted here from their definition (every input and
output array of the pass once; 383 B in FP64, 261 B with the tangent in
FP32 on the 100^3 cube), the node-block count of the 100^3 pattern from its
closed form, the source-hash gate of the recorded counter figures, and the
one-GPU exit."""
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def cube(n):
    return types.SimpleNamespace(n_elems=n ** 3, n_nodes=(n + 1) ** 3)


def nnz_of_cube(n):
    # each node couples to the nodes of its (clipped) 3x3x3 neighbourhood:
    # per axis 3 (interior) or 2 (face) choices, 3 (n + 1) - 2 in total
    return 9 * (3 * (n + 1) - 2) ** 3


def test_pattern_size_of_the_large_cube():
    assert nnz_of_cube(100) == 245_438_109


@pytest.mark.parametrize("mixed,per_gp", [(False, 383.256), (True, 260.537)])
def test_algorithmic_bytes_per_gauss_point(mixed, per_gp):
    p = cube(100)
    nnz = nnz_of_cube(100)
    ngp = 8 * p.n_elems
    kb = 4 if mixed else 8
    # per Gauss point: history in and out (7 doubles each), the tangent
    # values, coordinates and displacements, connectivity, three per-element
    # parameter columns, the element ranks, row pointers and the residual
    expect = (2 * 7 * 8 + nnz * kb / ngp + 2 * 3 * 8 * p.n_nodes / ngp + 8 * 4 / 8 + 3 * 8 / 8 + 64 / 8
              + (3 * p.n_nodes + 1) * 4 / ngp + 3 * 8 * p.n_nodes / ngp)
    got = bench.algorithmic_bytes(p, nnz, mixed, 3) / ngp
    assert got == pytest.approx(expect, rel=1e-12)
    assert got == pytest.approx(per_gp, abs=5e-4)


def test_design_bytes_include_the_element_scratch():
    p = cube(100)
    nnz = nnz_of_cube(100)
    for mixed in (False, True):
        kb = 4 if mixed else 8
        d = bench.design_bytes(p, nnz, mixed, 3, 0)
        alg = bench.algorithmic_bytes(p, nnz, mixed, 3)
        # the K^e scratch is written by the element kernel and read by the
        # assembly: twice 576 values per element beyond the method's bytes
        assert sum(d.values()) > alg + 2 * 576 * kb * p.n_elems * 0.99
        assert d["assemble_tangent"] >= nnz * kb + 576 * kb * p.n_elems


def test_counter_figures_are_gated_by_the_source_hash(monkeypatch):
    sha = bench.kernel_source_sha()
    monkeypatch.setitem(bench.PROFILED, "sha", sha)
    assert bench.profiled("fp64", "flop_per_gp") == bench.PROFILED["fp64"]["flop_per_gp"]
    assert bench.profiled("mixed", "traffic", "fwd_kernel") == bench.PROFILED["mixed"]["traffic"]["fwd_kernel"]
    monkeypatch.setitem(bench.PROFILED, "sha", "0" * 16)
    assert bench.profiled("fp64", "flop_per_gp") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
