"""The C ABI library loads on a host without a GPU, exports every function
declared in include/fem.h, and rejects invalid arguments before touching the
device (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fem.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2606_17390_amd import fem
    return fem.lib()


def test_header_declares_the_three_calls():
    names = declared_functions()
    for f in ("fem_csr_pattern", "fem_residual_tangent", "fem_residual_vjp"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_2606_17390_amd import fem
    assert sorted(fem.EXPORTS) == declared_functions()


def test_version_and_workspace_queries(lib):
    assert lib.fem_version() >= 100
    assert lib.fem_csr_workspace_bytes(125, 64) > 0
    assert lib.fem_csr_workspace_bytes(-1, 0) == 0
    assert lib.fem_forward_workspace_bytes(125, 64, 1) >= 64 * (24 * 8 + 576 * 4)
    assert lib.fem_forward_workspace_bytes(125, 64, 0) >= 64 * (24 * 8 + 576 * 8)
    assert lib.fem_vjp_workspace_bytes(64, 1) >= 7 * 64 * 8


def test_invalid_arguments_are_rejected_on_the_host(lib):
    from paper_2606_17390_amd import fem
    assert lib.fem_csr_pattern(None, None, None, 0, None) == fem.FEM_EINVAL
    assert b"must not be NULL" in lib.fem_last_error()
    rc = lib.fem_residual_tangent(None, None, None, None, None, None, None, 0, None, None, None, None, None,
                                  None, 0, None)
    assert rc == fem.FEM_EINVAL
    rc = lib.fem_residual_vjp(None, None, None, None, None, None, 0, None, None, None, None, 0, None)
    assert rc == fem.FEM_EINVAL
    # negative sizes
    m = fem.FemMesh(-1, 0, None, None)
    c = fem.FemCsr(0, 0, None, None, None, None, None)
    assert lib.fem_csr_pattern(ctypes.byref(m), ctypes.byref(c), None, 0, None) == fem.FEM_EINVAL
    # bad precision with otherwise empty problem
    m = fem.FemMesh(0, 0, None, None)
    p = fem.FemParams()
    assert lib.fem_residual_tangent(ctypes.byref(m), None, None, ctypes.byref(p), None, None, None, 9, None,
                                    None, None, None, None, None, 0, None) == fem.FEM_EINVAL


def test_launch_configuration_round_trip(lib):
    from paper_2606_17390_amd import fem
    cfg = fem.FemLaunch(256, 4, 0)
    assert lib.fem_set_launch(0, 1, ctypes.byref(cfg)) == fem.FEM_OK
    got = fem.FemLaunch()
    assert lib.fem_get_launch(0, 1, ctypes.byref(got)) == fem.FEM_OK
    assert (got.block, got.waves_per_cu, got.xcd_remap) == (256, 4, 0)
    assert lib.fem_set_launch(0, 1, None) == fem.FEM_OK
    bad = fem.FemLaunch(96, 4, 0)
    assert lib.fem_set_launch(0, 1, ctypes.byref(bad)) == fem.FEM_EINVAL
    assert lib.fem_set_launch(5, 1, None) == fem.FEM_EINVAL


def test_product_path_does_not_import_the_oracle():
    """The binding, kernels and bench's timed path never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2606_17390_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "oracle." not in txt.replace("the oracle", ""), f


def test_solver_arguments_are_rejected_on_the_host(lib):
    """fem_solve validates its arguments before any device work: the pointers
    below are never dereferenced."""
    from paper_2606_17390_amd import fem
    fake = ctypes.c_void_p(256)

    def solve(n_rows=6, nnz=18, prec=fem.FP64, method=1, pc=1, max_iter=10, rtol=1e-8, ws_bytes=1 << 40,
              b=fake, x=fake):
        c = fem.FemCsr(n_rows, nnz, fake, fake, None, None, None)
        it = ctypes.c_int32(-1)
        res = ctypes.c_double(-1.0)
        rc = lib.fem_solve(ctypes.byref(c), fake, prec, method, pc, b, x, max_iter, rtol, ctypes.byref(it),
                           ctypes.byref(res), fake, ws_bytes, None)
        return rc, it.value, res.value

    assert solve(method=4)[0] == fem.FEM_EINVAL and b"Krylov" in lib.fem_last_error()
    # GMRES needs its basis: FEM_GMRES_RESTART + 1 more vectors; FGMRES also
    # the FEM_GMRES_RESTART preconditioned ones
    assert solve(method=2, ws_bytes=lib.fem_solver_workspace_bytes(6, 18))[0] == fem.FEM_ENOMEM
    gm = lib.fem_solver_workspace_bytes_method(3000, 9 * 27 * 1000, 2)
    assert gm >= lib.fem_solver_workspace_bytes(3000, 9 * 27 * 1000) + 31 * 3000 * 8
    fgm = lib.fem_solver_workspace_bytes_method(3000, 9 * 27 * 1000, 3)
    assert fgm >= gm + 30 * 3000 * 8
    assert solve(method=3, ws_bytes=lib.fem_solver_workspace_bytes_method(6, 18, 2))[0] == fem.FEM_ENOMEM
    assert lib.fem_solver_workspace_bytes_method(3000, 9 * 27 * 1000, 0) == lib.fem_solver_workspace_bytes(
        3000, 9 * 27 * 1000)
    assert solve(pc=5)[0] == fem.FEM_EINVAL and b"preconditioner" in lib.fem_last_error()
    assert solve(prec=7)[0] == fem.FEM_EINVAL
    assert solve(n_rows=5)[0] == fem.FEM_EINVAL  # not 3 n_nodes
    assert solve(nnz=17)[0] == fem.FEM_EINVAL  # not whole 3x3 blocks
    assert solve(max_iter=-1)[0] == fem.FEM_EINVAL
    assert solve(rtol=float("nan"))[0] == fem.FEM_EINVAL
    assert solve(b=None)[0] == fem.FEM_EINVAL
    assert solve(ws_bytes=16)[0] == fem.FEM_ENOMEM and b"workspace" in lib.fem_last_error()
    # an empty system is solved without any device work
    assert solve(n_rows=0, nnz=0) == (fem.FEM_OK, 0, 0.0)
    # workspace: vectors, the block preconditioner and the node-column list
    small, big = lib.fem_solver_workspace_bytes(3000, 9 * 27 * 1000), lib.fem_solver_workspace_bytes(3000, 10 ** 8)
    assert small >= 8 * 3000 * 8 + 3 * 3000 * 8 + 27 * 1000 * 4 and big - small >= 4 * (10 ** 8 // 9 - 27 * 1000)
    assert lib.fem_solver_workspace_bytes(-3, 0) == 0 and lib.fem_solver_workspace_bytes(3, -1) == 0


def test_multigrid_arguments_are_rejected_on_the_host(lib):
    """The multigrid entry points validate their arguments before any device
    work (the fake pointers below are never dereferenced)."""
    from paper_2606_17390_amd import fem
    fake = ctypes.c_void_p(256)
    h = ctypes.c_void_p()

    def create(n_rows=6, nnz=18, prec=fem.FP64, K=fake, out=True):
        c = fem.FemCsr(n_rows, nnz, fake, fake, None, None, None)
        return lib.fem_amg_create(ctypes.byref(c), K, prec, None, ctypes.byref(h) if out else None, None)

    assert create(out=False) == fem.FEM_EINVAL
    assert create(K=None) == fem.FEM_EINVAL and h.value is None
    assert create(prec=fem.FP64_K32) == fem.FEM_EINVAL  # K is FP64 or FP32
    assert create(n_rows=0, nnz=0) == fem.FEM_EINVAL and b"non-empty" in lib.fem_last_error()
    assert create(n_rows=5) == fem.FEM_EINVAL
    assert create(nnz=17) == fem.FEM_EINVAL and b"multiple of 9" in lib.fem_last_error()
    assert lib.fem_amg_update(None, fake, fem.FP64, None) == fem.FEM_EINVAL
    assert lib.fem_amg_apply(None, fake, fake, None) == fem.FEM_EINVAL
    assert lib.fem_amg_info(None, None, None, None, None, None) == fem.FEM_EINVAL
    assert lib.fem_amg_aggregates(None, 1, fake) == fem.FEM_EINVAL
    assert lib.fem_amg_destroy(None) == fem.FEM_OK
    assert lib.fem_amg_set_cycle(None, 1, 0) == fem.FEM_EINVAL
    c = fem.FemCsr(6, 18, fake, fake, None, None, None)
    it, res = ctypes.c_int32(-1), ctypes.c_double(-1.0)
    assert lib.fem_solve_amg(ctypes.byref(c), fake, fem.FP64, 1, None, fake, fake, 10, 1e-8, ctypes.byref(it),
                             ctypes.byref(res), fake, 1 << 40, None) == fem.FEM_EINVAL
    assert b"multigrid" in lib.fem_last_error()
    # fem_solve itself does not take the multigrid preconditioner
    assert lib.fem_solve(ctypes.byref(c), fake, fem.FP64, 1, fem.PC_AMG, fake, fake, 10, 1e-8, ctypes.byref(it),
                         ctypes.byref(res), fake, 1 << 40, None) == fem.FEM_EINVAL


def test_noalloc_vjp_rejects_meshes_beyond_its_scratch(lib):
    """fem_residual_vjp_noalloc refuses, before any device work, a mesh whose
    workspace exceeds its static scratch (64 MiB: about 1.1M elements)."""
    from paper_2606_17390_amd import fem
    n = 1_200_000
    assert lib.fem_vjp_workspace_bytes(n, 1) > fem.VJP_SCRATCH_MAX_BYTES
    m = fem.FemMesh(3 * n, n, None, None)
    rc = lib.fem_residual_vjp_noalloc(ctypes.byref(m), None, None, None, None, None, 0, None, None, None, None)
    assert rc == fem.FEM_ENOMEM
    assert b"maximum" in lib.fem_last_error()
    assert lib.fem_residual_vjp_noalloc(None, None, None, None, None, None, 0, None, None, None, None) == \
        fem.FEM_EINVAL


def test_header_is_plain_c(tmp_path):
    """include/fem.h is a C header: it compiles as C99 with -pedantic, every
    declared entry point taken by address (so a C caller can link them)."""
    import re
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    hdr = open(os.path.join(root, "include", "fem.h")).read()
    names = sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s+(fem_\w+)\(", hdr, re.M)))
    assert "fem_solve_amg" in names and "fem_residual_tangent" in names
    src = tmp_path / "use.c"
    src.write_text('#include "fem.h"\ntypedef void (*fn)(void);\nfn table[] = {' + ", ".join(f"(fn){n}" for n in names)
                   + "};\n")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(root, "include"), "-c", str(src), "-o", str(tmp_path / "use.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_binding_constants_match_the_header():
    """The Python binding's copies of the header's constants and enum values
    (levels, dense threshold, Krylov methods, cycle types)."""
    from paper_2606_17390_amd import fem
    h = open(os.path.join(ROOT, "include", "fem.h")).read()

    def define(name):
        return int(re.search(r"#define %s (\d+)" % name, h).group(1))

    def enum(name):
        return int(re.search(r"\b%s = (\d+)" % name, h).group(1))

    assert define("FEM_AMG_MAX_LEVELS") == fem.AMG_MAX_LEVELS
    assert define("FEM_AMG_DENSE_NODES") == fem.AMG_DENSE_NODES
    for k, v in fem.KRYLOV.items():
        assert enum("FEM_KRYLOV_" + k.upper()) == v
    for k, v in fem.AMG_CYCLE.items():
        assert enum("FEM_AMG_CYCLE_" + k.upper()) == v
    assert enum("FEM_PC_AMG") == fem.PC_AMG
