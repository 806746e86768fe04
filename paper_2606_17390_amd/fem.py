"""ctypes binding of libfem.so (C ABI in include/fem.h).

Only argument marshalling lives here: every step of the hot path runs in the
HIP kernels of libfem.so.  Device buffers are torch tensors (torch is used for
device memory and streams only).  If libfem.so is missing the first call
raises; there is no fallback.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfem.so")

FEM_OK, FEM_EINVAL, FEM_EHIP, FEM_ENOMEM, FEM_EOVERFLOW, FEM_EMESH, FEM_ENOCONV = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_MIXED, FP64_K32 = 0, 1, 2
NPARAM, NGRAD = 11, 7
MODEL_VOCE, MODEL_FBAR, MODEL_BARLAT = 1, 2, 4  # fem_params.model flags
KERNEL_FORWARD, KERNEL_VJP, KERNEL_ASSEMBLE_K, KERNEL_ASSEMBLE_R = 0, 1, 2, 3

_c_i32, _c_i64, _c_u32, _c_p, _c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t


class FemMesh(ctypes.Structure):
    _fields_ = [("n_nodes", _c_i32), ("n_elems", _c_i32), ("X", _c_p), ("conn", _c_p)]


class FemParams(ctypes.Structure):
    _fields_ = [("p", _c_p * NPARAM), ("per_elem_mask", _c_u32), ("per_spec_mask", _c_u32), ("model", _c_u32),
                ("orient_per_elem", _c_u32), ("orient", _c_p), ("barlat", _c_p)]


class FemCsr(ctypes.Structure):
    _fields_ = [("n_rows", _c_i32), ("nnz", _c_i64), ("row_ptr", _c_p), ("col_idx", _c_p), ("elem_rank", _c_p),
                ("node_elem_ptr", _c_p), ("node_elem", _c_p)]


class FemBatch(ctypes.Structure):
    _fields_ = [("n_spec", _c_i32), ("elem_off", _c_p)]


class FemLaunch(ctypes.Structure):
    _fields_ = [("block", _c_i32), ("waves_per_cu", _c_i32), ("xcd_remap", _c_i32)]


class FemError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


_lib = None

EXPORTS = ("fem_version", "fem_last_error", "fem_set_launch", "fem_get_launch", "fem_csr_workspace_bytes",
           "fem_forward_workspace_bytes", "fem_vjp_workspace_bytes", "fem_csr_pattern", "fem_residual_tangent",
           "fem_residual_vjp", "fem_residual_vjp_noalloc", "fem_timing_enable", "fem_timing_read",
           "fem_graph_begin", "fem_graph_end", "fem_graph_launch", "fem_graph_destroy", "fem_solver_workspace_bytes",
           "fem_solver_workspace_bytes_method", "fem_csr_spmv", "fem_solve",
           "fem_csr_transpose", "fem_history_adjoint_workspace_bytes", "fem_history_adjoint", "fem_amg_create",
           "fem_amg_update", "fem_amg_apply", "fem_amg_info", "fem_amg_aggregates", "fem_amg_destroy",
           "fem_solve_amg", "fem_amg_plan_host", "fem_amg_set_cycle")


def lib():
    """Load libfem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2606_17390_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.fem_version.restype = ctypes.c_int
    L.fem_last_error.restype = ctypes.c_char_p
    L.fem_set_launch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(FemLaunch)]
    L.fem_get_launch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(FemLaunch)]
    L.fem_csr_workspace_bytes.argtypes = [_c_i32, _c_i32]
    L.fem_csr_workspace_bytes.restype = _c_sz
    L.fem_forward_workspace_bytes.argtypes = [_c_i32, _c_i32, ctypes.c_int]
    L.fem_forward_workspace_bytes.restype = _c_sz
    L.fem_vjp_workspace_bytes.argtypes = [_c_i32, _c_i32]
    L.fem_vjp_workspace_bytes.restype = _c_sz
    L.fem_csr_pattern.argtypes = [ctypes.POINTER(FemMesh), ctypes.POINTER(FemCsr), _c_p, _c_sz, _c_p]
    L.fem_residual_tangent.argtypes = [ctypes.POINTER(FemMesh), ctypes.POINTER(FemBatch), ctypes.POINTER(FemCsr),
                                       ctypes.POINTER(FemParams), _c_p, _c_p, _c_p, ctypes.c_int, _c_p, _c_p, _c_p,
                                       _c_p, _c_p, _c_p, _c_sz, _c_p]
    L.fem_residual_vjp.argtypes = [ctypes.POINTER(FemMesh), ctypes.POINTER(FemBatch), ctypes.POINTER(FemParams),
                                   _c_p, _c_p, _c_p, ctypes.c_int, _c_p, _c_p, _c_p, _c_p, _c_sz, _c_p]
    L.fem_residual_vjp_noalloc.argtypes = [ctypes.POINTER(FemMesh), ctypes.POINTER(FemBatch),
                                           ctypes.POINTER(FemParams), _c_p, _c_p, _c_p, ctypes.c_int, _c_p, _c_p,
                                           _c_p, _c_p]
    L.fem_timing_enable.argtypes = [ctypes.c_int]
    L.fem_timing_read.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_c_i32)]
    L.fem_graph_begin.argtypes = [_c_p]
    L.fem_graph_end.argtypes = [_c_p, ctypes.POINTER(_c_p)]
    L.fem_graph_launch.argtypes = [_c_p, _c_p]
    L.fem_graph_destroy.argtypes = [_c_p]
    L.fem_solver_workspace_bytes.argtypes = [_c_i32, ctypes.c_int64]
    L.fem_solver_workspace_bytes.restype = _c_sz
    L.fem_solver_workspace_bytes_method.argtypes = [_c_i32, ctypes.c_int64, ctypes.c_int]
    L.fem_solver_workspace_bytes_method.restype = _c_sz
    L.fem_csr_spmv.argtypes = [ctypes.POINTER(FemCsr), _c_p, ctypes.c_int, _c_p, _c_p, _c_p]
    L.fem_solve.argtypes = [ctypes.POINTER(FemCsr), _c_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_p, _c_p,
                            _c_i32, ctypes.c_double,
                            ctypes.POINTER(_c_i32), ctypes.POINTER(ctypes.c_double), _c_p, _c_sz, _c_p]
    L.fem_csr_transpose.argtypes = [ctypes.POINTER(FemCsr), _c_p, ctypes.c_int, _c_p, _c_p, _c_p]
    L.fem_amg_create.argtypes = [ctypes.POINTER(FemCsr), _c_p, ctypes.c_int, _c_p, ctypes.POINTER(_c_p), _c_p]
    L.fem_amg_update.argtypes = [_c_p, _c_p, ctypes.c_int, _c_p]
    L.fem_amg_apply.argtypes = [_c_p, _c_p, _c_p, _c_p]
    L.fem_amg_info.argtypes = [_c_p, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(_c_i32), ctypes.POINTER(ctypes.c_double)]
    L.fem_amg_aggregates.argtypes = [_c_p, _c_i32, _c_p]
    L.fem_amg_plan_host.argtypes = [_c_i32, _c_p, _c_p, _c_p, _c_p, ctypes.POINTER(_c_i32), _c_p, _c_p, _c_p]
    L.fem_amg_destroy.argtypes = [_c_p]
    L.fem_amg_set_cycle.argtypes = [_c_p, ctypes.c_int, _c_i32]
    L.fem_solve_amg.argtypes = [ctypes.POINTER(FemCsr), _c_p, ctypes.c_int, ctypes.c_int, _c_p, _c_p, _c_p,
                                _c_i32, ctypes.c_double,
                                ctypes.POINTER(_c_i32), ctypes.POINTER(ctypes.c_double), _c_p, _c_sz, _c_p]
    L.fem_history_adjoint_workspace_bytes.argtypes = [_c_i32, _c_i32]
    L.fem_history_adjoint_workspace_bytes.restype = _c_sz
    L.fem_history_adjoint.argtypes = [ctypes.POINTER(FemMesh), ctypes.POINTER(FemCsr), ctypes.POINTER(FemParams)] + \
        [_c_p] * 9 + [_c_p, _c_sz, _c_p]
    _lib = L
    return L


def _check(fn, code):
    if code != FEM_OK:
        raise FemError(fn, code, lib().fem_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _prec(p):
    if p in (FP64, "fp64", "f64", torch.float64):
        return FP64
    if p in (FP32_MIXED, "mixed", "fp32", "fp32_mixed", torch.float32):
        return FP32_MIXED
    if p in (FP64_K32, "fp64_k32"):
        return FP64_K32
    raise ValueError(f"unknown precision {p!r}")


def version():
    return lib().fem_version()


def set_launch(kernel, prec, block=None, waves_per_cu=None, xcd_remap=None):
    """Set the launch configuration of a kernel; with all None, reset it."""
    if block is None and waves_per_cu is None and xcd_remap is None:
        _check("fem_set_launch", lib().fem_set_launch(kernel, _prec(prec), None))
        return
    cur = get_launch(kernel, prec)
    cfg = FemLaunch(block if block is not None else cur.block,
                    waves_per_cu if waves_per_cu is not None else cur.waves_per_cu,
                    xcd_remap if xcd_remap is not None else cur.xcd_remap)
    _check("fem_set_launch", lib().fem_set_launch(kernel, _prec(prec), ctypes.byref(cfg)))


def timing_enable(on=True):
    _check("fem_timing_enable", lib().fem_timing_enable(1 if on else 0))


def timing_read(kernel):
    """(summed milliseconds, launch count) of the kernel since the last read."""
    ms = ctypes.c_double()
    n = _c_i32()
    _check("fem_timing_read", lib().fem_timing_read(kernel, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def get_launch(kernel, prec):
    cfg = FemLaunch()
    _check("fem_get_launch", lib().fem_get_launch(kernel, _prec(prec), ctypes.byref(cfg)))
    return cfg


# ---------------------------------------------------------------------------
# device-side containers
# ---------------------------------------------------------------------------

class Mesh:
    """Reference coordinates [n_nodes, 3] (float64) and connectivity [n_elems, 8]
    (int32, VTK order) resident on the device."""

    def __init__(self, X, conn, device="cuda"):
        self.X = torch.as_tensor(np.asarray(X, dtype=np.float64)).to(device).contiguous()
        self.conn = torch.as_tensor(np.asarray(conn, dtype=np.int32)).to(device).contiguous()
        self.n_nodes = int(self.X.shape[0])
        self.n_elems = int(self.conn.shape[0])
        self.device = self.X.device
        self._pattern = None

    def pattern(self):
        """The CSR pattern of this mesh (built on first use, then cached)."""
        if self._pattern is None:
            self._pattern = csr_pattern(self)
        return self._pattern

    def c(self):
        return FemMesh(self.n_nodes, self.n_elems, _ptr(self.X) if self.X.numel() else None,
                       _ptr(self.conn) if self.conn.numel() else None)


class Params:
    """The 11 material parameters: uniform (shape [11]), per element ([n_elems, 11])
    or per specimen ([n_spec, 11], batched mode); the model options: hardening
    "swift" or "voce" (slots 8-10 then hold sig0, Q, b), fbar (F-bar element),
    orient (None, one rotation [3, 3] / [9], or per element [n_elems, 3, 3] /
    [n_elems, 9]; columns = orthotropy axes), barlat (19 Yld2004-18p values:
    c'12 c'13 c'21 c'23 c'31 c'32 c'44 c'55 c'66, the same for c'', m; replaces
    the Hill-48 function)."""

    def __init__(self, prm, n_elems, device="cuda", per_spec=False, hardening="swift", fbar=False, orient=None,
                 barlat=None):
        if hardening not in ("swift", "voce"):
            raise ValueError(f"unknown hardening law {hardening!r}")
        self.model = (MODEL_VOCE if hardening == "voce" else 0) | (MODEL_FBAR if fbar else 0)
        self.barlat = None
        if barlat is not None:
            b = torch.as_tensor(np.asarray(barlat, dtype=np.float64)).reshape(-1)
            if b.numel() != 19:
                raise ValueError("barlat needs 19 values (18 coefficients and m)")
            self.barlat = b.to(device).contiguous()
            self.model |= MODEL_BARLAT
        self.orient = None
        self.orient_per_elem = 0
        if orient is not None:
            o = torch.as_tensor(np.asarray(orient, dtype=np.float64) if not torch.is_tensor(orient) else orient,
                                dtype=torch.float64)
            if o.numel() == 9:
                self.orient = o.reshape(9).to(device).contiguous()
            elif o.numel() == 9 * n_elems:
                self.orient = o.reshape(n_elems, 9).to(device).contiguous()
                self.orient_per_elem = 1
            else:
                raise ValueError("orient must hold one rotation or one per element")
        prm = torch.as_tensor(np.asarray(prm, dtype=np.float64) if not torch.is_tensor(prm) else prm,
                              dtype=torch.float64)
        self.cols = []
        self.per_elem_mask = 0
        self.per_spec_mask = 0
        if prm.dim() == 1:
            for k in range(NPARAM):
                self.cols.append(prm[k:k + 1].to(device).contiguous())
        else:
            if not per_spec and prm.shape[0] != n_elems:
                raise ValueError("per-element parameters need n_elems rows")
            for k in range(NPARAM):
                col = prm[:, k]
                if prm.shape[0] > 0 and bool((col == col[0]).all()):
                    # a constant column is passed as one uniform value
                    self.cols.append(col[:1].to(device).contiguous())
                    continue
                self.cols.append(col.to(device).contiguous())
                if per_spec:
                    self.per_spec_mask |= 1 << k
                else:
                    self.per_elem_mask |= 1 << k

    def c(self):
        p = FemParams()
        for k in range(NPARAM):
            p.p[k] = self.cols[k].data_ptr()
        p.per_elem_mask = self.per_elem_mask
        p.per_spec_mask = self.per_spec_mask
        p.model = self.model
        p.orient_per_elem = self.orient_per_elem
        p.orient = _ptr(self.orient) if self.orient is not None else None
        p.barlat = _ptr(self.barlat) if self.barlat is not None else None
        return p


class Batch:
    """Element offsets [n_spec + 1] of concatenated specimens."""

    def __init__(self, elem_off, device="cuda"):
        self.elem_off = torch.as_tensor(np.asarray(elem_off, dtype=np.int64)).to(device).contiguous()
        self.n_spec = int(self.elem_off.numel() - 1)

    def c(self):
        return FemBatch(self.n_spec, _ptr(self.elem_off))


class Csr:
    def __init__(self, row_ptr, col_idx, elem_rank, nnz, n_rows, node_elem_ptr, node_elem):
        self.row_ptr, self.col_idx, self.elem_rank = row_ptr, col_idx, elem_rank
        self.node_elem_ptr, self.node_elem = node_elem_ptr, node_elem
        self.nnz, self.n_rows = nnz, n_rows

    def c(self):
        return FemCsr(self.n_rows, self.nnz, _ptr(self.row_ptr), _ptr(self.col_idx) if self.nnz else None,
                      _ptr(self.elem_rank) if self.elem_rank is not None and self.elem_rank.numel() else None,
                      _ptr(self.node_elem_ptr), _ptr(self.node_elem) if self.node_elem.numel() else None)


def _ws(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def csr_pattern(mesh, stream=None, out=None):
    """Build the CSR pattern of the tangent (two calls of fem_csr_pattern).
    With `out` (a Csr of the same mesh) its buffers are filled again instead
    of allocating new ones."""
    L = lib()
    dev = mesh.device
    ws_bytes = L.fem_csr_workspace_bytes(mesh.n_nodes, mesh.n_elems)
    if out is not None and getattr(out, "_ws", None) is not None and out._ws.numel() >= ws_bytes:
        ws = out._ws
    else:
        ws = _ws(ws_bytes, dev)
    row_ptr = out.row_ptr if out is not None else torch.empty(3 * mesh.n_nodes + 1, dtype=torch.int32, device=dev)
    cm = mesh.c()
    c = FemCsr(3 * mesh.n_nodes, 0, _ptr(row_ptr), None, None)
    s = _stream(stream)
    _check("fem_csr_pattern", L.fem_csr_pattern(ctypes.byref(cm), ctypes.byref(c), _ptr(ws), ws_bytes, s))
    nnz = int(c.nnz)
    if out is not None and out.nnz == nnz and out.n_rows == 3 * mesh.n_nodes:
        col_idx, elem_rank, ne_ptr, ne_list = out.col_idx, out.elem_rank, out.node_elem_ptr, out.node_elem
    else:
        col_idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)[:nnz]
        elem_rank = torch.empty((max(mesh.n_elems, 1), 64), dtype=torch.uint8, device=dev)[:mesh.n_elems]
        ne_ptr = torch.zeros(mesh.n_nodes + 1, dtype=torch.int32, device=dev)
        ne_list = torch.empty(max(8 * mesh.n_elems, 1), dtype=torch.int32, device=dev)[:8 * mesh.n_elems]
    c.col_idx = col_idx.data_ptr()
    c.elem_rank = elem_rank.data_ptr()
    c.node_elem_ptr = ne_ptr.data_ptr()
    c.node_elem = ne_list.data_ptr()
    if nnz:
        _check("fem_csr_pattern", L.fem_csr_pattern(ctypes.byref(cm), ctypes.byref(c), _ptr(ws), ws_bytes, s))
    csr = Csr(row_ptr, col_idx, elem_rank, nnz, 3 * mesh.n_nodes, ne_ptr, ne_list)
    csr._ws = ws
    return csr


class Forward:
    """Preallocated outputs of fem_residual_tangent for repeated calls."""

    def __init__(self, mesh, csr, prec=FP64, want_K=True, want_hist=True, want_norm=True):
        dev = mesh.device
        self.prec = _prec(prec)
        self.R = torch.empty(3 * mesh.n_nodes, dtype=torch.float64, device=dev)
        kdt = torch.float64 if self.prec == FP64 else torch.float32
        nnz = csr.nnz if csr is not None else 0
        self.K = torch.empty(max(nnz, 1), dtype=kdt, device=dev)[:nnz] if (want_K and csr is not None) else None
        self.hist = torch.empty((7, 8 * mesh.n_elems), dtype=torch.float64, device=dev) if want_hist else None
        self.rnorm2 = torch.empty(1, dtype=torch.float64, device=dev) if want_norm else None
        self.diag = torch.empty(4, dtype=torch.int32, device=dev)
        nb = lib().fem_forward_workspace_bytes(mesh.n_nodes, mesh.n_elems, self.prec)
        self.ws = _ws(nb, dev)
        self.ws_bytes = nb


def residual_tangent(mesh, csr, params, d, hist_n, bc_mask=None, prec=FP64, out=None, batch=None,
                     want_K=True, want_hist=True, stream=None):
    """One residual + tangent + CSR assembly pass; returns the Forward buffers.
    With csr None the mesh's cached pattern is used (it carries the node
    incidence the assembly needs); K is then not requested."""
    L = lib()
    if csr is None:
        want_K = False
        if out is None or out.R is not None:
            csr = mesh.pattern()
    if out is None:
        out = Forward(mesh, csr, prec, want_K=want_K, want_hist=want_hist)
    cm, cp = mesh.c(), params.c()
    cc = csr.c() if csr is not None else None
    cb = batch.c() if batch is not None else None
    rc = L.fem_residual_tangent(ctypes.byref(cm), ctypes.byref(cb) if cb is not None else None,
                                ctypes.byref(cc) if cc is not None else None, ctypes.byref(cp), _ptr(d), _ptr(hist_n),
                                _ptr(bc_mask), out.prec, _ptr(out.R),
                                _ptr(out.K) if (want_K and out.K is not None and csr is not None and csr.nnz)
                                else None,
                                _ptr(out.hist), _ptr(out.rnorm2), _ptr(out.diag), _ptr(out.ws), out.ws_bytes,
                                _stream(stream))
    _check("fem_residual_tangent", rc)
    return out


class Vjp:
    def __init__(self, mesh, n_spec=1):
        dev = mesh.device
        self.g_uniform = torch.empty((n_spec, NGRAD), dtype=torch.float64, device=dev)
        self.g_elem = torch.empty((NGRAD, max(mesh.n_elems, 1)), dtype=torch.float64, device=dev)[:, :mesh.n_elems]
        self.diag = torch.empty(4, dtype=torch.int32, device=dev)
        nb = lib().fem_vjp_workspace_bytes(mesh.n_elems, n_spec)
        self.ws = _ws(nb, dev)
        self.ws_bytes = nb


def residual_vjp(mesh, params, d, hist_n, lam, prec=FP64, out=None, batch=None, want_elem=True, stream=None):
    """g = lam^T dR/dtheta for (F, G, H, N, K, eps0, n); returns the Vjp buffers."""
    L = lib()
    n_spec = batch.n_spec if batch is not None else 1
    if out is None:
        out = Vjp(mesh, n_spec)
    cm, cp = mesh.c(), params.c()
    cb = batch.c() if batch is not None else None
    ge = out.g_elem if (want_elem and mesh.n_elems) else None
    rc = L.fem_residual_vjp(ctypes.byref(cm), ctypes.byref(cb) if cb is not None else None, ctypes.byref(cp),
                            _ptr(d), _ptr(hist_n), _ptr(lam), _prec(prec), _ptr(out.g_uniform), _ptr(ge),
                            _ptr(out.diag), _ptr(out.ws), out.ws_bytes, _stream(stream))
    _check("fem_residual_vjp", rc)
    return out


VJP_SCRATCH_MAX_BYTES = 64 << 20  # FEM_VJP_SCRATCH_MAX_BYTES


def residual_vjp_noalloc(mesh, params, d, hist_n, lam, g_uniform, g_elem=None, diag=None, prec=FP64, batch=None,
                         stream=None):
    """fem_residual_vjp_noalloc: the VJP into caller-given outputs (g_uniform
    [n_spec, 7], g_elem [7, n_elems] or None, diag [4] int32 or None) with the
    library's static device scratch as workspace (nothing is allocated)."""
    cm, cp = mesh.c(), params.c()
    cb = batch.c() if batch is not None else None
    rc = lib().fem_residual_vjp_noalloc(ctypes.byref(cm), ctypes.byref(cb) if cb is not None else None,
                                        ctypes.byref(cp), _ptr(d), _ptr(hist_n), _ptr(lam), _prec(prec),
                                        _ptr(g_uniform), _ptr(g_elem) if g_elem is not None and mesh.n_elems
                                        else None, _ptr(diag), _stream(stream))
    _check("fem_residual_vjp_noalloc", rc)


# ---------------------------------------------------------------------------
# time-history adjoint
# ---------------------------------------------------------------------------

def csr_transpose(csr, K, bc_mask=None, out=None, stream=None):
    """K^T on the same pattern (float64 or float32 like K); rows of dofs marked in
    bc_mask become identity rows (the matrix of the adjoint solve)."""
    if out is None:
        out = torch.empty_like(K)
    _check("fem_csr_transpose", lib().fem_csr_transpose(ctypes.byref(csr.c()), _ptr(K), _kprec(K), _ptr(bc_mask),
                                                        _ptr(out), _stream(stream)))
    return out


class HistoryAdjoint:
    """Outputs and workspace of fem_history_adjoint for a mesh."""

    def __init__(self, mesh):
        dev = mesh.device
        ne, nn = mesh.n_elems, mesh.n_nodes
        self.g_uniform = torch.zeros(NGRAD, dtype=torch.float64, device=dev)
        self.g_elem = torch.zeros((NGRAD, ne), dtype=torch.float64, device=dev)
        self.hbar = torch.zeros((7, 8 * ne), dtype=torch.float64, device=dev)
        self.ubar = torch.zeros((nn, 3), dtype=torch.float64, device=dev)
        self.diag = torch.zeros(4, dtype=torch.int32, device=dev)
        self.ws_bytes = lib().fem_history_adjoint_workspace_bytes(nn, ne)
        self.ws = _ws(self.ws_bytes, dev)


def history_adjoint(mesh, csr, params, d, hist_n, lam=None, mu=None, out=None, want_hbar=True, want_ubar=True,
                    stream=None):
    """One load step of the time-history adjoint: g = lam^T dR/dtheta + mu^T dH/dtheta,
    hbar = lam^T dR/dh_n + mu^T dH/dh_n and ubar = mu^T dH/dd (FP64)."""
    if out is None:
        out = HistoryAdjoint(mesh)
    rc = lib().fem_history_adjoint(ctypes.byref(mesh.c()), ctypes.byref(csr.c()), ctypes.byref(params.c()), _ptr(d),
                                   _ptr(hist_n), _ptr(lam), _ptr(mu), _ptr(out.g_uniform),
                                   _ptr(out.g_elem) if mesh.n_elems else None,
                                   _ptr(out.hbar) if want_hbar and mesh.n_elems else None,
                                   _ptr(out.ubar) if want_ubar and mesh.n_nodes else None, _ptr(out.diag),
                                   _ptr(out.ws), out.ws_bytes, _stream(stream))
    _check("fem_history_adjoint", rc)
    return out


# ---------------------------------------------------------------------------
# HIP graphs
# ---------------------------------------------------------------------------

class Graph:
    """Capture the library calls made inside `with graph.capture(stream):` and
    replay them with graph.replay().  The stream must not be the null stream."""

    def __init__(self):
        self.exec = None

    def capture(self, stream):
        g = self

        class _Ctx:
            def __enter__(self_):
                _check("fem_graph_begin", lib().fem_graph_begin(_stream(stream)))
                return g

            def __exit__(self_, et, ev, tb):
                h = ctypes.c_void_p()
                rc = lib().fem_graph_end(_stream(stream), ctypes.byref(h))
                if et is None:
                    _check("fem_graph_end", rc)
                    g.exec = h
                return False
        return _Ctx()

    def replay(self, stream):
        _check("fem_graph_launch", lib().fem_graph_launch(self.exec, _stream(stream)))

    def __del__(self):
        if self.exec is not None and _lib is not None:
            _lib.fem_graph_destroy(self.exec)
            self.exec = None


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

class ResidualFn(torch.autograd.Function):
    """R(theta) with theta the 7 differentiated parameters (F, G, H, N, K, eps0, n),
    either uniform (shape [7]) or per element ([7, n_elems]).  Forward runs a
    residual-only pass of fem_residual_tangent; backward runs fem_residual_vjp
    with lam = grad_R.  Gradients with respect to d and the history are not
    provided (returned as None)."""

    GRAD_COLS = (2, 3, 4, 7, 8, 9, 10)

    @staticmethod
    def forward(ctx, theta, base_prm, mesh, d, hist_n, prec=FP64):
        prm = base_prm.clone().to(torch.float64)
        per_elem = theta.dim() == 2
        if per_elem:
            if prm.dim() == 1:
                prm = prm.unsqueeze(0).repeat(mesh.n_elems, 1)
            for i, c in enumerate(ResidualFn.GRAD_COLS):
                prm[:, c] = theta[i].detach().to(prm.device)
        else:
            for i, c in enumerate(ResidualFn.GRAD_COLS):
                if prm.dim() == 1:
                    prm[c] = theta[i].detach()
                else:
                    prm[:, c] = theta[i].detach()
        params = Params(prm, mesh.n_elems, device=mesh.device)
        out = residual_tangent(mesh, None, params, d, hist_n, prec=prec, want_K=False, want_hist=False)
        ctx.save_for_backward(d, hist_n)
        ctx.mesh, ctx.params, ctx.prec, ctx.per_elem = mesh, params, prec, per_elem
        ctx.uniform_prm = prm.dim() == 1
        ctx.theta_device = theta.device
        return out.R.clone()

    @staticmethod
    def backward(ctx, grad_R):
        d, hist_n = ctx.saved_tensors
        lam = grad_R.contiguous().to(torch.float64)
        v = residual_vjp(ctx.mesh, ctx.params, d, hist_n, lam, prec=ctx.prec, want_elem=ctx.per_elem)
        if ctx.per_elem:
            g = v.g_elem.clone()
        else:
            g = v.g_uniform[0].clone()
        return g.to(ctx.theta_device), None, None, None, None, None


# ---------------------------------------------------------------------------
# linear solve of the Newton iteration
# ---------------------------------------------------------------------------

def _kprec(K):
    return FP64 if K.dtype == torch.float64 else FP32_MIXED


def csr_spmv(csr, K, x, y=None, stream=None):
    """y = K x for the CSR values K (float64 or float32) of pattern csr."""
    if y is None:
        y = torch.empty(csr.n_rows, dtype=torch.float64, device=x.device)
    _check("fem_csr_spmv", lib().fem_csr_spmv(ctypes.byref(csr.c()), _ptr(K), _kprec(K), _ptr(x), _ptr(y),
                                              _stream(stream)))
    return y


PC_JACOBI, PC_BLOCK_JACOBI, PC_AMG = 0, 1, 2
KRYLOV = {"bicgstab": 0, "cg": 1, "gmres": 2, "fgmres": 3}
AMG_CYCLE = {"v": 0, "k": 1}


def default_krylov(precond, fbar):
    """The drivers' Krylov method: FGMRES (with the multigrid K-cycle) under
    the multigrid, else BiCGSTAB for the F-bar tangent and CG for the
    plain one (symmetric on the free dofs)."""
    if int(precond) == PC_AMG:
        return "fgmres"
    return "bicgstab" if fbar else "cg"
# levels of at least this many nodes take the K-cycle's two Krylov steps
AMG_K_MIN_NODES = 0
AMG_MAX_LEVELS = 12
AMG_DENSE_NODES = 32  # coarsest level inverted exactly at or below this many nodes


class AMG:
    """Aggregation multigrid hierarchy of fem_amg_create for pattern csr,
    aggregated from the block norms of K; bc_mask (device [n_rows] uint8 or
    bool, nonzero on constrained dofs) or None.  update(K) sets the numeric
    operators, apply(r) is one cycle (a V-cycle unless set_cycle("k"))."""

    def __init__(self, csr, K, bc_mask=None, stream=None):
        self.csr = csr
        self.h = _c_p()
        bc = None if bc_mask is None else bc_mask.reshape(-1).to(torch.uint8).contiguous()
        _check("fem_amg_create", lib().fem_amg_create(ctypes.byref(csr.c()), _ptr(K), _kprec(K), _ptr(bc),
                                                      ctypes.byref(self.h), _stream(stream)))

    def update(self, K, stream=None):
        self.K = K
        _check("fem_amg_update", lib().fem_amg_update(self.h, _ptr(K), _kprec(K), _stream(stream)))

    def set_cycle(self, cycle="v", k_min_nodes=None):
        """"v" or "k" (the K-cycle on levels of at least k_min_nodes nodes)"""
        kmin = AMG_K_MIN_NODES if k_min_nodes is None else int(k_min_nodes)
        _check("fem_amg_set_cycle", lib().fem_amg_set_cycle(self.h, AMG_CYCLE[cycle], kmin))
        self.cycle = cycle

    def apply(self, r, z=None, stream=None):
        if z is None:
            z = torch.empty_like(r)
        _check("fem_amg_apply", lib().fem_amg_apply(self.h, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def info(self, omega=False):
        """(levels as [(nodes, 3x3 blocks)], coarsest inverted exactly) and,
        with omega, the smoother damping per level"""
        nl, dense = _c_i32(0), _c_i32(0)
        nodes = (_c_i32 * AMG_MAX_LEVELS)()
        blocks = (ctypes.c_int64 * AMG_MAX_LEVELS)()
        om = (ctypes.c_double * AMG_MAX_LEVELS)()
        _check("fem_amg_info", lib().fem_amg_info(self.h, ctypes.byref(nl), nodes, blocks, ctypes.byref(dense),
                                                  om if omega else None))
        levels = [(int(nodes[i]), int(blocks[i])) for i in range(nl.value)]
        if omega:
            return levels, bool(dense.value), [float(om[i]) for i in range(nl.value)]
        return levels, bool(dense.value)

    def aggregates(self, level):
        """numpy int32 [nodes of level - 1]: aggregate of each node of the level above"""
        levels, _ = self.info()
        out = np.empty(levels[level - 1][0], dtype=np.int32)
        _check("fem_amg_aggregates", lib().fem_amg_aggregates(self.h, int(level),
                                                              out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def close(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            lib().fem_amg_destroy(self.h)
            self.h = _c_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def amg_plan_host(bptr, ncol, strength, bc_mask=None):
    """fem_amg_plan_host on numpy arrays: returns ([(nodes, blocks)] per
    level, [aggregate map of level l for l = 1 .. levels - 1])."""
    bptr = np.ascontiguousarray(bptr, dtype=np.int64)
    ncol = np.ascontiguousarray(ncol, dtype=np.int32)
    strength = np.ascontiguousarray(strength, dtype=np.float32)
    n = bptr.size - 1
    bc = None if bc_mask is None else np.ascontiguousarray(bc_mask, dtype=np.uint8)
    nl = _c_i32(0)
    nodes = np.zeros(AMG_MAX_LEVELS, dtype=np.int32)
    blocks = np.zeros(AMG_MAX_LEVELS, dtype=np.int64)
    agg = np.zeros(7 * n, dtype=np.int32)  # every level keeps at most 85 % of the one above

    def p(a):
        return None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    _check("fem_amg_plan_host", lib().fem_amg_plan_host(n, p(bptr), p(ncol), p(strength), p(bc), ctypes.byref(nl),
                                                        p(nodes), p(blocks), p(agg)))
    levels = [(int(nodes[i]), int(blocks[i])) for i in range(nl.value)]
    maps, off = [], 0
    for l in range(1, nl.value):
        maps.append(agg[off:off + levels[l - 1][0]].copy())
        off += levels[l - 1][0]
    return levels, maps


class Solver:
    """Workspace of fem_solve for a pattern (reused across solves).  With
    precond=PC_AMG the multigrid hierarchy is built at the first solve from
    that K (bc_mask: the constrained dofs, as for fem_residual_tangent) and
    its numeric operators are rebuilt for each K."""

    def __init__(self, csr, device="cuda", precond=PC_BLOCK_JACOBI, method="bicgstab", bc_mask=None, cycle=None,
                 k_min_nodes=None):
        self.csr = csr
        self.precond = int(precond)
        self.method = KRYLOV[method]
        # multigrid cycle: the K-cycle with the flexible method, else the V-cycle
        self.cycle = cycle if cycle is not None else ("k" if method == "fgmres" else "v")
        self.k_min_nodes = k_min_nodes
        self.device = device
        self.ws_bytes = lib().fem_solver_workspace_bytes_method(csr.n_rows, csr.nnz, self.method)
        self.ws = _ws(self.ws_bytes, device)
        self.bc_mask = bc_mask
        self.amg = None

    def solve(self, K, b, x=None, rtol=1e-10, max_iter=10000, stream=None, check=True, precond=None, method=None):
        """Solve K x = b (method "bicgstab", "gmres", "fgmres", or "cg" for
        a tangent symmetric on the free dofs; preconditioner PC_BLOCK_JACOBI,
        the 3x3 node blocks, unless given; with PC_AMG the K-cycle under
        "fgmres" unless the solver was made with cycle="v", else the
        V-cycle); returns (x, iterations, relative residual)."""
        if x is None:
            x = torch.zeros(self.csr.n_rows, dtype=torch.float64, device=b.device)
        it = _c_i32(0)
        res = ctypes.c_double(0.0)
        pc = self.precond if precond is None else int(precond)
        mt = self.method if method is None else KRYLOV[method]
        need = lib().fem_solver_workspace_bytes_method(self.csr.n_rows, self.csr.nnz, mt)
        if need > self.ws_bytes:  # GMRES asked of a solver made for another method
            self.ws_bytes = need
            self.ws = _ws(need, b.device)
        if pc == PC_AMG:
            if self.amg is None:
                self.amg = AMG(self.csr, K, self.bc_mask, stream)
            cyc = self.cycle if mt == KRYLOV["fgmres"] else "v"
            if getattr(self.amg, "cycle", "v") != cyc or cyc == "k":
                self.amg.set_cycle(cyc, self.k_min_nodes)
            fn = "fem_solve_amg"
            rc = lib().fem_solve_amg(ctypes.byref(self.csr.c()), _ptr(K), _kprec(K), mt, self.amg.h, _ptr(b), _ptr(x),
                                     int(max_iter), float(rtol), ctypes.byref(it), ctypes.byref(res), _ptr(self.ws),
                                     self.ws_bytes, _stream(stream))
        else:
            fn = "fem_solve"
            rc = lib().fem_solve(ctypes.byref(self.csr.c()), _ptr(K), _kprec(K), mt, pc, _ptr(b), _ptr(x),
                                 int(max_iter), float(rtol), ctypes.byref(it), ctypes.byref(res), _ptr(self.ws),
                                 self.ws_bytes, _stream(stream))
        if check:
            _check(fn, rc)
        return x, int(it.value), float(res.value)
