"""FP64 CPU oracle for the finite-strain Hill-48 hex8 path (ctypes binding).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` import this module.  The product
library never calls it, and it imports nothing from the product package.

The C source (``oracle.c``) follows the paper step by step; see its header for
the passages.  This module only marshals numpy arrays.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_ASAN_PATH = os.path.join(_HERE, "liboracle_asan.so")
# ORACLE_LIB names another build of oracle.c to load (the sanitizer build)
_lib = None

NPARAM = 11
NGRAD = 7
# model option flags (oracle.h)
MODEL_VOCE = 1
MODEL_FBAR = 2
MODEL_BARLAT = 4


def build(force=True, sanitize=False):
    """Compile liboracle.so with gcc (OpenMP, -O2).  sanitize=True builds
    liboracle_asan.so instead, with AddressSanitizer and UndefinedBehavior
    checks (host code; the test suite loads it in a child process with the
    ASan runtime preloaded)."""
    path = _ASAN_PATH if sanitize else _LIB_PATH
    if not force and os.path.exists(path):
        return path
    src = os.path.join(_HERE, "oracle.c")
    tmp = path + ".tmp"
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    cmd = ["gcc", *flags, "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", src, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, path)
    return path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ORACLE_LIB", _LIB_PATH)
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.oracle_eig_sym3.argtypes = [P, P, P]
    lib.oracle_log_strain.argtypes = [P, P]
    ci = ctypes.c_int
    lib.oracle_material_point.argtypes = [P] * 3 + [ci, P] + [P] * 9
    lib.oracle_material_point.restype = ctypes.c_int
    lib.oracle_element.argtypes = [P] * 4 + [ci, P] + [P] * 4
    lib.oracle_csr_pattern.argtypes = [i32, i32, P, P, P, P, P]
    lib.oracle_csr_pattern.restype = ctypes.c_int
    lib.oracle_residual_tangent.argtypes = [i32, i32] + [P] * 5 + [ci, P] + [P] * 8 + [ci]
    lib.oracle_residual_tangent.restype = ctypes.c_int
    lib.oracle_trial_yield.argtypes = [i32, i32] + [P] * 3 + [ci, P] + [P] * 3 + [ci]
    lib.oracle_residual_vjp.argtypes = [i32, i32] + [P] * 3 + [ci, P] + [P] * 6 + [ci]
    lib.oracle_residual_vjp.restype = ctypes.c_int
    lib.oracle_local_jacobian.argtypes = [P] * 3 + [ci, P, P]
    lib.oracle_local_jacobian.restype = ctypes.c_int
    lib.oracle_element_adjoint.argtypes = [P] * 4 + [ci] + [P] * 6
    lib.oracle_set_barlat.argtypes = [P]
    lib.oracle_effective_stress.argtypes = [P, P, ci, P, P]
    lib.oracle_effective_stress.restype = ctypes.c_double
    lib.oracle_local_return.argtypes = [P] * 3 + [ci, P, ci, ci, ci, P, P, ci, P]
    lib.oracle_local_return.restype = ctypes.c_int
    lib.oracle_local_merit.argtypes = [P] * 3 + [ci, P, ci, P]
    lib.oracle_local_merit.restype = ctypes.c_double
    lib.oracle_local_return_batch.argtypes = [i32] + [P] * 3 + [ci, P, ci, ci, ci, P, ci]
    _lib = lib
    del i64
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def eig_sym3(A):
    A = _f64(A).reshape(3, 3)
    w = np.zeros(3)
    Q = np.zeros((3, 3))
    _load().oracle_eig_sym3(_p(A), _p(w), _p(Q))
    return w, Q


def log_strain(F):
    F = _f64(F).reshape(3, 3)
    eps = np.zeros((3, 3))
    _load().oracle_log_strain(_p(F), _p(eps))
    return eps


def _theta(Theta):
    return None if Theta is None else _f64(Theta).reshape(9)


def expand_orient(orient, n_elems):
    """None, one rotation (3x3) or per-element rotations [n_elems, 3, 3] -> [n_elems, 9]."""
    if orient is None:
        return None
    o = _f64(orient)
    if o.size == 9:
        return np.ascontiguousarray(np.broadcast_to(o.reshape(9), (n_elems, 9)))
    return _f64(o.reshape(n_elems, 9))


def material_point(F, hist_n, prm, model=0, Theta=None):
    """Return a dict with S, P, T (3x3), hist (7), A (3,3,3,3), Cep, Cep_implicit,
    Cmat (6x6 Mandel), plastic, iters, converged, dgamma, ftr, sy_n.  model:
    MODEL_* flags (Voce hardening); Theta: orientation (3x3 rotation) or None."""
    F = _f64(F).reshape(3, 3)
    h = _f64(hist_n).reshape(7)
    p = _f64(prm).reshape(NPARAM)
    th = _theta(Theta)
    S, P, T = np.zeros((3, 3)), np.zeros((3, 3)), np.zeros((3, 3))
    hn = np.zeros(7)
    A = np.zeros(81)
    Cep, CepI, Cm = np.zeros((6, 6)), np.zeros((6, 6)), np.zeros((6, 6))
    info = np.zeros(6)
    rc = _load().oracle_material_point(_p(F), _p(h), _p(p), int(model), _p(th), _p(S), _p(P), _p(T),
                                       _p(hn), _p(A), _p(Cep), _p(CepI), _p(Cm), _p(info))
    return dict(S=S, P=P, T=T, hist=hn, A=A.reshape(3, 3, 3, 3), Cep=Cep, Cep_implicit=CepI,
                Cmat=Cm, plastic=bool(info[0]), iters=int(info[1]), converged=bool(info[2]),
                dgamma=info[3], ftr=info[4], sy_n=info[5], rc=rc)


def element(Xe, de, he, prm, want_K=True, model=0, Theta=None):
    """Element residual (24), tangent (24x24), updated history (8x7), diag (4);
    model: MODEL_* flags (Voce, F-bar); Theta: orientation or None."""
    Xe = _f64(Xe).reshape(8, 3)
    de = _f64(de).reshape(8, 3)
    he = _f64(he).reshape(8, 7)
    p = _f64(prm).reshape(NPARAM)
    th = _theta(Theta)
    R = np.zeros(24)
    K = np.zeros((24, 24)) if want_K else None
    hn = np.zeros((8, 7))
    diag = np.zeros(4, dtype=np.int32)
    _load().oracle_element(_p(Xe), _p(de), _p(he), _p(p), int(model), _p(th), _p(R), _p(K), _p(hn),
                           _p(diag))
    return R, K, hn, diag


def csr_pattern(conn, n_nodes, with_rank=True):
    """Return (row_ptr, col_idx, elem_rank [n_elems, 64]) or raise on a bad mesh."""
    conn = _i32(conn).reshape(-1, 8)
    ne = conn.shape[0]
    row_ptr = np.zeros(3 * n_nodes + 1, dtype=np.int32)
    nnz = np.zeros(1, dtype=np.int64)
    lib = _load()
    rc = lib.oracle_csr_pattern(n_nodes, ne, _p(conn), _p(nnz), _p(row_ptr), None, None)
    if rc != 0:
        raise ValueError(f"oracle_csr_pattern: invalid mesh (status {rc})")
    col_idx = np.zeros(int(nnz[0]), dtype=np.int32)
    rank = np.zeros((ne, 64), dtype=np.uint8) if with_rank else None
    rc = lib.oracle_csr_pattern(n_nodes, ne, _p(conn), _p(nnz), _p(row_ptr), _p(col_idx), _p(rank))
    if rc != 0:
        raise ValueError(f"oracle_csr_pattern: invalid mesh (status {rc})")
    return row_ptr, col_idx, rank


def expand_params(prm, n_elems):
    """Uniform [11] or per-element [n_elems, 11] parameters -> [n_elems, 11]."""
    prm = _f64(prm)
    if prm.ndim == 1:
        return np.ascontiguousarray(np.broadcast_to(prm, (n_elems, NPARAM)))
    return _f64(prm.reshape(n_elems, NPARAM))


def residual_tangent(X, conn, row_ptr, col_idx, prm, d, hist_n, bc_mask=None, want_K=True,
                     n_threads=0, model=0, orient=None):
    """Assembled residual R [3n], CSR values K [nnz] (or None), hist_np1 [7, 8ne],
    rnorm2 (double, long double), diag [4]."""
    X = _f64(X).reshape(-1, 3)
    conn = _i32(conn).reshape(-1, 8)
    nn, ne = X.shape[0], conn.shape[0]
    prm = expand_params(prm, ne)
    ori = expand_orient(orient, ne)
    d = _f64(d).reshape(nn, 3)
    hist_n = _f64(hist_n).reshape(7, 8 * ne)
    bc = None if bc_mask is None else np.ascontiguousarray(bc_mask, dtype=np.uint8)
    R = np.zeros(3 * nn)
    K = np.zeros(len(col_idx)) if want_K else None
    hn = np.zeros((7, 8 * ne))
    rn = np.zeros(2)
    diag = np.zeros(4, dtype=np.int32)
    rp = _i32(row_ptr)
    ci = _i32(col_idx)
    rc = _load().oracle_residual_tangent(nn, ne, _p(X), _p(conn), _p(rp), _p(ci), _p(prm), int(model),
                                         _p(ori), _p(d), _p(hist_n), _p(bc), _p(R), _p(K), _p(hn), _p(rn),
                                         _p(diag), int(n_threads))
    if rc != 0:
        raise RuntimeError("oracle_residual_tangent: element entry missing from the CSR pattern")
    return R, K, hn, rn, diag


def trial_yield(X, conn, prm, d, hist_n, n_threads=0, model=0, orient=None):
    X = _f64(X).reshape(-1, 3)
    conn = _i32(conn).reshape(-1, 8)
    nn, ne = X.shape[0], conn.shape[0]
    prm = expand_params(prm, ne)
    ori = expand_orient(orient, ne)
    d = _f64(d).reshape(nn, 3)
    hist_n = _f64(hist_n).reshape(7, 8 * ne)
    flag = np.zeros(8 * ne, dtype=np.uint8)
    _load().oracle_trial_yield(nn, ne, _p(X), _p(conn), _p(prm), int(model), _p(ori), _p(d), _p(hist_n),
                               _p(flag), int(n_threads))
    return flag


def residual_vjp(X, conn, prm, d, hist_n, lam, n_threads=0, model=0, orient=None):
    """Return (g_uniform [7], g_elem [7, n_elems], diag [4])."""
    X = _f64(X).reshape(-1, 3)
    conn = _i32(conn).reshape(-1, 8)
    nn, ne = X.shape[0], conn.shape[0]
    prm = expand_params(prm, ne)
    ori = expand_orient(orient, ne)
    d = _f64(d).reshape(nn, 3)
    hist_n = _f64(hist_n).reshape(7, 8 * ne)
    lam = _f64(lam).reshape(nn, 3)
    gu = np.zeros(7)
    ge = np.zeros((7, ne))
    diag = np.zeros(4, dtype=np.int32)
    _load().oracle_residual_vjp(nn, ne, _p(X), _p(conn), _p(prm), int(model), _p(ori), _p(d), _p(hist_n),
                                _p(lam), _p(gu), _p(ge), _p(diag), int(n_threads))
    return gu, ge, diag


def local_jacobian(F, hist_n, prm, model=0, Theta=None):
    """dz/dp [13, 20] of the local update: z = (T Mandel 6, hist_{n+1} 7),
    p = (eps Mandel 6, hist_n 7, theta 7)."""
    F = _f64(F).reshape(3, 3)
    h = _f64(hist_n).reshape(7)
    p = _f64(prm).reshape(NPARAM)
    th = _theta(Theta)
    Jz = np.zeros((13, 20))
    rc = _load().oracle_local_jacobian(_p(F), _p(h), _p(p), int(model), _p(th), _p(Jz))
    return Jz, rc


def element_adjoint(Xe, de, he, prm, lam=None, mu=None, model=0, Theta=None):
    """(theta_bar [7], hbar [8, 7], ubar [24]) of one element for the cotangents
    lam [8, 3] of R^e and mu [8, 7] of hist_{n+1} (either may be None)."""
    Xe = _f64(Xe).reshape(8, 3)
    de = _f64(de).reshape(8, 3)
    he = _f64(he).reshape(8, 7)
    p = _f64(prm).reshape(NPARAM)
    lm = None if lam is None else _f64(lam).reshape(24)
    mm = None if mu is None else _f64(mu).reshape(56)
    tb, hb, ub = np.zeros(7), np.zeros((8, 7)), np.zeros(24)
    _load().oracle_element_adjoint(_p(Xe), _p(de), _p(he), _p(p), int(model), _p(_theta(Theta)), _p(lm), _p(mm),
                                   _p(tb), _p(hb), _p(ub))
    return tb, hb, ub


def set_barlat(coef):
    """Barlat Yld2004-18p coefficients (c'12 c'13 c'21 c'23 c'31 c'32 c'44 c'55
    c'66, c''..., m) used by every call with MODEL_BARLAT."""
    c = _f64(coef).reshape(19)
    _load().oracle_set_barlat(_p(c))


def effective_stress(T, prm, model=0, Theta=None):
    """(phi, N [3, 3]) of the model's yield function at the stress T [3, 3]."""
    T = _f64(T).reshape(3, 3)
    p = _f64(prm).reshape(NPARAM)
    N = np.zeros((3, 3))
    phi = _load().oracle_effective_stress(_p(T), _p(p), int(model), _p(_theta(Theta)), _p(N))
    return phi, N


# layout of a line-search trace record (oracle.h, oracle_local_return)
TRACE_JMAX2 = 22
TRACE_REC = 22 + 2 * TRACE_JMAX2


def local_return(eps_m, hist_n, prm, model=0, Theta=None, line_search=True, kmax=100, merit_scaled=False,
                 trace_cap=200):
    """Local return map (Alg. C2, App. B line search) from the Mandel log strain
    eps_m [6] and stored history hist_n [7].  Returns (iterations (negative if
    not converged), y [8] = [T Mandel, alpha, dgamma], trace): trace is a list
    of dicts per Newton step with k, gnorm, psi0, psi1, zeta, y, dy and the
    line-search candidates zetas / psis (zetas[0] from Eq. (alpha_init))."""
    e = _f64(eps_m).reshape(6)
    h = _f64(hist_n).reshape(7)
    p = _f64(prm).reshape(NPARAM)
    y = np.zeros(8)
    tr = np.zeros((trace_cap, TRACE_REC))
    nrec = ctypes.c_int(0)
    it = _load().oracle_local_return(_p(e), _p(h), _p(p), int(model), _p(_theta(Theta)), int(bool(line_search)),
                                     int(kmax), int(bool(merit_scaled)), _p(y), _p(tr), int(trace_cap),
                                     ctypes.byref(nrec))
    recs = []
    for r in tr[:nrec.value]:
        m = int(r[5])
        recs.append(dict(k=int(r[0]), gnorm=r[1], psi0=r[2], psi1=r[3], zeta=r[4], y=r[6:14].copy(),
                         dy=r[14:22].copy(), zetas=r[22:22 + m].copy(),
                         psis=r[22 + TRACE_JMAX2:22 + TRACE_JMAX2 + m].copy()))
    return it, y, recs


def local_merit(eps_m, hist_n, prm, y, model=0, Theta=None, merit_scaled=False):
    """The merit psi(y) of the local system at y [8]."""
    e = _f64(eps_m).reshape(6)
    h = _f64(hist_n).reshape(7)
    p = _f64(prm).reshape(NPARAM)
    yy = _f64(y).reshape(8)
    return _load().oracle_local_merit(_p(e), _p(h), _p(p), int(model), _p(_theta(Theta)), int(bool(merit_scaled)),
                                      _p(yy))


def local_return_batch(eps_m, hist_n, prm, model=0, Theta=None, line_search=True, kmax=100, merit_scaled=False,
                       n_threads=0):
    """Iteration counts (negative: not converged) of local_return for many
    strains eps_m [n, 6] sharing hist_n."""
    e = _f64(eps_m).reshape(-1, 6)
    h = _f64(hist_n).reshape(7)
    p = _f64(prm).reshape(NPARAM)
    it = np.zeros(e.shape[0], dtype=np.int32)
    _load().oracle_local_return_batch(e.shape[0], _p(e), _p(h), _p(p), int(model), _p(_theta(Theta)),
                                      int(bool(line_search)), int(kmax), int(bool(merit_scaled)), _p(it),
                                      int(n_threads))
    return it
