"""Pins of the oracle parameter VJP lambda^T dR/dtheta (CPU only): central
finite differences of lambda^T R(theta) (the paper's verification protocol,
Alg. 2, with h = 1e-6 |theta_k|), per-element FD, the directional check
E_FD with D_i = 0.1 over a step sweep, and the all-elastic case."""
import numpy as np
import pytest

import oracle
from paper_2606_17390_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore")
GP = synth.GRAD_PARAM_INDEX


def lamR(p, prm, rp, ci):
    R, _, _, _, _ = oracle.residual_tangent(p.X, p.conn, rp, ci, prm, p.d, p.hist_n, want_K=False)
    return float(np.dot(p.lam.ravel(), R))


@pytest.fixture(scope="module")
def slab():
    p = synth.small_slab(31, 4, 3, 2, strain=0.01)
    rp, ci, _ = oracle.csr_pattern(p.conn, p.n_nodes, with_rank=False)
    return p, rp, ci


def test_uniform_vjp_matches_central_fd(slab):
    p, rp, ci = slab
    gu, ge, diag = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam)
    assert np.allclose(gu, ge.sum(axis=1), rtol=1e-14, atol=0)
    for k, col in enumerate(GP):
        h = 1e-6 * abs(p.prm[col])
        pp, pm = p.prm.copy(), p.prm.copy()
        pp[col] += h
        pm[col] -= h
        fd = (lamR(p, pp, rp, ci) - lamR(p, pm, rp, ci)) / (2 * h)
        assert abs(gu[k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gu).max()), (k, gu[k], fd)


def test_per_element_vjp_matches_fd(slab):
    p, rp, ci = slab
    prm_e = np.tile(p.prm, (p.n_elems, 1))
    gu, ge, _ = oracle.residual_vjp(p.X, p.conn, prm_e, p.d, p.hist_n, p.lam)
    rng = np.random.default_rng(0)
    for e in rng.choice(p.n_elems, 5, replace=False):
        for k, col in enumerate(GP):
            h = 1e-6 * abs(prm_e[e, col])
            pp, pm = prm_e.copy(), prm_e.copy()
            pp[e, col] += h
            pm[e, col] -= h
            fd = (lamR(p, pp, rp, ci) - lamR(p, pm, rp, ci)) / (2 * h)
            assert abs(ge[k, e] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(ge[:, e]).max() + 1e-300)


def test_directional_fd_check_has_v_shape(slab):
    """E_FD(h) = |g . D - (J(theta + hD) - J(theta - hD)) / 2h| with D_i = 0.1 on
    normalised parameters: truncation dominates at large h, rounding at small
    h, with a minimum in between."""
    p, rp, ci = slab
    gu, _, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam)
    scale = np.array([abs(p.prm[c]) for c in GP])
    D = 0.1 * np.ones(7)
    gD = np.dot(gu * scale, D)
    errs = []
    hs = 10.0 ** -np.arange(1, 12)
    for h in hs:
        pp, pm = p.prm.copy(), p.prm.copy()
        for k, c in enumerate(GP):
            pp[c] += h * D[k] * scale[k]
            pm[c] -= h * D[k] * scale[k]
        errs.append(abs(gD - (lamR(p, pp, rp, ci) - lamR(p, pm, rp, ci)) / (2 * h)))
    errs = np.array(errs)
    i = int(np.argmin(errs))
    assert 2 <= i <= 8
    assert errs[0] > 10 * errs[i] and errs[-1] > 10 * errs[i]
    assert errs[i] <= 1e-6 * abs(gD)


def test_all_elastic_gives_zero():
    p = synth.small_slab(32, 3, 2, 2, strain=1e-6, alpha_max=0.0)
    p.hist_n[:] = 0.0
    gu, ge, _ = oracle.residual_vjp(p.X, p.conn, p.prm, p.d, p.hist_n, p.lam)
    assert np.all(gu == 0.0) and np.all(ge == 0.0)
