"""Seeded synthetic inputs: hex8 meshes, material fields, displacement fields,
history and cotangents.

This module holds no arithmetic of the method (no kinematics, no constitutive
update, no assembly); it only draws inputs.  Both the HIP path (tests, bench)
and the CPU oracle (tests) read their inputs from here.  Everything is drawn
with numpy's PCG64 from an explicit seed; units are mm and MPa.

Workloads (they stand in for the paper's meshes; no dataset is involved):
  tiny_cube      4x4x4 unit cube, von Mises Hill parameters, uniaxial x-tension
  sheet_slab     40x40x4 jittered slab, one random Hill set, z=0 face clamped
  large_cube     100x100x100 cube, per-element Hill fields, 30% of Gauss
                 points yielding at the trial state
  void_specimen  200x200x2 slab with 25% voids, per-element fields for all
                 seven differentiated parameters, random unit cotangent
  batch64        64 uneven slabs, each with its own parameters
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PARAM_NAMES = ("E", "nu", "F", "G", "H", "L", "M", "N", "K", "eps0", "n")
GRAD_NAMES = ("F", "G", "H", "N", "K", "eps0", "n")
GRAD_PARAM_INDEX = (2, 3, 4, 7, 8, 9, 10)  # position of each GRAD_NAMES entry in PARAM_NAMES

E_DEFAULT, NU_DEFAULT = 200000.0, 0.3
SWIFT_DEFAULT = (500.0, 0.01, 0.2)  # K [MPa], eps0, n
# Voce law sigma_y = sig0 + Q (1 - exp(-b alpha)); its three parameters take
# the slots of (K, eps0, n) in a parameter row
VOCE_DEFAULT = (200.0, 150.0, 20.0)  # sig0 [MPa], Q [MPa], b
# Trial-state amplitude of the large_cube displacement field: the value for
# which 30% of the Gauss points have f_tr > 0 (tests/golden/calibrate_large_cube.py).
LARGE_CUBE_AMPLITUDE = 0.0041015625

# VTK hex corner order in (i, j, k) offsets
_HEX_OFF = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                     [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)


@dataclass
class Problem:
    name: str
    X: np.ndarray          # [n_nodes, 3]
    conn: np.ndarray       # [n_elems, 8] int32, VTK order
    d: np.ndarray          # [n_nodes, 3] displacement
    hist_n: np.ndarray     # [7, 8*n_elems]
    prm: np.ndarray        # [11] uniform or [n_elems, 11] per element
    bc_mask: Optional[np.ndarray] = None  # [3*n_nodes] uint8
    lam: Optional[np.ndarray] = None      # [n_nodes, 3] cotangent
    meta: dict = field(default_factory=dict)
    hardening: str = "swift"              # "swift" or "voce" (slots 8-10: K, eps0, n or sig0, Q, b)
    fbar: bool = False                    # F-bar element formulation
    orient: Optional[np.ndarray] = None   # None, [9] or [n_elems, 9] rotations (row-major)
    barlat: Optional[np.ndarray] = None   # Yld2004-18p coefficients [19] (replaces Hill-48), or None

    @property
    def n_nodes(self):
        return self.X.shape[0]

    @property
    def n_elems(self):
        return self.conn.shape[0]

    @property
    def per_element(self):
        return self.prm.ndim == 2


def params(F=0.5, G=0.5, H=0.5, L=1.5, M=1.5, N=1.5, K=SWIFT_DEFAULT[0], eps0=SWIFT_DEFAULT[1],
           n=SWIFT_DEFAULT[2], E=E_DEFAULT, nu=NU_DEFAULT):
    return np.array([E, nu, F, G, H, L, M, N, K, eps0, n], dtype=np.float64)


def voce_params(F=0.5, G=0.5, H=0.5, L=1.5, M=1.5, N=1.5, sig0=VOCE_DEFAULT[0], Q=VOCE_DEFAULT[1],
                b=VOCE_DEFAULT[2], E=E_DEFAULT, nu=NU_DEFAULT):
    return np.array([E, nu, F, G, H, L, M, N, sig0, Q, b], dtype=np.float64)


def random_rotation(rng):
    """A rotation drawn from the QR factors of a Gaussian matrix (det +1)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def rotation_z(angle):
    """Rotation by `angle` (radians) about the z axis; its columns are the rotated x, y, z axes."""
    c, s = np.cos(angle), np.sin(angle)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


# Yld2004-18p coefficients c'12 c'13 c'21 c'23 c'31 c'32 c'44 c'55 c'66, the
# same for c'', and m: the AA6111-T4 set of the paper's Barlat verification
# table (tests/golden/barlat_yld2004_aa6111.json holds the same values)
BARLAT_AA6111 = np.array([-0.069888, 0.936408, 0.079143, 1.003060, 0.524741, 1.363180, 1.023770, 1.069060, 0.954322,
                          0.981171, 0.476741, 0.575316, 0.866827, 1.145010, -0.079294, 1.051660, 1.147100, 1.404620,
                          8.0])


def with_model(p, seed, hardening="swift", fbar=False, orient=None, barlat=None):
    """Problem p with another hardening law, the F-bar element, an orientation
    and/or the Barlat yield function (barlat: 19 coefficients, e.g.
    BARLAT_AA6111): "voce" replaces slots 8-10 of the parameters by Voce values
    (per element draws if p is per element); orient is None, "uniform" (one
    random rotation) or "per_element" (one random in-plane angle per element)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    prm = p.prm.copy()
    if hardening == "voce":
        if prm.ndim == 2:
            ne = prm.shape[0]
            prm[:, 8] = rng.uniform(180.0, 220.0, ne)
            prm[:, 9] = rng.uniform(100.0, 200.0, ne)
            prm[:, 10] = rng.uniform(10.0, 30.0, ne)
        else:
            prm[8:11] = VOCE_DEFAULT
    ori = None
    if isinstance(orient, str):
        if orient == "uniform":
            ori = random_rotation(rng).ravel()
        elif orient == "per_element":
            ang = rng.uniform(0.0, np.pi, p.n_elems)
            c, s_ = np.cos(ang), np.sin(ang)
            ori = np.zeros((p.n_elems, 9))
            ori[:, 0], ori[:, 1], ori[:, 3], ori[:, 4], ori[:, 8] = c, -s_, s_, c, 1.0  # rotation_z(ang)
        else:
            raise ValueError(f"unknown orientation {orient!r}")
    elif orient is not None:
        ori = np.asarray(orient, dtype=np.float64)
    import dataclasses
    return dataclasses.replace(p, prm=prm, hardening=hardening, fbar=fbar, orient=ori,
                               barlat=None if barlat is None else np.asarray(barlat, dtype=np.float64),
                               name=f"{p.name}_{hardening}{'_fbar' if fbar else ''}{'_' + orient if isinstance(orient, str) else ''}")


def hex_grid(nx, ny, nz, lx=None, ly=None, lz=None):
    """Structured grid of nx*ny*nz hex8 cells; node id = i + (nx+1)(j + (ny+1)k)."""
    lx = float(nx) if lx is None else lx
    ly = float(ny) if ly is None else ly
    lz = float(nz) if lz is None else lz
    xs, ys, zs = np.linspace(0, lx, nx + 1), np.linspace(0, ly, ny + 1), np.linspace(0, lz, nz + 1)
    Z, Y, Xg = np.meshgrid(zs, ys, xs, indexing="ij")
    X = np.stack([Xg.ravel(), Y.ravel(), Z.ravel()], axis=1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    conn = np.zeros((base.shape[0], 8), dtype=np.int64)
    for c in range(8):
        ijk = base + _HEX_OFF[c]
        conn[:, c] = ijk[:, 0] + (nx + 1) * (ijk[:, 1] + (ny + 1) * ijk[:, 2])
    return X, conn.astype(np.int32)


def jitter_nodes(X, h, frac, rng):
    """Move every node by U[-frac, frac]*h per axis; boundary nodes keep their
    normal coordinate so the box faces stay flat."""
    lo, hi = X.min(axis=0), X.max(axis=0)
    dX = rng.uniform(-frac, frac, size=X.shape) * h
    on_face = np.isclose(X, lo) | np.isclose(X, hi)
    dX[on_face] = 0.0
    return X + dX


def gaussian_field(shape, sigma_cells, rng):
    """Periodic Gaussian random field: white noise convolved with a Gaussian of
    standard deviation sigma_cells (FFT), standardised to zero mean, unit std."""
    w = rng.standard_normal(shape)
    kern = np.ones(shape)
    for ax, n in enumerate(shape):
        f = np.fft.fftfreq(n)
        g = np.exp(-2.0 * (np.pi * f * sigma_cells) ** 2)
        sh = [1] * len(shape)
        sh[ax] = n
        kern = kern * g.reshape(sh)
    z = np.real(np.fft.ifftn(np.fft.fftn(w) * kern))
    return (z - z.mean()) / z.std()


def _field_to_range(z, lo, hi):
    """Map a standard normal field to [lo, hi] through the normal CDF."""
    from math import erf, sqrt
    cdf = 0.5 * (1.0 + np.vectorize(lambda v: erf(v / sqrt(2.0)))(z))
    return lo + (hi - lo) * cdf


class FourierField:
    """u(X) = sum_m a_m sin(2 pi k_m . (X / L) + phi_m), optionally multiplied by
    a linear ramp X_axis / L_axis so that the face X_axis = 0 stays fixed."""

    def __init__(self, rng, box, n_modes=3, kmax=2, ramp_axis=None):
        ks = []
        while len(ks) < n_modes:
            k = rng.integers(-kmax, kmax + 1, size=3)
            if np.any(k != 0):
                ks.append(k)
        self.k = np.array(ks, dtype=np.float64)
        self.a = rng.standard_normal((n_modes, 3))
        self.phi = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
        self.box = np.asarray(box, dtype=np.float64)
        self.ramp_axis = ramp_axis

    def _wave(self, X):
        arg = 2.0 * np.pi * (X / self.box) @ self.k.T + self.phi  # [n, m]
        return arg

    def value(self, X):
        arg = self._wave(X)
        u = np.sin(arg) @ self.a
        if self.ramp_axis is not None:
            u = u * (X[:, self.ramp_axis] / self.box[self.ramp_axis])[:, None]
        return u

    def grad(self, Xc):
        """Analytic displacement gradient [n, 3, 3] (du_i/dX_j) at the points Xc."""
        arg = self._wave(Xc)
        kk = 2.0 * np.pi * self.k / self.box  # [m, 3]
        grad = np.einsum("nm,mi,mj->nij", np.cos(arg), self.a, kk)
        if self.ramp_axis is not None:
            r = (Xc[:, self.ramp_axis] / self.box[self.ramp_axis])
            u = np.sin(arg) @ self.a
            grad = grad * r[:, None, None]
            grad[:, :, self.ramp_axis] += u / self.box[self.ramp_axis]
        return grad

    def max_strain(self, Xc):
        """max over the points Xc of the spectral norm of sym(grad u)."""
        g = self.grad(Xc)
        sym = 0.5 * (g + np.transpose(g, (0, 2, 1)))
        return float(np.max(np.abs(np.linalg.eigvalsh(sym))))


def centroids(X, conn):
    return X[conn].mean(axis=1)


def history(n_elems, rng, alpha_max=0.1, epsp_elem=None):
    """Per Gauss point history [7, 8*n_elems].  eps^p_n is element-constant:
    epsp_elem [n_elems, 3, 3] (or zero); alpha_n = sqrt(2/3)|eps^p_n| + U[0, alpha_max]."""
    n_gp = 8 * n_elems
    h = np.zeros((7, n_gp))
    extra = rng.uniform(0.0, alpha_max, size=n_gp)
    if epsp_elem is None:
        h[6] = extra
        return h
    D = np.repeat(np.asarray(epsp_elem, dtype=np.float64), 8, axis=0)
    h[0], h[1], h[2] = D[:, 0, 0], D[:, 1, 1], D[:, 2, 2]
    h[3], h[4], h[5] = D[:, 1, 2], D[:, 0, 2], D[:, 0, 1]
    h[6] = np.sqrt(2.0 / 3.0 * np.sum(D * D, axis=(1, 2))) + extra
    return h


def previous_plastic_strain(fld, scale, Xc):
    """Deviatoric part of sym(grad u_prev) at the element centroids: a stand-in
    for the plastic strain left by a previous load step."""
    g = scale * fld.grad(Xc)
    e = 0.5 * (g + np.transpose(g, (0, 2, 1)))
    tr = np.trace(e, axis1=1, axis2=2)
    e[:, [0, 1, 2], [0, 1, 2]] -= tr[:, None] / 3.0
    return e


def face_mask(X, axis, value=None, comps=(0, 1, 2)):
    """bc_mask [3n] with the listed components of nodes on X_axis == value set."""
    v = X[:, axis].min() if value is None else value
    on = np.isclose(X[:, axis], v)
    m = np.zeros((X.shape[0], 3), dtype=np.uint8)
    for c in comps:
        m[on, c] = 1
    return m.ravel()


def lam_unit(n_nodes, bc_mask, rng):
    lam = rng.standard_normal((n_nodes, 3))
    if bc_mask is not None:
        lam = lam * (1 - bc_mask.reshape(n_nodes, 3))
    return lam / np.linalg.norm(lam)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def tiny_cube(step=10, n_steps=10, seed=0):
    """4x4x4 unit cube, F=G=H=0.5, L=M=N=1.5, Swift K=500, eps0=0.01, n=0.2.
    Symmetry rollers on x=0, y=0, z=0; the face x=1 carries u_x = 0.002*step.
    d is the homogeneous uniaxial guess u_x = 0.002*step*x (a starting point;
    the other faces are free)."""
    X, conn = hex_grid(4, 4, 4, 1.0, 1.0, 1.0)
    ux = 0.02 * step / n_steps
    d = np.zeros_like(X)
    d[:, 0] = ux * X[:, 0]
    m = np.zeros((X.shape[0], 3), dtype=np.uint8)
    m[np.isclose(X[:, 0], 0.0), 0] = 1
    m[np.isclose(X[:, 1], 0.0), 1] = 1
    m[np.isclose(X[:, 2], 0.0), 2] = 1
    m[np.isclose(X[:, 0], 1.0), 0] = 1
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = np.zeros((7, 8 * conn.shape[0]))
    lam = lam_unit(X.shape[0], m.ravel(), rng)
    return Problem("tiny_cube", X, conn, d, hist, params(), m.ravel(), lam,
                   dict(ux=ux, nx=4, ny=4, nz=4))


def sheet_slab(seed=1, nx=40, ny=40, nz=4, strain=0.05, jitter=0.05):
    """Jittered slab [0,nx]x[0,ny]x[0,nz] (h = 1 mm), one Hill set F,G,H ~ U[0.2,0.8],
    Swift as tiny_cube, eps^p_n the deviatoric strain of a previous field at
    half the strain, alpha_n = sqrt(2/3)|eps^p_n| + U[0,0.1],
    displacement increment of 3 Fourier modes ramped in z (z=0 clamped)
    scaled to a maximum strain of `strain`, plus a previous displacement."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X0, conn = hex_grid(nx, ny, nz)
    X = jitter_nodes(X0, 1.0, jitter, rng)
    F, G, H = rng.uniform(0.2, 0.8, size=3)
    prm = params(F=F, G=G, H=H)
    box = np.array([nx, ny, nz], dtype=np.float64)
    Xc = centroids(X, conn)
    prev = FourierField(rng, box, ramp_axis=2)
    inc = FourierField(rng, box, ramp_axis=2)
    s_prev = 0.5 * strain / prev.max_strain(Xc)
    s_inc = strain / inc.max_strain(Xc)
    d = s_prev * prev.value(X) + s_inc * inc.value(X)
    hist = history(conn.shape[0], rng, epsp_elem=previous_plastic_strain(prev, s_prev, Xc))
    bc = face_mask(X, 2, 0.0)
    lam = lam_unit(X.shape[0], bc, rng)
    return Problem("sheet_slab", X, conn, d, hist, prm, bc, lam,
                   dict(nx=nx, ny=ny, nz=nz, seed=seed))


def large_cube(seed=2, n=100, amplitude=None, corr=10.0):
    """n^3 cube (h = 1 mm), per-element F,G,H = clip(0.5 + 0.15 z, 0.2, 0.8) from
    three Gaussian random fields of correlation length `corr` elements
    (sigma = corr/sqrt2), eps^p_n = 0, alpha_n ~ U[0, 0.1], Fourier displacement
    (no ramp) of the given amplitude, x = 0 face constrained."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X, conn = hex_grid(n, n, n)
    ne = conn.shape[0]
    prm = np.tile(params(), (ne, 1))
    for c, col in enumerate((2, 3, 4)):
        z = gaussian_field((n, n, n), corr / np.sqrt(2.0), rng)  # indexed [k, j, i]
        prm[:, col] = np.clip(0.5 + 0.15 * z.ravel(), 0.2, 0.8)
    hist = history(ne, rng)
    fld = FourierField(rng, np.array([n, n, n], dtype=np.float64), ramp_axis=None)
    amp = LARGE_CUBE_AMPLITUDE if amplitude is None else amplitude
    shape = fld.value(X)
    d = amp * shape
    bc = face_mask(X, 0, 0.0)
    lam = lam_unit(X.shape[0], bc, rng)
    return Problem("large_cube", X, conn, d, hist, prm, bc, lam,
                   dict(n=n, seed=seed, amplitude=amp, shape=shape))


def void_specimen(seed=3, nx=200, ny=200, nz=2, void_frac=0.25, strain=0.05):
    """nx x ny x nz slab; the lowest `void_frac` quantile of a 2-D Gaussian field
    (sigma = 8 elements) removes whole element columns; orphan nodes are dropped
    and nodes renumbered.  Per-element smooth fields: F,G,H in [0.2,0.8],
    N in [1.2,1.8], K in [450,550], eps0 in [0.005,0.015], n in [0.15,0.25].
    History and displacement as sheet_slab; unit random cotangent."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X, conn = hex_grid(nx, ny, nz)
    vf = gaussian_field((ny, nx), 8.0, rng)  # [j, i]
    cut = np.sort(vf.ravel())[int(round(void_frac * nx * ny))]
    keep_col = (vf >= cut).ravel()  # column index j*nx + i
    col_of_elem = np.tile(np.arange(nx * ny), nz)
    keep = keep_col[col_of_elem]
    conn = conn[keep]
    used = np.unique(conn)
    remap = -np.ones(X.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    X = X[used]
    conn = remap[conn].astype(np.int32)
    ne = conn.shape[0]
    prm = np.tile(params(), (ne, 1))
    ranges = {2: (0.2, 0.8), 3: (0.2, 0.8), 4: (0.2, 0.8), 7: (1.2, 1.8), 8: (450.0, 550.0),
              9: (0.005, 0.015), 10: (0.15, 0.25)}
    for col, (lo, hi) in ranges.items():
        z = gaussian_field((ny, nx), 8.0, rng).ravel()
        prm[:, col] = _field_to_range(z[col_of_elem[keep]], lo, hi)
    box = np.array([nx, ny, nz], dtype=np.float64)
    Xc = centroids(X, conn)
    prev = FourierField(rng, box, ramp_axis=2)
    inc = FourierField(rng, box, ramp_axis=2)
    s_prev = 0.5 * strain / prev.max_strain(Xc)
    d = s_prev * prev.value(X) + strain / inc.max_strain(Xc) * inc.value(X)
    hist = history(ne, rng, epsp_elem=previous_plastic_strain(prev, s_prev, Xc))
    bc = face_mask(X, 2, 0.0)
    lam = lam_unit(X.shape[0], bc, rng)
    grid_index = np.nonzero(keep)[0]
    return Problem("void_specimen", X, conn, d, hist, prm, bc, lam,
                   dict(nx=nx, ny=ny, nz=nz, seed=seed, grid_index=grid_index,
                        n_grid_elems=nx * ny * nz))


def uneven_slab(seed, n_target, strain=0.05):
    """One batch member: n_target ~ element count, n_z in {2,3,4}, aspect
    ~ logU[1,4]; own F,G,H ~ U[0.2,0.8], K ~ U[450,550], eps0 ~ U[0.005,0.015],
    n ~ U[0.15,0.25]; displacement and history as sheet_slab."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nz = int(rng.integers(2, 5))
    aspect = float(np.exp(rng.uniform(0.0, np.log(4.0))))
    nx = max(1, int(round(np.sqrt(n_target * aspect / nz))))
    ny = max(1, int(round(n_target / (nz * nx))))
    X0, conn = hex_grid(nx, ny, nz)
    X = jitter_nodes(X0, 1.0, 0.05, rng)
    prm = params(F=rng.uniform(0.2, 0.8), G=rng.uniform(0.2, 0.8), H=rng.uniform(0.2, 0.8),
                 K=rng.uniform(450, 550), eps0=rng.uniform(0.005, 0.015), n=rng.uniform(0.15, 0.25))
    box = np.array([nx, ny, nz], dtype=np.float64)
    Xc = centroids(X, conn)
    prev = FourierField(rng, box, ramp_axis=2)
    inc = FourierField(rng, box, ramp_axis=2)
    s_prev = 0.5 * strain / prev.max_strain(Xc)
    d = s_prev * prev.value(X) + strain / inc.max_strain(Xc) * inc.value(X)
    hist = history(conn.shape[0], rng, epsp_elem=previous_plastic_strain(prev, s_prev, Xc))
    bc = face_mask(X, 2, 0.0)
    lam = lam_unit(X.shape[0], bc, rng)
    return Problem(f"slab{seed}", X, conn, d, hist, prm, bc, lam, dict(nx=nx, ny=ny, nz=nz))


def batch64(n_spec=64, lo=2000, hi=60000, seed=4000):
    """n_spec uneven slabs; element counts log-uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_spec))
    return [uneven_slab(seed + i, int(round(s))) for i, s in enumerate(sizes)]


def hill_from_r(r11, r22, r33, r12, r13, r23):
    """F, G, H, L, M, N of the phi^2 form from the yield-stress ratios of App. A
    (G+H = 1/r11^2, F+H = 1/r22^2, F+G = 1/r33^2, N = 3/(2 r12^2),
    M = 3/(2 r13^2), L = 3/(2 r23^2))."""
    a, b, c = 1.0 / r11 ** 2, 1.0 / r22 ** 2, 1.0 / r33 ** 2
    return dict(F=0.5 * (b + c - a), G=0.5 * (a + c - b), H=0.5 * (a + b - c),
                L=1.5 / r23 ** 2, M=1.5 / r13 ** 2, N=1.5 / r12 ** 2)


def unit_cube_forward(n=100, ny=None, nz=None, nu=NU_DEFAULT):
    """The forward-simulation benchmark of the performance study (Sec. 3.1.3): the
    unit cube [0, 1]^3 mm in n^3 hex8 elements, Hill-48 with the yield-stress
    ratios r11..r23 = 1.5449, 1.0666, 1, 1.0307, 1, 1 and Voce hardening
    sigma0 = 138, Q = 410 MPa, b = 3.8, E = 219 GPa (nu not given: 0.3);
    the x = 0 face fixed, the x = 1 face moved by t (0.2, 0.1) mm in (x, y),
    its z motion free.  n x ny x nz elements (ny, nz default to n; the
    larger run of the study is 250 x 150 x 120).  Returns the Problem at
    t = 0 (hardening "voce") and the prescribed values at load factor t via
    meta["bc_at"](t)."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    X, conn = hex_grid(n, ny, nz, 1.0, 1.0, 1.0)
    hp = hill_from_r(1.5449, 1.0666, 1.0, 1.0307, 1.0, 1.0)
    prm = voce_params(sig0=138.0, Q=410.0, b=3.8, E=219000.0, nu=nu, **hp)
    left, right = np.isclose(X[:, 0], 0.0), np.isclose(X[:, 0], 1.0)
    bc = np.zeros((X.shape[0], 3), dtype=np.uint8)
    bc[left] = 1
    bc[right, 0] = 1
    bc[right, 1] = 1

    def bc_at(t):
        u = np.zeros((X.shape[0], 3))
        u[right, 0] = 0.2 * t
        u[right, 1] = 0.1 * t
        return u

    ne = conn.shape[0]
    return Problem(f"unit_cube_{n}x{ny}x{nz}", X, conn, np.zeros_like(X), np.zeros((7, 8 * ne)), prm, bc.ravel(),
                   None, dict(nx=n, ny=ny, nz=nz, bc_at=bc_at), hardening="voce")


# Load factors of the ten unequal steps of the tensile-specimen study (Sec. 3.2).
TENSILE_STEPS = (0.005, 0.006, 0.02, 0.045, 0.09, 0.15, 0.3, 0.5, 0.75, 1.0)


def tensile_specimen(nx=35, ny=30, nz=5, angle_deg=45.0):
    """Stand-in for the tensile specimen of the inverse study (Sec. 3.2: 5,250
    hex8, orientation 45 degrees to the load, bottom fixed, top moved 0.5 mm
    in y over TENSILE_STEPS, E = 200 GPa, nu = 0.3, r11 = r13 = r23 = 1): the
    specimen's shape is not given, so a 35 x 30 x 3 mm slab of nx x ny x nz
    elements (5,250 by default) with the y = 0 face fixed and the y = 30 face
    gripped (x, z fixed, y prescribed).  Hill-48 from r = (1, 1.1, 0.9, 1.05,
    1, 1), Voce (200, 150, 20) as the reference material.  Returns the
    Problem (hardening "voce", orientation set) with meta["bc_at"](t)."""
    X, conn = hex_grid(nx, ny, nz, 35.0, 30.0, 3.0)
    prm = voce_params(E=200000.0, nu=0.3, **hill_from_r(1.0, 1.1, 0.9, 1.05, 1.0, 1.0))
    bottom, top = np.isclose(X[:, 1], 0.0), np.isclose(X[:, 1], 30.0)
    bc = np.zeros((X.shape[0], 3), dtype=np.uint8)
    bc[bottom] = 1
    bc[top] = 1

    def bc_at(t):
        u = np.zeros((X.shape[0], 3))
        u[top, 1] = 0.5 * t
        return u

    ne = conn.shape[0]
    return Problem(f"tensile_{nx}x{ny}x{nz}", X, conn, np.zeros_like(X), np.zeros((7, 8 * ne)), prm, bc.ravel(),
                   None, dict(nx=nx, ny=ny, nz=nz, bc_at=bc_at, steps=TENSILE_STEPS), hardening="voce",
                   orient=rotation_z(np.deg2rad(angle_deg)).reshape(9))


def small_slab(seed, nx, ny, nz, per_element=False, strain=0.05, jitter=0.05, alpha_max=0.1):
    """Small jittered slab for parity tests with ragged element counts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X0, conn = hex_grid(nx, ny, nz)
    X = jitter_nodes(X0, 1.0, jitter, rng)
    ne = conn.shape[0]
    if per_element:
        prm = np.tile(params(), (ne, 1))
        prm[:, 2:5] = rng.uniform(0.2, 0.8, size=(ne, 3))
        prm[:, 5:8] = rng.uniform(1.2, 1.8, size=(ne, 3))
        prm[:, 8] = rng.uniform(450, 550, size=ne)
        prm[:, 9] = rng.uniform(0.005, 0.015, size=ne)
        prm[:, 10] = rng.uniform(0.15, 0.25, size=ne)
    else:
        prm = params(F=rng.uniform(0.2, 0.8), G=rng.uniform(0.2, 0.8), H=rng.uniform(0.2, 0.8))
    box = np.array([nx, ny, nz], dtype=np.float64)
    Xc = centroids(X, conn)
    prev = FourierField(rng, box, ramp_axis=None)
    fld = FourierField(rng, box, ramp_axis=None)
    s_prev = 0.5 * strain / prev.max_strain(Xc)
    d = s_prev * prev.value(X) + strain / fld.max_strain(Xc) * fld.value(X)
    hist = history(ne, rng, alpha_max=alpha_max, epsp_elem=previous_plastic_strain(prev, s_prev, Xc))
    bc = face_mask(X, 0, 0.0)
    lam = lam_unit(X.shape[0], bc, rng)
    return Problem(f"small{seed}_{nx}x{ny}x{nz}", X, conn, d, hist, prm, bc, lam,
                   dict(nx=nx, ny=ny, nz=nz))


def concat(problems):
    """Concatenate specimens into one mesh (node ids offset); returns the merged
    Problem (per-element parameters) and the element/node offsets."""
    node_off = np.zeros(len(problems) + 1, dtype=np.int64)
    elem_off = np.zeros(len(problems) + 1, dtype=np.int64)
    for i, p in enumerate(problems):
        node_off[i + 1] = node_off[i] + p.n_nodes
        elem_off[i + 1] = elem_off[i] + p.n_elems
    X = np.concatenate([p.X for p in problems])
    conn = np.concatenate([p.conn.astype(np.int64) + node_off[i] for i, p in enumerate(problems)])
    d = np.concatenate([p.d for p in problems])
    hist = np.concatenate([p.hist_n for p in problems], axis=1)
    prm = np.concatenate([np.broadcast_to(p.prm, (p.n_elems, 11)) if p.prm.ndim == 1 else p.prm
                          for p in problems])
    bc = np.concatenate([p.bc_mask for p in problems])
    lam = np.concatenate([p.lam for p in problems])
    spec_prm = np.stack([p.prm if p.prm.ndim == 1 else p.prm[0] for p in problems])
    merged = Problem("batch", X, conn.astype(np.int32), d, hist, np.ascontiguousarray(prm), bc, lam,
                     dict(node_off=node_off, elem_off=elem_off, spec_prm=spec_prm))
    return merged
