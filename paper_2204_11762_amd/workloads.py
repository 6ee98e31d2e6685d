"""Seeded synthetic inputs for MFA volume rendering.

This module only *draws* inputs: control-point grids, knot vectors, cameras,
transfer-function tables, render parameters and pixel subsets.  It holds
none of the renderer's arithmetic and is shared, as plain numpy arrays and
numbers, by the HIP library's tests and benchmark and by the CPU oracle.

Least-squares fits of the synthetic test field use scipy's B-spline
collocation matrices (an independent library routine); the fitting step is
input preparation, the MFA encoder itself being an offline step outside the
renderer (Sect. 3: the encoded model is the renderer's input).

All random draws use ``numpy.random.default_rng(seed)`` (PCG64).

Workloads (sizes of the paper-shaped synthetic configurations):

* ``c1``: degree 2, 16^3 control points i.i.d. U[0,1] (seed 0), clamped
  uniform knots; 128^2 orthographic image looking down -z; step 1/256;
  256-entry linear-ramp RGBA table over [0, 1].
* ``c2``: degree 3, 64^3 control points = least-squares fit of
  ``sin(6x) cos(5y) sin(7z) + 0.3 exp(-40 |r - 0.5|^2)`` sampled on a 128^3
  grid; clamped uniform knots; 512^2 perspective image (60 deg vertical
  field of view, orbit radius 2, azimuth 30 deg, elevation 20 deg);
  step 1/512; 8-node piecewise-linear RGBA table (seed 2) rasterised to 256
  entries over [min P, max P].
* ``c3``: degree 3, 256^3 control points = the same field fitted on a 512^3
  grid, plus N(0, 0.01^2) noise (seed 3); same camera at 1024^2; step
  1/1024; table as in c2 over this model's range; 4096-pixel subset drawn
  without replacement (seed 4).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# plain input records (numpy / python scalars only)
# ---------------------------------------------------------------------------

@dataclass
class ModelSpec:
    degree: tuple                      # (p_x, p_y, p_z)
    knots: tuple                       # three float64 arrays
    ctrl: np.ndarray                   # float64 (n_z, n_y, n_x), x fastest
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    weights: np.ndarray | None = None  # rational weights like ctrl (> 0), or None

    @property
    def n(self):
        nz, ny, nx = self.ctrl.shape
        return (nx, ny, nz)


@dataclass
class CameraSpec:
    kind: str                          # "ortho" | "persp"
    eye: tuple
    target: tuple
    up: tuple
    width: int
    height: int
    fov_y_deg: float = 60.0
    ortho_half_w: float = 0.5
    ortho_half_h: float = 0.5


@dataclass
class TFSpec:
    table: np.ndarray                  # float32 (n, 4) RGBA
    v_lo: float
    v_hi: float


@dataclass
class CurvatureTFSpec:
    table: np.ndarray                  # float32 (m, m, 4) RGBA: [i2, i1], k2 row, k1 column
    k_lo: float
    k_hi: float


def curvature_tf(m: int = 32, k_lo: float = -4.0, k_hi: float = 4.0) -> CurvatureTFSpec:
    """A table over the principal curvatures (k1, k2) in the manner of
    curvature-based transfer functions: red where both are positive (the
    surface curves around lower values), blue where both are negative, green
    on saddles, grey near flat; opacity grows with sqrt(k1^2 + k2^2) so that
    flat regions stay faint."""
    k = np.linspace(k_lo, k_hi, m)
    k2, k1 = np.meshgrid(k, k, indexing="ij")
    scale = max(abs(k_lo), abs(k_hi))
    mag = np.sqrt(k1 ** 2 + k2 ** 2) / scale
    conv = np.clip(np.minimum(k1, k2) / scale, 0, 1)
    conc = np.clip(-np.maximum(k1, k2) / scale, 0, 1)
    sadl = np.clip(np.minimum(k1, -k2) / scale, 0, 1) * (k1 * k2 < 0)
    grey = 0.5 * (1.0 - np.clip(conv + conc + sadl, 0, 1))
    table = np.stack([conv + grey, sadl + grey, conc + grey,
                      0.15 + 0.85 * np.clip(mag, 0, 1)], axis=-1)
    return CurvatureTFSpec(np.clip(table, 0, 1).astype(np.float32), float(k_lo), float(k_hi))


@dataclass
class ParamSpec:
    step: float
    ert_alpha: float = 0.99
    shading: bool = True
    ka: float = 0.1
    kd: float = 0.7
    ks: float = 0.2
    shininess: int = 10
    headlight: bool = True
    light_dir: tuple = (0.0, 0.0, 1.0)


@dataclass
class Workload:
    name: str
    model: ModelSpec
    camera: CameraSpec
    tf: TFSpec
    params: ParamSpec
    subset: np.ndarray | None = None   # flat pixel indices, or None = full
    extra: dict = field(default_factory=dict)


# ---------------------------------------------------------------------------
# knot vectors
# ---------------------------------------------------------------------------

def clamped_uniform_knots(n: int, p: int) -> np.ndarray:
    """``p+1`` zeros, interior knots ``k/(n-p)``, ``p+1`` ones."""
    m = n - p
    inner = np.array([k / m for k in range(1, m)], dtype=np.float64)
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def clamped_beta_knots(n: int, p: int, rng: np.random.Generator,
                       a: float = 2.0, b: float = 5.0) -> np.ndarray:
    """Clamped knots whose ``n-p`` spacings are i.i.d. Beta(a, b) draws,
    normalised to sum 1; a spacing below ``1e-3/(n-p)`` is redrawn."""
    m = n - p
    d = rng.beta(a, b, size=m)
    while True:
        small = d < 1e-3 / m
        if not small.any():
            break
        d[small] = rng.beta(a, b, size=int(small.sum()))
    d = d / d.sum()
    inner = np.cumsum(d)[:-1]
    inner = np.minimum(inner, np.nextafter(1.0, 0.0))
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


# ---------------------------------------------------------------------------
# least-squares fits of the synthetic field (scipy collocation matrices)
# ---------------------------------------------------------------------------

def _pinv_apply(knots: np.ndarray, p: int, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Least-squares 1-D coefficients c minimising |B c - ys| where B is the
    collocation matrix of the spline space at the sites xs."""
    from scipy.interpolate import BSpline
    B = BSpline.design_matrix(xs, knots, p).toarray()
    c, *_ = np.linalg.lstsq(B, ys, rcond=None)
    return c


def fit_test_field(n: int, p: int, grid: int) -> tuple[np.ndarray, np.ndarray]:
    """Separable least-squares fit of
    ``f = sin(6x) cos(5y) sin(7z) + 0.3 exp(-40 |r - 0.5|^2)`` sampled at
    ``x_g = g/(grid-1)`` on a ``grid^3`` lattice, with ``n^3`` control points
    on clamped uniform knots.

    Both terms are products of one-dimensional factors, and the least-squares
    operator of a tensor-product collocation matrix is the tensor product of
    the per-axis pseudo-inverses, so the 3-D fit equals the sum of outer
    products of 1-D fits (exactly, in exact arithmetic).
    Returns (control points (n,n,n) x fastest, knots).
    """
    U = clamped_uniform_knots(n, p)
    xs = np.arange(grid, dtype=np.float64) / (grid - 1)
    g = np.exp(-40.0 * (xs - 0.5) ** 2)
    ax = _pinv_apply(U, p, xs, np.sin(6.0 * xs))
    by = _pinv_apply(U, p, xs, np.cos(5.0 * xs))
    cz = _pinv_apply(U, p, xs, np.sin(7.0 * xs))
    gx = _pinv_apply(U, p, xs, g)
    # P[k, j, i] = a_i b_j c_k + 0.3 g_i g_j g_k
    P = (cz[:, None, None] * by[None, :, None] * ax[None, None, :]
         + 0.3 * gx[:, None, None] * gx[None, :, None] * gx[None, None, :])
    return P, U


def test_field(x, y, z):
    """The analytic field the c2/c3 models are fitted to."""
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    return np.sin(6 * x) * np.cos(5 * y) * np.sin(7 * z) + 0.3 * np.exp(-40 * r2)


# ---------------------------------------------------------------------------
# transfer functions and cameras
# ---------------------------------------------------------------------------

def ramp_tf(n: int = 256, v_lo: float = 0.0, v_hi: float = 1.0) -> TFSpec:
    e = np.arange(n, dtype=np.float64) / (n - 1)
    table = np.repeat(e[:, None], 4, axis=1).astype(np.float32)
    return TFSpec(table, v_lo, v_hi)


def pwl_tf(seed: int, v_lo: float, v_hi: float, nodes: int = 8, n: int = 256,
           alpha_max: float = 0.05) -> TFSpec:
    """``nodes`` equally spaced nodes, RGB ~ U[0,1], alpha ~ U[0, alpha_max],
    rasterised (FP64 linear interpolation) to ``n`` entries at e/(n-1)."""
    rng = np.random.default_rng(seed)
    rgb = rng.random((nodes, 3))
    alpha = rng.random(nodes) * alpha_max
    xn = np.linspace(0.0, 1.0, nodes)
    xe = np.arange(n, dtype=np.float64) / (n - 1)
    table = np.empty((n, 4))
    for ch in range(3):
        table[:, ch] = np.interp(xe, xn, rgb[:, ch])
    table[:, 3] = np.interp(xe, xn, alpha)
    return TFSpec(table.astype(np.float32), float(v_lo), float(v_hi))


def orbit_camera(width: int, height: int, az_deg: float, el_deg: float,
                 radius: float = 2.0, fov_y_deg: float = 60.0,
                 target=(0.5, 0.5, 0.5)) -> CameraSpec:
    az = math.radians(az_deg)
    el = math.radians(el_deg)
    eye = (target[0] + radius * math.cos(el) * math.sin(az),
           target[1] + radius * math.sin(el),
           target[2] + radius * math.cos(el) * math.cos(az))
    return CameraSpec("persp", eye, tuple(target), (0.0, 1.0, 0.0), width, height,
                      fov_y_deg=fov_y_deg)


def random_orbit_camera(rng: np.random.Generator, width: int, height: int,
                        radius: float = 2.0) -> CameraSpec:
    az = rng.uniform(0.0, 360.0)
    el = rng.uniform(-60.0, 60.0)
    return orbit_camera(width, height, az, el, radius)


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def c1() -> Workload:
    n, p = 16, 2
    rng = np.random.default_rng(0)
    ctrl = rng.random(n ** 3).reshape(n, n, n)
    U = clamped_uniform_knots(n, p)
    model = ModelSpec((p, p, p), (U, U.copy(), U.copy()), ctrl)
    cam = CameraSpec("ortho", (0.5, 0.5, 2.0), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0),
                     128, 128, ortho_half_w=0.5, ortho_half_h=0.5)
    return Workload("c1", model, cam, ramp_tf(256, 0.0, 1.0), ParamSpec(step=1.0 / 256))


_C2_CACHE: dict = {}


def c2() -> Workload:
    if "c2" not in _C2_CACHE:
        _C2_CACHE["c2"] = fit_test_field(64, 3, 128)
    P, U = _C2_CACHE["c2"]
    model = ModelSpec((3, 3, 3), (U, U.copy(), U.copy()), P.copy())
    cam = orbit_camera(512, 512, 30.0, 20.0)
    tf = pwl_tf(2, float(P.min()), float(P.max()))
    return Workload("c2", model, cam, tf, ParamSpec(step=1.0 / 512))


def c3(subset_size: int = 4096) -> Workload:
    P, U = fit_test_field(256, 3, 512)
    rng = np.random.default_rng(3)
    P = P + rng.normal(0.0, 0.01, size=P.size).reshape(P.shape)
    model = ModelSpec((3, 3, 3), (U, U.copy(), U.copy()), P)
    cam = orbit_camera(1024, 1024, 30.0, 20.0)
    tf = pwl_tf(2, float(P.min()), float(P.max()))
    sub = np.sort(np.random.default_rng(4).choice(1024 * 1024, size=subset_size,
                                                  replace=False))
    return Workload("c3", model, cam, tf, ParamSpec(step=1.0 / 1024), subset=sub)


def random_model(rng: np.random.Generator, n=(9, 7, 8), degree=(3, 2, 1),
                 beta_knots=False, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                 smooth=True) -> ModelSpec:
    """A small random model for parity cases (any degree, non-uniform knots,
    non-unit box).  ``smooth`` adds a low-frequency trend to the noise so
    that shading sees a meaningful gradient."""
    knots = []
    for k in range(3):
        if beta_knots:
            knots.append(clamped_beta_knots(n[k], degree[k], rng))
        else:
            knots.append(clamped_uniform_knots(n[k], degree[k]))
    nx, ny, nz = n
    ctrl = rng.random(nx * ny * nz).reshape(nz, ny, nx)
    if smooth:
        zz, yy, xx = np.meshgrid(np.linspace(0, 1, nz), np.linspace(0, 1, ny),
                                 np.linspace(0, 1, nx), indexing="ij")
        ctrl = 0.3 * ctrl + 0.7 * (np.sin(3 * xx) * np.cos(2 * yy) + zz)
    return ModelSpec(tuple(degree), tuple(knots), ctrl, tuple(map(float, lo)),
                     tuple(map(float, hi)))


def fit_field_on_knots(knots, degree, grid_factor: int = 2) -> np.ndarray:
    """Separable least-squares fit of the test field on the given knot
    vectors (one per axis, any clamped knots), sampled at ``grid_factor * n``
    equally spaced sites per axis.  Returns control points (n_z, n_y, n_x)."""
    fits = []
    for k in range(3):
        U = np.asarray(knots[k], dtype=np.float64)
        n = len(U) - degree[k] - 1
        xs = np.linspace(0.0, 1.0, grid_factor * n)
        g = np.exp(-40.0 * (xs - 0.5) ** 2)
        trig = (np.sin(6.0 * xs), np.cos(5.0 * xs), np.sin(7.0 * xs))[k]
        fits.append((_pinv_apply(U, degree[k], xs, trig), _pinv_apply(U, degree[k], xs, g)))
    (ax, gx), (by, gy), (cz, gz) = fits
    return (cz[:, None, None] * by[None, :, None] * ax[None, None, :]
            + 0.3 * gz[:, None, None] * gy[None, :, None] * gx[None, None, :])


@dataclass
class BatchRequest:
    model: int                         # index into the batch's model list
    camera: CameraSpec
    tf: TFSpec
    params: ParamSpec


def batch_mix_small(seed: int = 11):
    """Small mixed batch for parity tests: four models (uniform and Beta
    knots, degrees 1-4, mixed per axis, non-unit box, FP32 and BF16) and
    eight requests (ragged image sizes, perspective and orthographic,
    shading off, no early termination, one 2048-entry table).
    Returns ([(ModelSpec, store)], [BatchRequest])."""
    rng = np.random.default_rng(seed)
    models = [
        (random_model(rng, n=(9, 8, 7), degree=(3, 3, 3)), 0),
        (random_model(rng, n=(10, 9, 11), degree=(2, 3, 1), beta_knots=True,
                      lo=(-1.0, 0.0, 0.0), hi=(1.0, 1.0, 2.0)), 1),
        (random_model(rng, n=(8, 8, 8), degree=(4, 4, 4), beta_knots=True), 1),
        (random_model(rng, n=(12, 10, 9), degree=(2, 2, 2)), 0),
    ]
    sizes = [(37, 29), (40, 33), (23, 41), (64, 48), (31, 31), (48, 17), (56, 40), (33, 52)]
    reqs = []
    for i, (W, H) in enumerate(sizes):
        mi = i % len(models)
        spec = models[mi][0]
        lo, hi = np.asarray(spec.lo), np.asarray(spec.hi)
        ctr = tuple((lo + hi) / 2)
        ext = float(np.max(hi - lo))
        if i == 4:
            cam = CameraSpec("ortho", (ctr[0] + 0.3, ctr[1] + 0.2, ctr[2] + 3 * ext), ctr,
                             (0.0, 1.0, 0.0), W, H, ortho_half_w=0.6 * ext,
                             ortho_half_h=0.7 * ext)
        else:
            cam = orbit_camera(W, H, float(rng.uniform(0, 360)), float(rng.uniform(-50, 50)),
                               radius=2.2 * ext, target=ctr)
        P = np.asarray(spec.ctrl)
        tf = pwl_tf(seed + i, P.min(), P.max(), alpha_max=0.15, n=2048 if i == 6 else 256)
        prm = ParamSpec(step=ext / 97.0, ert_alpha=1.5 if i == 5 else 0.99,
                        shading=(i != 2), headlight=(i % 3 != 1), light_dir=(0.3, -0.5, 0.8))
        reqs.append(BatchRequest(mi, cam, tf, prm))
    return models, reqs


def batch_config(seed: int = 21, n_requests: int = 64):
    """The batching workload: four resident BF16 models with Beta(2,5)
    knot spacings, degrees 2/3/4/3, control grids 32^3, 96x128x80, 128^3
    and 200x200x100 (least-squares fits of the test field); n_requests
    requests over them with image sizes drawn from {256^2, 512^2, 768x432,
    1024^2}, step 1/512, random orbit cameras and per-model 8-node tables.
    Returns ([(ModelSpec, store)], [BatchRequest])."""
    rng = np.random.default_rng(seed)
    shapes = [((32, 32, 32), 2), ((96, 128, 80), 3), ((128, 128, 128), 4), ((200, 200, 100), 3)]
    models, tfs = [], []
    for (n, p) in shapes:
        knots = tuple(clamped_beta_knots(n[k], p, rng) for k in range(3))
        ctrl = fit_field_on_knots(knots, (p, p, p))
        models.append((ModelSpec((p, p, p), knots, ctrl), 1))
        tfs.append(pwl_tf(int(rng.integers(1 << 30)), float(ctrl.min()), float(ctrl.max())))
    sizes = [(256, 256), (512, 512), (768, 432), (1024, 1024)]
    reqs = []
    for _ in range(n_requests):
        mi = int(rng.integers(len(models)))
        W, H = sizes[int(rng.integers(len(sizes)))]
        reqs.append(BatchRequest(mi, random_orbit_camera(rng, W, H), tfs[mi],
                                 ParamSpec(step=1.0 / 512)))
    return models, reqs


def serve_config(seed: int = 41, rate: float = 400.0, duration_s: float = 2.0):
    """The serving workload: a Poisson request stream (mean ``rate`` per
    second for ``duration_s``) over 16 resident models (degree 2-4 on every
    axis; 32^3 to 256^3 control points; FP32 or BF16; uniform or Beta(2,5)
    knots; least-squares fits of the test field).  Each request draws its
    model, an orbit camera, an image size from {128^2, 256^2, 512^2,
    1024x768, 1280x720, 1920x1080}, N in {128, 256, 512, 1024} samples per
    unit length (step 1/N) and its own 8-node table.
    Returns ([(ModelSpec, store)], [BatchRequest], arrival times in s)."""
    rng = np.random.default_rng(seed)
    grids = [32, 64, 128, 256]
    models = []
    for i in range(16):
        p = 2 + i % 3
        n = grids[(i // 3) % 4] if i < 12 else grids[i % 4]
        beta = bool(i % 2)
        if beta:
            knots = tuple(clamped_beta_knots(n, p, rng) for _ in range(3))
        else:
            knots = tuple(clamped_uniform_knots(n, p) for _ in range(3))
        ctrl = fit_field_on_knots(knots, (p, p, p))
        models.append((ModelSpec((p, p, p), knots, ctrl), int(i % 4 >= 2)))
    sizes = [(128, 128), (256, 256), (512, 512), (1024, 768), (1280, 720), (1920, 1080)]
    n_req = int(round(rate * duration_s))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    reqs = []
    for i in range(n_req):
        mi = int(rng.integers(len(models)))
        W, H = sizes[int(rng.integers(len(sizes)))]
        N = int(rng.choice([128, 256, 512, 1024]))
        P = models[mi][0].ctrl
        tf = pwl_tf(int(rng.integers(1 << 30)), float(P.min()), float(P.max()))
        reqs.append(BatchRequest(mi, random_orbit_camera(rng, W, H), tf, ParamSpec(step=1.0 / N)))
    return models, reqs, arrivals


# ---------------------------------------------------------------------------
# the paper's closed-form fields (Sect. 4.1.1) on the box [-1, 1]^3
# ---------------------------------------------------------------------------

FIELD_LO = (-1.0, -1.0, -1.0)
FIELD_HI = (1.0, 1.0, 1.0)


def gaussian_beam(x, y, z, v_min=0.0, v_max=255.0, mu=0.0, sigma=1.0 / 3.0, radius=math.sqrt(3.0)):
    """Eq. (1): V_min + (V_max - V_min) G(|r| / R), G(l) = exp(-(l - mu)^2 / (2 sigma^2)).
    Returns (value, gradient (..., 3))."""
    x, y, z = (np.asarray(t, dtype=np.float64) for t in (x, y, z))
    r = np.sqrt(x * x + y * y + z * z)
    l = r / radius
    G = np.exp(-(l - mu) ** 2 / (2.0 * sigma ** 2))
    f = v_min + (v_max - v_min) * G
    # dG/dl = -(l - mu) / sigma^2 G; dl/dx_k = x_k / (R r)  (mu = 0: smooth at r = 0)
    with np.errstate(invalid="ignore", divide="ignore"):
        dl = np.where(r > 0, 1.0 / (radius * r), 0.0)
    dGdl = -(l - mu) / sigma ** 2 * G
    if mu == 0.0:
        fac = (v_max - v_min) * (-G / (sigma ** 2 * radius ** 2))   # d/dx_k = fac x_k
        g = np.stack([fac * x, fac * y, fac * z], axis=-1)
    else:
        g = np.stack([(v_max - v_min) * dGdl * dl * t for t in (x, y, z)], axis=-1)
    return f, g


def marschner_lobb(x, y, z, f_m=6.0, alpha=0.25):
    """Eq. (2): (1 - sin(pi z / 2) + alpha (1 + rho(sqrt(x^2 + y^2)))) / (2 (1 + alpha)),
    rho(r) = cos(2 pi f_M cos(pi r / 2)).  Returns (value, gradient (..., 3))."""
    x, y, z = (np.asarray(t, dtype=np.float64) for t in (x, y, z))
    r = np.sqrt(x * x + y * y)
    inner = 2.0 * np.pi * f_m * np.cos(np.pi * r / 2.0)
    rho = np.cos(inner)
    den = 2.0 * (1.0 + alpha)
    f = (1.0 - np.sin(np.pi * z / 2.0) + alpha * (1.0 + rho)) / den
    # drho/dr = sin(inner) 2 pi f_M sin(pi r / 2) pi / 2; dr/dx = x / r
    drho_dr = np.sin(inner) * 2.0 * np.pi * f_m * np.sin(np.pi * r / 2.0) * (np.pi / 2.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        q = np.where(r > 0, drho_dr / r, 0.0)   # drho_dr ~ r near 0: limit is finite
    small = r < 1e-12
    if np.any(small):
        # drho/dr / r -> 2 pi f_M sin(2 pi f_M) (pi / 2)^2 as r -> 0
        q = np.where(small, 2.0 * np.pi * f_m * np.sin(2.0 * np.pi * f_m) * (np.pi / 2.0) ** 2, q)
    gx = alpha * q * x / den
    gy = alpha * q * y / den
    gz = -(np.pi / 2.0) * np.cos(np.pi * z / 2.0) / den
    return f, np.stack([gx, gy, gz * np.ones_like(gx)], axis=-1)


def field_grid(field, N: int) -> np.ndarray:
    """The discrete dataset: the field at N^3 equally spaced points of
    [-1, 1]^3, shape (N, N, N) indexed (z, y, x)."""
    t = np.linspace(-1.0, 1.0, N)
    zz, yy, xx = np.meshgrid(t, t, t, indexing="ij")
    return field(xx, yy, zz)[0]


def fit_grid(data: np.ndarray, n: int, p: int) -> ModelSpec:
    """Least-squares MFA of an (N, N, N) grid dataset on [-1, 1]^3 with n
    control points of degree p per axis on clamped uniform knots: the
    tensor-product least-squares solution, applied one axis at a time (the
    pseudo-inverse of a Kronecker product is the Kronecker product of the
    pseudo-inverses).  Input preparation standing in for the MFA encoder."""
    from scipy.interpolate import BSpline
    N = data.shape[0]
    U = clamped_uniform_knots(n, p)
    sites = np.linspace(0.0, 1.0, N)
    B = BSpline.design_matrix(sites, U, p).toarray()
    Bp = np.linalg.pinv(B)                      # (n, N)
    P = np.einsum("az,zyx->ayx", Bp, data)
    P = np.einsum("by,ayx->abx", Bp, P)
    P = np.einsum("cx,abx->abc", Bp, P)
    return ModelSpec((p, p, p), (U, U.copy(), U.copy()), P, FIELD_LO, FIELD_HI)


def pixel_subset(width: int, height: int, size: int, seed: int) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(width * height, size=size,
                                                      replace=False))


def uniform_points(rng: np.random.Generator, m: int, lo=(0.0, 0.0, 0.0),
                   hi=(1.0, 1.0, 1.0)) -> np.ndarray:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + rng.random((m, 3)) * (hi - lo)


def morton_order(xyz: np.ndarray, bits: int = 10) -> np.ndarray:
    """Permutation that sorts points in [0,1]^3 along a Morton (Z-order) curve."""
    q = np.clip((xyz * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(len(xyz), dtype=np.int64)
    for bit in range(bits):
        for k in range(3):
            code |= ((q[:, k] >> bit) & 1) << (3 * bit + k)
    return np.argsort(code, kind="stable")
