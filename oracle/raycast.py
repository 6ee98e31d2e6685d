"""FP64 direct volume ray caster for an MFA model -- oracle, test only.

Follows the rendering steps of Sect. 3.1 and Algorithm 1: a ray per pixel
(fixed-point ray-cast model), samples at a constant distance from the first
to the last sample inside the volume, normalisation of each sample position
to the unit cube, the value query, the colour/opacity transfer function,
(with shading on) the gradient query and Phong lighting, front-to-back
compositing, and early ray termination once the accumulated opacity exceeds
the maximum opacity (tested after the sample has been composited).

Where the paper is silent, the readings below are used (each one is listed
with its reason in the design notes of the repository):

* camera: pixel centres, row 0 at the top; perspective with a vertical
  field of view; orthographic window of half extents ``half_w, half_h``;
* sampling: ``N = floor((t_exit - t_enter) / step)`` samples at the
  midpoints ``t_enter + (s + 1/2) step``; ``t_enter`` is clamped to 0 when
  the eye is inside the box;
* parameters ``u = clamp((x - lo) / (hi - lo), 0, 1)``, world gradient by
  the chain rule;
* one RGBA table with linear interpolation over ``[v_lo, v_hi]``; no
  opacity correction for the step;
* Phong with one light: ``n = g / max(|g|, 1e-6)``, two-sided diffuse
  ``|n.l|``, reflection ``r = 2 (n.l) n - l``, specular ``max(0, r.v)^k``
  (integer ``k``), ``c' = min(1, (k_a + k_d diff) c + k_s spec)``;
  the light is the headlight ``l = -F`` (F the viewing axis) unless a light
  direction is given; ``v = -d``;
* premultiplied output ``(C_r, C_g, C_b, A)``, transparent black for rays
  that miss the box;
* curvature transfer function (optional; the use the model's analytic
  second derivatives are for): the principal curvatures of the isosurface
  through the sample, ``k1 >= k2``, are the two tangential eigenvalues of
  ``G = P H P / |g|`` (``H`` the world Hessian, ``P = I - n n^T``,
  ``n = g / |g|``), i.e. ``k1,2 = (T +- |k1 - k2|) / 2`` with
  ``T = trace G`` and ``|k1 - k2| = sqrt(2) |G - (T/2) P|_F`` (the traceless
  tangential part, whose entries carry no cancellation, unlike
  ``2 |G|_F^2 - T^2``; a sphere around lower values has ``k1 = k2 = 1/r``;
  both are 0 where ``|g|^2 < 1e-12``); an
  ``m x m`` RGBA table over ``[k_lo, k_hi]^2`` (k1 along the first table
  axis) interpolated bilinearly with clamping gives the sample's colour,
  and its opacity multiplies the value table's.

Pixel-level arithmetic of the camera and slab steps is written operation by
operation (no library reductions) so that the ray parameters are the plain
IEEE results of the stated formulas.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .bspline import HESS_PAIRS, Model, eval_local, hessian_from_models, hessian_models

GRAD_EPS = 1e-6


@dataclass
class Camera:
    kind: str                     # "ortho" or "persp"
    eye: tuple
    target: tuple
    up: tuple
    width: int
    height: int
    fov_y_deg: float = 60.0
    ortho_half_w: float = 0.5
    ortho_half_h: float = 0.5


@dataclass
class TransferFunction:
    table: np.ndarray             # (n, 4) RGBA, float32 values
    v_lo: float
    v_hi: float


@dataclass
class CurvatureTF:
    table: np.ndarray             # (m, m, 4) RGBA, float32 values; [i2, i1]: k2 row, k1 column
    k_lo: float
    k_hi: float


@dataclass
class RenderParams:
    step: float
    ert_alpha: float = 0.99       # >= 1 disables early termination
    shading: bool = True
    ka: float = 0.1
    kd: float = 0.7
    ks: float = 0.2
    shininess: int = 10
    headlight: bool = True
    light_dir: tuple = field(default=(0.0, 0.0, 1.0))


# ---------------------------------------------------------------------------
# camera and rays
# ---------------------------------------------------------------------------

def _unit(x, y, z):
    ln = math.sqrt(x * x + y * y + z * z)
    return x / ln, y / ln, z / ln


def camera_frame(cam: Camera):
    """Viewing axis F, right R and true up V (unit vectors, plain floats)."""
    F = _unit(cam.target[0] - cam.eye[0], cam.target[1] - cam.eye[1],
              cam.target[2] - cam.eye[2])
    ux, uy, uz = cam.up
    R = _unit(F[1] * uz - F[2] * uy, F[2] * ux - F[0] * uz, F[0] * uy - F[1] * ux)
    V = (R[1] * F[2] - R[2] * F[1], R[2] * F[0] - R[0] * F[2], R[0] * F[1] - R[1] * F[0])
    return F, R, V


def camera_rays(cam: Camera, rows: np.ndarray, cols: np.ndarray):
    """Origins and unit directions (m, 3) of the rays through pixel centres."""
    F, R, V = camera_frame(cam)
    W, H = float(cam.width), float(cam.height)
    c = cols.astype(np.float64)
    r = rows.astype(np.float64)
    o = np.empty((len(r), 3))
    d = np.empty((len(r), 3))
    if cam.kind == "ortho":
        a = (2.0 * (c + 0.5) / W - 1.0) * cam.ortho_half_w
        b = (1.0 - 2.0 * (r + 0.5) / H) * cam.ortho_half_h
        for k in range(3):
            o[:, k] = cam.eye[k] + a * R[k] + b * V[k]
            d[:, k] = F[k]
    elif cam.kind == "persp":
        half = cam.fov_y_deg * (math.pi / 180.0) * 0.5
        tau = math.tan(half)
        aspect = W / H
        a = (2.0 * (c + 0.5) / W - 1.0) * tau * aspect
        b = (1.0 - 2.0 * (r + 0.5) / H) * tau
        dx = F[0] + a * R[0] + b * V[0]
        dy = F[1] + a * R[1] + b * V[1]
        dz = F[2] + a * R[2] + b * V[2]
        ln = np.sqrt(dx * dx + dy * dy + dz * dz)
        d[:, 0], d[:, 1], d[:, 2] = dx / ln, dy / ln, dz / ln
        for k in range(3):
            o[:, k] = cam.eye[k]
    else:
        raise ValueError(f"unknown camera kind {cam.kind!r}")
    return o, d


def slab(o: np.ndarray, d: np.ndarray, lo, hi):
    """Entry/exit ray parameters with the box [lo, hi] (t_enter >= 0).

    Returns ``t_enter, t_exit, hit``.  An axis with zero direction component
    constrains nothing when the origin lies within the slab and makes the
    ray miss otherwise.
    """
    m = len(o)
    t0 = np.zeros(m)
    t1 = np.full(m, np.inf)
    miss = np.zeros(m, dtype=bool)
    for k in range(3):
        dk = d[:, k]
        ok = o[:, k]
        nz = dk != 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (lo[k] - ok) / dk
            tb = (hi[k] - ok) / dk
        tn = np.where(nz, np.minimum(ta, tb), -np.inf)
        tf = np.where(nz, np.maximum(ta, tb), np.inf)
        miss |= (~nz) & ((ok < lo[k]) | (ok > hi[k]))
        t0 = np.maximum(t0, tn)
        t1 = np.minimum(t1, tf)
    hit = (~miss) & (t1 > t0)
    return t0, t1, hit


def sample_counts(t_enter, t_exit, hit, step: float) -> np.ndarray:
    """Number of samples ``floor((t_exit - t_enter) / step)`` (0 on a miss)."""
    n = np.zeros(len(t_enter), dtype=np.int64)
    L = (t_exit[hit] - t_enter[hit]) / step
    n[hit] = np.floor(L).astype(np.int64)
    return n


# ---------------------------------------------------------------------------
# shading pieces
# ---------------------------------------------------------------------------

def tf_lookup(tf: TransferFunction, v: np.ndarray) -> np.ndarray:
    """RGBA by linear interpolation of the table over [v_lo, v_hi]."""
    T = np.asarray(tf.table, dtype=np.float64)
    n = len(T)
    x = (v - tf.v_lo) / (tf.v_hi - tf.v_lo)
    x = np.clip(x, 0.0, 1.0) * (n - 1)
    i = np.minimum(np.floor(x).astype(np.int64), n - 2)
    t = (x - i)[:, None]
    return T[i] + t * (T[i + 1] - T[i])


def principal_curvatures(g: np.ndarray, h: np.ndarray):
    """(k1, k2), k1 >= k2, of the isosurfaces at points with world gradient
    ``g`` (m, 3) and world Hessian ``h`` (m, 6: xx yy zz xy xz yz)."""
    m = len(g)
    H = np.zeros((m, 3, 3))
    for c, (a, b) in enumerate(HESS_PAIRS):
        H[:, a, b] = h[:, c]
        H[:, b, a] = h[:, c]
    g2 = (g * g).sum(axis=1)
    ok = g2 >= 1e-12
    glen = np.sqrt(np.where(ok, g2, 1.0))
    n = g / glen[:, None]
    P = np.eye(3)[None, :, :] - n[:, :, None] * n[:, None, :]
    G = P @ H @ P / glen[:, None, None]
    T = np.trace(G, axis1=1, axis2=2)
    D = G - 0.5 * T[:, None, None] * P
    disc = np.sqrt(2.0 * (D * D).sum(axis=(1, 2)))
    k1 = np.where(ok, 0.5 * (T + disc), 0.0)
    k2 = np.where(ok, 0.5 * (T - disc), 0.0)
    return k1, k2


def curvature_lookup(ctf: CurvatureTF, k1: np.ndarray, k2: np.ndarray) -> np.ndarray:
    """RGBA by bilinear interpolation of the table over [k_lo, k_hi]^2."""
    T = np.asarray(ctf.table, dtype=np.float64)
    m = T.shape[0]

    def coord(k):
        x = np.clip((k - ctf.k_lo) / (ctf.k_hi - ctf.k_lo), 0.0, 1.0) * (m - 1)
        i = np.minimum(np.floor(x).astype(np.int64), m - 2)
        return i, (x - i)[:, None]

    i1, t1 = coord(k1)
    i2, t2 = coord(k2)
    low = T[i2, i1] + t1 * (T[i2, i1 + 1] - T[i2, i1])
    high = T[i2 + 1, i1] + t1 * (T[i2 + 1, i1 + 1] - T[i2 + 1, i1])
    return low + t2 * (high - low)


def ipow(x: np.ndarray, k: int) -> np.ndarray:
    """x**k for an integer k >= 0 by plain repeated multiplication."""
    out = np.ones_like(x)
    for _ in range(k):
        out = out * x
    return out


def phong(rgb: np.ndarray, g: np.ndarray, light: np.ndarray, view: np.ndarray,
          prm: RenderParams) -> np.ndarray:
    """Shaded colour from the gradient ``g`` (m,3), light and view (m,3)."""
    glen = np.sqrt((g * g).sum(axis=1))
    nrm = g / np.maximum(glen, GRAD_EPS)[:, None]
    ndl = (nrm * light).sum(axis=1)
    diff = np.abs(ndl)
    refl = 2.0 * ndl[:, None] * nrm - light
    rv = (refl * view).sum(axis=1)
    spec = ipow(np.maximum(rv, 0.0), prm.shininess)
    out = (prm.ka + prm.kd * diff)[:, None] * rgb + (prm.ks * spec)[:, None]
    return np.minimum(out, 1.0)


# ---------------------------------------------------------------------------
# rendering
# ---------------------------------------------------------------------------

@dataclass
class RenderResult:
    rgba: np.ndarray        # (m, 4) premultiplied
    samples: np.ndarray     # (m,) samples composited per ray
    n_nominal: np.ndarray   # (m,) samples per ray without termination
    near_threshold: np.ndarray  # (m,) min |A_s - O_max| over composited samples


def render_pixels(model: Model, cam: Camera, tf: TransferFunction, prm: RenderParams,
                  pix: np.ndarray, o_max: float | None = None,
                  chunk: int = 4096, field=None, curvature: CurvatureTF | None = None
                  ) -> RenderResult:
    """Render the pixels with flat indices ``pix`` (row-major, row 0 top).

    ``field``, if given, replaces the MFA by a closed-form field: a callable
    taking world points (k, 3) and returning the values (k,) and world
    gradients (k, 3); the model then only supplies the box.  Used to render
    the ground truth of the closed-form test fields.  ``curvature``, if
    given, colours each sample by the curvature table (non-rational models,
    no ``field``)."""
    pix = np.asarray(pix, dtype=np.int64)
    m = len(pix)
    rgba = np.zeros((m, 4))
    used = np.zeros(m, dtype=np.int64)
    nom = np.zeros(m, dtype=np.int64)
    near = np.full(m, np.inf)
    omax = prm.ert_alpha if o_max is None else o_max
    for c0 in range(0, m, chunk):
        sl = slice(c0, min(m, c0 + chunk))
        res = _render_chunk(model, cam, tf, prm, pix[sl], omax, field, curvature)
        rgba[sl], used[sl], nom[sl], near[sl] = res
    return RenderResult(rgba, used, nom, near)


def _render_chunk(model, cam, tf, prm, pix, omax, field=None, curvature=None):
    W = cam.width
    rows = pix // W
    cols = pix % W
    o, d = camera_rays(cam, rows, cols)
    lo = np.asarray(model.lo, dtype=np.float64)
    hi = np.asarray(model.hi, dtype=np.float64)
    t0, t1, hit = slab(o, d, lo, hi)
    nr = sample_counts(t0, t1, hit, prm.step)
    m = len(pix)
    C = np.zeros((m, 3))
    A = np.zeros(m)
    used = np.zeros(m, dtype=np.int64)
    near = np.full(m, np.inf)
    alive = nr > 0
    F, _, _ = camera_frame(cam)
    if prm.headlight:
        lvec = -np.asarray(F, dtype=np.float64)
    else:
        lvec = np.asarray(prm.light_dir, dtype=np.float64)
        lvec = lvec / math.sqrt(float((lvec * lvec).sum()))
    ext = hi - lo
    if curvature is not None:
        if field is not None or model.weights is not None:
            raise ValueError("curvature rendering: non-rational MFA models only")
        hmodels = hessian_models(model)
        hscale = np.array([1.0 / (ext[a] * ext[b]) for a, b in HESS_PAIRS])
    s = 0
    while alive.any():
        idx = np.nonzero(alive)[0]
        t = t0[idx] + (s + 0.5) * prm.step
        x = o[idx] + t[:, None] * d[idx]
        uvw = np.clip((x - lo) / ext, 0.0, 1.0)
        if field is None:
            f, df = eval_local(model, uvw)
            g = df / ext
        else:
            f, g = field(lo + uvw * ext)
        col = tf_lookup(tf, f)
        rgb, alpha = col[:, :3], col[:, 3]
        if curvature is not None:
            hw = hessian_from_models(hmodels, uvw) * hscale
            k1, k2 = principal_curvatures(g, hw)
            cc = curvature_lookup(curvature, k1, k2)
            rgb = cc[:, :3]
            alpha = alpha * cc[:, 3]
        if prm.shading:
            light = np.broadcast_to(lvec, g.shape)
            rgb = phong(rgb, g, light, -d[idx], prm)
        w = (1.0 - A[idx]) * alpha
        C[idx] += w[:, None] * rgb
        A[idx] += w
        used[idx] += 1
        near[idx] = np.minimum(near[idx], np.abs(A[idx] - omax))
        done = (s + 1 >= nr[idx]) | (A[idx] > omax)
        alive[idx[done]] = False
        s += 1
    rgba = np.concatenate([C, A[:, None]], axis=1)
    return rgba, used, nr, near


def render(model: Model, cam: Camera, tf: TransferFunction, prm: RenderParams,
           o_max: float | None = None) -> RenderResult:
    """Whole image; ``rgba`` has shape (H, W, 4)."""
    npx = cam.width * cam.height
    res = render_pixels(model, cam, tf, prm, np.arange(npx), o_max=o_max)
    res.rgba = res.rgba.reshape(cam.height, cam.width, 4)
    return res
