"""Tensor-product B-spline (MFA) evaluation in plain FP64 -- oracle, test only.

The MFA model (Sect. 2.3) represents a field by a tensor product of B-spline
bases: per axis a degree ``p`` and a clamped, non-decreasing knot vector
``U_0 .. U_{n+p}``, plus an ``n_x x n_y x n_z`` grid of control points.  The
paper's renderer queries the value and the first derivatives in all three
directions at arbitrary points of the normalised domain (Sect. 3.1,
Algorithm 1: value query and gradient query; the three derivatives are
obtained together).  The paper names rational B-splines but states no
weights and uses non-rational models in its experiments: a model without
weights is non-rational; with weights ``w_ijk > 0`` the field is the
rational quotient ``f = sum N N N w P / sum N N N w`` and its gradient
follows from the quotient rule.

Definitions used (textbook B-splines; Cox--de Boor, de Boor):

* span of ``u``: the largest ``s`` in ``[p, n-1]`` with ``U_s <= u``; at the
  right end ``u = U_n`` the last span ``n-1`` is used (spans are closed on
  the left, the last one also on the right);
* ``N_{i,0}(u) = 1`` on ``[U_i, U_{i+1})`` (and on the closed last non-empty
  span), else 0;
* ``N_{i,q} = (u-U_i)/(U_{i+q}-U_i) N_{i,q-1}
  + (U_{i+q+1}-u)/(U_{i+q+1}-U_{i+1}) N_{i+1,q-1}``, a term with a zero
  denominator being 0;
* ``N'_{i,p} = p/(U_{i+p}-U_i) N_{i,p-1} - p/(U_{i+p+1}-U_{i+1}) N_{i+1,p-1}``;
* value ``f(u,v,w) = sum_{ijk} N_i(u) N_j(v) N_k(w) P_{ijk}``, and each
  partial derivative is the same sum with one factor differentiated;
* rational: numerator ``A = sum N N N w P`` and denominator
  ``D = sum N N N w`` as above, ``f = A / D``, ``grad f = (grad A - f grad D) / D``.

Control points are stored x-fastest: ``ctrl[k, j, i] = P_{ijk}``.

Two evaluators are provided: ``eval_full`` sums over every control point
with the literal recursion (brute force, tiny models only), ``eval_local``
uses the span and the ``p+1`` non-zero functions per axis (local support
makes the two equal).  ``grad_hodograph`` differentiates through derivative
control points, an algebraically different route to the same gradient.
Second derivatives: ``hessian_full`` (literal recursion, brute force) and
``hessian_hodograph`` (derivative control points applied twice).
"""

from __future__ import annotations

from dataclasses import dataclass
from math import comb

import numpy as np


@dataclass
class Model:
    """A tensor-product B-spline volume over a box (rational when weights
    are given)."""

    degree: tuple            # (p_x, p_y, p_z)
    knots: tuple             # three float64 arrays, len n_k + p_k + 1
    ctrl: np.ndarray         # float64, shape (n_z, n_y, n_x), x fastest
    lo: np.ndarray           # float64 (3,), domain box corner
    hi: np.ndarray           # float64 (3,)
    weights: np.ndarray | None = None   # float64 like ctrl, > 0; None: all 1

    @property
    def n(self):
        nz, ny, nx = self.ctrl.shape
        return (nx, ny, nz)


# ---------------------------------------------------------------------------
# knot-span search
# ---------------------------------------------------------------------------

def find_span(n: int, p: int, U, u: float) -> int:
    """Span index of scalar ``u`` by bisection over ``[p, n]``.

    Returns the largest ``s`` in ``[p, n-1]`` with ``U[s] <= u``; ``u`` at or
    beyond ``U[n]`` gives ``n-1``.
    """
    if u >= U[n]:
        return n - 1
    if u < U[p]:
        return p
    lo, hi = p, n          # invariant: U[lo] <= u < U[hi]
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if U[mid] <= u:
            lo = mid
        else:
            hi = mid
    return lo


def find_span_vec(n: int, p: int, U: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Vectorised span search (sorted search on the knot vector)."""
    s = np.searchsorted(U, u, side="right") - 1
    return np.clip(s, p, n - 1)


# ---------------------------------------------------------------------------
# basis functions: brute-force recursion over the whole knot vector
# ---------------------------------------------------------------------------

def _last_nonempty(U) -> int:
    """Index i of the last non-empty knot interval [U_i, U_{i+1})."""
    i = len(U) - 2
    while i > 0 and not (U[i] < U[i + 1]):
        i -= 1
    return i


def basis_full(i: int, q: int, U, u: float) -> float:
    """``N_{i,q}(u)`` by the literal Cox--de Boor recursion (scalar)."""
    if q == 0:
        if U[i] <= u < U[i + 1]:
            return 1.0
        # the last non-empty interval is closed on the right
        if u == U[-1] and i == _last_nonempty(U):
            return 1.0
        return 0.0
    acc = 0.0
    den1 = U[i + q] - U[i]
    if den1 != 0.0:
        acc += (u - U[i]) / den1 * basis_full(i, q - 1, U, u)
    den2 = U[i + q + 1] - U[i + 1]
    if den2 != 0.0:
        acc += (U[i + q + 1] - u) / den2 * basis_full(i + 1, q - 1, U, u)
    return acc


def dbasis_full(i: int, q: int, U, u: float) -> float:
    """``N'_{i,q}(u)`` by de Boor's derivative formula on the full recursion."""
    if q == 0:
        return 0.0
    acc = 0.0
    den1 = U[i + q] - U[i]
    if den1 != 0.0:
        acc += q / den1 * basis_full(i, q - 1, U, u)
    den2 = U[i + q + 1] - U[i + 1]
    if den2 != 0.0:
        acc -= q / den2 * basis_full(i + 1, q - 1, U, u)
    return acc


# ---------------------------------------------------------------------------
# basis functions: the p+1 functions that are non-zero on one span
# ---------------------------------------------------------------------------

def basis_local(s, u, p: int, U):
    """Values and first derivatives of ``N_{s-p..s, p}`` at ``u``.

    ``s`` and ``u`` may be scalars or equal-length arrays.  Returns two
    arrays of shape ``(..., p+1)``: entry ``r`` belongs to ``N_{s-p+r,p}``.
    The degree is raised one step at a time; at degree ``q`` the non-zero
    functions on span ``s`` are ``N_{s-q..s, q}`` and the two neighbours
    that fall outside (``N_{s-q,q-1}`` and ``N_{s+1,q-1}``) are zero.
    On a non-empty span none of the denominators used here vanish.
    """
    U = np.asarray(U, dtype=np.float64)
    s = np.asarray(s)
    u = np.asarray(u, dtype=np.float64)
    prev = [np.ones_like(u)]                 # degree 0: N_{s,0} = 1
    lower = prev                             # degree p-1 values, kept for N'
    for q in range(1, p + 1):
        cur = []
        for r in range(q + 1):
            i = s - q + r
            val = np.zeros_like(u)
            if r >= 1:                       # (u-U_i)/(U_{i+q}-U_i) N_{i,q-1}
                val = val + (u - U[i]) / (U[i + q] - U[i]) * prev[r - 1]
            if r <= q - 1:                   # (U_{i+q+1}-u)/(...) N_{i+1,q-1}
                val = val + (U[i + q + 1] - u) / (U[i + q + 1] - U[i + 1]) * prev[r]
            cur.append(val)
        if q == p:
            lower = prev
        prev = cur
    vals = np.stack(prev, axis=-1)
    ders = []
    for r in range(p + 1):
        i = s - p + r
        d = np.zeros_like(u)
        if p >= 1:
            if r >= 1:
                d = d + p / (U[i + p] - U[i]) * lower[r - 1]
            if r <= p - 1:
                d = d - p / (U[i + p + 1] - U[i + 1]) * lower[r]
        ders.append(d)
    return vals, np.stack(ders, axis=-1)


# ---------------------------------------------------------------------------
# volume evaluation
# ---------------------------------------------------------------------------

def _axis_basis(model: Model, axis: int, u: np.ndarray):
    p = model.degree[axis]
    U = np.asarray(model.knots[axis], dtype=np.float64)
    n = model.n[axis]
    s = find_span_vec(n, p, U, u)
    N, dN = basis_local(s, u, p, U)
    return s, N, dN


def eval_local(model: Model, uvw: np.ndarray):
    """Value and parametric gradient at points ``uvw`` (m, 3) in [0,1]^3.

    Returns ``f`` (m,) and ``df`` (m, 3) = (df/du, df/dv, df/dw).
    Only the ``(p_x+1)(p_y+1)(p_z+1)`` control points whose basis functions
    are non-zero at the point enter the sum; the weights are the plain
    products of the three axis bases.
    """
    uvw = np.atleast_2d(np.asarray(uvw, dtype=np.float64))
    sx, Nx, dNx = _axis_basis(model, 0, uvw[:, 0])
    sy, Ny, dNy = _axis_basis(model, 1, uvw[:, 1])
    sz, Nz, dNz = _axis_basis(model, 2, uvw[:, 2])
    px, py, pz = model.degree
    a = np.arange(px + 1)
    b = np.arange(py + 1)
    c = np.arange(pz + 1)
    ix = (sx - px)[:, None] + a[None, :]           # (m, px+1)
    iy = (sy - py)[:, None] + b[None, :]
    iz = (sz - pz)[:, None] + c[None, :]
    # block[m, c, b, a] = P[iz, iy, ix]
    sel = (iz[:, :, None, None], iy[:, None, :, None], ix[:, None, None, :])
    block = model.ctrl[sel]

    def contract(wx, wy, wz, blk):
        w = wz[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :]
        return (w * blk).sum(axis=(1, 2, 3))

    def value_and_grad(blk):
        return (contract(Nx, Ny, Nz, blk),
                np.stack([contract(dNx, Ny, Nz, blk), contract(Nx, dNy, Nz, blk),
                          contract(Nx, Ny, dNz, blk)], axis=-1))

    if model.weights is None:
        return value_and_grad(block)
    wblock = model.weights[sel]
    A, dA = value_and_grad(wblock * block)
    D, dD = value_and_grad(wblock)
    f = A / D
    return f, (dA - f[:, None] * dD) / D[:, None]


def eval_full(model: Model, uvw: np.ndarray):
    """Brute force: sum over every control point with the literal recursion.

    Scalar Python loops; only for models with a few hundred control points.
    """
    uvw = np.atleast_2d(np.asarray(uvw, dtype=np.float64))
    nx, ny, nz = model.n
    px, py, pz = model.degree
    Ux, Uy, Uz = (list(map(float, k)) for k in model.knots)
    out_f = np.zeros(len(uvw))
    out_g = np.zeros((len(uvw), 3))
    for m, (u, v, w) in enumerate(uvw):
        Bx = [basis_full(i, px, Ux, u) for i in range(nx)]
        By = [basis_full(j, py, Uy, v) for j in range(ny)]
        Bz = [basis_full(k, pz, Uz, w) for k in range(nz)]
        Dx = [dbasis_full(i, px, Ux, u) for i in range(nx)]
        Dy = [dbasis_full(j, py, Uy, v) for j in range(ny)]
        Dz = [dbasis_full(k, pz, Uz, w) for k in range(nz)]
        acc = np.zeros((2, 4))              # rows: numerator, denominator
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    w = 1.0 if model.weights is None else float(model.weights[k, j, i])
                    terms = (Bx[i] * By[j] * Bz[k], Dx[i] * By[j] * Bz[k],
                             Bx[i] * Dy[j] * Bz[k], Bx[i] * By[j] * Dz[k])
                    for r, t in enumerate(terms):
                        acc[0, r] += t * w * float(model.ctrl[k, j, i])
                        acc[1, r] += t * w
        if model.weights is None:
            out_f[m] = acc[0, 0]
            out_g[m] = acc[0, 1:]
        else:
            f = acc[0, 0] / acc[1, 0]
            out_f[m] = f
            out_g[m] = (acc[0, 1:] - f * acc[1, 1:]) / acc[1, 0]
    return out_f, out_g


def grad_hodograph(model: Model, uvw: np.ndarray) -> np.ndarray:
    """Parametric gradient through derivative control points.

    Along axis ``a`` the derivative of a degree-p spline is a degree p-1
    spline on the knot vector with its first and last knot removed, with
    control points ``Q_i = p (P_{i+1} - P_i) / (U_{i+p+1} - U_{i+1})``.
    """
    uvw = np.atleast_2d(np.asarray(uvw, dtype=np.float64))
    if model.weights is not None:
        raise ValueError("grad_hodograph: non-rational models only")
    out = np.zeros((len(uvw), 3))
    for axis in range(3):
        p = model.degree[axis]
        U = np.asarray(model.knots[axis], dtype=np.float64)
        n = model.n[axis]
        ctrl_ax = 2 - axis                      # numpy axis of this direction
        P = np.moveaxis(model.ctrl, ctrl_ax, 0)   # (n, ...)
        den = U[p + 1:p + n] - U[1:n]             # U_{i+p+1} - U_{i+1}, i=0..n-2
        Q = p * (P[1:] - P[:-1]) / den.reshape((-1,) + (1,) * (P.ndim - 1))
        Q = np.moveaxis(Q, 0, ctrl_ax)
        deg = list(model.degree)
        deg[axis] = p - 1
        knots = list(model.knots)
        knots[axis] = U[1:-1]
        dm = Model(tuple(deg), tuple(knots), Q, model.lo, model.hi)
        f, _ = eval_local(dm, uvw)
        out[:, axis] = f
    return out


# ---------------------------------------------------------------------------
# second derivatives (Hessian)
# ---------------------------------------------------------------------------
# The model has analytic derivatives of every order (Sect. 3.1 notes that
# the B-spline representation yields all derivatives together); second
# derivatives are what curvature-based transfer functions need.  The six
# components are ordered uu, vv, ww, uv, uw, vw.

HESS_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def d2basis_full(i: int, q: int, U, u: float) -> float:
    """``N''_{i,q}(u)``: de Boor's derivative formula applied to the first
    derivatives of the two degree q-1 functions."""
    if q <= 1:
        return 0.0
    acc = 0.0
    den1 = U[i + q] - U[i]
    if den1 != 0.0:
        acc += q / den1 * dbasis_full(i, q - 1, U, u)
    den2 = U[i + q + 1] - U[i + 1]
    if den2 != 0.0:
        acc -= q / den2 * dbasis_full(i + 1, q - 1, U, u)
    return acc


def hessian_full(model: Model, uvw: np.ndarray) -> np.ndarray:
    """Brute force parametric Hessian (m, 6): every control point, with each
    axis factor differentiated as often as the axis occurs in the pair.
    Scalar loops; tiny non-rational models only."""
    if model.weights is not None:
        raise ValueError("hessian_full: non-rational models only")
    uvw = np.atleast_2d(np.asarray(uvw, dtype=np.float64))
    nx, ny, nz = model.n
    deg = model.degree
    knots = [list(map(float, k)) for k in model.knots]
    fns = (basis_full, dbasis_full, d2basis_full)
    out = np.zeros((len(uvw), 6))
    for m, pt in enumerate(uvw):
        # B[axis][order][index]
        B = [[[fns[o](i, deg[ax], knots[ax], pt[ax]) for i in range(model.n[ax])]
              for o in range(3)] for ax in range(3)]
        for h, (a, b) in enumerate(HESS_PAIRS):
            order = [0, 0, 0]
            order[a] += 1
            order[b] += 1
            acc = 0.0
            for k in range(nz):
                for j in range(ny):
                    for i in range(nx):
                        acc += (B[0][order[0]][i] * B[1][order[1]][j] * B[2][order[2]][k]
                                * float(model.ctrl[k, j, i]))
            out[m, h] = acc
    return out


def derivative_model(model: Model, axis: int):
    """The derivative along ``axis`` as a B-spline model: degree p-1 on the
    knot vector without its first and last knot, with control points
    ``Q_i = p (P_{i+1} - P_i) / (U_{i+p+1} - U_{i+1})``.  A zero denominator
    belongs to a degree p-1 function that vanishes everywhere, so its
    ``Q_i`` is 0.  ``None`` when p = 0: the derivative is identically 0."""
    if model.weights is not None:
        raise ValueError("derivative_model: non-rational models only")
    p = model.degree[axis]
    if p == 0:
        return None
    U = np.asarray(model.knots[axis], dtype=np.float64)
    n = model.n[axis]
    ctrl_ax = 2 - axis                              # numpy axis of this direction
    P = np.moveaxis(model.ctrl, ctrl_ax, 0)          # (n, ...)
    den = U[p + 1:p + n] - U[1:n]                    # U_{i+p+1} - U_{i+1}, i = 0..n-2
    shape = (-1,) + (1,) * (P.ndim - 1)
    safe = np.where(den != 0.0, den, 1.0).reshape(shape)
    Q = np.where((den != 0.0).reshape(shape), p * (P[1:] - P[:-1]) / safe, 0.0)
    deg = list(model.degree)
    deg[axis] = p - 1
    knots = list(model.knots)
    knots[axis] = U[1:-1]
    return Model(tuple(deg), tuple(knots), np.moveaxis(Q, 0, ctrl_ax), model.lo, model.hi)


def hessian_models(model: Model) -> list:
    """The six second-derivative splines (pair order of ``HESS_PAIRS``):
    the model differentiated along a, then along b; ``None`` where the
    derivative is identically 0."""
    out = []
    for a, b in HESS_PAIRS:
        da = derivative_model(model, a)
        out.append(None if da is None else derivative_model(da, b))
    return out


def hessian_from_models(models: list, uvw: np.ndarray) -> np.ndarray:
    """Parametric Hessian (m, 6): the values of the six derivative splines."""
    uvw = np.atleast_2d(np.asarray(uvw, dtype=np.float64))
    out = np.zeros((len(uvw), 6))
    for h, dab in enumerate(models):
        if dab is not None:
            out[:, h], _ = eval_local(dab, uvw)
    return out


def hessian_hodograph(model: Model, uvw: np.ndarray) -> np.ndarray:
    """Parametric Hessian (m, 6) through derivative control points: for each
    pair (a, b) the model is differentiated along a, then along b, and the
    resulting spline's value is evaluated."""
    return hessian_from_models(hessian_models(model), uvw)


def eval_world_hessian(model: Model, xyz: np.ndarray):
    """Value, world gradient and world Hessian (m, 6) at world points: each
    parametric second derivative d2f/du_a du_b is divided by the two box
    extents (chain rule of the affine normalisation)."""
    f, g = eval_world(model, xyz)
    H = hessian_hodograph(model, to_param(model, xyz))
    ext = np.asarray(model.hi, dtype=np.float64) - np.asarray(model.lo, dtype=np.float64)
    scale = np.array([1.0 / (ext[a] * ext[b]) for a, b in HESS_PAIRS])
    return f, g, H * scale


def to_param(model: Model, xyz: np.ndarray) -> np.ndarray:
    """World coordinates -> parameters in [0,1]^3 (affine, then clamped)."""
    xyz = np.atleast_2d(np.asarray(xyz, dtype=np.float64))
    u = (xyz - model.lo) / (model.hi - model.lo)
    return np.clip(u, 0.0, 1.0)


def eval_world(model: Model, xyz: np.ndarray):
    """Value and world-space gradient at world points (chain rule of the
    affine normalisation to the unit cube)."""
    f, df = eval_local(model, to_param(model, xyz))
    return f, df / (model.hi - model.lo)


# ---------------------------------------------------------------------------
# helpers for pins
# ---------------------------------------------------------------------------

def marsden_coeffs(p: int, U, m: int) -> np.ndarray:
    """Control points that reproduce ``u**m`` exactly (m <= p):
    ``c_i = e_m(U_{i+1}, ..., U_{i+p}) / C(p, m)`` with ``e_m`` the
    elementary symmetric polynomial (Marsden's identity)."""
    U = np.asarray(U, dtype=np.float64)
    n = len(U) - p - 1
    out = np.empty(n)
    for i in range(n):
        xs = U[i + 1:i + p + 1]
        e = np.zeros(m + 1)
        e[0] = 1.0
        for x in xs:                      # expand prod (1 + x t)
            for k in range(m, 0, -1):
                e[k] += x * e[k - 1]
        out[i] = e[m] / comb(p, m)
    return out
