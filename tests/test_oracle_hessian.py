"""Pins of the oracle's second derivatives (Hessian) against facts outside
it: closed forms through Marsden's identity (monomials are reproduced, so
their second derivatives are known exactly), scipy's NdBSpline derivatives,
central differences of the oracle's own gradient, the symmetry of mixed
derivatives (taken in both orders), the brute-force literal recursion, and
the chain rule of the world normalisation."""

import numpy as np
import pytest
from scipy.interpolate import NdBSpline

from oracle import bspline as ob
from paper_2204_11762_amd import workloads as wl


def _knots(n, p, kind, rng):
    if kind == "uniform":
        return wl.clamped_uniform_knots(n, p)
    if kind == "beta":
        return wl.clamped_beta_knots(n, p, rng)
    # a repeated interior knot of multiplicity p - 1 (still C^1, so second
    # derivatives exist on both sides and jump only at the knot)
    m = max(p - 1, 1)
    inner = [0.35] * m + list(np.linspace(0.5, 0.9, n - p - 1 - m))
    U = np.array([0.0] * (p + 1) + inner + [1.0] * (p + 1))
    assert len(U) == n + p + 1
    return U


def _model(rng, degree, kind="beta", extra=(4, 5, 3), lo=(0, 0, 0), hi=(1, 1, 1)):
    n = tuple(degree[k] + extra[k] + (2 if kind == "repeated" else 0) for k in range(3))
    knots = tuple(_knots(n[k], degree[k], kind, rng) for k in range(3))
    ctrl = rng.standard_normal((n[2], n[1], n[0]))
    return ob.Model(tuple(degree), knots, ctrl, np.asarray(lo, float), np.asarray(hi, float))


def _monomial_hessian(uvw, e):
    """Exact parametric Hessian of u^a v^b w^c, components uu vv ww uv uw vw."""
    u, v, w = uvw.T
    x = (u, v, w)

    def term(order):
        out = np.ones(len(uvw))
        for ax in range(3):
            k, d = e[ax], order[ax]
            coef = 1.0
            for j in range(d):
                coef *= (k - j)
            out = out * (coef * x[ax] ** max(k - d, 0) if k >= d else 0.0)
        return out

    cols = []
    for a, b in ob.HESS_PAIRS:
        order = [0, 0, 0]
        order[a] += 1
        order[b] += 1
        cols.append(term(order))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("degree", [(2, 2, 2), (3, 2, 4), (4, 3, 1), (1, 3, 2)])
@pytest.mark.parametrize("kind", ["uniform", "beta", "repeated"])
def test_monomials_closed_form(degree, kind):
    """Every monomial u^a v^b w^c with a <= p_x, ... is reproduced exactly
    (Marsden), so its Hessian is the textbook one, on any clamped knots."""
    rng = np.random.default_rng(31)
    M0 = _model(rng, degree, kind)
    uvw = rng.random((250, 3))
    for a in range(degree[0] + 1):
        for b in range(degree[1] + 1):
            for c in range(degree[2] + 1):
                cx = ob.marsden_coeffs(degree[0], M0.knots[0], a)
                cy = ob.marsden_coeffs(degree[1], M0.knots[1], b)
                cz = ob.marsden_coeffs(degree[2], M0.knots[2], c)
                ctrl = cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
                M = ob.Model(M0.degree, M0.knots, ctrl, M0.lo, M0.hi)
                H = ob.hessian_hodograph(M, uvw)
                np.testing.assert_allclose(H, _monomial_hessian(uvw, (a, b, c)), rtol=0,
                                           atol=1e-10)


@pytest.mark.parametrize("degree", [(2, 3, 4), (3, 3, 3), (4, 1, 2), (1, 1, 1)])
def test_matches_scipy_ndbspline_second_derivatives(degree):
    rng = np.random.default_rng(32)
    M = _model(rng, degree, "beta", extra=(5, 4, 6))
    nd = NdBSpline(M.knots, np.transpose(M.ctrl, (2, 1, 0)), degree)
    uvw = rng.random((300, 3))
    H = ob.hessian_hodograph(M, uvw)
    for h, (a, b) in enumerate(ob.HESS_PAIRS):
        nu = [0, 0, 0]
        nu[a] += 1
        nu[b] += 1
        ref = nd(uvw, nu=tuple(nu))
        np.testing.assert_allclose(H[:, h], ref, rtol=0,
                                   atol=1e-10 * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("degree", [(2, 2, 2), (3, 3, 3), (4, 2, 3)])
def test_central_differences_of_gradient(degree):
    rng = np.random.default_rng(33)
    M = _model(rng, degree, "beta", extra=(6, 6, 6))
    h = 1e-6
    pts = rng.uniform(0.05, 0.95, size=(300, 3))
    ok = np.ones(len(pts), dtype=bool)
    for ax in range(3):
        d = np.abs(pts[:, ax][:, None] - np.unique(M.knots[ax])[None, :]).min(axis=1)
        ok &= d > 2 * h
    pts = pts[ok]
    H = ob.hessian_hodograph(M, pts)
    scale = np.abs(H).max()
    for hh, (a, b) in enumerate(ob.HESS_PAIRS):
        e = np.zeros(3)
        e[b] = h
        _, gp = ob.eval_local(M, pts + e)
        _, gm = ob.eval_local(M, pts - e)
        fd = (gp[:, a] - gm[:, a]) / (2 * h)
        np.testing.assert_allclose(H[:, hh], fd, rtol=0, atol=1e-6 * scale)


def test_mixed_derivatives_in_both_orders():
    """d/dv(d/du f) through the derivative models equals d/du(d/dv f)."""
    rng = np.random.default_rng(34)
    M = _model(rng, (3, 4, 2), "beta")
    uvw = rng.random((400, 3))
    H = ob.hessian_hodograph(M, uvw)
    for h, (a, b) in enumerate(ob.HESS_PAIRS):
        if a == b:
            continue
        swapped, _ = ob.eval_local(ob.derivative_model(ob.derivative_model(M, b), a), uvw)
        np.testing.assert_allclose(H[:, h], swapped, rtol=0, atol=1e-10 * np.abs(H).max())


@pytest.mark.parametrize("degree", [(1, 2, 3), (3, 3, 3), (2, 1, 4)])
@pytest.mark.parametrize("kind", ["beta", "repeated"])
def test_brute_force_equals_hodograph(degree, kind):
    rng = np.random.default_rng(35)
    M = _model(rng, degree, kind, extra=(2, 1, 2))
    uvw = rng.random((12, 3))
    Hf = ob.hessian_full(M, uvw)
    Hh = ob.hessian_hodograph(M, uvw)
    np.testing.assert_allclose(Hh, Hf, rtol=0, atol=1e-10 * max(1.0, np.abs(Hf).max()))


def test_degree_one_axes_have_no_second_derivative():
    rng = np.random.default_rng(36)
    M = _model(rng, (1, 3, 1), "beta")
    H = ob.hessian_hodograph(M, rng.random((100, 3)))
    assert np.all(H[:, 0] == 0.0) and np.all(H[:, 2] == 0.0)      # uu, ww
    # mixed derivatives of linear axes need not vanish (u w has d2/du dw = 1)
    assert np.abs(H[:, 1]).max() > 0 and np.abs(H[:, 4]).max() > 0


def test_world_hessian_chain_rule():
    """World second derivatives against central differences of the world
    gradient on a non-unit box."""
    rng = np.random.default_rng(37)
    lo, hi = (-1.0, 0.5, 2.0), (1.0, 3.0, 2.5)
    M = _model(rng, (3, 2, 4), "uniform", lo=lo, hi=hi)
    lo, hi = np.asarray(lo), np.asarray(hi)
    xyz = lo + (hi - lo) * rng.uniform(0.05, 0.95, size=(200, 3))
    f, g, H = ob.eval_world_hessian(M, xyz)
    f2, g2 = ob.eval_world(M, xyz)
    np.testing.assert_array_equal(f, f2)
    np.testing.assert_array_equal(g, g2)
    h = 1e-6
    for hh, (a, b) in enumerate(ob.HESS_PAIRS):
        e = np.zeros(3)
        e[b] = h * (hi[b] - lo[b])
        _, gp = ob.eval_world(M, xyz + e)
        _, gm = ob.eval_world(M, xyz - e)
        fd = (gp[:, a] - gm[:, a]) / (2 * e[b])
        np.testing.assert_allclose(H[:, hh], fd, rtol=0, atol=2e-5 * np.abs(H[:, hh]).max())


def test_rational_models_are_refused():
    rng = np.random.default_rng(38)
    M = _model(rng, (2, 2, 2), "uniform")
    R = ob.Model(M.degree, M.knots, M.ctrl, M.lo, M.hi, weights=np.ones_like(M.ctrl))
    with pytest.raises(ValueError):
        ob.hessian_hodograph(R, rng.random((3, 3)))
    with pytest.raises(ValueError):
        ob.hessian_full(R, rng.random((3, 3)))
