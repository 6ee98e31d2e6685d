"""Pins of the FP64 oracle's B-spline evaluation against facts that do not
depend on the oracle itself: closed forms (Bernstein, Marsden's identity),
brute force over the literal recursion, invariants (partition of unity,
convex hull), finite differences, and independent library routines
(scipy's BSpline / NdBSpline / RegularGridInterpolator)."""

from math import comb

import numpy as np
import pytest
from scipy.interpolate import BSpline, NdBSpline, RegularGridInterpolator

from oracle import bspline as ob
from oracle import quant
from paper_2204_11762_amd import workloads as wl


def _knot_cases():
    rng = np.random.default_rng(11)
    cases = []
    for p in (1, 2, 3, 4):
        for n in (p + 1, p + 2, 7, 10):
            cases.append((n, p, wl.clamped_uniform_knots(n, p)))
            if n > p + 1:
                cases.append((n, p, wl.clamped_beta_knots(n, p, rng)))
        # a repeated interior knot (multiplicity p, still C^0)
        n = 2 * p + 3
        inner = [0.3] * p + list(np.linspace(0.45, 0.9, n - p - 1 - p))
        U = np.array([0.0] * (p + 1) + inner + [1.0] * (p + 1))
        assert len(U) == n + p + 1
        cases.append((n, p, U))
    return cases


KNOT_CASES = _knot_cases()


def _sites(U, rng, k=40):
    """Random sites plus every knot, the ends and points next to knots."""
    u = list(rng.random(k))
    for x in np.unique(U):
        u += [x, min(1.0, x + 1e-9), max(0.0, x - 1e-9)]
    return np.array(sorted(set(u)))


@pytest.mark.parametrize("n,p,U", KNOT_CASES)
def test_find_span_definition(n, p, U):
    rng = np.random.default_rng(1)
    for u in _sites(U, rng):
        # the definition, by exhaustive scan
        cand = [s for s in range(p, n) if U[s] <= u]
        want = max(cand)
        assert ob.find_span(n, p, U, u) == want
        assert ob.find_span_vec(n, p, U, np.array([u]))[0] == want
        s = want
        assert U[s] < U[s + 1], "a located span must be non-empty"


@pytest.mark.parametrize("n,p,U", KNOT_CASES)
def test_partition_of_unity_and_derivative_sum(n, p, U):
    rng = np.random.default_rng(2)
    u = _sites(U, rng)
    s = ob.find_span_vec(n, p, U, u)
    N, dN = ob.basis_local(s, u, p, U)
    np.testing.assert_allclose(N.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    scale = np.abs(dN).sum(axis=1).max()
    np.testing.assert_allclose(dN.sum(axis=1), 0.0, rtol=0, atol=1e-14 * max(1.0, scale))
    assert (N >= -1e-15).all()


@pytest.mark.parametrize("n,p,U", [c for c in KNOT_CASES if c[0] <= 10])
def test_local_triangle_equals_full_recursion(n, p, U):
    rng = np.random.default_rng(3)
    Ul = list(map(float, U))
    for u in _sites(U, rng, k=15):
        s = ob.find_span(n, p, U, u)
        N, dN = ob.basis_local(s, np.array([u]), p, U)
        full = np.array([ob.basis_full(i, p, Ul, u) for i in range(n)])
        dfull = np.array([ob.dbasis_full(i, p, Ul, u) for i in range(n)])
        want = np.zeros(n)
        want[s - p:s + 1] = N[0]
        dwant = np.zeros(n)
        dwant[s - p:s + 1] = dN[0]
        np.testing.assert_allclose(full, want, rtol=0, atol=1e-14)
        # at a knot of multiplicity p the derivative jumps; the left-closed
        # span convention is then the one the full recursion also uses
        np.testing.assert_allclose(dfull, dwant, rtol=0, atol=1e-12 * max(1, np.abs(dwant).max()))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_bernstein_closed_form(p):
    n = p + 1
    U = wl.clamped_uniform_knots(n, p)
    u = np.linspace(0, 1, 101)
    s = ob.find_span_vec(n, p, U, u)
    assert (s == p).all()
    N, dN = ob.basis_local(s, u, p, U)
    for i in range(p + 1):
        B = comb(p, i) * u ** i * (1 - u) ** (p - i)
        np.testing.assert_allclose(N[:, i], B, rtol=0, atol=1e-14)
        # d/du B_{i,p} = p (B_{i-1,p-1} - B_{i,p-1})
        left = comb(p - 1, i - 1) * u ** (i - 1) * (1 - u) ** (p - i) if i >= 1 else 0 * u
        right = comb(p - 1, i) * u ** i * (1 - u) ** (p - 1 - i) if i <= p - 1 else 0 * u
        np.testing.assert_allclose(dN[:, i], p * (left - right), rtol=0, atol=1e-13)


@pytest.mark.parametrize("n,p,U", [c for c in KNOT_CASES if c[0] > c[1] + 1])
def test_basis_matches_scipy_design_matrix(n, p, U):
    rng = np.random.default_rng(4)
    u = rng.random(200)
    s = ob.find_span_vec(n, p, U, u)
    N, dN = ob.basis_local(s, u, p, U)
    D = BSpline.design_matrix(u, U, p).toarray()
    mine = np.zeros_like(D)
    dmine = np.zeros_like(D)
    for m in range(len(u)):
        mine[m, s[m] - p:s[m] + 1] = N[m]
        dmine[m, s[m] - p:s[m] + 1] = dN[m]
    np.testing.assert_allclose(mine, D, rtol=0, atol=1e-13)
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1.0
        der = BSpline(U, c, p).derivative()(u)
        np.testing.assert_allclose(dmine[:, i], der, rtol=0, atol=1e-11 * max(1, np.abs(der).max()))


def _rand_model(rng, n=(6, 5, 7), degree=(2, 3, 1), beta=True):
    return ob.Model(tuple(degree),
                    tuple((wl.clamped_beta_knots(n[k], degree[k], rng) if beta
                           else wl.clamped_uniform_knots(n[k], degree[k])) for k in range(3)),
                    rng.standard_normal((n[2], n[1], n[0])),
                    np.zeros(3), np.ones(3))


@pytest.mark.parametrize("degree", [(1, 1, 1), (2, 3, 1), (3, 3, 3), (4, 2, 3)])
def test_local_equals_brute_force_full_sum(degree):
    rng = np.random.default_rng(5)
    n = tuple(d + 3 for d in degree)
    M = _rand_model(rng, n=(n[0], n[1] + 1, n[2] + 2), degree=degree)
    uvw = rng.random((25, 3))
    uvw[0] = (0, 0, 0)
    uvw[1] = (1, 1, 1)
    uvw[2] = (1, 0, 0.5)
    f, g = ob.eval_local(M, uvw)
    F, G = ob.eval_full(M, uvw)
    np.testing.assert_allclose(f, F, rtol=0, atol=1e-14 * np.abs(M.ctrl).max() * 4)
    np.testing.assert_allclose(g, G, rtol=0, atol=1e-12 * max(1, np.abs(G).max()))


@pytest.mark.parametrize("degree", [(1, 2, 3), (2, 2, 2), (3, 3, 3), (4, 3, 2)])
@pytest.mark.parametrize("beta", [False, True])
def test_polynomial_reproduction(degree, beta):
    """Marsden's identity: u^a v^b w^c (a<=p_x, ...) is reproduced exactly,
    value and gradient."""
    rng = np.random.default_rng(6)
    n = (degree[0] + 4, degree[1] + 5, degree[2] + 3)
    knots = tuple((wl.clamped_beta_knots(n[k], degree[k], rng) if beta
                   else wl.clamped_uniform_knots(n[k], degree[k])) for k in range(3))
    uvw = rng.random((300, 3))
    for a in range(degree[0] + 1):
        for b in range(degree[1] + 1):
            for c in range(degree[2] + 1):
                cx = ob.marsden_coeffs(degree[0], knots[0], a)
                cy = ob.marsden_coeffs(degree[1], knots[1], b)
                cz = ob.marsden_coeffs(degree[2], knots[2], c)
                ctrl = cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
                M = ob.Model(degree, knots, ctrl, np.zeros(3), np.ones(3))
                f, g = ob.eval_local(M, uvw)
                u, v, w = uvw.T
                np.testing.assert_allclose(f, u ** a * v ** b * w ** c, rtol=0, atol=1e-13)
                gu = a * u ** max(a - 1, 0) * v ** b * w ** c
                gv = b * u ** a * v ** max(b - 1, 0) * w ** c
                gw = c * u ** a * v ** b * w ** max(c - 1, 0)
                np.testing.assert_allclose(g, np.stack([gu, gv, gw], 1), rtol=0, atol=1e-12)


@pytest.mark.parametrize("degree", [(1, 2, 3), (3, 3, 3), (4, 1, 2)])
def test_matches_scipy_ndbspline(degree):
    rng = np.random.default_rng(7)
    M = _rand_model(rng, n=(degree[0] + 5, degree[1] + 4, degree[2] + 6), degree=degree)
    # NdBSpline indexes coefficients as c[i, j, k] with t = (U^x, U^y, U^z)
    nd = NdBSpline(M.knots, np.transpose(M.ctrl, (2, 1, 0)), degree)
    uvw = rng.random((200, 3))
    f, g = ob.eval_local(M, uvw)
    np.testing.assert_allclose(f, nd(uvw), rtol=0, atol=1e-12)
    for ax in range(3):
        nu = [0, 0, 0]
        nu[ax] = 1
        ref = nd(uvw, nu=tuple(nu))
        np.testing.assert_allclose(g[:, ax], ref, rtol=0, atol=1e-11 * max(1, np.abs(ref).max()))


def test_degree_one_is_trilinear():
    rng = np.random.default_rng(8)
    n = (7, 5, 6)
    M = _rand_model(rng, n=n, degree=(1, 1, 1), beta=False)
    grids = tuple(np.arange(n[k]) / (n[k] - 1) for k in range(3))
    rgi = RegularGridInterpolator(grids, np.transpose(M.ctrl, (2, 1, 0)), method="linear")
    uvw = rng.random((500, 3))
    f, _ = ob.eval_local(M, uvw)
    np.testing.assert_allclose(f, rgi(uvw), rtol=0, atol=1e-13)


@pytest.mark.parametrize("degree", [(2, 2, 2), (3, 3, 3), (4, 2, 3)])
def test_gradient_central_differences(degree):
    rng = np.random.default_rng(9)
    M = _rand_model(rng, n=(degree[0] + 6, degree[1] + 6, degree[2] + 6), degree=degree)
    h = 1e-6
    pts = rng.uniform(0.05, 0.95, size=(200, 3))
    # keep the stencil away from knots so that one polynomial piece is used
    ok = np.ones(len(pts), dtype=bool)
    for ax in range(3):
        d = np.abs(pts[:, ax][:, None] - np.unique(M.knots[ax])[None, :]).min(axis=1)
        ok &= d > 2 * h
    pts = pts[ok]
    _, g = ob.eval_local(M, pts)
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        fp, _ = ob.eval_local(M, pts + e)
        fm, _ = ob.eval_local(M, pts - e)
        fd = (fp - fm) / (2 * h)
        np.testing.assert_allclose(g[:, ax], fd, rtol=1e-7, atol=1e-7 * np.abs(g).max())


@pytest.mark.parametrize("degree", [(1, 1, 1), (2, 3, 4), (3, 3, 3)])
def test_hodograph_gradient_equals_direct(degree):
    rng = np.random.default_rng(10)
    M = _rand_model(rng, n=(degree[0] + 5, degree[1] + 3, degree[2] + 4), degree=degree)
    uvw = rng.random((300, 3))
    _, g = ob.eval_local(M, uvw)
    gh = ob.grad_hodograph(M, uvw)
    np.testing.assert_allclose(g, gh, rtol=0, atol=1e-12 * max(1, np.abs(g).max()))


def test_convex_hull():
    rng = np.random.default_rng(12)
    M = _rand_model(rng, n=(9, 8, 7), degree=(3, 2, 4))
    f, _ = ob.eval_local(M, rng.random((2000, 3)))
    assert f.min() >= M.ctrl.min() - 1e-14
    assert f.max() <= M.ctrl.max() + 1e-14


def test_world_gradient_chain_rule():
    """A box [lo, hi] maps affinely to the unit cube: f_world(x) =
    f(u(x)) and grad_world = grad_u / (hi - lo) (checked by differences)."""
    rng = np.random.default_rng(13)
    M = _rand_model(rng, n=(8, 8, 8), degree=(3, 3, 3))
    M.lo = np.array([-1.0, 2.0, 0.5])
    M.hi = np.array([3.0, 2.5, 4.0])
    x = M.lo + rng.uniform(0.1, 0.9, size=(100, 3)) * (M.hi - M.lo)
    f, g = ob.eval_world(M, x)
    f0, _ = ob.eval_local(M, (x - M.lo) / (M.hi - M.lo))
    np.testing.assert_allclose(f, f0, rtol=0, atol=1e-14)
    h = 1e-6
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h * (M.hi[ax] - M.lo[ax])
        fd = (ob.eval_world(M, x + e)[0] - ob.eval_world(M, x - e)[0]) / (2 * e[ax])
        np.testing.assert_allclose(g[:, ax], fd, rtol=1e-6, atol=1e-6 * np.abs(g[:, ax]).max())
    # outside points clamp to the box
    fo, _ = ob.eval_world(M, np.array([[M.hi[0] + 5, M.lo[1] - 1, M.lo[2]]]))
    fc, _ = ob.eval_local(M, np.array([[1.0, 0.0, 0.0]]))
    assert fo[0] == fc[0]


def test_bf16_rounding_known_values_and_torch():
    import torch
    one = 1.0
    cases = {
        one: one,
        one + 2.0 ** -8: one,                       # tie -> even
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,       # tie -> even (upwards)
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,
        -2.5: -2.5,
        0.0: 0.0,
    }
    x = np.array(list(cases.keys()))
    np.testing.assert_array_equal(quant.dequant_bf16(x), np.array(list(cases.values())))
    rng = np.random.default_rng(14)
    y = rng.standard_normal(100000) * 3
    ref = torch.from_numpy(y.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(quant.dequant_bf16(y), ref)
    np.testing.assert_array_equal(quant.dequant_f32(y), y.astype(np.float32).astype(np.float64))


def test_f16_rounding_known_values_and_libraries():
    import torch
    one = 1.0
    cases = {
        one: one,
        one + 2.0 ** -11: one,                      # tie -> even
        one + 3 * 2.0 ** -11: one + 2.0 ** -9,      # tie -> even (upwards)
        one + 2.0 ** -11 + 2.0 ** -20: one + 2.0 ** -10,
        65504.0: 65504.0,                           # largest finite
        2.0 ** -14: 2.0 ** -14,                     # smallest normal
        2.0 ** -24: 2.0 ** -24,                     # smallest subnormal
        2.0 ** -25: 0.0,                            # tie -> even (zero)
        3 * 2.0 ** -26: 2.0 ** -24,
        -2.5: -2.5,
        0.0: 0.0,
        1.0 / 3.0: 0.333251953125,                  # 0x3555
    }
    x = np.array(list(cases.keys()))
    np.testing.assert_array_equal(quant.dequant_f16(x), np.array(list(cases.values())))
    assert quant.f16_bits(np.array([1.0 / 3.0]))[0] == 0x3555
    assert quant.f16_bits(np.array([-65504.0]))[0] == 0xFBFF
    rng = np.random.default_rng(15)
    y = np.concatenate([rng.standard_normal(100000) * 3, rng.standard_normal(20000) * 1e-5,
                        rng.uniform(-65000, 65000, 1000)])
    f32 = y.astype(np.float32)
    np.testing.assert_array_equal(quant.dequant_f16(y), f32.astype(np.float16).astype(np.float64))
    ref = torch.from_numpy(f32).to(torch.float16).to(torch.float64).numpy()
    np.testing.assert_array_equal(quant.dequant_f16(y), ref)


def _golden_pieces():
    import os
    from fractions import Fraction
    path = os.path.join(os.path.dirname(__file__), "golden", "cardinal_pieces.txt")
    rows = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        p, t, i, n, dn = line.split()
        rows.append((int(p), float(Fraction(t)), int(i), float(Fraction(n)),
                     float(Fraction(dn))))
    return rows


def test_uniform_pieces_match_hand_derived_fixture():
    """Interior spans of uniform clamped knots carry the cardinal pieces:
    N at u = (j + t)/m and m dN/dt equal the exact rationals of the fixture,
    on every interior span of a long knot vector (m = 12)."""
    rows = _golden_pieces()
    assert len(rows) == 4 * (2 + 3 + 4)
    for p in (1, 2, 3):
        m = 12
        n = m + p
        U = wl.clamped_uniform_knots(n, p)
        for j in range(p, m - p):          # spans whose p+1 functions are all interior
            s = j + p
            for (q, t, i, nv, dv) in rows:
                if q != p:
                    continue
                u = (j + t) / m
                assert ob.find_span(n, p, U, u) == s
                N, dN = ob.basis_local(s, u, p, U)
                assert abs(N[i] - nv) <= 1e-14, (p, j, t, i)
                assert abs(dN[i] - m * dv) <= 1e-12, (p, j, t, i)


def _rational_reciprocal_model():
    """Degree 2 along x with weights (1, 1, 2) and values (1, 1, 1/2): the
    denominator is (1-u)^2 + 2u(1-u) + 2u^2 = 1 + u^2 and the numerator
    (1-u)^2 + 2u(1-u) + u^2 = 1, so f = 1 / (1 + u^2) exactly; constant in
    y and z (degree 1, two control points each)."""
    U2 = np.array([0, 0, 0, 1, 1, 1], float)
    U1 = np.array([0, 0, 1, 1], float)
    ctrl = np.empty((2, 2, 3))
    ctrl[:, :, :] = [1.0, 1.0, 0.5]
    w = np.empty((2, 2, 3))
    w[:, :, :] = [1.0, 1.0, 2.0]
    return ob.Model((2, 1, 1), (U2, U1, U1), ctrl, np.zeros(3), np.ones(3), weights=w)


def test_rational_reproduces_reciprocal_quadratic():
    M = _rational_reciprocal_model()
    rng = np.random.default_rng(21)
    uvw = rng.random((500, 3))
    uvw[:5, 0] = [0.0, 1.0, 0.5, 0.25, 1e-9]
    u = uvw[:, 0]
    f, g = ob.eval_local(M, uvw)
    np.testing.assert_allclose(f, 1.0 / (1.0 + u * u), rtol=0, atol=1e-15)
    np.testing.assert_allclose(g[:, 0], -2.0 * u / (1.0 + u * u) ** 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(g[:, 1:], 0.0, atol=1e-15)
    fb, gb = ob.eval_full(M, uvw[:40])
    np.testing.assert_allclose(fb, f[:40], atol=1e-15)
    np.testing.assert_allclose(gb, g[:40], atol=1e-14)


@pytest.mark.parametrize("degree", [(1, 2, 3), (3, 3, 3), (4, 2, 2)])
def test_rational_constant_weights_and_brute_force(degree):
    rng = np.random.default_rng(22)
    spec = wl.random_model(rng, n=(6, 7, 5), degree=degree, beta_knots=True)
    M0 = ob.Model(spec.degree, spec.knots, spec.ctrl, np.zeros(3), np.ones(3))
    Mc = ob.Model(spec.degree, spec.knots, spec.ctrl, np.zeros(3), np.ones(3),
                  weights=np.full(spec.ctrl.shape, 3.7))
    uvw = rng.random((60, 3))
    f0, g0 = ob.eval_local(M0, uvw)
    fc, gc = ob.eval_local(Mc, uvw)
    np.testing.assert_allclose(fc, f0, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(gc, g0, rtol=1e-13, atol=1e-13)
    Mw = ob.Model(spec.degree, spec.knots, spec.ctrl, np.zeros(3), np.ones(3),
                  weights=rng.uniform(0.2, 5.0, spec.ctrl.shape))
    fl, gl = ob.eval_local(Mw, uvw)
    fb, gb = ob.eval_full(Mw, uvw)
    np.testing.assert_allclose(fl, fb, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(gl, gb, rtol=1e-12, atol=1e-12)
    # the rational value is a convex combination of the control points
    assert (fl >= spec.ctrl.min() - 1e-12).all() and (fl <= spec.ctrl.max() + 1e-12).all()
    # central differences of the rational value
    h = 1e-6
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        inner = np.clip(uvw, 2 * h, 1 - 2 * h)
        fd = (ob.eval_local(Mw, inner + e)[0] - ob.eval_local(Mw, inner - e)[0]) / (2 * h)
        ga = ob.eval_local(Mw, inner)[1][:, ax]
        assert np.abs(fd - ga).max() <= 1e-6 * max(1.0, np.abs(ga).max())
