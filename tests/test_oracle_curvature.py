"""Pins of the oracle's curvature transfer function: principal curvatures
against closed forms (sphere, cylinder, saddle) and against an
eigen-decomposition of the geometry tensor, through the model's own Hessian
on a reproduced quadric, the bilinear table lookup against a bilinear
function it must reproduce exactly, and the render integration against a
plain render with the colour moved into the value table."""

import numpy as np
import pytest

from oracle import bspline as ob
from oracle import raycast as orc
from paper_2204_11762_amd import workloads as wl


def _sym6(H):
    return np.stack([H[:, a, b] for a, b in ob.HESS_PAIRS], axis=1)


def test_sphere_and_cylinder_closed_forms():
    rng = np.random.default_rng(41)
    c = np.array([0.4, 0.55, 0.5])
    p = rng.uniform(-1, 1, size=(200, 3))
    r = np.linalg.norm(p - c, axis=1)
    keep = r > 0.05
    p, r = p[keep], r[keep]
    # f = |x - c|^2: g = 2 (x - c), H = 2 I; isosurfaces are spheres around lower values
    g = 2.0 * (p - c)
    H = np.repeat(2.0 * np.eye(3)[None], len(p), axis=0)
    k1, k2 = orc.principal_curvatures(g, _sym6(H))
    np.testing.assert_allclose(k1, 1.0 / r, rtol=1e-12)
    np.testing.assert_allclose(k2, 1.0 / r, rtol=1e-12)
    # f = (x - cx)^2 + (y - cy)^2: cylinders about the z axis, curvatures 1/r and 0
    rc = np.linalg.norm((p - c)[:, :2], axis=1)
    ok = rc > 0.05
    g = 2.0 * (p - c) * np.array([1.0, 1.0, 0.0])
    H = np.repeat(np.diag([2.0, 2.0, 0.0])[None], len(p), axis=0)
    k1, k2 = orc.principal_curvatures(g[ok], _sym6(H[ok]))
    np.testing.assert_allclose(k1, 1.0 / rc[ok], rtol=1e-12)
    np.testing.assert_allclose(k2, 0.0, atol=1e-12)


def test_saddle_at_the_stationary_point_of_the_surface():
    # f = x^2 - y^2 + z at the origin: n = (0, 0, 1), curvatures +2 and -2
    g = np.array([[0.0, 0.0, 1.0]])
    H = np.diag([2.0, -2.0, 0.0])[None]
    k1, k2 = orc.principal_curvatures(g, _sym6(H))
    np.testing.assert_allclose([k1[0], k2[0]], [2.0, -2.0], atol=1e-14)


def test_formula_equals_eigenvalues_of_the_geometry_tensor():
    rng = np.random.default_rng(42)
    m = 500
    g = rng.standard_normal((m, 3))
    A = rng.standard_normal((m, 3, 3))
    H = A + np.transpose(A, (0, 2, 1))
    k1, k2 = orc.principal_curvatures(g, _sym6(H))
    for i in range(m):
        n = g[i] / np.linalg.norm(g[i])
        P = np.eye(3) - np.outer(n, n)
        G = P @ H[i] @ P / np.linalg.norm(g[i])
        w, V = np.linalg.eigh(G)
        # drop the eigenvalue whose eigenvector is the normal
        j = int(np.argmax(np.abs(V.T @ n)))
        rest = np.sort(np.delete(w, j))
        np.testing.assert_allclose([k1[i], k2[i]], rest[::-1], atol=1e-10 * max(1, abs(w).max()))


def test_vanishing_gradient_gives_zero():
    k1, k2 = orc.principal_curvatures(np.array([[1e-7, 0.0, 0.0]]),
                                      np.array([[5.0, 1.0, 2.0, 0.5, 0.1, 0.3]]))
    assert k1[0] == 0.0 and k2[0] == 0.0


def test_through_the_model_hessian_on_a_reproduced_sphere():
    """A degree-2 model reproducing |x - c|^2 exactly (Marsden): the oracle's
    gradient and Hessian give curvature 1/r at every point."""
    rng = np.random.default_rng(43)
    deg = (2, 3, 2)
    n = (7, 8, 6)
    knots = tuple(wl.clamped_beta_knots(n[k], deg[k], rng) for k in range(3))
    c = np.array([0.45, 0.5, 0.55])
    ctrl = np.zeros((n[2], n[1], n[0]))
    for ax in range(3):
        # (u - c)^2 = u^2 - 2 c u + c^2 on this axis, constants on the others
        q = (ob.marsden_coeffs(deg[ax], knots[ax], 2) - 2 * c[ax]
             * ob.marsden_coeffs(deg[ax], knots[ax], 1) + c[ax] ** 2)
        shape = [1, 1, 1]
        shape[2 - ax] = n[ax]
        ctrl = ctrl + q.reshape(shape)
    M = ob.Model(deg, knots, ctrl, np.zeros(3), np.ones(3))
    u = rng.random((300, 3))
    r = np.linalg.norm(u - c, axis=1)
    u, r = u[r > 0.05], r[r > 0.05]
    _, g = ob.eval_local(M, u)
    k1, k2 = orc.principal_curvatures(g, ob.hessian_hodograph(M, u))
    np.testing.assert_allclose(k1, 1.0 / r, rtol=1e-9)
    np.testing.assert_allclose(k2, 1.0 / r, rtol=1e-9)


def test_bilinear_lookup_reproduces_bilinear_tables():
    m = 9
    i2, i1 = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    table = np.stack([i1, i2, i1 * i2, 0.5 + 0 * i1], axis=-1).astype(np.float64)
    ctf = orc.CurvatureTF(table, -2.0, 6.0)
    rng = np.random.default_rng(44)
    k1 = rng.uniform(-3, 7, 400)
    k2 = rng.uniform(-3, 7, 400)
    out = orc.curvature_lookup(ctf, k1, k2)
    x1 = np.clip((k1 + 2.0) / 8.0, 0, 1) * (m - 1)
    x2 = np.clip((k2 + 2.0) / 8.0, 0, 1) * (m - 1)
    np.testing.assert_allclose(out[:, 0], x1, atol=1e-12)
    np.testing.assert_allclose(out[:, 1], x2, atol=1e-12)
    np.testing.assert_allclose(out[:, 2], x1 * x2, atol=1e-11)
    np.testing.assert_allclose(out[:, 3], 0.5, atol=1e-15)
    # the upper corner is reached exactly
    top = orc.curvature_lookup(ctf, np.array([6.0]), np.array([100.0]))
    np.testing.assert_allclose(top[0], table[m - 1, m - 1], atol=1e-12)


@pytest.mark.parametrize("shading", [False, True])
def test_constant_curvature_table_equals_recoloured_value_table(shading):
    """A constant curvature table (colour q, opacity s) renders as a plain
    render whose value table has colour q and opacity s times its own."""
    wk = wl.c1()
    M = ob.Model(wk.model.degree, tuple(wk.model.knots), np.asarray(wk.model.ctrl, float),
                 np.zeros(3), np.ones(3))
    cam = orc.Camera(wk.camera.kind, wk.camera.eye, wk.camera.target, wk.camera.up, 24, 24,
                     wk.camera.fov_y_deg, wk.camera.ortho_half_w, wk.camera.ortho_half_h)
    T = np.asarray(wk.tf.table, dtype=np.float64)
    tf = orc.TransferFunction(T, wk.tf.v_lo, wk.tf.v_hi)
    prm = orc.RenderParams(step=wk.params.step, shading=shading)
    q = np.array([0.2, 0.7, 0.4, 0.8])
    ctf = orc.CurvatureTF(np.tile(q, (4, 4, 1)), -1.0, 1.0)
    pix = np.arange(24 * 24)
    a = orc.render_pixels(M, cam, tf, prm, pix, curvature=ctf)
    T2 = T.copy()
    T2[:, :3] = q[:3]
    T2[:, 3] = T[:, 3] * q[3]
    b = orc.render_pixels(M, cam, orc.TransferFunction(T2, wk.tf.v_lo, wk.tf.v_hi), prm, pix)
    np.testing.assert_allclose(a.rgba, b.rgba, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(a.samples, b.samples)
