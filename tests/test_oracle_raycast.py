"""Pins of the FP64 oracle's ray caster: camera and slab closed forms,
transfer-function and Phong hand cases, and whole-image closed forms
(constant field, linear field) plus a mirror symmetry.  None of these
expected values comes from the oracle itself."""

import math

import numpy as np
import pytest

from helpers import oracle_workload
from oracle import bspline as ob
from oracle import raycast as orc
from paper_2204_11762_amd import workloads as wl


def _c1_camera(W=128, H=128):
    return orc.Camera("ortho", (0.5, 0.5, 2.0), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), W, H)


def test_camera_frame_c1():
    F, R, V = orc.camera_frame(_c1_camera())
    assert F == (0.0, 0.0, -1.0)
    assert R == (1.0, 0.0, 0.0)
    assert V == (0.0, 1.0, 0.0)


def test_ortho_rays_and_slab_c1():
    cam = _c1_camera()
    r, c = np.divmod(np.arange(128 * 128), 128)
    o, d = orc.camera_rays(cam, r, c)
    np.testing.assert_array_equal(o[:, 0], (c + 0.5) / 128)
    np.testing.assert_array_equal(o[:, 1], 1 - (r + 0.5) / 128)
    assert (o[:, 2] == 2.0).all()
    assert (d == np.array([0.0, 0.0, -1.0])).all()
    t0, t1, hit = orc.slab(o, d, np.zeros(3), np.ones(3))
    assert hit.all() and (t0 == 1.0).all() and (t1 == 2.0).all()
    n = orc.sample_counts(t0, t1, hit, 1 / 256)
    assert (n == 256).all()


def test_perspective_rays():
    W, H = 64, 48
    cam = orc.Camera("persp", (0.0, 0.0, 5.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H,
                     fov_y_deg=60.0)
    r, c = np.divmod(np.arange(W * H), W)
    o, d = orc.camera_rays(cam, r, c)
    assert np.allclose(o, [0, 0, 5])
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    # pixel centres: tan of the angle to the axis is linear in the pixel index
    tan_x = d[:, 0] / -d[:, 2]
    tan_y = d[:, 1] / -d[:, 2]
    tau = math.tan(math.radians(30.0))
    np.testing.assert_allclose(tan_y, (1 - 2 * (r + 0.5) / H) * tau, atol=1e-14)
    np.testing.assert_allclose(tan_x, (2 * (c + 0.5) / W - 1) * tau * W / H, atol=1e-14)
    # row 0 is the top of the image, column 0 the left
    assert d[0, 1] > 0 and d[0, 0] < 0


def test_slab_special_rays():
    lo, hi = np.zeros(3), np.ones(3)
    o = np.array([[0.5, 0.5, 3.0],     # straight through the middle
                  [1.0, 0.5, 3.0],     # along the face x = 1 (inside, closed box)
                  [1.5, 0.5, 3.0],     # parallel to z, outside in x -> miss
                  [0.5, 0.5, 0.5],     # eye inside the box
                  [-1.0, -1.0, -1.0],  # body diagonal
                  [2.0, 2.0, 0.5]])    # misses the box
    d = np.array([[0, 0, -1.0], [0, 0, -1.0], [0, 0, -1.0], [1.0, 0, 0],
                  [1, 1, 1.0] / np.sqrt(3), [0, 0, 1.0]])
    t0, t1, hit = orc.slab(o, d, lo, hi)
    assert hit.tolist() == [True, True, False, True, True, False]
    assert (t0[0], t1[0]) == (2.0, 3.0)
    assert (t0[1], t1[1]) == (2.0, 3.0)
    assert (t0[3], t1[3]) == (0.0, 0.5)
    np.testing.assert_allclose([t0[4], t1[4]], [np.sqrt(3), 2 * np.sqrt(3)], rtol=1e-15)
    n = orc.sample_counts(t0, t1, hit, 0.1)
    assert n.tolist() == [10, 10, 0, 5, 17, 0]


def test_tf_lookup_hand_cases():
    T = np.array([[0, 0, 0, 0], [1, 0.5, 0.25, 1], [0, 1, 0, 0.5]], dtype=np.float32)
    tf = orc.TransferFunction(T, -1.0, 3.0)
    v = np.array([-5.0, -1.0, 1.0, 3.0, 9.0, 0.0, 2.0])
    out = orc.tf_lookup(tf, v)
    np.testing.assert_array_equal(out[0], T[0])
    np.testing.assert_array_equal(out[1], T[0])
    np.testing.assert_array_equal(out[2], T[1])
    np.testing.assert_array_equal(out[3], T[2])
    np.testing.assert_array_equal(out[4], T[2])
    np.testing.assert_allclose(out[5], (T[0] + T[1]) / 2, atol=1e-15)
    np.testing.assert_allclose(out[6], (T[1] + T[2]) / 2, atol=1e-15)


def test_phong_hand_cases():
    prm = orc.RenderParams(step=0.1)
    rgb = np.array([[0.5, 0.2, 1.0]] * 4)
    z = np.array([0, 0, 1.0])
    g = np.array([[0, 0, 3.0],      # n = l = v: diff 1, spec 1
                  [0, 0, -2.0],     # two-sided: same as above
                  [1.0, 0, 0],      # n perpendicular to l: diff 0, r = -l -> spec 0
                  [0, 0, 0.0]])     # zero gradient: n = 0, diff 0, spec 0
    L = np.broadcast_to(z, (4, 3))
    out = orc.phong(rgb, g, L, L, prm)
    lit = np.minimum((0.1 + 0.7) * rgb[0] + 0.2, 1.0)
    np.testing.assert_allclose(out[0], lit, atol=1e-15)
    np.testing.assert_allclose(out[1], lit, atol=1e-15)
    np.testing.assert_allclose(out[2], 0.1 * rgb[2], atol=1e-15)
    np.testing.assert_allclose(out[3], 0.1 * rgb[3], atol=1e-15)
    # 45 degrees: n.l = cos45, r = 2 cos45 n - l lies along x; view at 45 deg
    # on the other side of n sees the mirror direction: r.v = 1
    n45 = np.array([[0, 0, 1.0]])
    l45 = np.array([[1.0, 0, 1.0]]) / math.sqrt(2)
    v45 = np.array([[-1.0, 0, 1.0]]) / math.sqrt(2)
    out = orc.phong(rgb[:1], n45, l45, v45, prm)
    np.testing.assert_allclose(out[0], np.minimum((0.1 + 0.7 * math.sqrt(0.5)) * rgb[0] + 0.2, 1),
                               atol=1e-15)
    # specular exponent: r.v = cos(theta) -> cos^10
    th = 0.3
    vth = np.array([[-math.sin(math.pi / 4 + th), 0, math.cos(math.pi / 4 + th)]])
    out = orc.phong(np.zeros((1, 3)), n45, l45, vth, prm)
    np.testing.assert_allclose(out[0], 0.2 * math.cos(th) ** 10, atol=1e-15)


def _constant_pixel(c0, nr, omax, ka=0.1):
    """Closed form for a constant field: every sample has the same colour
    and alpha; k* = min(N_r, first k with 1-(1-a)^k > O_max)."""
    a = c0
    k = 0
    A = 0.0
    while k < nr:
        k += 1
        A = 1 - (1 - a) ** k
        if A > omax:
            break
    return np.array([ka * c0 * A] * 3 + [A]), k


@pytest.mark.parametrize("c0", [0.5, 0.03, 0.0])
def test_constant_field_image(c0):
    n, p = 6, 2
    U = wl.clamped_uniform_knots(n, p)
    M = ob.Model((p, p, p), (U, U, U), np.full((n, n, n), c0), np.zeros(3), np.ones(3))
    cam = _c1_camera(16, 16)
    e = np.arange(5) / 4.0          # a ramp that is exact in float32
    tf = orc.TransferFunction(np.repeat(e[:, None], 4, 1).astype(np.float32), 0.0, 1.0)
    prm = orc.RenderParams(step=1 / 64)
    res = orc.render(M, cam, tf, prm)
    want, k = _constant_pixel(c0, 64, 0.99)
    # the computed gradient of a constant field is zero up to rounding
    # (~1e-16); the 1e-6 clamp of |g| turns that into a normal of length
    # up to ~1e-9, hence the tolerance
    np.testing.assert_allclose(res.rgba.reshape(-1, 4), np.broadcast_to(want, (256, 4)),
                               rtol=0, atol=1e-9)
    assert (res.samples == k).all()
    if c0 == 0.5:
        assert k == 7


def test_linear_field_image():
    """f = w reproduced exactly (Marsden, m = 1 along z); with the c1
    camera sample s sits at w = 1 - (s+1/2)/256, the world gradient is +z
    and n = l = v, so diff = spec = 1."""
    n, p = 16, 2
    U = wl.clamped_uniform_knots(n, p)
    cz = ob.marsden_coeffs(p, U, 1)
    ctrl = np.broadcast_to(cz[:, None, None], (n, n, n)).copy()
    M = ob.Model((p, p, p), (U, U, U), ctrl, np.zeros(3), np.ones(3))
    cam = _c1_camera(8, 8)
    tf = orc.TransferFunction(wl.ramp_tf().table, 0.0, 1.0)
    for omax in (0.99, 1.0):
        prm = orc.RenderParams(step=1 / 256, ert_alpha=omax)
        res = orc.render(M, cam, tf, prm)
        C = A = 0.0
        k = 0
        for s in range(256):
            w = 1 - (s + 0.5) / 256
            a = w                               # ramp table: colour = alpha = value
            cs = min(1.0, (0.1 + 0.7) * w + 0.2)
            C += (1 - A) * a * cs
            A += (1 - A) * a
            k += 1
            if A > omax:
                break
        want = np.array([C, C, C, A])
        np.testing.assert_allclose(res.rgba.reshape(-1, 4), np.broadcast_to(want, (64, 4)),
                                   rtol=0, atol=1e-7)  # table is float32: e/255 rounded
        assert (res.samples == k).all()


def test_linear_field_image_exact_table():
    """As above with a table that is exact in float32 (steps of 1/4)."""
    n, p = 10, 3
    U = wl.clamped_uniform_knots(n, p)
    cz = ob.marsden_coeffs(p, U, 1)
    ctrl = np.broadcast_to(cz[:, None, None], (n, n, n)).copy()
    M = ob.Model((p, p, p), (U, U, U), ctrl, np.zeros(3), np.ones(3))
    cam = _c1_camera(4, 4)
    e = np.arange(5) / 4.0
    tf = orc.TransferFunction(np.repeat(e[:, None], 4, 1).astype(np.float32), 0.0, 1.0)
    prm = orc.RenderParams(step=1 / 32)
    res = orc.render(M, cam, tf, prm)
    C = A = 0.0
    for s in range(32):
        w = 1 - (s + 0.5) / 32
        cs = min(1.0, 0.8 * w + 0.2)
        C += (1 - A) * w * cs
        A += (1 - A) * w
        if A > 0.99:
            break
    np.testing.assert_allclose(res.rgba.reshape(-1, 4), np.broadcast_to([C, C, C, A], (16, 4)),
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("light, diff, spec", [
    # l = (0, 3, 4)/5 (given unnormalised): n.l = 0.8, r = 2(n.l)n - l =
    # (0, -0.6, 0.8), r.v = 0.8
    ((0.0, 3.0, 4.0), 0.8, 0.8 ** 10),
    # the opposite light: two-sided diffuse |n.l| = 0.8, r = (0, 0.6, -0.8)
    # points away from the eye, r.v = -0.8, no specular
    ((0.0, -3.0, -4.0), 0.8, 0.0),
    # tilted in x: l = (12, 0, 5)/13, n.l = 5/13, r = (-12, 0, 5)/13, r.v = 5/13
    ((12.0, 0.0, 5.0), 5 / 13, (5 / 13) ** 10),
])
def test_linear_field_explicit_light(light, diff, spec):
    """The explicit-light branch (headlight off): f = w reproduced exactly,
    the c1 camera (v = +z, world gradient +z, so n = +z), and a light
    direction given unnormalised.  Diffuse and specular terms follow from
    the hand-normalised light, so every pixel is one closed-form sum; a
    missing normalisation or a one-sided diffuse fails."""
    n, p = 10, 3
    U = wl.clamped_uniform_knots(n, p)
    cz = ob.marsden_coeffs(p, U, 1)
    ctrl = np.broadcast_to(cz[:, None, None], (n, n, n)).copy()
    M = ob.Model((p, p, p), (U, U, U), ctrl, np.zeros(3), np.ones(3))
    cam = _c1_camera(4, 4)
    e = np.arange(5) / 4.0
    tf = orc.TransferFunction(np.repeat(e[:, None], 4, 1).astype(np.float32), 0.0, 1.0)
    prm = orc.RenderParams(step=1 / 32, headlight=False, light_dir=light)
    res = orc.render(M, cam, tf, prm)
    C = A = 0.0
    for s in range(32):
        w = 1 - (s + 0.5) / 32
        cs = min(1.0, (0.1 + 0.7 * diff) * w + 0.2 * spec)
        C += (1 - A) * w * cs
        A += (1 - A) * w
        if A > 0.99:
            break
    np.testing.assert_allclose(res.rgba.reshape(-1, 4), np.broadcast_to([C, C, C, A], (16, 4)),
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("light, diff, spec", [
    # n = +x, v = +z (n.v = 0): r = 2 (n.l) n - l = (0.6, 0, 0.8), r.v = 0.8
    ((3.0, 0.0, -4.0), 0.6, 0.8 ** 10),
    # mirrored light: r = (-0.6, 0, -0.8) faces away from the eye
    ((-3.0, 0.0, 4.0), 0.6, 0.0),
])
def test_linear_field_x_explicit_light(light, diff, spec):
    """Headlight off with the normal across the view: f = u reproduced
    exactly (Marsden along x), so n = +x while v = +z.  Every sample of the
    ray through column c has f = (c + 1/2)/W (u is constant along a z ray),
    so the pixel is the constant-colour closed form with opacity f and the
    shaded colour min(1, (k_a + k_d |n.l|) f + k_s max(0, r.v)^k).  Here r.v
    comes only from the reflected light (n.v = 0): a sign or term slip in
    r = 2 (n.l) n - l shows."""
    n, p = 10, 3
    U = wl.clamped_uniform_knots(n, p)
    cx = ob.marsden_coeffs(p, U, 1)
    ctrl = np.broadcast_to(cx[None, None, :], (n, n, n)).copy()
    M = ob.Model((p, p, p), (U, U, U), ctrl, np.zeros(3), np.ones(3))
    W, H = 8, 3
    cam = _c1_camera(W, H)
    e = np.arange(5) / 4.0
    tf = orc.TransferFunction(np.repeat(e[:, None], 4, 1).astype(np.float32), 0.0, 1.0)
    prm = orc.RenderParams(step=1 / 32, headlight=False, light_dir=light)
    res = orc.render(M, cam, tf, prm)
    for c in range(W):
        a = (c + 0.5) / W
        cs = min(1.0, (0.1 + 0.7 * diff) * a + 0.2 * spec)
        k = 0
        A = 0.0
        while k < 32:
            k += 1
            A = 1 - (1 - a) ** k
            if A > 0.99:
                break
        want = np.array([cs * A, cs * A, cs * A, A])
        np.testing.assert_allclose(res.rgba[:, c, :], np.broadcast_to(want, (H, 4)),
                                   rtol=0, atol=1e-14)
        assert (res.samples.reshape(H, W)[:, c] == k).all()


def test_mirror_symmetry():
    """A model symmetric under x <-> y seen from a camera in the plane x = y
    with up = +z renders a left-right mirror-symmetric image."""
    rng = np.random.default_rng(21)
    n, p = 9, 3
    U = wl.clamped_uniform_knots(n, p)
    P = rng.random((n, n, n))
    P = 0.5 * (P + np.transpose(P, (0, 2, 1)))       # P[k, j, i] = P[k, i, j]
    M = ob.Model((p, p, p), (U, U, U), P, np.zeros(3), np.ones(3))
    cam = orc.Camera("persp", (2.2, 2.2, 0.9), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 24, 20)
    tf = orc.TransferFunction(wl.pwl_tf(5, P.min(), P.max(), alpha_max=0.2).table,
                              P.min(), P.max())
    res = orc.render(M, cam, tf, orc.RenderParams(step=1 / 64))
    img = res.rgba
    assert img[..., 3].max() > 0.1
    np.testing.assert_allclose(img, img[:, ::-1], rtol=0, atol=1e-12)


def test_miss_pixels_are_transparent_black():
    wk = wl.c2()
    wk.camera.width = wk.camera.height = 48
    M, cam, tf, prm = oracle_workload(wk)
    res = orc.render(M, cam, tf, prm)
    miss = res.n_nominal.reshape(48, 48) == 0
    assert miss.any() and (~miss).any()
    assert (res.rgba[miss] == 0).all()
    assert (res.rgba[~miss][:, 3] > 0).all()


def test_c1_workload_facts():
    """The c1 inputs: 256 nominal samples on every ray; value range of the
    model inside [0, 1] so the ramp table is never clamped."""
    wk = wl.c1()
    M, cam, tf, prm = oracle_workload(wk)
    assert wk.model.ctrl.shape == (16, 16, 16)
    assert (M.knots[0][:3] == 0).all() and M.knots[0][3] == 1 / 14
    res = orc.render_pixels(M, cam, tf, prm, np.arange(0, 128 * 128, 97))
    assert (res.n_nominal == 256).all()
    assert (res.samples >= 1).all() and (res.samples < 256).all()


def test_field_callback_reproduces_model_path():
    """A closed-form field given as a callback is rendered by the same
    steps: passing the model's own world evaluation as the field gives the
    default image exactly."""
    from oracle import bspline as ob
    wk = wl.c1()
    M, cam, tf, prm = oracle_workload(wk)
    pix = np.arange(0, 128 * 128, 37)
    ref = orc.render_pixels(M, cam, tf, prm, pix)
    got = orc.render_pixels(M, cam, tf, prm, pix, field=lambda xyz: ob.eval_world(M, xyz))
    np.testing.assert_allclose(got.rgba, ref.rgba, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(got.samples, ref.samples)
