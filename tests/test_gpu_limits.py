"""GPU parity at the ABI's size limits, through the C ABI: the largest image
(2^26 pixels) and a BF16 model whose control points fill the 2^31-byte
limit on 32-bit element offsets, each against the FP64 oracle on sampled
outputs and on properties that hold at any size, and the first sizes past
each limit refused."""

import numpy as np
import pytest

from gpu_helpers import FP32_REL, FP32_RMSE, compare_image, gpu_eval, gpu_render, normwise, torch_mod
from helpers import oracle_model
from oracle import bspline as ob
from paper_2204_11762_amd import workloads as wl

pytestmark = pytest.mark.gpu

TAU32 = 2e-5
PX32 = 2e-4


def test_largest_image(mfa):
    """8192 x 8192 pixels, an orthographic view whose window is the box's
    front face: every ray crosses the whole depth, so with termination off
    each takes exactly 1 / step samples and the frame's count is known in
    closed form (2^32, beyond 32 bits)."""
    b, ctx = mfa
    torch = torch_mod()
    rng = np.random.default_rng(401)
    spec = wl.random_model(rng, n=(12, 11, 10), degree=(2, 2, 2))
    side = 8192
    cam = wl.CameraSpec("ortho", (0.5, 0.5, 3.0), (0.5, 0.5, 0.0), (0.0, 1.0, 0.0), side, side,
                        ortho_half_w=0.5, ortho_half_h=0.5)
    P = np.asarray(spec.ctrl)
    tf = wl.pwl_tf(41, P.min(), P.max(), alpha_max=0.05)
    prm = wl.ParamSpec(step=1.0 / 64, ert_alpha=1.0)
    wk = wl.Workload("largest image", spec, cam, tf, prm)
    h = b.mfa_model_upload(ctx, spec)
    try:
        img, cnt = gpu_render(b, ctx, h, wk)
        assert cnt == 64 * side * side
        assert np.isfinite(img).all() and (img[..., 3] > 0).all()
        # corners, last row and column, and random pixels
        last = side * side - 1
        pix = np.concatenate([[0, side - 1, last - side + 1, last],
                              last - side + 1 + np.arange(0, side, 997),
                              np.arange(side - 1, side * side, side * 991),
                              wl.pixel_subset(side, side, 400, seed=42)])
        rep = compare_image(img, cnt, wk, pix, TAU32, PX32)
        print(f"\n  8192^2: rmse {rep.rmse:.2e} max {rep.max_abs:.2e} on {len(pix)} pixels")
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        del img
        # one pixel more, or a side beyond 32768, is refused
        out = torch.zeros((1, 1, 4), dtype=torch.float32, device="cuda")
        for w, hgt in ((side, side + 1), (32769, 1)):
            bad = wl.CameraSpec("ortho", cam.eye, cam.target, cam.up, w, hgt,
                                ortho_half_w=0.5, ortho_half_h=0.5)
            st = b.lib.mfa_render(ctx, h, b.C.byref(b.camera_struct(bad)),
                                  b.C.byref(b.tf_struct(tf)[0]),
                                  b.C.byref(b.params_struct(prm)), out.data_ptr(), None, None)
            assert st == b.MFA_ERR_INVALID, (w, hgt)
    finally:
        b.mfa_model_free(ctx, h)


def test_largest_bf16_model(mfa):
    """1024 x 1024 x 1020 cubic control points in BF16 (just under 2^31 bytes
    with the row padding): point queries over the box and at its far corner,
    and a frame through the far corner, against the oracle.  The values are
    exact in BF16, so the oracle sees the stored model."""
    b, ctx = mfa
    rng = np.random.default_rng(402)
    n = (1024, 1024, 1020)
    knots = tuple(wl.clamped_uniform_knots(n[k], 3) for k in range(3))
    # (128 + k) / 256, k < 128: eight significant bits, exact in BF16
    ctrl = rng.integers(0, 128, size=n[0] * n[1] * n[2], dtype=np.uint16)
    ctrl = ((ctrl.astype(np.float64) + 128.0) / 256.0).reshape(n[2], n[1], n[0])
    spec = wl.ModelSpec((3, 3, 3), knots, ctrl)
    h = b.mfa_model_upload(ctx, spec, b.MFA_STORE_BF16)
    try:
        M = oracle_model(spec)
        xyz = np.concatenate([wl.uniform_points(rng, 3000, np.zeros(3), np.ones(3)),
                              wl.uniform_points(rng, 200, np.full(3, 0.999), np.ones(3)),
                              np.array([[a, c, d] for a in (0, 1) for c in (0, 1) for d in (0, 1)],
                                       float)])
        f, g = gpu_eval(b, ctx, h, xyz)
        F, G = ob.eval_world(M, xyz)
        ev, eg = normwise(f, F), normwise(g, G)
        print(f"\n  1024x1024x1020 BF16: value rel {ev:.2e} gradient rel {eg:.2e}")
        assert ev <= FP32_REL and eg <= FP32_REL
        cam = wl.CameraSpec("persp", (1.45, 1.4, 1.5), (0.96, 0.96, 0.96), (0.0, 1.0, 0.0), 48, 40,
                            fov_y_deg=6.0)
        tf = wl.pwl_tf(43, 0.5, 1.0, alpha_max=0.05)
        wk = wl.Workload("largest model", spec, cam, tf, wl.ParamSpec(step=1.0 / 1024))
        img, cnt = gpu_render(b, ctx, h, wk)
        rep = compare_image(img, cnt, wk, np.arange(48 * 40), TAU32, PX32, model=M)
        print(f"  frame through the far corner: rmse {rep.rmse:.2e} samples "
              f"{rep.samples_gpu}/{rep.samples_ref}")
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        assert abs(rep.samples_gpu - rep.samples_ref) <= rep.samples_slack
        assert rep.samples_ref > 1000
    finally:
        b.mfa_model_free(ctx, h)
    # 1024^3 BF16 is past the limit: refused from the counts alone
    small = wl.ModelSpec((3, 3, 3), tuple(wl.clamped_uniform_knots(1024, 3) for _ in range(3)),
                         np.zeros((1, 1, 1)))
    d, keep = b.model_desc(small, b.MFA_STORE_BF16)
    d.n_ctrl[0] = d.n_ctrl[1] = d.n_ctrl[2] = 1024
    out = b.C.c_int64()
    assert b.lib.mfa_model_upload(ctx, b.C.byref(d), b.C.byref(out)) == b.MFA_ERR_INVALID
    assert "too large" in b.last_error()
