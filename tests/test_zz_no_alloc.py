"""The allocation-free render entry point (mfa_render_noalloc), called
through the C ABI: two calls in a row, the second with a smaller image and
on another stream, each equal to mfa_render's image and sample count bit
for bit and to the FP64 oracle within the FP32 bar on sampled pixels; a
frame on the global-memory caster (no tile planning); an image beyond the
fixed scratch's limit refused before anything is enqueued."""

from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import FP32_RMSE, compare_image, gpu_render
from paper_2204_11762_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _noalloc(b, ctx, model, wk, stream=None):
    import torch
    cam = wk.camera
    out = torch.full((cam.height, cam.width, 4), -1.0, dtype=torch.float32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    b.mfa_render_noalloc(ctx, model, cam, wk.tf, wk.params, out, cnt, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), int(cnt.cpu().item())


def _check_oracle(img, cnt, wk, seed):
    W, H = wk.camera.width, wk.camera.height
    pix = np.sort(np.random.default_rng(seed).choice(W * H, min(600, W * H), replace=False))
    rep = compare_image(img, cnt, wk, pix, 2e-5, 2e-4)
    assert rep.rmse <= FP32_RMSE and rep.n_bad == 0, rep


def test_noalloc_two_calls_equal_render(mfa):
    import torch
    b, ctx = mfa
    big = wl.c2()
    big.camera = wl.orbit_camera(480, 360, 30.0, 20.0)
    small = wl.c2()
    small.camera = wl.orbit_camera(96, 72, 200.0, -35.0)
    h = b.mfa_model_upload(ctx, big.model)
    try:
        ref_big = gpu_render(b, ctx, h, big)
        ref_small = gpu_render(b, ctx, h, small)
        got_big = _noalloc(b, ctx, h, big)
        side = torch.cuda.Stream()
        got_small = _noalloc(b, ctx, h, small, stream=side)
        # the first image again after the smaller one: nothing left over
        again = _noalloc(b, ctx, h, big)
        for (img, cnt), (rimg, rcnt), name in ((got_big, ref_big, "first"),
                                               (got_small, ref_small, "second"),
                                               (again, ref_big, "third")):
            assert np.array_equal(img, rimg), f"{name} call: image differs from mfa_render"
            assert cnt == rcnt, f"{name} call: count {cnt} != {rcnt}"
        _check_oracle(got_big[0], got_big[1], big, 1)
        _check_oracle(got_small[0], got_small[1], small, 2)
    finally:
        b.mfa_model_free(ctx, h)


def test_noalloc_global_kernel_and_ortho(mfa):
    """A 4096-entry transfer function leaves too little LDS for bricks, so
    the frame takes the global-memory caster (no tile planning); then a
    small orthographic frame on the brick caster."""
    b, ctx = mfa
    wk = wl.c1()
    wk.camera.width, wk.camera.height = 40, 24
    wide = wl.c1()
    wide.camera.width, wide.camera.height = 40, 24
    wide.tf = wl.ramp_tf(4096)
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        for w in (wide, wk):
            ref = gpu_render(b, ctx, h, w)
            got = _noalloc(b, ctx, h, w)
            assert np.array_equal(got[0], ref[0]) and got[1] == ref[1]
            _check_oracle(got[0], got[1], w, 3)
    finally:
        b.mfa_model_free(ctx, h)


def test_noalloc_rejects_beyond_limit(mfa):
    import torch
    b, ctx = mfa
    wk = wl.c1()
    wk.camera = wl.orbit_camera(5700, 5700, 30.0, 20.0)
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        out = torch.full((5700, 5700, 4), -1.0, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(b.MFAError) as ei:
            b.mfa_render_noalloc(ctx, h, wk.camera, wk.tf, wk.params, out)
        assert ei.value.status == b.MFA_ERR_INVALID
        assert "at most" in str(ei.value)
        torch.cuda.synchronize()
        assert bool((out[::97, ::89] == -1.0).all().item())
        # the largest square image within the limit renders
        del out
        wk.camera = wl.orbit_camera(5600, 5600, 30.0, 20.0)
        ref = gpu_render(b, ctx, h, wk)
        got = _noalloc(b, ctx, h, wk)
        assert np.array_equal(got[0], ref[0]) and got[1] == ref[1]
    finally:
        b.mfa_model_free(ctx, h)
