"""GPU parity of rendering with a curvature transfer function
(mfa_render_curvature) against the FP64 oracle, through the C ABI.  Up to
degree 3 the brick ray caster renders it (second derivatives from the span
tables on both of its paths); degree 4 uses the global-memory kernel.

Principal curvatures are well conditioned where the gradient is large
against the Hessian and ill conditioned near critical points (the
isosurface normal is undefined where g = 0).  The quadric cases keep |g|
bounded away from 0 by construction (centre outside the box); the seeded
random-model and full-size cases contain critical points, but no sample
falls close enough to one for FP32 and FP64 to part, and all cases are held
to the FP32 image bar."""

import copy

import numpy as np
import pytest

from gpu_helpers import FP32_RMSE, compare_image, gpu_render, torch_mod
from helpers import oracle_model
from oracle import bspline as ob
from oracle import quant
from paper_2204_11762_amd import workloads as wl

pytestmark = pytest.mark.gpu

TAU32 = 2e-5
PX32 = 2e-4


def _sphere_spec(seed, degree=(2, 3, 2), n=(10, 9, 11), centre=(-0.6, 0.45, 0.5), noise=2e-3,
                 uniform=False):
    """|x - c|^2 reproduced on Beta(2,5) knots (uniform knots if asked;
    centre outside the box, so 1.2 <= |g| everywhere), plus small
    control-point noise."""
    rng = np.random.default_rng(seed)
    knots = tuple(wl.clamped_uniform_knots(n[k], degree[k]) if uniform
                  else wl.clamped_beta_knots(n[k], degree[k], rng) for k in range(3))
    ctrl = np.zeros((n[2], n[1], n[0]))
    for ax in range(3):
        c = centre[ax]
        q = (ob.marsden_coeffs(degree[ax], knots[ax], 2)
             - 2 * c * ob.marsden_coeffs(degree[ax], knots[ax], 1) + c * c)
        shape = [1, 1, 1]
        shape[2 - ax] = n[ax]
        ctrl = ctrl + q.reshape(shape)
    ctrl = ctrl + noise * rng.standard_normal(ctrl.shape)
    return wl.ModelSpec(tuple(degree), knots, ctrl)


def _workload(spec, size=48, ert=0.99, shading=True, seed=5):
    cam = wl.orbit_camera(size, size, 35.0, 25.0, radius=2.6, target=(0.5, 0.5, 0.5))
    tf = wl.pwl_tf(seed, 0.3, 2.5)
    prm = wl.ParamSpec(step=1.0 / 128, ert_alpha=ert, shading=shading)
    return wl.Workload("curvature", spec, cam, tf, prm)


def gpu_curvature_render(b, ctx, h, wk, ctf):
    torch = torch_mod()
    W, H = wk.camera.width, wk.camera.height
    out = torch.full((H, W, 4), -1.0, dtype=torch.float32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    b.mfa_render_curvature(ctx, h, wk.camera, wk.tf, ctf, wk.params, out, cnt)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), int(cnt.item())


def _run(mfa, spec, wk, ctf, store=0, pix=None, deq=None):
    b, ctx = mfa
    h = b.mfa_model_upload(ctx, spec, store)
    try:
        img, cnt = gpu_curvature_render(b, ctx, h, wk, ctf)
    finally:
        b.mfa_model_free(ctx, h)
    W, H = wk.camera.width, wk.camera.height
    pix = np.arange(W * H) if pix is None else pix
    M = None if deq is None else oracle_model(spec, ctrl=deq(spec.ctrl))
    rep = compare_image(img, cnt, wk, pix, TAU32, PX32, model=M, curvature=ctf)
    return img, rep


@pytest.mark.parametrize("shading", [False, True])
def test_quadric_exact_no_termination(mfa, shading):
    spec = _sphere_spec(51)
    wk = _workload(spec, ert=1.0, shading=shading)
    ctf = wl.curvature_tf(32, 0.0, 2.5)
    img, rep = _run(mfa, spec, wk, ctf)
    print(f"\n  quadric shading={shading}: rmse {rep.rmse:.2e} max {rep.max_abs:.2e} "
          f"samples {rep.samples_gpu}/{rep.samples_ref}")
    assert np.isfinite(img).all()
    assert rep.n_bad == 0 and rep.rmse <= FP32_RMSE
    assert rep.samples_gpu == rep.samples_ref
    # the curvature table changes the image: not the plain render
    assert np.abs(img[..., :3]).max() > 0


@pytest.mark.parametrize("store", [1, 2])
def test_quadric_storages_with_termination(mfa, store):
    spec = _sphere_spec(52, degree=(3, 3, 3), n=(9, 10, 8))
    wk = _workload(spec, ert=0.99)
    ctf = wl.curvature_tf(24, 0.0, 2.5)
    deq = quant.dequant_bf16 if store == 1 else quant.dequant_f16
    _, rep = _run(mfa, spec, wk, ctf, store=store, deq=deq)
    print(f"\n  quadric store {store}: rmse {rep.rmse:.2e} ambiguous {rep.n_ambiguous} "
          f"samples {rep.samples_gpu}/{rep.samples_ref}")
    assert rep.n_bad == 0 and rep.rmse <= FP32_RMSE
    assert abs(rep.samples_gpu - rep.samples_ref) <= rep.samples_slack


# (degree, uniform knots): the brick caster's uniform-knot path with equal
# and mixed degrees, its general path with mixed degrees, and degree 4,
# which renders curvature with the global-memory kernel
VARIANTS = [((2, 2, 2), True), ((2, 3, 3), True), ((3, 2, 3), False), ((4, 4, 4), True),
            ((4, 3, 4), False)]


@pytest.mark.parametrize("variant", range(len(VARIANTS)))
def test_quadric_kernel_variants(mfa, variant):
    deg, uniform = VARIANTS[variant]
    n = tuple(d + 8 for d in deg)
    spec = _sphere_spec(60 + variant, degree=deg, n=n, uniform=uniform)
    wk = _workload(spec, size=40, ert=0.99, shading=variant % 2 == 0)
    ctf = wl.curvature_tf(24, 0.0, 2.5)
    img, rep = _run(mfa, spec, wk, ctf)
    print(f"\n  degree {deg} uniform={uniform}: rmse {rep.rmse:.2e} max {rep.max_abs:.2e} "
          f"ambiguous {rep.n_ambiguous} samples {rep.samples_gpu}/{rep.samples_ref}")
    assert np.isfinite(img).all()
    assert rep.n_bad == 0 and rep.rmse <= FP32_RMSE
    assert abs(rep.samples_gpu - rep.samples_ref) <= rep.samples_slack


def test_random_model_near_critical_points(mfa):
    """A random smooth model (critical points inside the box)."""
    spec = wl.random_model(np.random.default_rng(53), n=(12, 11, 10), degree=(3, 3, 3),
                           beta_knots=True)
    cam = wl.orbit_camera(48, 48, 30.0, 20.0, radius=2.6, target=(0.5, 0.5, 0.5))
    wk = wl.Workload("curvature", spec, cam, wl.pwl_tf(6, float(spec.ctrl.min()),
                                                       float(spec.ctrl.max())),
                     wl.ParamSpec(step=1.0 / 128))
    ctf = wl.curvature_tf(32, -30.0, 30.0)
    _, rep = _run(mfa, spec, wk, ctf)
    print(f"\n  random model: rmse {rep.rmse:.2e} max {rep.max_abs:.2e} bad {rep.n_bad} "
          f"ambiguous {rep.n_ambiguous}")
    assert rep.rmse <= FP32_RMSE and rep.n_bad == 0


def test_c3_model_sampled(mfa):
    """The 256^3 degree-3 model at 512^2 with the curvature table: 200 sampled
    pixels against the oracle."""
    w3 = wl.c3()
    cam = copy.copy(w3.camera)
    cam.width = cam.height = 512
    wk = wl.Workload("curvature", w3.model, cam, w3.tf, w3.params)
    ctf = wl.curvature_tf(32, -60.0, 60.0)
    pix = wl.pixel_subset(512, 512, 200, seed=54)
    _, rep = _run(mfa, w3.model, wk, ctf, pix=pix)
    print(f"\n  c3 512^2: rmse {rep.rmse:.2e} max {rep.max_abs:.2e} bad {rep.n_bad} "
          f"ambiguous {rep.n_ambiguous}")
    assert rep.rmse <= FP32_RMSE and rep.n_bad == 0


def test_curvature_errors(mfa):
    torch = torch_mod()
    b, ctx = mfa
    spec = _sphere_spec(55)
    wk = _workload(spec, size=16)
    out = torch.zeros((16, 16, 4), dtype=torch.float32, device="cuda")
    h = b.mfa_model_upload(ctx, spec)
    good = wl.curvature_tf(8, -1.0, 1.0)
    try:
        bad = {
            "one entry": wl.CurvatureTFSpec(good.table[:1, :1], -1.0, 1.0),
            "too large": wl.CurvatureTFSpec(np.zeros((65, 65, 4), np.float32), -1.0, 1.0),
            "empty range": wl.CurvatureTFSpec(good.table, 1.0, 1.0),
            "nan entry": wl.CurvatureTFSpec(np.full((4, 4, 4), np.nan, np.float32), -1.0, 1.0),
            "opacity above 1": wl.CurvatureTFSpec(np.full((4, 4, 4), 1.5, np.float32), -1.0, 1.0),
        }
        for name, ctf in bad.items():
            with pytest.raises(b.MFAError) as e:
                b.mfa_render_curvature(ctx, h, wk.camera, wk.tf, ctf, wk.params, out)
            assert e.value.status == b.MFA_ERR_INVALID, name
        st = b.lib.mfa_render_curvature(ctx, h, None, None, None, None, None, None, None)
        assert st == b.MFA_ERR_INVALID
        b.mfa_render_curvature(ctx, h, wk.camera, wk.tf, good, wk.params, out)
        torch.cuda.synchronize()
    finally:
        b.mfa_model_free(ctx, h)
    rspec = _sphere_spec(56)
    rspec.weights = np.full(rspec.ctrl.shape, 2.0)
    hr = b.mfa_model_upload(ctx, rspec)
    try:
        with pytest.raises(b.MFAError) as e:
            b.mfa_render_curvature(ctx, hr, wk.camera, wk.tf, good, wk.params, out)
        assert e.value.status == b.MFA_ERR_MODEL
    finally:
        b.mfa_model_free(ctx, hr)


def test_concurrent_with_plain_renders(mfa):
    """Curvature frames and plain frames of another model enqueued
    alternately on two streams without synchronising in between (each
    stream has its own tile-planning space) equal their solo renders bit for
    bit."""
    torch = torch_mod()
    b, ctx = mfa
    spec = _sphere_spec(58, degree=(3, 3, 3), n=(11, 11, 11), uniform=True)
    ctf = wl.curvature_tf(16, 0.0, 2.5)
    curv = [_workload(spec, size=sz, seed=9) for sz in (40, 56)]
    plain = wl.c2()
    plain.camera = wl.orbit_camera(96, 80, 60.0, 25.0)
    hc = b.mfa_model_upload(ctx, spec)
    hp = b.mfa_model_upload(ctx, plain.model)
    try:
        ref_c = [gpu_curvature_render(b, ctx, hc, w, ctf) for w in curv]
        ref_p = gpu_render(b, ctx, hp, plain)
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        outs = [torch.zeros((w.camera.height, w.camera.width, 4), dtype=torch.float32,
                            device="cuda") for w in curv]
        out_p = torch.zeros((80, 96, 4), dtype=torch.float32, device="cuda")
        cnts = [torch.zeros((1,), dtype=torch.int64, device="cuda") for _ in range(3)]
        torch.cuda.synchronize()
        for rep in range(3):
            for i, w in enumerate(curv):
                s = streams[i % 2]
                with torch.cuda.stream(s):
                    b.mfa_render_curvature(ctx, hc, w.camera, w.tf, ctf, w.params, outs[i],
                                           cnts[i], stream=s)
                    if i == 0:
                        b.mfa_render(ctx, hp, plain.camera, plain.tf, plain.params, out_p,
                                     cnts[2], stream=s)
            torch.cuda.synchronize()
            for i in range(2):
                assert np.array_equal(outs[i].cpu().numpy().astype(np.float64), ref_c[i][0]), \
                    f"repeat {rep}, curvature frame {i}"
                assert int(cnts[i].item()) == ref_c[i][1]
            assert np.array_equal(out_p.cpu().numpy().astype(np.float64), ref_p[0])
            assert int(cnts[2].item()) == ref_p[1]
            for o in outs + [out_p]:
                o.fill_(-1.0)
    finally:
        b.mfa_model_free(ctx, hc)
        b.mfa_model_free(ctx, hp)


def test_curvature_frames_are_timed(mfa):
    """Kernel timing records curvature frames like plain ones, without
    changing the image."""
    torch = torch_mod()
    b, ctx = mfa
    spec = _sphere_spec(57)
    wk = _workload(spec, size=32)
    ctf = wl.curvature_tf(16, 0.0, 2.5)
    h = b.mfa_model_upload(ctx, spec)
    try:
        ref, _ = gpu_curvature_render(b, ctx, h, wk, ctf)
        out = torch.zeros((32, 32, 4), dtype=torch.float32, device="cuda")
        b.mfa_kernel_timing(ctx, True)
        for _ in range(2):
            b.mfa_render_curvature(ctx, h, wk.camera, wk.tf, ctf, wk.params, out)
        b.mfa_render(ctx, h, wk.camera, wk.tf, wk.params, out)
        ms = b.mfa_kernel_times(ctx)
        b.mfa_kernel_timing(ctx, False)
        assert ms.shape == (3,) and np.all(ms > 0)
        b.mfa_render_curvature(ctx, h, wk.camera, wk.tf, ctf, wk.params, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
    finally:
        b.mfa_model_free(ctx, h)
