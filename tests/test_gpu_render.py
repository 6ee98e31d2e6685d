"""GPU parity of the ray caster (mfa_render) against the FP64 oracle, through
the C ABI: full frames at small sizes with ragged tiles, the c1 and c2
frames in full (with and without termination), and the 4096-pixel subset of
c3 in FP32 and BF16 storage."""

import copy

import numpy as np
import pytest

from gpu_helpers import (BF16_REL, BF16_RMSE, F16_RMSE, FP32_REL, FP32_RMSE, compare_image, gpu_eval,
                         gpu_render, normwise, oracle_on_pixels, small_workload)
from helpers import oracle_workload, oracle_model
from oracle import bspline as ob
from oracle import quant
from oracle import raycast as orc
from paper_2204_11762_amd import workloads as wl

pytestmark = pytest.mark.gpu

TAU32 = 2e-5      # band around the termination threshold for FP32 opacity
PX32 = 2e-4       # per-pixel sanity bound (RMSE is the criterion)


def _report(tag, rep):
    print(f"\n  {tag}: rmse {rep.rmse:.3e} max {rep.max_abs:.3e} ambiguous {rep.n_ambiguous} "
          f"bad {rep.n_bad} samples gpu {rep.samples_gpu} ref {rep.samples_ref} "
          f"slack {rep.samples_slack}")


def _check_counts(rep, pix_is_full):
    if pix_is_full:
        assert abs(rep.samples_gpu - rep.samples_ref) <= rep.samples_slack


def test_c1_full_frame(mfa):
    b, ctx = mfa
    wk = wl.c1()
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        img, cnt = gpu_render(b, ctx, h, wk)
        pix = np.arange(128 * 128)
        rep = compare_image(img, cnt, wk, pix, TAU32, PX32)
        _report("c1", rep)
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        _check_counts(rep, True)
        # no termination: continuous, nominal 256 samples per ray
        p2 = copy.copy(wk.params)
        p2.ert_alpha = 1.0
        img2, cnt2 = gpu_render(b, ctx, h, wk, p2)
        assert cnt2 == 256 * 128 * 128
        wk2 = copy.copy(wk)
        wk2.params = p2
        rep2 = compare_image(img2, cnt2, wk2, pix, TAU32, PX32)
        _report("c1 no-ERT", rep2)
        # without termination the image is a continuous function of the
        # samples: FP32 rounding only
        assert rep2.rmse <= 1e-6 and rep2.n_bad == 0
    finally:
        b.mfa_model_free(ctx, h)


SMALL = [
    # (seed, n, degree, beta, lo, hi, image, kind, shading, ert, headlight)
    (1, (9, 8, 7), (3, 3, 3), False, (0, 0, 0), (1, 1, 1), (37, 29), "persp", True, 0.99, True),
    (2, (10, 9, 11), (2, 3, 1), True, (-1, 0, 0), (1, 1, 2), (40, 33), "persp", True, 0.95, False),
    (3, (8, 8, 8), (4, 4, 4), True, (0, 0, 0), (1, 1, 1), (23, 41), "ortho", True, 0.99, True),
    (4, (7, 9, 6), (1, 1, 1), False, (0, 0, 0), (1, 1, 1), (31, 31), "persp", False, 0.99, True),
    (5, (12, 10, 9), (3, 4, 2), True, (0, 0, 0), (2, 1, 1), (48, 17), "persp", True, 1.5, True),
]


@pytest.mark.parametrize("case", range(len(SMALL)))
@pytest.mark.parametrize("store", [0, 1, 2])
def test_small_full_frames(mfa, case, store):
    spec, wk = small_workload(*SMALL[case])
    W, H = wk.camera.width, wk.camera.height
    b, ctx = mfa
    h = b.mfa_model_upload(ctx, spec, store)
    try:
        img, cnt = gpu_render(b, ctx, h, wk)
        pix = np.arange(W * H)
        if store == 0:
            rep = compare_image(img, cnt, wk, pix, TAU32, PX32)
            _report(f"small{case} fp32", rep)
            assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
            _check_counts(rep, True)
        else:
            name = "bf16" if store == 1 else "f16"
            deq = quant.dequant_bf16 if store == 1 else quant.dequant_f16
            # arithmetic error only: against the de-quantised model
            Mq = oracle_model(spec, ctrl=deq(spec.ctrl))
            rep = compare_image(img, cnt, wk, pix, TAU32, PX32, model=Mq)
            _report(f"small{case} {name} vs dequantised", rep)
            assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
            # and the total error against the FP64 model
            rep = compare_image(img, cnt, wk, pix, 3e-3, 5e-2)
            _report(f"small{case} {name} vs fp64", rep)
            assert rep.rmse <= (BF16_RMSE if store == 1 else F16_RMSE)
        # misses are exactly transparent black, and nothing is left unwritten
        M, c, _, p = oracle_workload(wk)
        r, cc = np.divmod(pix, W)
        o, d = orc.camera_rays(c, r, cc)
        t0, t1, hit = orc.slab(o, d, M.lo, M.hi)
        nr = orc.sample_counts(t0, t1, hit, p.step)
        flat = img.reshape(-1, 4)
        assert (flat[nr == 0] == 0).all()
        assert (flat >= 0).all()
    finally:
        b.mfa_model_free(ctx, h)


@pytest.mark.parametrize("store", [0, 1])
def test_rational_full_frames(mfa, store):
    """Rational models (random positive weights) on the global-memory ray
    caster, full frames against the oracle on the stored homogeneous values."""
    b, ctx = mfa
    rng = np.random.default_rng(60 + store)
    spec = wl.random_model(rng, n=(9, 8, 10), degree=(3, 2, 3), beta_knots=True)
    spec.weights = rng.uniform(0.3, 3.0, spec.ctrl.shape)
    cam = wl.orbit_camera(45, 37, 120.0, 25.0, radius=2.2)
    P = np.asarray(spec.ctrl)
    tf = wl.pwl_tf(9, P.min(), P.max(), alpha_max=0.15)
    prm = wl.ParamSpec(step=1.0 / 97.0, light_dir=(0.3, -0.5, 0.8))
    wk = wl.Workload("rational", spec, cam, tf, prm)
    deq = quant.dequant_f32 if store == 0 else quant.dequant_bf16
    wq = deq(spec.weights)
    Mq = oracle_model(spec, ctrl=deq(spec.weights * spec.ctrl) / wq)
    Mq.weights = wq
    h = b.mfa_model_upload(ctx, spec, store)
    try:
        img, cnt = gpu_render(b, ctx, h, wk)
        rep = compare_image(img, cnt, wk, np.arange(45 * 37), TAU32, PX32, model=Mq)
        _report(f"rational store {store}", rep)
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        _check_counts(rep, True)
    finally:
        b.mfa_model_free(ctx, h)


def test_determinism_and_stream(mfa):
    import torch
    b, ctx = mfa
    wk = wl.c2()
    wk.camera.width = wk.camera.height = 200
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        a1, c1 = gpu_render(b, ctx, h, wk)
        s = torch.cuda.Stream()
        out = torch.zeros((200, 200, 4), dtype=torch.float32, device="cuda")
        cnt = torch.zeros((1,), dtype=torch.int64, device="cuda")
        with torch.cuda.stream(s):
            b.mfa_render(ctx, h, wk.camera, wk.tf, wk.params, out, cnt, stream=s)
        s.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.float64), a1)
        assert int(cnt.item()) == c1
    finally:
        b.mfa_model_free(ctx, h)


def test_concurrent_streams(mfa):
    """Frames of different sizes and views enqueued on two streams without
    synchronising in between (so their planning and ray casting can
    overlap on the device) equal their solo renders bit for bit."""
    import copy

    import torch
    b, ctx = mfa
    wk = wl.c2()
    views = []
    for w, az in ((320, 30.0), (256, 75.0), (384, 150.0), (200, 250.0)):
        v = copy.copy(wk)
        v.camera = wl.orbit_camera(w, w, az, 20.0)
        views.append(v)
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        ref = [gpu_render(b, ctx, h, v) for v in views]
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        outs = [torch.zeros((v.camera.height, v.camera.width, 4), dtype=torch.float32,
                            device="cuda") for v in views]
        cnts = [torch.zeros((1,), dtype=torch.int64, device="cuda") for _ in views]
        torch.cuda.synchronize()
        for rep in range(3):
            for i, v in enumerate(views):
                s = streams[i % 2]
                with torch.cuda.stream(s):
                    b.mfa_render(ctx, h, v.camera, v.tf, v.params, outs[i], cnts[i], stream=s)
            torch.cuda.synchronize()
            for i in range(len(views)):
                assert np.array_equal(outs[i].cpu().numpy().astype(np.float64), ref[i][0]), \
                    f"repeat {rep}, view {i}"
                assert int(cnts[i].item()) == ref[i][1]
                outs[i].fill_(-1.0)
    finally:
        b.mfa_model_free(ctx, h)


def test_frame_sequence_one_stream(mfa):
    """Frames of changing size enqueued back to back on one fresh stream
    (the planning scratch grows between them, and consecutive frames plan
    with alternating counter sets) equal the same frames rendered each as
    the first frame of a fresh context, bit for bit, and write every pixel."""
    import torch
    b, ctx = mfa
    wk = wl.c2()
    sizes = (96, 96, 300, 64, 300, 300, 130, 96, 417)
    views = []
    for k, w in enumerate(sizes):
        v = copy.copy(wk)
        v.camera = wl.orbit_camera(w, w - 7 * (k % 3), 40.0 * k, 15.0)
        views.append(v)
    ref = []
    for v in views:
        c2 = b.mfa_create(0)
        try:
            h2 = b.mfa_model_upload(c2, wk.model)
            ref.append(gpu_render(b, c2, h2, v))
        finally:
            b.mfa_destroy(c2)
        assert (ref[-1][0] >= 0.0).all()
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        s = torch.cuda.Stream()
        outs = [torch.full((v.camera.height, v.camera.width, 4), -1.0, dtype=torch.float32,
                           device="cuda") for v in views]
        cnts = [torch.zeros((1,), dtype=torch.int64, device="cuda") for _ in views]
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            for i, v in enumerate(views):
                b.mfa_render(ctx, h, v.camera, v.tf, v.params, outs[i], cnts[i], stream=s)
        s.synchronize()
        for i in range(len(views)):
            assert np.array_equal(outs[i].cpu().numpy().astype(np.float64), ref[i][0]), f"frame {i}"
            assert int(cnts[i].item()) == ref[i][1], f"frame {i}"
    finally:
        b.mfa_model_free(ctx, h)


def test_kernel_timing(mfa):
    """The optional kernel events time every render while enabled, leave the
    image unchanged, and record nothing once disabled."""
    import time

    import torch
    b, ctx = mfa
    wk = wl.c2()
    wk.camera.width = wk.camera.height = 200
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        ref, _ = gpu_render(b, ctx, h, wk)
        out = torch.zeros((200, 200, 4), dtype=torch.float32, device="cuda")
        b.mfa_kernel_timing(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            b.mfa_render(ctx, h, wk.camera, wk.tf, wk.params, out)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
        ms = b.mfa_kernel_times(ctx)
        assert ms.shape == (3,) and np.all(ms > 0) and ms.sum() <= wall_ms
        assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
        assert b.mfa_kernel_times(ctx).shape == (0,)      # cleared by the read
        b.mfa_kernel_timing(ctx, False)
        b.mfa_render(ctx, h, wk.camera, wk.tf, wk.params, out)
        assert b.mfa_kernel_times(ctx).shape == (0,)
    finally:
        b.mfa_kernel_timing(ctx, False)
        b.mfa_model_free(ctx, h)


def test_autotune_keeps_parity(mfa):
    """The autotuner picks one of its candidate configurations (round
    length and lanes per ray), never one slower than the default it timed,
    and renders after tuning still match the oracle."""
    import torch
    b, ctx = mfa
    wk = wl.c2()
    wk.camera.width = wk.camera.height = 256
    h = b.mfa_model_upload(ctx, wk.model, 1)
    try:
        scratch = torch.zeros((256, 256, 4), dtype=torch.float32, device="cuda")
        res = b.mfa_autotune(ctx, h, wk.camera, wk.tf, wk.params, scratch, repeats=3)
        print(f"\n  tuned round spans {res.round_spans}, {res.lanes_per_ray} lanes per ray, "
              f"{res.candidates} candidates, best {res.best_ms:.4f} ms, "
              f"default {res.default_ms:.4f} ms")
        assert res.candidates == 15
        assert res.round_spans in (1.5, 2.0, 3.0, 4.0, 6.0)
        assert res.lanes_per_ray in (1, 2, 4)
        assert 0 < res.best_ms <= res.default_ms
        img, cnt = gpu_render(b, ctx, h, wk)
        pix = wl.pixel_subset(256, 256, 1500, seed=8)
        Mq = oracle_model(wk.model, ctrl=quant.dequant_bf16(wk.model.ctrl))
        rep = compare_image(img, cnt, wk, pix, TAU32, PX32, model=Mq, count_exact=False)
        _report("autotuned c2 256^2 bf16", rep)
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        with pytest.raises(b.MFAError) as ei:
            b.mfa_autotune(ctx, h, wk.camera, wk.tf, wk.params, scratch, repeats=0)
        assert ei.value.status == b.MFA_ERR_INVALID
    finally:
        b.mfa_model_free(ctx, h)


def test_camera_inside_volume(mfa):
    b, ctx = mfa
    wk = wl.c2()
    wk.camera = wl.CameraSpec("persp", (0.45, 0.5, 0.55), (0.9, 0.6, 0.2), (0, 1, 0), 64, 48,
                              fov_y_deg=70.0)
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        img, cnt = gpu_render(b, ctx, h, wk)
        rep = compare_image(img, cnt, wk, np.arange(64 * 48), TAU32, PX32)
        _report("inside", rep)
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        _check_counts(rep, True)
    finally:
        b.mfa_model_free(ctx, h)


OFF_IMAGE_CASES = {
    # the box small in a wide view: most pixels miss it
    "distant": wl.CameraSpec("persp", (3.5, 2.9, 6.2), (0.5, 0.5, 0.5), (0, 1, 0), 160, 120,
                             fov_y_deg=40.0),
    # the box across the image border
    "edge": wl.CameraSpec("persp", (0.5, 0.6, 2.6), (1.25, 0.9, 0.5), (0, 1, 0), 144, 100,
                          fov_y_deg=50.0),
    # every corner in front of the eye, the box beside the view: every ray misses
    "beside": wl.CameraSpec("persp", (0.5, 0.5, 4.0), (4.0, 0.5, 0.0), (0, 1, 0), 96, 64,
                            fov_y_deg=30.0),
    # orthographic window much wider than the box
    "ortho": wl.CameraSpec("ortho", (0.5, 0.5, 3.0), (0.5, 0.5, 0.0), (0, 1, 0), 128, 96,
                           ortho_half_w=1.6, ortho_half_h=1.2),
}


@pytest.mark.parametrize("name", sorted(OFF_IMAGE_CASES))
def test_box_partly_or_wholly_off_image(mfa, name):
    """Frames in which most rays, or all, miss the box: the full image and
    the sample count equal the oracle's, and every missing ray gives
    transparent black."""
    b, ctx = mfa
    wk = wl.c2()
    wk.camera = OFF_IMAGE_CASES[name]
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        W, H = wk.camera.width, wk.camera.height
        img, cnt = gpu_render(b, ctx, h, wk)
        rep = compare_image(img, cnt, wk, np.arange(W * H), TAU32, PX32)
        _report(f"off-image {name}", rep)
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        _check_counts(rep, True)
        M, cam, _, p = oracle_workload(wk)
        r, c = np.divmod(np.arange(W * H), W)
        o, d = orc.camera_rays(cam, r, c)
        t0, t1, hit = orc.slab(o, d, M.lo, M.hi)
        nr = orc.sample_counts(t0, t1, hit, p.step)
        assert (img.reshape(-1, 4)[nr == 0] == 0).all()
        if name == "beside":
            assert (nr == 0).all() and cnt == 0 and (img == 0).all()
        else:
            assert (nr > 0).sum() > 100
    finally:
        b.mfa_model_free(ctx, h)


def test_c2_full_frame(mfa):
    """The production-size frame (64^3 cubic fit, 512^2 perspective, step
    1/512) in full: every pixel against the oracle, and the frame's sample
    count equal to the oracle's apart from the slack of the pixels whose
    termination is ambiguous in FP32."""
    b, ctx = mfa
    wk = wl.c2()
    h = b.mfa_model_upload(ctx, wk.model)
    try:
        img, cnt = gpu_render(b, ctx, h, wk)
        pix = np.arange(512 * 512)
        rep = compare_image(img, cnt, wk, pix, TAU32, PX32)
        _report("c2 full frame", rep)
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        _check_counts(rep, True)
        # and without termination: continuous, the count is the nominal one
        p2 = copy.copy(wk.params)
        p2.ert_alpha = 1.0
        img2, cnt2 = gpu_render(b, ctx, h, wk, p2)
        wk2 = copy.copy(wk)
        wk2.params = p2
        ref2 = oracle_on_pixels(wk2, pix)
        err2 = img2.reshape(-1, 4) - ref2.rgba
        rmse2 = float(np.sqrt((err2 ** 2).mean()))
        print(f"\n  c2 full frame no-ERT: rmse {rmse2:.3e} max {np.abs(err2).max():.3e} "
              f"samples gpu {cnt2} ref {int(ref2.samples.sum())}")
        assert rmse2 <= 1e-6 and np.abs(err2).max() <= PX32
        assert cnt2 == int(ref2.samples.sum()) == int(ref2.n_nominal.sum())
    finally:
        b.mfa_model_free(ctx, h)


@pytest.fixture(scope="module")
def c3():
    return wl.c3()


def _subset_sample_positions(wk, every=5):
    """World positions of the oracle's samples on the subset rays (every
    ``every``-th sample), for value/gradient parity at those positions."""
    M, cam, _, p = oracle_workload(wk)
    pix = wk.subset
    r, c = np.divmod(pix, cam.width)
    o, d = orc.camera_rays(cam, r, c)
    t0, t1, hit = orc.slab(o, d, M.lo, M.hi)
    nr = orc.sample_counts(t0, t1, hit, p.step)
    pts = []
    for i in np.nonzero(nr > 0)[0]:
        s = np.arange(0, nr[i], every)
        t = t0[i] + (s + 0.5) * p.step
        pts.append(o[i] + t[:, None] * d[i])
    return np.concatenate(pts)


@pytest.mark.parametrize("store", [0, 1])
def test_c3_subset(mfa, c3, store):
    b, ctx = mfa
    wk = c3
    h = b.mfa_model_upload(ctx, wk.model, store)
    try:
        # value / gradient at the oracle's sample positions
        xyz = _subset_sample_positions(wk)
        f, g = gpu_eval(b, ctx, h, xyz)
        M = oracle_model(wk.model)
        F = np.empty(len(xyz))
        G = np.empty((len(xyz), 3))
        for i in range(0, len(xyz), 100000):
            F[i:i + 100000], G[i:i + 100000] = ob.eval_world(M, xyz[i:i + 100000])
        ev, eg = normwise(f, F), normwise(g, G)
        print(f"\n  c3 store={store}: value rel {ev:.3e} grad rel {eg:.3e} at {len(xyz)} positions")
        img, cnt = gpu_render(b, ctx, h, wk)
        if store == 0:
            assert ev <= FP32_REL and eg <= FP32_REL
            rep = compare_image(img, cnt, wk, wk.subset, TAU32, PX32)
            _report("c3 fp32", rep)
            assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        else:
            assert ev <= BF16_REL
            rep = compare_image(img, cnt, wk, wk.subset, 3e-3, 5e-2)
            _report("c3 bf16 vs fp64", rep)
            assert rep.rmse <= BF16_RMSE
    finally:
        b.mfa_model_free(ctx, h)


@pytest.mark.parametrize("variant", ["large_tf", "coarse_step"])
@pytest.mark.parametrize("store", [0, 1])
def test_fallback_paths(mfa, variant, store):
    """A 2048-entry table leaves no LDS room for bricks (global-memory
    kernel); a step of several knot spans makes every round's brick exceed
    its capacity (rounds gather from global memory)."""
    rng = np.random.default_rng(31)
    if variant == "large_tf":
        spec = wl.random_model(rng, n=(14, 12, 13), degree=(3, 3, 3))
        P = np.asarray(spec.ctrl)
        tf = wl.pwl_tf(7, P.min(), P.max(), n=2048, alpha_max=0.1)
        step = 1 / 90
    else:
        spec = wl.random_model(rng, n=(160, 150, 170), degree=(2, 3, 2), smooth=True)
        P = np.asarray(spec.ctrl)
        tf = wl.pwl_tf(8, P.min(), P.max(), alpha_max=0.1)
        step = 1 / 12
    cam = wl.orbit_camera(45, 38, 40.0, 25.0)
    wk = wl.Workload(variant, spec, cam, tf, wl.ParamSpec(step=step))
    b, ctx = mfa
    h = b.mfa_model_upload(ctx, spec, store)
    try:
        img, cnt = gpu_render(b, ctx, h, wk)
        model = None if store == 0 else oracle_model(spec, ctrl=quant.dequant_bf16(spec.ctrl))
        rep = compare_image(img, cnt, wk, np.arange(45 * 38), TAU32, PX32, model=model)
        _report(f"{variant} store={store}", rep)
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        _check_counts(rep, True)
    finally:
        b.mfa_model_free(ctx, h)
