"""The ray caster with one, two and four lanes per ray (the configurations
the autotuner chooses between), through the C ABI: full small frames on
uniform and Beta knots and degrees 1-4 against the FP64 oracle, the
production-size model on sampled pixels, a batch mixing models of
different lanes per ray against their single renders, and the tuning
setter's argument checks."""

from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import FP32_RMSE, compare_image, gpu_render, small_workload
from helpers import oracle_model
from oracle import quant
from paper_2204_11762_amd import workloads as wl

pytestmark = pytest.mark.gpu

TAU32 = 2e-5
PX32 = 2e-4

CASES = [
    # (seed, n, degree, beta, lo, hi, image, kind, shading, ert, headlight)
    (1, (9, 8, 7), (3, 3, 3), False, (0, 0, 0), (1, 1, 1), (37, 29), "persp", True, 0.99, True),
    (2, (10, 9, 11), (2, 3, 1), True, (-1, 0, 0), (1, 1, 2), (40, 33), "persp", True, 0.95, False),
    (3, (8, 8, 8), (4, 4, 4), True, (0, 0, 0), (1, 1, 1), (23, 41), "ortho", True, 0.99, True),
    (6, (11, 12, 10), (2, 2, 2), False, (0, 0, 0), (1, 1, 1), (45, 38), "persp", False, 0.99, True),
]


@pytest.mark.parametrize("lanes", [1, 2])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_lanes_per_ray_small_frames(mfa, case, lanes):
    b, ctx = mfa
    spec, wk = small_workload(*CASES[case])
    W, H = wk.camera.width, wk.camera.height
    h = b.mfa_model_upload(ctx, spec)
    try:
        b.mfa_model_set_tuning(ctx, h, 3.0, lanes)
        img, cnt = gpu_render(b, ctx, h, wk)
        rep = compare_image(img, cnt, wk, np.arange(W * H), TAU32, PX32)
        print(f"\n  case {case}, {lanes} lanes per ray: rmse {rep.rmse:.2e} ambiguous "
              f"{rep.n_ambiguous} samples {rep.samples_gpu}/{rep.samples_ref}")
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
        assert abs(rep.samples_gpu - rep.samples_ref) <= rep.samples_slack
        assert (img >= 0).all()
    finally:
        b.mfa_model_free(ctx, h)


@pytest.mark.parametrize("lanes,spans", [(1, 1.5), (2, 6.0), (4, 2.0)])
def test_lanes_per_ray_production_model(mfa, lanes, spans):
    """The 64^3 degree-3 least-squares model (BF16) at 320x240 on sampled
    pixels: the FP32 bar against the de-quantised model."""
    b, ctx = mfa
    wk = wl.c2()
    wk.camera = wl.orbit_camera(320, 240, 130.0, 35.0)
    h = b.mfa_model_upload(ctx, wk.model, 1)
    try:
        b.mfa_model_set_tuning(ctx, h, spans, lanes)
        img, cnt = gpu_render(b, ctx, h, wk)
        pix = wl.pixel_subset(320, 240, 2500, seed=12)
        Mq = oracle_model(wk.model, ctrl=quant.dequant_bf16(wk.model.ctrl))
        rep = compare_image(img, cnt, wk, pix, TAU32, PX32, model=Mq)
        print(f"\n  c2 model, {lanes} lanes, {spans} spans: rmse {rep.rmse:.2e} "
              f"ambiguous {rep.n_ambiguous}")
        assert rep.rmse <= FP32_RMSE and rep.n_bad == 0
    finally:
        b.mfa_model_free(ctx, h)


def test_batch_mixes_lanes_per_ray(mfa):
    """Models tuned to different lanes per ray land in different batch
    classes; every request equals its single render bit for bit."""
    import torch
    b, ctx = mfa
    models, reqs = wl.batch_mix_small()
    handles = [b.mfa_model_upload(ctx, spec, store) for spec, store in models]
    lanes = [1, 2, 4, 1]
    outs, breqs = [], []
    batch = None
    try:
        for i, hdl in enumerate(handles):
            b.mfa_model_set_tuning(ctx, hdl, 3.0, lanes[i % len(lanes)])
        for r in reqs:
            out = torch.full((r.camera.height, r.camera.width, 4), -1.0, dtype=torch.float32,
                             device="cuda")
            cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
            outs.append((out, cnt))
            breqs.append((handles[r.model], r.camera, r.tf, r.params, out, cnt))
        batch = b.mfa_batch_create(ctx, breqs)
        b.mfa_batch_render(ctx, batch)
        torch.cuda.synchronize()
        for i, r in enumerate(reqs):
            wk = wl.Workload("batch", models[r.model][0], r.camera, r.tf, r.params)
            img, cnt = gpu_render(b, ctx, handles[r.model], wk)
            got = outs[i][0].cpu().numpy().astype(np.float64)
            assert np.array_equal(got, img), f"request {i}"
            assert int(outs[i][1].item()) == cnt
    finally:
        if batch is not None:
            b.mfa_batch_free(ctx, batch)
        for hdl in handles:
            b.mfa_model_free(ctx, hdl)


def test_set_tuning_errors(mfa):
    b, ctx = mfa
    spec, _ = small_workload(*CASES[0])
    h = b.mfa_model_upload(ctx, spec)
    try:
        for spans, lanes in ((3.0, 3), (3.0, 8), (0.1, 4), (40.0, 2), (float("nan"), 4)):
            with pytest.raises(b.MFAError) as ei:
                b.mfa_model_set_tuning(ctx, h, spans, lanes)
            assert ei.value.status == b.MFA_ERR_INVALID
        with pytest.raises(b.MFAError) as ei:
            b.mfa_model_set_tuning(ctx, 987654, 3.0, 4)
        assert ei.value.status == b.MFA_ERR_HANDLE
    finally:
        b.mfa_model_free(ctx, h)
