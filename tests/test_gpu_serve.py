"""The render server (continuous batching): every request submitted into
the mix, from several host threads and at random times, gives the image and
sample count of the same request rendered alone; the byte budget and the
batch limit are respected; bad requests are refused at submission."""

from __future__ import annotations

import threading
import time

import numpy as np
import pytest

from gpu_helpers import gpu_render
from paper_2204_11762_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _requests(seed, n):
    """n requests over the four small mixed models (cameras re-drawn)."""
    models, base = wl.batch_mix_small(seed)
    rng = np.random.default_rng(seed + 100)
    reqs = []
    for i in range(n):
        r = base[i % len(base)]
        spec = models[r.model][0]
        lo, hi = np.asarray(spec.lo), np.asarray(spec.hi)
        ctr = tuple((lo + hi) / 2)
        ext = float(np.max(hi - lo))
        cam = r.camera
        if cam.kind == "persp":
            cam = wl.orbit_camera(cam.width, cam.height, float(rng.uniform(0, 360)),
                                  float(rng.uniform(-50, 50)), radius=2.2 * ext, target=ctr)
        reqs.append(wl.BatchRequest(r.model, cam, r.tf, r.params))
    return models, reqs


def _references(b, ctx, handles, models, reqs):
    refs = []
    for r in reqs:
        wk = wl.Workload("serve", models[r.model][0], r.camera, r.tf, r.params)
        refs.append(gpu_render(b, ctx, handles[r.model], wk))
    return refs


def _run_server(b, ctx, handles, reqs, threads=2, **cfg):
    import torch
    outs = [torch.full((r.camera.height, r.camera.width, 4), -1.0, dtype=torch.float32,
                       device="cuda") for r in reqs]
    cnts = [torch.full((1,), -7, dtype=torch.int64, device="cuda") for _ in reqs]
    torch.cuda.synchronize()
    server = b.mfa_server_create(ctx, **cfg)
    tickets = [None] * len(reqs)
    try:
        def submit(part, seed):
            rng = np.random.default_rng(seed)
            for i in part:
                time.sleep(float(rng.uniform(0, 2e-3)))
                r = reqs[i]
                tickets[i] = b.mfa_server_submit(server, handles[r.model], r.camera, r.tf,
                                                 r.params, outs[i], cnts[i])
        parts = [list(range(k, len(reqs), threads)) for k in range(threads)]
        ths = [threading.Thread(target=submit, args=(p, 7 + k)) for k, p in enumerate(parts)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        infos = [b.mfa_server_wait(server, t, -1) for t in tickets]
    finally:
        b.mfa_server_destroy(server)
    torch.cuda.synchronize()
    return outs, cnts, infos


def _upload(b, ctx, models):
    return [b.mfa_model_upload(ctx, spec, store) for spec, store in models]


def test_server_mix_equals_alone(mfa):
    b, ctx = mfa
    models, reqs = _requests(31, 24)
    handles = _upload(b, ctx, models)
    try:
        refs = _references(b, ctx, handles, models, reqs)
        outs, cnts, infos = _run_server(b, ctx, handles, reqs, threads=2, streams=2)
        sizes = [inf.batch_size for inf in infos]
        print(f"\n  batch sizes seen: {sorted(set(sizes))}")
        for i, (img, cnt) in enumerate(refs):
            assert np.array_equal(outs[i].cpu().numpy().astype(np.float64), img), f"request {i}"
            assert int(cnts[i].item()) == cnt, f"request {i} count"
            inf = infos[i]
            assert inf.status == b.MFA_OK
            assert inf.submit_ns <= inf.launch_ns <= inf.done_ns
            assert 1 <= inf.batch_size <= 24
    finally:
        for h in handles:
            b.mfa_model_free(ctx, h)


def test_server_budget_and_batch_limit(mfa):
    b, ctx = mfa
    models, reqs = _requests(32, 12)
    handles = _upload(b, ctx, models)
    try:
        refs = _references(b, ctx, handles, models, reqs)
        biggest = max(r.camera.width * r.camera.height for r in reqs) * 16
        # budget for about two requests in flight, at most three per batch
        outs, cnts, infos = _run_server(b, ctx, handles, reqs, threads=1, streams=1,
                                        max_batch=3, max_bytes=2 * biggest + 65536)
        assert max(inf.batch_size for inf in infos) <= 3
        for i, (img, cnt) in enumerate(refs):
            assert np.array_equal(outs[i].cpu().numpy().astype(np.float64), img), f"request {i}"
            assert int(cnts[i].item()) == cnt
    finally:
        for h in handles:
            b.mfa_model_free(ctx, h)


def test_server_errors(mfa):
    import copy

    import torch
    b, ctx = mfa
    models, reqs = _requests(33, 2)
    handles = _upload(b, ctx, models)
    r = reqs[0]
    out = torch.zeros((r.camera.height, r.camera.width, 4), dtype=torch.float32, device="cuda")
    try:
        server = b.mfa_server_create(ctx, max_bytes=1024)
        try:
            with pytest.raises(b.MFAError) as ei:       # larger than the whole budget
                b.mfa_server_submit(server, handles[r.model], r.camera, r.tf, r.params, out)
            assert ei.value.status == b.MFA_ERR_NOMEM
            p = copy.copy(r.params)
            p.step = 0.0
            with pytest.raises(b.MFAError) as ei:
                b.mfa_server_submit(server, handles[r.model], r.camera, r.tf, p, out)
            assert ei.value.status == b.MFA_ERR_INVALID
            with pytest.raises(b.MFAError) as ei:
                b.mfa_server_submit(server, 987654, r.camera, r.tf, r.params, out)
            assert ei.value.status == b.MFA_ERR_HANDLE
            with pytest.raises(b.MFAError) as ei:
                b.mfa_server_wait(server, 12345, 0)
            assert ei.value.status == b.MFA_ERR_HANDLE
        finally:
            b.mfa_server_destroy(server)
        with pytest.raises(b.MFAError):
            b.mfa_server_create(ctx, streams=9)
    finally:
        for h in handles:
            b.mfa_model_free(ctx, h)
