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



def test_server_two_waits_on_one_ticket(mfa):
    """Two host threads waiting for the same ticket: one receives the
    request's record, the other the error for an already waited-for ticket;
    neither is left waiting (each wait has a 10 s limit, so a wait that
    missed the other's hand-over shows up as a time-out, not a hang)."""
    import torch
    b, ctx = mfa
    models, reqs = _requests(35, 1)
    handles = _upload(b, ctx, models)
    r = reqs[0]
    out = torch.zeros((r.camera.height, r.camera.width, 4), dtype=torch.float32, device="cuda")
    try:
        server = b.mfa_server_create(ctx)
        try:
            results = [None, None]

            def wait(k, ticket):
                try:
                    results[k] = b.mfa_server_wait(server, ticket, 10_000_000)
                except b.MFAError as exc:
                    results[k] = exc.status

            for _ in range(3):
                t = b.mfa_server_submit(server, handles[r.model], r.camera, r.tf, r.params, out)
                ths = [threading.Thread(target=wait, args=(k, t)) for k in range(2)]
                for th in ths:
                    th.start()
                for th in ths:
                    th.join()
                infos = [x for x in results if isinstance(x, b.RequestInfo)]
                errors = [x for x in results if not isinstance(x, b.RequestInfo)]
                assert len(infos) == 1 and infos[0].status == b.MFA_OK, results
                assert errors == [b.MFA_ERR_HANDLE], results
        finally:
            b.mfa_server_destroy(server)
    finally:
        for h in handles:
            b.mfa_model_free(ctx, h)

# Requests shaped like the serving workload: (model of the serving set, image
# size, samples per unit length).  Models 9, 10, 11 and 15 are the 256^3 ones
# (p 2 FP32 Beta, p 3 BF16 uniform, p 4 BF16 Beta, p 2 BF16 Beta).
SERVE_MIX = [(10, (1920, 1080), 1024), (11, (1920, 1080), 1024), (9, (1280, 720), 512),
             (15, (1024, 768), 256), (7, (512, 512), 1024), (4, (128, 128), 128),
             (8, (256, 256), 512), (1, (1920, 1080), 128)]


def test_server_serving_mix_against_oracle(mfa):
    """Requests of the serving workload's shape (256^3 models in FP32 and
    BF16, uniform and Beta knots, degrees 2-4, images up to 1920x1080, up to
    1024 samples per unit length) served under a byte budget that holds the
    second full-HD request back while the first is in flight.  Each served
    image equals its solo render bit for bit, and sampled pixels match the
    FP64 oracle: FP32 models at the FP32 bar; BF16 models at the FP32 bar
    against the de-quantised model and at the BF16 bar against FP64."""
    import torch

    from gpu_helpers import BF16_RMSE, FP32_RMSE, compare_image
    from helpers import oracle_model, oracle_workload
    from oracle import quant
    from oracle import raycast as orc
    b, ctx = mfa
    models, _, _ = wl.serve_config()
    rng = np.random.default_rng(81)
    reqs = []
    for mi, (W, H), N in SERVE_MIX:
        P = models[mi][0].ctrl
        tf = wl.pwl_tf(int(rng.integers(1 << 30)), float(P.min()), float(P.max()))
        reqs.append(wl.BatchRequest(mi, wl.random_orbit_camera(rng, W, H), tf,
                                    wl.ParamSpec(step=1.0 / N)))
    used = sorted({r.model for r in reqs})
    handles = {mi: b.mfa_model_upload(ctx, *models[mi]) for mi in used}
    try:
        refs = [gpu_render(b, ctx, handles[r.model],
                           wl.Workload("serve", models[r.model][0], r.camera, r.tf, r.params))
                for r in reqs]
        outs = [torch.full((r.camera.height, r.camera.width, 4), -1.0, dtype=torch.float32,
                           device="cuda") for r in reqs]
        cnts = [torch.full((1,), -7, dtype=torch.int64, device="cuda") for _ in reqs]
        torch.cuda.synchronize()
        fhd = 1920 * 1080 * 16
        server = b.mfa_server_create(ctx, streams=2, max_batch=4, max_bytes=fhd * 3 // 2)
        try:
            tickets = [b.mfa_server_submit(server, handles[r.model], r.camera, r.tf, r.params,
                                           outs[i], cnts[i]) for i, r in enumerate(reqs)]
            infos = [b.mfa_server_wait(server, t, -1) for t in tickets]
        finally:
            b.mfa_server_destroy(server)
        torch.cuda.synchronize()
        assert sum(inf.deferred for inf in infos) >= 1, "the byte budget never held a request"
        for i, r in enumerate(reqs):
            spec, store = models[r.model]
            got = outs[i].cpu().numpy().astype(np.float64)
            cnt = int(cnts[i].item())
            assert np.array_equal(got, refs[i][0]), f"request {i}: served image differs"
            assert cnt == refs[i][1], f"request {i}: count"
            wk = wl.Workload("serve", spec, r.camera, r.tf, r.params)
            M, cam, _, prm = oracle_workload(wk)
            W, H = r.camera.width, r.camera.height
            rr, cc = np.divmod(np.arange(W * H), W)
            o, d = orc.camera_rays(cam, rr, cc)
            t0, t1, hit = orc.slab(o, d, M.lo, M.hi)
            nr = orc.sample_counts(t0, t1, hit, prm.step)
            assert (got.reshape(-1, 4)[nr == 0] == 0).all()
            prng = np.random.default_rng(90 + i)
            hits, misses = np.nonzero(nr > 0)[0], np.nonzero(nr == 0)[0]
            pix = np.sort(np.concatenate([
                prng.choice(hits, min(150, len(hits)), replace=False),
                prng.choice(misses, min(20, len(misses)), replace=False)]))
            if store == 0:
                rep = compare_image(got, cnt, wk, pix, 2e-5, 2e-4)
                msg = f"fp32 rmse {rep.rmse:.2e}"
                assert rep.rmse <= FP32_RMSE and rep.n_bad == 0, f"request {i}: {rep}"
            else:
                Mq = oracle_model(spec, ctrl=quant.dequant_bf16(spec.ctrl))
                rep = compare_image(got, cnt, wk, pix, 2e-5, 2e-4, model=Mq)
                assert rep.rmse <= FP32_RMSE and rep.n_bad == 0, f"request {i}: {rep}"
                rep64 = compare_image(got, cnt, wk, pix, 3e-3, 5e-2)
                assert rep64.rmse <= BF16_RMSE, f"request {i}: {rep64}"
                msg = f"bf16 rmse {rep.rmse:.2e} (de-quantised), {rep64.rmse:.2e} (FP64)"
            print(f"\n  request {i}: model {r.model} p{spec.degree[0]} {W}x{H} step 1/"
                  f"{round(1 / r.params.step)}, batch {infos[i].batch_size}, deferred "
                  f"{infos[i].deferred}: {msg}")
    finally:
        for h in handles.values():
            b.mfa_model_free(ctx, h)
