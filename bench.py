#!/usr/bin/env python3
"""Benchmark of the MFA ray caster on one MI355X.

A step is one frame: one launch of the fused render kernel over the whole
image (ray setup, span location, basis and derivatives, (p+1)^3 contraction
to value and gradient, transfer function, Phong shading, compositing with
early termination).  The workload is the 256^3-control-point degree-3 model
(least-squares fit plus N(0, 0.01^2) noise), 1024x1024 perspective frame,
step 1/1024, with the control points stored once in FP32 and once in BF16.

Printed: one JSON line with MFA samples/s (samples actually composited,
value + gradient each), frames/s, p50/p99 frame latency (HIP events on the
render stream), the roofline of the render kernel, and the FP64 CPU oracle
timed on this host on a bounded sample of the same frame (whose pixels also
give the accuracy of the GPU frame).
"""

from __future__ import annotations

import argparse
import copy
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2204_11762_amd import workloads as wl  # noqa: E402

METRIC = "MFA samples/s (value+grad) BF16 vs FP32 at stated err; p50/p99 frame latency"
PEAK_FP32_VALU = 157.3e12     # MI355X FP32 vector peak (packed issue)
PEAK_HBM = 8.0e12             # MI355X HBM3E bytes/s
CLOCK_HZ = 2.4e9              # MI355X peak engine clock
N_CU = 256                    # MI355X compute units
CSRC = os.path.join(ROOT, "paper_2204_11762_amd", "csrc")
# every source that the device code is compiled from
KERNEL_SOURCES = ["mfa_dev.h", "kernels_impl.h", "kernels.hip", "kernels_f32.hip",
                  "kernels_bf16.hip", "kernels_f16.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_256cubed_traffic.json")


def kernel_source_hash() -> str:
    """SHA-256 over the device sources (names and contents, in a fixed order)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode() + b"\0")
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(store: str):
    """HBM bytes per launch of the render kernel from the committed counter
    summary, or None if the summary was taken on different device sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    leg = rec.get("legs", {}).get(store)
    return None if leg is None else leg.get("hbm_bytes_per_launch")


def hbm_rate(traffic, kern_ms):
    """Measured HBM bytes per launch over the kernel's mean duration, against
    the 8 TB/s peak (None without a matching counter summary)."""
    if traffic is None or not kern_ms:
        return None
    gbps = traffic / (kern_ms * 1e-3) / 1e9
    return {"gb_per_s": gbps, "frac": gbps / (PEAK_HBM / 1e9)}


def lds_rate(p: int, samples: int, kern_ms):
    """Algorithmic LDS read bytes of the brick kernel: each composited sample
    gathers its (p+1)^3 control points (FP32 in LDS) and two transfer-function
    entries (16 B each).  Reported per compute unit and clock against the
    LDS's 128 bytes per clock."""
    if not kern_ms:
        return None
    per_sample = 4 * (p + 1) ** 3 + 32
    per_clk = samples * per_sample / (kern_ms * 1e-3 * CLOCK_HZ * N_CU)
    return {"bytes_per_sample": per_sample, "bytes_per_clk_per_cu": per_clk,
            "peak_bytes_per_clk_per_cu": 128, "frac": per_clk / 128}


def flops_per_sample(p: int) -> int:
    """Algorithmic FP32 operations per sample at degree p: sum-factorised
    contraction to value + 3 derivatives, basis and derivative triangles on
    three axes, and ~50 for position, transfer function, shading and
    compositing."""
    q = p + 1
    contraction = 2 * (2 * q ** 3 + 3 * q ** 2 + 4 * q)
    basis = 3 * (2 * p + 5 * p * (p + 1) // 2 + 3 * q)
    return contraction + basis + 50


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on host cores (before the GPU is touched)
# ---------------------------------------------------------------------------

_ORACLE_STATE = {}


def _oracle_chunk(pix):
    from oracle import raycast as orc
    M, cam, tf, prm = _ORACLE_STATE["args"]
    res = orc.render_pixels(M, cam, tf, prm, pix)
    return pix, res.rgba, res.samples


def cpu_baseline(wk, n_rays: int, seed: int, workers: int):
    import multiprocessing as mp

    from oracle import bspline as ob
    from oracle import raycast as orc
    m = wk.model
    M = ob.Model(tuple(m.degree), tuple(np.asarray(k) for k in m.knots), np.asarray(m.ctrl),
                 np.asarray(m.lo, float), np.asarray(m.hi, float))
    c = wk.camera
    cam = orc.Camera(c.kind, c.eye, c.target, c.up, c.width, c.height, c.fov_y_deg,
                     c.ortho_half_w, c.ortho_half_h)
    tf = orc.TransferFunction(wk.tf.table, wk.tf.v_lo, wk.tf.v_hi)
    p = wk.params
    prm = orc.RenderParams(step=p.step, ert_alpha=p.ert_alpha, shading=p.shading, ka=p.ka,
                           kd=p.kd, ks=p.ks, shininess=p.shininess, headlight=p.headlight,
                           light_dir=p.light_dir)
    # sample among the pixels whose ray meets the volume
    allpix = np.arange(c.width * c.height)
    r, cc = np.divmod(allpix, c.width)
    o, d = orc.camera_rays(cam, r, cc)
    t0, t1, hit = orc.slab(o, d, M.lo, M.hi)
    hits = np.nonzero(hit)[0]
    if n_rays < 0 or n_rays >= len(hits):
        pix = hits
    else:
        pix = np.sort(np.random.default_rng(seed).choice(hits, size=n_rays, replace=False))
    _ORACLE_STATE["args"] = (M, cam, tf, prm)
    chunks = np.array_split(pix, max(workers * 4, 1))
    t_start = time.perf_counter()
    if workers > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_oracle_chunk, chunks)
    else:
        parts = [_oracle_chunk(ch) for ch in chunks]
    wall = time.perf_counter() - t_start
    rgba = np.concatenate([q[1] for q in parts])
    samples = int(sum(q[2].sum() for q in parts))
    return {"pix": pix, "rgba": rgba, "samples": samples, "wall": wall}


FRAME_NAMES = {
    "c1": "16^3 p2 random control points, 128^2 orthographic, step 1/256 (every ray)",
    "c2": "64^3 p3 least-squares fit, 512^2 perspective, step 1/512 (every ray that meets "
          "the volume)",
}


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# GPU leg
# ---------------------------------------------------------------------------

def gpu_leg(b, ctx, wk, store: int, steps: int, warmup: int, log, nominal_frames=True,
            autotune=False):
    import torch
    cam = wk.camera
    h = b.mfa_model_upload(ctx, wk.model, store)
    try:
        out = torch.zeros((cam.height, cam.width, 4), dtype=torch.float32, device="cuda")
        cnt = torch.zeros((1,), dtype=torch.int64, device="cuda")
        tune = None
        if autotune:
            r = b.mfa_autotune(ctx, h, cam, wk.tf, wk.params, out, repeats=10)
            tune = {"round_spans": r.round_spans, "best_ms": r.best_ms, "default_ms": r.default_ms}
            log(f"autotune: {r.round_spans} spans per round ({r.best_ms:.4f} ms; "
                f"default {r.default_ms:.4f} ms)")
        b.mfa_render(ctx, h, cam, wk.tf, wk.params, out, cnt)
        torch.cuda.synchronize()
        samples = int(cnt.item())
        image = out.cpu().numpy()
        nominal_prm = copy.copy(wk.params)
        nominal_prm.ert_alpha = 1.0
        nominal = None
        if nominal_frames:
            b.mfa_render(ctx, h, cam, wk.tf, nominal_prm, out, cnt)
            torch.cuda.synchronize()
            nominal = int(cnt.item())
        for _ in range(warmup):
            b.mfa_render(ctx, h, cam, wk.tf, wk.params, out, None)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        b.mfa_kernel_timing(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ev0[i].record(stream)
            b.mfa_render(ctx, h, cam, wk.tf, wk.params, out, None, stream=stream)
            ev1[i].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # frame latency: events around the whole call (tile planning + kernel);
        # kernel duration: the library's events around the ray-casting kernel
        lat = np.array([a.elapsed_time(e) for a, e in zip(ev0, ev1)])  # ms
        kern = b.mfa_kernel_times(ctx).astype(np.float64)
        b.mfa_kernel_timing(ctx, False)
        assert len(kern) == steps, (len(kern), steps)
        # nominal (no termination) frames, a few, for the ERT-free rate
        nominal_ms = nominal_kern_ms = None
        if nominal_frames:
            nsteps = max(3, steps // 10)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            b.mfa_kernel_timing(ctx, True)
            e0.record(stream)
            for _ in range(nsteps):
                b.mfa_render(ctx, h, cam, wk.tf, nominal_prm, out, None, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            nominal_ms = e0.elapsed_time(e1) / nsteps
            nominal_kern_ms = float(b.mfa_kernel_times(ctx).astype(np.float64).mean())
            b.mfa_kernel_timing(ctx, False)
        log(f"store={('fp32', 'bf16', 'fp16')[store]}: {samples} samples/frame, "
            f"{wall / steps * 1e3:.3f} ms/frame wall, frame p50 {np.median(lat):.3f} ms, "
            f"render kernel mean {kern.mean():.4f} ms")
        return {"samples": samples, "nominal": nominal, "wall": wall, "lat": lat, "kern": kern,
                "tune": tune,
                "nominal_ms": nominal_ms, "nominal_kern_ms": nominal_kern_ms, "image": image,
                "model_bytes": b.mfa_model_bytes(ctx, h)}
    finally:
        b.mfa_model_free(ctx, h)


def batch_leg(b, ctx, steps: int, warmup: int, log):
    """The batching workload (64 requests over four resident BF16 models with
    Beta(2,5) knots, degrees 2/3/4/3, mixed image sizes): the same requests
    rendered one by one with mfa_render, as one batch, and as a replayed HIP
    graph of the batch, first with the default configuration, then after
    the autotuner has chosen each model's round length and lanes per ray
    (on the model's largest request of the batch) and the batch has been
    prepared again."""
    import torch
    models, reqs = wl.batch_config()
    p_of = [int(max(spec.degree)) for spec, _ in models]
    handles = [b.mfa_model_upload(ctx, spec, store) for spec, store in models]
    batch = None
    try:
        outs = [torch.zeros((r.camera.height, r.camera.width, 4), dtype=torch.float32,
                            device="cuda") for r in reqs]
        cnts = [torch.zeros((1,), dtype=torch.int64, device="cuda") for _ in reqs]
        breqs = [(handles[r.model], r.camera, r.tf, r.params, o, c)
                 for r, o, c in zip(reqs, outs, cnts)]
        batch = b.mfa_batch_create(ctx, breqs)
        b.mfa_batch_render(ctx, batch)
        torch.cuda.synchronize()
        per_req = [int(c.item()) for c in cnts]
        samples = sum(per_req)
        flops = sum(n * flops_per_sample(p_of[r.model]) for n, r in zip(per_req, reqs))
        stream = torch.cuda.current_stream()

        def timed(fn, n):
            e0 = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
            e1 = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(n):
                e0[i].record(stream)
                fn()
                e1[i].record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            return wall / n * 1e3, np.array([a.elapsed_time(z) for a, z in zip(e0, e1)])

        def one_by_one():
            for r, o, c in zip(reqs, outs, cnts):
                b.mfa_render(ctx, handles[r.model], r.camera, r.tf, r.params, o, c, stream=stream)

        def batched():
            b.mfa_batch_render(ctx, batch, stream=stream)

        def graph_of_batch():
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                b.mfa_batch_render(ctx, batch)
            for _ in range(warmup):
                g.replay()
            return g

        for _ in range(warmup):
            one_by_one()
            batched()
        seq_ms, seq_lat = timed(one_by_one, steps)
        bat_ms, bat_lat = timed(batched, steps)
        g = graph_of_batch()
        gr_ms, gr_lat = timed(g.replay, steps)
        del g
        log(f"batch: {len(reqs)} requests, {samples} samples; one by one {seq_ms:.3f} ms, "
            f"batch {bat_ms:.3f} ms, graph {gr_ms:.3f} ms")
        # autotune every model on its largest request, then prepare the batch again
        tuned = []
        for m, h in enumerate(handles):
            mine = [i for i, r in enumerate(reqs) if r.model == m]
            i = max(mine, key=lambda k: reqs[k].camera.width * reqs[k].camera.height)
            r = reqs[i]
            res = b.mfa_autotune(ctx, h, r.camera, r.tf, r.params, outs[i], repeats=5)
            tuned.append({"model": m, "degree": p_of[m], "round_spans": float(res.round_spans),
                          "lanes_per_ray": int(res.lanes_per_ray),
                          "candidates": int(res.candidates), "best_ms": float(res.best_ms),
                          "default_ms": float(res.default_ms)})
            log(f"autotune model {m} (p {p_of[m]}) on a {r.camera.width}x{r.camera.height} "
                f"request: {res.round_spans} spans, {res.lanes_per_ray} lanes per ray, "
                f"{res.best_ms:.4f} ms against {res.default_ms:.4f} ms by default")
        b.mfa_batch_free(ctx, batch)
        batch = None
        batch = b.mfa_batch_create(ctx, breqs)
        b.mfa_batch_render(ctx, batch)
        torch.cuda.synchronize()
        tuned_samples = sum(int(c.item()) for c in cnts)
        for _ in range(warmup):
            batched()
        tb_ms, tb_lat = timed(batched, steps)
        g = graph_of_batch()
        tg_ms, tg_lat = timed(g.replay, steps)
        del g
        log(f"tuned batch: {tuned_samples} samples; batch {tb_ms:.3f} ms, graph {tg_ms:.3f} ms")
        return {"workload": "64 requests, 4 BF16 models (Beta(2,5) knots; p 2/3/4/3; 32^3, "
                            "96x128x80, 128^3, 200x200x100), images {256^2, 512^2, 768x432, "
                            "1024^2}, step 1/512, random orbit cameras",
                "requests": len(reqs), "samples_per_batch": samples,
                "flops_per_batch": flops,
                "one_by_one": {"ms": seq_ms, "samples_per_s": samples / (seq_ms * 1e-3),
                               "p50_ms": float(np.percentile(seq_lat, 50)),
                               "p99_ms": float(np.percentile(seq_lat, 99))},
                "batch": {"ms": bat_ms, "samples_per_s": samples / (bat_ms * 1e-3),
                          "p50_ms": float(np.percentile(bat_lat, 50)),
                          "p99_ms": float(np.percentile(bat_lat, 99))},
                "graph": {"ms": gr_ms, "samples_per_s": samples / (gr_ms * 1e-3),
                          "p50_ms": float(np.percentile(gr_lat, 50)),
                          "p99_ms": float(np.percentile(gr_lat, 99)),
                          "tflops": flops / (gr_ms * 1e-3) / 1e12},
                "autotune": tuned,
                "tuned": {"samples_per_batch": tuned_samples,
                          "batch": {"ms": tb_ms, "samples_per_s": tuned_samples / (tb_ms * 1e-3),
                                    "p50_ms": float(np.percentile(tb_lat, 50)),
                                    "p99_ms": float(np.percentile(tb_lat, 99))},
                          "graph": {"ms": tg_ms, "samples_per_s": tuned_samples / (tg_ms * 1e-3),
                                    "p50_ms": float(np.percentile(tg_lat, 50)),
                                    "p99_ms": float(np.percentile(tg_lat, 99))},
                          "gain_over_one_by_one": seq_ms / tg_ms,
                          "gain_over_untuned_graph": gr_ms / tg_ms}}
    finally:
        if batch is not None:
            b.mfa_batch_free(ctx, batch)
        for h in handles:
            b.mfa_model_free(ctx, h)


def serve_leg(b, ctx, log, rate: float, duration: float, max_bytes: int):
    """The serving workload: requests submitted to the library's render
    server at their Poisson arrival times; throughput over the whole run and
    per-request latency (submission to completion).  The server admits
    requests within a device-byte budget (max_bytes); the requests it held
    back for it while a launch slot was free are counted."""
    import torch
    models, reqs, arrivals = wl.serve_config(rate=rate, duration_s=duration)
    p_of = [int(max(spec.degree)) for spec, _ in models]
    handles = [b.mfa_model_upload(ctx, spec, store) for spec, store in models]
    try:
        outs = [torch.empty((r.camera.height, r.camera.width, 4), dtype=torch.float32,
                            device="cuda") for r in reqs]
        cnt = torch.zeros((len(reqs),), dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        server = b.mfa_server_create(ctx, streams=2, max_batch=64, max_bytes=max_bytes)
        infos = []
        try:
            # a few requests first, so that the slots' buffers are sized
            warm = [b.mfa_server_submit(server, handles[r.model], r.camera, r.tf, r.params,
                                        outs[i], cnt[i:i + 1]) for i, r in enumerate(reqs[:8])]
            for t in warm:
                b.mfa_server_wait(server, t, -1)
            tickets = []
            t0 = time.perf_counter()
            for i, r in enumerate(reqs):
                delay = t0 + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets.append(b.mfa_server_submit(server, handles[r.model], r.camera, r.tf,
                                                   r.params, outs[i], cnt[i:i + 1]))
            infos = [b.mfa_server_wait(server, t, -1) for t in tickets]
        finally:
            b.mfa_server_destroy(server)
        per_req = cnt.cpu().numpy()
        samples = int(per_req.sum())
        flops = int(sum(int(n) * flops_per_sample(p_of[r.model]) for n, r in zip(per_req, reqs)))
        sub = np.array([inf.submit_ns for inf in infos], dtype=np.float64)
        done = np.array([inf.done_ns for inf in infos], dtype=np.float64)
        span = (done.max() - sub.min()) * 1e-9
        lat = (done - sub) * 1e-6
        bsz = np.array([inf.batch_size for inf in infos])
        deferred = int(sum(inf.deferred for inf in infos))
        log(f"serve: {len(reqs)} requests in {span:.2f} s, {samples} samples, "
            f"p50 {np.percentile(lat, 50):.2f} ms, p99 {np.percentile(lat, 99):.2f} ms, "
            f"mean batch {bsz.mean():.1f}, {deferred} held back by the "
            f"{max_bytes / 2**20:.0f} MiB budget")
        return {"workload": f"Poisson {rate:g} req/s for {duration:g} s over 16 resident models "
                            "(p 2-4, 32^3-256^3, FP32/BF16, uniform/Beta(2,5) knots); images "
                            "128^2-1920x1080, 128-1024 samples per unit length, per-request table",
                "requests": len(reqs), "offered_req_per_s": rate,
                "frames_per_s": len(reqs) / span, "samples_per_s": samples / span,
                "tflops": flops / span / 1e12, "samples": samples,
                "latency_p50_ms": float(np.percentile(lat, 50)),
                "latency_p99_ms": float(np.percentile(lat, 99)),
                "latency_max_ms": float(lat.max()), "mean_batch": float(bsz.mean()),
                "deferred_by_budget": deferred,
                "server": {"streams": 2, "max_batch": 64, "max_bytes": max_bytes}}
    finally:
        for h in handles:
            b.mfa_model_free(ctx, h)


def eval_leg(b, ctx, wk, steps: int, log, n_points: int = 1 << 24):
    """Value + gradient queries at n_points points of the 256^3 model
    (uniformly random, then sorted along a Morton curve).  Each entry gives
    the time per call and the rate of the query's own input and output
    (24 B position + 16 B value and gradient per point, and the control
    points once per call) against 8 TB/s: the sorted, binned evaluation
    reads each control point about twice per call, so the queries are bound
    by instruction issue (sorted input) or by the scattered position reads
    and result writes (random input), not by HBM bandwidth.  FP32 storage
    also times the second-derivative query (value, gradient and six second
    derivatives: 40 B of results per point)."""
    import torch
    xyz = wl.uniform_points(np.random.default_rng(9), n_points)
    orders = {"random": np.arange(n_points), "morton": wl.morton_order(xyz)}
    n_ctrl = int(np.prod(wk.model.ctrl.shape))

    def entry(ms, io_bytes):
        gbs = n_points * io_bytes / (ms * 1e-3) / 1e9
        return {"ms": ms, "points_per_s": n_points / (ms * 1e-3),
                "ns_per_point": ms * 1e6 / n_points, "io_bytes_per_point": io_bytes,
                "io_GBps": gbs, "io_frac_of_8TBps": gbs / 8000.0}

    out = {}
    for store, name in ((0, "fp32"), (1, "bf16")):
        h = b.mfa_model_upload(ctx, wk.model, store)
        try:
            elem = 4 if store == 0 else 2
            io = 24 + 16 + n_ctrl * elem / n_points
            for oname, perm in orders.items():
                x = torch.from_numpy(np.ascontiguousarray(xyz[perm])).cuda()
                v = torch.empty(n_points, dtype=torch.float32, device="cuda")
                g = torch.empty((n_points, 3), dtype=torch.float32, device="cuda")
                b.mfa_eval_points(ctx, h, x, v, g)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(steps):
                    b.mfa_eval_points(ctx, h, x, v, g)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / steps
                out[f"{name}_{oname}"] = entry(ms, io)
                log(f"eval {name} {oname}: {ms:.3f} ms for {n_points} points, "
                    f"{n_points / (ms * 1e-3):.3g} points/s")
                if store == 0:
                    hs = torch.empty((n_points, 6), dtype=torch.float32, device="cuda")
                    b.mfa_eval_hessian(ctx, h, x, v, hs, grad=g)
                    torch.cuda.synchronize()
                    e0.record()
                    for _ in range(steps):
                        b.mfa_eval_hessian(ctx, h, x, v, hs, grad=g)
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / steps
                    out[f"{name}_{oname}_hessian"] = entry(ms, io + 24)
                    log(f"eval {name} {oname} with second derivatives: {ms:.3f} ms")
                    del hs
                del x, v, g
        finally:
            b.mfa_model_free(ctx, h)
    out["points"] = n_points
    return out


def curvature_leg(b, ctx, wk, steps: int, log):
    """The render frame with a curvature transfer function (principal
    curvatures from the analytic Hessian colour the samples): FP32 storage,
    one lane per ray, timed around the whole call on the caller's stream."""
    import torch
    ctf = wl.curvature_tf(32, -60.0, 60.0)
    h = b.mfa_model_upload(ctx, wk.model, 0)
    try:
        W, H = wk.camera.width, wk.camera.height
        out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        b.mfa_render_curvature(ctx, h, wk.camera, wk.tf, ctf, wk.params, out, cnt)
        torch.cuda.synchronize()
        samples = int(cnt.item())
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            b.mfa_render_curvature(ctx, h, wk.camera, wk.tf, ctf, wk.params, out, cnt)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
    finally:
        b.mfa_model_free(ctx, h)
    log(f"curvature: {samples} samples in {ms:.3f} ms, {samples / (ms * 1e-3):.3e} samples/s")
    return {"store": "fp32", "samples_per_frame": samples, "ms_per_frame": ms,
            "samples_per_s": samples / (ms * 1e-3),
            "table": "32x32 over k1, k2 in [-60, 60]"}


def fields_leg(b, ctx, log, n_points: int = 1 << 22):
    """Sect. 4 shaped measurements on the Gaussian beam (Eq. 1) sampled on a
    128^3 grid: (i) point-query time against the number of control points
    and the degree (least-squares fits, n in {32, 64, 128}, p in 1..4);
    (ii) a 1000 x 1000 render of the fit with control points = data size and
    degree 2."""
    import torch
    data = wl.field_grid(wl.gaussian_beam, 128)
    rng = np.random.default_rng(17)
    xyz = torch.from_numpy(np.ascontiguousarray(
        wl.uniform_points(rng, n_points, wl.FIELD_LO, wl.FIELD_HI))).cuda()
    v = torch.empty(n_points, dtype=torch.float32, device="cuda")
    g = torch.empty((n_points, 3), dtype=torch.float32, device="cuda")
    sweep = []
    for n in (32, 64, 128):
        for p in (1, 2, 3, 4):
            spec = wl.fit_grid(data, n, p)
            h = b.mfa_model_upload(ctx, spec)
            try:
                b.mfa_eval_points(ctx, h, xyz, v, g)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(5):
                    b.mfa_eval_points(ctx, h, xyz, v, g)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / 5
            finally:
                b.mfa_model_free(ctx, h)
            sweep.append({"n": n, "p": p, "ns_per_query": ms * 1e6 / n_points,
                          "queries_per_s": n_points / (ms * 1e-3)})
    log("eval sweep (ns per value+gradient query): " + ", ".join(
        f"n{r['n']}p{r['p']} {r['ns_per_query']:.3f}" for r in sweep))
    # paper-shaped render: control points = data size, degree 2, 1000 x 1000
    spec = wl.fit_grid(data, 128, 2)
    e = np.arange(256) / 255.0
    table = np.stack([np.ones(256), np.zeros(256), np.zeros(256), 0.08 * e], axis=1)
    wk = wl.Workload("gaussian-beam", spec,
                     wl.orbit_camera(1000, 1000, 30.0, 20.0, radius=3.5, target=(0.0, 0.0, 0.0)),
                     wl.TFSpec(table.astype(np.float32), 0.0, 255.0), wl.ParamSpec(step=2.0 / 256))
    leg = gpu_leg(b, ctx, wk, 0, 50, 5, log, nominal_frames=False, autotune=False)
    render = {"workload": "Gaussian beam (Eq. 1) 128^3 samples, least-squares MFA with 128^3 "
                          "control points, degree 2, FP32; 1000x1000 perspective, step 1/128 of "
                          "the box, ramp opacity, Phong",
              "samples_per_frame": leg["samples"],
              "ms_per_frame": leg["wall"] / 50 * 1e3,
              "kernel_mean_ms": float(leg["kern"].mean()),
              "samples_per_s": leg["samples"] / (float(leg["kern"].mean()) * 1e-3)}
    return {"eval_sweep": sweep, "paper_shaped_render": render, "points": n_points}


def rmse_on(image, base):
    if base is None:
        return None
    got = image.reshape(-1, 4)[base["pix"]].astype(np.float64)
    err = got - base["rgba"]
    return {"rmse": float(np.sqrt((err ** 2).mean())), "max_abs": float(np.abs(err).max()),
            "pixels": int(len(base["pix"])), "reference": "FP64 oracle, ERT on"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--store", choices=["bf16", "fp32", "fp16"], default="bf16",
                    help="storage of the headline number (both are measured)")
    ap.add_argument("--cpu-rays", type=int, default=-1,
                    help="rays of the oracle's bounded sample: -1 = every ray that meets "
                         "the volume, 0 = skip the CPU leg")
    ap.add_argument("--no-nominal", action="store_true",
                    help="skip the frames without early termination (so that every render "
                         "launch of a profiled run is a timed-type frame)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes: 0 = the host CPUs this process may run on, at most "
                         "16 (the CPU share of one GPU on the measurement hosts)")
    ap.add_argument("--no-cpu-frames", action="store_true",
                    help="skip the oracle's full-frame timings of the small (128^2) and "
                         "production (512^2) frames")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (a plain copy "
                         "kernel of known traffic, for scaling HBM counters)")
    ap.add_argument("--legs", default="fp32,bf16,fp16", help="storages to measure")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="timed repetitions of the batching workload (0 = skip it)")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="duration of the served request stream (0 = skip it)")
    ap.add_argument("--serve-rate", type=float, default=400.0, help="requests per second")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner on each storage leg's frame before timing")
    ap.add_argument("--no-fields", action="store_true",
                    help="skip the closed-form field measurements")
    ap.add_argument("--eval-steps", type=int, default=10,
                    help="timed repetitions of the point-query micro-benchmark (0 = skip it)")
    ap.add_argument("--curvature-steps", type=int, default=5,
                    help="timed frames with the curvature transfer function (0 = skip them)")
    args = ap.parse_args()

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the ray caster would "
              "shard by image tiles across GPUs, which is not implemented.", file=sys.stderr)
        sys.exit(2)

    log(f"kernel source sha256 {kernel_source_hash()}")
    log("generating the 256^3 degree-3 workload")
    wk = wl.c3()
    p = int(max(wk.model.degree))

    base = None
    cores = 0
    if args.cpu_rays != 0:
        cores = args.cpu_workers or min(16, len(os.sched_getaffinity(0)))
        log(f"CPU oracle on {'all hit' if args.cpu_rays < 0 else args.cpu_rays} rays "
            f"with {cores} processes")
        base = cpu_baseline(wk, args.cpu_rays, args.seed, cores)
        log(f"CPU oracle: {base['samples']} samples in {base['wall']:.2f} s")
        if not args.no_cpu_frames:
            frames = {}
            for name, fw in (("c1", wl.c1()), ("c2", wl.c2())):
                r = cpu_baseline(fw, -1, args.seed, cores)
                frames[name] = {"workload": FRAME_NAMES[name], "rays": int(len(r["pix"])),
                                "samples": r["samples"], "wall_s": r["wall"],
                                "samples_per_s": r["samples"] / r["wall"]}
                log(f"CPU oracle, {name} frame: {r['samples']} samples in {r['wall']:.2f} s")
            base["frames"] = frames

    import torch

    from paper_2204_11762_amd import binding as b
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calib > 0:
        n = args.copy_calib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calib} MiB read + {args.copy_calib} MiB written")
        del src, dst
    ctx = b.mfa_create(0)
    try:
        legs = {}
        for name, store in (("fp32", 0), ("bf16", 1), ("fp16", 2)):
            if name in args.legs.split(","):
                legs[name] = gpu_leg(b, ctx, wk, store, args.steps, args.warmup, log,
                                     nominal_frames=not args.no_nominal, autotune=args.autotune)
        value_only = None
        if "bf16" in legs:
            # the same frame without shading: value queries only, no gradient
            wk_v = copy.copy(wk)
            wk_v.params = copy.copy(wk.params)
            wk_v.params.shading = False
            vleg = gpu_leg(b, ctx, wk_v, 1, max(20, args.steps // 4), 5, log, nominal_frames=False,
                           autotune=args.autotune)
            value_only = {"store": "bf16", "shading": False,
                          "samples_per_frame": vleg["samples"],
                          "samples_per_s": vleg["samples"] / (float(vleg["kern"].mean()) * 1e-3),
                          "kernel_mean_ms": float(vleg["kern"].mean()),
                          "note": "value only (no gradient, no Phong); a different frame, since "
                                  "unshaded colours change where rays terminate"}
        # the attainable FP32 vector rate without packed FP32 (micro-loop)
        fma_tflops = b.mfa_measure_fma_peak(ctx)
        log(f"FP32 FMA micro-loop: {fma_tflops:.1f} TFLOP/s")
        evals = None
        if args.eval_steps > 0:
            evals = eval_leg(b, ctx, wk, args.eval_steps, log)
        curvature = None
        if args.curvature_steps > 0:
            curvature = curvature_leg(b, ctx, wk, args.curvature_steps, log)
        fields = None if args.no_fields else fields_leg(b, ctx, log)
        batch = None
        if args.batch_steps > 0:
            batch = batch_leg(b, ctx, args.batch_steps, 2, log)
        serve = saturated = None
        if args.serve_seconds > 0:
            # a budget of 48 MiB in flight: one full-HD request (33 MB of
            # image) leaves room for smaller ones but not for a second one
            serve = serve_leg(b, ctx, log, args.serve_rate, args.serve_seconds, 48 << 20)
            # the same request mix offered 20 times faster: the server's
            # capacity, with a budget that still binds (a 64-request batch of
            # this mix holds about 1.1 GB of images)
            saturated = serve_leg(b, ctx, log, 20 * args.serve_rate, args.serve_seconds / 8,
                                  512 << 20)
    finally:
        b.mfa_destroy(ctx)
    if args.store not in legs:
        args.store = next(iter(legs))

    head = legs[args.store]
    fps = args.steps / head["wall"]
    value = head["samples"] * fps
    kern_ms = float(head["kern"].mean())
    flops = head["samples"] * flops_per_sample(p)
    achieved = flops / (kern_ms * 1e-3)

    def summary(leg, name):
        return {"store": name, "samples_per_frame": leg["samples"],
                "samples_per_s": leg["samples"] * args.steps / leg["wall"],
                "ms_per_frame": leg["wall"] / args.steps * 1e3,
                "p50_ms": float(np.percentile(leg["lat"], 50)),
                "p99_ms": float(np.percentile(leg["lat"], 99)),
                "kernel_mean_ms": float(leg["kern"].mean()),
                "autotune": leg["tune"],
                "nominal_samples_per_frame": leg["nominal"],
                "nominal_samples_per_s": (None if leg["nominal"] is None
                                          else leg["nominal"] / (leg["nominal_ms"] * 1e-3)),
                "model_bytes": leg["model_bytes"],
                "error": rmse_on(leg["image"], base)}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mfa-256^3-p3-1024x1024-persp-step1/1024 "
                               "(LS fit of sin6x cos5y sin7z + 0.3 exp(-40|r-0.5|^2) + N(0,0.01^2))",
                   "store": args.store, "degree": p, "image": [1024, 1024],
                   "step": wk.params.step, "ert_alpha": wk.params.ert_alpha,
                   "shading": "phong"},
        "frames_per_s": fps,
        "p50_ms": float(np.percentile(head["lat"], 50)),
        "p99_ms": float(np.percentile(head["lat"], 99)),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                     "traffic": measured_traffic(args.store),
                     "kernel": "render_brick_kernel<3,%d,shade,fast,eq,4>" % (
                         {"fp32": 0, "bf16": 1, "fp16": 2}[args.store]),
                     "kernel_ms": kern_ms, "flops_per_sample": flops_per_sample(p),
                     "flops_per_launch": flops,
                     "measured_fma_tflops": fma_tflops,
                     "frac_of_measured_fma": achieved / (fma_tflops * 1e12),
                     "hbm": hbm_rate(measured_traffic(args.store), kern_ms),
                     "lds": lds_rate(p, head["samples"], kern_ms),
                     "ert_off": None if head["nominal"] is None else {
                         "achieved": head["nominal"] * flops_per_sample(p)
                         / (head["nominal_kern_ms"] * 1e-3) / 1e12,
                         "frac": head["nominal"] * flops_per_sample(p)
                         / (head["nominal_kern_ms"] * 1e-3) / PEAK_FP32_VALU,
                         "kernel_ms": head["nominal_kern_ms"],
                         "call_ms": head["nominal_ms"],
                         "note": "the same frame with termination off (the configuration "
                                 "the VALU roofline fraction is defined on): composited "
                                 "samples x F(p) over the mean duration of the ray-casting "
                                 "kernel"}},
        "legs": {k: summary(v, k) for k, v in legs.items()},
    }
    if value_only is not None:
        line["value_only"] = value_only
    if curvature is not None:
        line["curvature"] = curvature
    if evals is not None:
        line["eval"] = evals
    if fields is not None:
        line["fields"] = fields
    if batch is not None:
        line["batch"] = batch
    if serve is not None:
        line["serve"] = serve
        line["serve_saturated"] = saturated
    if base is not None:
        line["cpu_baseline"] = {"value": base["samples"] / base["wall"], "unit": "samples/s",
                                "cores": cores,
                                "processes": cores,
                                "host_cpus_visible": len(os.sched_getaffinity(0)),
                                "per_process": base["samples"] / base["wall"] / cores,
                                "kind": "oracle",
                                "sample": f"{len(base['pix'])} rays of the same frame that meet the "
                                          f"volume, {base['samples']} samples, "
                                          f"{base['wall']:.1f} s wall",
                                "host_cpu": host_cpu_model(),
                                "full_frames": base.get("frames")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
