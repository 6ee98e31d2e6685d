"""Render or query workload for profiler runs (rocprofv3 kernel traces and
counter passes): a fixed number of identical launches of one kind, so that
every dispatch of the profiled kernel is of that kind.

``python -m paper_2204_11762_amd.profile_frames frame --store bf16 --ert on``
renders the 256^3 degree-3 frame (1024x1024, step 1/1024) ``--frames``
times after ``--warmup`` frames; ``--ert off`` renders it without early
termination, ``--shading off`` without gradient and shading.  ``eval``
runs value+gradient queries at 2^24 points of the same model, in random or
Morton order.  Each run prints, per launch kind, the samples (or points)
per launch and the mean duration of the ray-casting kernel (HIP events
around it on the launch stream), which the counter summaries divide by.
"""

from __future__ import annotations

import argparse
import copy
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

STORES = {"fp32": 0, "bf16": 1, "fp16": 2}
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
KERNEL_SOURCES = ["mfa_dev.h", "kernels_impl.h", "kernels.hip", "kernels_f32.hip",
                  "kernels_bf16.hip", "kernels_f16.hip"]


def source_hash() -> str:
    """SHA-256 over the device sources (names and contents, in a fixed
    order), so that a summary names what it profiled."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode() + b"\0")
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg: str) -> None:
    print(f"[profile] {msg}", flush=True)


def run_frames(args, b, ctx, wk) -> None:
    import torch
    prm = copy.copy(wk.params)
    if args.ert == "off":
        prm.ert_alpha = 1.0
    if args.shading == "off":
        prm.shading = False
    cam = wk.camera
    h = b.mfa_model_upload(ctx, wk.model, STORES[args.store])
    try:
        out = torch.zeros((cam.height, cam.width, 4), dtype=torch.float32, device="cuda")
        cnt = torch.zeros((1,), dtype=torch.int64, device="cuda")
        b.mfa_render(ctx, h, cam, wk.tf, prm, out, cnt)
        torch.cuda.synchronize()
        samples = int(cnt.item())
        for _ in range(args.warmup):
            b.mfa_render(ctx, h, cam, wk.tf, prm, out, None)
        torch.cuda.synchronize()
        b.mfa_kernel_timing(ctx, True)
        t0 = time.perf_counter()
        for _ in range(args.frames):
            b.mfa_render(ctx, h, cam, wk.tf, prm, out, None)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / max(1, args.frames)
        kern = b.mfa_kernel_times(ctx).astype(np.float64)
        b.mfa_kernel_timing(ctx, False)
        log(f"frame store={args.store} ert={args.ert} shading={args.shading}: "
            f"samples_per_launch {samples} launches {args.frames + args.warmup + 1} "
            f"kernel_mean_ms {kern.mean():.4f} kernel_min_ms {kern.min():.4f} "
            f"kernel_max_ms {kern.max():.4f} wall_ms {wall * 1e3:.4f}")
    finally:
        b.mfa_model_free(ctx, h)


def run_eval(args, b, ctx, wk) -> None:
    import torch
    from paper_2204_11762_amd import workloads as wl
    n = args.points
    xyz = wl.uniform_points(np.random.default_rng(9), n)
    if args.order == "morton":
        xyz = np.ascontiguousarray(xyz[wl.morton_order(xyz)])
    h = b.mfa_model_upload(ctx, wk.model, STORES[args.store])
    try:
        x = torch.from_numpy(xyz).cuda()
        v = torch.empty(n, dtype=torch.float32, device="cuda")
        g = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        for _ in range(args.warmup + 1):
            b.mfa_eval_points(ctx, h, x, v, g)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.frames):
            b.mfa_eval_points(ctx, h, x, v, g)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / max(1, args.frames)
        log(f"eval store={args.store} order={args.order}: points_per_launch {n} "
            f"launches {args.frames + args.warmup + 1} call_mean_ms {ms:.4f}")
    finally:
        b.mfa_model_free(ctx, h)


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("kind", choices=["frame", "eval"])
    ap.add_argument("--store", choices=list(STORES), default="bf16")
    ap.add_argument("--ert", choices=["on", "off"], default="on")
    ap.add_argument("--shading", choices=["on", "off"], default="on")
    ap.add_argument("--order", choices=["random", "morton"], default="random")
    ap.add_argument("--points", type=int, default=1 << 24)
    ap.add_argument("--frames", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    args = ap.parse_args()
    import torch

    from paper_2204_11762_amd import binding as b
    from paper_2204_11762_amd import workloads as wl
    assert torch.cuda.is_available(), "profiling runs need a GPU"
    log(f"kernel source sha256 {source_hash()}")
    wk = wl.c3()
    ctx = b.mfa_create(0)
    try:
        if args.kind == "frame":
            run_frames(args, b, ctx, wk)
        else:
            run_eval(args, b, ctx, wk)
    finally:
        b.mfa_destroy(ctx)


if __name__ == "__main__":
    main()
