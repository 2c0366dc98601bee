#!/usr/bin/env python3
"""Benchmark: full four-quadrant FHT of a 4096 x 4096 float32 image on one GPU.

One step = one full forward transform (all four quadrants, merged full Hough
image of 16381 x 8192 float32) of a synthetic, seeded image already resident
in HBM.  Prints one JSON line:
  value        input Gpixels/s of the forward (4096^2 pixels per step)
  fwd_adjoint  Gpixels/s of forward + adjoint (the backward of the transform)
  batched      Gpixels/s of the batched forward over 8 such images
  roofline     the dominant kernel against the 8 TB/s HBM roof
  cpu_baseline the CPU oracle on this host's cores (bounded sample)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def _timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def cpu_baseline(img, target_s: float = 10.0):
    """The CPU oracle (float64 stage recurrence, OpenMP over rows) on the same
    4096^2 image: repeated full transforms until about target_s seconds."""
    import oracle

    x = img.astype("float64")
    reps, total = 0, 0.0
    while total < target_s and reps < 8:
        t = time.perf_counter()
        oracle.full(x)
        total += time.perf_counter() - t
        reps += 1
    px = x.shape[0] * x.shape[1] * reps
    return {"value": round(px / total / 1e9, 6), "unit": "Gpixels/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "%d full float64 transform(s) of the same 4096x4096 image, %.1f s" % (reps, total)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--fwd-only", action="store_true", help="time only the forward (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the transform shards "
              "by image, quadrant or column band; see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1811_06378_amd import fht, synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(max(1, args.steps)):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "launches": max(1, args.steps)}))
        return
    side = 4096
    img_np = synth.dense4096(0, size=side)
    x = torch.from_numpy(img_np).cuda()
    rows, cols = fht.hough_shape(side, side)
    out = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
    ws = torch.empty(max(fht.workspace_size(side, side, "full", torch.float32), 256), dtype=torch.uint8,
                     device="cuda")
    print("bench: forward %dx%d float32 -> %dx%d, %d steps after %d warmup" % (side, side, rows, cols, args.steps,
                                                                             args.warmup), file=sys.stderr, flush=True)

    ms_fwd, wall_fwd = _timed(lambda: fht.forward(x, out=out, workspace=ws), args.steps, args.warmup, torch)
    px = side * side
    value = px / (ms_fwd * 1e-3) / 1e9

    result = {
        "metric": "Gpixels/s full 4-quadrant FHT 4096^2 (fwd, fwd+adjoint, batched); % HBM peak",
        "value": round(value, 3),
        "unit": "Gpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_fwd, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Exp(1) image with 16 planted lines)",
        "config": {"workload": "dense4096", "image": [side, side], "hough": [rows, cols], "quads": "full",
                   "fhtshift": False, "parallelism": "single GPU"},
    }

    # compulsory traffic of one forward: read the image once, write the Hough image once
    in_bytes = px * 4
    out_bytes = rows * cols * 4
    compulsory = in_bytes + out_bytes
    result["hbm_compulsory_frac"] = round(compulsory / (ms_fwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    result["roofline"] = {
        "bound": "hbm",
        "achieved": round(compulsory / (ms_fwd * 1e-3) / 1e9, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(compulsory / (ms_fwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "traffic": None,
        "kernel": "forward (all launches of one step)",
        "algorithmic_bytes": compulsory,
    }

    if not args.fwd_only:
        g = torch.empty_like(out).normal_()
        gimg = torch.empty_like(x)
        ms_fa, _ = _timed(lambda: (fht.forward(x, out=out, workspace=ws), fht.adjoint(g, side, side, out=gimg)),
                          max(1, args.steps // 2), 1, torch)
        result["fwd_adjoint"] = {"value": round(px / (ms_fa * 1e-3) / 1e9, 3), "unit": "Gpixels/s",
                                 "ms_per_step": round(ms_fa, 4)}

    if not args.no_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(img_np)

    print(json.dumps(result))


if __name__ == "__main__":
    main()
