#!/usr/bin/env python3
"""Benchmark: full four-quadrant FHT of a 4096 x 4096 float32 image on one GPU.

One step = one full forward transform (all four quadrants, merged full Hough
image of 16381 x 8192 float32) of a synthetic, seeded image already resident
in HBM.  Prints one JSON line:
  value         input Gpixels/s of the forward (4096^2 pixels per step)
  roofline      the dominant kernel (last pass) against the 8 TB/s HBM roof:
                the transform's compulsory bytes (image once + Hough image
                once; one launch completes one transform) over its average
                launch time,
                measured with HIP events on its launch stream in the timed
                region; traffic = HBM bytes per launch from the committed
                counter summary (null when the kernel sources have changed)
  fwd_adjoint   forward + adjoint (the backward of the transform)
  batched       8 such images through one batch plan (HIP graph replay),
                beside a loop of 8 single-image forwards
  sparse1024    1024^2 uint8: forward, forward + fused fhtshift, standalone
                fhtshift, angle range [-15, 15] degrees (microseconds)
  batch512      512 uint8 images with sides uniform in 64..2048 (graph
                replay), beside a loop of 512 single-image forwards
  cpu_baseline  the CPU oracle on this host's cores (bounded sample)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
CSRC = os.path.join(ROOT, "paper_1811_06378_amd", "csrc")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "fht_pass_kernel_last_dense4096_traffic.txt")


# the sources the forward pass kernels and their launches are built from
PASS_SOURCES = ("fht_api.hip", "fht_device.h", "fht_fwd_f32.hip", "fht_internal.h", "fht_launch.h", "fht_misc.hip",
                "fht_plan.h")


def sources_digest() -> str:
    """sha256 over the forward pass kernel's sources (name + bytes, in order)."""
    h = hashlib.sha256()
    for f in PASS_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def committed_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if absent, for another kernel, or taken on other sources."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    kv = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or kv.get("sources_sha256") != sources_digest():
        return None
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def committed_forward_traffic():
    """Counter bytes of one whole forward (every pass kernel) from the
    committed summary, or None when absent or taken on other sources."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    kv = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_sha256") != sources_digest():
        return None
    try:
        return int(float(kv["forward_traffic_bytes"]))
    except (KeyError, ValueError):
        return None


def _timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def last_pass_algorithmic_bytes(fht, w: int, h: int, elem: int) -> int:
    """Bytes the last pass of a two-pass full transform must move: read every
    quadrant's first-pass band (n rows of other + 2^G1 - 1 columns, where G1
    is the first pass's stage count) and write the full Hough image once."""
    wp, hp = 1 << max(0, (w - 1).bit_length()), 1 << max(0, (h - 1).bit_length())
    total = 0
    for n, other in ((hp, wp), (hp, wp), (wp, hp), (wp, hp)):
        split = fht.pass_split(n)
        assert len(split) == 2, "the roofline formula covers two-pass sizes"
        total += n * (other + (1 << split[0]) - 1) * elem
    rows, cols = fht.hough_shape(w, h)
    return total + rows * cols * elem


def cpu_baseline(img, reps: int = 3):
    """The CPU oracle (stage recurrence, OpenMP over rows) on the same 4096^2
    image: `reps` full transforms in float64 (the oracle's own precision; the
    reported value) and `reps` in its float32 mode, median of each."""
    import statistics

    import oracle

    x = img.astype("float64")

    def median_s(single):
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            oracle.full(x, single=single)
            ts.append(time.perf_counter() - t)
        return statistics.median(ts), sum(ts)

    t64, tot64 = median_s(False)
    t32, tot32 = median_s(True)
    px = x.shape[0] * x.shape[1]
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(px / t64 / 1e9, 6), "unit": "Gpixels/s", "cores": oracle.threads(),
            "kind": "oracle", "cpu_model": model, "host_cpus": os.cpu_count(),
            "fp32": {"value": round(px / t32 / 1e9, 6), "unit": "Gpixels/s", "median_s": round(t32, 4)},
            "median_s": round(t64, 4),
            "sample": "median of %d full float64 transforms (value) and of %d float32-mode transforms of the "
                      "same 4096x4096 image, %.1f s in total" % (reps, reps, tot64 + tot32)}


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def bench_stack(fht, torch, x, steps, warmup, label):
    """Stack forward (fht_forward_stack, captured once in a HIP graph and
    replayed) and the same images through single-image forwards, into the
    same output."""
    n, h, w = x.shape
    rows, cols = fht.hough_shape(w, h)
    out = torch.empty((n, rows, cols), dtype=torch.float32 if x.dtype == torch.float32 else torch.int32, device="cuda")
    ws = torch.empty(max(fht.forward_stack_workspace_size(w, h, n, "full", x.dtype), 256), dtype=torch.uint8,
                     device="cuda")
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fht.batch_forward(x, out=out, workspace=ws)  # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(s)
    with torch.cuda.graph(graph):
        fht.batch_forward(x, out=out, workspace=ws)
    ms_stack = _timed(graph.replay, steps, warmup, torch)
    ws1 = torch.empty(max(fht.workspace_size(w, h, "full", x.dtype), 256), dtype=torch.uint8, device="cuda")

    def loop():
        for i in range(n):
            fht.forward(x[i], out=out[i], workspace=ws1)

    ms_loop = _timed(loop, steps, warmup, torch)
    px = n * h * w
    out_bytes = out.numel() * out.element_size()
    in_bytes = x.numel() * x.element_size()
    res = {"value": round(px / (ms_stack * 1e-3) / 1e9, 3), "unit": "Gpixels/s", "ms_per_step": round(ms_stack, 4),
           "images": n, "pixels": px, "hough_cells": out.numel(),
           "hbm_compulsory_frac": round((in_bytes + out_bytes) / (ms_stack * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "single_image_loop": {"value": round(px / (ms_loop * 1e-3) / 1e9, 3), "ms_per_step": round(ms_loop, 4)},
           "launch": "fht_forward_stack (one launch per pass kind over the stack), captured in a HIP graph and "
                     "replayed"}
    log("%s: stacked %.3f ms, single-image loop %.3f ms" % (label, ms_stack, ms_loop))
    del graph, out, ws, ws1
    torch.cuda.empty_cache()
    return res


def bench_batch(fht, torch, imgs, steps, warmup, label):
    """Batched forward (captured once in a HIP graph, replayed) and the same
    images through single-image forwards, into the same packed output."""
    sizes = [tuple(x.shape) for x in imgs]
    plan = fht.BatchPlan(sizes, in_dtype=imgs[0].dtype)
    table = plan.pointer_table(imgs)
    packed = plan.output()
    graph = plan.capture(table, packed)
    ms_batch = _timed(graph.replay, steps, warmup, torch)
    views = plan.views(packed)
    ws = torch.empty(max(max(fht.workspace_size(w, h, "full", imgs[0].dtype) for h, w in sizes), 256),
                     dtype=torch.uint8, device="cuda")

    def loop():
        for x, v in zip(imgs, views):
            fht.forward(x, out=v, workspace=ws)

    ms_loop = _timed(loop, steps, warmup, torch)
    px = sum(h * w for h, w in sizes)
    out_bytes = plan.out_elems * 4
    in_bytes = sum(x.numel() * x.element_size() for x in imgs)
    res = {"value": round(px / (ms_batch * 1e-3) / 1e9, 3), "unit": "Gpixels/s", "ms_per_step": round(ms_batch, 4),
           "images": len(imgs), "pixels": px, "hough_cells": plan.out_elems,
           "hbm_compulsory_frac": round((in_bytes + out_bytes) / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "single_image_loop": {"value": round(px / (ms_loop * 1e-3) / 1e9, 3), "ms_per_step": round(ms_loop, 4)},
           "launch": "one batch plan, captured in a HIP graph and replayed"}
    log("%s: batched %.3f ms, single-image loop %.3f ms" % (label, ms_batch, ms_loop))
    del graph, packed, views, plan
    torch.cuda.empty_cache()
    return res


def batch_graph_ms(fht, torch, imgs, steps, packed=None):
    """ms per replay of one batch plan captured in a HIP graph (the current
    stage splits and tile heights), into `packed` when given."""
    plan = fht.BatchPlan([tuple(x.shape) for x in imgs], in_dtype=imgs[0].dtype)
    table = plan.pointer_table(imgs)
    out = plan.output() if packed is None else packed
    graph = plan.capture(table, out)
    ms = _timed(graph.replay, steps, 2, torch)
    del graph, out, table, plan
    torch.cuda.empty_cache()
    return ms


def stage_configs(k):
    """(split, tile rows) candidates for quadrants of 2^k rows: every split
    into the fewest passes of 3..6 stages, each with 64-row tiles and, when
    some pass has at most 5 stages, 32-row tiles (the candidates
    fht_autotune times on one image)."""
    n_pass = -(-k // 6)
    splits = []

    def extend(prefix, left, parts):
        if parts == 0:
            if left == 0:
                splits.append(prefix)
            return
        for g in range(3, 7):
            if g <= left:
                extend(prefix + [g], left - g, parts - 1)

    extend([], k, n_pass)
    out = []
    for sp in splits:
        out.append((sp, 64))
        if min(sp) <= 5:
            out.append((sp, 32))
    return out


def tune_on_workload(fht, ks, time_fn):
    """Stage split and tile height tuned on the workload itself: from the
    default rules, for each stage count in turn every candidate is set and
    the whole workload timed (time_fn), and the fastest setting is kept
    before the next stage count.  Returns the default time, the best time
    and the setting per stage count."""
    for k in ks:
        fht.set_pass_split(k, None)
        fht.set_tile_rows(k, None)
    time_fn()  # warm-up: first-call costs stay out of the comparison
    ms_default = time_fn()
    best_ms = ms_default
    chosen = {}
    for k in ks:
        best = None
        for split, rows in stage_configs(k):
            fht.set_pass_split(k, split)
            fht.set_tile_rows(k, rows)
            ms = time_fn()
            if ms < best_ms:
                best_ms, best = ms, (split, rows)
        if best is None:
            fht.set_pass_split(k, None)
            fht.set_tile_rows(k, None)
        else:
            fht.set_pass_split(k, best[0])
            fht.set_tile_rows(k, best[1])
        chosen[str(k)] = {"split": fht.pass_split(1 << k), "tile_rows": fht.tile_rows(1 << k)}
    return ms_default, best_ms, chosen


def reset_tuning(fht, ks):
    for k in ks:
        fht.set_pass_split(k, None)
        fht.set_tile_rows(k, None)


def bench_diff16(fht, synth, torch, steps):
    """The differentiable workload: a 16 x 1024^2 float32 stack through the
    autograd wrapper, forward plus backward for a fixed upstream gradient
    (the weighted-square loss's gradient shape), against the same work as a
    loop of single-image forwards and adjoints."""
    xs = torch.from_numpy(synth.normal1024(0)).cuda()
    n, h, w = xs.shape
    rows, cols = fht.hough_shape(w, h)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    up = torch.rand((n, rows, cols), generator=gen, device="cuda")
    x = xs.clone().requires_grad_()

    def step():
        x.grad = None
        fht.fht(x).backward(up)

    # stage split and tile height of the 1024-row quadrants tuned on the
    # whole step (every candidate timed on it), then measured again
    k = max(0, (h - 1).bit_length())
    default = {"split": fht.pass_split(h), "tile_rows": fht.tile_rows(h)}
    ms_default, ms_tuned, chosen = tune_on_workload(fht, [k], lambda: _timed(step, max(3, steps // 2), 1, torch))
    ms = _timed(step, steps, 2, torch)
    outs = torch.empty((n, rows, cols), device="cuda")
    grads = torch.empty_like(xs)

    def loop():
        for i in range(n):
            fht.forward(xs[i], out=outs[i])
            fht.adjoint(up[i], w, h, out=grads[i])

    ms_loop = _timed(loop, steps, 2, torch)
    px = n * h * w
    log("diff16x1024: autograd fwd+bwd %.3f ms, single-image loop %.3f ms" % (ms, ms_loop))
    res = {"workload": "16 x 1024x1024 float32 (standard normal), forward + backward through the autograd "
                       "wrapper for a fixed upstream gradient", "unit": "Gpixels/s",
           "value": round(px / (ms * 1e-3) / 1e9, 3), "ms_per_step": round(ms, 4),
           "single_image_loop": {"value": round(px / (ms_loop * 1e-3) / 1e9, 3), "ms_per_step": round(ms_loop, 4)},
           "tuning": {"default": default, "default_ms": round(ms_default, 4), "used": chosen[str(k)],
                      "tuned_ms": round(ms_tuned, 4),
                      "how": "every (split, tile height) of the 1024-row quadrants timed on the whole step"}}
    reset_tuning(fht, [k])
    return res


def bench_sparse1024(fht, synth, torch, steps):
    """1024^2 uint8 image: full forward, forward with fhtshift fused into the
    stores, standalone fhtshift of the full image, and the angle range
    [-15, +15] degrees (int32 Hough images)."""
    side = 1024
    x = torch.from_numpy(synth.sparse1024(0)).cuda()
    rows, cols = fht.hough_shape(side, side)
    out = torch.empty((rows, cols), dtype=torch.int32, device="cuda")
    out2 = torch.empty_like(out)
    ws = torch.empty(max(fht.workspace_size(side, side, "full", torch.uint8), 256), dtype=torch.uint8, device="cuda")
    S1, S = fht.range_params(side, -15.0, 15.0)
    rr, rc = fht.range_shape(side, side, S1, S)
    rout = torch.empty((rr, rc), dtype=torch.int32, device="cuda")
    px = side * side
    res = {"workload": "1024x1024 uint8, 2% of pixels uniform in 0..255 plus 8 lines of 255; int32 Hough images",
           "unit": "microseconds per call"}
    res["forward_us"] = round(_timed(lambda: fht.forward(x, out=out, workspace=ws), steps, 2, torch) * 1e3, 2)
    res["forward_shifted_us"] = round(
        _timed(lambda: fht.forward(x, shifted=True, out=out, workspace=ws), steps, 2, torch) * 1e3, 2)
    res["fhtshift_us"] = round(_timed(lambda: fht.shift(out, side, side, out=out2), steps, 2, torch) * 1e3, 2)
    res["range_us"] = round(_timed(lambda: fht.range_transform(x, S1, S, out=rout), steps, 2, torch) * 1e3, 2)
    res["range"] = {"deg": [-15, 15], "S1": S1, "S": S, "rows": rr}
    res["forward_gpx_s"] = round(px / (res["forward_us"] * 1e-6) / 1e9, 3)
    log("sparse1024: forward %.1f us, shifted %.1f us, fhtshift %.1f us, range %.1f us"
        % (res["forward_us"], res["forward_shifted_us"], res["fhtshift_us"], res["range_us"]))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--fwd-only", action="store_true", help="time only the forward (profiling runs)")
    ap.add_argument("--fwd-adjoint-only", action="store_true",
                    help="time only the forward and the forward + adjoint step (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the transform shards "
              "by image, quadrant or column band without a collective on the hot path).", file=sys.stderr)
        sys.exit(2)

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
    log("forward %dx%d float32 -> %dx%d, %d steps after %d warmup" % (side, side, rows, cols, args.steps,
                                                                   args.warmup))

    def step():
        fht.forward(x, out=out, workspace=ws)

    def timed_region(kernel_filter):
        """K steps between two events on the launch stream, with the pass
        launches whose kernel name contains kernel_filter (all if None)
        bracketed by HIP events on the same stream."""
        fht.timing_filter(kernel_filter)
        fht.timing_enable(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        fht.timing_enable(False)
        fht.timing_filter(None)
        return e0.elapsed_time(e1) / args.steps, fht.timing_report()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # every kernel timed: finds the dominant kernel (largest summed time)
    ms_all, kernels_all = timed_region(None)
    dominant = max(kernels_all.items(), key=lambda kv: kv[1][1])[0]
    # the timed region of value and roofline: only the dominant kernel's
    # launches carry events (each pair delays the next launch slightly)
    ms_fwd, kernels = timed_region(dominant)
    # the same steps without any launch events
    ms_plain = _timed(step, args.steps, 1, torch)
    px = side * side
    value = px / (ms_fwd * 1e-3) / 1e9

    result = {
        "metric": "Gpixels/s full 4-quadrant FHT 4096² (fwd, fwd+adjoint, batched); % HBM peak",
        "value": round(value, 3),
        "unit": "Gpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_fwd, 4),
        "ms_per_step_without_launch_events": round(ms_plain, 4),
        "ms_per_step_all_launches_timed": round(ms_all, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Exp(1) 4096x4096 image with 16 planted lines of +20)",
        "config": {"workload": "dense4096: 4096x4096 float32, full four-quadrant Hough image 16381x8192 float32",
                   "image": [side, side], "hough": [rows, cols], "quads": "full", "fhtshift": False},
    }

    # whole-transform compulsory traffic: read the image once, write the Hough image once
    compulsory = px * 4 + rows * cols * 4
    result["hbm_compulsory_frac"] = round(compulsory / (ms_fwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    # dominant kernel: the largest summed launch time with every kernel timed.
    # Its algorithmic bytes are the whole transform's compulsory traffic (the
    # image read once, the Hough image written once): one launch of the last
    # pass completes one transform.  The pass's own bytes (bands in, Hough
    # image out) are reported beside it.
    name = dominant
    launches, total_ms = kernels[name]
    avg_ms = total_ms / launches
    alg = compulsory if "fht_pass_kernel<float, float, 3, false, true, 0, 8, 0>" in name else None
    pass_bytes = last_pass_algorithmic_bytes(fht, side, side, 4) if alg else None
    achieved = alg / (avg_ms * 1e-3) / 1e9 if alg else None
    traffic = committed_traffic(name)
    result["roofline"] = {
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": traffic,
        "kernel": name,
        "launch_ms": round(avg_ms, 4),
        "launches": launches,
        "algorithmic_bytes_per_launch": alg,
        "algorithmic_bytes": "image once + Hough image once (4096^2 x 4 B + 16381 x 8192 x 4 B)",
        "pass_bytes_per_launch": pass_bytes,
        "pass_frac": round(pass_bytes / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if pass_bytes else None,
        "traffic_over_algorithmic": round(traffic / alg, 3) if (traffic and alg) else None,
        "kernel_times_ms": {k: round(v[1] / v[0], 4) for k, v in kernels_all.items()},
    }
    forward_traffic = committed_forward_traffic()
    if forward_traffic:
        result["forward_traffic_bytes"] = forward_traffic
        result["forward_traffic_over_compulsory"] = round(forward_traffic / compulsory, 3)

    if not args.fwd_only:
        g = torch.empty_like(out).normal_()
        gimg = torch.empty_like(x)
        ms_fa = _timed(lambda: (fht.forward(x, out=out, workspace=ws), fht.adjoint(g, side, side, out=gimg)),
                       max(1, args.steps // 2), 1, torch)
        result["fwd_adjoint"] = {"value": round(px / (ms_fa * 1e-3) / 1e9, 3), "unit": "Gpixels/s",
                                 "ms_per_step": round(ms_fa, 4),
                                 "hbm_compulsory_frac": round(2 * compulsory / (ms_fa * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                                              4)}
        del g, gimg
        log("fwd+adjoint %.3f ms" % ms_fa)

    if not args.fwd_only and not args.fwd_adjoint_only:
        imgs8 = [x] + [torch.from_numpy(synth.dense4096(s, size=side)).cuda() for s in range(1, 8)]
        x8 = torch.stack(imgs8)
        result["batched"] = bench_stack(fht, torch, x8, max(1, args.steps // 4), 1, "batched 8x4096^2 f32")
        result["batched"]["workload"] = "8 dense4096 images (seeds 0..7), float32, one (8, 4096, 4096) stack"
        plan_line = bench_batch(fht, torch, imgs8, max(1, args.steps // 4), 1, "batch plan 8x4096^2 f32")
        result["batched"]["batch_plan"] = {"value": plan_line["value"], "ms_per_step": plan_line["ms_per_step"],
                                           "launch": plan_line["launch"]}
        del imgs8, x8

        result["sparse1024"] = bench_sparse1024(fht, synth, torch, max(5, args.steps))
        result["diff16x1024"] = bench_diff16(fht, synth, torch, max(5, args.steps // 2))
        torch.cuda.empty_cache()

        imgs512 = [torch.from_numpy(a).cuda() for a in synth.batch512(0)]
        # Stage split and tile height per stage count tuned on the batch's
        # own work list: each candidate timed on the whole batch (graph
        # replay), one stage count at a time, then the line measured again.
        ks = [k for k in sorted({max(0, (s - 1).bit_length()) for a in imgs512 for s in a.shape})
              if len(stage_configs(k)) > 1]
        default = {str(k): {"split": fht.pass_split(1 << k), "tile_rows": fht.tile_rows(1 << k)} for k in ks}
        probe = fht.BatchPlan([tuple(a.shape) for a in imgs512], in_dtype=torch.uint8)
        packed = probe.output()
        del probe
        ms_default, ms_tuned, chosen = tune_on_workload(
            fht, ks, lambda: batch_graph_ms(fht, torch, imgs512, 3, packed=packed))
        del packed
        torch.cuda.empty_cache()
        result["batch512"] = bench_batch(fht, torch, imgs512, 6, 2, "batch512 u8")
        result["batch512"]["workload"] = "512 uint8 images, sides uniform in 64..2048 (seed 0), int32 Hough images"
        result["batch512"]["tuning"] = {"default": default, "default_ms": round(ms_default, 3), "used": chosen,
                                        "tuned_ms": round(ms_tuned, 3),
                                        "how": "every (split, tile height) per stage count timed on the whole batch"}
        reset_tuning(fht, ks)
        del imgs512
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log("CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(img_np)

    print(json.dumps(result))


if __name__ == "__main__":
    main()
