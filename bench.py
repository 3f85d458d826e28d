#!/usr/bin/env python3
"""Benchmark of the gfx950 oil-paint filter.

One JSON line on stdout.  The headline `value` is the plain single-image
kernel's throughput (megapixels/s) over one pass of the 1920x1080 sweep --
r in {1, 2, 5, 10, 15} at L = 20 and L in {8, 64} at r = 5, seven filter
launches per step -- with the image already resident in device memory.  The
same line carries:
  * per-(r, L) MP/s of that sweep, the 256x256 (r=2, L=20) case and the
    4000x3000 (r=10, L=32) camera case;
  * `batched`: 64 uneven images in one hipGraph-replayed persistent launch
    against 64 back-to-back plain launches;
  * `serving`: 2000 Poisson-arriving requests through the continuous-batching
    queue against the plain kernel run request by request (p50/p99 latency
    and MP/s), plus a saturation run, with every served output compared to
    the plain kernel's and a sample to the CPU oracle;
  * `roofline` of the plain kernel against LDS bandwidth, and
  * `cpu_baseline`: the CPU oracle on the host's cores over the same sweep.

usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--quick]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "megapixels/sec at (r, L), batched/served vs plain kernel; p50/p99 request latency"
LDS_PEAK_GBS = 256 * 2.4e9 * 256 / 1e9  # 256 CUs x 2.4 GHz x 256 B/clk LDS read path


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def lds_bytes_per_pixel(r: int, L: int) -> int:
    """Algorithmic LDS bytes per output pixel of the sliding-window method:
    2(2r+1) window updates, each reading a 4-byte staged pixel and applying
    one 8-byte bin update, plus the mode search reading L bins of 8 bytes and
    the winning bin once more."""
    u = 2 * (2 * r + 1)
    return u * (4 + 8) + (L + 1) * 8


def kernel_source_hash() -> str:
    from paper_1405_1020_amd import tune
    return tune.code_hash()


def autotune(synth, quick: bool) -> dict:
    """Tune the launch shape of every (r, L) the workloads use, each on an
    image of the size it is used at (a few ms of GPU time per pair)."""
    from paper_1405_1020_amd import tune
    out = {}
    out.update(tune.ensure(synth.FHD_SWEEP, 1920, 1080))
    if not quick:
        out.update(tune.ensure([synth.CAMERA_RL], 4000, 3000))
        out.update(tune.ensure([(2, 20)], 256, 256))
        out.update(tune.ensure([(r, L) for r in (2, 3, 5, 8) for L in (16, 20, 32)], 2048, 1536))
        out.update(tune.ensure([(r, L) for r in range(1, 16) for L in (8, 16, 20, 32, 64)], 2400, 1800))
    return {k: v["variant"] for k, v in out.items()}


class Timer:
    """HIP events on torch's current stream, where the binding launches."""

    def __init__(self, torch):
        self.torch = torch

    def time(self, fn, reps: int, warmup: int) -> float:
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps  # ms per call


def bench_plain(torch, B, synth, timer, steps, warmup):
    img = synth.fhd_image()
    src = torch.from_numpy(img).cuda()
    dst = torch.empty_like(src)
    runs = synth.FHD_SWEEP
    mp = img.shape[0] * img.shape[1] / 1e6

    def step():
        for r, L in runs:
            B.oilpaint_async(src, dst, r, L)

    ms_step = timer.time(step, steps, warmup)
    per = {}
    for r, L in runs:
        ms = timer.time(lambda: B.oilpaint_async(src, dst, r, L), max(steps, 10), 2)
        v = B.pick_variant(img.shape[1], img.shape[0], r, L)
        per["r%d_L%d" % (r, L)] = {"ms": round(ms, 5), "mp_per_s": round(mp / (ms / 1e3), 1),
                                   "lds_gbs": round(lds_bytes_per_pixel(r, L) * mp * 1e6 / (ms / 1e3) / 1e9, 1),
                                   "variant": list(v.as_tuple())}
    total_bytes = sum(lds_bytes_per_pixel(r, L) for r, L in runs) * mp * 1e6
    achieved = total_bytes / (ms_step / 1e3) / 1e9
    return img, src, ms_step, mp * len(runs), per, achieved


def bench_single(torch, B, timer, img, r, L, reps):
    src = torch.from_numpy(img).cuda()
    dst = torch.empty_like(src)
    ms = timer.time(lambda: B.oilpaint_async(src, dst, r, L), reps, 3)
    mp = img.shape[0] * img.shape[1] / 1e6
    return {"ms": round(ms, 5), "mp_per_s": round(mp / (ms / 1e3), 1),
            "lds_gbs": round(lds_bytes_per_pixel(r, L) * mp * 1e6 / (ms / 1e3) / 1e9, 1)}


def bench_batched(torch, B, synth, timer, reps):
    specs = synth.batch_items()
    srcs = [synth.batch_image(it) for it in specs]
    dsts = [torch.empty_like(s) for s in srcs]
    mp = sum(s.shape[0] * s.shape[1] for s in srcs) / 1e6
    items = [B.Item(s, d, it.radius, it.levels) for s, d, it in zip(srcs, dsts, specs)]

    def plain():
        for it in items:
            B.oilpaint_async(it.src, it.dst, it.radius, it.levels)

    ms_plain = timer.time(plain, reps, 2)
    ref = [d.clone() for d in dsts]
    plan = B.Plan(items)
    tiles, wgs = plan.info()
    ms_graph = timer.time(plan.launch, reps, 2)
    same = all(torch.equal(a, b) for a, b in zip(ref, dsts))
    ms_batch = timer.time(lambda: B.batch(items), reps, 2)
    same = same and all(torch.equal(a, b) for a, b in zip(ref, dsts))
    plan.close()
    return {
        "workload": "64 images, W~U{320..4096}, H~U{240..3072}, r~U{2,3,5,8}, L~U{16,20,32}",
        "megapixels": round(mp, 2),
        "plain_ms": round(ms_plain, 4), "plain_mp_per_s": round(mp / (ms_plain / 1e3), 1),
        "graph_ms": round(ms_graph, 4), "graph_mp_per_s": round(mp / (ms_graph / 1e3), 1),
        "batch_call_ms": round(ms_batch, 4), "batch_call_mp_per_s": round(mp / (ms_batch / 1e3), 1),
        "graph_vs_plain": round(ms_plain / ms_graph, 3),
        "tiles": tiles, "workgroups": wgs,
        "outputs_equal_plain": bool(same),
    }


def bench_serving(torch, B, synth, serve, n_requests, oracle_mod):
    wl = synth.serve_workload(n=n_requests)
    torch.cuda.synchronize()
    budget = 32 * (1 << 30)
    out = {"workload": "%d requests, Poisson 200/s, 0.1-24 MP log-uniform, r~U{1..15}, "
                       "L~U{8,16,20,32,64}, crops of 8 resident 5700x4300 canvases" % n_requests,
           "budget_bytes": budget}

    def one(kind, saturate):
        rs = serve.make_requests(wl)
        if saturate:
            for q in rs:
                q.arrival_s = 0.0
        ex = serve.QueueExecutor(capacity=4096, step_pixels=16 << 20) if kind == "queue" else serve.PlainExecutor()
        alloc, free = serve.device_allocator(keep=(kind == "queue" and not saturate))
        s = serve.Server(ex, budget_bytes=budget, capacity=4096, allocate=alloc, free=free)
        st = serve.run_open_loop(s, rs)
        ex.close()
        torch.cuda.synchronize()
        return st, rs

    st_q, rs_q = one("queue", False)
    log("served (queue):", st_q)
    st_p, _ = one("plain", False)
    log("served (plain):", st_p)
    sat_q, _ = one("queue", True)
    sat_p, _ = one("plain", True)
    # verification: every served output against the plain kernel, a sample
    # against the CPU oracle (pixels whose windows are cut out and filtered)
    equal = 0
    for q in rs_q:
        ref = torch.empty_like(q.dst)
        B.run(B.Item(q.src, ref, q.radius, q.levels))
        equal += int(torch.equal(ref, q.dst))
    torch.cuda.synchronize()
    import numpy as np
    rng = np.random.default_rng(5)
    sample = [rs_q[i] for i in rng.choice(len(rs_q), size=min(12, len(rs_q)), replace=False)]
    oracle_ok = 0
    checked = 0
    for q in sample:
        h, w = q.height, q.width
        for _ in range(4):
            x, y = int(rng.integers(0, w)), int(rng.integers(0, h))
            r = q.radius
            y0, y1, x0, x1 = max(0, y - r), min(h, y + r + 1), max(0, x - r), min(w, x + r + 1)
            crop = q.src[y0:y1, x0:x1].contiguous().cpu().numpy()
            want = oracle_mod.oilpaint_ref(crop, r, q.levels)[y - y0, x - x0]
            got = q.dst[y, x].cpu().numpy()
            oracle_ok += int((want == got).all())
            checked += 1
    for q in rs_q:
        q.dst = None

    def pick(st):
        return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()
                if k in ("completed", "failed", "megapixels", "span_s", "mp_per_s", "p50_ms", "p99_ms",
                         "mean_ms", "peak_bytes")}
    out.update({
        "queue": pick(st_q), "plain": pick(st_p),
        "saturation_queue": pick(sat_q), "saturation_plain": pick(sat_p),
        "p99_gain": round(st_p["p99_ms"] / st_q["p99_ms"], 3) if st_q["p99_ms"] > 0 else None,
        "saturation_mp_gain": round(sat_q["mp_per_s"] / sat_p["mp_per_s"], 3) if sat_p["mp_per_s"] > 0 else None,
        "outputs_equal_plain": "%d/%d" % (equal, len(rs_q)),
        "oracle_pixels": "%d/%d" % (oracle_ok, checked),
    })
    return out


def cpu_baseline(oracle_mod, img, runs):
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    threads = max(1, min(16, ncpu))
    t0 = time.perf_counter()
    for r, L in runs:
        oracle_mod.oilpaint_ref(img, r, L, nthreads=threads)
    dt = time.perf_counter() - t0
    mp = img.shape[0] * img.shape[1] / 1e6 * len(runs)
    return {"value": round(mp / dt, 3), "unit": "MP/s", "cores": threads, "kind": "oracle",
            "sample": "the full 1920x1080 sweep (7 runs), row bands over %d threads, %.1f s wall" % (threads, dt)}


def hbm_traffic(achieved_launch_bytes):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "k_plain_fhd_sweep_hbm.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="main sweep only (for profiling)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--copy-ref", action="store_true",
                    help="run only a plain 1 GiB device copy kernel (HBM counter scaling) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1405_1020_amd import binding as B, synth, serve
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B.lib()

    if args.copy_ref:
        n = 1 << 30
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 0, out=b)  # elementwise kernel: reads n bytes, writes n bytes
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes": n}))
        return

    timer = Timer(torch)
    log("autotune ...")
    tuned = autotune(synth, args.quick)
    log("plain sweep ...")
    img, src, ms_step, mp_step, per, achieved = bench_plain(torch, B, synth, timer, args.steps, args.warmup)
    value = mp_step / (ms_step / 1e3)
    launch_ms = ms_step / len(synth.FHD_SWEEP)
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "MP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "fhd_1920x1080_sweep", "width": 1920, "height": 1080,
                   "runs": [list(x) for x in synth.FHD_SWEEP], "image": "40 Gaussian colour blobs + U{-8..8} noise, seed 2",
                   "launches_per_step": len(synth.FHD_SWEEP)},
    }
    res["roofline"] = {"bound": "lds", "achieved": round(achieved, 1), "peak": round(LDS_PEAK_GBS, 1),
                       "unit": "GB/s", "frac": round(achieved / LDS_PEAK_GBS, 4),
                       "traffic": hbm_traffic(None), "kernel": "k_plain",
                       "avg_launch_ms": round(launch_ms, 5)}
    res["sweep"] = per
    res["tuned_variants"] = tuned
    if not args.quick:
        small_img, r, L = synth.small_case()
        res["small_256x256_r2_L20"] = bench_single(torch, B, timer, small_img, r, L, 50)
        log("camera ...")
        res["camera_4000x3000_r10_L32"] = bench_single(torch, B, timer, synth.camera_image(), 10, 32, 10)
        log("batched ...")
        res["batched"] = bench_batched(torch, B, synth, timer, 5)
        import oracle as oracle_mod
        log("serving ...")
        res["serving"] = bench_serving(torch, B, synth, serve, args.serve_requests, oracle_mod)
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(oracle_mod, img, synth.FHD_SWEEP)
        # parity of the timed configuration: the sweep's outputs against the oracle
        bad = 0
        for r, L in synth.FHD_SWEEP:
            out = B.oilpaint(src, r, L)
            torch.cuda.synchronize()
            want = oracle_mod.oilpaint_ref(img, r, L, nthreads=res["cpu_baseline"]["cores"])
            bad += int((out.cpu().numpy() != want).any(axis=-1).sum())
        res["parity"] = {"fhd_sweep_pixels_differing": bad}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
