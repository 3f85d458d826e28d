#!/usr/bin/env python3
"""Benchmark of the gfx950 oil-paint filter.

One JSON line on stdout.  The headline `value` is the plain single-image
kernel's throughput (megapixels/s) over one pass of the 1920x1080 sweep --
r in {1, 2, 5, 10, 15} at L = 20 and L in {8, 64} at r = 5, seven filter
launches per step -- with the image already resident in device memory,
timed over K steps after W warmup steps, which follow 30 ms of untimed steps
(`settle_steps`) that bring the GPU out of its idle state.  The same line
carries:
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
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "megapixels/sec at (r, L), batched/served vs plain kernel; p50/p99 request latency"
# How the HBM counter summary is made, from the repository root ($REPO) on the
# GPU host, with $OUT an output directory (the first line fills the tuning
# cache so that the profiled runs launch only the timed shapes).
HBM_COMMANDS = [
    "python3 bench.py --quick --steps 20 --warmup 3 > $OUT/quick.json",
    "cd /tmp && export TMPDIR=/tmp",
    "timeout -s KILL 180 rocprofv3 --pmc FETCH_SIZE -d $OUT/sweep_fetch --output-format csv -- "
    "python3 $REPO/bench.py --quick --steps 5 --warmup 2",
    "timeout -s KILL 180 rocprofv3 --pmc WRITE_SIZE -d $OUT/sweep_write --output-format csv -- "
    "python3 $REPO/bench.py --quick --steps 5 --warmup 2",
    "timeout -s KILL 180 rocprofv3 --pmc FETCH_SIZE -d $OUT/copy_fetch --output-format csv -- "
    "python3 $REPO/bench.py --copy-ref",
    "timeout -s KILL 180 rocprofv3 --pmc WRITE_SIZE -d $OUT/copy_write --output-format csv -- "
    "python3 $REPO/bench.py --copy-ref",
    "cd $REPO && python3 bench.py --hbm-summary $OUT --sweep-json $OUT/quick.json",
]
LDS_PEAK_GBS = 256 * 2.4e9 * 256 / 1e9  # 256 CUs x 2.4 GHz x 256 B/clk LDS read path
# Counter passes over the LDS and VALU units (one rocprofv3 --pmc run each,
# with the kernel trace for durations), as bench.py --counter-summary reads
# them: sub-folder name -> counters.
COUNTER_PASSES = {
    "derived": ["LdsUtil", "VALUBusy", "LdsBankConflict", "OccupancyPercent", "VALUUtilization"],
    "lds": ["SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_LDS", "SQ_ACTIVE_INST_LDS", "SQ_WAVES",
            "GRBM_GUI_ACTIVE"],
    "valu": ["SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES",
             "SQ_INSTS_SALU", "GRBM_GUI_ACTIVE"],
}
# GRBM_GUI_ACTIVE is counted by each of the GPU's XCDs and the raw output sums
# them; rocprofiler-sdk's derived figures take their maximum.
XCDS = 8
COUNTER_WORKLOADS = {
    "sweep": "bench.py --quick --steps 3 --warmup 1",
    "camera": "bench.py --counter-workload camera",
    "batched": "bench.py --counter-workload batched",
}
COUNTER_PROFILE = os.path.join(ROOT, "profiles", "lds_valu_counters.json")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "lds_valu_counters.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def lds_bytes_per_pixel(r: int, L: int) -> int:
    """Algorithmic LDS bytes per output pixel of the sliding-window method:
    U = 2(2r+1) window updates, each reading a 4-byte staged pixel and
    reading and writing one 8-byte bin (20 B), plus the mode search reading
    L bins of 8 bytes: 20 U + 8 L."""
    u = 2 * (2 * r + 1)
    return 20 * u + 8 * L


HBM_PROFILE = os.path.join(ROOT, "profiles", "k_plain_fhd_sweep_hbm.json")


def lds_probe_leg(torch, B, iters: int = 2048, per_cu: int = 4) -> dict:
    """Measured LDS rates of this GPU (oilpaint_lds_probe): four 256-lane
    workgroups of 32 KB per CU, every wavefront issuing iters x 16 LDS
    operations of one kind on distinct, conflict-free words.  Per CU and
    shader clock (s_memtime between barriers, per workgroup, median): bytes
    of 8-byte and of 4-byte reads, and clocks per 64-lane 64-bit atomic add.
    The shader clock comes from the same counters against the 100 MHz real
    time."""
    import statistics
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"cus": cus, "iters": iters, "workgroups_per_cu": per_cu}
    clocks_hz = []
    for name, kind, lane_bytes in (("read64", B.PROBE_READ64, 8), ("read32", B.PROBE_READ32, 4),
                                   ("add64", B.PROBE_ADD64, 0)):
        B.lds_probe(kind, 64, per_cu)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        wg, clocks = B.lds_probe(kind, iters, per_cu)
        e1.record()
        torch.cuda.synchronize()
        c = clocks.cpu().numpy().astype("float64")
        cyc = c[:, 1] - c[:, 0]
        real_s = (c[:, 3] - c[:, 2]) / 100e6
        med_cyc = statistics.median(cyc.tolist())
        hz = statistics.median((cyc / real_s).tolist())
        clocks_hz.append(hz)
        instr = per_cu * 4 * iters * 16  # per CU
        per_clk = instr / med_cyc
        e = {"workgroups": wg, "cycles_median": int(med_cyc), "clock_mhz": round(hz / 1e6, 1),
             "kernel_ms": round(e0.elapsed_time(e1), 4), "instr_per_clk_per_cu": round(per_clk, 4),
             "clk_per_instr": round(1.0 / per_clk, 3)}
        if lane_bytes:
            e["bytes_per_clk_per_cu"] = round(per_clk * 64 * lane_bytes, 1)
        out[name] = e
    hz = statistics.median(clocks_hz)
    out["clock_mhz"] = round(hz / 1e6, 1)
    out["read64_gbs"] = round(out["read64"]["bytes_per_clk_per_cu"] * cus * hz / 1e9, 1)
    out["read32_gbs"] = round(out["read32"]["bytes_per_clk_per_cu"] * cus * hz / 1e9, 1)
    out["add64_g_lane_ops"] = round(64 * out["add64"]["instr_per_clk_per_cu"] * cus * hz / 1e9, 1)
    return out


def lds_model_ms(r: int, L: int, pixels: float, rates: dict) -> float:
    """Time the sliding method's LDS work would take at the measured LDS
    rates: per output pixel U = 2(2r+1) bin updates (64-bit atomic adds, 64
    lanes per instruction) and U staged-pixel reads (4 bytes, at the 4-byte
    read rate), plus L bin reads (8 bytes, at the 8-byte read rate); spread
    over every CU at the probe's shader clock."""
    u = 2 * (2 * r + 1)
    cyc = (u * rates["add64"]["clk_per_instr"] / 64.0 + 4.0 * u / rates["read32"]["bytes_per_clk_per_cu"] +
           8.0 * L / rates["read64"]["bytes_per_clk_per_cu"])
    return pixels * cyc / (rates["cus"] * rates["clock_mhz"] * 1e6) * 1e3


def kernel_name(r: int, L: int, v) -> str:
    """Name of the plain kernel a (radius, levels, variant) launch runs, as
    the profiler reports it."""
    scan = (L + 7) // 8 * 8
    mb = 2 if L <= 8 else 4 if L <= 16 else 5 if L <= 20 else 8 if L <= 32 else 16  # bins per wavefront
    if v.hist == 1 and v.waves == 4:  # streamed rows, four wavefronts per strip
        return "k_plain_split<%d, %d>" % (r, mb)
    if v.hist == 3 and v.waves == 4:  # streamed rows, 8-byte entries, four wavefronts per strip
        return "k_plain_split8<%d, %d>" % (r, mb)
    if v.hist == 1:  # streamed rows
        return "k_plain_stream<%d, %d>" % (r, 32 if scan <= 32 else 64)
    if v.hist == 3:  # streamed rows, 8-byte entries
        return "k_plain_stream8<%d>" % r
    if v.hist == 5:  # histograms in registers
        return "k_plain_regs<%d, %d>" % (r, 8 if L <= 8 else 16)
    if v.hist == 4 and r <= 15 and L <= 64:  # column histograms, radius <= 15 form
        words = 3 if L <= 9 else 7 if L <= 21 else 11 if L <= 33 else 22
        return "k_plain_column15<%d, %d>" % (words, v.waves)
    if v.hist == 4 and 16 <= r <= 31 and L <= 64 and v.waves in (2, 4):  # column histograms, radius 16..31 form
        words = 4 if L <= 8 else 10 if L <= 20 else 16 if L <= 32 else 32
        return "k_plain_column31<%d, %d>" % (words, v.waves)
    if v.hist == 4:  # column histograms
        return "k_plain_column<%d>" % ((64 + 2 * r + 63) // 64)
    if v.hist == 0 and v.lanes == 64 and r <= 15 and L <= 64:
        return "k_plain_fast<%d, %d>" % (r, 16 if scan <= 16 else 32 if scan <= 32 else 64)
    return "k_plain"


# Sources that define the plain kernels the sweep launches; the HBM counter
# summary is valid while they are unchanged.
SWEEP_KERNEL_SOURCES = ("oilpaint_internal.h", "oilpaint_device.h", "oilpaint_k_regs.hip", "oilpaint_k_stream_lo.hip",
                        "oilpaint_k_stream_hi.hip", "oilpaint_k_stream8.hip", "oilpaint_k_split.hip",
                        "oilpaint_k_split_lo.hip", "oilpaint_k_split_hi.hip", "oilpaint_k_fast_lo.hip",
                        "oilpaint_k_fast_hi.hip", "oilpaint_column.h", "oilpaint_k_column.hip")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1405_1020_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


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
        out.update(tune.ensure([(r, 20) for r in LARGE_RADII], 1920, 1080))
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

    def each(self, fn, reps: int) -> list:
        """Sorted per-call times (ms), an event pair around every call."""
        torch = self.torch
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return sorted(a.elapsed_time(b) for a, b in ev)


def transfers(torch, img) -> dict:
    """Host-device copy times of one image (pinned host buffer): context for
    callers that hand over host images; the filter itself takes device
    pointers and the timed figures exclude copies."""
    host = torch.from_numpy(img).pin_memory()
    dev = torch.empty(host.shape, dtype=torch.uint8, device="cuda")
    for _ in range(3):
        dev.copy_(host, non_blocking=True)
        host.copy_(dev, non_blocking=True)
    torch.cuda.synchronize()
    out = {}
    for name, fn in (("h2d", lambda: dev.copy_(host, non_blocking=True)),
                     ("d2h", lambda: host.copy_(dev, non_blocking=True))):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        out[name + "_ms"] = round(ms, 4)
        out[name + "_gbs"] = round(img.nbytes / (ms / 1e3) / 1e9, 1)
    out["bytes"] = int(img.nbytes)
    return out


def host_cpu() -> dict:
    """The host's CPU model and counts, and the oracle's thread count: the
    CPUs this process may run on, at most 16 (the host's share per GPU)."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return {"model": model, "cpu_count": os.cpu_count(), "affinity": aff, "threads": max(1, min(16, aff))}


def oracle_timings(oracle_mod, synth, threads: int) -> dict:
    """The oracle in the paper's two forms (Section 4's serial loop, T1;
    Section 5's row-parallel loop, T2, here row bands on `threads` threads):
    one thread on the 256x256 case and on the whole 1920x1080 sweep; all
    threads on the 256x256 case, the 4000x3000 camera image and the 64-image
    batch (the 1920x1080 sweep on all threads is cpu_baseline)."""
    out = {}

    def timed(name, imgs_rl, th):
        t0 = time.perf_counter()
        px = 0
        for img, r, L in imgs_rl:
            oracle_mod.oilpaint_ref(img, r, L, nthreads=th)
            px += img.shape[0] * img.shape[1]
        dt = time.perf_counter() - t0
        out[name] = {"s": round(dt, 3), "mp_per_s": round(px / 1e6 / dt, 3), "threads": th,
                     "megapixels": round(px / 1e6, 2)}
    small, r, L = synth.small_case()
    fhd = synth.fhd_image()
    timed("256x256_r2_L20_T1", [(small, r, L)], 1)
    timed("256x256_r2_L20_T2", [(small, r, L)], threads)
    timed("1920x1080_sweep_T1", [(fhd, r_, L_) for r_, L_ in synth.FHD_SWEEP], 1)
    timed("4000x3000_r10_L32_T2", [(synth.camera_image(),) + tuple(synth.CAMERA_RL)], threads)
    batch = [(synth.batch_image(it).cpu().numpy(), it.radius, it.levels) for it in synth.batch_items()]
    timed("batch64_T2", batch, threads)
    for name in ("256x256_r2_L20", ):
        out[name + "_speedup_T1_over_T2"] = round(out[name + "_T1"]["s"] / out[name + "_T2"]["s"], 2)
    return out


SETTLE_S = 0.03


def settle(torch, step, seconds: float = SETTLE_S, max_steps: int = 2000) -> int:
    """Run `step` untimed, eight at a time, until `seconds` of wall time have
    passed: after the host-side set-up (the image, tuning) the GPU comes back
    from idle, and the first few milliseconds of work run slower (the first
    20 sweep steps timed straight after set-up: 260 us each, then 250, then
    246 once settled).  Returns the number of steps run."""
    n = 0
    t0 = time.perf_counter()
    while n < max_steps and time.perf_counter() - t0 < seconds:
        for _ in range(8):
            step()
        torch.cuda.synchronize()
        n += 8
    return n


def bench_plain(torch, B, synth, timer, steps, warmup):
    img = synth.fhd_image()
    src = torch.from_numpy(img).cuda()
    dst = torch.empty_like(src)
    runs = synth.FHD_SWEEP
    mp = img.shape[0] * img.shape[1] / 1e6

    def step():
        for r, L in runs:
            B.oilpaint_async(src, dst, r, L)

    settle_steps = settle(torch, step)
    ms_step = timer.time(step, steps, warmup)
    per = {}
    for r, L in runs:
        reps = max(steps, 20)
        ms = timer.time(lambda: B.oilpaint_async(src, dst, r, L), reps, 3)
        each = timer.each(lambda: B.oilpaint_async(src, dst, r, L), reps)
        v = B.pick_variant(img.shape[1], img.shape[0], r, L)
        per["r%d_L%d" % (r, L)] = {"r": r, "L": L, "ms": round(ms, 5), "mp_per_s": round(mp / (ms / 1e3), 1),
                                   "median_ms": round(each[len(each) // 2], 5), "min_ms": round(each[0], 5),
                                   "reps": reps,
                                   "lds_gbs": round(lds_bytes_per_pixel(r, L) * mp * 1e6 / (ms / 1e3) / 1e9, 1),
                                   "kernel": kernel_name(r, L, v), "variant": list(v.as_tuple())}
    total_bytes = sum(lds_bytes_per_pixel(r, L) for r, L in runs) * mp * 1e6
    achieved = total_bytes / (ms_step / 1e3) / 1e9
    return img, src, ms_step, mp * len(runs), per, achieved, settle_steps


def bench_single(torch, B, timer, img, r, L, reps):
    src = torch.from_numpy(img).cuda()
    dst = torch.empty_like(src)
    ms = timer.time(lambda: B.oilpaint_async(src, dst, r, L), reps, 3)
    mp = img.shape[0] * img.shape[1] / 1e6
    return {"ms": round(ms, 5), "mp_per_s": round(mp / (ms / 1e3), 1),
            "lds_gbs": round(lds_bytes_per_pixel(r, L) * mp * 1e6 / (ms / 1e3) / 1e9, 1)}


LARGE_RADII = (16, 32, 64, 128)


def bench_large_radius(torch, B, synth, timer, oracle_mod) -> dict:
    """Radii above the streamed layout's 15 on the 1920x1080 image (L = 20):
    the tuned launch (column histograms) against the wide layout, whose
    work grows with the radius, and a seeded sample of output pixels against
    the oracle (each pixel filtered on the crop of its own window)."""
    import numpy as np
    img = synth.fhd_image()
    src = torch.from_numpy(img).cuda()
    dst = torch.empty_like(src)
    h, w = img.shape[:2]
    mp = w * h / 1e6
    rng = np.random.default_rng(13)
    out = {}
    for r in LARGE_RADII:
        L = 20
        v = B.pick_variant(w, h, r, L)
        reps = 10 if r <= 32 else 3
        ms = timer.time(lambda: B.oilpaint_async(src, dst, r, L), reps, 1)
        wide = B.tune_times(w, h, r, L, [B.Variant(16, 2, B.HIST_WIDE, 64, 1)], reps=1 if r > 32 else 3)[0]
        B.oilpaint_async(src, dst, r, L)
        got = dst.cpu().numpy()
        ok = 0
        pts = [(int(rng.integers(0, w)), int(rng.integers(0, h))) for _ in range(12)] + [(0, 0), (w - 1, h - 1)]
        for x, y in pts:
            y0, y1, x0, x1 = max(0, y - r), min(h, y + r + 1), max(0, x - r), min(w, x + r + 1)
            want = oracle_mod.oilpaint_ref(np.ascontiguousarray(img[y0:y1, x0:x1]), r, L)[y - y0, x - x0]
            ok += int((got[y, x] == want).all())
        out["r%d_L%d" % (r, L)] = {"ms": round(ms, 4), "mp_per_s": round(mp / (ms / 1e3), 1),
                                   "kernel": kernel_name(r, L, v), "variant": list(v.as_tuple()),
                                   "wide_ms": round(wide, 4), "wide_mp_per_s": round(mp / (wide / 1e3), 1),
                                   "speedup_vs_wide": round(wide / ms, 2),
                                   "oracle_pixels": "%d/%d" % (ok, len(pts))}
    return out


def bench_median(torch, B, synth, timer, oracle_mod, threads: int) -> dict:
    """The windowed median of one channel (the second filter of the class) on
    the 1920x1080 image, channel 1, with each radius's tuned kernel form (one
    or four wavefronts per strip, or column histograms): MP/s per radius; the
    whole output against the median oracle at r = 1, 5, 15 and 32, sampled
    pixels (each by sorting its window) at r = 64 and 127."""
    import numpy as np
    from paper_1405_1020_amd import tune
    img = synth.fhd_image()
    src = torch.from_numpy(img).cuda()
    h, w = img.shape[:2]
    dst = torch.empty(h, w, dtype=torch.uint8, device="cuda")
    mp = w * h / 1e6
    radii = (1, 2, 5, 10, 15, 16, 32, 64, 127)
    tuned = tune.ensure_median(radii, w, h)
    rng = np.random.default_rng(17)
    out = {}
    for r in radii:
        reps = 20 if r <= 32 else 5
        ms = timer.time(lambda: B.median_async(src, dst, r, 1), reps, 2)
        e = {"ms": round(ms, 5), "mp_per_s": round(mp / (ms / 1e3), 1), "kind": tuned[str(r)]["kind"],
             "forms_ms": {str(k): round(t, 4) for k, t in tuned[str(r)]["all"]}}
        B.median_async(src, dst, r, 1)
        torch.cuda.synchronize()
        got = dst.cpu().numpy()
        if r in (1, 5, 15, 32):
            want = oracle_mod.median_ref(img, r, 1, nthreads=threads)
            e["pixels_differing"] = int((got != want).sum())
        elif r in (64, 127):
            pts = [(0, 0), (w - 1, h - 1)] + [(int(rng.integers(0, w)), int(rng.integers(0, h))) for _ in range(14)]
            ok = 0
            for x, y in pts:
                ok += int(oracle_mod.median_at(img, x, y, r, 1) == got[y, x])
            e["oracle_pixels"] = "%d/%d" % (ok, len(pts))
        out["r%d" % r] = e
    return out

def bench_register_histograms(B, tune) -> dict:
    """Histograms in registers (OILPAINT_HIST_REGS) against the tuned launch
    shape, on a 1920x1080 tuning image (the library's photo-like fill), by
    the library's own timer: the fastest register-histogram density and the
    tuned shape's time, per (r, L)."""
    out = {}
    for r, L in ((1, 8), (2, 8), (3, 8), (5, 8), (1, 16), (2, 16), (3, 16), (5, 16)):
        regs = [v for v in tune.candidates(r, L) if v.hist == B.HIST_REGS]
        t_regs = B.tune_times(1920, 1080, r, L, regs, reps=5)
        tuned = B.pick_variant(1920, 1080, r, L)
        t_tuned = B.tune_times(1920, 1080, r, L, [tuned], reps=5)[0]
        k = min((i for i in range(len(regs)) if t_regs[i] >= 0), key=lambda i: t_regs[i])
        out["r%d_L%d" % (r, L)] = {"regs_ms": round(t_regs[k], 4), "regs_per_cu": regs[k].per_cu,
                                   "tuned_ms": round(t_tuned, 4), "tuned_variant": list(tuned.as_tuple()),
                                   "regs_over_tuned": round(t_regs[k] / t_tuned, 2)}
    return out


PAPER_SIZES = ((640, 480), (800, 600), (1024, 768), (1920, 1080), (2560, 1600))


def bench_jpeg(torch, B, synth, oracle_mod, threads: int, reps: int = 5) -> dict:
    """The paper's program around the filter (Section 3: decode a JPEG file,
    filter, encode; the three steps timed apart), at the paper's image sizes
    and radii (r = 2, 4, 6, 8; L = 20, the paper states none): a JPEG file in
    host memory (the blob image at that size, encoded by PIL at quality 90,
    4:2:0) is decoded onto the device (markers parsed and stripped on the
    host, upload, Huffman decoding, inverse DCT and colour kernels), filtered
    there, and encoded from there
    (colour, FDCT and quantization kernels, Huffman statistics on the
    device, tables fitted on the host, Huffman coding and byte stuffing on
    the device, download; same quality and subsampling).  Each step is timed
    on the host clock around the call and a device synchronization (median
    of `reps`); the host's share (decode: parsing, stripping the markers and
    planning the subsequences; encode: fitting the tables and writing the
    headers) is reported beside it.  The
    filter's output on the 1920x1080 decoded image is checked against the
    oracle on those decoded pixels."""
    import io
    import statistics
    import numpy as np
    from PIL import Image
    out = {"format": "baseline JPEG, quality 90, 4:2:0 (input by PIL; output by this library)", "L": 20,
           "sizes": {}}
    for w, h in PAPER_SIZES:
        img = synth.make_image(w, h, seed=w, **synth.LARGE_BLOBS)
        b = io.BytesIO()
        Image.fromarray(img).save(b, format="JPEG", quality=90, subsampling=2)
        data = b.getvalue()
        dev = torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(dev)
        dec, dec_host, enc, enc_host = [], [], [], []
        proc = {r: [] for r in (2, 4, 6, 8)}
        for k in range(reps + 1):
            t = {}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.jpeg_decode(data, out=dev, times=t)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            dh = t["host_ms"]
            for r in proc:
                t2 = time.perf_counter()
                B.oilpaint_async(dev, dst, r, 20)
                torch.cuda.synchronize()
                if k:
                    proc[r].append((time.perf_counter() - t2) * 1e3)
            t3 = time.perf_counter()
            enc_bytes = B.jpeg_encode(dst, quality=90, subsampling=2, times=t)
            t4 = time.perf_counter()
            if k:  # the first pass warms up
                dec.append((t1 - t0) * 1e3)
                dec_host.append(dh)
                enc.append((t4 - t3) * 1e3)
                enc_host.append(t["host_ms"])
        mp = w * h / 1e6
        e = {"jpeg_bytes": len(data), "encoded_bytes": len(enc_bytes),
             "decode_ms": round(statistics.median(dec), 3), "decode_host_ms": round(statistics.median(dec_host), 3),
             "encode_ms": round(statistics.median(enc), 3), "encode_host_tables_ms": round(statistics.median(enc_host), 3),
             "process_ms": {"r%d" % r: round(statistics.median(v), 4) for r, v in proc.items()}}
        e["decode_mp_per_s"] = round(mp / (e["decode_ms"] / 1e3), 1)
        e["encode_mp_per_s"] = round(mp / (e["encode_ms"] / 1e3), 1)
        if (w, h) == (1920, 1080):
            B.oilpaint_async(dev, dst, 2, 20)
            torch.cuda.synchronize()
            want = oracle_mod.oilpaint_ref(dev.cpu().numpy(), 2, 20, nthreads=threads)
            e["filter_on_decoded_pixels_differing"] = int((dst.cpu().numpy() != want).any(axis=-1).sum())
        out["sizes"]["%dx%d" % (w, h)] = e
    return out


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
    model = sum(lds_bytes_per_pixel(it.radius, it.levels) * it.width * it.height for it in specs)

    def frac(ms):
        return round(model / (ms / 1e3) / 1e9 / LDS_PEAK_GBS, 4)
    return {
        "workload": "64 images, W~U{320..4096}, H~U{240..3072}, r~U{2,3,5,8}, L~U{16,20,32}",
        "megapixels": round(mp, 2),
        "model_lds_bytes": model,
        "graph_roofline_frac": frac(ms_graph), "plain_roofline_frac": frac(ms_plain),
        "batch_call_roofline_frac": frac(ms_batch),
        "plain_ms": round(ms_plain, 4), "plain_mp_per_s": round(mp / (ms_plain / 1e3), 1),
        "graph_ms": round(ms_graph, 4), "graph_mp_per_s": round(mp / (ms_graph / 1e3), 1),
        "batch_call_ms": round(ms_batch, 4), "batch_call_mp_per_s": round(mp / (ms_batch / 1e3), 1),
        "graph_vs_plain": round(ms_plain / ms_graph, 3),
        "tiles": tiles, "workgroups": wgs,
        "outputs_equal_plain": bool(same),
    }


def bench_serving(torch, B, synth, serve, n_requests, oracle_mod, oracle_threads: int):
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
        # light load: outputs allocated up front and kept (verification);
        # saturation: allocated at admission, released at completion
        alloc, free = serve.device_allocator(keep=not saturate, preallocate=None if saturate else rs)
        s = serve.Server(ex, budget_bytes=budget, capacity=4096, allocate=alloc, free=free)
        st = serve.run_open_loop(s, rs)
        ex.close()
        torch.cuda.synchronize()
        return st, rs

    st_q, rs_q = one("queue", False)
    log("served (queue):", st_q)
    st_p, rs_p = one("plain", False)
    log("served (plain):", st_p)
    # verification: every served output equals the same request filtered by
    # the plain kernel alone; a sample against the CPU oracle (pixels whose
    # windows are cut out and filtered)
    equal = sum(int(torch.equal(a.dst, b.dst)) for a, b in zip(rs_q, rs_p))
    for q in rs_p:
        q.dst = None
    torch.cuda.synchronize()
    import numpy as np
    rng = np.random.default_rng(5)
    # whole outputs against the oracle: every request of at most 0.5 MP, and
    # a seeded 5 % of the larger ones
    small = [q for q in rs_q if q.pixels <= 500_000]
    large = [q for q in rs_q if q.pixels > 500_000]
    pick_l = sorted(rng.choice(len(large), size=max(1, len(large) // 20), replace=False).tolist()) if large else []
    sample = small + [large[i] for i in pick_l]
    oracle_ok = 0
    t0 = time.perf_counter()
    for q in sample:
        img = q.src.contiguous().cpu().numpy()
        want = oracle_mod.oilpaint_ref(img, q.radius, q.levels, nthreads=oracle_threads)
        oracle_ok += int(np.array_equal(want, q.dst.cpu().numpy()))
    oracle_s = time.perf_counter() - t0
    for q in rs_q:
        q.dst = None
    torch.cuda.synchronize()
    sat_q, _ = one("queue", True)
    sat_p, _ = one("plain", True)
    model = sum(lds_bytes_per_pixel(q.radius, q.levels) * q.width * q.height for q in wl.requests)

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
        "oracle_outputs": "%d/%d" % (oracle_ok, len(sample)),
        "oracle_sample": "whole outputs of all %d requests <= 0.5 MP and a seeded 5 %% (%d) of the %d larger "
                         "ones, %.1f MP, %.1f s on %d threads" % (len(small), len(pick_l), len(large),
                                                                 sum(q.pixels for q in sample) / 1e6, oracle_s,
                                                                 oracle_threads),
        "model_lds_bytes": model,
        "saturation_roofline_frac": round(model / sat_q["span_s"] / 1e9 / LDS_PEAK_GBS, 4),
        "saturation_plain_roofline_frac": round(model / sat_p["span_s"] / 1e9 / LDS_PEAK_GBS, 4),
    })
    return out


def cpu_baseline(oracle_mod, img, runs, cpu: dict):
    threads = cpu["threads"]
    t0 = time.perf_counter()
    for r, L in runs:
        oracle_mod.oilpaint_ref(img, r, L, nthreads=threads)
    dt = time.perf_counter() - t0
    mp = img.shape[0] * img.shape[1] / 1e6 * len(runs)
    return {"value": round(mp / dt, 3), "unit": "MP/s", "cores": threads, "kind": "oracle",
            "sample": "the full 1920x1080 sweep (7 runs), row bands over %d threads, %.1f s wall" % (threads, dt),
            "cpu_model": cpu["model"], "host_cpus": cpu["cpu_count"], "affinity_cpus": cpu["affinity"]}


def hbm_traffic(kernel: str, config: str, variant=None):
    """HBM bytes per launch of `kernel` on sweep run `config`, from the
    committed counter summary, if it was taken on the current kernel source
    and (when given) the same resolved launch shape (else None)."""
    try:
        d = json.load(open(HBM_PROFILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    e = d.get("launches", {}).get(config)
    if not e or e.get("kernel") != kernel:
        return None
    if variant is not None and list(e.get("variant", [])) != list(variant):
        return None
    return e.get("hbm_bytes_per_launch")


def _kernel_short_name(full: str) -> str:
    import re
    m = re.search(r"(k_\w+(?:<[\d, ]+>)?)\(", full)
    return m.group(1) if m else full


def _pmc_rows(folder: str, counter: str):
    """(file, dispatch id, kernel name, grid size, value) of every dispatch
    in a rocprofv3 --pmc CSV output under `folder` (a file per process), in
    dispatch order."""
    import csv
    import glob
    out = []
    for f in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            if row.get("Counter_Name") != counter:
                continue
            out.append((f, int(row.get("Dispatch_Id", 0) or 0), _kernel_short_name(row["Kernel_Name"]),
                        int(row.get("Grid_Size", 0) or 0), float(row["Counter_Value"])))
    return sorted(out)


def _trace_rows(folder: str):
    """(file, dispatch id, kernel name, grid size, duration in ns) of every
    dispatch in a rocprofv3 --kernel-trace CSV output under `folder`, in
    dispatch order."""
    import csv
    import glob
    out = []
    for f in glob.glob(os.path.join(folder, "**", "*kernel_trace.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            grid = int(row["Grid_Size_X"]) * int(row["Grid_Size_Y"]) * int(row["Grid_Size_Z"])
            out.append((f, int(row["Dispatch_Id"]), _kernel_short_name(row["Kernel_Name"]), grid,
                        float(row["End_Timestamp"]) - float(row["Start_Timestamp"])))
    return sorted(out)


def sweep_run_values(rows, runs) -> dict:
    """Per sweep run, the values of its dispatches.  `rows` are (file,
    dispatch id, kernel, grid, value) in dispatch order; `runs` are (run,
    kernel, grid) in the order one step launches them.  A dispatch belongs to
    the run with its kernel and grid.  Runs that share both (a kernel whose
    radius is an argument) follow each other in the sweep and are launched
    the same number of times in each phase of bench_plain (a step launches
    every run once; then each run is timed alone), so each maximal block of
    consecutive such dispatches splits into equal parts, in run order; a
    block that does not split evenly is left out."""
    out = {run: [] for run, _, _ in runs}
    index = {}
    for i, (_, k, g) in enumerate(runs):
        index.setdefault((k, g), []).append(i)
    i = 0
    while i < len(rows):
        f, _, k, g, _ = rows[i]
        j = i
        while j < len(rows) and rows[j][0] == f and rows[j][2] == k and rows[j][3] == g:
            j += 1
        idx = index.get((k, g), [])
        n, m = j - i, len(idx)
        if m and n % m == 0:
            for part, ri in enumerate(idx):
                out[runs[ri][0]].extend(v for *_, v in rows[i + part * (n // m):i + (part + 1) * (n // m)])
        i = j
    return out


def sweep_runs(sweep_json: str, w: int = 1920, h: int = 1080):
    """(run, kernel, grid work-items, variant) of the 1920x1080 sweep's runs
    in launch order, as the bench output `sweep_json` (the last JSON line of
    a `bench.py --quick` run) records them."""
    from paper_1405_1020_amd import synth
    line = [x for x in open(sweep_json).read().splitlines() if x.startswith("{")][-1]
    sweep = json.loads(line)["sweep"]
    out = []
    for r, L in synth.FHD_SWEEP:
        e = sweep["r%d_L%d" % (r, L)]
        out.append(("r%d_L%d" % (r, L), e["kernel"], launch_threads(w, h, e["variant"]), list(e["variant"])))
    return out


def trace_summary(folder: str, sweep_json: str) -> dict:
    """Per sweep run, the kernel-trace durations of its dispatches (the
    `--kernel-trace` output under `folder` of `bench.py --quick`, whose
    launch shapes `sweep_json` records)."""
    import statistics
    runs = sweep_runs(sweep_json)
    vals = sweep_run_values(_trace_rows(folder), [(n, k, g) for n, k, g, _ in runs])
    return {n: {"kernel": k, "grid_threads": g, "dispatches": len(vals[n]),
                "mean_us": round(statistics.fmean(vals[n]) / 1e3, 2) if vals[n] else None,
                "median_us": round(statistics.median(vals[n]) / 1e3, 2) if vals[n] else None}
            for n, k, g, _ in runs}


def launch_threads(w: int, h: int, variant) -> int:
    """Work-items of a plain launch of a w x h image with a resolved variant
    (rows, waves, hist, lanes, per_cu): one workgroup of 64 x waves per tile
    (the profiler's grid size); a tile spans waves x rows output rows, except
    in the streamed and column layouts (hist 1, 3 and 4), whose wavefronts
    share one run."""
    rows, waves, hist, lanes = variant[0], variant[1], variant[2], variant[3]
    runs = 1 if hist in (1, 3, 4) else waves
    tiles = -(-w // lanes) * -(-h // (runs * rows))
    return tiles * 64 * waves


def hbm_entry(folder: str, run: str, runs, w: int, h: int, scale: dict) -> dict:
    """Counters per dispatch of one sweep run (its dispatches as
    sweep_run_values attributes them); `runs` as sweep_runs gives them."""
    import statistics
    name, grid, variant = next((k, g, v) for n, k, g, v in runs if n == run)
    e = {"kernel": name, "variant": variant, "grid_threads": grid}
    for c, sub in (("FETCH_SIZE", "sweep_fetch"), ("WRITE_SIZE", "sweep_write")):
        vals = sweep_run_values(_pmc_rows(os.path.join(folder, sub), c), [(n, k, g) for n, k, g, _ in runs])[run]
        e[c.lower() + "_kib_per_dispatch"] = round(statistics.median(vals), 1) if vals else None
        e[c.lower() + "_dispatches"] = len(vals)
    if e["fetch_size_kib_per_dispatch"] is not None and e["write_size_kib_per_dispatch"] is not None:
        e["hbm_bytes_per_launch"] = round(e["fetch_size_kib_per_dispatch"] * 1024 * scale["FETCH_SIZE"] +
                                          e["write_size_kib_per_dispatch"] * 1024 * scale["WRITE_SIZE"])
        e["algorithmic_hbm_bytes"] = 6 * w * h
    return e


def write_hbm_summary(folder: str, sweep_json: str, commands: list[str]):
    """Turn four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE over
    `bench.py --quick` and over `bench.py --copy-ref`, in the sub-folders
    sweep_fetch, sweep_write, copy_fetch and copy_write of `folder`) into
    the committed HBM summary: per sweep run, the counters per dispatch of
    its kernel, scaled so that the copy kernel's counters read its known
    bytes."""
    import statistics
    copy_bytes = 1 << 30
    scale = {}
    for c, sub in (("FETCH_SIZE", "copy_fetch"), ("WRITE_SIZE", "copy_write")):
        vals = [v for _, _, n, g, v in _pmc_rows(os.path.join(folder, sub), c) if g >= (1 << 20)]
        scale[c] = copy_bytes / (statistics.median(vals) * 1024.0)
    w, h = 1920, 1080
    runs = sweep_runs(sweep_json, w, h)
    launches = {n: hbm_entry(folder, n, runs, w, h, scale) for n, _, _, _ in runs}
    out = {"kernel_source_sha": kernel_source_hash(), "workload": "fhd_1920x1080_sweep",
           "commands": commands, "copy_reference": {"bytes_read": copy_bytes, "bytes_written": copy_bytes,
                                                     "scale": {k: round(v_, 4) for k, v_ in scale.items()}},
           "launches": launches}
    with open(HBM_PROFILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def _pmc_all(folder: str):
    """{(file, dispatch id): {"kernel", "grid", counter: value, ...}} from a
    rocprofv3 --pmc CSV output under `folder`."""
    import csv
    import glob
    out = {}
    for f in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            key = (f, int(row.get("Dispatch_Id", 0) or 0))
            e = out.setdefault(key, {"kernel": _kernel_short_name(row["Kernel_Name"]),
                                     "grid": int(row.get("Grid_Size", 0) or 0)})
            e[row["Counter_Name"]] = e.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    return out


def _trace_by_kernel(folder: str) -> dict:
    """{(kernel, grid): [durations in ns]} from a --kernel-trace output."""
    out = {}
    for _, _, k, g, d in _trace_rows(folder):
        out.setdefault((k, g), []).append(d)
    return out


def counter_metrics(disp: list, durations_ns: list, cus: int, pixels: float) -> dict:
    """Figures of a group of dispatches of one kernel (counters averaged per
    dispatch).  rocprofiler-sdk's own gfx950 metrics where the derived pass
    recorded them (LdsUtil, VALUBusy and OccupancyPercent in per cent,
    LdsBankConflict as a ratio, VALUUtilization in per cent); else the same
    definitions from the raw counters: LdsUtil = LDS_IDX_ACTIVE /
    (GRBM_GUI_ACTIVE x CUs), LdsBankConflict = BANK_CONFLICT /
    (LDS_IDX_ACTIVE - BANK_CONFLICT), VALUBusy = ACTIVE_INST_VALU / (CUs x
    GRBM_GUI_ACTIVE), VALUUtilization = THREAD_CYCLES_VALU /
    (ACTIVE_INST_VALU x 64), occupancy = 4 x WAVE_CYCLES / (GRBM_GUI_ACTIVE
    x CUs x 32), with GRBM_GUI_ACTIVE per XCD (the raw sum over XCDS)."""
    import statistics

    def mean(c):
        vals = [d[c] for d in disp if c in d]
        return statistics.fmean(vals) if vals else None
    m = {c: mean(c) for c in set().union(*[set(d) for d in disp]) if c not in ("kernel", "grid")}
    gui = m.get("GRBM_GUI_ACTIVE")
    if gui:
        gui /= XCDS
    out = {"dispatches": len(disp)}
    if durations_ns:
        out["trace_mean_us"] = round(statistics.fmean(durations_ns) / 1e3, 2)
    if gui:
        if m.get("SQ_LDS_IDX_ACTIVE") is not None:
            out["lds_util"] = round(m["SQ_LDS_IDX_ACTIVE"] / (gui * cus), 4)
            act = m["SQ_LDS_IDX_ACTIVE"] - m.get("SQ_LDS_BANK_CONFLICT", 0.0)
            if act > 0:
                out["lds_bank_conflict_rate"] = round(m.get("SQ_LDS_BANK_CONFLICT", 0.0) / act, 4)
        if m.get("SQ_ACTIVE_INST_VALU") is not None:
            out["valu_busy"] = round(m["SQ_ACTIVE_INST_VALU"] / (cus * gui), 4)
            if m["SQ_ACTIVE_INST_VALU"] > 0 and m.get("SQ_THREAD_CYCLES_VALU") is not None:
                out["valu_utilization"] = round(m["SQ_THREAD_CYCLES_VALU"] / (m["SQ_ACTIVE_INST_VALU"] * 64), 4)
        if m.get("SQ_WAVE_CYCLES") is not None:
            out["occupancy"] = round(4 * m["SQ_WAVE_CYCLES"] / (gui * cus * 32), 4)
    if pixels:
        for c, k in (("SQ_INSTS_LDS", "lds_insts_per_pixel"), ("SQ_INSTS_VALU", "valu_insts_per_pixel"),
                     ("SQ_INSTS_SALU", "salu_insts_per_pixel")):
            if m.get(c) is not None:
                out[k] = round(m[c] / pixels, 3)
    # rocprofiler-sdk's own figures, where recorded, take precedence
    for c, k, scale in (("LdsUtil", "lds_util", 0.01), ("VALUBusy", "valu_busy", 0.01),
                        ("LdsBankConflict", "lds_bank_conflict_rate", 1.0), ("OccupancyPercent", "occupancy", 0.01),
                        ("VALUUtilization", "valu_utilization", 0.01)):
        if m.get(c) is not None:
            if k in out:
                out[k + "_raw"] = out[k]
            out[k] = round(m[c] * scale, 4)
    if "lds_util" in out and "valu_busy" in out:
        out["binding_unit"] = "lds" if out["lds_util"] >= out["valu_busy"] else "valu"
    out["counters_mean"] = {c: round(v, 1) for c, v in sorted(m.items()) if v is not None}
    return out


def write_counter_summary(folder: str, sweep_json: str, cus: int = 256):
    """Per sweep run (and per kernel of the camera and batched workloads) the
    LDS and VALU counters of COUNTER_PASSES, from rocprofv3 --pmc runs in the
    sub-folders <workload>_<pass> of `folder` (COUNTER_WORKLOADS), into
    profiles/lds_valu_counters.json and .md."""
    from paper_1405_1020_amd import synth
    runs = sweep_runs(sweep_json)
    line = [x for x in open(sweep_json).read().splitlines() if x.startswith("{")][-1]
    per = json.loads(line)["sweep"]
    out = {"kernel_source_sha": kernel_source_hash(), "cus": cus,
           "passes": COUNTER_PASSES, "workloads": COUNTER_WORKLOADS, "sweep": {}, "camera": {}, "batched": {}}
    # sweep: attribute dispatches to runs as the HBM summary does
    sweep_disp = {}
    sweep_dur = {}
    for pname in COUNTER_PASSES:
        sub = os.path.join(folder, "sweep_" + pname)
        allc = _pmc_all(sub)
        rows = sorted((f, i, e["kernel"], e["grid"], e) for (f, i), e in allc.items())
        vals = sweep_run_values(rows, [(n, k, g) for n, k, g, _ in runs])
        for n in vals:
            sweep_disp.setdefault(n, []).extend(vals[n])
        tr = sweep_run_values(_trace_rows(sub), [(n, k, g) for n, k, g, _ in runs])
        for n in tr:
            sweep_dur.setdefault(n, []).extend(tr[n])
    for n, k, g, v in runs:
        e = counter_metrics(sweep_disp.get(n, []), sweep_dur.get(n, []), cus, 1920 * 1080)
        e.update({"kernel": k, "variant": v, "event_ms": per[n]["ms"]})
        out["sweep"][n] = e
    camera_px = 4000 * 3000
    batch_px = sum(it.width * it.height for it in synth.batch_items())
    for wl, px in (("camera", camera_px), ("batched", batch_px)):
        groups, durs = {}, {}
        for pname in COUNTER_PASSES:
            sub = os.path.join(folder, wl + "_" + pname)
            for (_, _), e in _pmc_all(sub).items():
                if e["kernel"].startswith(("k_plain", "k_batch")):
                    groups.setdefault(e["kernel"], []).append(e)
            for (k, g), d in _trace_by_kernel(sub).items():
                if k.startswith(("k_plain", "k_batch")):
                    durs.setdefault(k, []).extend(d)
        for k, disp in groups.items():
            out[wl][k] = counter_metrics(disp, durs.get(k, []), cus, px if wl == "camera" else 0)
    with open(COUNTER_PROFILE, "w") as f:
        json.dump(out, f, indent=1)
    md = ["# LDS and VALU counters: 1920x1080 sweep, 4000x3000 camera, 64-image batch", "",
          "Counter passes (one `rocprofv3 --pmc` run each, with `--kernel-trace` for durations), per workload "
          "(`$REPO` the repository root, `$OUT` an output folder; the first line fills the tuning cache and "
          "records the sweep's launch shapes):", "", "```",
          "python3 bench.py --quick --steps 20 --warmup 3 > $OUT/quick.json", "cd /tmp && export TMPDIR=/tmp"]
    for wl, cmd in COUNTER_WORKLOADS.items():
        for pname, cs in COUNTER_PASSES.items():
            md.append("timeout -s KILL 120 rocprofv3 --kernel-trace --pmc %s -d $OUT/%s_%s --output-format csv -- "
                      "python3 $REPO/%s" % (" ".join(cs), wl, pname, cmd))
    md += ["cd $REPO && python3 bench.py --counter-summary $OUT --sweep-json $OUT/quick.json", "```", "",
           "Figures per dispatch (averages over a kernel's dispatches; %d CUs): LDS busy, bank conflicts, VALU "
           "busy, VALU lanes and occupancy are rocprofiler-sdk's gfx950 metrics LdsUtil (SQ_LDS_IDX_ACTIVE / "
           "(GRBM_GUI_ACTIVE x CUs)), LdsBankConflict (SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - "
           "SQ_LDS_BANK_CONFLICT)), VALUBusy (SQ_ACTIVE_INST_VALU / (GRBM_GUI_ACTIVE x CUs)), VALUUtilization "
           "(SQ_THREAD_CYCLES_VALU / (64 x SQ_ACTIVE_INST_VALU)) and OccupancyPercent (4 x SQ_WAVE_CYCLES / "
           "(GRBM_GUI_ACTIVE x CUs x 32)), from the derived pass; instructions per output pixel from the raw "
           "passes (SQ_INSTS_LDS, SQ_INSTS_VALU: wavefront instructions). Traced us: the kernel trace of the "
           "counter runs (counter collection serializes and slows dispatches a little). The binding unit is the "
           "busier of LDS and VALU." % cus, "",
           "| Workload | Kernel | Dispatches | Traced us | LDS busy | Bank conflicts | VALU busy | "
           "VALU lanes | Occupancy | LDS instr/px | VALU instr/px | Binding |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|"]

    def row(wl, k, e):
        def f(x, pct=False):
            if x is None:
                return "-"
            return "%.1f %%" % (100 * x) if pct else str(x)
        return "| %s | `%s` | %s | %s | %s | %s | %s | %s | %s | %s | %s | %s |" % (
            wl, k, e.get("dispatches"), f(e.get("trace_mean_us")),
            f(e.get("lds_util"), True), f(e.get("lds_bank_conflict_rate"), True), f(e.get("valu_busy"), True),
            f(e.get("valu_utilization"), True), f(e.get("occupancy"), True), f(e.get("lds_insts_per_pixel")),
            f(e.get("valu_insts_per_pixel")), e.get("binding_unit", "-"))
    for n, e in out["sweep"].items():
        md.append(row("sweep " + n, e["kernel"], e))
    for wl in ("camera", "batched"):
        for k, e in sorted(out[wl].items()):
            md.append(row(wl, k, e))
    md += ["", "Kernel source hash of these figures: `%s`." % out["kernel_source_sha"], ""]
    with open(COUNTER_SUMMARY, "w") as f:
        f.write("\n".join(md))
    print(json.dumps(out))


def counter_fields(run: str):
    """Counter-derived figures of a sweep run from the committed summary, if
    it was taken on the current kernel sources (else None)."""
    try:
        d = json.load(open(COUNTER_PROFILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    e = d.get("sweep", {}).get(run)
    if not e:
        return None
    return {k: e[k] for k in ("lds_util", "lds_bank_conflict_rate", "valu_busy", "valu_utilization", "occupancy",
                              "binding_unit", "kernel") if k in e}


def counter_workload(name: str, torch, B, synth):
    """The camera (4000x3000, r = 10, L = 32: five plain launches) or the
    64-image batch (three replays of its captured plan), after tuning, for
    the counter passes; or the JPEG leg's decode / filter (r = 2, 4, 6, 8,
    L = 20) / encode at 640x480 or 1920x1080, six rounds, for a kernel
    trace."""
    from paper_1405_1020_amd import tune
    if name in ("jpeg640", "jpeg1920"):
        import io
        from PIL import Image
        w, h = (640, 480) if name == "jpeg640" else (1920, 1080)
        tune.ensure([(r, 20) for r in (2, 4, 6, 8)], w, h)
        img = synth.make_image(w, h, seed=w, **synth.LARGE_BLOBS)
        b = io.BytesIO()
        Image.fromarray(img).save(b, format="JPEG", quality=90, subsampling=2)
        data = b.getvalue()
        dev = torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(dev)
        for _ in range(6):
            B.jpeg_decode(data, out=dev)
            for r in (2, 4, 6, 8):
                B.oilpaint_async(dev, dst, r, 20)
            B.jpeg_encode(dst, quality=90, subsampling=2)
    elif name == "camera":
        tune.ensure([synth.CAMERA_RL], 4000, 3000)
        src = torch.from_numpy(synth.camera_image()).cuda()
        dst = torch.empty_like(src)
        for _ in range(5):
            B.oilpaint_async(src, dst, *synth.CAMERA_RL)
    elif name == "batched":
        tune.ensure([(r, L) for r in (2, 3, 5, 8) for L in (16, 20, 32)], 2048, 1536)
        specs = synth.batch_items()
        srcs = [synth.batch_image(it) for it in specs]
        items = [B.Item(s_, torch.empty_like(s_), it.radius, it.levels) for s_, it in zip(srcs, specs)]
        plan = B.Plan(items)
        for _ in range(3):
            plan.launch()
        torch.cuda.synchronize()
        plan.close()
    else:
        raise ValueError(name)
    torch.cuda.synchronize()
    print(json.dumps({"counter_workload": name}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="main sweep only (for profiling)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--copy-ref", action="store_true",
                    help="run only a plain 1 GiB device copy kernel (HBM counter scaling) and exit")
    ap.add_argument("--hbm-summary", metavar="DIR",
                    help="write the HBM counter summary under profiles/ from rocprofv3 --pmc outputs in DIR")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="print per sweep run the kernel-trace durations from rocprofv3 --kernel-trace output in DIR")
    ap.add_argument("--counter-summary", metavar="DIR",
                    help="write the LDS/VALU counter summary under profiles/ from the counter passes in DIR")
    ap.add_argument("--counter-workload", choices=["camera", "batched", "jpeg640", "jpeg1920"],
                    help="run only that workload (for a counter pass) and exit")
    ap.add_argument("--sweep-json", metavar="FILE",
                    help="with --hbm-summary or --trace-summary: the output of the profiled bench.py --quick run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.counter_summary:
        if not args.sweep_json:
            ap.error("--sweep-json is required with --counter-summary")
        write_counter_summary(args.counter_summary, args.sweep_json)
        return
    if args.hbm_summary or args.trace_summary:
        if not args.sweep_json:
            ap.error("--sweep-json is required with --hbm-summary and --trace-summary")
        if args.hbm_summary:
            write_hbm_summary(args.hbm_summary, args.sweep_json, HBM_COMMANDS)
        else:
            print(json.dumps(trace_summary(args.trace_summary, args.sweep_json), indent=1))
        return

    import torch
    from paper_1405_1020_amd import binding as B, synth, serve
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B.lib()

    if args.counter_workload:
        counter_workload(args.counter_workload, torch, B, synth)
        return

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
    img, src, ms_step, mp_step, per, achieved, settle_steps = bench_plain(torch, B, synth, timer, args.steps,
                                                                           args.warmup)
    value = mp_step / (ms_step / 1e3)
    launch_ms = ms_step / len(synth.FHD_SWEEP)
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "MP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "settle_steps": settle_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "fhd_1920x1080_sweep", "width": 1920, "height": 1080,
                   "image_sha256": synth.sha256(img),
                   "runs": [list(x) for x in synth.FHD_SWEEP], "image": "40 Gaussian colour blobs + U{-8..8} noise, seed 2",
                   "launches_per_step": len(synth.FHD_SWEEP)},
    }
    # roofline of the dominant kernel: the sweep run with the longest launch
    dom = max(per, key=lambda k: per[k]["ms"])
    d = per[dom]
    r_d, L_d = d["r"], d["L"]
    d_bytes = lds_bytes_per_pixel(r_d, L_d) * img.shape[0] * img.shape[1]
    d_ach = d_bytes / (d["ms"] / 1e3) / 1e9
    res["roofline"] = {"bound": "lds", "achieved": round(d_ach, 1), "peak": round(LDS_PEAK_GBS, 1),
                       "unit": "GB/s", "frac": round(d_ach / LDS_PEAK_GBS, 4),
                       "traffic": hbm_traffic(d["kernel"], dom, d["variant"]), "kernel": d["kernel"], "run": dom,
                       "lds_bytes_per_launch": d_bytes, "avg_launch_ms": d["ms"],
                       "sweep_achieved": round(achieved, 1), "sweep_avg_launch_ms": round(launch_ms, 5)}
    # the same LDS work priced at this GPU's measured LDS rates, and the
    # counters of the committed summary (when taken on these sources)
    log("lds probe ...")
    rates = lds_probe_leg(torch, B)
    px = img.shape[0] * img.shape[1]
    for name, e in per.items():
        e["lds_model_ms_measured_rates"] = round(lds_model_ms(e["r"], e["L"], px, rates), 5)
        e["lds_frac_measured_rates"] = round(e["lds_model_ms_measured_rates"] / e["ms"], 4)
        c = counter_fields(name)
        if c:
            e["counters"] = c
    res["roofline"]["measured_lds_rates"] = rates
    res["roofline"]["frac_at_measured_rates"] = d["lds_frac_measured_rates"]
    res["roofline"]["counters"] = counter_fields(dom)
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
        log("large radii ...")
        res["large_radius_1920x1080"] = bench_large_radius(torch, B, synth, timer, oracle_mod)
        log("median ...")
        cpu = host_cpu()
        res["median_1920x1080_channel1"] = bench_median(torch, B, synth, timer, oracle_mod, cpu["threads"])
        log("register histograms ...")
        from paper_1405_1020_amd import tune as tune_mod
        res["register_histograms_1920x1080"] = bench_register_histograms(B, tune_mod)
        log("jpeg ...")
        res["jpeg_decode_process_encode"] = bench_jpeg(torch, B, synth, oracle_mod, cpu["threads"])
        log("serving ...")
        res["serving"] = bench_serving(torch, B, synth, serve, args.serve_requests, oracle_mod, cpu["threads"])
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(oracle_mod, img, synth.FHD_SWEEP, cpu)
        res["oracle_timings"] = oracle_timings(oracle_mod, synth, cpu["threads"])
        res["transfers_1920x1080"] = transfers(torch, img)
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
