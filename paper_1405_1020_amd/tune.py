"""Autotuner: the launch shape per (radius, levels).

For each (radius, levels) the candidates -- streamed rows with several
workgroup densities (and, for radius 8..15 with at most 32 levels, the
same with 8-byte on-chip row entries), histograms in registers for radius
<= 7 and at most 16 levels, tile-staged workgroups of 2 or 4 wavefronts
with several densities, column histograms for radii from 3 (at most 64
levels; one, two or four wavefronts per strip) and above 15, and the wide
layout above 15 -- are
timed by the library itself (oilpaint_tune, HIP
events around repeated launches on a representative image) and the fastest
is installed with oilpaint_set_variant, so that oilpaint_async, batches and
the request queue use it.  Shapes whose rows are derived from a workgroup
density (rows = 0, per_cu) adapt to the image size they are used on.

Results are cached as JSON, keyed by the GPU architecture and a hash of the
kernel sources, in $OILPAINT_TUNE_CACHE or ~/.cache/oilpaint/tune.json.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import binding as B

HERE = os.path.dirname(os.path.abspath(__file__))


def code_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cpp", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def cache_path() -> str:
    return os.environ.get("OILPAINT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "oilpaint", "tune.json"))


def candidates(radius: int, levels: int) -> list[B.Variant]:
    out = []
    if radius <= 15 and levels <= 64:
        for per_cu in (2, 4, 8, 16, 32):
            out.append(B.Variant(0, 1, B.HIST_STREAM, 64, per_cu))
        # four wavefronts per strip
        for per_cu in (2, 3, 4, 5, 6, 8, 16):
            out.append(B.Variant(0, 4, B.HIST_STREAM, 64, per_cu))
    if 8 <= radius <= 15 and levels <= 32:
        for per_cu in (2, 4, 8, 16):
            out.append(B.Variant(0, 1, B.HIST_STREAM8, 64, per_cu))
        # four wavefronts per strip
        for per_cu in (1, 2, 3, 4, 5, 8):
            out.append(B.Variant(0, 4, B.HIST_STREAM8, 64, per_cu))
    if radius <= 7 and levels <= 16:
        # each lane's histogram in its registers (window updates as VALU
        # compare-selects over every bin instead of LDS atomics)
        for per_cu in (2, 4, 8, 16, 32):
            out.append(B.Variant(0, 1, B.HIST_REGS, 64, per_cu))
    if radius <= 15 and levels <= 255:
        for waves in (2, 4):
            for per_cu in (1, 2, 4, 8):
                out.append(B.Variant(0, waves, B.HIST_PACKED, 64, per_cu))
    if radius > 15:
        for per_cu in (1, 2, 4, 8, 16):
            out.append(B.Variant(0, 1, B.HIST_COLUMN, 64, per_cu))
        if radius <= 31 and levels <= 64:
            # the count-word form with wider fields, two or four wavefronts per strip
            for waves, per_cu in ((2, 4), (2, 8), (4, 2), (4, 4), (4, 5), (4, 6), (4, 8)):
                out.append(B.Variant(0, waves, B.HIST_COLUMN, 64, per_cu))
    elif radius >= 3 and levels <= 64:
        # column histograms cost O(levels) per row (and 2r+1 reads for the
        # winning level): they can win at wide windows and few levels; one,
        # two or four wavefronts per strip
        for waves, per_cu in ((1, 8), (2, 8), (4, 4), (4, 5), (4, 6), (4, 7), (4, 8)):
            out.append(B.Variant(0, waves, B.HIST_COLUMN, 64, per_cu))
    if not out or radius > 15:
        for per_cu in (1, 2, 4):
            out.append(B.Variant(0, 2, B.HIST_WIDE, 64, per_cu))
    return out


def _key(radius: int, levels: int) -> str:
    return "%d,%d" % (radius, levels)


def _load_file(section: str = "entries") -> dict:
    try:
        d = json.load(open(cache_path()))
    except (OSError, ValueError):
        return {}
    if d.get("arch") != arch() or d.get("code") != code_hash():
        return {}
    return d.get(section, {})


def _save_file(entries: dict, section: str = "entries"):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        d = {"arch": arch(), "code": code_hash(), "entries": _load_file("entries"), "median": _load_file("median")}
        d[section] = entries
        tmp = p + ".tmp%d" % os.getpid()
        json.dump(d, open(tmp, "w"), indent=1)
        os.replace(tmp, p)
    except OSError:
        pass


def install(entries: dict) -> int:
    n = 0
    for k, e in entries.items():
        r, L = (int(v) for v in k.split(","))
        if B.set_variant(r, L, B.Variant(*e["variant"])) == B.OK:
            n += 1
    return n


def load() -> int:
    """Install every cached result for this GPU and kernel source."""
    return install(_load_file())


# A later candidate replaces an earlier one only when it is faster by more
# than this fraction, so that near-ties resolve the same way from run to run.
TIE = 0.02


def pick(timed):
    """The first (candidate, ms) within TIE of the fastest."""
    fastest = min(t for _, t in timed)
    return next((c, t) for c, t in timed if t <= fastest * (1.0 + TIE))


def tune(radius: int, levels: int, width: int = 1920, height: int = 1080, reps: int = 5) -> dict:
    """Time the candidates for (radius, levels) on a width x height image and
    return {"variant": [...], "ms": best, "all": [(variant, ms), ...]}; near
    ties go to the earlier candidate (pick)."""
    cands = candidates(radius, levels)
    times = B.tune_times(width, height, radius, levels, cands, reps=reps)
    ok = [(c, t) for c, t in zip(cands, times) if t > 0]
    if not ok:
        raise B.OilpaintError(B.ERR_UNSUPPORTED, "no candidate runs (r=%d, L=%d)" % (radius, levels))
    best, ms = pick(ok)
    return {"variant": list(best.as_tuple()), "ms": ms, "size": [width, height],
            "all": [(list(c.as_tuple()), t) for c, t in zip(cands, times)]}


def ensure(pairs, width: int = 1920, height: int = 1080, reps: int = 5, retune: bool = False) -> dict:
    """Make sure every (radius, levels) in `pairs` has a tuned shape
    installed: taken from the cache, or tuned now and added to it."""
    entries = {} if retune else _load_file()
    changed = False
    for r, L in pairs:
        k = _key(r, L)
        if k not in entries:
            entries[k] = tune(r, L, width, height, reps)
            changed = True
    if changed:
        _save_file(entries)
    install({k: entries[k] for k in (_key(r, L) for r, L in pairs)})
    return {k: entries[k] for k in (_key(r, L) for r, L in pairs)}


# ---------------------------------------------------------------------------
# The windowed median: which kernel form per radius (one or four wavefronts
# per strip with per-lane histograms up to radius 15, column histograms up to
# 127), timed on a photo-like image with HIP events.
# ---------------------------------------------------------------------------
def median_candidates(radius: int) -> list[int]:
    out = []
    if radius <= 15:
        out += [B.MEDIAN_ONE, B.MEDIAN_FOUR]
    if radius <= 127:
        out.append(B.MEDIAN_COLUMN)
    return out


def tune_median(radius: int, width: int = 1920, height: int = 1080, reps: int = 5) -> dict:
    """Time every form for `radius` on channel 1 of a width x height blob
    image and return {"kind": best, "ms": ..., "all": [(kind, ms), ...]}."""
    import torch
    from . import synth
    src = synth.make_image_device(width, height, seed=7)
    dst = torch.empty((height, width), dtype=torch.uint8, device=src.device)
    timed = []
    for kind in median_candidates(radius):
        B.median_async(src, dst, radius, 1, kind=kind)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            B.median_async(src, dst, radius, 1, kind=kind)
        e1.record()
        torch.cuda.synchronize()
        timed.append((kind, e0.elapsed_time(e1) / reps))
    best, ms = pick(timed)
    return {"kind": best, "ms": ms, "size": [width, height], "all": timed}


def ensure_median(radii, width: int = 1920, height: int = 1080, reps: int = 5, retune: bool = False) -> dict:
    """Make sure every radius has its median form installed: from the cache,
    or tuned now and added to it."""
    entries = {} if retune else _load_file("median")
    changed = False
    for r in radii:
        k = str(r)
        if k not in entries:
            entries[k] = tune_median(r, width, height, reps)
            changed = True
    if changed:
        _save_file(entries, "median")
    for r in radii:
        B.median_set_kind(r, entries[str(r)]["kind"])
    return {str(r): entries[str(r)] for r in radii}
