"""ctypes binding of liboilpaint.so (include/oilpaint.h), same names.

Argument marshalling only: torch supplies device memory and streams, every
step of the filter runs in the library's HIP kernels.  There is no CPU
fallback: if the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "liboilpaint.so")
HEADER = os.path.join(ROOT, "include", "oilpaint.h")

OK = 0
ERR_NULL = -1
ERR_ARG = -2
ERR_OVERLAP = -3
ERR_NOT_DEVICE = -4
ERR_HIP = -5
ERR_NOMEM = -6
ERR_FULL = -7
ERR_UNSUPPORTED = -8

HIST_PACKED = 0
HIST_STREAM = 1
HIST_WIDE = 2
HIST_STREAM8 = 3
HIST_COLUMN = 4
HIST_REGS = 5
FLAG_PAPER = 1


class OilpaintError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = strerror(status) if _lib is not None else str(status)
        if status == ERR_HIP and _lib is not None:
            msg += " [" + _lib.oilpaint_last_error().decode() + "]"
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


class Variant(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("hist", ctypes.c_int32), ("lanes", ctypes.c_int32), ("per_cu", ctypes.c_int32)]

    def __init__(self, rows=0, waves=1, hist=0, lanes=64, per_cu=8):
        super().__init__(rows, waves, hist, lanes, per_cu)

    def as_tuple(self):
        return (self.rows, self.waves, self.hist, self.lanes, self.per_cu)

    def __repr__(self):
        return "Variant(rows=%d, waves=%d, hist=%d, lanes=%d, per_cu=%d)" % self.as_tuple()


class Desc(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("stride", ctypes.c_int32), ("dst_stride", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("row_begin", ctypes.c_int32), ("row_end", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_lib = None

_SIGS = {
    "oilpaint_version": ([], ctypes.c_int),
    "oilpaint_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "oilpaint_last_error": ([], ctypes.c_char_p),
    "oilpaint_validate": ([ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 5, ctypes.c_int),
    "oilpaint": ([ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 5, ctypes.c_int),
    "oilpaint_async": ([ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 5 + [ctypes.c_void_p], ctypes.c_int),
    "oilpaint_pick_variant": ([ctypes.c_int] * 4 + [ctypes.POINTER(Variant)], ctypes.c_int),
    "oilpaint_set_variant": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(Variant)], ctypes.c_int),
    "oilpaint_clear_variants": ([], ctypes.c_int),
    "oilpaint_async_variant": ([ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 5
                               + [ctypes.POINTER(Variant), ctypes.c_void_p], ctypes.c_int),
    "oilpaint_run": ([ctypes.POINTER(Desc), ctypes.c_void_p], ctypes.c_int),
    "oilpaint_median_async": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                               ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p],
                              ctypes.c_int),
    "oilpaint_median_async_kind": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p], ctypes.c_int),
    "oilpaint_median_set_kind": ([ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "oilpaint_median_pick_kind": ([ctypes.c_int], ctypes.c_int),
    "oilpaint_median": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "oilpaint_tune": ([ctypes.c_int] * 4 + [ctypes.POINTER(Variant), ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                       ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "oilpaint_batch": ([ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)],
                       ctypes.c_int),
    "oilpaint_batch_noalloc": ([ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)],
                               ctypes.c_int),
    "oilpaint_lds_probe": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_int), ctypes.c_void_p], ctypes.c_int),
    "oilpaint_jpeg_header": ([ctypes.c_char_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "oilpaint_jpeg_coefficients": ([ctypes.c_char_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "oilpaint_jpeg_decode": ([ctypes.c_char_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                              ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "oilpaint_jpeg_decode_planes": ([ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p),
                                     ctypes.POINTER(ctypes.c_int), ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)],
                                    ctypes.c_int),
    "oilpaint_jpeg_encode": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t), ctypes.c_void_p,
                              ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "oilpaint_jpeg_encode_bound": ([ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
    "oilpaint_jpeg_set_subsequence_bits": ([ctypes.c_int], ctypes.c_int),
    "oilpaint_jpeg_encode_info": ([ctypes.c_int] * 4 + [ctypes.c_void_p], ctypes.c_int),
    "oilpaint_jpeg_write": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "oilpaint_plan_create": ([ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_void_p,
                              ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "oilpaint_plan_launch": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "oilpaint_plan_info": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
                           ctypes.c_int),
    "oilpaint_plan_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "oilpaint_queue_create": ([ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "oilpaint_queue_push": ([ctypes.c_void_p, ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_uint64)],
                            ctypes.c_int),
    "oilpaint_queue_step": ([ctypes.c_void_p], ctypes.c_int),
    "oilpaint_queue_poll": ([ctypes.c_void_p, ctypes.c_uint64], ctypes.c_int),
    "oilpaint_queue_completed": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int),
                                  ctypes.c_int], ctypes.c_int),
    "oilpaint_queue_fail_next": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "oilpaint_queue_drain": ([ctypes.c_void_p], ctypes.c_int),
    "oilpaint_queue_stream": ([ctypes.c_void_p], ctypes.c_void_p),
    "oilpaint_queue_destroy": ([ctypes.c_void_p], ctypes.c_int),
}


def header_functions() -> list[str]:
    """Names of the functions declared in include/oilpaint.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(oilpaint\w*)\s*\(", text)))


def lib():
    """Load liboilpaint.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OilpaintError(ERR_UNSUPPORTED,
                                "liboilpaint.so is not built (python -m paper_1405_1020_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (argt, rest) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = argt
            fn.restype = rest
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().oilpaint_strerror(status).decode()


def version() -> int:
    return lib().oilpaint_version()


def _check(st: int, what: str):
    if st != OK:
        raise OilpaintError(st, what)
    return st


# ---------------------------------------------------------------------------
# torch marshalling
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def image_geometry(t) -> tuple[int, int, int]:
    """(width, height, stride) of a uint8 [H, W, 3] tensor whose pixels are
    packed (strides (S, 3, 1)); S is the row stride in bytes."""
    torch = _torch()
    if t.dtype != torch.uint8 or t.dim() != 3 or t.shape[2] != 3:
        raise ValueError("expected a uint8 [H, W, 3] tensor")
    h, w, _ = t.shape
    sh, sw, sc = t.stride()
    if h > 0 and w > 0 and (sc != 1 or sw != 3 or (h > 1 and sh < 3 * w)):
        raise ValueError("pixels must be packed: strides (S >= 3W, 3, 1), got %s" % (t.stride(),))
    stride = sh if h > 1 else 3 * w
    return w, h, stride


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _require_cuda(*ts):
    for t in ts:
        if not t.is_cuda:
            raise OilpaintError(ERR_NOT_DEVICE, "tensor is not on a GPU")


def validate(src_ptr: int, dst_ptr: int, width: int, height: int, stride: int, radius: int,
             levels: int) -> int:
    """oilpaint_validate on raw addresses (pure host, no GPU needed)."""
    return lib().oilpaint_validate(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), width, height,
                                   stride, radius, levels)


def oilpaint_async(src, dst, radius: int, levels: int, stream=None, variant: Variant | None = None):
    """Enqueue the filter of src into dst (uint8 [H, W, 3] CUDA tensors with
    the same geometry) on `stream` (default: torch's current stream)."""
    _require_cuda(src, dst)
    w, h, s = image_geometry(src)
    w2, h2, s2 = image_geometry(dst)
    if (w, h) != (w2, h2) or (h > 1 and s != s2):
        raise ValueError("src and dst must have the same width, height and row stride")
    L = lib()
    if w == 0 or h == 0:
        return OK  # nothing to filter (an empty tensor has no storage pointer)
    if variant is None:
        st = L.oilpaint_async(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                              w, h, s, radius, levels, _stream_ptr(stream))
    else:
        st = L.oilpaint_async_variant(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                      w, h, s, radius, levels, ctypes.byref(variant), _stream_ptr(stream))
    return _check(st, "oilpaint_async")


def oilpaint(src, radius: int, levels: int, out=None, stream=None, variant: Variant | None = None):
    """Filter a uint8 [H, W, 3] CUDA tensor; returns `out` (allocated if None)."""
    torch = _torch()
    if out is None:
        # one row stride serves both buffers: give dst the source's
        w, h, s = image_geometry(src)
        buf = torch.empty(max(h - 1, 0) * s + 3 * w, dtype=torch.uint8, device=src.device)
        out = buf.as_strided((h, w, 3), (s, 3, 1))
    oilpaint_async(src, out, radius, levels, stream=stream, variant=variant)
    return out


def _plane_geometry(t, channels: int | None) -> tuple[int, int, int, int]:
    """(width, height, row stride, channels) of a uint8 [H, W, C] (C = 1..4)
    or [H, W] tensor with packed pixels."""
    torch = _torch()
    if t.dtype != torch.uint8 or t.dim() not in (2, 3) or (t.dim() == 3 and not 1 <= t.shape[2] <= 4):
        raise ValueError("expected a uint8 [H, W] or [H, W, C<=4] tensor")
    h, w = t.shape[0], t.shape[1]
    c = t.shape[2] if t.dim() == 3 else 1
    st = t.stride()
    if h > 0 and w > 0 and (st[1] != c or (t.dim() == 3 and st[2] != 1) or (h > 1 and st[0] < c * w)):
        raise ValueError("pixels must be packed, got strides %s" % (st,))
    return w, h, (st[0] if h > 1 else c * w), c


MEDIAN_AUTO = 0
MEDIAN_ONE = 1
MEDIAN_FOUR = 2
MEDIAN_COLUMN = 3


def median_async(src, dst, radius: int, channel: int, stream=None, kind: int = MEDIAN_AUTO) -> int:
    """oilpaint_median_async (or, with a kind, oilpaint_median_async_kind):
    the windowed median of channel `channel` of src (uint8 [H, W, C] CUDA
    tensor) into dst (uint8 [H, W] or [H, W, 1]), each with its own row
    stride, on `stream`."""
    _require_cuda(src, dst)
    w, h, s, c = _plane_geometry(src, None)
    w2, h2, s2, c2 = _plane_geometry(dst, None)
    if (w, h) != (w2, h2) or c2 != 1:
        raise ValueError("dst must be a one-channel image of src's width and height")
    if w == 0 or h == 0:
        return OK
    if kind == MEDIAN_AUTO:
        st = lib().oilpaint_median_async(ctypes.c_void_p(src.data_ptr()), s, c, channel,
                                         ctypes.c_void_p(dst.data_ptr()), s2, w, h, radius, _stream_ptr(stream))
    else:
        st = lib().oilpaint_median_async_kind(ctypes.c_void_p(src.data_ptr()), s, c, channel,
                                              ctypes.c_void_p(dst.data_ptr()), s2, w, h, radius, kind,
                                              _stream_ptr(stream))
    return _check(st, "oilpaint_median_async")


def median_set_kind(radius: int, kind: int):
    _check(lib().oilpaint_median_set_kind(radius, kind), "oilpaint_median_set_kind")


def median_pick_kind(radius: int) -> int:
    st = lib().oilpaint_median_pick_kind(radius)
    if st < 0:
        raise OilpaintError(st, "oilpaint_median_pick_kind")
    return st


def median(src, radius: int, channel: int, out=None, stream=None, kind: int = MEDIAN_AUTO):
    """Windowed median of one channel; returns `out` (uint8 [H, W],
    allocated if None)."""
    torch = _torch()
    if out is None:
        out = torch.empty(src.shape[0], src.shape[1], dtype=torch.uint8, device=src.device)
    median_async(src, out, radius, channel, stream=stream, kind=kind)
    return out


def pick_variant(width: int, height: int, radius: int, levels: int) -> Variant:
    v = Variant()
    _check(lib().oilpaint_pick_variant(width, height, radius, levels, ctypes.byref(v)), "pick_variant")
    return v


def set_variant(radius: int, levels: int, v: Variant) -> int:
    return lib().oilpaint_set_variant(radius, levels, ctypes.byref(v))


def clear_variants():
    lib().oilpaint_clear_variants()


def tune_times(width: int, height: int, radius: int, levels: int, candidates, reps: int = 5,
               stream=None) -> list[float]:
    """oilpaint_tune: average ms per launch of each candidate (-1 when it
    cannot run this (radius, levels))."""
    n = len(candidates)
    arr = (Variant * n)(*candidates)
    out = (ctypes.c_float * n)()
    _check(lib().oilpaint_tune(width, height, radius, levels, arr, n, reps, _stream_ptr(stream), out),
           "oilpaint_tune")
    return [float(v) for v in out]


@dataclass
class Item:
    """One image of a batch: src/dst CUDA tensors and its parameters."""
    src: object
    dst: object
    radius: int
    levels: int
    row_begin: int = 0
    row_end: int = 0
    flags: int = 0


def make_desc(it: Item) -> Desc:
    """Descriptor of an Item; src and dst may have different row strides."""
    _require_cuda(it.src, it.dst)
    w, h, s = image_geometry(it.src)
    w2, h2, s2 = image_geometry(it.dst)
    if (w, h) != (w2, h2):
        raise ValueError("src and dst must have the same width and height")
    return Desc(it.src.data_ptr(), it.dst.data_ptr(), w, h, s, s2, it.radius, it.levels,
                it.row_begin, it.row_end, it.flags, 0)


def run(item, stream=None) -> None:
    """oilpaint_run: the plain kernel on one descriptor (own dst stride, row
    band and flags)."""
    if isinstance(item, Item):
        w, h, _ = image_geometry(item.src)
        if w == 0 or h == 0:
            return
    d = item if isinstance(item, Desc) else make_desc(item)
    _check(lib().oilpaint_run(ctypes.byref(d), _stream_ptr(stream)), "oilpaint_run")


def _desc_array(items):
    arr = (Desc * max(1, len(items)))()
    for i, it in enumerate(items):
        arr[i] = it if isinstance(it, Desc) else make_desc(it)
    return arr


def batch(items, stream=None) -> None:
    """oilpaint_batch: one persistent launch over every item."""
    arr = _desc_array(items)
    bad = ctypes.c_int(-1)
    st = lib().oilpaint_batch(arr, len(items), _stream_ptr(stream), ctypes.byref(bad))
    if st != OK:
        raise OilpaintError(st, "oilpaint_batch (item %d)" % bad.value)


def batch_noalloc(items, stream=None) -> None:
    """oilpaint_batch_noalloc: oilpaint_batch with its argument block in the
    library's static device array (no device allocation)."""
    arr = _desc_array(items)
    bad = ctypes.c_int(-1)
    st = lib().oilpaint_batch_noalloc(arr, len(items), _stream_ptr(stream), ctypes.byref(bad))
    if st != OK:
        raise OilpaintError(st, "oilpaint_batch_noalloc (item %d)" % bad.value)


class JpegInfo(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("components", ctypes.c_int32),
                ("h_samp", ctypes.c_int32 * 3), ("v_samp", ctypes.c_int32 * 3),
                ("comp_width", ctypes.c_int32 * 3), ("comp_height", ctypes.c_int32 * 3),
                ("blocks_w", ctypes.c_int32 * 3), ("blocks_h", ctypes.c_int32 * 3),
                ("first_block", ctypes.c_int32 * 3), ("blocks", ctypes.c_int64),
                ("restart_interval", ctypes.c_int32), ("scans", ctypes.c_int32)]


def jpeg_header(data: bytes) -> JpegInfo:
    """oilpaint_jpeg_header (host only)."""
    info = JpegInfo()
    _check(lib().oilpaint_jpeg_header(data, len(data), ctypes.byref(info)), "oilpaint_jpeg_header")
    return info


def jpeg_coefficients(data: bytes):
    """oilpaint_jpeg_coefficients (host only): (JpegInfo, int16 numpy array of
    every block's 64 coefficients, natural order)."""
    import numpy as np
    info = jpeg_header(data)
    out = np.zeros(int(info.blocks) * 64, np.int16)
    n = ctypes.c_size_t(0)
    _check(lib().oilpaint_jpeg_coefficients(data, len(data), out.ctypes.data, out.size, ctypes.byref(n)),
           "oilpaint_jpeg_coefficients")
    return info, out[:n.value]


def jpeg_encode_info(width: int, height: int, quality: int, subsampling: int) -> JpegInfo:
    info = JpegInfo()
    _check(lib().oilpaint_jpeg_encode_info(width, height, quality, subsampling, ctypes.byref(info)),
           "oilpaint_jpeg_encode_info")
    return info


def jpeg_write(coef, width: int, height: int, quality: int, subsampling: int) -> bytes:
    """oilpaint_jpeg_write (host only): entropy-code int16 coefficients."""
    import numpy as np
    coef = np.ascontiguousarray(coef, dtype=np.int16)
    n = ctypes.c_size_t(0)
    st = lib().oilpaint_jpeg_write(coef.ctypes.data, width, height, quality, subsampling, None, 0, ctypes.byref(n))
    if st not in (OK, ERR_NOMEM):
        raise OilpaintError(st, "oilpaint_jpeg_write")
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().oilpaint_jpeg_write(coef.ctypes.data, width, height, quality, subsampling, buf, n.value,
                                     ctypes.byref(n)), "oilpaint_jpeg_write")
    return buf.raw[:n.value]


def jpeg_set_subsequence_bits(bits: int) -> None:
    """oilpaint_jpeg_set_subsequence_bits (process-wide; 0: chosen per scan)."""
    _check(lib().oilpaint_jpeg_set_subsequence_bits(int(bits)), "oilpaint_jpeg_set_subsequence_bits")


def jpeg_decode(data: bytes, out=None, stream=None, times: dict | None = None):
    """oilpaint_jpeg_decode: a uint8 [H, W, 3] CUDA tensor (or `out`)."""
    torch = _torch()
    info = jpeg_header(data)
    if out is None:
        out = torch.empty((info.height, info.width, 3), dtype=torch.uint8, device="cuda")
    _require_cuda(out)
    w, h, s = image_geometry(out)
    if (w, h) != (info.width, info.height):
        raise ValueError("out must be [%d, %d, 3]" % (info.height, info.width))
    ms = ctypes.c_double(0)
    _check(lib().oilpaint_jpeg_decode(data, len(data), out.data_ptr(), s, _stream_ptr(stream), ctypes.byref(ms)),
           "oilpaint_jpeg_decode")
    if times is not None:
        times["host_ms"] = ms.value
    return out


def jpeg_decode_planes(data: bytes, stream=None):
    """oilpaint_jpeg_decode_planes: one uint8 [comp_height, comp_width] CUDA
    tensor per component."""
    torch = _torch()
    info = jpeg_header(data)
    planes = [torch.empty((info.comp_height[c], info.comp_width[c]), dtype=torch.uint8, device="cuda")
              for c in range(info.components)]
    ptrs = (ctypes.c_void_p * 3)(*([p.data_ptr() for p in planes] + [None] * (3 - len(planes))))
    strides = (ctypes.c_int * 3)(*([p.shape[1] for p in planes] + [0] * (3 - len(planes))))
    _check(lib().oilpaint_jpeg_decode_planes(data, len(data), ptrs, strides, _stream_ptr(stream), None),
           "oilpaint_jpeg_decode_planes")
    return planes


_jpeg_out = None


def jpeg_encode(src, quality: int = 90, subsampling: int = 2, stream=None, times: dict | None = None) -> bytes:
    """oilpaint_jpeg_encode of a uint8 [H, W, 3] CUDA tensor: the file bytes."""
    import numpy as np
    _require_cuda(src)
    w, h, s = image_geometry(src)
    global _jpeg_out
    # a reused output block of the raw image's size (a JPEG file rarely
    # exceeds it); a larger file is encoded again into a block of its size
    need = 3 * w * h + 65536
    if _jpeg_out is None or _jpeg_out.size < need:
        _jpeg_out = np.empty(need, np.uint8)
    n = ctypes.c_size_t(0)
    ms = ctypes.c_double(0)
    for _ in range(2):
        st = lib().oilpaint_jpeg_encode(src.data_ptr(), w, h, s, quality, subsampling, _jpeg_out.ctypes.data,
                                        _jpeg_out.size, ctypes.byref(n), _stream_ptr(stream), ctypes.byref(ms))
        if st != ERR_NOMEM or n.value <= _jpeg_out.size:
            break
        _jpeg_out = np.empty(n.value, np.uint8)
    _check(st, "oilpaint_jpeg_encode")
    if times is not None:
        times["host_ms"] = ms.value
    return _jpeg_out[:n.value].tobytes()


PROBE_READ64 = 0
PROBE_ADD64 = 1
PROBE_READ32 = 2


def lds_probe(kind: int, iters: int, per_cu: int = 4, stream=None):
    """oilpaint_lds_probe: returns (workgroups, clocks) with clocks a device
    tensor [workgroups, 4] (shader clock start/end, 100 MHz real time
    start/end per workgroup), after the kernel has run."""
    torch = _torch()
    n = 4096
    clocks = torch.zeros((n, 4), dtype=torch.int64, device="cuda")
    wg = ctypes.c_int(0)
    _check(lib().oilpaint_lds_probe(kind, iters, per_cu, clocks.data_ptr(), n, ctypes.byref(wg),
                                    _stream_ptr(stream)), "oilpaint_lds_probe")
    return wg.value, clocks[:wg.value]


class Plan:
    """oilpaint_plan: the batch laid out once and captured in a hipGraph."""

    def __init__(self, items, stream=None):
        self._items = list(items)  # keep the tensors alive
        arr = _desc_array(self._items)
        h = ctypes.c_void_p()
        bad = ctypes.c_int(-1)
        st = lib().oilpaint_plan_create(arr, len(self._items), _stream_ptr(stream), ctypes.byref(h),
                                        ctypes.byref(bad))
        if st != OK:
            raise OilpaintError(st, "oilpaint_plan_create (item %d)" % bad.value)
        self._h = h

    def launch(self, stream=None):
        _check(lib().oilpaint_plan_launch(self._h, _stream_ptr(stream)), "oilpaint_plan_launch")

    def info(self) -> tuple[int, int]:
        t, g = ctypes.c_int(), ctypes.c_int()
        _check(lib().oilpaint_plan_info(self._h, ctypes.byref(t), ctypes.byref(g)), "oilpaint_plan_info")
        return t.value, g.value

    def close(self):
        if getattr(self, "_h", None):
            lib().oilpaint_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Queue:
    """oilpaint_queue: continuous batching of filter requests."""

    def __init__(self, capacity: int = 4096, step_pixels: int = 0):
        h = ctypes.c_void_p()
        _check(lib().oilpaint_queue_create(capacity, step_pixels, ctypes.byref(h)), "oilpaint_queue_create")
        self._h = h

    def push(self, item) -> int:
        d = item if isinstance(item, Desc) else make_desc(item)
        t = ctypes.c_uint64()
        st = lib().oilpaint_queue_push(self._h, ctypes.byref(d), ctypes.byref(t))
        if st != OK:
            raise OilpaintError(st, "oilpaint_queue_push")
        return t.value

    def try_push(self, item) -> tuple[int, int]:
        """(status, ticket) without raising on ERR_FULL."""
        d = item if isinstance(item, Desc) else make_desc(item)
        t = ctypes.c_uint64()
        st = lib().oilpaint_queue_push(self._h, ctypes.byref(d), ctypes.byref(t))
        return st, t.value

    def step(self) -> int:
        st = lib().oilpaint_queue_step(self._h)
        if st < 0:
            raise OilpaintError(st, "oilpaint_queue_step")
        return st

    def poll(self, ticket: int) -> bool:
        st = lib().oilpaint_queue_poll(self._h, ticket)
        if st < 0:
            raise OilpaintError(st, "oilpaint_queue_poll")
        return st == 1

    def completed(self, max_tickets: int = 4096) -> list[int]:
        """Tickets completed since last reported (each reported once),
        failed requests included (see completed_status)."""
        return [t for t, _ in self.completed_status(max_tickets)]

    def completed_status(self, max_tickets: int = 4096) -> list[tuple[int, int]]:
        """(ticket, status) of the requests completed since last reported:
        status OK, or the error code of a request whose launch failed."""
        if getattr(self, "_buf", None) is None or len(self._buf) < max_tickets:
            self._buf = (ctypes.c_uint64 * max_tickets)()
            self._sbuf = (ctypes.c_int * max_tickets)()
        n = lib().oilpaint_queue_completed(self._h, self._buf, self._sbuf, max_tickets)
        if n < 0:
            raise OilpaintError(n, "oilpaint_queue_completed")
        return list(zip(self._buf[:n], self._sbuf[:n]))

    def fail_next(self, n: int):
        """Test hook: the next n launches fail before anything is enqueued."""
        _check(lib().oilpaint_queue_fail_next(self._h, n), "oilpaint_queue_fail_next")

    def drain(self):
        _check(lib().oilpaint_queue_drain(self._h), "oilpaint_queue_drain")

    def stream_ptr(self) -> int:
        return lib().oilpaint_queue_stream(self._h) or 0

    def close(self):
        if getattr(self, "_h", None):
            lib().oilpaint_queue_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
