"""CPU oracle for the oil-paint filter.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library
(paper_1405_1020_amd) never imports it and shares no code with it.

`oilpaint_ref` wraps the plain C implementation in oilpaint_ref.c through
ctypes on numpy arrays; `brute` is an independent Python brute force for tiny
images.  `median_ref` wraps median_ref.c, the windowed median filter (the
second filter of the same class); `brute.brute_median` is its brute force.
`jpeg_ref` (imported as `oracle.jpeg_ref`) is the plain baseline JPEG codec of
ITU-T T.81 and JFIF for the decode and encode steps either side of the filter.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .brute import brute, brute_median, level_of, median_at  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oilpaint_ref.c")
_SRCS = [_SRC, os.path.join(_HERE, "median_ref.c")]
_LIB = os.path.join(_HERE, "liboilpaint_ref.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oilpaint_ref.c and median_ref.c with gcc -O2 into
    liboilpaint_ref.so."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-pthread"] + _SRCS + ["-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        for name in ("oilpaint_ref", "oilpaint_ref_paper"):
            fn = getattr(lib, name)
            fn.argtypes = [u8p, u8p] + [ctypes.c_int] * 6
            fn.restype = ctypes.c_int
        lib.median_ref.argtypes = [u8p, u8p] + [ctypes.c_int] * 8
        lib.median_ref.restype = ctypes.c_int
        for name in ("oilpaint_ref_level", "oilpaint_ref_level_paper"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.c_uint] * 4
            fn.restype = ctypes.c_uint
        _lib = lib
    return _lib


def _u8p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _as_rows(img: np.ndarray, stride: int | None):
    """Return (flat uint8 buffer, width, height, stride) for an image given as
    [H, W, 3] (dense rows) or as a flat/2-D byte buffer with explicit stride."""
    if img.ndim == 3:
        h, w, c = img.shape
        assert c == 3 and img.dtype == np.uint8
        buf = np.ascontiguousarray(img).reshape(-1)
        return buf, w, h, 3 * w
    raise ValueError("pass an [H, W, 3] uint8 array, or use oilpaint_ref_buffer")


def oilpaint_ref(img: np.ndarray, radius: int, levels: int, nthreads: int = 1,
                 paper_mode: bool = False, out: np.ndarray | None = None) -> np.ndarray:
    """Filter an [H, W, 3] uint8 image on the CPU.  Returns a new array (or
    fills `out`, which in paper mode keeps its bytes outside the interior)."""
    buf, w, h, stride = _as_rows(img, None)
    if out is None:
        out = np.zeros_like(np.ascontiguousarray(img))
    assert out.shape == img.shape and out.dtype == np.uint8 and out.flags.c_contiguous
    oilpaint_ref_buffer(buf, out.reshape(-1), w, h, stride, radius, levels, nthreads, paper_mode)
    return out


def oilpaint_ref_buffer(src: np.ndarray, dst: np.ndarray, width: int, height: int, stride: int,
                        radius: int, levels: int, nthreads: int = 1,
                        paper_mode: bool = False) -> int:
    """Filter flat byte buffers with an explicit row stride (bytes)."""
    lib = _load()
    assert src.dtype == np.uint8 and dst.dtype == np.uint8
    assert src.flags.c_contiguous and dst.flags.c_contiguous
    if width > 0 and height > 0:
        need = (height - 1) * stride + 3 * width
        assert src.size >= need and dst.size >= need
    fn = lib.oilpaint_ref_paper if paper_mode else lib.oilpaint_ref
    rc = fn(_u8p(src), _u8p(dst), width, height, stride, radius, levels, nthreads)
    if rc != 0:
        raise ValueError("oilpaint_ref rejected the arguments (status %d)" % rc)
    return rc


def ref_level(r: int, g: int, b: int, levels: int, paper_mode: bool = False) -> int:
    lib = _load()
    fn = lib.oilpaint_ref_level_paper if paper_mode else lib.oilpaint_ref_level
    return int(fn(r, g, b, levels))


def median_ref(img: np.ndarray, radius: int, channel: int, nthreads: int = 1) -> np.ndarray:
    """Windowed lower median of one channel of an [H, W, C] uint8 image
    (window clipped to the image).  Returns an [H, W] uint8 array."""
    a = np.ascontiguousarray(img)
    assert a.dtype == np.uint8 and a.ndim == 3
    h, w, c = a.shape
    out = np.zeros((h, w), np.uint8)
    if w == 0 or h == 0:
        return out
    st = _load().median_ref(_u8p(a.reshape(-1)), _u8p(out.reshape(-1)), w, h, c * w, w, c, channel, radius,
                            nthreads)
    if st != 0:
        raise ValueError("median_ref: status %d" % st)
    return out
