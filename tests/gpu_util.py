"""Helpers shared by the GPU tests: move images to the device with padded
row strides (garbage in the padding), run the filter through the C-ABI, and
compare with the CPU oracle."""
from __future__ import annotations

import os

import numpy as np

import oracle

ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def to_device(img: np.ndarray, pad: int = 0, fill: int | None = None, seed: int = 0):
    """Copy an [H, W, 3] uint8 image into a device buffer with row stride
    3W + pad; the padding bytes hold seeded garbage (or `fill`).  Returns
    (view [H, W, 3] with strides (S, 3, 1), whole backing buffer)."""
    torch = torch_mod()
    h, w, _ = img.shape
    s = 3 * w + pad
    n = max(h - 1, 0) * s + 3 * w
    rng = np.random.default_rng(seed)
    host = rng.integers(0, 256, size=max(n, 1), dtype=np.uint8) if fill is None else np.full(max(n, 1), fill, np.uint8)
    for y in range(h):
        host[y * s:y * s + 3 * w] = img[y].reshape(-1)
    buf = torch.from_numpy(host).cuda()
    view = buf.as_strided((h, w, 3), (max(s, 1), 3, 1))
    return view, buf


def empty_like_device(img: np.ndarray, pad: int = 0, seed: int = 1):
    """A destination buffer of the same geometry, pre-filled with garbage."""
    h, w, _ = img.shape
    rng = np.random.default_rng(seed)
    junk = rng.integers(0, 256, size=img.shape, dtype=np.uint8)
    return to_device(junk, pad=pad, seed=seed + 7)


def from_device(view) -> np.ndarray:
    return view.cpu().numpy().copy() if view.numel() else np.zeros(tuple(view.shape), np.uint8)


def padding_bytes(buf, h: int, w: int, s: int) -> np.ndarray:
    host = buf.cpu().numpy()
    parts = [host[y * s + 3 * w:(y + 1) * s] for y in range(h - 1)]
    return np.concatenate(parts) if parts else np.zeros(0, np.uint8)


def ref(img: np.ndarray, r: int, L: int, paper: bool = False, out: np.ndarray | None = None):
    return oracle.oilpaint_ref(img, r, L, nthreads=ORACLE_THREADS, paper_mode=paper, out=out)


def ref_pixel(img: np.ndarray, x: int, y: int, r: int, L: int) -> np.ndarray:
    """Oracle value of one output pixel: the filter restricted to the crop
    that is exactly the pixel's clipped window (the pixel's window inside the
    crop is the same set of pixels)."""
    h, w, _ = img.shape
    y0, y1 = max(0, y - r), min(h, y + r + 1)
    x0, x1 = max(0, x - r), min(w, x + r + 1)
    crop = np.ascontiguousarray(img[y0:y1, x0:x1])
    out = oracle.oilpaint_ref(crop, r, L, nthreads=1)
    return out[y - y0, x - x0]


def first_mismatch(a: np.ndarray, b: np.ndarray):
    d = np.argwhere((a != b).any(axis=-1))
    if len(d) == 0:
        return None
    y, x = d[0]
    return (int(y), int(x), tuple(a[y, x]), tuple(b[y, x]), len(d))
