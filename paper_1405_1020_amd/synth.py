"""Seeded synthetic inputs for the oil-paint filter.

This module holds no part of the filter's arithmetic: it only draws images and
workload descriptions.  The GPU path, the tests and the CPU oracle all consume
the same bytes from here, so parity never depends on how the images look.

The paper measures on undisclosed JPEG photographs (Section 4, experimental
results).  They are not available, so photo-like stand-ins are drawn here:
a sum of Gaussian colour blobs plus small uniform integer noise, clamped to
8 bits, optionally with salt-and-pepper pixels.

    img = clamp(round(sum_k a_k * exp(-|p - c_k|^2 / (2 s_k^2))) + n, 0, 255)

with, per blob k, a centre c_k uniform over the image, s_k ~ U[s_min, s_max]
and one amplitude per channel a_k ~ U[0, 255]; n ~ U{-noise..noise} i.i.d.
per channel.  Each blob is evaluated separably (outer product of two 1-D
Gaussians) inside its +-4 s_k box, which is part of this generator's
definition.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np


def make_image(width: int, height: int, seed: int, n_blobs: int = 40,
               sigma: tuple[float, float] = (30.0, 200.0), noise: int = 8,
               salt_pepper: float = 0.0) -> np.ndarray:
    """Return an [height, width, 3] uint8 photo-like image."""
    rng = np.random.default_rng(seed)
    acc = np.zeros((height, width, 3), dtype=np.float32)
    for _ in range(n_blobs):
        cx = rng.uniform(0, width)
        cy = rng.uniform(0, height)
        s = rng.uniform(sigma[0], sigma[1])
        amp = rng.uniform(0, 255, size=3).astype(np.float32)
        x0 = max(0, int(math.floor(cx - 4 * s)))
        x1 = min(width, int(math.ceil(cx + 4 * s)) + 1)
        y0 = max(0, int(math.floor(cy - 4 * s)))
        y1 = min(height, int(math.ceil(cy + 4 * s)) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        gx = np.exp(-((np.arange(x0, x1, dtype=np.float32) - cx) ** 2) / (2 * s * s))
        gy = np.exp(-((np.arange(y0, y1, dtype=np.float32) - cy) ** 2) / (2 * s * s))
        block = gy[:, None, None] * gx[None, :, None] * amp[None, None, :]
        acc[y0:y1, x0:x1, :] += block
    img = np.rint(acc).astype(np.int16)
    if noise > 0:
        img += rng.integers(-noise, noise + 1, size=img.shape, dtype=np.int16)
    np.clip(img, 0, 255, out=img)
    out = img.astype(np.uint8)
    if salt_pepper > 0:
        npx = width * height
        m = int(round(salt_pepper * npx))
        idx = rng.choice(npx, size=m, replace=False)
        flat = out.reshape(-1, 3)
        half = m // 2
        flat[idx[:half]] = 0
        flat[idx[half:]] = 255
    return out


def make_image_device(width: int, height: int, seed: int, n_blobs: int = 40,
                      sigma: tuple[float, float] = (30.0, 200.0), noise: int = 8,
                      salt_pepper: float = 0.0, device: str = "cuda"):
    """The same recipe as make_image, drawn and rendered on the GPU with
    torch (for the large batch and serving workloads).  Blob parameters come
    from numpy's generator with `seed`; the noise and the salt-and-pepper
    positions from a torch generator seeded with `seed` on `device`.  The
    bytes are deterministic for a given device and software stack but are not
    the bytes make_image returns.  Returns a uint8 [H, W, 3] CUDA tensor."""
    import torch
    rng = np.random.default_rng(seed)
    acc = torch.zeros((height, width, 3), dtype=torch.float32, device=device)
    for _ in range(n_blobs):
        cx = rng.uniform(0, width)
        cy = rng.uniform(0, height)
        s = rng.uniform(sigma[0], sigma[1])
        amp = torch.tensor(rng.uniform(0, 255, size=3), dtype=torch.float32, device=device)
        x0 = max(0, int(math.floor(cx - 4 * s)))
        x1 = min(width, int(math.ceil(cx + 4 * s)) + 1)
        y0 = max(0, int(math.floor(cy - 4 * s)))
        y1 = min(height, int(math.ceil(cy + 4 * s)) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        gx = torch.exp(-((torch.arange(x0, x1, device=device, dtype=torch.float32) - cx) ** 2) / (2 * s * s))
        gy = torch.exp(-((torch.arange(y0, y1, device=device, dtype=torch.float32) - cy) ** 2) / (2 * s * s))
        acc[y0:y1, x0:x1, :] += gy[:, None, None] * gx[None, :, None] * amp[None, None, :]
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    img = torch.round(acc).to(torch.int16)
    del acc
    if noise > 0:
        img += torch.randint(-noise, noise + 1, img.shape, generator=g, device=device, dtype=torch.int16)
    out = img.clamp_(0, 255).to(torch.uint8)
    del img
    if salt_pepper > 0:
        npx = width * height
        m = int(round(salt_pepper * npx))
        idx = torch.randperm(npx, generator=g, device=device)[:m]
        flat = out.view(-1, 3)
        half = m // 2
        flat[idx[:half]] = 0
        flat[idx[half:]] = 255
    return out


def make_random(width: int, height: int, seed: int) -> np.ndarray:
    """Uniform random bytes: the worst case for level agreement."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=(height, width, 3), dtype=np.uint8)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---------------------------------------------------------------------------
# Workloads.  Sizes, radii and level counts follow the benchmark configurations
# of this project; the paper's own images are 640x480 .. 2560x1600 photographs
# filtered at r in {2, 4, 6, 8} with an unstated L.
# ---------------------------------------------------------------------------

SMALL_BLOBS = dict(n_blobs=8, sigma=(20.0, 60.0))
LARGE_BLOBS = dict(n_blobs=40, sigma=(30.0, 200.0))


def small_case() -> tuple[np.ndarray, int, int]:
    """256x256, 8 blobs (sigma 20..60), seed 1; r = 2, L = 20."""
    return make_image(256, 256, seed=1, **SMALL_BLOBS), 2, 20


def fhd_image() -> np.ndarray:
    """1920x1080, 40 blobs (sigma 30..200), seed 2."""
    return make_image(1920, 1080, seed=2, **LARGE_BLOBS)


# (r, L) runs on the 1920x1080 image: r sweep at L = 20, then L sweep at r = 5.
FHD_SWEEP = [(1, 20), (2, 20), (5, 20), (10, 20), (15, 20), (5, 8), (5, 64)]


def camera_image() -> np.ndarray:
    """4000x3000, 40 blobs (sigma 30..200), 2 % salt-and-pepper, seed 3."""
    return make_image(4000, 3000, seed=3, salt_pepper=0.02, **LARGE_BLOBS)


CAMERA_RL = (10, 32)


@dataclass
class BatchItem:
    width: int
    height: int
    radius: int
    levels: int
    seed: int


def batch_items(n: int = 64, seed: int = 4) -> list[BatchItem]:
    """n images, W ~ U{320..4096}, H ~ U{240..3072} independently,
    r ~ U{2,3,5,8}, L ~ U{16,20,32}."""
    rng = np.random.default_rng(seed)
    items = []
    for i in range(n):
        w = int(rng.integers(320, 4097))
        h = int(rng.integers(240, 3073))
        r = int(rng.choice([2, 3, 5, 8]))
        lv = int(rng.choice([16, 20, 32]))
        items.append(BatchItem(w, h, r, lv, seed * 1000 + i))
    return items


def batch_image(item: BatchItem, device: str | None = "cuda"):
    """The item's image: images below 0.5 MP use the small-image blob
    parameters, the rest the large-image ones.  Rendered on `device` (a CUDA
    tensor) or, with device=None, by make_image (a numpy array)."""
    blobs = SMALL_BLOBS if item.width * item.height < 500_000 else LARGE_BLOBS
    if device is None:
        return make_image(item.width, item.height, seed=item.seed, **blobs)
    return make_image_device(item.width, item.height, seed=item.seed, device=device, **blobs)


@dataclass
class Request:
    rid: int
    arrival_s: float
    width: int
    height: int
    radius: int
    levels: int
    canvas: int
    x0: int
    y0: int


@dataclass
class ServeWorkload:
    requests: list[Request]
    canvases: list = field(default_factory=list)   # uint8 [H, W, 3] CUDA tensors

    def image(self, req: Request):
        """The request's image: a strided view into its canvas (row stride =
        the canvas's)."""
        c = self.canvases[req.canvas]
        return c[req.y0:req.y0 + req.height, req.x0:req.x0 + req.width, :]


def serve_workload(n: int = 2000, rate: float = 200.0, seed: int = 5,
                   mp_range: tuple[float, float] = (0.1, 24.0),
                   n_canvas: int = 8, canvas_wh: tuple[int, int] = (5700, 4300),
                   radii: tuple[int, int] = (1, 15),
                   levels: tuple[int, ...] = (8, 16, 20, 32, 64),
                   with_canvases: bool = True) -> ServeWorkload:
    """Open-loop Poisson arrivals at `rate` req/s; megapixels log-uniform in
    mp_range with W = round(sqrt(MP * 1e6 * 4 / 3)), H = round(MP * 1e6 / W);
    r ~ U{radii}, L ~ U{levels}; every image is a seeded crop of one of
    n_canvas pre-drawn canvases."""
    rng = np.random.default_rng(seed)
    cw, ch = canvas_wh
    t = 0.0
    reqs = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        mp = math.exp(rng.uniform(math.log(mp_range[0]), math.log(mp_range[1])))
        w = int(round(math.sqrt(mp * 1e6 * 4.0 / 3.0)))
        h = int(round(mp * 1e6 / w))
        w = max(1, min(w, cw))
        h = max(1, min(h, ch))
        r = int(rng.integers(radii[0], radii[1] + 1))
        lv = int(rng.choice(list(levels)))
        c = int(rng.integers(0, n_canvas))
        x0 = int(rng.integers(0, cw - w + 1))
        y0 = int(rng.integers(0, ch - h + 1))
        reqs.append(Request(i, t, w, h, r, lv, c, x0, y0))
    wl = ServeWorkload(reqs)
    if with_canvases:
        wl.canvases = [make_image_device(cw, ch, seed=seed * 100 + k, **LARGE_BLOBS) for k in range(n_canvas)]
    return wl
