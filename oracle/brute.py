"""Second, independent brute force of the oil-paint filter, for tiny images.

TEST INFRASTRUCTURE ONLY: used by the test suite to cross-check the C oracle
(oilpaint_ref.c).  It is written in a different style on purpose (a dict of
per-level pixel lists, min() with a key for the selection) so that the two do
not share a mistake.

Definition followed (Section 4 of the paper, the histogram-based algorithm and
its serial listing), with the clipped-window reading:
  level(p)  = ((R+G+B) // 3) * L // 256
  window    = the in-image pixels of the (2r+1)x(2r+1) square around (x, y)
  chosen    = the level holding the most window pixels, lowest level on ties
  output    = per-channel floor(mean) of the chosen level's pixels
"""
from __future__ import annotations

from collections import defaultdict


def level_of(rgb, levels: int) -> int:
    r, g, b = (int(v) for v in rgb)
    mean = (r + g + b) // 3
    return (mean * levels) // 256


def brute(pixels, radius: int, levels: int):
    """pixels: list of rows, each a list of (R, G, B) tuples.  Returns the
    filtered image in the same nested-list form."""
    height = len(pixels)
    width = len(pixels[0]) if height else 0
    out = []
    for y in range(height):
        row_out = []
        for x in range(width):
            groups = defaultdict(list)
            for yy in range(max(0, y - radius), min(height, y + radius + 1)):
                for xx in range(max(0, x - radius), min(width, x + radius + 1)):
                    px = pixels[yy][xx]
                    groups[level_of(px, levels)].append(px)
            # most pixels first, then the lowest level
            chosen = min(groups, key=lambda k: (-len(groups[k]), k))
            members = groups[chosen]
            n = len(members)
            row_out.append(tuple(sum(int(p[c]) for p in members) // n for c in range(3)))
        out.append(row_out)
    return out


def brute_median(img, radius: int, channel: int):
    """Windowed lower median by sorting each clipped window (tiny images):
    element floor((n - 1) / 2) of the sorted window values of one channel."""
    h, w = len(img), len(img[0])
    out = [[0] * w for _ in range(h)]
    for y in range(h):
        for x in range(w):
            vals = sorted(int(img[yy][xx][channel])
                          for yy in range(max(0, y - radius), min(h, y + radius + 1))
                          for xx in range(max(0, x - radius), min(w, x + radius + 1)))
            out[y][x] = vals[(len(vals) - 1) // 2]
    return out


def median_at(img, x: int, y: int, radius: int, channel: int) -> int:
    """The lower median of one output pixel by sorting its clipped window
    (numpy array [H, W, C]): element floor((n - 1) / 2) of the sorted values."""
    import numpy as np
    h, w = img.shape[0], img.shape[1]
    win = np.asarray(img[max(0, y - radius):min(h, y + radius + 1), max(0, x - radius):min(w, x + radius + 1), channel])
    vals = np.sort(win.reshape(-1))
    return int(vals[(vals.size - 1) // 2])
