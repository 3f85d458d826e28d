import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_fixture(name):
    """Parse a tests/golden/*.txt image fixture -> (img, radius, levels, expects)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", name)
    pixels, expects, meta = {}, [], {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "pixel":
                y, x, r, g, b = map(int, tok[1:])
                pixels[(y, x)] = (r, g, b)
            elif tok[0] == "expect":
                y, x, r, g, b = map(int, tok[1:])
                expects.append(((y, x), (r, g, b)))
            else:
                meta[tok[0]] = int(tok[1])
    h = 1 + max(y for y, _ in pixels)
    w = 1 + max(x for _, x in pixels)
    img = np.zeros((h, w, 3), dtype=np.uint8)
    for (y, x), v in pixels.items():
        img[y, x] = v
    return img, meta["radius"], meta["levels"], expects
