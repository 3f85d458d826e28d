"""Pins for the CPU oracle: facts that do not come from the oracle itself.

Each test checks the oracle against something the paper or mathematics fixes:
hand-computed fixtures (tests/golden), closed forms, invariants, special cases
that reduce to a textbook operation, and an independent brute force.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck
from scipy import ndimage

import oracle
from conftest import load_fixture, ROOT
from paper_1405_1020_amd import synth

LEVEL_SET = [1, 2, 3, 5, 8, 16, 20, 32, 64, 255, 256]


def ref(img, r, L, **kw):
    return oracle.oilpaint_ref(img, r, L, **kw)


# --------------------------------------------------------------------------
# Level step (Section 4 listing; the integer reading of it)
# --------------------------------------------------------------------------

def test_levels_hand_values():
    path = f"{ROOT}/tests/golden/levels_hand.txt"
    n = 0
    for line in open(path):
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        r, g, b, L, k, kp = map(int, line)
        assert oracle.ref_level(r, g, b, L) == k, (r, g, b, L)
        assert oracle.ref_level(r, g, b, L, paper_mode=True) == kp, (r, g, b, L)
        n += 1
    assert n >= 10


def test_levels_range_monotone_and_reachable():
    # every level lies in [0, L), the level never decreases with R+G+B, and
    # all L levels are reachable (the reading gives exactly L bins)
    for L in range(1, 257):
        prev = -1
        seen = set()
        for s in range(766):
            r = min(255, s)
            g = min(255, s - r)
            b = s - r - g
            k = oracle.ref_level(r, g, b, L)
            assert 0 <= k < L
            assert k >= prev
            prev = k
            seen.add(k)
        assert seen == set(range(L)), L


def test_levels_special_cases():
    # L = 256: the level is the integer mean intensity; L = 2^j: the top j
    # bits of the mean intensity; the level depends on R+G+B only
    rng = np.random.default_rng(0)
    for _ in range(2000):
        r, g, b = (int(v) for v in rng.integers(0, 256, 3))
        mean = (r + g + b) // 3
        assert oracle.ref_level(r, g, b, 256) == mean
        for j in range(0, 9):
            assert oracle.ref_level(r, g, b, 1 << j) == mean >> (8 - j)
        L = int(rng.integers(1, 257))
        assert oracle.ref_level(r, g, b, L) == oracle.ref_level(b, r, g, L)


def test_paper_levels_extra_white_level():
    # the listing's double formula reaches level L only at pure white
    for L in (1, 8, 20, 64, 255, 256):
        assert oracle.ref_level(255, 255, 255, L, paper_mode=True) == L
        assert oracle.ref_level(255, 255, 254, L, paper_mode=True) < L


# --------------------------------------------------------------------------
# Hand-computed fixtures
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["worked_example_3x3.txt", "tie_1x4.txt"])
def test_hand_fixtures(name):
    img, r, L, expects = load_fixture(name)
    out = ref(img, r, L)
    for (y, x), rgb in expects:
        assert tuple(int(v) for v in out[y, x]) == rgb, (name, y, x)
    # the independent brute force agrees on the fixture too
    bf = oracle.brute(img.tolist(), r, L)
    for (y, x), rgb in expects:
        assert tuple(bf[y][x]) == rgb


def test_paper_mode_worked_example():
    # the listing writes only the interior; with r = 1 on a 3x3 image that is
    # the centre pixel, whose value is the hand-computed (241, 240, 238)
    img, r, L, _ = load_fixture("worked_example_3x3.txt")
    dst = np.full_like(img, 7)
    oracle.oilpaint_ref(img, r, L, paper_mode=True, out=dst)
    assert tuple(dst[1, 1]) == (241, 240, 238)
    mask = np.ones(img.shape[:2], bool)
    mask[1, 1] = False
    assert (dst[mask] == 7).all()


def test_paper_mode_white_window_not_written():
    # pure white falls in the extra level L, which the listing never selects:
    # every count it scans is zero, so nothing is written
    img = np.full((5, 5, 3), 255, np.uint8)
    dst = np.full_like(img, 3)
    oracle.oilpaint_ref(img, 1, 20, paper_mode=True, out=dst)
    assert (dst == 3).all()
    # one non-white pixel in the window is then the only candidate
    img[2, 2] = (250, 251, 252)
    oracle.oilpaint_ref(img, 1, 20, paper_mode=True, out=dst)
    assert tuple(dst[2, 2]) == (250, 251, 252)
    assert tuple(dst[1, 1]) == (250, 251, 252)


# --------------------------------------------------------------------------
# Invariants and special cases
# --------------------------------------------------------------------------

def test_radius_zero_is_identity():
    img = synth.make_random(37, 23, seed=11)
    for L in LEVEL_SET:
        assert np.array_equal(ref(img, 0, L), img)


def test_constant_image_unchanged():
    for rgb in [(0, 0, 0), (255, 255, 255), (13, 200, 77)]:
        img = np.empty((9, 14, 3), np.uint8)
        img[:] = rgb
        for r in (1, 3, 20):
            for L in (1, 20, 256):
                assert np.array_equal(ref(img, r, L), img)


def test_output_within_window_min_max():
    img = synth.make_image(61, 47, seed=3, n_blobs=6, sigma=(5, 15))
    for r, L in [(1, 20), (2, 8), (4, 64), (7, 256)]:
        out = ref(img, r, L).astype(int)
        size = 2 * r + 1
        for c in range(3):
            lo = ndimage.minimum_filter(img[..., c], size=size, mode="nearest")
            hi = ndimage.maximum_filter(img[..., c], size=size, mode="nearest")
            assert (out[..., c] >= lo).all() and (out[..., c] <= hi).all()


def box_mean_floor(img, r):
    """Floored mean over the clipped (2r+1)^2 window via integral images."""
    h, w, _ = img.shape
    integ = np.zeros((h + 1, w + 1, 3), np.int64)
    integ[1:, 1:] = img.astype(np.int64).cumsum(0).cumsum(1)
    ys = np.arange(h)
    xs = np.arange(w)
    y0 = np.clip(ys - r, 0, h)[:, None]
    y1 = np.clip(ys + r + 1, 0, h)[:, None]
    x0 = np.clip(xs - r, 0, w)[None, :]
    x1 = np.clip(xs + r + 1, 0, w)[None, :]
    tot = integ[y1, x1] - integ[y0, x1] - integ[y1, x0] + integ[y0, x0]
    cnt = ((y1 - y0) * (x1 - x0))[..., None]
    return (tot // cnt).astype(np.uint8)


def test_single_level_is_box_mean():
    # L = 1 puts every pixel in level 0, so the filter is a floored box mean
    for (w, h, seed) in [(40, 31, 5), (7, 3, 6), (1, 9, 7)]:
        img = synth.make_random(w, h, seed)
        for r in (1, 2, 5, 12):
            assert np.array_equal(ref(img, r, 1), box_mean_floor(img, r)), (w, h, r)


def _edge_expect(W, e, r, left, right, l_left, l_right):
    """Closed form for an image whose columns x < e hold `left` and x >= e
    hold `right`: in a clipped window of h rows the two levels hold
    (#left columns)*h and (#right columns)*h pixels; ties go to the lower
    level."""
    want = []
    for x in range(W):
        x0, x1 = max(0, x - r), min(W - 1, x + r)
        nl = max(0, min(x1, e - 1) - x0 + 1)
        nr = (x1 - x0 + 1) - nl
        if nl > nr or (nl == nr and l_left < l_right):
            want.append(left)
        else:
            want.append(right)
    return want


def test_two_colour_edge_closed_form():
    A = (30, 40, 50)     # level at L=20: 40*20/256 = 3
    B = (200, 210, 220)  # level at L=20: 210*20/256 = 16
    W, H = 23, 6
    for e in (9, 12):
        for left, right, ll, lr in [(A, B, 3, 16), (B, A, 16, 3)]:
            img = np.empty((H, W, 3), np.uint8)
            img[:, :e] = left
            img[:, e:] = right
            for r in (1, 2, 4, 7):
                out = ref(img, r, 20)
                want = _edge_expect(W, e, r, left, right, ll, lr)
                for x in range(W):
                    for y in range(H):
                        assert tuple(out[y, x]) == want[x], (e, r, x, y)


def test_symmetries():
    img = synth.make_image(33, 21, seed=9, n_blobs=5, sigma=(3, 10))
    for r, L in [(1, 20), (3, 8), (5, 32)]:
        base = ref(img, r, L)
        assert np.array_equal(ref(img[:, ::-1].copy(), r, L), base[:, ::-1])
        assert np.array_equal(ref(img[::-1].copy(), r, L), base[::-1])
        assert np.array_equal(ref(img.transpose(1, 0, 2).copy(), r, L), base.transpose(1, 0, 2))
        for perm in ([1, 2, 0], [2, 0, 1], [0, 2, 1]):
            assert np.array_equal(ref(img[..., perm].copy(), r, L), base[..., perm])


def test_crop_consistency():
    # an output pixel whose whole window lies inside a crop is unchanged by
    # the crop
    img = synth.make_image(50, 40, seed=12, n_blobs=6, sigma=(4, 12))
    r, L = 3, 20
    full = ref(img, r, L)
    y0, y1, x0, x1 = 5, 31, 8, 44
    crop = ref(img[y0:y1, x0:x1].copy(), r, L)
    inner = crop[r:(y1 - y0) - r, r:(x1 - x0) - r]
    assert np.array_equal(inner, full[y0 + r:y1 - r, x0 + r:x1 - r])


def test_threads_match_single_thread():
    img = synth.make_image(97, 61, seed=13, n_blobs=6, sigma=(4, 12))
    one = ref(img, 4, 20, nthreads=1)
    for t in (2, 3, 8, 500):
        assert np.array_equal(ref(img, 4, 20, nthreads=t), one)


def test_stride_padding_neither_read_nor_written():
    img = synth.make_random(13, 11, seed=14)
    w, h = 13, 11
    stride = 3 * w + 7
    rng = np.random.default_rng(1)
    src = rng.integers(0, 256, size=h * stride, dtype=np.uint8)
    for y in range(h):
        src[y * stride:y * stride + 3 * w] = img[y].reshape(-1)
    dst = rng.integers(0, 256, size=h * stride, dtype=np.uint8)
    before = dst.copy()
    oracle.oilpaint_ref_buffer(src, dst, w, h, stride, 2, 20)
    want = ref(img, 2, 20)
    for y in range(h):
        assert np.array_equal(dst[y * stride:y * stride + 3 * w], want[y].reshape(-1))
        assert np.array_equal(dst[y * stride + 3 * w:(y + 1) * stride],
                              before[y * stride + 3 * w:(y + 1) * stride])


def test_rejects_bad_arguments():
    img = np.zeros((4, 4, 3), np.uint8)
    with pytest.raises(ValueError):
        ref(img, -1, 20)
    with pytest.raises(ValueError):
        ref(img, 1, 0)
    with pytest.raises(ValueError):
        ref(img, 1, 257)
    buf = np.zeros(64, np.uint8)
    with pytest.raises(ValueError):
        oracle.oilpaint_ref_buffer(buf, buf.copy(), 4, 2, 11, 1, 20)


def test_empty_images_are_noops():
    for shape in [(0, 5, 3), (5, 0, 3), (0, 0, 3)]:
        img = np.zeros(shape, np.uint8)
        assert ref(img, 2, 20).shape == shape


# --------------------------------------------------------------------------
# Independent brute force on tiny images
# --------------------------------------------------------------------------

@st.composite
def tiny_case(draw):
    w = draw(st.integers(1, 9))
    h = draw(st.integers(1, 9))
    r = draw(st.integers(0, 5))
    L = draw(st.sampled_from(LEVEL_SET))
    palette = draw(st.integers(1, 6))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.default_rng(seed)
    if palette < 6:
        # few distinct colours make ties and shared levels common
        cols = rng.integers(0, 256, size=(palette, 3))
        img = cols[rng.integers(0, palette, size=(h, w))].astype(np.uint8)
    else:
        img = rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8)
    return img, r, L


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_case())
def test_brute_force_agrees(case):
    img, r, L = case
    got = ref(img, r, L)
    want = np.array(oracle.brute(img.tolist(), r, L), dtype=np.uint8).reshape(img.shape)
    assert np.array_equal(got, want)
