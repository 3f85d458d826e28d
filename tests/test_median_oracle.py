"""Pins of the median oracle (oracle/median_ref.c) against facts that do not
come from it: a hand-computed fixture, an independent brute force that sorts
every window, scipy's median filter on windows the image does not clip,
closed forms (r = 0, constant images, a window covering the whole image) and
the commutation of order statistics with non-decreasing value maps."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from conftest import load_fixture


def rand(h, w, c, seed):
    return np.random.default_rng(seed).integers(0, 256, (h, w, c), dtype=np.uint8)


def test_hand_fixture():
    img, r, _, expects = load_fixture("median_3x3.txt")
    out = oracle.median_ref(img, r, 1)
    for (y, x), (v, _, _) in expects:
        assert out[y, x] == v, (y, x, out[y, x], v)
    # the other channels are not the answer
    assert not np.array_equal(out, oracle.median_ref(img, r, 0))


@settings(max_examples=150, deadline=None)
@given(h=st.integers(1, 7), w=st.integers(1, 7), c=st.integers(1, 4), r=st.integers(0, 4),
       seed=st.integers(0, 10 ** 6), data=st.data())
def test_brute_force(h, w, c, r, seed, data):
    ch = data.draw(st.integers(0, c - 1))
    img = rand(h, w, c, seed)
    want = np.array(oracle.brute_median(img, r, ch), np.uint8)
    assert np.array_equal(oracle.median_ref(img, r, ch), want)


@pytest.mark.parametrize("r", [1, 2, 4, 7])
def test_interior_matches_scipy(r):
    from scipy import ndimage
    img = rand(40, 55, 3, seed=r)
    for ch in range(3):
        out = oracle.median_ref(img, r, ch)
        ref = ndimage.median_filter(img[:, :, ch], size=2 * r + 1, mode="nearest")
        # windows the image does not clip hold (2r+1)^2 values, an odd count:
        # the lower median is the median
        assert np.array_equal(out[r:-r, r:-r], ref[r:-r, r:-r])


def test_closed_forms():
    img = rand(13, 17, 3, seed=5)
    assert np.array_equal(oracle.median_ref(img, 0, 2), img[:, :, 2])
    const = np.full((9, 11, 3), 77, np.uint8)
    assert (oracle.median_ref(const, 3, 0) == 77).all()
    # a window that always covers the whole image: every output is the lower
    # median of all the channel's values
    vals = np.sort(img[:, :, 1].reshape(-1))
    assert (oracle.median_ref(img, 20, 1) == vals[(vals.size - 1) // 2]).all()


def test_monotone_maps_commute():
    img = rand(21, 19, 3, seed=9)
    f = (np.arange(256) // 3).astype(np.uint8)  # non-decreasing
    for r in (1, 3):
        assert np.array_equal(oracle.median_ref(f[img], r, 0), f[oracle.median_ref(img, r, 0)])


def test_threads_and_bad_args():
    img = rand(37, 23, 3, seed=3)
    a = oracle.median_ref(img, 2, 1, nthreads=1)
    assert np.array_equal(a, oracle.median_ref(img, 2, 1, nthreads=5))
    with pytest.raises(ValueError):
        oracle.median_ref(img, 2, 3)
    assert oracle.median_ref(np.zeros((0, 5, 3), np.uint8), 2, 0).shape == (0, 5)


def test_median_at_matches_brute_and_table():
    rng = np.random.default_rng(4)
    for (w, h, c, r) in [(7, 5, 3, 1), (9, 9, 1, 3), (4, 11, 2, 6)]:
        img = rng.integers(0, 256, (h, w, c), dtype=np.uint8)
        want = oracle.brute_median(img.tolist(), r, c - 1)
        table = oracle.median_ref(img, r, c - 1)
        for y in range(h):
            for x in range(w):
                assert oracle.median_at(img, x, y, r, c - 1) == want[y][x] == table[y, x]
