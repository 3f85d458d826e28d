"""GPU parity of the windowed median (oilpaint_median_async) against the CPU
median oracle, bit-exact, through the C-ABI: every radius 0..15 (both count
widths), 1 to 4 channels, every channel, padded strides on both sides,
ragged sizes around the strip width, radii clipped by the image, the
1920x1080 image in full, the column-histogram form (every strip chunk count,
radius up to 127, and forced onto small radii), the installed-form switch,
and error paths leaving dst untouched."""
import numpy as np
import pytest

import oracle
from paper_1405_1020_amd import binding as B
from paper_1405_1020_amd import synth
from gpu_util import first_mismatch, torch_mod, ORACLE_THREADS

pytestmark = pytest.mark.gpu


def device_planes(img, spad, dpad, seed):
    """src [H, W, C] with row padding spad, dst [H, W] with row padding dpad
    prefilled with seeded junk; returns (src, dst, dst_buffer)."""
    torch = torch_mod()
    h, w, c = img.shape
    sbuf = torch.from_numpy(np.random.default_rng(seed).integers(0, 256, (h, w * c + spad), dtype=np.uint8)).cuda()
    sbuf[:, :w * c] = torch.from_numpy(img.reshape(h, w * c)).cuda()
    src = sbuf.as_strided((h, w, c), (w * c + spad, c, 1))
    dbuf = torch.from_numpy(np.random.default_rng(seed + 1).integers(0, 256, (h, w + dpad), dtype=np.uint8)).cuda()
    dst = dbuf.as_strided((h, w), (w + dpad, 1))
    return src, dst, dbuf


def check(img, r, ch, spad=0, dpad=0, kind=B.MEDIAN_AUTO):
    torch = torch_mod()
    h, w, _ = img.shape
    src, dst, dbuf = device_planes(img, spad, dpad, seed=r + 7 * ch)
    before = dbuf[:, w:].clone()
    B.median_async(src, dst, r, ch, kind=kind)
    torch.cuda.synchronize()
    assert torch.equal(before, dbuf[:, w:]), "dst padding was written"
    got = dst.cpu().numpy()
    want = oracle.median_ref(img, r, ch, nthreads=ORACLE_THREADS)
    mm = first_mismatch(got[..., None], want[..., None])
    assert mm is None, (img.shape, r, ch, spad, dpad, kind, mm)


@pytest.mark.parametrize("r", list(range(16)))
def test_median_every_radius(r):
    for (w, h, c) in [(1, 1, 3), (63, 2 * r + 1, 1), (65, 2 * r + 3, 4), (130, 57, 3)]:
        img = (synth.make_image(w, h, seed=500 + r + w, n_blobs=4, sigma=(2, 15)) if c == 3 and w * h > 100
               else np.random.default_rng(500 + r + w).integers(0, 256, (h, w, c), dtype=np.uint8))
        for ch in range(c):
            check(img, r, ch, spad=(w + r) % 5, dpad=(h + r) % 3)


def test_median_fhd_full():
    img = synth.fhd_image()
    for r in (1, 5, 15):
        check(img, r, 1)


def test_median_errors_leave_dst_untouched():
    torch = torch_mod()
    img = synth.make_random(40, 30, seed=1)
    src, dst, dbuf = device_planes(img, 0, 0, seed=3)
    before = dbuf.clone()
    wide = synth.make_random(200, 30, seed=2)
    wsrc, wdst, wbuf = device_planes(wide, 0, 0, seed=4)
    wbefore = wbuf.clone()
    with pytest.raises(B.OilpaintError) as e:
        B.median_async(wsrc, wdst, 128, 0)  # effective radius 128
    assert e.value.status == B.ERR_UNSUPPORTED
    with pytest.raises(B.OilpaintError) as e:
        B.median_async(src, dst, 20, 0, kind=B.MEDIAN_FOUR)  # the LDS forms stop at 15
    assert e.value.status == B.ERR_UNSUPPORTED
    with pytest.raises(B.OilpaintError) as e:
        B.median_async(src, dst, 2, 0, kind=7)
    assert e.value.status == B.ERR_ARG
    with pytest.raises(B.OilpaintError) as e:
        B.median_async(src, dst, 2, 3)
    assert e.value.status == B.ERR_ARG
    torch.cuda.synchronize()
    assert torch.equal(before, dbuf) and torch.equal(wbefore, wbuf)
    # the synchronous form on the default stream
    out = torch.empty(30, 40, dtype=torch.uint8, device="cuda")
    L = B.lib()
    import ctypes
    st = L.oilpaint_median(ctypes.c_void_p(src.data_ptr()), 120, 3, 2, ctypes.c_void_p(out.data_ptr()), 40, 40, 30, 3)
    assert st == B.OK
    assert np.array_equal(out.cpu().numpy(), oracle.median_ref(img, 3, 2))


@pytest.mark.parametrize("r", [1, 2, 7, 16, 31, 32, 33, 63, 64, 95, 96, 127])
def test_median_column_form(r):
    # the column-histogram form on ragged sizes: strips of 1 .. 5 chunks of 64
    # columns with their halo, windows clipped by the image on every side
    for (w, h, c) in [(70, 2 * r + 3, 1), (150, 90, 3), (203, 131, 4)]:
        img = (synth.make_image(w, h, seed=900 + r + w, n_blobs=5, sigma=(2, 30)) if c == 3
               else np.random.default_rng(900 + r + w).integers(0, 256, (h, w, c), dtype=np.uint8))
        for ch in range(c):
            check(img, r, ch, spad=(w + r) % 5, dpad=(h + r) % 3, kind=B.MEDIAN_COLUMN)
    # the built-in choice above radius 15 is the column form
    if r > 15:
        assert B.median_pick_kind(r) == B.MEDIAN_COLUMN


def test_median_column_fhd_full():
    img = synth.fhd_image()
    for r in (16, 40):
        check(img, r, 1)


def test_median_installed_kind():
    torch = torch_mod()
    img = synth.make_image(150, 97, seed=31, n_blobs=5, sigma=(2, 30))
    try:
        B.median_set_kind(5, B.MEDIAN_COLUMN)
        assert B.median_pick_kind(5) == B.MEDIAN_COLUMN
        check(img, 5, 0)
        B.median_set_kind(5, B.MEDIAN_FOUR)
        assert B.median_pick_kind(5) == B.MEDIAN_FOUR
        check(img, 5, 2)
        with pytest.raises(B.OilpaintError):
            B.median_set_kind(20, B.MEDIAN_ONE)
    finally:
        for r in range(128):
            B.median_set_kind(r, B.MEDIAN_AUTO)
    torch.cuda.synchronize()
