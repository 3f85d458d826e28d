"""GPU parity: the HIP path, called through the C-ABI, against the CPU oracle.

The bar is bit-exact equality (all arithmetic is integer).  Sizes span
several tiles with ragged tails; the benchmark images (256x256 r=2 L=20,
1920x1080 over the r/L sweep, 4000x3000 r=10 L=32) are compared in full.
"""
import numpy as np
import pytest

from paper_1405_1020_amd import binding as B
from paper_1405_1020_amd import synth
from gpu_util import (to_device, empty_like_device, from_device, padding_bytes, ref, ref_pixel,
                      first_mismatch, torch_mod)

pytestmark = pytest.mark.gpu


def run_plain(img, r, L, pad=0, variant=None):
    torch = torch_mod()
    h, w, _ = img.shape
    src, sbuf = to_device(img, pad=pad, seed=3)
    dst, dbuf = empty_like_device(img, pad=pad, seed=5)
    before = padding_bytes(dbuf, h, w, 3 * w + pad)
    B.oilpaint_async(src, dst, r, L, variant=variant)
    torch.cuda.synchronize()
    after = padding_bytes(dbuf, h, w, 3 * w + pad)
    assert np.array_equal(before, after), "dst padding was written"
    return from_device(dst)


def check(img, r, L, **kw):
    got = run_plain(img, r, L, **kw)
    want = ref(img, r, L)
    mm = first_mismatch(got, want)
    assert mm is None, ("mismatch (y, x, got, want, count)", mm, img.shape, r, L, kw)


def test_small_case_exact():
    img, r, L = synth.small_case()
    print("small case 256x256", r, L, flush=True)
    check(img, r, L)


@pytest.mark.parametrize("r,L", synth.FHD_SWEEP)
def test_fhd_sweep_exact(r, L):
    print("fhd", r, L, flush=True)
    check(synth.fhd_image(), r, L)


# the column layout's radius <= 15 form at full size, in the launch shapes
# the tuner installs for the sweep (four wavefronts, eight per CU) and with
# one and two wavefronts per strip; L = 32 takes the 11-word bucket
@pytest.mark.parametrize("r,L,waves,per_cu", [(10, 20, 4, 8), (15, 20, 4, 8), (15, 20, 1, 8), (15, 20, 2, 8),
                                              (12, 32, 4, 4), (7, 16, 4, 6)])
def test_fhd_column15_exact(r, L, waves, per_cu):
    print("fhd column15", r, L, waves, per_cu, flush=True)
    check(synth.fhd_image(), r, L, variant=B.Variant(0, waves, B.HIST_COLUMN, 64, per_cu))


# Plain launches deal their tiles to the XCDs in chunks of neighbours, with
# the last partial round of chunks in launch order: grids just below, at
# and above whole rounds (32 tiles), one strip wide and three, in each
# layout family (fixed 8-row runs, so the tile count is set by the height)
@pytest.mark.parametrize("tiles_x,tiles_y", [(1, 31), (1, 32), (1, 33), (1, 97), (3, 11), (3, 21), (5, 13)])
@pytest.mark.parametrize("variant", [B.Variant(8, 1, B.HIST_STREAM, 64, 8), B.Variant(8, 4, B.HIST_STREAM, 64, 4),
                                     B.Variant(8, 4, B.HIST_COLUMN, 64, 4)], ids=["stream", "split", "column15"])
def test_tile_dealing_grid_sizes(tiles_x, tiles_y, variant):
    w, h = 64 * tiles_x - 17, 8 * tiles_y - 3  # ragged last strip and run
    img = synth.make_image(w, h, seed=tiles_x * 100 + tiles_y, n_blobs=6, sigma=(3, 25))
    print("tile grid", tiles_x, tiles_y, variant, flush=True)
    check(img, 5, 20, variant=variant)


def test_camera_exact():
    img = synth.camera_image()
    r, L = synth.CAMERA_RL
    print("camera 4000x3000", r, L, flush=True)
    check(img, r, L)


RAGGED = [(1, 1), (1, 7), (7, 1), (2, 3), (63, 5), (64, 64), (65, 17), (129, 70), (200, 33), (31, 300)]


@pytest.mark.parametrize("w,h", RAGGED)
def test_ragged_sizes(w, h):
    rng = np.random.default_rng(w * 1000 + h)
    img = synth.make_image(w, h, seed=w + h, n_blobs=4, sigma=(2, 20)) if w * h > 100 else \
        synth.make_random(w, h, seed=w + h)
    for r in (0, 1, 2, 5, 15):
        L = int(rng.choice([1, 2, 8, 20, 32, 64, 255]))
        print("ragged", w, h, r, L, flush=True)
        check(img, r, L, pad=int(rng.integers(0, 9)))


@pytest.mark.parametrize("r,L", [(16, 20), (20, 8), (40, 32), (3, 256), (1, 256), (60, 64)])
def test_wide_layout(r, L):
    img = synth.make_image(150, 97, seed=r + L, n_blobs=5, sigma=(5, 30))
    print("wide", r, L, flush=True)
    check(img, r, L, pad=5)


def test_radius_larger_than_image():
    img = synth.make_random(9, 6, seed=2)
    for r in (8, 9, 100, 5000, 65535):
        check(img, r, 20)


def test_every_variant_same_bytes():
    img = synth.make_image(333, 211, seed=77, n_blobs=8, sigma=(4, 40))
    for r, L in [(2, 20), (7, 64), (15, 8), (9, 32), (3, 16)]:
        want = ref(img, r, L)
        for rows in (1, 3, 8, 16, 64):
            for waves in (1, 2, 4, 8):
                for lanes in (16, 32, 64):
                    for hist in (B.HIST_PACKED, B.HIST_STREAM, B.HIST_WIDE, B.HIST_STREAM8, B.HIST_REGS):
                        v = B.Variant(rows, waves, hist, lanes)
                        try:
                            got = run_plain(img, r, L, pad=3, variant=v)
                        except B.OilpaintError as e:
                            assert e.status == B.ERR_UNSUPPORTED, (v, e)
                            continue
                        mm = first_mismatch(got, want)
                        assert mm is None, (r, L, v, mm)


@pytest.mark.parametrize("r", list(range(16)))
def test_stream_every_radius(r):
    # the streamed-row kernels, one per radius, on sizes around the strip
    # width and the ring height, several run lengths and level counts
    for (w, h) in [(1, 1), (63, 2 * r + 1), (65, 2 * r + 3), (130, 57)]:
        img = synth.make_image(w, h, seed=100 + r + w, n_blobs=4, sigma=(2, 15)) if w * h > 100 else \
            synth.make_random(w, h, seed=100 + r + w)
        want = {L: ref(img, r, L) for L in (1, 8, 9, 16, 20, 32, 33, 64)}
        for rows in (1, 2, 5, 16, 300):
            for L in (1, 8, 9, 16, 20, 32, 33, 64):
                for hist, waves in ((B.HIST_STREAM, 1), (B.HIST_STREAM, 4), (B.HIST_STREAM8, 1), (B.HIST_STREAM8, 4),
                                    (B.HIST_REGS, 1)):
                    v = B.Variant(rows, waves, hist, 64)
                    reff = min(r, max(w, h) - 1)
                    if (hist == B.HIST_STREAM8 and not (8 <= reff and L <= 32)) or \
                            (hist == B.HIST_REGS and not (reff <= 7 and L <= 16)):
                        with pytest.raises(B.OilpaintError) as e:
                            run_plain(img, r, L, pad=(w + rows) % 5, variant=v)
                        assert e.value.status == B.ERR_UNSUPPORTED
                        continue
                    got = run_plain(img, r, L, pad=(w + rows) % 5, variant=v)
                    mm = first_mismatch(got, want[L])
                    assert mm is None, (w, h, r, L, rows, hist, waves, mm)


def test_repeat_is_deterministic():
    img = synth.fhd_image()
    a = run_plain(img, 10, 20)
    b = run_plain(img, 10, 20)
    assert np.array_equal(a, b)


def test_errors_leave_dst_untouched():
    torch = torch_mod()
    img = synth.make_random(40, 30, seed=9)
    src, _ = to_device(img)
    dst, dbuf = empty_like_device(img)
    before = dbuf.cpu().numpy().copy()
    with pytest.raises(B.OilpaintError) as e:
        B.oilpaint_async(src, dst, -1, 20)
    assert e.value.status == B.ERR_ARG
    with pytest.raises(B.OilpaintError) as e:
        B.oilpaint_async(src, dst, 2, 0)
    assert e.value.status == B.ERR_ARG
    # src and dst overlapping: the same buffer
    with pytest.raises(B.OilpaintError) as e:
        B.oilpaint_async(src, src, 2, 20)
    assert e.value.status == B.ERR_OVERLAP
    # host memory is rejected
    lib = B.lib()
    host = np.zeros(40 * 30 * 3, np.uint8)
    import ctypes
    st = lib.oilpaint_async(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(host.ctypes.data), 40, 30, 120, 2,
                            20, None)
    assert st == B.ERR_NOT_DEVICE
    torch.cuda.synchronize()
    assert np.array_equal(before, dbuf.cpu().numpy())


def test_sync_entry_point():
    torch = torch_mod()
    import ctypes
    img = synth.make_image(300, 200, seed=4, n_blobs=5, sigma=(5, 40))
    src, _ = to_device(img)
    dst, _ = empty_like_device(img)
    st = B.lib().oilpaint(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), 300, 200, 900, 3, 16)
    assert st == B.OK
    assert first_mismatch(from_device(dst), ref(img, 3, 16)) is None
    torch.cuda.synchronize()


def test_empty_images_noop():
    torch = torch_mod()
    import ctypes
    for (w, h) in [(0, 5), (5, 0)]:
        src = torch.zeros((h, w, 3), dtype=torch.uint8, device="cuda")
        dst = torch.zeros((h, w, 3), dtype=torch.uint8, device="cuda")
        B.oilpaint_async(src, dst, 2, 20)
    # through the C-ABI with real pointers and a zero size
    a = torch.full((64,), 9, dtype=torch.uint8, device="cuda")
    b = torch.full((64,), 9, dtype=torch.uint8, device="cuda")
    for (w, h) in [(0, 5), (5, 0), (0, 0)]:
        st = B.lib().oilpaint_async(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), w, h, 15, 2, 20,
                                    None)
        assert st == B.OK
    torch.cuda.synchronize()
    assert int(b.eq(9).all()) == 1


def test_sampled_pixels_full_size_camera():
    # the camera image in the launch configuration the benchmark uses, with
    # oracle values computed pixel by pixel at sampled positions (borders,
    # corners and random interior points)
    img = synth.camera_image()
    r, L = synth.CAMERA_RL
    got = run_plain(img, r, L)
    h, w, _ = img.shape
    rng = np.random.default_rng(0)
    pts = [(0, 0), (w - 1, 0), (0, h - 1), (w - 1, h - 1), (r, r), (w // 2, h // 2)]
    pts += [(int(x), int(y)) for x, y in zip(rng.integers(0, w, 200), rng.integers(0, h, 200))]
    for x, y in pts:
        assert tuple(got[y, x]) == tuple(ref_pixel(img, x, y, r, L)), (x, y)


@pytest.mark.parametrize("r", [1, 3, 7, 10, 15])
def test_paper_form_every_default_layout(r):
    # the listing's literal form (interior pixels only, the pure-white level
    # never chosen, nothing written where the winning count is 0) through the
    # library's own launch shapes: one wavefront per strip below radius 7,
    # four from 7 on, the tile-staged or wide layouts beyond 64 levels
    torch = torch_mod()
    img = synth.make_image(203, 149, seed=40 + r, n_blobs=6, sigma=(4, 40))
    img[20:60, 30:90] = 255
    img[100:104, :] = 255
    junk = np.random.default_rng(r).integers(0, 256, size=img.shape, dtype=np.uint8)
    for L in (8, 20, 33, 64, 200):
        print("paper", r, L, flush=True)
        src, _ = to_device(img, pad=3, seed=1)
        dst, dbuf = to_device(junk, pad=3, seed=2)
        B.run(B.Item(src, dst, r, L, flags=B.FLAG_PAPER))
        torch.cuda.synchronize()
        want = ref(img, r, L, paper=True, out=junk.copy())
        mm = first_mismatch(from_device(dst), want)
        assert mm is None, (r, L, B.pick_variant(203, 149, r, L).as_tuple(), mm)


def test_row_bands_four_wavefronts():
    # output-row bands through the descriptor path (each band a launch of its
    # own, its windows reaching rows outside the band) with the four-wavefront
    # streamed shapes, against the whole image's oracle output
    torch = torch_mod()
    img = synth.make_image(190, 141, seed=71, n_blobs=6, sigma=(4, 40))
    for r, L, hist in ((10, 20, B.HIST_STREAM), (12, 32, B.HIST_STREAM8), (15, 64, B.HIST_STREAM)):
        want = ref(img, r, L)
        src, _ = to_device(img, pad=2)
        dst, _ = empty_like_device(img, pad=2)
        B.set_variant(r, L, B.Variant(0, 4, hist, 64, 4))
        try:
            for a, b in ((0, 1), (1, 30), (30, 31), (31, 100), (100, 141)):
                B.run(B.Item(src, dst, r, L, row_begin=a, row_end=b))
            torch.cuda.synchronize()
        finally:
            B.clear_variants()
        mm = first_mismatch(from_device(dst), want)
        assert mm is None, (r, L, hist, mm)


def test_paper_form_tiny_images():
    # the listing's form filters [r, W-r) x [r, H-r) with the radius as given,
    # so on images with 2r >= W or 2r >= H nothing is written (the clipped
    # form clamps the radius to the image instead)
    torch = torch_mod()
    for w, h in ((1, 1), (2, 2), (1, 5), (3, 2), (5, 5), (7, 3)):
        img = synth.make_image(w, h, seed=w * 10 + h, n_blobs=2, sigma=(1, 3))
        for r in (1, 2, 3):
            junk = np.random.default_rng(w * 100 + h * 10 + r).integers(0, 256, size=img.shape, dtype=np.uint8)
            src, _ = to_device(img, pad=1, seed=3)
            dst, _ = to_device(junk, pad=1, seed=4)
            B.run(B.Item(src, dst, r, 20, flags=B.FLAG_PAPER))
            torch.cuda.synchronize()
            want = ref(img, r, 20, paper=True, out=junk.copy())
            mm = first_mismatch(from_device(dst), want)
            assert mm is None, (w, h, r, mm)
