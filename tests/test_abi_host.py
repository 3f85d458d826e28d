"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every function include/oilpaint.h declares, and its pure-host argument
validation returns the documented status codes."""
import ctypes

import pytest

from paper_1405_1020_amd import binding as B


def test_library_loads_and_exports_every_declared_symbol():
    lib = B.lib()
    names = B.header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # and the binding knows every one of them, with the same names
    assert set(names) == set(B._SIGS)


def test_version_and_strerror():
    assert B.version() == 1
    for st in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert B.strerror(st) and B.strerror(st) != "unknown status"
    assert B.strerror(-99) == "unknown status"


BASE = 1 << 32  # fake, never dereferenced: validation is pure host


def v(src=BASE, dst=BASE + (1 << 30), w=64, h=48, s=192, r=2, L=20):
    return B.validate(src, dst, w, h, s, r, L)


def test_validate_ok_and_noop_sizes():
    assert v() == B.OK
    assert v(w=0) == B.OK
    assert v(h=0) == B.OK
    assert v(w=0, h=0, s=0) == B.OK
    assert v(r=0) == B.OK and v(r=65535) == B.OK
    assert v(L=1) == B.OK and v(L=256) == B.OK
    assert v(s=193) == B.OK


def test_validate_null():
    assert v(src=0) == B.ERR_NULL
    assert v(dst=0) == B.ERR_NULL
    assert v(src=0, w=0) == B.ERR_NULL


@pytest.mark.parametrize("kw", [dict(w=-1), dict(h=-1), dict(r=-1), dict(r=65536), dict(L=0),
                                dict(L=257), dict(s=191), dict(s=-3), dict(w=1 << 30, s=1 << 30)])
def test_validate_bad_args(kw):
    assert v(**kw) == B.ERR_ARG


def test_validate_overlap():
    span = 47 * 192 + 192
    assert v(src=BASE, dst=BASE) == B.ERR_OVERLAP
    assert v(src=BASE, dst=BASE + span - 1) == B.ERR_OVERLAP
    assert v(src=BASE + span - 1, dst=BASE) == B.ERR_OVERLAP
    assert v(src=BASE, dst=BASE + span) == B.OK
    # the padding of the last row is not part of the range
    assert v(src=BASE, dst=BASE + 47 * 200 + 192, s=200) == B.OK


def test_median_argument_checks():
    # the median entry point's checks that come before any device call
    L = B.lib()
    buf = (ctypes.c_uint8 * 4096)()
    a = ctypes.addressof(buf)
    src, dst = ctypes.c_void_p(a), ctypes.c_void_p(a + 2048)
    call = lambda s, ss, c, ch, d, ds, w, h, r: L.oilpaint_median_async(s, ss, c, ch, d, ds, w, h, r, None)
    assert call(None, 30, 3, 0, dst, 10, 10, 5, 2) == B.ERR_NULL
    assert call(src, 30, 3, 0, None, 10, 10, 5, 2) == B.ERR_NULL
    assert call(src, 30, 3, 3, dst, 10, 10, 5, 2) == B.ERR_ARG   # channel
    assert call(src, 30, 5, 0, dst, 10, 10, 5, 2) == B.ERR_ARG   # channels
    assert call(src, 29, 3, 0, dst, 10, 10, 5, 2) == B.ERR_ARG   # src stride
    assert call(src, 30, 3, 0, dst, 9, 10, 5, 2) == B.ERR_ARG    # dst stride
    assert call(src, 30, 3, 0, dst, 10, 10, 5, -1) == B.ERR_ARG
    assert call(src, 30, 3, 0, dst, 10, -1, 5, 2) == B.ERR_ARG
    assert call(src, 30, 3, 0, dst, 10, 0, 5, 2) == B.OK         # empty: nothing to do
    assert call(src, 30, 3, 0, ctypes.c_void_p(a + 100), 10, 10, 5, 2) == B.ERR_OVERLAP
    # radius 128 on a 129 x 1 image is 128 effective: beyond the median kernels
    assert call(src, 387, 3, 0, dst, 129, 129, 1, 128) == B.ERR_UNSUPPORTED
    # an explicit form that does not cover the radius, and an unknown form
    kcall = lambda r, k: L.oilpaint_median_async_kind(src, 60, 3, 0, dst, 20, 20, 20, r, k, None)
    assert kcall(16, B.MEDIAN_ONE) == B.ERR_UNSUPPORTED and kcall(16, B.MEDIAN_FOUR) == B.ERR_UNSUPPORTED
    assert kcall(2, 4) == B.ERR_ARG and kcall(2, -1) == B.ERR_ARG
    assert L.oilpaint_median_set_kind(16, B.MEDIAN_ONE) == B.ERR_UNSUPPORTED
    assert L.oilpaint_median_set_kind(128, B.MEDIAN_COLUMN) == B.ERR_ARG
    assert L.oilpaint_median_pick_kind(16) == B.MEDIAN_COLUMN and L.oilpaint_median_pick_kind(128) == B.ERR_UNSUPPORTED
    # on a 10 x 5 image it is 9 effective: valid, and host memory is refused
    assert call(src, 30, 3, 0, dst, 10, 10, 5, 16) == B.ERR_NOT_DEVICE


def test_pick_variant_shapes():
    # the choice is pure host logic once the device facts are cached; without
    # a GPU it falls back to nominal facts
    vv = B.pick_variant(1920, 1080, 5, 20)
    assert vv.hist == B.HIST_STREAM and vv.lanes == 64 and vv.waves == 1 and vv.rows >= 1
    # four wavefronts per strip for wide windows and many levels
    for r, L in ((7, 20), (15, 20), (5, 64)):
        vv = B.pick_variant(1920, 1080, r, L)
        assert vv.hist == B.HIST_STREAM and vv.lanes == 64 and vv.waves == 4 and vv.rows >= 1, (r, L)
    vv = B.pick_variant(1920, 1080, 5, 100)
    assert vv.hist == B.HIST_PACKED and vv.lanes in (16, 32, 64) and 1 <= vv.waves <= 8 and vv.rows >= 1
    assert B.pick_variant(1920, 1080, 16, 20).hist == B.HIST_COLUMN
    # (without a GPU the on-chip budget is the nominal 64 KB)
    assert B.pick_variant(1920, 1080, 100, 20).hist == B.HIST_COLUMN
    assert B.pick_variant(1920, 1080, 255, 64).hist == B.HIST_WIDE   # 65 x 574 x 8 B do not fit
    assert B.pick_variant(1920, 1080, 256, 20).hist == B.HIST_WIDE   # beyond the column layout
    assert B.pick_variant(1920, 1080, 200, 256).hist == B.HIST_WIDE  # column histograms do not fit
    assert B.pick_variant(1920, 1080, 5, 256).hist == B.HIST_WIDE
    # a radius beyond the image behaves as the image size
    assert B.pick_variant(12, 10, 1000, 20).hist == B.HIST_STREAM
    # rows derived from the workgroup density: about per_cu (8 by default for
    # one wavefront) workgroups per CU, at least 2 rows, at most 1024
    assert B.pick_variant(1920, 1080, 2, 20).rows == 16    # 30 strips x 1080 rows / (8 x 256)
    assert B.pick_variant(640, 480, 2, 20).rows == 3       # 10 x 480 / 2048
    assert B.pick_variant(256, 256, 2, 20).rows == 2       # half a row per workgroup: the floor
    assert B.pick_variant(64, 100000, 2, 20).rows == 49
    assert B.pick_variant(20, 10, 1000, 20).hist == B.HIST_COLUMN  # effective radius 19


def test_stream_split_limits():
    # four wavefronts per strip: radius <= 15, levels <= 64, 64 lanes; other
    # wavefront counts are refused for the streamed layout
    try:
        assert B.set_variant(0, 1, B.Variant(0, 4, B.HIST_STREAM, 64, 4)) == B.OK
        assert B.set_variant(5, 64, B.Variant(0, 4, B.HIST_STREAM, 64, 4)) == B.OK
        assert B.set_variant(15, 20, B.Variant(16, 4, B.HIST_STREAM, 64, 0)) == B.OK
        assert B.set_variant(5, 65, B.Variant(0, 4, B.HIST_STREAM, 64, 4)) == B.ERR_UNSUPPORTED
        assert B.set_variant(16, 20, B.Variant(0, 4, B.HIST_STREAM, 64, 4)) == B.ERR_UNSUPPORTED
        assert B.set_variant(5, 20, B.Variant(0, 2, B.HIST_STREAM, 64, 4)) == B.ERR_UNSUPPORTED
        assert B.set_variant(5, 20, B.Variant(0, 4, B.HIST_STREAM, 32, 4)) == B.ERR_UNSUPPORTED
    finally:
        B.clear_variants()


def test_stream8_limits():
    # 8-byte on-chip row entries: radius 8..15 (effective) and <= 32 levels
    ok = B.Variant(0, 1, B.HIST_STREAM8, 64, 4)
    try:
        assert B.set_variant(10, 32, ok) == B.OK
        assert B.set_variant(8, 1, ok) == B.OK
        assert B.set_variant(7, 20, ok) == B.ERR_UNSUPPORTED
        assert B.set_variant(16, 20, ok) == B.ERR_UNSUPPORTED
        assert B.set_variant(10, 33, ok) == B.ERR_UNSUPPORTED
        assert B.set_variant(10, 20, B.Variant(0, 2, B.HIST_STREAM8, 64, 4)) == B.ERR_UNSUPPORTED
        assert B.set_variant(10, 20, B.Variant(0, 8, B.HIST_STREAM8, 64, 4)) == B.ERR_UNSUPPORTED
        # four wavefronts sharing a strip
        assert B.set_variant(10, 20, B.Variant(0, 4, B.HIST_STREAM8, 64, 4)) == B.OK
        assert B.set_variant(15, 32, B.Variant(0, 4, B.HIST_STREAM8, 64, 2)) == B.OK
        assert B.set_variant(15, 33, B.Variant(0, 4, B.HIST_STREAM8, 64, 2)) == B.ERR_UNSUPPORTED
        assert B.set_variant(7, 20, B.Variant(0, 4, B.HIST_STREAM8, 64, 2)) == B.ERR_UNSUPPORTED
        assert B.set_variant(10, 20, B.Variant(0, 1, B.HIST_STREAM8, 32, 4)) == B.ERR_UNSUPPORTED
    finally:
        B.clear_variants()


def test_column_limits():
    # column histograms: 64 lanes, radius <= 255, and the (levels + 1) x
    # (64 + 2r) 8-byte histograms within the on-chip budget; one wavefront
    # per strip, or two or four in the count-word forms (radius <= 31, at most
    # 64 levels)
    v = B.Variant(0, 1, B.HIST_COLUMN, 64, 2)
    try:
        assert B.set_variant(0, 1, v) == B.OK
        assert B.set_variant(100, 20, v) == B.OK
        assert B.set_variant(32, 40, v) == B.OK
        assert B.set_variant(256, 20, v) == B.ERR_UNSUPPORTED
        assert B.set_variant(200, 256, v) == B.ERR_UNSUPPORTED
        assert B.set_variant(32, 20, B.Variant(0, 2, B.HIST_COLUMN, 64, 2)) == B.ERR_UNSUPPORTED
        assert B.set_variant(20, 20, B.Variant(0, 1, B.HIST_COLUMN, 32, 2)) == B.ERR_UNSUPPORTED
        # two or four wavefronts per strip: radius <= 31 and at most 64 levels
        for waves in (2, 4):
            assert B.set_variant(15, 20, B.Variant(0, waves, B.HIST_COLUMN, 64, 4)) == B.OK
            assert B.set_variant(0, 64, B.Variant(0, waves, B.HIST_COLUMN, 64, 4)) == B.OK
            assert B.set_variant(16, 20, B.Variant(0, waves, B.HIST_COLUMN, 64, 4)) == B.OK
            assert B.set_variant(31, 40, B.Variant(0, waves, B.HIST_COLUMN, 64, 4)) == B.OK
            assert B.set_variant(32, 20, B.Variant(0, waves, B.HIST_COLUMN, 64, 4)) == B.ERR_UNSUPPORTED
            assert B.set_variant(15, 65, B.Variant(0, waves, B.HIST_COLUMN, 64, 4)) == B.ERR_UNSUPPORTED
            assert B.set_variant(20, 65, B.Variant(0, waves, B.HIST_COLUMN, 64, 4)) == B.ERR_UNSUPPORTED
        assert B.set_variant(15, 20, B.Variant(0, 3, B.HIST_COLUMN, 64, 4)) == B.ERR_UNSUPPORTED
        assert B.set_variant(20, 20, B.Variant(0, 3, B.HIST_COLUMN, 64, 4)) == B.ERR_UNSUPPORTED
    finally:
        B.clear_variants()


def test_column_counts_fit():
    # the column layout's packed fields and 32-bit window sums hold their
    # largest values (radius 255: columns of 511 pixels, windows of 511^2)
    col = 2 * 255 + 1
    assert col < 2 ** 13 and 255 * col < 2 ** 17
    assert col * col < 2 ** 32 and 255 * col * col < 2 ** 27
    # prefix sums over a whole strip with its halo stay below 2^32
    assert 255 * col * (64 + 2 * 255) < 2 ** 32
    # the largest strip with its halo spans at most nine wavefront widths
    assert -(-(64 + 2 * 255) // 64) == 9


def test_kernel_integer_identities():
    # facts the kernels' integer arithmetic relies on, checked exhaustively
    # over their whole domains (no GPU, no oracle involved)
    assert all(((s * 43691) >> 17) == s // 3 for s in range(766))
    assert all(((x * 5614337) >> 32) == x // 765 for x in range(765 * 256 + 1))
    for n in range(2, 962):
        m = -(-(1 << 32) // n)
        for s in range(0, 255 * n + 1, max(1, n // 7)):
            assert ((s * m) >> 32) == s // n
        s = 255 * n
        assert ((s * m) >> 32) == s // n and (((s - 1) * m) >> 32) == (s - 1) // n
    for L in range(1, 257):
        for s in range(766):
            assert int(((s * L) / 3.0) / 255.0) == (s * L) // 765


def test_jpeg_subsequence_bits_range():
    # 0 (chosen per scan) or a fixed 64 .. 16384 bits; pure host state
    lib = B.lib()
    try:
        for bits in (0, 64, 512, 16384):
            assert lib.oilpaint_jpeg_set_subsequence_bits(bits) == B.OK
        for bits in (-1, 1, 63, 16385):
            assert lib.oilpaint_jpeg_set_subsequence_bits(bits) == B.ERR_ARG
    finally:
        assert lib.oilpaint_jpeg_set_subsequence_bits(0) == B.OK
