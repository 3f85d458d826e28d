"""Pins of the JPEG oracle (oracle/jpeg_ref.py) against things other than
itself: scipy's orthonormal DCT-II (the T.81 8 x 8 DCT pair is that
transform), libjpeg through PIL (zig-zag order via the quantization tables it
reports in natural order, Huffman decoding with and without restart
intervals, the inverse DCT within IEEE 1180's one-level peak error, colour
conversion within its fixed-point rounding, forward DCT and quantization),
and hand-computed closed forms."""
import io

import numpy as np
import pytest
import scipy.fft

import oracle.jpeg_ref as J
from paper_1405_1020_amd import synth

PIL = pytest.importorskip("PIL.Image")


def pil_jpeg(img, quality, subsampling, **kw) -> bytes:
    b = io.BytesIO()
    PIL.fromarray(img).save(b, format="JPEG", quality=quality, subsampling=subsampling, **kw)
    return b.getvalue()


def pil_ycc(data: bytes) -> np.ndarray:
    """libjpeg's decoded YCbCr samples (its inverse DCT, no colour conversion;
    chroma upsampled by libjpeg)."""
    im = PIL.open(io.BytesIO(data))
    im.draft("YCbCr", im.size)
    assert im.mode == "YCbCr"
    return np.asarray(im).astype(np.int64)


def test_zigzag_is_figure_a6():
    zz = J.ZIGZAG
    assert sorted(zz) == list(range(64))
    assert zz[:10] == [0, 1, 8, 16, 9, 2, 3, 10, 17, 24]  # (0,0) (0,1) (1,0) (2,0) (1,1) (0,2) ...
    assert zz[-6:] == [61, 54, 47, 55, 62, 63]  # (7,5) (6,6) (5,7) (6,7) (7,6) (7,7)
    # consecutive entries are neighbours: a step along a row or column at the
    # edges, else one diagonal step
    for a, b in zip(zz, zz[1:]):
        ra, ca, rb, cb = a // 8, a % 8, b // 8, b % 8
        assert max(abs(ra - rb), abs(ca - cb)) == 1


@pytest.mark.parametrize("quality", [10, 50, 75, 95])
def test_dqt_dezigzag_matches_libjpeg(quality):
    # PIL reports the quantization tables in natural order; the file stores
    # them in zig-zag order
    img = synth.make_image(40, 24, seed=quality, n_blobs=3, sigma=(3, 10))
    data = pil_jpeg(img, quality, 2)
    j = J.parse(data)
    ref = PIL.open(io.BytesIO(data)).quantization
    assert set(j.qtables) == set(ref)
    for k in ref:
        assert list(j.qtables[k]) == list(ref[k]), k


def test_dct_pair_is_orthonormal_dct2():
    rng = np.random.default_rng(0)
    for _ in range(20):
        s = rng.integers(-128, 128, size=(8, 8)).astype(np.float64)
        F = J.fdct(s)
        assert np.allclose(F, scipy.fft.dctn(s, type=2, norm="ortho"), atol=1e-9)
        C = rng.normal(0, 200, size=(8, 8))
        assert np.allclose(J.idct(C), scipy.fft.idctn(C, type=2, norm="ortho"), atol=1e-9)
        assert np.allclose(J.idct(F), s, atol=1e-9)
    # a flat block has only a DC term: S(0,0) = 8 x the sample
    assert np.allclose(J.fdct(np.full((8, 8), 5.0)), np.pad([[40.0]], ((0, 7), (0, 7))), atol=1e-12)


def test_rounding_rules():
    assert list(J.round_half_up(np.array([0.5, 1.5, -0.5, -1.5, 2.4999, 2.5 - 1e-12]))) == [1, 2, 0, -1, 2, 3]
    assert list(J.round_half_away(np.array([0.5, -0.5, 1.5, -1.5, -0.49]))) == [1, -1, 2, -2, 0]


def test_colour_closed_forms():
    # greys are unchanged both ways (the luma weights sum to 1, the chroma
    # weights to 0)
    k = np.arange(256)
    y, cb, cr = J.rgb_to_ycc(np.stack([k, k, k], -1))
    assert np.array_equal(y, k) and (cb == 128).all() and (cr == 128).all()
    assert np.array_equal(J.ycc_to_rgb(k, np.full(256, 128), np.full(256, 128)), np.stack([k, k, k], -1))
    # pure red: Y = 76.245 -> 76, Cb = 128 - 43.02768 -> 85, Cr = 255.5 -> 256 -> 255
    y, cb, cr = J.rgb_to_ycc(np.array([[255, 0, 0]]))
    assert (int(y[0]), int(cb[0]), int(cr[0])) == (76, 85, 255)
    # Y = 100, Cb = 150, Cr = 90: R = 100 - 53.276 -> 47, G = 100 - 7.570992
    # + 27.137168 -> 119.566 -> 120, B = 100 + 38.984 -> 139
    assert tuple(J.ycc_to_rgb(np.array([100]), np.array([150]), np.array([90]))[0]) == (47, 120, 139)
    # Cr - 128 = 51: R = 100 + 71.502 -> 172 (a coefficient of 1.400 would give
    # 171), G = 100 - 36.420936 -> 64
    assert tuple(J.ycc_to_rgb(np.array([100]), np.array([128]), np.array([179]))[0]) == (172, 64, 100)
    # Cb - 128 = -77: B = 100 - 136.444 -> 0 (clamped); Cb - 128 = 43: B = 100 +
    # 76.196 -> 176, G = 100 - 14.797848 -> 85.202 -> 85
    assert tuple(J.ycc_to_rgb(np.array([100]), np.array([51]), np.array([128]))[0])[2] == 0
    assert tuple(J.ycc_to_rgb(np.array([100]), np.array([171]), np.array([128]))[0]) == (100, 85, 176)


def test_colour_against_pil():
    rng = np.random.default_rng(1)
    rgb = rng.integers(0, 256, size=(1, 200_000, 3), dtype=np.uint8)
    ours = np.stack(J.rgb_to_ycc(rgb), -1)
    pil = np.asarray(PIL.fromarray(rgb).convert("YCbCr")).astype(np.int64)
    assert np.abs(ours - pil).max() <= 1
    ycc = rng.integers(0, 256, size=(1, 200_000, 3), dtype=np.uint8)
    ours = J.ycc_to_rgb(ycc[..., 0], ycc[..., 1], ycc[..., 2]).astype(np.int64)
    pil = np.asarray(PIL.fromarray(ycc, mode="YCbCr").convert("RGB")).astype(np.int64)
    assert np.abs(ours - pil).max() <= 1


@pytest.mark.parametrize("subsampling,quality", [(0, 50), (0, 90), (1, 75), (2, 60), (2, 95)])
def test_decode_matches_libjpeg(subsampling, quality):
    img = synth.make_image(203, 117, seed=3 + quality, n_blobs=8, sigma=(5, 40))
    data = pil_jpeg(img, quality, subsampling)
    j = J.parse(data)
    planes = J.reconstruct_planes(j, J.decode_coefficients(j))
    h, w, _ = img.shape
    ref = pil_ycc(data)
    # luma: the inverse DCT against libjpeg's (IEEE 1180: peak error 1)
    d = np.abs(planes[0][:h, :w].astype(np.int64) - ref[..., 0])
    assert d.max() <= 1 and d.mean() < 0.05
    if subsampling == 0:
        for c in (1, 2):
            d = np.abs(planes[c][:h, :w].astype(np.int64) - ref[..., c])
            assert d.max() <= 1 and d.mean() < 0.05
        # the whole decode: one level per stage, times at most 1.772 in colour
        rgb = J.planes_to_rgb(j, planes).astype(np.int64)
        pil = np.asarray(PIL.open(io.BytesIO(data)).convert("RGB")).astype(np.int64)
        assert np.abs(rgb - pil).max() <= 3 and np.abs(rgb - pil).mean() < 0.1


def test_decode_restart_intervals_and_grey():
    img = synth.make_image(150, 71, seed=9, n_blobs=6, sigma=(4, 30))
    plain = pil_jpeg(img, 80, 2)
    rst = pil_jpeg(img, 80, 2, restart_marker_blocks=3)
    assert J.parse(rst).restart == 3 and J.parse(plain).restart == 0
    a = J.decode_coefficients(J.parse(plain))
    b = J.decode_coefficients(J.parse(rst))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # one component
    grey = img[..., 1].copy()
    bio = io.BytesIO()
    PIL.fromarray(grey).save(bio, format="JPEG", quality=85)
    data = bio.getvalue()
    out = J.decode(data)
    ref = np.asarray(PIL.open(io.BytesIO(data))).astype(np.int64)
    assert np.abs(out[..., 0].astype(np.int64) - ref).max() <= 1
    assert np.array_equal(out[..., 0], out[..., 1]) and np.array_equal(out[..., 0], out[..., 2])


def test_rejects_progressive():
    img = synth.make_image(32, 32, seed=1, n_blobs=2, sigma=(3, 9))
    data = pil_jpeg(img, 80, 2, progressive=True)
    with pytest.raises(ValueError):
        J.parse(data)


def test_replication_upsampling():
    # 4:2:0 planes with a distinct value per chroma sample: each covers 2 x 2
    # luma samples, clipped at the image edge
    j = J.Jpeg(width=5, height=3, components=[J.Component(1, 2, 2, 0), J.Component(2, 1, 1, 1),
                                               J.Component(3, 1, 1, 1)])
    y = np.full((16, 16), 100, np.uint8)
    cb = np.full((8, 8), 128, np.uint8)
    cr = (np.arange(64).reshape(8, 8) + 100).astype(np.uint8)
    rgb = J.planes_to_rgb(j, [y, cb, cr])
    assert rgb.shape == (3, 5, 3)
    want_cr = np.array([[100, 100, 101, 101, 102], [100, 100, 101, 101, 102], [108, 108, 109, 109, 110]])
    assert np.array_equal(rgb[..., 0], J.ycc_to_rgb(np.full((3, 5), 100), np.full((3, 5), 128), want_cr)[..., 0])


def test_replication_upsampling_422():
    # 4:2:2 (chroma half width, full height): a chroma sample covers 2 x 1
    j = J.Jpeg(width=5, height=2, components=[J.Component(1, 2, 1, 0), J.Component(2, 1, 1, 1),
                                               J.Component(3, 1, 1, 1)])
    y = np.full((8, 16), 100, np.uint8)
    cb = np.full((8, 8), 128, np.uint8)
    cr = (np.arange(64).reshape(8, 8) + 100).astype(np.uint8)
    rgb = J.planes_to_rgb(j, [y, cb, cr])
    want_cr = np.array([[100, 100, 101, 101, 102], [108, 108, 109, 109, 110]])
    assert np.array_equal(rgb, J.ycc_to_rgb(np.full((2, 5), 100), np.full((2, 5), 128), want_cr))


def test_encode_planes_hand_example():
    # 3 x 2 image, 4:2:0: extended to 16 x 16 by repeating the last column and
    # row; a grey image keeps Y = the grey and Cb = Cr = 128
    img = np.array([[[10, 10, 10], [20, 20, 20], [31, 31, 31]],
                    [[40, 40, 40], [50, 50, 50], [60, 60, 60]]], np.uint8)
    y, cb, cr = J.encode_planes(img, (2, 1, 1), (2, 1, 1))
    assert y.shape == (16, 16) and cb.shape == (8, 8)
    assert list(y[0, :5]) == [10, 20, 31, 31, 31] and list(y[1, :3]) == [40, 50, 60] and list(y[15, :3]) == [40, 50, 60]
    assert (cb == 128).all() and (cr == 128).all()
    # a chroma sample is the mean of its 2 x 2 block, half up: make Cb differ
    img2 = np.zeros((2, 2, 3), np.uint8)
    img2[..., 2] = [[0, 1], [1, 1]]   # blue adds 0.5 per level to Cb
    _, cb2, _ = J.encode_planes(img2, (2, 1, 1), (2, 1, 1))
    full = J.rgb_to_ycc(img2)[1]
    assert cb2[0, 0] == (full.sum() + 2) // 4


def test_quantize_flat_block_closed_form():
    # a flat block of value k: S(0,0) = 8 (k - 128), all else 0
    q = np.arange(1, 65)
    for k in (0, 37, 128, 200, 255):
        qc, ratio, _ = J.quantize_blocks(np.full((8, 8), k, np.int64), q)
        want = np.zeros(64, np.int64)
        want[0] = J.round_half_away(np.array([8.0 * (k - 128) / 1.0]))[0]
        assert np.array_equal(qc[0, 0], want), k


@pytest.mark.parametrize("quality", [50, 90])
def test_forward_path_matches_libjpeg(quality):
    # the luma coefficients libjpeg writes (read back with the oracle's
    # decoder) against the oracle's colour conversion, FDCT and quantization
    # of the same image with the same table: libjpeg's integer FDCT is off by
    # one level now and then; blocks that only pad the MCU grid are left out
    # (libjpeg fills them differently)
    img = synth.make_image(203, 117, seed=30 + quality, n_blobs=8, sigma=(5, 40))
    for ss, hv in ((0, ((1, 1, 1), (1, 1, 1))), (2, ((2, 1, 1), (2, 1, 1)))):
        data = pil_jpeg(img, quality, ss)
        j = J.parse(data)
        coefs = J.decode_coefficients(j)
        planes = J.encode_planes(img, *hv)
        qc, _, _ = J.quantize_blocks(planes[0], j.qtables[j.components[0].tq])
        bw, bh = -(-203 // 8), -(-117 // 8)
        d = np.abs(qc[:bh, :bw] - coefs[0][:bh, :bw])
        assert d.max() <= 1 and (d == 0).mean() > 0.99, (ss, d.max(), (d == 0).mean())
        if ss == 0:
            for c in (1, 2):
                qc, _, _ = J.quantize_blocks(planes[c], j.qtables[j.components[c].tq])
                d = np.abs(qc - coefs[c])
                assert d.max() <= 2 and (d == 0).mean() > 0.99


@pytest.mark.parametrize("ss,restart", [(2, 0), (0, 7), (1, 1)])
def test_split_scans_helper_keeps_coefficients(ss, restart):
    """The test helper that rewrites a file with one scan per component keeps
    every coefficient of each component's own block grid (read back by the
    oracle's decoder, which follows T.81's non-interleaved order)."""
    from jpeg_scans import split_scans
    img = np.random.default_rng(ss).integers(0, 256, (37, 53, 3), dtype=np.uint8)
    data = pil_jpeg(img, 85, ss)
    split = split_scans(data, restart)
    j0, j1 = J.parse(data), J.parse(split)
    assert len(j1.scans) == 3 and j1.restart == restart
    a, b = J.decode_coefficients(j0), J.decode_coefficients(j1)
    _, _, _, _, grids = J.block_grid(j0)
    for c in range(3):
        (_, _), (bw, bh) = grids[c]
        assert np.array_equal(a[c][:bh, :bw], b[c][:bh, :bw])
        assert not b[c][bh:].any() and not b[c][:, bw:].any()
