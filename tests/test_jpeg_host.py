"""Host half of the library's JPEG codec (no GPU): header parsing and
entropy decoding against the JPEG oracle's (every coefficient, bit-exact),
entropy encoding checked by decoding its files with the oracle and with
libjpeg (through PIL), the quality-scaled tables against T.81's Annex K and
libjpeg's, and the error paths."""
import io

import numpy as np
import pytest

import oracle.jpeg_ref as J
from paper_1405_1020_amd import binding as B
from paper_1405_1020_amd import synth

PIL = pytest.importorskip("PIL.Image")


def pil_jpeg(img, quality, subsampling=2, **kw) -> bytes:
    b = io.BytesIO()
    PIL.fromarray(img).save(b, format="JPEG", quality=quality, subsampling=subsampling, **kw)
    return b.getvalue()


def oracle_flat(data: bytes) -> np.ndarray:
    """The oracle's coefficients in the library's layout (components one after
    another, blocks raster order over the MCU-padded grid, natural order)."""
    j = J.parse(data)
    return np.concatenate([c.reshape(-1) for c in J.decode_coefficients(j)])


CASES = [((203, 117), 75, 2, {}), ((203, 117), 90, 0, {}), ((64, 48), 30, 1, {}), ((1, 1), 80, 2, {}),
         ((7, 9), 95, 2, {}), ((33, 17), 100, 0, {}), ((150, 71), 80, 2, {"restart_marker_blocks": 3}),
         ((97, 61), 60, 0, {"restart_marker_rows": 1}), ((16, 16), 5, 2, {})]


@pytest.mark.parametrize("size,quality,ss,kw", CASES)
def test_entropy_decode_matches_oracle(size, quality, ss, kw):
    w, h = size
    img = synth.make_image(w, h, seed=w * 7 + quality, n_blobs=5, sigma=(2, 30))
    data = pil_jpeg(img, quality, ss, **kw)
    info, coef = B.jpeg_coefficients(data)
    j = J.parse(data)
    assert (info.width, info.height, info.components) == (j.width, j.height, len(j.components))
    assert [info.h_samp[c] for c in range(3)] == [c.h for c in j.components]
    assert [info.v_samp[c] for c in range(3)] == [c.v for c in j.components]
    assert info.restart_interval == j.restart
    assert np.array_equal(coef.astype(np.int64), oracle_flat(data))


def test_entropy_decode_grey():
    img = synth.make_image(45, 31, seed=5, n_blobs=4, sigma=(2, 20))[..., 0].copy()
    b = io.BytesIO()
    PIL.fromarray(img).save(b, format="JPEG", quality=70)
    data = b.getvalue()
    info, coef = B.jpeg_coefficients(data)
    assert info.components == 1
    assert np.array_equal(coef.astype(np.int64), oracle_flat(data))


def test_annex_k_tables_and_quality_scaling():
    k1 = [16, 11, 10, 16, 24, 40, 51, 61, 12, 12, 14, 19, 26, 58, 60, 55, 14, 13, 16, 24, 40, 57, 69, 56,
          14, 17, 22, 29, 51, 87, 80, 62, 18, 22, 37, 56, 68, 109, 103, 77, 24, 35, 55, 64, 81, 104, 113, 92,
          49, 64, 78, 87, 103, 121, 120, 101, 72, 92, 95, 98, 112, 100, 103, 99]   # T.81 Table K.1
    k2 = [17, 18, 24, 47] + [99] * 4 + [18, 21, 26, 66] + [99] * 4 + [24, 26, 56] + [99] * 5 + \
         [47, 66] + [99] * 6 + [99] * 32                                              # T.81 Table K.2
    info = B.jpeg_encode_info(16, 16, 50, 0)
    coef = np.zeros(int(info.blocks) * 64, np.int16)
    j = J.parse(B.jpeg_write(coef, 16, 16, 50, 0))
    assert list(j.qtables[0]) == k1 and list(j.qtables[1]) == k2
    # other qualities: the same tables libjpeg makes (PIL reports them in
    # natural order)
    img = synth.make_image(16, 16, seed=1, n_blobs=2, sigma=(2, 5))
    for q in (1, 10, 49, 51, 75, 90, 99, 100):
        ours = J.parse(B.jpeg_write(coef, 16, 16, q, 0)).qtables
        ref = PIL.open(io.BytesIO(pil_jpeg(img, q, 0))).quantization
        assert list(ours[0]) == list(ref[0]) and list(ours[1]) == list(ref[1]), q


@pytest.mark.parametrize("ss", [0, 1, 2])
def test_entropy_encode_round_trip(ss):
    # coefficients the oracle computes for a photo-like image (so that the
    # symbol statistics are realistic), plus blocks with long zero runs,
    # extreme values and every AC position
    img = synth.make_image(77, 45, seed=10 + ss, n_blobs=6, sigma=(2, 25))
    q = 85
    info = B.jpeg_encode_info(77, 45, q, ss)
    hv = ((1, 1, 1), (1, 1, 1)) if ss == 0 else (((2, 1, 1), (1, 1, 1)) if ss == 1 else ((2, 1, 1), (2, 1, 1)))
    probe = J.parse(B.jpeg_write(np.zeros(int(info.blocks) * 64, np.int16), 77, 45, q, ss))
    planes = J.encode_planes(img, *hv)
    parts = [J.quantize_blocks(planes[c], probe.qtables[probe.components[c].tq])[0].reshape(-1) for c in range(3)]
    coef = np.concatenate(parts).astype(np.int16)
    rng = np.random.default_rng(ss)
    blocks = coef.reshape(-1, 64)
    blocks[0] = 0
    blocks[0, 63] = -1023                       # run of 62 zeros (three ZRL) then the last position
    blocks[1] = rng.integers(-1023, 1024, 64)   # no zeros at all
    blocks[2, 0] = 2047                         # DC difference of category 11
    blocks[3, 0] = -2047
    data = B.jpeg_write(coef, 77, 45, q, ss)
    back = oracle_flat(data)
    assert np.array_equal(back, coef.astype(np.int64))
    # libjpeg reads the file too
    out = np.asarray(PIL.open(io.BytesIO(data)).convert("RGB"))
    assert out.shape == (45, 77, 3)


def test_errors():
    img = synth.make_image(32, 32, seed=2, n_blobs=2, sigma=(2, 9))
    prog = pil_jpeg(img, 80, 2, progressive=True)
    with pytest.raises(B.OilpaintError) as e:
        B.jpeg_header(prog)
    assert e.value.status == B.ERR_UNSUPPORTED
    good = pil_jpeg(img, 80, 2)
    for bad in (b"", b"\xff\xd8", good[:len(good) // 2], b"\x00" + good[1:]):
        with pytest.raises(B.OilpaintError) as e:
            B.jpeg_coefficients(bad)
        assert e.value.status == B.ERR_ARG
    with pytest.raises(B.OilpaintError):
        B.jpeg_encode_info(0, 10, 50, 0)
    with pytest.raises(B.OilpaintError):
        B.jpeg_encode_info(10, 10, 0, 0)
    with pytest.raises(B.OilpaintError):
        B.jpeg_encode_info(10, 10, 50, 3)


@pytest.mark.parametrize("ss,restart", [(2, 0), (0, 7), (1, 1)])
def test_entropy_decode_per_component_scans(ss, restart):
    """The host decoder on files with one scan per component (T.81 A.2.2),
    written by the test helper, against the oracle's decoder."""
    from jpeg_scans import split_scans
    img = synth.make_image(71, 45, seed=ss, n_blobs=4, sigma=(2, 20))
    data = split_scans(pil_jpeg(img, 85, ss), restart)
    info, coef = B.jpeg_coefficients(data)
    j = J.parse(data)
    want = J.decode_coefficients(j)
    for c in range(3):
        first, bw, bh = info.first_block[c], info.blocks_w[c], info.blocks_h[c]
        got = coef.reshape(-1, 64)[first:first + bw * bh].reshape(bh, bw, 64)
        assert np.array_equal(got, want[c])
