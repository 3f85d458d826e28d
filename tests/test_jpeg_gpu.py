"""GPU parity of the JPEG steps either side of the filter, through the C-ABI,
against the JPEG oracle (oracle/jpeg_ref.py: T.81 and JFIF in fp64 and exact
integers).

Tolerance.  Colour conversion is integer arithmetic on both sides: bit-exact.
The inverse and forward DCTs run in fp32 on the GPU: every sample (or
quantized coefficient) must equal the oracle's, except where the oracle's
exact value lies within the fp32 error bound of a rounding boundary (half an
integer), where it may differ by one.  The bound is 2^-17 x the block's sum
of |dequantized coefficients| (inverse) or of |sample - 128| (forward, divided
by the quantizer), with 2^-20 of the value itself for the division: two
passes of eight fp32 multiply-adds over basis entries below 1 each round at
most 2^-24 relative per step, which this exceeds several times over."""
import io

import numpy as np
import pytest

import oracle
import oracle.jpeg_ref as J
from paper_1405_1020_amd import binding as B
from paper_1405_1020_amd import synth
from gpu_util import torch_mod
from jpeg_scans import split_scans

pytestmark = pytest.mark.gpu
PIL = pytest.importorskip("PIL.Image")

HV = {0: ((1, 1, 1), (1, 1, 1)), 1: ((2, 1, 1), (1, 1, 1)), 2: ((2, 1, 1), (2, 1, 1))}


def pil_jpeg(img, quality, subsampling=2, **kw) -> bytes:
    b = io.BytesIO()
    PIL.fromarray(img).save(b, format="JPEG", quality=quality, subsampling=subsampling, **kw)
    return b.getvalue()


def near_half(v: np.ndarray, window: np.ndarray) -> np.ndarray:
    f = v - np.floor(v)
    return np.abs(f - 0.5) < window


def check_planes(data: bytes, planes_gpu, coefs=None) -> int:
    """Every sample of every component against the oracle (its inverse DCT
    of `coefs`, by default its own decoding of the file's coefficients);
    returns how many sat within the fp32 bound of a rounding boundary."""
    j = J.parse(data)
    if coefs is None:
        coefs = J.decode_coefficients(j)
    want = J.reconstruct_planes(j, coefs)
    vals, sums = J.idct_values(j, coefs)
    flagged = 0
    for c, p in enumerate(planes_gpu):
        got = p.cpu().numpy().astype(np.int64)
        h, w = got.shape
        ref = want[c][:h, :w].astype(np.int64)
        win = np.repeat(np.repeat(sums[c], 8, 0), 8, 1)[:h, :w] * 2.0 ** -17
        tie = near_half(vals[c][:h, :w], win)
        d = np.abs(got - ref)
        assert d.max() <= 1, (c, int(d.max()))
        bad = (d != 0) & ~tie
        assert not bad.any(), (c, np.argwhere(bad)[:5].tolist())
        flagged += int(tie.sum())
    return flagged


CASES = [((203, 117), 75, 2, {}), ((203, 117), 95, 0, {}), ((64, 48), 30, 1, {}), ((1, 1), 80, 2, {}),
         ((7, 9), 100, 2, {}), ((150, 71), 80, 2, {"restart_marker_blocks": 3}), ((640, 480), 90, 2, {})]


@pytest.mark.parametrize("size,quality,ss,kw", CASES)
def test_decode_matches_oracle(size, quality, ss, kw):
    torch = torch_mod()
    w, h = size
    img = synth.make_image(w, h, seed=w + quality, n_blobs=6, sigma=(2, 40))
    data = pil_jpeg(img, quality, ss, **kw)
    planes = B.jpeg_decode_planes(data)
    rgb = B.jpeg_decode(data)
    torch.cuda.synchronize()
    check_planes(data, planes)
    # colour: exact integers, applied by the oracle to the GPU's own planes
    j = J.parse(data)
    want = J.planes_to_rgb(j, [p.cpu().numpy() for p in planes])
    assert np.array_equal(rgb.cpu().numpy(), want)


def test_decode_grey_and_strided_output():
    torch = torch_mod()
    img = synth.make_image(97, 53, seed=4, n_blobs=4, sigma=(2, 20))[..., 2].copy()
    b = io.BytesIO()
    PIL.fromarray(img).save(b, format="JPEG", quality=85)
    data = b.getvalue()
    planes = B.jpeg_decode_planes(data)
    check_planes(data, planes)
    buf = torch.full((53, 97 * 3 + 5), 77, dtype=torch.uint8, device="cuda")
    view = buf[:, :97 * 3].view(53, 97, 3)
    B.jpeg_decode(data, out=view)
    torch.cuda.synchronize()
    y = planes[0].cpu().numpy()
    got = buf.cpu().numpy()
    assert np.array_equal(got[:, :97 * 3].reshape(53, 97, 3), np.stack([y, y, y], -1))
    assert (got[:, 97 * 3:] == 77).all()


def test_decode_full_hd():
    torch = torch_mod()
    img = synth.fhd_image()
    data = pil_jpeg(img, 90, 2)
    planes = B.jpeg_decode_planes(data)
    rgb = B.jpeg_decode(data)
    torch.cuda.synchronize()
    check_planes(data, planes)
    want = J.planes_to_rgb(J.parse(data), [p.cpu().numpy() for p in planes])
    assert np.array_equal(rgb.cpu().numpy(), want)


@pytest.mark.parametrize("ss,restart", [(2, 0), (0, 7), (1, 1)])
def test_decode_per_component_scans(ss, restart):
    """Files with one scan per component (blocks over each component's own
    grid), with and without restart intervals."""
    torch = torch_mod()
    img = synth.make_image(203, 117, seed=11 + ss, n_blobs=6, sigma=(2, 40))
    data = split_scans(pil_jpeg(img, 85, ss), restart)
    assert len(J.parse(data).scans) == 3
    planes = B.jpeg_decode_planes(data)
    torch.cuda.synchronize()
    check_planes(data, planes)


def test_decode_any_subsequence_length():
    """The device decoder gives the same samples whatever the subsequences'
    length, 64 bits (many subsequences and links, a short checkpoint) to
    16384, and with the length chosen per scan; interleaved, restart-marked and per-component files, and noise at
    quality 100 (long codes, stuffed bytes, few end-of-block codes, so that
    tracks rarely meet the true decoding and the host decodes many
    subsequences itself)."""
    torch = torch_mod()
    img = synth.make_image(640, 480, seed=21, n_blobs=12, sigma=(2, 60))
    noise = np.random.default_rng(8).integers(0, 256, (96, 160, 3), dtype=np.uint8)
    files = [pil_jpeg(img, 90, 2), pil_jpeg(img, 75, 0, restart_marker_blocks=5),
             split_scans(pil_jpeg(img[:200, :300].copy(), 80, 1), 9), pil_jpeg(noise, 100, 0)]
    ref = [[p.cpu().numpy() for p in B.jpeg_decode_planes(f)] for f in files]
    check_planes(files[1], [torch.from_numpy(p) for p in ref[1]])
    check_planes(files[3], [torch.from_numpy(p) for p in ref[3]])
    try:
        for bits in (64, 100, 333, 4096, 16384, 0):
            B.jpeg_set_subsequence_bits(bits)
            for f, r in zip(files, ref):
                got = [p.cpu().numpy() for p in B.jpeg_decode_planes(f)]
                assert all(np.array_equal(a, b) for a, b in zip(got, r)), bits
    finally:
        B.jpeg_set_subsequence_bits(0)
    with pytest.raises(B.OilpaintError):
        B.jpeg_set_subsequence_bits(63)


def test_decode_corrupt_streams_as_host_decoder():
    """Bits flipped in the entropy-coded data: the device decoder reports a
    malformed stream (ERR_ARG) exactly when the library's host decoder does,
    and otherwise decodes the host decoder's coefficients (the oracle's
    inverse DCT of them gives its samples)."""
    torch = torch_mod()
    img = synth.make_image(160, 120, seed=31, n_blobs=6, sigma=(2, 40))
    data = pil_jpeg(img, 80, 2, restart_marker_blocks=4)
    begin = data.index(b"\xff\xda") + 2 + (data[data.index(b"\xff\xda") + 2] << 8 | data[data.index(b"\xff\xda") + 3])
    end = len(data) - 2
    rng = np.random.default_rng(5)
    outcomes = set()
    cases = []
    for trial in range(24):
        b = bytearray(data)
        while True:
            pos = int(rng.integers(begin + 1, end - 1))
            new = b[pos] ^ (1 << int(rng.integers(0, 8)))
            if 0xFF not in (b[pos - 1], b[pos], new):
                break
        b[pos] = new
        cases.append(bytes(b))
    # 64 one bits (stuffed 0xFF bytes) in the middle of the data: no code is
    # all ones (T.81 C), so both decoders must stop there
    mid = (begin + end) // 2
    while 0xFF in data[mid - 1:mid + 1]:
        mid += 1
    cases.append(data[:mid] + b"\xff\x00" * 8 + data[mid:])
    B.jpeg_set_subsequence_bits(64)
    try:
        for trial, bad in enumerate(cases):
            try:
                B.jpeg_coefficients(bad)
                host_ok = True
            except B.OilpaintError as e:
                assert e.status == B.ERR_ARG
                host_ok = False
            try:
                planes = B.jpeg_decode_planes(bad)
                torch.cuda.synchronize()
                dev_ok = True
            except B.OilpaintError as e:
                assert e.status == B.ERR_ARG
                dev_ok = False
            assert host_ok == dev_ok, trial
            if dev_ok:
                # the oracle's decoder stops at a marker where the library
                # reads zero bits (an interval whose data runs short), so
                # the coefficients here are the host decoder's
                info, coef = B.jpeg_coefficients(bad)
                coefs = [coef.reshape(-1, 64)[info.first_block[c]:info.first_block[c] + info.blocks_w[c] *
                                               info.blocks_h[c]].reshape(info.blocks_h[c], info.blocks_w[c], 64)
                         .astype(np.int64) for c in range(info.components)]
                check_planes(bad, planes, coefs)
            outcomes.add(dev_ok)
    finally:
        B.jpeg_set_subsequence_bits(0)
    assert outcomes == {True, False}


@pytest.mark.parametrize("restart,bits", [(0, 64), (0, 0), (3, 0)])
def test_decode_shifted_streams_as_host_decoder(restart, bits):
    """A byte deleted from or repeated in the entropy-coded data shifts
    every later code: the device's tracks, links and host walk must still
    find the same decoding as the library's host decoder (status and every
    coefficient), whatever the subsequence length and restart intervals."""
    torch = torch_mod()
    img = synth.make_image(176, 96, seed=37, n_blobs=6, sigma=(2, 40))
    kw = {"restart_marker_blocks": restart} if restart else {}
    data = pil_jpeg(img, 85, 2, **kw)
    sos = data.index(b"\xff\xda")
    begin = sos + 2 + (data[sos + 2] << 8 | data[sos + 3])
    end = len(data) - 2
    rng = np.random.default_rng(11 + restart + bits)
    cases = []
    while len(cases) < 12:
        pos = int(rng.integers(begin + 2, end - 2))
        if 0xFF in data[pos - 1:pos + 2]:
            continue
        b = bytearray(data)
        if len(cases) % 2:
            del b[pos]
        else:
            b.insert(pos, b[pos])
        cases.append(bytes(b))
    B.jpeg_set_subsequence_bits(bits)
    try:
        for trial, bad in enumerate(cases):
            try:
                info, coef = B.jpeg_coefficients(bad)
                host_ok = True
            except B.OilpaintError as e:
                assert e.status == B.ERR_ARG
                host_ok = False
            try:
                planes = B.jpeg_decode_planes(bad)
                torch.cuda.synchronize()
                dev_ok = True
            except B.OilpaintError as e:
                assert e.status == B.ERR_ARG
                dev_ok = False
            assert host_ok == dev_ok, trial
            if dev_ok:
                coefs = [coef.reshape(-1, 64)[info.first_block[c]:info.first_block[c] + info.blocks_w[c] *
                                               info.blocks_h[c]].reshape(info.blocks_h[c], info.blocks_w[c], 64)
                         .astype(np.int64) for c in range(info.components)]
                check_planes(bad, planes, coefs)
    finally:
        B.jpeg_set_subsequence_bits(0)


def check_encoded(img: np.ndarray, data: bytes, quality: int, ss: int) -> int:
    """The file's quantized coefficients (read with the oracle's decoder)
    against the oracle's colour, chroma averaging, FDCT and quantization of
    the source with the file's tables; returns the near-boundary count."""
    j = J.parse(data)
    assert (j.width, j.height) == (img.shape[1], img.shape[0])
    h, v = HV[ss]
    assert [c.h for c in j.components] == list(h) and [c.v for c in j.components] == list(v)
    coefs = J.decode_coefficients(j)
    planes = J.encode_planes(img, h, v)
    flagged = 0
    for c in range(3):
        q = j.qtables[j.components[c].tq]
        qc, ratio, sums = J.quantize_blocks(planes[c], q)
        win = sums[..., None] * 2.0 ** -17 / q[None, None, :] + np.abs(ratio) * 2.0 ** -20
        tie = near_half(np.abs(ratio), win)
        d = np.abs(qc - coefs[c])
        assert d.max() <= 1, (c, int(d.max()))
        assert not ((d != 0) & ~tie).any(), c
        flagged += int(tie.sum())
    return flagged


@pytest.mark.parametrize("size,quality,ss", [((203, 117), 75, 2), ((203, 117), 95, 0), ((64, 48), 30, 1),
                                             ((1, 1), 80, 2), ((7, 9), 100, 2), ((33, 17), 50, 1),
                                             ((640, 480), 90, 2)])
def test_encode_matches_oracle(size, quality, ss):
    torch = torch_mod()
    w, h = size
    img = synth.make_image(w, h, seed=3 * w + quality, n_blobs=6, sigma=(2, 40))
    src = torch.from_numpy(img).cuda()
    data = B.jpeg_encode(src, quality=quality, subsampling=ss)
    check_encoded(img, data, quality, ss)
    # libjpeg reads it, and it is close to the source
    out = np.asarray(PIL.open(io.BytesIO(data)).convert("RGB")).astype(np.int64)
    assert out.shape == img.shape
    if quality >= 90 and w * h > 100:
        assert np.abs(out - img).mean() < 3.0


@pytest.mark.parametrize("size,quality,ss,noise", [((203, 117), 75, 2, False), ((64, 48), 30, 1, False),
                                                   ((1, 1), 80, 2, False), ((7, 9), 100, 0, True),
                                                   ((640, 480), 100, 0, True), ((1920, 1080), 90, 2, False)])
def test_device_coder_matches_host_coder(size, quality, ss, noise):
    """The device's Huffman coding (statistics, code sizes, bit placement,
    byte stuffing) against the library's host coder on the same quantized
    coefficients: the files are the same bytes.  Noise at quality 100 fills
    the stream with 0xFF bytes (about one in 256) and long codes; 1920x1080
    spans many prefix-sum tiles of blocks and of bytes."""
    torch = torch_mod()
    w, h = size
    if noise:
        img = np.random.default_rng(w * h).integers(0, 256, (h, w, 3), dtype=np.uint8)
    else:
        img = synth.make_image(w, h, seed=5 * w + quality, n_blobs=6, sigma=(2, 40))
    data = B.jpeg_encode(torch.from_numpy(img).cuda(), quality=quality, subsampling=ss)
    _, coef = B.jpeg_coefficients(data)
    assert data == B.jpeg_write(coef, w, h, quality, ss)
    if noise and w * h > 1000:
        scan = data[data.index(b"\xff\xda"):]
        assert scan.count(b"\xff\x00") > 100
    check_encoded(img, data, quality, ss)


def test_encode_capacity():
    """An output of exactly the file's length, or more, receives the same
    file; one byte short is ERR_NOMEM with the output untouched."""
    import ctypes
    torch = torch_mod()
    img = np.random.default_rng(3).integers(0, 256, (96, 160, 3), dtype=np.uint8)
    src = torch.from_numpy(img).cuda()
    want = B.jpeg_encode(src, quality=100, subsampling=0)
    n = len(want)
    w, h, s = B.image_geometry(src)
    got = ctypes.c_size_t(0)
    for cap in (n, n + 1, 2 * n):
        buf = (ctypes.c_uint8 * cap)()
        st = B.lib().oilpaint_jpeg_encode(src.data_ptr(), w, h, s, 100, 0, buf, cap, ctypes.byref(got), None, None)
        assert st == B.OK and got.value == n and bytes(buf)[:n] == want, cap
    buf = (ctypes.c_uint8 * (n - 1))(*([7] * (n - 1)))
    st = B.lib().oilpaint_jpeg_encode(src.data_ptr(), w, h, s, 100, 0, buf, n - 1, ctypes.byref(got), None, None)
    assert st == B.ERR_NOMEM and got.value == n and bytes(buf) == bytes([7] * (n - 1))


def test_file_driver_decode_filter_encode():
    """The paper's program shape: a JPEG file decoded onto the device, the oil
    paint filter run there, the result encoded: the decoded image against
    the oracle (as above), the filtered one against the filter's oracle on
    those decoded pixels (bit-exact), the file against the oracle encoder."""
    torch = torch_mod()
    img = synth.make_image(320, 240, seed=77, n_blobs=10, sigma=(5, 60))
    data = pil_jpeg(img, 90, 2)
    dec = B.jpeg_decode(data)
    planes = B.jpeg_decode_planes(data)
    out = B.oilpaint(dec, 3, 20)
    enc = B.jpeg_encode(out, quality=90, subsampling=2)
    torch.cuda.synchronize()
    check_planes(data, planes)
    decoded = dec.cpu().numpy()
    filtered = out.cpu().numpy()
    assert np.array_equal(filtered, oracle.oilpaint_ref(decoded, 3, 20, nthreads=4))
    check_encoded(filtered, enc, 90, 2)


def test_encode_errors():
    torch = torch_mod()
    src = torch.zeros((10, 10, 3), dtype=torch.uint8, device="cuda")
    for q, ss in ((0, 2), (101, 2), (50, 3), (50, -1)):
        with pytest.raises(B.OilpaintError) as e:
            B.jpeg_encode(src, quality=q, subsampling=ss)
        assert e.value.status == B.ERR_ARG
    host = torch.zeros((10, 10, 3), dtype=torch.uint8)
    data = pil_jpeg(np.zeros((10, 10, 3), np.uint8), 80)
    assert B.lib().oilpaint_jpeg_decode(data, len(data), host.data_ptr(), 30, None, None) == B.ERR_NOT_DEVICE
    assert B.lib().oilpaint_jpeg_decode(data, len(data), src.data_ptr(), 29, None, None) == B.ERR_ARG
