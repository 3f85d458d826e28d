"""CPU oracle for the JPEG steps either side of the filter: baseline
sequential DCT-based JPEG (Huffman coding, 8-bit samples) as ITU-T T.81
(ISO/IEC 10918-1) defines it, with JFIF's YCbCr colour space.

TEST INFRASTRUCTURE ONLY.  Only the test suite and the benchmark's CPU legs may
import this module.  It shares no code, table or constant with the GPU library:
every table here (zig-zag order, DCT basis, Huffman decoding tables) is built
from the standard's definitions in this file.

The paper's program decodes a JPEG file, runs the filter on the pixel buffer
and encodes the result (its Section 3 file driver with the decoder and encoder
listings); the codec itself it leaves to the operating system's imaging
library.  What is computed here:

  * marker syntax (T.81 Annex B): SOI, APPn/COM (skipped), DQT, DHT, SOF0 /
    SOF1 (8-bit, Huffman, sequential), DRI, SOS, RSTn, EOI;
  * Huffman table generation (Annex C: the size and code tables from BITS and
    HUFFVAL) and the decoder tables MINCODE, MAXCODE, VALPTR (F.2.2.3);
  * entropy decoding (F.2.2): DECODE, RECEIVE, EXTEND; DC prediction per
    component (F.1.2.1), reset at each restart interval; AC run/size symbols
    with ZRL and EOB (F.1.2.2); stuffed zero bytes after 0xFF (F.1.2.3);
  * block order (A.2): non-interleaved scans in raster order over the
    component's own blocks, interleaved scans MCU by MCU, each component's
    H x V blocks in raster order inside the MCU;
  * the zig-zag order of Figure A.6;
  * dequantization R = Sq x Q (A.3.5) and the 8 x 8 inverse DCT (A.3.3),
    level shift +128 (A.3.1), each sample rounded half up and clamped to
    [0, 255];
  * forward DCT (A.3.3) of samples - 128 and quantization (A.3.4), rounded
    to the nearest integer, half away from zero;
  * JFIF YCbCr <-> RGB with JFIF's decimal coefficients, evaluated exactly
    (integers scaled by 10^3 or 10^6) and rounded half up, clamped;
  * chroma resampling, which neither document fixes: on decode every chroma
    sample covers its Hmax/H x Vmax/V luma samples (replication); on encode
    the image is first extended to whole MCUs by repeating its last column
    and row (A.2.4), then each chroma sample is the mean of the luma-grid
    samples it covers, rounded half up.

Floating point (the DCT pair) is fp64.  A reconstructed value whose exact
value is a half-integer is rounded up; fp64 puts such values within 1e-9 of
the half-integer (these sums stay below 2^16 in magnitude, so their fp64
error is far smaller), and values that close are taken as the tie.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TIE_EPS = 1e-9


# ---------------------------------------------------------------------------
# Zig-zag order (T.81 Figure A.6): anti-diagonals u + v = s in turn, odd s
# walked from the top row down, even s from the bottom up.  ZIGZAG[k] is the
# natural (row-major, row = vertical frequency) index of the k-th coefficient.
# ---------------------------------------------------------------------------
def _zigzag() -> list[int]:
    out = []
    for s in range(15):
        rows = range(0, s + 1) if s % 2 == 1 else range(s, -1, -1)
        for r in rows:
            c = s - r
            if r < 8 and c < 8:
                out.append(r * 8 + c)
    return out


ZIGZAG = _zigzag()


# ---------------------------------------------------------------------------
# The DCT pair of A.3.3 as 8 x 8 matrices: A[u][x] = C(u)/2 cos((2x+1) u pi/16)
# with C(0) = 1/sqrt(2), C(u) = 1 otherwise; then
#   S(v,u) = sum_y sum_x A[v][y] s(y,x) A[u][x]     (FDCT:  S = A s A^T)
#   s(y,x) = sum_v sum_u A[v][y] S(v,u) A[u][x]     (IDCT:  s = A^T S A)
# ---------------------------------------------------------------------------
def dct_matrix() -> np.ndarray:
    a = np.zeros((8, 8))
    for u in range(8):
        cu = 1.0 / math.sqrt(2.0) if u == 0 else 1.0
        for x in range(8):
            a[u, x] = cu / 2.0 * math.cos((2 * x + 1) * u * math.pi / 16.0)
    return a


_A = dct_matrix()


def fdct(block: np.ndarray) -> np.ndarray:
    """8 x 8 forward DCT (A.3.3) of level-shifted samples, fp64."""
    return _A @ np.asarray(block, dtype=np.float64) @ _A.T


def idct(coef: np.ndarray) -> np.ndarray:
    """8 x 8 inverse DCT (A.3.3) of dequantized coefficients S[v][u], fp64."""
    return _A.T @ np.asarray(coef, dtype=np.float64) @ _A


def round_half_up(v: np.ndarray) -> np.ndarray:
    """floor(v + 1/2), with values within TIE_EPS of a half-integer taken as
    the half-integer."""
    v = np.asarray(v, dtype=np.float64)
    f = np.floor(v)
    frac = v - f
    tie = np.abs(frac - 0.5) < TIE_EPS
    return np.where(tie, f + 1, np.floor(v + 0.5)).astype(np.int64)


def round_half_away(v: np.ndarray) -> np.ndarray:
    """Nearest integer, halves away from zero (ties as in round_half_up)."""
    v = np.asarray(v, dtype=np.float64)
    return np.sign(v).astype(np.int64) * round_half_up(np.abs(v))


# ---------------------------------------------------------------------------
# Colour (JFIF): exact decimal coefficients, rounded half up, clamped.
# ---------------------------------------------------------------------------
def _clamp8(v):
    return np.clip(v, 0, 255).astype(np.uint8)


def ycc_to_rgb(y, cb, cr) -> np.ndarray:
    """R = Y + 1.402 (Cr-128); G = Y - 0.344136 (Cb-128) - 0.714136 (Cr-128);
    B = Y + 1.772 (Cb-128); each rounded half up and clamped.  Integer
    arrays of equal shape in, [.., 3] uint8 out."""
    y = np.asarray(y, np.int64)
    cb = np.asarray(cb, np.int64) - 128
    cr = np.asarray(cr, np.int64) - 128
    m = 1_000_000
    r = y + (1_402_000 * cr + m // 2) // m
    g = y + (-344_136 * cb - 714_136 * cr + m // 2) // m
    b = y + (1_772_000 * cb + m // 2) // m
    return np.stack([_clamp8(r), _clamp8(g), _clamp8(b)], axis=-1)


def rgb_to_ycc(rgb) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Y = 0.299 R + 0.587 G + 0.114 B; Cb = -0.168736 R - 0.331264 G + 0.5 B
    + 128; Cr = 0.5 R - 0.418688 G - 0.081312 B + 128; rounded half up and
    clamped."""
    rgb = np.asarray(rgb, np.int64)
    r, g, b = rgb[..., 0], rgb[..., 1], rgb[..., 2]
    m = 1_000_000
    y = (299_000 * r + 587_000 * g + 114_000 * b + m // 2) // m
    cb = (-168_736 * r - 331_264 * g + 500_000 * b + 128 * m + m // 2) // m
    cr = (500_000 * r - 418_688 * g - 81_312 * b + 128 * m + m // 2) // m
    return _clamp8(y).astype(np.int64), _clamp8(cb).astype(np.int64), _clamp8(cr).astype(np.int64)


# ---------------------------------------------------------------------------
# Marker syntax (Annex B)
# ---------------------------------------------------------------------------
@dataclass
class Component:
    cid: int
    h: int
    v: int
    tq: int


@dataclass
class Scan:
    comps: list            # [(component index, td, ta)]
    data: bytes            # entropy-coded segment(s), markers included


@dataclass
class Jpeg:
    width: int = 0
    height: int = 0
    components: list = field(default_factory=list)
    qtables: dict = field(default_factory=dict)    # id -> natural-order int array of 64
    htables: dict = field(default_factory=dict)    # (class, id) -> (bits[16], vals)
    restart: int = 0
    scans: list = field(default_factory=list)      # Scan, each with the tables in force
    scan_tables: list = field(default_factory=list)


def parse(data: bytes) -> Jpeg:
    """Split a JPEG stream into its tables, frame and scans."""
    if data[:2] != b"\xff\xd8":
        raise ValueError("no SOI")
    j = Jpeg()
    i = 2
    frame_seen = False
    while i < len(data):
        if data[i] != 0xFF:
            raise ValueError("marker expected at %d" % i)
        while data[i] == 0xFF:
            i += 1
        m = data[i]
        i += 1
        if m == 0xD9:  # EOI
            break
        seg_len = data[i] << 8 | data[i + 1]
        seg = data[i + 2:i + seg_len]
        i += seg_len
        if m == 0xDB:  # DQT
            k = 0
            while k < len(seg):
                pq, tq = seg[k] >> 4, seg[k] & 15
                k += 1
                n = 2 if pq else 1
                zz = [int.from_bytes(seg[k + n * t:k + n * t + n], "big") for t in range(64)]
                k += 64 * n
                nat = np.zeros(64, np.int64)
                for t in range(64):
                    nat[ZIGZAG[t]] = zz[t]
                j.qtables[tq] = nat
        elif m == 0xC4:  # DHT
            k = 0
            while k < len(seg):
                tc, th = seg[k] >> 4, seg[k] & 15
                bits = list(seg[k + 1:k + 17])
                nvals = sum(bits)
                vals = list(seg[k + 17:k + 17 + nvals])
                j.htables[(tc, th)] = (bits, vals)
                k += 17 + nvals
        elif m in (0xC0, 0xC1):  # SOF0 / SOF1: sequential, Huffman
            if seg[0] != 8:
                raise ValueError("only 8-bit samples")
            j.height = seg[1] << 8 | seg[2]
            j.width = seg[3] << 8 | seg[4]
            nc = seg[5]
            j.components = [Component(seg[6 + 3 * c], seg[7 + 3 * c] >> 4, seg[7 + 3 * c] & 15, seg[8 + 3 * c])
                            for c in range(nc)]
            frame_seen = True
        elif 0xC2 <= m <= 0xCF and m not in (0xC4, 0xC8, 0xCC):
            raise ValueError("frame type 0x%02X is not baseline/extended sequential Huffman" % m)
        elif m == 0xDD:  # DRI
            j.restart = seg[0] << 8 | seg[1]
        elif m == 0xDA:  # SOS: the entropy-coded data follows up to the next non-RST marker
            if not frame_seen:
                raise ValueError("SOS before SOF")
            ns = seg[0]
            ids = [c.cid for c in j.components]
            comps = [(ids.index(seg[1 + 2 * k]), seg[2 + 2 * k] >> 4, seg[2 + 2 * k] & 15) for k in range(ns)]
            start = i
            while True:
                if i + 1 >= len(data):
                    raise ValueError("unterminated scan")
                if data[i] == 0xFF and data[i + 1] != 0 and not (0xD0 <= data[i + 1] <= 0xD7):
                    break
                i += 1
            j.scans.append(Scan(comps, data[start:i]))
            j.scan_tables.append(dict(j.htables))
        # APPn, COM and anything else: skipped
    return j


# ---------------------------------------------------------------------------
# Huffman decoding (Annex C, F.2.2)
# ---------------------------------------------------------------------------
class HuffDecoder:
    """MAXCODE, MINCODE, VALPTR from BITS and HUFFVAL (C.2, F.2.2.3)."""

    def __init__(self, bits, vals):
        huffsize = [l + 1 for l in range(16) for _ in range(bits[l])]
        huffcode = []
        code = 0
        si = huffsize[0] if huffsize else 0
        k = 0
        while k < len(huffsize):
            while k < len(huffsize) and huffsize[k] == si:
                huffcode.append(code)
                code += 1
                k += 1
            code <<= 1
            si += 1
        self.vals = list(vals)
        self.maxcode = [-1] * 17
        self.mincode = [0] * 17
        self.valptr = [0] * 17
        j = 0
        for l in range(1, 17):
            if bits[l - 1] == 0:
                self.maxcode[l] = -1
                continue
            self.valptr[l] = j
            self.mincode[l] = huffcode[j]
            j += bits[l - 1]
            self.maxcode[l] = huffcode[j - 1]


class BitReader:
    """NEXTBIT over an entropy-coded segment: a 0x00 after 0xFF is a stuffed
    byte; RSTn markers are met only at interval boundaries (restart())."""

    def __init__(self, data: bytes):
        self.d = data
        self.i = 0
        self.cnt = 0
        self.b = 0

    def bit(self) -> int:
        if self.cnt == 0:
            b = self.d[self.i] if self.i < len(self.d) else 0
            self.i += 1
            if b == 0xFF:
                nxt = self.d[self.i] if self.i < len(self.d) else 0
                if nxt == 0:
                    self.i += 1
                else:
                    raise ValueError("marker inside an interval")
            self.b = b
            self.cnt = 8
        self.cnt -= 1
        return (self.b >> self.cnt) & 1

    def restart(self):
        """Drop the remaining bits of the byte and skip the RSTn marker."""
        self.cnt = 0
        while self.i + 1 < len(self.d) and not (self.d[self.i] == 0xFF and 0xD0 <= self.d[self.i + 1] <= 0xD7):
            self.i += 1
        self.i += 2

    def decode(self, t: HuffDecoder) -> int:
        code = self.bit()
        l = 1
        while code > t.maxcode[l]:
            code = (code << 1) | self.bit()
            l += 1
            if l > 16:
                raise ValueError("bad Huffman code")
        return t.vals[t.valptr[l] + code - t.mincode[l]]

    def receive(self, s: int) -> int:
        v = 0
        for _ in range(s):
            v = (v << 1) | self.bit()
        return v


def extend(v: int, t: int) -> int:
    return v - (1 << t) + 1 if t and v < (1 << (t - 1)) else v


def block_grid(j: Jpeg):
    """(Hmax, Vmax, MCUs across, MCUs down, per component (blocks across,
    blocks down) of the MCU-padded grid, (blocks across, down) of its own
    samples)."""
    hmax = max(c.h for c in j.components)
    vmax = max(c.v for c in j.components)
    mx = -(-j.width // (8 * hmax))
    my = -(-j.height // (8 * vmax))
    grids = []
    for c in j.components:
        xc = -(-j.width * c.h // hmax)
        yc = -(-j.height * c.v // vmax)
        grids.append(((mx * c.h, my * c.v), (-(-xc // 8), -(-yc // 8))))
    return hmax, vmax, mx, my, grids


def decode_coefficients(j: Jpeg) -> list[np.ndarray]:
    """Quantized coefficients per component, [blocks down, blocks across, 64]
    in NATURAL order over the MCU-padded grid (blocks a scan does not cover
    stay 0)."""
    hmax, vmax, mx, my, grids = block_grid(j)
    out = [np.zeros((g[0][1], g[0][0], 64), np.int64) for g in grids]
    for scan, tables in zip(j.scans, j.scan_tables):
        br = BitReader(scan.data)
        dcs = {ci: HuffDecoder(*tables[(0, td)]) for ci, td, _ in scan.comps}
        acs = {ci: HuffDecoder(*tables[(1, ta)]) for ci, _, ta in scan.comps}
        pred = {ci: 0 for ci, _, _ in scan.comps}

        def block(ci, by, bx):
            t = br.decode(dcs[ci])
            pred[ci] += extend(br.receive(t), t)
            zz = [0] * 64
            zz[0] = pred[ci]
            k = 1
            while k < 64:
                rs = br.decode(acs[ci])
                r, s = rs >> 4, rs & 15
                if s == 0:
                    if r == 15:
                        k += 16
                        continue
                    break
                k += r
                zz[k] = extend(br.receive(s), s)
                k += 1
            nat = out[ci][by, bx]
            for t in range(64):
                nat[ZIGZAG[t]] = zz[t]

        if len(scan.comps) == 1:
            ci = scan.comps[0][0]
            (_, _), (bw, bh) = grids[ci]
            units = [(by, bx) for by in range(bh) for bx in range(bw)]
            for n, (by, bx) in enumerate(units):
                if j.restart and n and n % j.restart == 0:
                    br.restart()
                    pred = {c: 0 for c in pred}
                block(ci, by, bx)
        else:
            n = 0
            for my_ in range(my):
                for mx_ in range(mx):
                    if j.restart and n and n % j.restart == 0:
                        br.restart()
                        pred = {c: 0 for c in pred}
                    for ci, _, _ in scan.comps:
                        c = j.components[ci]
                        for v in range(c.v):
                            for h in range(c.h):
                                block(ci, my_ * c.v + v, mx_ * c.h + h)
                    n += 1
    return out


def reconstruct_planes(j: Jpeg, coefs: list[np.ndarray]) -> list[np.ndarray]:
    """Dequantize, inverse DCT, level shift, round half up and clamp: one
    uint8 plane per component over its MCU-padded block grid."""
    planes = []
    for ci, c in enumerate(j.components):
        q = j.qtables[c.tq]
        bh, bw, _ = coefs[ci].shape
        plane = np.zeros((bh * 8, bw * 8), np.uint8)
        for by in range(bh):
            for bx in range(bw):
                s = idct((coefs[ci][by, bx] * q).reshape(8, 8)) + 128.0
                plane[by * 8:by * 8 + 8, bx * 8:bx * 8 + 8] = np.clip(round_half_up(s), 0, 255)
        planes.append(plane)
    return planes


def idct_values(j: Jpeg, coefs: list[np.ndarray]) -> list[np.ndarray]:
    """The level-shifted inverse DCT values before rounding (fp64), and per
    block sum |S| of the dequantized coefficients: [planes], [sums]."""
    vals, sums = [], []
    for ci, c in enumerate(j.components):
        q = j.qtables[c.tq]
        bh, bw, _ = coefs[ci].shape
        v = np.zeros((bh * 8, bw * 8))
        sm = np.zeros((bh, bw))
        for by in range(bh):
            for bx in range(bw):
                dq = (coefs[ci][by, bx] * q).reshape(8, 8)
                v[by * 8:by * 8 + 8, bx * 8:bx * 8 + 8] = idct(dq) + 128.0
                sm[by, bx] = np.abs(dq).sum()
        vals.append(v)
        sums.append(sm)
    return vals, sums


def planes_to_rgb(j: Jpeg, planes: list[np.ndarray]) -> np.ndarray:
    """Chroma replicated onto the luma grid, then JFIF YCbCr -> RGB (one
    component: R = G = B = Y).  [H, W, 3] uint8."""
    hmax = max(c.h for c in j.components)
    vmax = max(c.v for c in j.components)
    ys = np.arange(j.height)
    xs = np.arange(j.width)
    up = []
    for c, p in zip(j.components, planes):
        yi = ys * c.v // vmax
        xi = xs * c.h // hmax
        up.append(p[yi][:, xi].astype(np.int64))
    if len(up) == 1:
        y = np.clip(up[0], 0, 255).astype(np.uint8)
        return np.stack([y, y, y], axis=-1)
    return ycc_to_rgb(up[0], up[1], up[2])


def decode(data: bytes) -> np.ndarray:
    """JPEG bytes -> [H, W, 3] uint8 RGB."""
    j = parse(data)
    return planes_to_rgb(j, reconstruct_planes(j, decode_coefficients(j)))


# ---------------------------------------------------------------------------
# Encoding side: colour, chroma subsampling, FDCT and quantization
# ---------------------------------------------------------------------------
def encode_planes(rgb: np.ndarray, h: tuple, v: tuple) -> list[np.ndarray]:
    """Integer sample planes of the three components for sampling factors
    h = (h_Y, h_Cb, h_Cr), v = (...): the image extended to whole MCUs by
    repeating its last column and row, converted to YCbCr, each chroma plane
    the rounded-half-up mean of the luma-grid samples each of its samples
    covers.  Each plane spans its component's MCU-padded block grid."""
    hgt, wid, _ = rgb.shape
    hmax, vmax = max(h), max(v)
    mx = -(-wid // (8 * hmax))
    my = -(-hgt // (8 * vmax))
    W, H = mx * 8 * hmax, my * 8 * vmax
    yi = np.minimum(np.arange(H), hgt - 1)
    xi = np.minimum(np.arange(W), wid - 1)
    ext = np.asarray(rgb)[yi][:, xi]
    full = rgb_to_ycc(ext)
    out = []
    for c in range(3):
        fh, fv = hmax // h[c], vmax // v[c]
        p = full[c].reshape(H // fv, fv, W // fh, fh).sum(axis=(1, 3))
        n = fh * fv
        out.append((p + n // 2) // n)
    return out


def quantize_blocks(plane: np.ndarray, q: np.ndarray):
    """FDCT of (samples - 128) per 8 x 8 block and quantization: returns the
    quantized coefficients [blocks down, blocks across, 64] (natural order),
    the values S/Q before rounding, and per block sum |samples - 128|."""
    H, W = plane.shape
    bh, bw = H // 8, W // 8
    qc = np.zeros((bh, bw, 64), np.int64)
    ratio = np.zeros((bh, bw, 64))
    sums = np.zeros((bh, bw))
    q = np.asarray(q, np.float64).reshape(8, 8)
    for by in range(bh):
        for bx in range(bw):
            s = plane[by * 8:by * 8 + 8, bx * 8:bx * 8 + 8].astype(np.float64) - 128.0
            r = fdct(s) / q
            ratio[by, bx] = r.reshape(-1)
            qc[by, bx] = round_half_away(r).reshape(-1)
            sums[by, bx] = np.abs(s).sum()
    return qc, ratio, sums
