"""Test helper: a baseline JPEG file rewritten with one scan per component
(T.81 A.2.2, non-interleaved order: each component's blocks in raster order
over its own block grid), optionally with a restart interval (B.2.4.4, E.1.4),
from the coefficients the oracle decodes and the file's own Huffman tables.

Test infrastructure only.  It writes the entropy-coded data with its own
canonical code construction (T.81 C.2) and bit writer, sharing nothing with
the library, so that the device decoder can be tried on files that PIL does
not write."""
import oracle.jpeg_ref as J


def _codes(bits, vals):
    """Symbol -> (code, length) from BITS and HUFFVAL (T.81 C.2)."""
    out, code, k = {}, 0, 0
    for length in range(1, 17):
        for _ in range(bits[length - 1]):
            out[vals[k]] = (code, length)
            code += 1
            k += 1
        code <<= 1
    return out


class _Bits:
    """MSB-first bit writer with a zero byte after every 0xFF (B.1.1.5)."""

    def __init__(self):
        self.out = bytearray()
        self.acc = 0
        self.n = 0

    def put(self, v: int, n: int):
        for i in range(n - 1, -1, -1):
            self.acc = (self.acc << 1) | ((v >> i) & 1)
            self.n += 1
            if self.n == 8:
                self.out.append(self.acc)
                if self.acc == 0xFF:
                    self.out.append(0)
                self.acc = 0
                self.n = 0

    def pad(self):
        while self.n:
            self.put(1, 1)


def _cat(v: int) -> int:
    return abs(v).bit_length()


def _mag(v: int, s: int) -> int:
    return (v if v >= 0 else v + (1 << s) - 1) & ((1 << s) - 1)


def split_scans(data: bytes, restart: int = 0) -> bytes:
    j = J.parse(data)
    assert len(j.scans) == 1
    coefs = J.decode_coefficients(j)
    _, _, _, _, grids = J.block_grid(j)
    # the headers before the first SOS, without any DRI
    head = bytearray(data[:2])
    i = 2
    while True:
        m = data[i + 1]
        n = data[i + 2] << 8 | data[i + 3]
        if m == 0xDA:
            break
        if m != 0xDD:
            head += data[i:i + 2 + n]
        i += 2 + n
    out = bytearray(head)
    if restart:
        out += bytes([0xFF, 0xDD, 0, 4, restart >> 8, restart & 255])
    tables = j.scan_tables[0]
    for ci, td, ta in j.scans[0].comps:
        dc = _codes(*tables[(0, td)])
        ac = _codes(*tables[(1, ta)])
        out += bytes([0xFF, 0xDA, 0, 8, 1, j.components[ci].cid, td << 4 | ta, 0, 63, 0])
        (_, _), (bw, bh) = grids[ci]
        w = _Bits()
        pred = 0
        rst = 0
        for n in range(bw * bh):
            if restart and n and n % restart == 0:
                w.pad()
                w.out += bytes([0xFF, 0xD0 + rst])
                rst = (rst + 1) & 7
                pred = 0
            blk = coefs[ci][n // bw, n % bw]
            zz = [int(blk[J.ZIGZAG[k]]) for k in range(64)]
            d = zz[0] - pred
            pred = zz[0]
            s = _cat(d)
            w.put(*dc[s])
            w.put(_mag(d, s), s)
            run = 0
            for k in range(1, 64):
                if zz[k] == 0:
                    run += 1
                    continue
                while run > 15:
                    w.put(*ac[0xF0])
                    run -= 16
                s = _cat(zz[k])
                w.put(*ac[run << 4 | s])
                w.put(_mag(zz[k], s), s)
                run = 0
            if run:
                w.put(*ac[0x00])
        w.pad()
        out += w.out
    out += b"\xff\xd9"
    return bytes(out)
