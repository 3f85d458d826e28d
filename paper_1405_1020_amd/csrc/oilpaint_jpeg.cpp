// JPEG decode and encode around the filter: baseline sequential DCT-based
// JPEG (ITU-T T.81; Huffman coding, 8-bit samples) in JFIF's YCbCr colour
// space.  The host parses markers, decodes the entropy-coded data, fits the
// encoder's Huffman tables and writes the headers; everything per sample
// (dequantization, inverse DCT, colour, chroma resampling; colour, chroma
// averaging, forward DCT, quantization) runs in the kernels of
// oilpaint_k_jpeg.hip and the encoder's Huffman coding in those of
// oilpaint_k_huff.hip, so a decoded image lands in device memory, ready for
// the filter, and an encoded one is read from there.
#include <algorithm>
#include <atomic>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "oilpaint_internal.h"
#include "oilpaint_jpeg.h"

namespace oilpaint_impl {
int check_device_ptr(const void* p);

namespace {

// Zig-zag order (T.81 Figure A.6): entry k is the natural (row-major) index
// of the k-th coefficient of the zig-zag sequence.
constexpr uint8_t kZigzag[64] = {
    0,  1,  8,  16, 9,  2,  3,  10, 17, 24, 32, 25, 18, 11, 4,  5,  12, 19, 26, 33, 40, 48,
    41, 34, 27, 20, 13, 6,  7,  14, 21, 28, 35, 42, 49, 56, 57, 50, 43, 36, 29, 22, 15, 23,
    30, 37, 44, 51, 58, 59, 52, 45, 38, 31, 39, 46, 53, 60, 61, 54, 47, 55, 62, 63};

// T.81 Annex K, Tables K.1 (luminance) and K.2 (chrominance), natural order.
constexpr uint8_t kLumaQ[64] = {16, 11, 10, 16, 24,  40,  51,  61,  12, 12, 14, 19, 26,  58,  60,  55,
                                14, 13, 16, 24, 40,  57,  69,  56,  14, 17, 22, 29, 51,  87,  80,  62,
                                18, 22, 37, 56, 68,  109, 103, 77,  24, 35, 55, 64, 81,  104, 113, 92,
                                49, 64, 78, 87, 103, 121, 120, 101, 72, 92, 95, 98, 112, 100, 103, 99};
constexpr uint8_t kChromaQ[64] = {17, 18, 24, 47, 99, 99, 99, 99, 18, 21, 26, 66, 99, 99, 99, 99,
                                  24, 26, 56, 99, 99, 99, 99, 99, 47, 66, 99, 99, 99, 99, 99, 99,
                                  99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99,
                                  99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99};

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------------------
// Marker syntax
// ---------------------------------------------------------------------------
struct HuffSpec {
    uint8_t bits[16];
    uint8_t vals[256];
    int nvals = 0;
    bool set = false;
};

struct ScanComp {
    int comp, td, ta;
};

struct Scan {
    std::vector<ScanComp> comps;
    size_t begin = 0, end = 0;  // entropy-coded bytes (RST markers included)
    HuffSpec dc[4], ac[4];      // tables in force at this scan
};

struct Frame {
    int width = 0, height = 0, ncomp = 0;
    int id[kJpegMaxComps] = {}, h[kJpegMaxComps] = {}, v[kJpegMaxComps] = {}, tq[kJpegMaxComps] = {};
    int hmax = 1, vmax = 1, mcux = 0, mcuy = 0, restart = 0;
    int bw[kJpegMaxComps] = {}, bh[kJpegMaxComps] = {};      // MCU-padded block grid
    int own_bw[kJpegMaxComps] = {}, own_bh[kJpegMaxComps] = {};  // blocks of the component's own samples
    int xc[kJpegMaxComps] = {}, yc[kJpegMaxComps] = {};      // component's own samples
    uint16_t q[4][64] = {};
    bool qset[4] = {};
    std::vector<Scan> scans;
    size_t blocks = 0;
    int first[kJpegMaxComps + 1] = {};
};

int parse_frame(const uint8_t* d, size_t n, Frame& f) {
    if (n < 4 || d[0] != 0xFF || d[1] != 0xD8) return OILPAINT_ERR_ARG;
    HuffSpec dc[4], ac[4];
    bool have_frame = false;
    size_t i = 2;
    for (;;) {
        if (i >= n) return OILPAINT_ERR_ARG;
        if (d[i] != 0xFF) return OILPAINT_ERR_ARG;
        while (i < n && d[i] == 0xFF) ++i;
        if (i >= n) return OILPAINT_ERR_ARG;
        const uint8_t m = d[i++];
        if (m == 0xD9) break;                                    // EOI
        if (m == 0x01 || (m >= 0xD0 && m <= 0xD7)) continue;     // TEM, stray RST
        if (i + 2 > n) return OILPAINT_ERR_ARG;
        const size_t len = (size_t)d[i] << 8 | d[i + 1];
        if (len < 2 || i + len > n) return OILPAINT_ERR_ARG;
        const uint8_t* s = d + i + 2;
        const size_t sl = len - 2;
        i += len;
        if (m == 0xDB) {  // DQT
            size_t k = 0;
            while (k < sl) {
                const int pq = s[k] >> 4, tq = s[k] & 15;
                if (tq > 3 || pq > 1) return OILPAINT_ERR_ARG;
                if (pq) return OILPAINT_ERR_UNSUPPORTED;  // 16-bit tables go with 12-bit samples (B.2.4.1)
                ++k;
                const size_t need = 64 * (pq ? 2 : 1);
                if (k + need > sl) return OILPAINT_ERR_ARG;
                for (int t = 0; t < 64; ++t) {
                    const int val = pq ? (s[k + 2 * t] << 8 | s[k + 2 * t + 1]) : s[k + t];
                    if (val == 0) return OILPAINT_ERR_ARG;
                    f.q[tq][kZigzag[t]] = (uint16_t)val;
                }
                f.qset[tq] = true;
                k += need;
            }
        } else if (m == 0xC4) {  // DHT
            size_t k = 0;
            while (k < sl) {
                const int tc = s[k] >> 4, th = s[k] & 15;
                if (tc > 1 || th > 3 || k + 17 > sl) return OILPAINT_ERR_ARG;
                HuffSpec& h = tc ? ac[th] : dc[th];
                int total = 0;
                for (int l = 0; l < 16; ++l) total += (h.bits[l] = s[k + 1 + l]);
                if (total > 256 || k + 17 + total > sl) return OILPAINT_ERR_ARG;
                std::memcpy(h.vals, s + k + 17, total);
                h.nvals = total;
                h.set = true;
                k += 17 + total;
            }
        } else if (m == 0xC0 || m == 0xC1) {  // SOF0, SOF1
            if (have_frame || sl < 6 || s[0] != 8) return OILPAINT_ERR_UNSUPPORTED;
            f.height = s[1] << 8 | s[2];
            f.width = s[3] << 8 | s[4];
            f.ncomp = s[5];
            if (f.width == 0 || f.height == 0) return OILPAINT_ERR_UNSUPPORTED;  // height from DNL
            if ((f.ncomp != 1 && f.ncomp != 3) || sl < 6 + 3 * (size_t)f.ncomp) return OILPAINT_ERR_UNSUPPORTED;
            for (int c = 0; c < f.ncomp; ++c) {
                f.id[c] = s[6 + 3 * c];
                f.h[c] = s[7 + 3 * c] >> 4;
                f.v[c] = s[7 + 3 * c] & 15;
                f.tq[c] = s[8 + 3 * c];
                if (f.h[c] < 1 || f.h[c] > 4 || f.v[c] < 1 || f.v[c] > 4 || f.tq[c] > 3) return OILPAINT_ERR_ARG;
            }
            have_frame = true;
        } else if ((m >= 0xC2 && m <= 0xCF) && m != 0xC4 && m != 0xC8 && m != 0xCC) {
            return OILPAINT_ERR_UNSUPPORTED;  // progressive, lossless, hierarchical, arithmetic
        } else if (m == 0xDD) {  // DRI
            if (sl < 2) return OILPAINT_ERR_ARG;
            f.restart = s[0] << 8 | s[1];
        } else if (m == 0xDA) {  // SOS
            if (!have_frame || sl < 1) return OILPAINT_ERR_ARG;
            Scan sc;
            const int ns = s[0];
            if (ns < 1 || ns > f.ncomp || sl < 1 + 2 * (size_t)ns + 3) return OILPAINT_ERR_ARG;
            for (int k = 0; k < ns; ++k) {
                int c = 0;
                while (c < f.ncomp && f.id[c] != s[1 + 2 * k]) ++c;
                if (c == f.ncomp) return OILPAINT_ERR_ARG;
                const int td = s[2 + 2 * k] >> 4, ta = s[2 + 2 * k] & 15;
                if (td > 3 || ta > 3 || !dc[td].set || !ac[ta].set) return OILPAINT_ERR_ARG;
                sc.comps.push_back({c, td, ta});
            }
            for (int t = 0; t < 4; ++t) {
                sc.dc[t] = dc[t];
                sc.ac[t] = ac[t];
            }
            sc.begin = i;
            // the data ends at the first 0xFF followed by neither a stuffed
            // zero nor RSTn
            for (;;) {
                const void* hit = i < n ? std::memchr(d + i, 0xFF, n - i) : nullptr;
                i = hit ? (size_t)(static_cast<const uint8_t*>(hit) - d) : n;
                if (i + 1 >= n) break;
                const uint8_t nx = d[i + 1];
                if (nx != 0 && !(nx >= 0xD0 && nx <= 0xD7)) break;
                i += 2;
            }
            if (i + 1 >= n) return OILPAINT_ERR_ARG;
            sc.end = i;
            f.scans.push_back(sc);
        }
        // APPn, COM, DNL and the rest: skipped
    }
    if (!have_frame || f.scans.empty()) return OILPAINT_ERR_ARG;
    for (int c = 0; c < f.ncomp; ++c)
        if (!f.qset[f.tq[c]]) return OILPAINT_ERR_ARG;
    f.hmax = f.vmax = 1;
    for (int c = 0; c < f.ncomp; ++c) {
        f.hmax = std::max(f.hmax, f.h[c]);
        f.vmax = std::max(f.vmax, f.v[c]);
    }
    f.mcux = (f.width + 8 * f.hmax - 1) / (8 * f.hmax);
    f.mcuy = (f.height + 8 * f.vmax - 1) / (8 * f.vmax);
    f.first[0] = 0;
    for (int c = 0; c < f.ncomp; ++c) {
        f.bw[c] = f.mcux * f.h[c];
        f.bh[c] = f.mcuy * f.v[c];
        f.xc[c] = (int)(((int64_t)f.width * f.h[c] + f.hmax - 1) / f.hmax);
        f.yc[c] = (int)(((int64_t)f.height * f.v[c] + f.vmax - 1) / f.vmax);
        f.own_bw[c] = (f.xc[c] + 7) / 8;
        f.own_bh[c] = (f.yc[c] + 7) / 8;
        f.first[c + 1] = f.first[c] + f.bw[c] * f.bh[c];
    }
    for (int c = f.ncomp; c < kJpegMaxComps; ++c) f.first[c + 1] = f.first[c];
    f.blocks = (size_t)f.first[f.ncomp];
    return OILPAINT_OK;
}

// ---------------------------------------------------------------------------
// Huffman decoding: codes from BITS (Annex C), a 9-bit lookup for short
// codes, the MAXCODE/VALPTR walk (F.2.2.3) for longer ones.
// ---------------------------------------------------------------------------
struct HuffDec {
    int32_t maxcode[18];
    int32_t valoff[17];  // value index = code + valoff[len]
    uint8_t vals[256];
    uint16_t fast[512];  // (length << 8) | value, 0 if longer than 9 bits
    bool ok = false;
};

bool build_dec(const HuffSpec& s, HuffDec& h) {
    std::memcpy(h.vals, s.vals, sizeof(h.vals));
    std::memset(h.fast, 0, sizeof(h.fast));
    int code = 0, k = 0;
    for (int len = 1; len <= 16; ++len) {
        const int cnt = s.bits[len - 1];
        h.valoff[len] = k - code;
        for (int j = 0; j < cnt; ++j, ++k, ++code) {
            if (code >= (1 << len)) return false;
            if (len <= 9) {
                const int shift = 9 - len;
                for (int f = code << shift; f < ((code + 1) << shift); ++f) h.fast[f] = (uint16_t)(len << 8 | s.vals[k]);
            }
        }
        h.maxcode[len] = cnt ? code - 1 : -1;
        code <<= 1;
    }
    h.maxcode[17] = 0x7fffffff;
    h.ok = true;
    return true;
}

class BitIn {
  public:
    BitIn(const uint8_t* d, size_t begin, size_t end) : d_(d), i_(begin), end_(end) {}
    // Reads 0 bits beyond a marker or the segment's end.
    void fill() {
        while (nbits_ <= 56) {
            uint64_t b = 0;
            if (!marker_ && i_ < end_) {
                b = d_[i_];
                if (b == 0xFF) {
                    const uint8_t nx = i_ + 1 < end_ ? d_[i_ + 1] : 0xD9;
                    if (nx == 0x00) {
                        i_ += 2;
                    } else {
                        marker_ = true;
                        b = 0;
                    }
                } else {
                    ++i_;
                }
            }
            buf_ |= b << (56 - nbits_);
            nbits_ += 8;
        }
    }
    uint32_t peek(int n) {
        if (nbits_ < n) fill();
        return (uint32_t)(buf_ >> (64 - n));
    }
    void skip(int n) {
        buf_ <<= n;
        nbits_ -= n;
    }
    int receive(int s) {
        if (s == 0) return 0;
        const int v = (int)peek(s);
        skip(s);
        return v;
    }
    int decode(const HuffDec& h) {
        const uint32_t p = peek(16);
        const uint16_t e = h.fast[p >> 7];
        if (e) {
            skip(e >> 8);
            return e & 255;
        }
        int len = 10;
        int code = (int)(p >> (16 - len));
        while (code > h.maxcode[len]) {
            ++len;
            if (len > 16) return -1;
            code = (int)(p >> (16 - len));
        }
        skip(len);
        return h.vals[(code + h.valoff[len]) & 255];
    }
    // At a restart boundary: drop the buffered bits and step over RSTn.
    bool restart() {
        buf_ = 0;
        nbits_ = 0;
        marker_ = false;
        while (i_ + 1 < end_ && !(d_[i_] == 0xFF && d_[i_ + 1] >= 0xD0 && d_[i_ + 1] <= 0xD7)) ++i_;
        if (i_ + 1 >= end_) return false;
        i_ += 2;
        return true;
    }

  private:
    const uint8_t* d_;
    size_t i_, end_;
    uint64_t buf_ = 0;
    int nbits_ = 0;
    bool marker_ = false;
};

inline int extend(int v, int t) { return (t && v < (1 << (t - 1))) ? v - (1 << t) + 1 : v; }

// Every scan's blocks into `coef` (natural order, component c's block (bx,
// by) at (first[c] + by * bw[c] + bx) * 64); blocks no scan covers are 0.
int entropy_decode(const uint8_t* d, const Frame& f, int16_t* coef) {
    std::memset(coef, 0, f.blocks * 64 * sizeof(int16_t));
    for (const Scan& sc : f.scans) {
        HuffDec dcd[4], acd[4];
        for (const ScanComp& c : sc.comps) {
            if (!dcd[c.td].ok && !build_dec(sc.dc[c.td], dcd[c.td])) return OILPAINT_ERR_ARG;
            if (!acd[c.ta].ok && !build_dec(sc.ac[c.ta], acd[c.ta])) return OILPAINT_ERR_ARG;
        }
        BitIn in(d, sc.begin, sc.end);
        int pred[kJpegMaxComps] = {};
        auto block = [&](const ScanComp& c, int by, int bx) -> bool {
            int16_t* out = coef + ((size_t)f.first[c.comp] + (size_t)by * f.bw[c.comp] + bx) * 64;
            const int t = in.decode(dcd[c.td]);
            if (t < 0 || t > 11) return false;
            pred[c.comp] += extend(in.receive(t), t);
            out[0] = (int16_t)pred[c.comp];
            for (int k = 1; k < 64;) {
                const int rs = in.decode(acd[c.ta]);
                if (rs < 0) return false;
                const int r = rs >> 4, s = rs & 15;
                if (s == 0) {
                    if (r != 15) break;
                    k += 16;
                    continue;
                }
                k += r;
                if (k > 63 || s > 10) return false;
                out[kZigzag[k]] = (int16_t)extend(in.receive(s), s);
                ++k;
            }
            return true;
        };
        if (sc.comps.size() == 1) {
            const ScanComp& c = sc.comps[0];
            int64_t n = 0;
            for (int by = 0; by < f.own_bh[c.comp]; ++by)
                for (int bx = 0; bx < f.own_bw[c.comp]; ++bx, ++n) {
                    if (f.restart && n && n % f.restart == 0) {
                        if (!in.restart()) return OILPAINT_ERR_ARG;
                        pred[c.comp] = 0;
                    }
                    if (!block(c, by, bx)) return OILPAINT_ERR_ARG;
                }
        } else {
            int64_t n = 0;
            for (int my = 0; my < f.mcuy; ++my)
                for (int mx = 0; mx < f.mcux; ++mx, ++n) {
                    if (f.restart && n && n % f.restart == 0) {
                        if (!in.restart()) return OILPAINT_ERR_ARG;
                        for (int& p : pred) p = 0;
                    }
                    for (const ScanComp& c : sc.comps)
                        for (int v = 0; v < f.v[c.comp]; ++v)
                            for (int h = 0; h < f.h[c.comp]; ++h)
                                if (!block(c, my * f.v[c.comp] + v, mx * f.h[c.comp] + h)) return OILPAINT_ERR_ARG;
                }
        }
    }
    return OILPAINT_OK;
}

// ---------------------------------------------------------------------------
// Huffman encoding with tables fitted to the image (T.81 K.2: code sizes
// from symbol frequencies, lengths limited to 16 bits, one code point
// reserved so that no code is all ones).
// ---------------------------------------------------------------------------
struct HuffEnc {
    uint8_t bits[16];
    uint8_t vals[256];
    int nvals = 0;
    uint16_t code[256];
    uint8_t size[256];
};

void fit_table(const int64_t* freq_in, HuffEnc& t) {
    int64_t freq[257];
    int codesize[257] = {};
    int others[257];
    for (int i = 0; i < 256; ++i) freq[i] = freq_in[i];
    freq[256] = 1;  // reserved
    for (int i = 0; i < 257; ++i) others[i] = -1;
    for (;;) {
        int v1 = -1, v2 = -1;
        for (int i = 0; i < 257; ++i)  // least frequency, the larger index on ties
            if (freq[i] > 0 && (v1 < 0 || freq[i] <= freq[v1])) v1 = i;
        for (int i = 0; i < 257; ++i)
            if (freq[i] > 0 && i != v1 && (v2 < 0 || freq[i] <= freq[v2])) v2 = i;
        if (v2 < 0) break;
        freq[v1] += freq[v2];
        freq[v2] = 0;
        ++codesize[v1];
        while (others[v1] >= 0) {
            v1 = others[v1];
            ++codesize[v1];
        }
        others[v1] = v2;
        ++codesize[v2];
        while (others[v2] >= 0) {
            v2 = others[v2];
            ++codesize[v2];
        }
    }
    int cnt[33] = {};
    for (int i = 0; i < 257; ++i)
        if (codesize[i]) ++cnt[std::min(codesize[i], 32)];
    for (int i = 32; i > 16; --i) {  // limit the lengths to 16
        while (cnt[i] > 0) {
            int j = i - 2;
            while (cnt[j] == 0) --j;
            cnt[i] -= 2;
            ++cnt[i - 1];
            cnt[j + 1] += 2;
            --cnt[j];
        }
    }
    int i = 16;
    while (i > 0 && cnt[i] == 0) --i;
    if (i > 0) --cnt[i];  // drop the reserved code point
    for (int l = 0; l < 16; ++l) t.bits[l] = (uint8_t)cnt[l + 1];
    t.nvals = 0;
    for (int l = 1; l <= 32; ++l)
        for (int s = 0; s < 256; ++s)
            if (codesize[s] == l) t.vals[t.nvals++] = (uint8_t)s;
    // codes (Annex C)
    std::memset(t.size, 0, sizeof(t.size));
    int code = 0, k = 0;
    for (int len = 1; len <= 16; ++len) {
        for (int j = 0; j < t.bits[len - 1]; ++j, ++k, ++code) {
            t.code[t.vals[k]] = (uint16_t)code;
            t.size[t.vals[k]] = (uint8_t)len;
        }
        code <<= 1;
    }
}

class BitOut {
  public:
    explicit BitOut(std::vector<uint8_t>& o) : o_(o) {}
    void put(uint32_t v, int n) {
        if (n == 0) return;
        acc_ = (acc_ << n) | (v & ((1u << n) - 1));
        nb_ += n;
        while (nb_ >= 8) {
            const uint8_t b = (uint8_t)(acc_ >> (nb_ - 8));
            o_.push_back(b);
            if (b == 0xFF) o_.push_back(0);
            nb_ -= 8;
        }
    }
    void flush() {  // pad with one bits
        if (nb_ > 0) put(0x7F, 8 - nb_);
    }

  private:
    std::vector<uint8_t>& o_;
    uint64_t acc_ = 0;
    int nb_ = 0;
};

inline int category(int v) {
    int a = v < 0 ? -v : v, s = 0;
    while (a) {
        ++s;
        a >>= 1;
    }
    return s;
}

// Walk the blocks of one interleaved scan: fn(component, block coefficients).
template <typename Fn>
void for_blocks(const Frame& f, const int16_t* coef, Fn fn) {
    for (int my = 0; my < f.mcuy; ++my)
        for (int mx = 0; mx < f.mcux; ++mx)
            for (int c = 0; c < f.ncomp; ++c)
                for (int v = 0; v < f.v[c]; ++v)
                    for (int h = 0; h < f.h[c]; ++h) {
                        const int by = my * f.v[c] + v, bx = mx * f.h[c] + h;
                        fn(c, coef + ((size_t)f.first[c] + (size_t)by * f.bw[c] + bx) * 64);
                    }
}

void put16(std::vector<uint8_t>& o, int v) {
    o.push_back((uint8_t)(v >> 8));
    o.push_back((uint8_t)v);
}

// Symbol counts of the scan (DC and AC, luminance and chrominance tables).
void count_symbols(const Frame& f, const int16_t* coef, int64_t* fdc, int64_t* fac) {
    int pred[kJpegMaxComps] = {};
    for_blocks(f, coef, [&](int c, const int16_t* b) {
        const int t = c ? 1 : 0;
        ++fdc[t * 256 + category(b[0] - pred[c])];
        pred[c] = b[0];
        int run = 0;
        for (int k = 1; k < 64; ++k) {
            const int v = b[kZigzag[k]];
            if (v == 0) {
                ++run;
                continue;
            }
            while (run > 15) {
                ++fac[t * 256 + 0xF0];
                run -= 16;
            }
            ++fac[t * 256 + (run << 4 | category(v))];
            run = 0;
        }
        if (run) ++fac[t * 256 + 0x00];
    });
}

// Everything before the entropy-coded data: SOI, JFIF APP0, the quantization
// tables, SOF0, the fitted Huffman tables and SOS.
void write_headers(const Frame& f, const HuffEnc* dc, const HuffEnc* ac, std::vector<uint8_t>& o) {
    const int ntab = f.ncomp == 1 ? 1 : 2;
    o.insert(o.end(), {0xFF, 0xD8, 0xFF, 0xE0});
    put16(o, 16);
    o.insert(o.end(), {'J', 'F', 'I', 'F', 0, 1, 1, 0, 0, 1, 0, 1, 0, 0});
    for (int t = 0; t < ntab; ++t) {
        o.insert(o.end(), {0xFF, 0xDB});
        put16(o, 67);
        o.push_back((uint8_t)t);
        for (int k = 0; k < 64; ++k) o.push_back((uint8_t)f.q[t][kZigzag[k]]);
    }
    o.insert(o.end(), {0xFF, 0xC0});
    put16(o, 8 + 3 * f.ncomp);
    o.push_back(8);
    put16(o, f.height);
    put16(o, f.width);
    o.push_back((uint8_t)f.ncomp);
    for (int c = 0; c < f.ncomp; ++c) {
        o.push_back((uint8_t)(c + 1));
        o.push_back((uint8_t)(f.h[c] << 4 | f.v[c]));
        o.push_back((uint8_t)f.tq[c]);
    }
    for (int t = 0; t < ntab; ++t)
        for (int cls = 0; cls < 2; ++cls) {
            const HuffEnc& h = cls ? ac[t] : dc[t];
            o.insert(o.end(), {0xFF, 0xC4});
            put16(o, 2 + 17 + h.nvals);
            o.push_back((uint8_t)(cls << 4 | t));
            o.insert(o.end(), h.bits, h.bits + 16);
            o.insert(o.end(), h.vals, h.vals + h.nvals);
        }
    o.insert(o.end(), {0xFF, 0xDA});
    put16(o, 6 + 2 * f.ncomp);
    o.push_back((uint8_t)f.ncomp);
    for (int c = 0; c < f.ncomp; ++c) {
        o.push_back((uint8_t)(c + 1));
        const int t = c ? 1 : 0;
        o.push_back((uint8_t)(t << 4 | t));
    }
    o.insert(o.end(), {0, 63, 0});
}

// The whole file on the host (oilpaint_jpeg_write).
void entropy_encode(const Frame& f, const int16_t* coef, std::vector<uint8_t>& o) {
    const int ntab = f.ncomp == 1 ? 1 : 2;
    std::vector<int64_t> fdc(2 * 256, 0), fac(2 * 256, 0);
    count_symbols(f, coef, fdc.data(), fac.data());
    HuffEnc dc[2], ac[2];
    for (int t = 0; t < ntab; ++t) {
        fit_table(&fdc[t * 256], dc[t]);
        fit_table(&fac[t * 256], ac[t]);
    }
    write_headers(f, dc, ac, o);
    BitOut bo(o);
    int pred[kJpegMaxComps] = {};
    for_blocks(f, coef, [&](int c, const int16_t* b) {
        const HuffEnc& hd = dc[c ? 1 : 0];
        const HuffEnc& ha = ac[c ? 1 : 0];
        const int diff = b[0] - pred[c];
        pred[c] = b[0];
        const int s = category(diff);
        bo.put(hd.code[s], hd.size[s]);
        bo.put((uint32_t)(diff < 0 ? diff - 1 : diff), s);
        int run = 0;
        for (int k = 1; k < 64; ++k) {
            const int v = b[kZigzag[k]];
            if (v == 0) {
                ++run;
                continue;
            }
            while (run > 15) {
                bo.put(ha.code[0xF0], ha.size[0xF0]);
                run -= 16;
            }
            const int sz = category(v);
            const int sym = run << 4 | sz;
            bo.put(ha.code[sym], ha.size[sym]);
            bo.put((uint32_t)(v < 0 ? v - 1 : v), sz);
            run = 0;
        }
        if (run) bo.put(ha.code[0], ha.size[0]);
    });
    bo.flush();
    o.insert(o.end(), {0xFF, 0xD9});
}

// The scan as the device coder walks it (every component interleaved).
JpegScanMap scan_map(const Frame& f) {
    JpegScanMap m;
    std::memset(&m, 0, sizeof(m));
    int j = 0;
    for (int c = 0; c < f.ncomp; ++c) {
        for (int v = 0; v < f.v[c]; ++v)
            for (int h = 0; h < f.h[c]; ++h, ++j) {
                m.comp[j] = c;
                m.dx[j] = h;
                m.dy[j] = v;
                m.prev[j] = (v || h) ? j - 1 : -1;
            }
        m.last[c] = j - 1;
        m.h[c] = f.h[c];
        m.v[c] = f.v[c];
        m.bw[c] = f.bw[c];
        m.first[c] = f.first[c];
        m.tab[c] = c ? 1 : 0;
    }
    m.bpm = j;
    m.mcux = f.mcux;
    m.blocks = (int64_t)f.mcux * f.mcuy * j;
    return m;
}

// Quality scaling of the Annex K tables (the Independent JPEG Group's
// convention: 50 keeps them, lower scales them up, higher down).
void scaled_table(const uint8_t* base, int quality, uint16_t* out) {
    quality = std::min(100, std::max(1, quality));
    const int scale = quality < 50 ? 5000 / quality : 200 - 2 * quality;
    for (int k = 0; k < 64; ++k) out[k] = (uint16_t)std::min(255, std::max(1, (base[k] * scale + 50) / 100));
}

// The frame the encoder writes: three components, Y sampled (hl, vl) = (1,
// 1), (2, 1) or (2, 2) for subsampling 0, 1, 2 (4:4:4, 4:2:2, 4:2:0), Cb and
// Cr (1, 1); tables 0 (luminance) and 1 (chrominance) at `quality`.
int encode_frame(int width, int height, int quality, int subsampling, Frame& f) {
    if (width < 1 || height < 1 || width > 65535 || height > 65535) return OILPAINT_ERR_ARG;
    if (quality < 1 || quality > 100 || subsampling < 0 || subsampling > 2) return OILPAINT_ERR_ARG;
    f = Frame();
    f.width = width;
    f.height = height;
    f.ncomp = 3;
    const int hl = subsampling == 0 ? 1 : 2, vl = subsampling == 2 ? 2 : 1;
    for (int c = 0; c < 3; ++c) {
        f.id[c] = c + 1;
        f.h[c] = c ? 1 : hl;
        f.v[c] = c ? 1 : vl;
        f.tq[c] = c ? 1 : 0;
    }
    scaled_table(kLumaQ, quality, f.q[0]);
    scaled_table(kChromaQ, quality, f.q[1]);
    f.qset[0] = f.qset[1] = true;
    f.hmax = hl;
    f.vmax = vl;
    f.mcux = (width + 8 * hl - 1) / (8 * hl);
    f.mcuy = (height + 8 * vl - 1) / (8 * vl);
    f.first[0] = 0;
    for (int c = 0; c < 3; ++c) {
        f.bw[c] = f.mcux * f.h[c];
        f.bh[c] = f.mcuy * f.v[c];
        f.xc[c] = (int)(((int64_t)width * f.h[c] + hl - 1) / hl);
        f.yc[c] = (int)(((int64_t)height * f.v[c] + vl - 1) / vl);
        f.own_bw[c] = (f.xc[c] + 7) / 8;
        f.own_bh[c] = (f.yc[c] + 7) / 8;
        f.first[c + 1] = f.first[c] + f.bw[c] * f.bh[c];
    }
    f.blocks = (size_t)f.first[3];
    return OILPAINT_OK;
}

void fill_info(const Frame& f, oilpaint_jpeg_info* info) {
    std::memset(info, 0, sizeof(*info));
    info->width = f.width;
    info->height = f.height;
    info->components = f.ncomp;
    for (int c = 0; c < f.ncomp; ++c) {
        info->h_samp[c] = f.h[c];
        info->v_samp[c] = f.v[c];
        info->comp_width[c] = f.xc[c];
        info->comp_height[c] = f.yc[c];
        info->blocks_w[c] = f.bw[c];
        info->blocks_h[c] = f.bh[c];
        info->first_block[c] = f.first[c];
    }
    info->blocks = (int64_t)f.blocks;
    info->restart_interval = f.restart;
    info->scans = (int)f.scans.size();
}

// ---------------------------------------------------------------------------
// Per-device buffers: coefficients and sample planes, grown on demand;
// `done` marks the end of the last call's device work on them.
// ---------------------------------------------------------------------------
struct JpegDevice {
    std::mutex mu;
    int16_t* coef = nullptr;
    size_t coef_cap = 0;  // coefficients
    uint8_t* planes = nullptr;
    size_t plane_cap = 0;
    hipEvent_t done = nullptr;
    // the decoder's tracks come down on `side` while the links are decoded
    hipStream_t side = nullptr;
    hipEvent_t tracks_done = nullptr;
    bool pending = false;
    // Huffman coding on the device: symbol counts, code tables and the two
    // totals (bits, 0xFF bytes) in `small` (device) and `small_host`
    // (pinned); per-block bits and offsets, prefix-sum tiles, the stream's
    // words and the stuffed bytes.
    struct Small {
        unsigned long long freq[4 * 256];
        uint32_t tabs[4 * 256];
        uint64_t totals[2];
    };
    Small* small = nullptr;
    Small* small_host = nullptr;
    uint32_t* bits = nullptr;
    uint64_t* offset = nullptr;
    uint64_t* tiles = nullptr;
    uint32_t* words = nullptr;
    uint8_t* stuffed = nullptr;
    size_t bits_cap = 0, offset_cap = 0, tiles_cap = 0, words_cap = 0, stuffed_cap = 0;
    int cus = 0;
    // Huffman decoding on the device: the staged upload (stripped data,
    // tables, subsequences, intervals) in `stage` (pinned) and `dstage`, the
    // tracks, links and entries of the subsequences, the DC differences and
    // their sums.
    uint8_t* stage = nullptr;
    uint8_t* dstage = nullptr;
    size_t stage_cap = 0, dstage_cap = 0;
    JpegTrack* tracks = nullptr;   // 2 x bpm per subsequence
    JpegLink* links = nullptr;
    JpegEntry* entries = nullptr;
    uint32_t* dflags = nullptr;    // [0] malformed, [2..3] a prefix-sum total
    uint32_t* dcdiff = nullptr;    // 2 x blocks: differences, then their component order
    uint64_t* dsum = nullptr;      // blocks: prefix sums
    uint8_t* hwork = nullptr;      // pinned: tracks and links down, entries up; the coded stream down
    size_t tracks_cap = 0, links_cap = 0, entries_cap = 0, dcdiff_cap = 0, dsum_cap = 0, hwork_cap = 0;
    ~JpegDevice() {
        if (pending) (void)hipEventSynchronize(done);
        if (coef) (void)hipFree(coef);
        if (planes) (void)hipFree(planes);
        if (done) (void)hipEventDestroy(done);
        if (tracks_done) (void)hipEventDestroy(tracks_done);
        if (side) (void)hipStreamDestroy(side);
        if (small) (void)hipFree(small);
        if (small_host) (void)hipHostFree(small_host);
        for (void* p : {(void*)bits, (void*)offset, (void*)tiles, (void*)words, (void*)stuffed, (void*)dstage,
                        (void*)tracks, (void*)links, (void*)entries, (void*)dflags, (void*)dcdiff, (void*)dsum})
            if (p) (void)hipFree(p);
        if (stage) (void)hipHostFree(stage);
        if (hwork) (void)hipHostFree(hwork);
    }
    template <typename T>
    static int grow(T*& p, size_t& cap, size_t n) {
        if (n <= cap) return OILPAINT_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        const size_t c = std::max(n, (size_t)1 << 16);
        if (hipMalloc(reinterpret_cast<void**>(&p), c * sizeof(T)) != hipSuccess) return OILPAINT_ERR_NOMEM;
        cap = c;
        return OILPAINT_OK;
    }
    int reserve_hwork(size_t n) {
        if (n <= hwork_cap) return OILPAINT_OK;
        if (hwork) (void)hipHostFree(hwork);
        hwork = nullptr;
        hwork_cap = 0;
        const size_t c = std::max(n, (size_t)1 << 20);
        if (hipHostMalloc(reinterpret_cast<void**>(&hwork), c, hipHostMallocDefault) != hipSuccess)
            return OILPAINT_ERR_NOMEM;
        hwork_cap = c;
        return OILPAINT_OK;
    }
    int reserve_stage(size_t n) {
        if (n > stage_cap) {
            if (stage) (void)hipHostFree(stage);
            stage = nullptr;
            stage_cap = 0;
            const size_t c = std::max(n, (size_t)1 << 20);
            if (hipHostMalloc(reinterpret_cast<void**>(&stage), c, hipHostMallocDefault) != hipSuccess)
                return OILPAINT_ERR_NOMEM;
            stage_cap = c;
        }
        return grow(dstage, dstage_cap, n);
    }
    int reserve_coder(int device) {
        if (!small) {
            if (hipMalloc(reinterpret_cast<void**>(&small), sizeof(Small)) != hipSuccess) return OILPAINT_ERR_NOMEM;
            if (hipHostMalloc(reinterpret_cast<void**>(&small_host), sizeof(Small), hipHostMallocDefault) !=
                hipSuccess)
                return OILPAINT_ERR_NOMEM;
        }
        if (!cus && note_hip("hipDeviceGetAttribute", hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                                                            device)) != hipSuccess)
            return OILPAINT_ERR_HIP;
        if (!side && note_hip("hipStreamCreate", hipStreamCreateWithFlags(&side, hipStreamNonBlocking)) != hipSuccess)
            return OILPAINT_ERR_HIP;
        if (!tracks_done &&
            note_hip("hipEventCreate", hipEventCreateWithFlags(&tracks_done, hipEventDisableTiming)) != hipSuccess)
            return OILPAINT_ERR_HIP;
        return OILPAINT_OK;
    }
    int reserve(size_t ncoef, size_t nplane) {
        if (!done && note_hip("hipEventCreate", hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess)
            return OILPAINT_ERR_HIP;
        if (ncoef > coef_cap) {
            if (coef) (void)hipFree(coef);
            coef = nullptr;
            coef_cap = 0;
            const size_t cap = std::max(ncoef, (size_t)1 << 20);
            if (hipMalloc(&coef, cap * sizeof(int16_t)) != hipSuccess) return OILPAINT_ERR_NOMEM;
            coef_cap = cap;
        }
        if (nplane > plane_cap) {
            if (planes) (void)hipFree(planes);
            planes = nullptr;
            plane_cap = 0;
            const size_t cap = std::max(nplane, (size_t)1 << 20);
            if (hipMalloc(&planes, cap) != hipSuccess) return OILPAINT_ERR_NOMEM;
            plane_cap = cap;
        }
        return OILPAINT_OK;
    }
    // Wait (host) until the previous call's work on the buffers is done.
    int wait() {
        if (pending && note_hip("hipEventSynchronize", hipEventSynchronize(done)) != hipSuccess)
            return OILPAINT_ERR_HIP;
        pending = false;
        return OILPAINT_OK;
    }
    int mark(hipStream_t s) {
        if (note_hip("hipEventRecord", hipEventRecord(done, s)) != hipSuccess) return OILPAINT_ERR_HIP;
        pending = true;
        return OILPAINT_OK;
    }
};

JpegDevice& jpeg_device(int device) {
    static std::mutex mu;
    static std::map<int, std::unique_ptr<JpegDevice>> m;
    std::lock_guard<std::mutex> lock(mu);
    auto& p = m[device];
    if (!p) p.reset(new JpegDevice);
    return *p;
}

// Planes of the frame's components over their MCU-padded grids, one after
// another in `base`.
void plane_layout(const Frame& f, uint8_t* base, uint8_t** plane, int32_t* stride, size_t* total) {
    size_t off = 0;
    for (int c = 0; c < kJpegMaxComps; ++c) {
        if (c < f.ncomp) {
            stride[c] = f.bw[c] * 8;
            plane[c] = base ? base + off : nullptr;
            off += ((size_t)f.bw[c] * 8 * f.bh[c] * 8 + 255) & ~(size_t)255;
        } else {
            stride[c] = 0;
            plane[c] = nullptr;
        }
    }
    *total = off;
}

JpegIdctArgs idct_args(const Frame& f, const int16_t* coef) {
    JpegIdctArgs a;
    std::memset(&a, 0, sizeof(a));
    a.coef = coef;
    for (int c = 0; c <= kJpegMaxComps; ++c) a.first[c] = f.first[c];
    for (int c = 0; c < f.ncomp; ++c) {
        a.bw[c] = f.bw[c];
        std::memcpy(a.q[c], f.q[f.tq[c]], sizeof(a.q[c]));
    }
    return a;
}

// ---------------------------------------------------------------------------
// Huffman decoding on the device (oilpaint_k_huffdec.hip): the host strips
// the markers and plans the subsequences, the kernels decode.
// ---------------------------------------------------------------------------
std::atomic<int> g_sub_bits{0};  // 0: automatic (auto_sub_bits)

// The subsequence length for a scan of `bits` bits of data.  A thread
// decodes its subsequence serially, so the tracks, links and decode passes
// last in proportion to the length while the GPU has threads to spare; the
// host's walk and the subsequences it decodes itself grow with their number.
// The sum is least near a length proportional to the square root of the
// data: about 0.35 sqrt(bits), in multiples of 64 between 128 and 1024
// (measured best at 640x480, 1024x768, 1920x1080 and 2560x1600, quality 90:
// 128, 192-256, 384-512 and 512-1024 bits).
uint64_t auto_sub_bits(uint64_t bits) {
    const double s = 0.35 * std::sqrt((double)bits);
    const uint64_t r = (uint64_t)(s / 64.0 + 0.5) * 64;
    return std::min<uint64_t>(1024, std::max<uint64_t>(128, r));
}

// Scan sc's entropy-coded bytes without the stuffed zero bytes and the RST
// markers (T.81 B.1.1.5, E.1.4), appended to out; starts receives the byte
// offset in out of each restart interval's data, then the end.  Inside a
// scan's data every 0xFF is followed by 0x00 or RSTn (the parser ends the
// data at any other marker).
void strip_scan(const uint8_t* d, const Scan& sc, std::vector<uint8_t>& out, std::vector<size_t>& starts) {
    starts.push_back(out.size());
    size_t i = sc.begin;
    while (i < sc.end) {
        const void* hit = std::memchr(d + i, 0xFF, sc.end - i);
        const size_t k = hit ? (size_t)(static_cast<const uint8_t*>(hit) - d) : sc.end;
        out.insert(out.end(), d + i, d + k);
        if (k + 1 >= sc.end) break;
        if (d[k + 1] == 0x00) {
            out.push_back(0xFF);
        } else {
            starts.push_back(out.size());  // RSTn
        }
        i = k + 2;
    }
    starts.push_back(out.size());
}

void to_dev_table(const HuffSpec& spec, const HuffDec& h, JpegHuffTable& t) {
    // the canonical codes (T.81 C.2) again; every code of at most
    // kJpegFastBits bits fills the entries it prefixes (build_dec has
    // checked that the codes fit their lengths)
    std::memset(t.fast, 0, sizeof(t.fast));
    int code = 0, k = 0;
    for (int len = 1; len <= 16; ++len) {
        for (int n = 0; n < spec.bits[len - 1]; ++n, ++k, ++code)
            if (len <= kJpegFastBits) {
                const int shift = kJpegFastBits - len;
                for (int f = code << shift; f < ((code + 1) << shift); ++f) t.fast[f] = (uint16_t)(len << 8 | spec.vals[k]);
            }
        code <<= 1;
    }
    for (int l = 0; l < 18; ++l) t.maxcode[l] = l < 17 ? h.maxcode[l] : INT32_MAX;
    std::memcpy(t.valoff, h.valoff, sizeof(t.valoff));
    std::memcpy(t.vals, h.vals, sizeof(t.vals));
}

// One scan's plan: its map, tables, subsequences and intervals, and where its
// pieces sit in the staged upload.
struct ScanPlan {
    JpegDecScan s;
    int sub_bits = 0;
    size_t words_off = 0, tables_off = 0, subs_off = 0, segs_off = 0;
    std::vector<JpegSub> subs;
    std::vector<JpegSeg> segs;
    JpegHuffTable tables[8];
    HuffDec hdec[8];  // the same tables for the host's own decoding
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Plans every scan, stages the upload in jd.stage and returns its size.
int plan_scans(const uint8_t* data, const Frame& f, std::vector<ScanPlan>& plans, std::vector<uint8_t>& bytes,
               size_t* stage_bytes) {
    const uint64_t fixed_bits = (uint64_t)g_sub_bits.load();
    plans.resize(f.scans.size());
    for (ScanPlan& pl : plans) {
        pl.subs.clear();
        pl.segs.clear();
    }
    for (size_t si = 0; si < f.scans.size(); ++si) {
        const Scan& sc = f.scans[si];
        ScanPlan& pl = plans[si];
        JpegDecScan& s = pl.s;
        std::memset(&s, 0, sizeof(s));
        // tables: the scan's DC and AC tables in force
        std::memset(pl.tables, 0, sizeof(pl.tables));
        for (int t = 0; t < 8; ++t)
            for (int l = 0; l < 18; ++l) pl.tables[t].maxcode[l] = -1;
        bool built[8] = {};
        for (const ScanComp& c : sc.comps) {
            for (int cls = 0; cls < 2; ++cls) {
                const int id = cls ? 4 + c.ta : c.td;
                if (built[id]) continue;
                HuffDec& h = pl.hdec[id];
                const HuffSpec& spec = cls ? sc.ac[c.ta] : sc.dc[c.td];
                if (!build_dec(spec, h)) return OILPAINT_ERR_ARG;
                to_dev_table(spec, h, pl.tables[id]);
                built[id] = true;
            }
        }
        // the MCU: every scan component's blocks in turn
        int j = 0;
        s.ns = (int)sc.comps.size();
        const bool inter = s.ns > 1;
        for (int k = 0; k < s.ns; ++k) {
            const ScanComp& c = sc.comps[k];
            const int hh = inter ? f.h[c.comp] : 1, vv = inter ? f.v[c.comp] : 1;
            s.off[k] = j;
            s.nb[k] = hh * vv;
            if (j + hh * vv > kJpegMaxMcuBlocks) return OILPAINT_ERR_ARG;  // T.81 B.2.3: at most 10
            for (int v = 0; v < vv; ++v)
                for (int h = 0; h < hh; ++h, ++j) {
                    s.comp[j] = c.comp;
                    s.dx[j] = h;
                    s.dy[j] = v;
                    s.dct[j] = c.td;
                    s.act[j] = c.ta;
                }
            s.h[c.comp] = hh;
            s.v[c.comp] = vv;
        }
        for (int c = 0; c < f.ncomp; ++c) {
            s.bw[c] = f.bw[c];
            s.first[c] = f.first[c];
        }
        s.bpm = j;
        for (int b = 0; b < j; ++b) {
            s.dsel |= (uint32_t)s.dct[b] << (2 * b);
            s.asel |= (uint32_t)s.act[b] << (2 * b);
        }
        s.mcux = inter ? f.mcux : f.own_bw[sc.comps[0].comp];
        s.mcus = inter ? (int64_t)f.mcux * f.mcuy
                       : (int64_t)f.own_bw[sc.comps[0].comp] * f.own_bh[sc.comps[0].comp];
        s.blocks = s.mcus * s.bpm;
        s.restart = f.restart;
        // the data, word aligned, and its restart intervals
        bytes.resize(align_up(bytes.size(), 4));
        pl.words_off = bytes.size();
        std::vector<size_t> starts;
        strip_scan(data, sc, bytes, starts);
        bytes.insert(bytes.end(), 16, 0);  // readable words past the end
        s.nwords = (int64_t)((bytes.size() - pl.words_off) / 4);
        const int64_t nseg = f.restart ? (s.mcus + f.restart - 1) / f.restart : 1;
        if ((int64_t)starts.size() - 1 < nseg) return OILPAINT_ERR_ARG;  // a restart marker is missing
        const uint64_t sub_bits = fixed_bits ? fixed_bits : auto_sub_bits(8 * (uint64_t)(starts.back() - starts.front()));
        pl.segs.reserve((size_t)nseg);
        pl.subs.reserve((size_t)nseg + 8 * (starts.back() - starts.front()) / sub_bits + 1);
        for (int64_t g = 0; g < nseg; ++g) {
            JpegSeg seg;
            seg.first_block = (f.restart ? g * f.restart : 0) * s.bpm;
            seg.end_block = std::min<int64_t>(s.mcus, f.restart ? (g + 1) * f.restart : s.mcus) * s.bpm;
            seg.first_sub = (int32_t)pl.subs.size();
            seg.pad = 0;
            pl.segs.push_back(seg);
            const uint64_t b0 = 8 * (uint64_t)(starts[g] - starts[0]);
            const uint64_t b1 = 8 * (uint64_t)(starts[g + 1] - starts[0]);
            const uint64_t n = std::max<uint64_t>(1, (b1 - b0 + sub_bits - 1) / sub_bits);
            for (uint64_t q = 0; q < n; ++q) {
                JpegSub sb;
                sb.begin = b0 + q * sub_bits;
                sb.end = q + 1 == n ? b1 : b0 + (q + 1) * sub_bits;
                sb.seg_end = b1;
                sb.seg = (int32_t)g;
                sb.flags = (q == 0 ? 1 : 0) | (q + 1 == n ? 2 : 0);
                pl.subs.push_back(sb);
            }
        }
        if (pl.subs.size() > (size_t)INT32_MAX / 2) return OILPAINT_ERR_UNSUPPORTED;
        s.nsub = (int32_t)pl.subs.size();
        s.check_bits = (int32_t)std::min<uint64_t>(kJpegCheckBits, sub_bits / 2);
        pl.sub_bits = (int)sub_bits;
    }
    // tables, subsequences and intervals after the data
    size_t off = align_up(bytes.size(), 16);
    for (ScanPlan& pl : plans) {
        pl.tables_off = off;
        off += sizeof(pl.tables);
        pl.subs_off = off = align_up(off, 16);
        off += pl.subs.size() * sizeof(JpegSub);
        pl.segs_off = off = align_up(off, 16);
        off += pl.segs.size() * sizeof(JpegSeg);
        off = align_up(off, 16);
    }
    *stage_bytes = off;
    return OILPAINT_OK;
}

// The device's decoding step on the host, for the subsequences whose true
// decoding meets no track: the same state (bit, block of the MCU,
// coefficient), the same tables and rules, over the same stripped data.
struct HostStepper {
    const uint8_t* data;  // the scan's stripped bytes, 16 zero bytes after
    const ScanPlan* pl;
    uint32_t peek32(uint64_t p, uint64_t end) const {
        if (p >= end) return 0u;
        const uint8_t* b = data + (p >> 3);
        const uint64_t x = (uint64_t)b[0] << 32 | (uint64_t)b[1] << 24 | (uint64_t)b[2] << 16 | (uint64_t)b[3] << 8 | b[4];
        uint32_t v = (uint32_t)(x >> (8 - (p & 7)));
        if (end - p < 32) v &= 0xFFFFFFFFu << (32 - (uint32_t)(end - p));
        return v;
    }
    static int lookup(const HuffDec& t, uint32_t top, uint32_t& len) {
        const uint32_t e = t.fast[top >> 7];
        if (e) {
            len = e >> 8;
            return (int)(e & 255u);
        }
        for (uint32_t l = 10; l <= 16; ++l) {
            const int32_t code = (int32_t)(top >> (16 - l));
            if (code <= t.maxcode[l]) {
                len = l;
                return t.vals[(code + t.valoff[l]) & 255];
            }
        }
        len = 1;
        return -1;
    }
    // One symbol; false for a malformed code (the state then moves one bit).
    bool step(uint64_t& p, uint32_t& j, uint32_t& z, uint32_t& done, uint64_t end) const {
        const JpegDecScan& s = pl->s;
        const uint32_t v = peek32(p, end);
        uint32_t len;
        if (z == 0) {
            const int cat = lookup(pl->hdec[s.dct[j]], v >> 16, len);
            if (cat < 0 || cat > 11) {
                p += 1;
                return false;
            }
            p += len + (uint32_t)cat;
            z = 1;
        } else {
            const int rs = lookup(pl->hdec[4 + s.act[j]], v >> 16, len);
            if (rs < 0) {
                p += 1;
                return false;
            }
            const uint32_t r = (uint32_t)rs >> 4, sz = (uint32_t)rs & 15u;
            if (sz == 0) {
                p += len;
                z = r == 15 ? z + 16 : 64;
            } else {
                if (z + r > 63 || sz > 10) {
                    p += 1;
                    return false;
                }
                p += len + sz;
                z += r + 1;
            }
        }
        if (z >= 64) {
            z = 0;
            j = j + 1 == (uint32_t)s.bpm ? 0u : j + 1;
            ++done;
        }
        return true;
    }
    // Decode from `state` until the position reaches `until`; the blocks
    // completed.
    uint32_t run_until(uint64_t& state, uint64_t seg_end, uint64_t until) const {
        uint64_t p = state >> 16;
        uint32_t j = (uint32_t)(state >> 8) & 255u, z = (uint32_t)state & 255u, done = 0;
        while (p < until) (void)step(p, j, z, done, seg_end);
        state = p << 16 | (uint64_t)j << 8 | z;
        return done;
    }
};

// Follow the links from every restart interval's start: the two parts of
// every subsequence's true decoding into entries[2i], entries[2i + 1].
void walk_links(const ScanPlan& pl, const uint8_t* data, const JpegTrack* tracks, const JpegLink* links,
                JpegEntry* entries) {
    const int nt = 2 * pl.s.bpm;
    const uint64_t ck = (uint64_t)pl.s.check_bits;
    const HostStepper hs{data, &pl};
    for (const JpegSeg& seg : pl.segs) {
        int i = seg.first_sub;
        uint64_t state = pl.subs[i].begin << 16;  // block 0, its DC: track 0
        int u = 0;
        uint32_t pre = tracks[(size_t)i * nt].pre;
        int64_t block = seg.first_block;
        for (;; ++i) {
            const JpegSub& sub = pl.subs[i];
            JpegEntry& a = entries[2 * (size_t)i];
            JpegEntry& b = entries[2 * (size_t)i + 1];
            a.state = state;
            a.block = block;
            b.block = -1;
            b.state = 0;
            b.stop = 0;
            if (sub.flags & 2) {
                a.stop = kJpegStopAtBlocks;
                break;
            }
            const JpegSub& nx = pl.subs[i + 1];
            uint32_t blocks;
            if (u >= 0) {  // the true decoding follows track u from its checkpoint
                const JpegTrack& t = tracks[(size_t)i * nt + u];
                const JpegLink& l = links[(size_t)i * nt + u];
                a.stop = sub.begin + ck;
                b.state = t.check;
                b.block = block + pre;
                b.stop = sub.end;
                blocks = pre + t.post;
                state = t.exit;
                u = l.next == kJpegNoTrack ? -1 : (int)l.next;
                pre = l.blocks;
            } else {  // no track: decode this subsequence here, in one part there
                a.stop = sub.end;
                blocks = hs.run_until(state, sub.seg_end, sub.end);
                uint64_t probe = state;
                pre = hs.run_until(probe, nx.seg_end, nx.begin + ck);
                for (int v = 0; v < nt; ++v)
                    if (tracks[(size_t)(i + 1) * nt + v].check == probe) {
                        u = v;
                        break;
                    }
            }
            block += blocks;
        }
    }
}

// Entropy-decode every scan on the device into jd.coef (zeroed first; the
// blocks no scan covers stay 0).  Waits for each scan's tracks and, at the
// end, for the decoding, to report a malformed stream.
int device_entropy_decode(const uint8_t* data, const Frame& f, JpegDevice& jd, int device, hipStream_t s,
                          double* host_ms, std::chrono::steady_clock::time_point t0) {
    // kept from call to call on each thread (their pages stay mapped)
    static thread_local std::vector<ScanPlan> plans;
    static thread_local std::vector<uint8_t> bytes;
    bytes.clear();
    bytes.reserve(f.scans.empty() ? 0 : f.scans.back().end - f.scans.front().begin + 64 * f.scans.size());
    size_t total = 0;
    int st = plan_scans(data, f, plans, bytes, &total);
    if (st != OILPAINT_OK) return st;
    if ((st = jd.reserve_stage(total)) != OILPAINT_OK) return st;
    std::memcpy(jd.stage, bytes.data(), bytes.size());
    size_t max_sub = 1, max_tracks = 1;
    for (ScanPlan& pl : plans) {
        std::memcpy(jd.stage + pl.tables_off, pl.tables, sizeof(pl.tables));
        std::memcpy(jd.stage + pl.subs_off, pl.subs.data(), pl.subs.size() * sizeof(JpegSub));
        std::memcpy(jd.stage + pl.segs_off, pl.segs.data(), pl.segs.size() * sizeof(JpegSeg));
        max_sub = std::max(max_sub, pl.subs.size());
        max_tracks = std::max(max_tracks, pl.subs.size() * 2 * (size_t)pl.s.bpm);
    }
    double host = ms_since(t0);
    if ((st = jd.reserve_coder(device)) != OILPAINT_OK) return st;
    const size_t nblk = std::max<size_t>(f.blocks, 1);
    if ((st = JpegDevice::grow(jd.tracks, jd.tracks_cap, max_tracks)) != OILPAINT_OK ||
        (st = JpegDevice::grow(jd.links, jd.links_cap, max_tracks)) != OILPAINT_OK ||
        (st = JpegDevice::grow(jd.entries, jd.entries_cap, 2 * max_sub)) != OILPAINT_OK ||
        (st = JpegDevice::grow(jd.dcdiff, jd.dcdiff_cap, 2 * nblk)) != OILPAINT_OK ||
        (st = JpegDevice::grow(jd.dsum, jd.dsum_cap, nblk)) != OILPAINT_OK ||
        (st = JpegDevice::grow(jd.tiles, jd.tiles_cap, (size_t)huff_scan_tiles((int64_t)nblk))) != OILPAINT_OK ||
        (st = jd.reserve_hwork(max_tracks * (sizeof(JpegTrack) + sizeof(JpegLink)) + 2 * max_sub * sizeof(JpegEntry))) !=
            OILPAINT_OK)
        return st;
    if (!jd.dflags && hipMalloc(reinterpret_cast<void**>(&jd.dflags), 16) != hipSuccess) return OILPAINT_ERR_NOMEM;
    if (note_hip("hipMemcpyAsync", hipMemcpyAsync(jd.dstage, jd.stage, total, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        note_hip("hipMemsetAsync", hipMemsetAsync(jd.coef, 0, f.blocks * 64 * sizeof(int16_t), s)) != hipSuccess ||
        note_hip("hipMemsetAsync", hipMemsetAsync(jd.dflags, 0, 16, s)) != hipSuccess)
        return OILPAINT_ERR_HIP;
    JpegTrack* htracks = reinterpret_cast<JpegTrack*>(jd.hwork);
    JpegLink* hlinks = reinterpret_cast<JpegLink*>(jd.hwork + max_tracks * sizeof(JpegTrack));
    JpegEntry* hentries =
        reinterpret_cast<JpegEntry*>(jd.hwork + max_tracks * (sizeof(JpegTrack) + sizeof(JpegLink)));
    for (ScanPlan& pl : plans) {
        JpegDecScan sc = pl.s;
        sc.words = reinterpret_cast<const uint32_t*>(jd.dstage + pl.words_off);
        sc.tables = reinterpret_cast<const JpegHuffTable*>(jd.dstage + pl.tables_off);
        sc.subs = reinterpret_cast<const JpegSub*>(jd.dstage + pl.subs_off);
        sc.segs = reinterpret_cast<const JpegSeg*>(jd.dstage + pl.segs_off);
        sc.coef = jd.coef;
        sc.dcdiff = jd.dcdiff;
        const size_t ntr = pl.subs.size() * 2 * (size_t)pl.s.bpm;
        // the tracks come down on the side stream while the links decode
        if (launch_huff_tracks(sc, pl.sub_bits, jd.tracks, jd.links, jd.tracks_done, s) != hipSuccess ||
            note_hip("hipStreamWaitEvent", hipStreamWaitEvent(jd.side, jd.tracks_done, 0)) != hipSuccess ||
            note_hip("hipMemcpyAsync", hipMemcpyAsync(htracks, jd.tracks, ntr * sizeof(JpegTrack),
                                                      hipMemcpyDeviceToHost, jd.side)) != hipSuccess ||
            note_hip("hipMemcpyAsync", hipMemcpyAsync(hlinks, jd.links, ntr * sizeof(JpegLink),
                                                      hipMemcpyDeviceToHost, s)) != hipSuccess ||
            note_hip("hipStreamSynchronize", hipStreamSynchronize(s)) != hipSuccess ||
            note_hip("hipStreamSynchronize", hipStreamSynchronize(jd.side)) != hipSuccess)
            return OILPAINT_ERR_HIP;
        const auto t1 = std::chrono::steady_clock::now();
        walk_links(pl, bytes.data() + pl.words_off, htracks, hlinks, hentries);
        host += ms_since(t1);
        if (note_hip("hipMemcpyAsync", hipMemcpyAsync(jd.entries, hentries, 2 * pl.subs.size() * sizeof(JpegEntry),
                                                      hipMemcpyHostToDevice, s)) != hipSuccess ||
            launch_huff_decode(sc, pl.sub_bits, jd.entries, jd.dflags, jd.tiles, reinterpret_cast<uint64_t*>(jd.dflags + 2),
                               jd.dcdiff + nblk, jd.dsum, s) != hipSuccess)
            return OILPAINT_ERR_HIP;
    }
    uint32_t* flags_host = reinterpret_cast<uint32_t*>(jd.small_host->totals);
    if (note_hip("hipMemcpyAsync", hipMemcpyAsync(flags_host, jd.dflags, 4, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        note_hip("hipStreamSynchronize", hipStreamSynchronize(s)) != hipSuccess)
        return OILPAINT_ERR_HIP;
    if (host_ms) *host_ms = host;
    return flags_host[0] ? OILPAINT_ERR_ARG : OILPAINT_OK;
}

// Parse, entropy-decode on the device and start the inverse DCT on `stream`;
// planes as given (device pointers, component samples only) or the
// library's own (whole padded grids).
int decode_to_planes(const uint8_t* data, size_t len, JpegDevice& jd, int device, Frame& f, uint8_t* const* user_planes,
                     const int* user_strides, hipStream_t stream, double* host_ms) {
    const auto t0 = std::chrono::steady_clock::now();
    int st = parse_frame(data, len, f);
    if (st != OILPAINT_OK) return st;
    uint8_t* lib_planes[kJpegMaxComps];
    int32_t lib_strides[kJpegMaxComps];
    size_t plane_bytes = 0;
    plane_layout(f, nullptr, lib_planes, lib_strides, &plane_bytes);
    if ((st = jd.wait()) != OILPAINT_OK) return st;
    if ((st = jd.reserve(f.blocks * 64, user_planes ? 0 : plane_bytes)) != OILPAINT_OK) return st;
    if ((st = device_entropy_decode(data, f, jd, device, stream, host_ms, t0)) != OILPAINT_OK) return st;
    JpegIdctArgs a = idct_args(f, jd.coef);
    if (user_planes) {
        for (int c = 0; c < f.ncomp; ++c) {
            a.plane[c] = user_planes[c];
            a.stride[c] = user_strides[c];
            a.limit_w[c] = f.xc[c];
            a.limit_h[c] = f.yc[c];
        }
    } else {
        plane_layout(f, jd.planes, lib_planes, lib_strides, &plane_bytes);
        for (int c = 0; c < f.ncomp; ++c) {
            a.plane[c] = lib_planes[c];
            a.stride[c] = lib_strides[c];
            a.limit_w[c] = f.bw[c] * 8;
            a.limit_h[c] = f.bh[c] * 8;
        }
    }
    if (launch_jpeg_idct(a, stream) != hipSuccess) return OILPAINT_ERR_HIP;
    return OILPAINT_OK;
}

}  // namespace
}  // namespace oilpaint_impl

using namespace oilpaint_impl;

extern "C" {

int oilpaint_jpeg_header(const uint8_t* data, size_t len, oilpaint_jpeg_info* info) {
    if (!data || !info) return OILPAINT_ERR_NULL;
    Frame f;
    const int st = parse_frame(data, len, f);
    if (st != OILPAINT_OK) return st;
    fill_info(f, info);
    return OILPAINT_OK;
}

int oilpaint_jpeg_coefficients(const uint8_t* data, size_t len, int16_t* coef, size_t capacity, size_t* count) {
    if (!data || !count) return OILPAINT_ERR_NULL;
    Frame f;
    int st = parse_frame(data, len, f);
    if (st != OILPAINT_OK) return st;
    *count = f.blocks * 64;
    if (!coef || capacity < f.blocks * 64) return OILPAINT_ERR_NOMEM;
    return entropy_decode(data, f, coef);
}

int oilpaint_jpeg_encode_info(int width, int height, int quality, int subsampling, oilpaint_jpeg_info* info) {
    if (!info) return OILPAINT_ERR_NULL;
    Frame f;
    const int st = encode_frame(width, height, quality, subsampling, f);
    if (st != OILPAINT_OK) return st;
    fill_info(f, info);
    return OILPAINT_OK;
}

int oilpaint_jpeg_write(const int16_t* coef, int width, int height, int quality, int subsampling, uint8_t* out,
                        size_t capacity, size_t* out_len) {
    if (!coef || !out_len) return OILPAINT_ERR_NULL;
    Frame f;
    const int st = encode_frame(width, height, quality, subsampling, f);
    if (st != OILPAINT_OK) return st;
    std::vector<uint8_t> bytes;
    bytes.reserve(f.blocks * 16 + 1024);
    entropy_encode(f, coef, bytes);
    *out_len = bytes.size();
    if (!out || bytes.size() > capacity) return OILPAINT_ERR_NOMEM;
    std::memcpy(out, bytes.data(), bytes.size());
    return OILPAINT_OK;
}

int oilpaint_jpeg_decode(const uint8_t* data, size_t len, uint8_t* dst, int dst_stride, void* stream,
                         double* host_ms) {
    if (!data || !dst) return OILPAINT_ERR_NULL;
    int device = 0;
    if (note_hip("hipGetDevice", hipGetDevice(&device)) != hipSuccess) return OILPAINT_ERR_HIP;
    Frame hdr;
    int st = parse_frame(data, len, hdr);
    if (st != OILPAINT_OK) return st;
    if (dst_stride < 3 * hdr.width) return OILPAINT_ERR_ARG;
    if ((st = check_device_ptr(dst)) != OILPAINT_OK) return st;
    JpegDevice& jd = jpeg_device(device);
    std::lock_guard<std::mutex> lock(jd.mu);
    const hipStream_t s = (hipStream_t)stream;
    Frame f;
    if ((st = decode_to_planes(data, len, jd, device, f, nullptr, nullptr, s, host_ms)) != OILPAINT_OK) return st;
    JpegColorArgs c;
    std::memset(&c, 0, sizeof(c));
    uint8_t* planes[kJpegMaxComps];
    int32_t strides[kJpegMaxComps];
    size_t bytes = 0;
    plane_layout(f, jd.planes, planes, strides, &bytes);
    for (int k = 0; k < f.ncomp; ++k) {
        c.plane[k] = planes[k];
        c.stride[k] = strides[k];
        c.h[k] = f.h[k];
        c.v[k] = f.v[k];
    }
    c.hmax = f.hmax;
    c.vmax = f.vmax;
    c.ncomp = f.ncomp;
    c.width = f.width;
    c.height = f.height;
    c.dst = dst;
    c.dst_stride = dst_stride;
    if (launch_jpeg_color(c, s) != hipSuccess) return OILPAINT_ERR_HIP;
    return jd.mark(s);
}

int oilpaint_jpeg_decode_planes(const uint8_t* data, size_t len, uint8_t* const* planes, const int* strides,
                                void* stream, double* host_ms) {
    if (!data || !planes || !strides) return OILPAINT_ERR_NULL;
    int device = 0;
    if (note_hip("hipGetDevice", hipGetDevice(&device)) != hipSuccess) return OILPAINT_ERR_HIP;
    Frame hdr;
    int st = parse_frame(data, len, hdr);
    if (st != OILPAINT_OK) return st;
    for (int c = 0; c < hdr.ncomp; ++c) {
        if (!planes[c]) return OILPAINT_ERR_NULL;
        if (strides[c] < hdr.xc[c]) return OILPAINT_ERR_ARG;
        if ((st = check_device_ptr(planes[c])) != OILPAINT_OK) return st;
    }
    JpegDevice& jd = jpeg_device(device);
    std::lock_guard<std::mutex> lock(jd.mu);
    const hipStream_t s = (hipStream_t)stream;
    Frame f;
    if ((st = decode_to_planes(data, len, jd, device, f, planes, strides, s, host_ms)) != OILPAINT_OK) return st;
    return jd.mark(s);
}

int oilpaint_jpeg_set_subsequence_bits(int bits) {
    if (bits != 0 && (bits < 64 || bits > kJpegMaxSubBits)) return OILPAINT_ERR_ARG;
    g_sub_bits.store(bits);
    return OILPAINT_OK;
}

size_t oilpaint_jpeg_encode_bound(int width, int height) {
    if (width <= 0 || height <= 0) return 0;
    const size_t blocks = (size_t)((width + 15) / 16) * ((height + 15) / 16) * 6 * 2;  // up to 4:4:4
    return 1024 + 4 * 17 * 2 + 4 * 256 + blocks * 64 * 8;
}

int oilpaint_jpeg_encode(const uint8_t* src, int width, int height, int stride, int quality, int subsampling,
                         uint8_t* out, size_t capacity, size_t* out_len, void* stream, double* host_ms) {
    if (!src || !out_len) return OILPAINT_ERR_NULL;
    Frame f;
    int st = encode_frame(width, height, quality, subsampling, f);
    if (st != OILPAINT_OK) return st;
    if (stride < 3 * width) return OILPAINT_ERR_ARG;
    const int hl = f.hmax, vl = f.vmax;
    int device = 0;
    if (note_hip("hipGetDevice", hipGetDevice(&device)) != hipSuccess) return OILPAINT_ERR_HIP;
    if ((st = check_device_ptr(src)) != OILPAINT_OK) return st;
    JpegDevice& jd = jpeg_device(device);
    std::lock_guard<std::mutex> lock(jd.mu);
    const hipStream_t s = (hipStream_t)stream;
    uint8_t* planes[kJpegMaxComps];
    int32_t strides[kJpegMaxComps];
    size_t plane_bytes = 0;
    plane_layout(f, nullptr, planes, strides, &plane_bytes);
    if ((st = jd.wait()) != OILPAINT_OK) return st;
    if ((st = jd.reserve(f.blocks * 64, plane_bytes)) != OILPAINT_OK) return st;
    plane_layout(f, jd.planes, planes, strides, &plane_bytes);
    JpegRgbArgs r;
    std::memset(&r, 0, sizeof(r));
    r.src = src;
    r.stride = stride;
    r.width = width;
    r.height = height;
    r.ymcu_w = f.bw[0] * 8;
    r.ymcu_h = f.bh[0] * 8;
    r.fh = hl;
    r.fv = vl;
    JpegFdctArgs q;
    std::memset(&q, 0, sizeof(q));
    for (int c = 0; c < 3; ++c) {
        r.plane[c] = planes[c];
        r.pstride[c] = strides[c];
        q.plane[c] = planes[c];
        q.stride[c] = strides[c];
        q.bw[c] = f.bw[c];
        std::memcpy(q.q[c], f.q[f.tq[c]], sizeof(q.q[c]));
    }
    for (int c = 0; c <= 3; ++c) q.first[c] = f.first[c];
    q.coef = jd.coef;
    if (launch_jpeg_rgb(r, s) != hipSuccess || launch_jpeg_fdct(q, s) != hipSuccess) return OILPAINT_ERR_HIP;
    // symbol statistics on the device, the tables fitted here
    if ((st = jd.reserve_coder(device)) != OILPAINT_OK) return st;
    JpegDevice::Small* dev = jd.small;
    JpegDevice::Small* hs = jd.small_host;
    const JpegScanMap m = scan_map(f);
    if (note_hip("hipMemsetAsync", hipMemsetAsync(dev->freq, 0, sizeof(dev->freq), s)) != hipSuccess ||
        launch_huff_stats(m, jd.coef, dev->freq, jd.cus, s) != hipSuccess ||
        note_hip("hipMemcpyAsync", hipMemcpyAsync(hs->freq, dev->freq, sizeof(hs->freq), hipMemcpyDeviceToHost,
                                                  s)) != hipSuccess ||
        note_hip("hipStreamSynchronize", hipStreamSynchronize(s)) != hipSuccess)
        return OILPAINT_ERR_HIP;
    const auto t0 = std::chrono::steady_clock::now();
    HuffEnc dc[2], ac[2];
    int64_t freq[4 * 256];
    for (int i = 0; i < 4 * 256; ++i) freq[i] = (int64_t)hs->freq[i];
    uint64_t nbits = 0;
    for (int t = 0; t < 2; ++t) {
        fit_table(freq + t * 256, dc[t]);
        fit_table(freq + (2 + t) * 256, ac[t]);
        for (int sym = 0; sym < 256; ++sym) {
            nbits += (uint64_t)freq[t * 256 + sym] * (uint64_t)(dc[t].size[sym] + sym);
            nbits += (uint64_t)freq[(2 + t) * 256 + sym] * (uint64_t)(ac[t].size[sym] + (sym & 15));
        }
    }
    for (int t = 0; t < 4; ++t) {
        const HuffEnc& h = t < 2 ? dc[t] : ac[t - 2];
        for (int sym = 0; sym < 256; ++sym) hs->tabs[t * 256 + sym] = (uint32_t)h.size[sym] << 16 | h.code[sym];
    }
    std::vector<uint8_t> head;
    write_headers(f, dc, ac, head);
    if (host_ms) *host_ms = ms_since(t0);
    // the coding passes
    const uint64_t nbytes = (nbits + 7) / 8;
    const size_t nwords = (size_t)(nbits / 32) + 2;
    if ((st = JpegDevice::grow(jd.bits, jd.bits_cap, (size_t)m.blocks)) != OILPAINT_OK ||
        (st = JpegDevice::grow(jd.offset, jd.offset_cap, (size_t)m.blocks)) != OILPAINT_OK ||
        (st = JpegDevice::grow(jd.tiles, jd.tiles_cap,
                               (size_t)std::max(huff_scan_tiles(m.blocks), huff_scan_tiles((int64_t)nbytes)))) !=
            OILPAINT_OK ||
        (st = JpegDevice::grow(jd.words, jd.words_cap, nwords)) != OILPAINT_OK ||
        (st = JpegDevice::grow(jd.stuffed, jd.stuffed_cap, (size_t)(2 * nbytes + 16))) != OILPAINT_OK ||
        (st = jd.reserve_hwork((size_t)(2 * nbytes + 16))) != OILPAINT_OK)
        return st;
    if (note_hip("hipMemcpyAsync", hipMemcpyAsync(dev->tabs, hs->tabs, sizeof(hs->tabs), hipMemcpyHostToDevice,
                                                  s)) != hipSuccess ||
        note_hip("hipMemsetAsync", hipMemsetAsync(jd.words, 0, nwords * sizeof(uint32_t), s)) != hipSuccess ||
        launch_huff_code(m, jd.coef, dev->tabs, jd.bits, jd.offset, jd.tiles, &dev->totals[0], jd.words, jd.cus, s) !=
            hipSuccess ||
        launch_huff_stuff(jd.words, nbits, jd.tiles, &dev->totals[1], jd.stuffed, s) != hipSuccess ||
        note_hip("hipMemcpyAsync", hipMemcpyAsync(hs->totals, dev->totals, sizeof(hs->totals),
                                                  hipMemcpyDeviceToHost, s)) != hipSuccess)
        return OILPAINT_ERR_HIP;
    // The stuffed stream's whole room (twice the bytes, the most stuffing can
    // make) comes down into pinned memory in the same wait as the totals,
    // which say how much of it is the stream.
    if (note_hip("hipMemcpyAsync", hipMemcpyAsync(jd.hwork, jd.stuffed, 2 * (size_t)nbytes, hipMemcpyDeviceToHost,
                                                  s)) != hipSuccess ||
        note_hip("hipStreamSynchronize", hipStreamSynchronize(s)) != hipSuccess)
        return OILPAINT_ERR_HIP;
    if (hs->totals[0] != nbits) {
        note_error("oilpaint_jpeg_encode: the device's bit count disagrees with the symbol statistics");
        return OILPAINT_ERR_HIP;
    }
    const size_t data = (size_t)(nbytes + hs->totals[1]);
    *out_len = head.size() + data + 2;
    if (!out || *out_len > capacity) return OILPAINT_ERR_NOMEM;
    std::memcpy(out, head.data(), head.size());
    std::memcpy(out + head.size(), jd.hwork, data);
    out[*out_len - 2] = 0xFF;
    out[*out_len - 1] = 0xD9;
    return OILPAINT_OK;
}

}  // extern "C"
