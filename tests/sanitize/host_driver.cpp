// The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_host_sanitizers.py builds it with the host half instrumented and
// runs it without a GPU): status strings, and the host JPEG codec -- header
// parsing and entropy decoding of the files named on the command line and of
// truncated and corrupted copies of them, entropy encoding of random
// coefficients read back by the decoder.  Any sanitizer report ends the run
// with a non-zero status; so does a wrong result.
#include "oilpaint.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

int failures = 0;

#define EXPECT(c)                                                              \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "%s:%d: failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

// xorshift64*: a small seeded generator for the mutations and coefficients
struct Rng {
    uint64_t s;
    uint64_t next() {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        return s * 0x2545F4914F6CDD1Dull;
    }
    uint32_t below(uint32_t n) { return (uint32_t)(next() >> 33) % n; }
};

// Coefficient budget of one decode here: larger claimed frames are only
// checked for the capacity refusal.
constexpr int64_t kMaxCoefs = int64_t(1) << 22;

// Header and entropy decoding of one (possibly malformed) file: any status
// the header documents is fine; a frame that parses must decode into exactly
// its blocks, and a short buffer must be refused untouched.
void decode_once(const std::vector<uint8_t>& d, int* parsed) {
    oilpaint_jpeg_info info;
    const int st = oilpaint_jpeg_header(d.data(), d.size(), &info);
    if (d.empty()) {  // no bytes: a null data pointer
        EXPECT(st == OILPAINT_ERR_NULL);
        return;
    }
    if (!(st == OILPAINT_OK || st == OILPAINT_ERR_ARG || st == OILPAINT_ERR_UNSUPPORTED))
        std::fprintf(stderr, "header status %d, %zu bytes\n", st, d.size());
    EXPECT(st == OILPAINT_OK || st == OILPAINT_ERR_ARG || st == OILPAINT_ERR_UNSUPPORTED);
    if (st != OILPAINT_OK) return;
    ++*parsed;
    EXPECT(info.blocks > 0 && info.components >= 1 && info.components <= 3);
    int16_t small[64];
    std::memset(small, 0x5A, sizeof(small));
    size_t count = 0;
    const int s2 = oilpaint_jpeg_coefficients(d.data(), d.size(), small, 63, &count);
    EXPECT(s2 != OILPAINT_OK);
    for (int16_t v : small) EXPECT(v == 0x5A5A);
    if (info.blocks * 64 > kMaxCoefs) return;
    std::vector<int16_t> coef((size_t)info.blocks * 64 + 64, (int16_t)0x7777);
    const int s3 = oilpaint_jpeg_coefficients(d.data(), d.size(), coef.data(), (size_t)info.blocks * 64, &count);
    EXPECT(s3 == OILPAINT_OK || s3 == OILPAINT_ERR_ARG || s3 == OILPAINT_ERR_UNSUPPORTED);
    if (s3 == OILPAINT_OK) EXPECT(count == (size_t)info.blocks * 64);
    for (size_t i = (size_t)info.blocks * 64; i < coef.size(); ++i) EXPECT(coef[i] == (int16_t)0x7777);
}

void fuzz_file(const char* path, Rng& rng) {
    FILE* f = std::fopen(path, "rb");
    if (!f) {
        std::fprintf(stderr, "cannot open %s\n", path);
        ++failures;
        return;
    }
    std::vector<uint8_t> d;
    int c;
    while ((c = std::fgetc(f)) != EOF) d.push_back((uint8_t)c);
    std::fclose(f);
    int parsed = 0;
    decode_once(d, &parsed);
    EXPECT(parsed == 1);  // the file itself is well formed
    // every truncation near the ends, a spread of them in between
    const size_t n = d.size();
    const size_t step = n > 400 ? n / 200 : 1;
    for (size_t len = 0; len <= n; len += (len < 64 || len + 64 > n) ? 1 : step) {
        std::vector<uint8_t> t(d.begin(), d.begin() + (ptrdiff_t)len);
        decode_once(t, &parsed);
    }
    // single-byte corruptions, most of them in the headers
    for (int k = 0; k < 3000; ++k) {
        std::vector<uint8_t> m = d;
        const size_t span = (k & 3) ? std::min<size_t>(n, 640) : n;
        const size_t pos = rng.below((uint32_t)span);
        if (k & 1)
            m[pos] ^= (uint8_t)(1u << rng.below(8));
        else
            m[pos] = (uint8_t)rng.below(256);
        decode_once(m, &parsed);
    }
    // a few bytes deleted or duplicated
    for (int k = 0; k < 400; ++k) {
        std::vector<uint8_t> m = d;
        const size_t pos = rng.below((uint32_t)n);
        if (k & 1)
            m.erase(m.begin() + (ptrdiff_t)pos);
        else
            m.insert(m.begin() + (ptrdiff_t)pos, m[pos]);
        decode_once(m, &parsed);
    }
    std::printf("%s: %zu bytes, %d variants parsed\n", path, n, parsed);
}

// Host entropy encoding of random coefficients (DC within +-1000, sparse AC
// within +-1023, so every symbol is codable) read back bit-exact; a buffer
// one byte short is refused untouched.
void encode_roundtrip(int w, int h, int quality, int subsampling, Rng& rng) {
    oilpaint_jpeg_info info;
    EXPECT(oilpaint_jpeg_encode_info(w, h, quality, subsampling, &info) == OILPAINT_OK);
    const size_t nc = (size_t)info.blocks * 64;
    std::vector<int16_t> coef(nc, 0);
    for (size_t b = 0; b < (size_t)info.blocks; ++b) {
        coef[b * 64] = (int16_t)((int)rng.below(2001) - 1000);
        const uint32_t density = rng.below(4);  // empty, sparse, denser, full blocks
        for (int k = 1; k < 64; ++k) {
            const bool on = density == 3 || (density > 0 && rng.below(8) < density);
            if (on) coef[b * 64 + k] = (int16_t)((int)rng.below(2047) - 1023);
        }
    }
    std::vector<uint8_t> out(oilpaint_jpeg_encode_bound(w, h) + 4096);
    size_t len = 0;
    const int st = oilpaint_jpeg_write(coef.data(), w, h, quality, subsampling, out.data(), out.size(), &len);
    EXPECT(st == OILPAINT_OK);
    if (st != OILPAINT_OK) return;
    std::vector<uint8_t> file(out.begin(), out.begin() + (ptrdiff_t)len);
    std::vector<int16_t> back(nc, 0);
    size_t count = 0;
    EXPECT(oilpaint_jpeg_coefficients(file.data(), file.size(), back.data(), nc, &count) == OILPAINT_OK);
    EXPECT(count == nc && back == coef);
    std::vector<uint8_t> shortbuf(len - 1, 0xA5);
    size_t len2 = 0;
    EXPECT(oilpaint_jpeg_write(coef.data(), w, h, quality, subsampling, shortbuf.data(), shortbuf.size(), &len2) ==
           OILPAINT_ERR_NOMEM);
    for (uint8_t v : shortbuf) EXPECT(v == 0xA5);
}

}  // namespace

int main(int argc, char** argv) {
    for (int s = -32; s <= 4; ++s) EXPECT(oilpaint_strerror(s) != nullptr && oilpaint_strerror(s)[0] != 0);
    EXPECT(oilpaint_version() > 0);
    oilpaint_jpeg_info info;
    EXPECT(oilpaint_jpeg_header(nullptr, 10, &info) != OILPAINT_OK);
    EXPECT(oilpaint_jpeg_header((const uint8_t*)"", 0, &info) != OILPAINT_OK);
    Rng rng{0x9E3779B97F4A7C15ull};
    for (int i = 1; i < argc; ++i) fuzz_file(argv[i], rng);
    const int sizes[][2] = {{1, 1}, {9, 7}, {33, 17}, {64, 48}, {130, 3}};
    for (const auto& s : sizes)
        for (int ss = 0; ss < 3; ++ss)
            for (int q : {1, 50, 100}) encode_roundtrip(s[0], s[1], q, ss, rng);
    std::printf("%d failures\n", failures);
    return failures ? 1 : 0;
}
