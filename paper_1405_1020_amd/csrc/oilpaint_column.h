// Device code of the column-histogram layout (OILPAINT_HIST_COLUMN), used by
// oilpaint_k_column.hip only.
#pragma once

#include "oilpaint_device.h"

namespace oilpaint_impl {
namespace dev {

// ---------------------------------------------------------------------------
// COLUMN layout (any radius up to 255): the window histogram of every lane
// from column histograms, with no per-radius work per output row.
// ---------------------------------------------------------------------------
// One wavefront per workgroup, 64 output columns, a run of rows.  LDS holds,
// for each of the 64+2r columns of the strip, the histogram of its 2r+1
// window rows (column histograms; L levels plus a sink row for outside
// pixels and the paper form's white level).  Per output row and level, an
// inclusive prefix sum of the column histograms across the strip -- a
// wavefront scan per 64 columns -- gives every lane its window as the
// difference of two prefix entries; the running maximum over levels (first
// strictly larger count wins, so the lowest level wins ties) is the mode.
// Moving one row down changes each column histogram by two pixels.
//   LDS: [column histograms: (L+1) x (64+2r) x 8 B][prefix: (64+2r+1) x 16 B]
//        [output row buffer: 192 B]
// Column histogram entry: count:13 @51 | sum2:17 @34 | sum1:17 @17 |
// sum0:17 @0 (count <= 511, sums <= 130,305 for r <= 255).  Prefix entries
// and window sums are four 32-bit fields (window count <= 261,121, sums <=
// 66,585,855).

// Inclusive prefix sum over the 64 lanes of a wavefront: shifts within the
// 16-lane rows, then the last lane of each row broadcast into the next rows.
// Every lane must be active.
__device__ __forceinline__ uint32_t wave_scan_add(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

__device__ __forceinline__ uint64_t column_inc(uint32_t c0, uint32_t c1, uint32_t c2) {
    return (uint64_t)c0 | ((uint64_t)c1 << 17) | ((uint64_t)c2 << 34) | (1ull << 51);
}

struct Sums4 {
    uint32_t n, a, b, c;  // count, sum0, sum1, sum2
};

__device__ __forceinline__ Sums4 column_unpack(uint64_t e) {
    const uint32_t lo = (uint32_t)e, hi = (uint32_t)(e >> 32);
    Sums4 r;
    r.a = lo & 0x1FFFFu;
    r.b = (lo >> 17) | ((hi & 0x3u) << 15);
    r.c = (hi >> 2) & 0x1FFFFu;
    r.n = hi >> 19;
    return r;
}

// floor(s / n) for s < 2^27 and 1 <= n < 2^19: the product with the correctly
// rounded double reciprocal is within a tiny fraction of s/n, so truncating
// it gives the quotient or one less; the integer checks correct either way.
__device__ __forceinline__ uint32_t div_exact32(uint32_t s, uint32_t n, double rn) {
    uint32_t q = (uint32_t)((double)s * rn);
    q += ((q + 1u) * n <= s) ? 1u : 0u;
    q -= (q * n > s) ? 1u : 0u;
    return q;
}

// Three bytes of an image pixel at (gx, gy), coordinates clamped into the
// image (so the load needs no branch) and `in` telling whether it is real.
struct PixelBytes {
    uint32_t c0, c1, c2;
    bool in;
    __device__ __forceinline__ void load(const Job& j, int gx, int gy, bool valid) {
        in = valid && gy >= 0 && gy < j.height && gx >= 0 && gx < j.width;
        const int gyc = min(max(gy, 0), j.height - 1);
        const int gxc = min(max(gx, 0), j.width - 1);
        gsrc_t q = gsrc(j.src) + (size_t)gyc * (size_t)j.stride + 3 * gxc;
        c0 = q[0];
        c1 = q[1];
        c2 = q[2];
    }
    // column-histogram row: the level, or the sink (row L) for outside
    // pixels and the paper form's white level
    __device__ __forceinline__ uint32_t row(const Job& j) const {
        if (!in) return (uint32_t)j.levels;
        const uint32_t lev = level_of(c0 + c1 + c2, (uint32_t)j.levels, j.paper != 0);
        return lev >= (uint32_t)j.levels ? (uint32_t)j.levels : lev;
    }
};

// NT: 64-column chunks of the strip with its halo, ceil((64 + 2r) / 64).
template <int NT>
__device__ __forceinline__ void tile_column(const Job& j, int unit, uint8_t* lds) {
    const int R = j.radius;
    const int TW = 64 + 2 * R;
    const int L = j.levels;
    const int lane = threadIdx.x & 63;
    const int tx = unit % j.tiles_x;
    const int ty = unit / j.tiles_x;
    const int x0 = tx * 64;
    const int ya = j.row_begin + ty * j.rows;
    const int yb = min(ya + j.rows, j.row_end);
    const size_t chb = ((size_t)(L + 1) * TW * 8 + 15) & ~(size_t)15;
    uint8_t* ch = lds;
    uint32_t* P = reinterpret_cast<uint32_t*>(lds + chb);  // (TW + 1) entries of 4 words
    uint8_t* obuf = lds + chb + (size_t)(TW + 1) * 16;
    auto entry = [&](uint32_t row, int c) { return reinterpret_cast<uint64_t*>(ch + ((size_t)row * TW + c) * 8); };

    {
        const int n16 = (int)((size_t)(L + 1) * TW * 8 / 16);
        for (int e = lane; e < n16; e += 64) *reinterpret_cast<uint4*>(ch + (size_t)e * 16) = make_uint4(0u, 0u, 0u, 0u);
        if (lane == 0) *reinterpret_cast<uint4*>(P) = make_uint4(0u, 0u, 0u, 0u);
    }
    lds_order();
    // column histograms of rows ya-R .. ya+R, the (2R+1) x TW pixels spread
    // over the lanes (no two lanes of one instruction share a column)
    {
        // pixel p = base + 64 i sits at (p / TW, p % TW), tracked by steps of
        // 64 (TW >= 64, so one wrap at most); sixteen pixels per lane in
        // flight
        const int NP = (2 * R + 1) * TW;
        constexpr int CH = 16;
        int row = 0, col = lane;
        for (int base = lane; base < NP; base += CH * 64) {
            PixelBytes px[CH];
            int cl[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                cl[i] = col;
                px[i].load(j, x0 - R + col, ya - R + row, base + i * 64 < NP);
                col += 64;
                if (col >= TW) {
                    col -= TW;
                    ++row;
                }
            }
#pragma unroll
            for (int i = 0; i < CH; ++i)
                if (base + i * 64 < NP)
                    lds_add(entry(px[i].row(j), cl[i]), column_inc(px[i].c0, px[i].c1, px[i].c2));
        }
    }
    lds_order();
#pragma unroll 1
    for (int y = ya; y < yb; ++y) {
        // pixels of the step y -> y+1, fetched now and applied after the row:
        // the leaving row y-R and the entering row y+1+R of every column
        const bool step = y + 1 < yb;
        PixelBytes lv[NT], ev[NT];
        if (step) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int c = lane + 64 * t;
                lv[t].load(j, x0 - R + c, y - R, c < TW);
                ev[t].load(j, x0 - R + c, y + 1 + R, c < TW);
            }
        }
        // pass 1: the window count of every level for every lane (prefix sums
        // of the column counts across the strip), four levels at a time --
        // four independent scans, one prefix entry of four counts, one LDS
        // round trip; levels are compared in increasing order and the first
        // strictly larger count wins, so the lowest level wins ties
        Sums4 best = {0u, 0u, 0u, 0u};
        uint32_t bk = 0;
        auto count_of = [&](int k, int c) -> uint32_t {
            return reinterpret_cast<const uint32_t*>(entry((uint32_t)k, c))[1] >> 19;
        };
#pragma unroll 1
        for (int k0 = 0; k0 < L; k0 += 4) {
            const bool h1 = k0 + 1 < L, h2 = k0 + 2 < L, h3 = k0 + 3 < L;
            uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0;  // totals of the chunks before
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int c = lane + 64 * t;
                uint32_t n0 = 0, n1 = 0, n2 = 0, n3 = 0;
                if (c < TW) {
                    n0 = count_of(k0, c);
                    if (h1) n1 = count_of(k0 + 1, c);
                    if (h2) n2 = count_of(k0 + 2, c);
                    if (h3) n3 = count_of(k0 + 3, c);
                }
                n0 = wave_scan_add(n0) + q0;
                n1 = wave_scan_add(n1) + q1;
                n2 = wave_scan_add(n2) + q2;
                n3 = wave_scan_add(n3) + q3;
                if (c < TW) *reinterpret_cast<uint4*>(P + (size_t)(c + 1) * 4) = make_uint4(n0, n1, n2, n3);
                if (t + 1 < NT) {
                    q0 = (uint32_t)__builtin_amdgcn_readlane((int)n0, 63);
                    q1 = (uint32_t)__builtin_amdgcn_readlane((int)n1, 63);
                    q2 = (uint32_t)__builtin_amdgcn_readlane((int)n2, 63);
                    q3 = (uint32_t)__builtin_amdgcn_readlane((int)n3, 63);
                }
            }
            lds_order();
            const uint4 hi = *reinterpret_cast<const uint4*>(P + (size_t)(lane + 2 * R + 1) * 4);
            const uint4 lo = *reinterpret_cast<const uint4*>(P + (size_t)lane * 4);
            const uint32_t w0 = hi.x - lo.x, w1 = hi.y - lo.y, w2 = hi.z - lo.z, w3 = hi.w - lo.w;
            if (w0 > best.n) {
                best.n = w0;
                bk = (uint32_t)k0;
            }
            if (w1 > best.n) {
                best.n = w1;
                bk = (uint32_t)k0 + 1;
            }
            if (w2 > best.n) {
                best.n = w2;
                bk = (uint32_t)k0 + 2;
            }
            if (w3 > best.n) {
                best.n = w3;
                bk = (uint32_t)k0 + 3;
            }
            lds_order();
        }
        // pass 2: the channel sums of each lane's winning level, one set of
        // prefix sums per distinct winner in the wavefront (neighbouring
        // pixels mostly share their mode)
        uint64_t pending = __ballot(best.n > 0);
        while (pending) {
            const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)bk, (int)__builtin_ctzll(pending));
            uint32_t ca = 0, cb = 0, cc = 0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int c = lane + 64 * t;
                uint64_t e = 0;
                if (c < TW) e = *entry(k, c);
                Sums4 v = column_unpack(e);
                v.a = wave_scan_add(v.a) + ca;
                v.b = wave_scan_add(v.b) + cb;
                v.c = wave_scan_add(v.c) + cc;
                if (c < TW) *reinterpret_cast<uint4*>(P + (size_t)(c + 1) * 4) = make_uint4(0u, v.a, v.b, v.c);
                if (t + 1 < NT) {
                    ca = (uint32_t)__builtin_amdgcn_readlane((int)v.a, 63);
                    cb = (uint32_t)__builtin_amdgcn_readlane((int)v.b, 63);
                    cc = (uint32_t)__builtin_amdgcn_readlane((int)v.c, 63);
                }
            }
            lds_order();
            const bool mine = best.n > 0 && bk == k;
            if (mine) {
                const uint4 hi = *reinterpret_cast<const uint4*>(P + (size_t)(lane + 2 * R + 1) * 4);
                const uint4 lo = *reinterpret_cast<const uint4*>(P + (size_t)lane * 4);
                best.a = hi.y - lo.y;
                best.b = hi.z - lo.z;
                best.c = hi.w - lo.w;
            }
            pending &= ~__ballot(mine);
            lds_order();
        }
        uint32_t px = 0;
        if (best.n > 0) {
            const double rn = 1.0 / (double)best.n;
            px = div_exact32(best.a, best.n, rn) | (div_exact32(best.b, best.n, rn) << 8) |
                 (div_exact32(best.c, best.n, rn) << 16);
        }
        store_row(j, x0, y, best.n, px, obuf);
        if (step) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int c = lane + 64 * t;
                if (c < TW) {
                    lds_sub(entry(lv[t].row(j), c), column_inc(lv[t].c0, lv[t].c1, lv[t].c2));
                    lds_add(entry(ev[t].row(j), c), column_inc(ev[t].c0, ev[t].c1, ev[t].c2));
                }
            }
            lds_order();
        }
    }
}

// ---------------------------------------------------------------------------
// COLUMN layout for radius <= 15 (tile_column15): the same column histograms
// and prefix sums, shaped for windows of at most 31 x 31.
// ---------------------------------------------------------------------------
// Column entries use the streamed layout's F18 bin word (count:10 @54 |
// 3 x 18-bit sums), so the window word of a level is the plain 64-bit sum of
// its 2r+1 column entries.  Beside them, each column keeps its counts three
// levels to a 32-bit word, 10 bits each (word w: levels 3w .. 3w+2).  Pass 1
// prefix-sums those words across the strip: the sums wrap, but a window
// count is below 1024 and 32-bit addition is exact modulo 2^32, so the
// difference of two prefix words holds the three window counts exactly.
// Pass 2 sums the 2r+1 entries of each lane's winning level directly: a
// fixed cost, however many distinct winners a row has.  Outside pixels and
// the paper form's white level are counted nowhere.
//   LDS: [column histograms: L level rows x 94 columns x 8 B]
//        [count words: NW x 94 x 4 B] ...

// Prefix sum of the wavefront's column words at column lane + 2R (chunk 0
// holds columns 0..63, chunk 1 columns 64..): a lane permute of either
// chunk's inclusive scan.
__device__ __forceinline__ uint32_t shifted_prefix(uint32_t s0, uint32_t s1, int lane, int r2) {
    const int src = lane + r2;
    const int a = (src & 63) << 2;
    const uint32_t p0 = (uint32_t)__builtin_amdgcn_ds_bpermute(a, (int)s0);
    const uint32_t p1 = (uint32_t)__builtin_amdgcn_ds_bpermute(a, (int)s1);
    return src < 64 ? p0 : p1;
}

// NV wavefronts share a strip (1, 2 or 4).  Per output row: pass 1's
// words are dealt round the wavefronts, each posting the best key of its
// levels; a barrier; every wavefront takes the largest key, applies its
// share of the step's count-word updates and sums its share of the 2r+1
// winning entries; a barrier; one wavefront, rotating by row, adds the
// partial words and stores the row while all make their share of the entry
// updates.  The updates of the step y -> y+1 are the two pixels of each
// column of the strip, leaving row y-R and entering row y+1+R, dealt as
// (leave/enter, 64-column chunk) pairs.
//   LDS, after the count words: [keys: NV x 64 x 4 B][partial words:
//   (NV - 1) x 64 x 8 B, slot (w - finalizer - 1) mod NV][output row
//   buffer: 192 B]
//
// WIDE: the form for radius 16..31 (tile_column31 below): windows up to
// 63 x 63, so window counts need 12 bits -- two 16-bit counts per word (word
// w: levels 2w, 2w+1) -- and window sums 20 bits, more than a 64-bit word
// holds beside them: pass 2 sums the column entries into two words, sums 0
// and 2 in one, sum 1 and the count in the other, each field with room to
// grow.  Column entries keep the F18 word (a column holds at most 63
// pixels).  Partial words are 16 bytes per lane.
template <int NW, int NV, bool WIDE = false>
__device__ __forceinline__ void tile_column15(const Job& j, int unit, uint8_t* lds) {
    static_assert(NV == 1 || NV == 2 || NV == 4, "one, two or four wavefronts per strip");
    constexpr int CS = WIDE ? kColumn31Stride : kColumn15Stride;
    constexpr int FB = WIDE ? 16 : 10;                 // bits of a count field
    constexpr int NF = WIDE ? 2 : 3;                   // count fields per word
    constexpr uint32_t FM = (1u << FB) - 1u;
    constexpr int RS = CS * 8;  // bytes per level row
    constexpr int NT = 64 * NV;
    constexpr int NPX = 4 / NV;  // step pixels per lane of each wavefront
    const int R = j.radius;
    const int TW = 64 + 2 * R;
    const int L = j.levels;
    const int lane = threadIdx.x & 63;
    const int wv = NV == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int tx = unit % j.tiles_x;
    const int ty = unit / j.tiles_x;
    const int x0 = tx * 64;
    const int ya = j.row_begin + ty * j.rows;
    const int yb = min(ya + j.rows, j.row_end);
    uint8_t* ch = lds;
    uint32_t* cw = reinterpret_cast<uint32_t*>(lds + (size_t)L * RS);
    uint32_t* keys = cw + NW * CS;
    uint64_t* words = reinterpret_cast<uint64_t*>(keys + NV * 64);
    uint8_t* obuf = reinterpret_cast<uint8_t*>(words + (NV - 1) * 64 * (WIDE ? 2 : 1));
    const bool paper = j.paper != 0;
    auto barrier = [] {
        if constexpr (NV > 1)
            lds_barrier();
        else
            lds_order();
    };
    // level of a pixel, or L for outside pixels and the paper form's white
    auto level = [&](const PixelBytes& p) -> uint32_t {
        const uint32_t lev = level_of(p.c0 + p.c1 + p.c2, (uint32_t)L, paper);
        return (p.in && lev < (uint32_t)L) ? lev : (uint32_t)L;
    };
    auto inc = [](const PixelBytes& p) -> uint64_t {
        return ((uint64_t)((p.c2 << 4) | (1u << 22)) << 32) | (p.c0 | (p.c1 << 18));
    };
    // count word and field of level k < 128: k / 3 == (43 k) >> 7, or k / 2
    auto count_word = [](uint32_t k) { return WIDE ? k >> 1 : mul24(k, 43u) >> 7; };
    auto count_bit = [&](uint32_t k) {
        return WIDE ? 1u << (16u * (k & 1u)) : 1u << mul24(10u, k - mul24(3u, count_word(k)));
    };
    auto entry_at = [&](uint32_t k, int c) {
        return reinterpret_cast<uint64_t*>(ch + mul24(k, RS) + (uint32_t)c * 8u);
    };

    {
        // (rounded up into the keys, which are written before they are read)
        const int n16 = (int)(((size_t)L * RS + (size_t)NW * CS * 4 + 15) / 16);
        for (int e = (int)threadIdx.x; e < n16; e += NT)
            *reinterpret_cast<uint4*>(ch + (size_t)e * 16) = make_uint4(0u, 0u, 0u, 0u);
    }
    barrier();
    {
        // column histograms of rows ya-R .. ya+R; pixel p = t + NT i sits
        // at (p / TW, p % TW), tracked in steps of NT
        const int NP = (2 * R + 1) * TW;
        constexpr int CH = 16 / NV;
        const int dq = NT / TW, dr = NT % TW;
        int row = (int)threadIdx.x / TW, col = (int)threadIdx.x % TW;
        for (int base = (int)threadIdx.x; base < NP; base += CH * NT) {
            PixelBytes px[CH];
            int cl[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                cl[i] = col;
                px[i].load(j, x0 - R + col, ya - R + row, base + i * NT < NP);
                row += dq;
                col += dr;
                if (col >= TW) {
                    col -= TW;
                    ++row;
                }
            }
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const uint32_t k = level(px[i]);
                if (k < (uint32_t)L) {
                    lds_add(entry_at(k, cl[i]), inc(px[i]));
                    lds_add(cw + mul24(count_word(k), CS) + cl[i], count_bit(k));
                }
            }
        }
    }
    barrier();
    const int span = 2 * R + 1;
    const int part = (span + NV - 1) / NV;
    const int d0 = min(span, wv * part), d1 = min(span, d0 + part);
    // this wavefront's pixels of each step: (leave/enter) << 1 | chunk
    int pc[NPX];
    bool enter[NPX];
#pragma unroll
    for (int q = 0; q < NPX; ++q) {
        const int id = wv * NPX + q;
        enter[q] = (id >> 1) != 0;
        pc[q] = lane + 64 * (id & 1);
    }
    // the pixels of the step y -> y+1: leaving row y-R or entering row y+1+R
    auto fetch = [&](int y, PixelBytes (&px)[NPX]) {
        if (y + 1 < yb) {
#pragma unroll
            for (int q = 0; q < NPX; ++q) px[q].load(j, x0 - R + pc[q], enter[q] ? y + 1 + R : y - R, pc[q] < TW);
        }
    };
    // Output row y, then the step y -> y+1 with the pixels px.
    auto row = [&](int y, const PixelBytes (&px)[NPX]) {
        const bool step = y + 1 < yb;
        // pass 1: window counts, three levels per word; the most populated
        // level, lowest among equals, is the largest key (count << 7) |
        // (127 - level).  Chunk-1 columns past the strip read whatever
        // follows in LDS: only scan entries at lanes they precede are used.
        // Every wavefront takes the same number of words, the last one again
        // where the words run out (a repeated word repeats its keys), so
        // that the words' scans interleave without branches.
        uint32_t key = 0;
#pragma unroll
        for (int i = 0; i < (NW + NV - 1) / NV; ++i) {
            const int w = min(i * NV + wv, NW - 1);
            const uint32_t v0 = cw[w * CS + lane];
            const uint32_t v1 = cw[w * CS + 64 + lane];
            const uint32_t s0 = wave_scan_add(v0);
            const uint32_t s1 = wave_scan_add(v1) + (uint32_t)__builtin_amdgcn_readlane((int)s0, 63);
            const uint32_t dd = shifted_prefix(s0, s1, lane, 2 * R) - (s0 - v0);
#pragma unroll
            for (int k = 0; k < NF; ++k)
                key = max(key, (((dd >> (FB * k)) & FM) << 7) | (127u - (uint32_t)(NF * w + k)));
        }
        if constexpr (NV > 1) keys[wv * 64 + lane] = key;
        barrier();
        if constexpr (NV > 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v) key = max(key, keys[v * 64 + lane]);
        }
        uint32_t lev[NPX];
#pragma unroll
        for (int q = 0; q < NPX; ++q) {
            lev[q] = (step && pc[q] < TW) ? level(px[q]) : (uint32_t)L;
            if (lev[q] < (uint32_t)L) {
                uint32_t* c = cw + mul24(count_word(lev[q]), CS) + pc[q];
                if (enter[q])
                    lds_add(c, count_bit(lev[q]));
                else
                    lds_sub(c, count_bit(lev[q]));
            }
        }
        // pass 2: this wavefront's share of the winning level's window word
        const uint32_t n = key >> 7;
        const uint64_t* ent = entry_at(127u - (key & 127u), lane);
        const int fin = NV == 1 ? 0 : ((y - ya) & (NV - 1));
        if constexpr (!WIDE) {
            uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
            int d = d0;
#pragma unroll 1
            for (; d + 4 <= d1; d += 4) {
                a0 += ent[d];
                a1 += ent[d + 1];
                a2 += ent[d + 2];
                a3 += ent[d + 3];
            }
            for (; d < d1; ++d) a0 += ent[d];
            uint64_t word = (a0 + a1) + (a2 + a3);
            if constexpr (NV > 1)
                if (wv != fin) words[((wv - fin - 1) & (NV - 1)) * 64 + lane] = word;
            barrier();
            if (wv == fin) {
                if constexpr (NV > 1) {
#pragma unroll
                    for (int v = 0; v < NV - 1; ++v) word += words[v * 64 + lane];
                }
                store_row(j, x0, y, n, finalize_packed<false>(n, word), obuf);
            }
        } else {
            // sums 0 and 2 (bits 0 and 36) in one word, sum 1 and the count
            // (bits 0 and 36 after a shift by 18) in the other: each total
            // stays below 2^20, clear of the next field
            constexpr uint64_t MA = 0x3FFFFull | (0x3FFFFull << 36);
            constexpr uint64_t MB = 0x3FFFFull | (0x3FFull << 36);
            uint64_t a0 = 0, b0 = 0, a1 = 0, b1 = 0;
            int d = d0;
#pragma unroll 1
            for (; d + 2 <= d1; d += 2) {
                const uint64_t e0 = ent[d], e1 = ent[d + 1];
                a0 += e0 & MA;
                b0 += (e0 >> 18) & MB;
                a1 += e1 & MA;
                b1 += (e1 >> 18) & MB;
            }
            if (d < d1) {
                const uint64_t e0 = ent[d];
                a0 += e0 & MA;
                b0 += (e0 >> 18) & MB;
            }
            uint64_t wa = a0 + a1, wb = b0 + b1;
            if constexpr (NV > 1)
                if (wv != fin) {
                    uint64_t* slot = words + (size_t)((wv - fin - 1) & (NV - 1)) * 128 + 2 * lane;
                    slot[0] = wa;
                    slot[1] = wb;
                }
            barrier();
            if (wv == fin) {
                if constexpr (NV > 1) {
#pragma unroll
                    for (int v = 0; v < NV - 1; ++v) {
                        const uint64_t* slot = words + (size_t)v * 128 + 2 * lane;
                        wa += slot[0];
                        wb += slot[1];
                    }
                }
                const uint32_t nn = n ? n : 1u;
                const double rn = 1.0 / (double)nn;
                const uint32_t s0 = (uint32_t)wa & 0xFFFFFu, s2 = (uint32_t)(wa >> 36) & 0xFFFFFu;
                const uint32_t s1 = (uint32_t)wb & 0xFFFFFu;
                store_row(j, x0, y, n,
                          div_exact32(s0, nn, rn) | (div_exact32(s1, nn, rn) << 8) | (div_exact32(s2, nn, rn) << 16),
                          obuf);
            }
        }
#pragma unroll
        for (int q = 0; q < NPX; ++q)
            if (lev[q] < (uint32_t)L) {
                uint64_t* c = entry_at(lev[q], pc[q]);
                if (enter[q])
                    lds_add(c, inc(px[q]));
                else
                    lds_sub(c, inc(px[q]));
            }
        lds_order();
    };
    PixelBytes pa[NPX];
    if constexpr (NV == 1) {
        // one wavefront: a step's pixels are fetched one row ahead, into two
        // register sets taken in turn
        PixelBytes pb[NPX];
        fetch(ya, pa);
#pragma unroll 1
        for (int y = ya; y < yb; y += 2) {
            fetch(y + 1, pb);
            row(y, pa);
            if (y + 1 < yb) {
                fetch(y + 2, pa);
                row(y + 1, pb);
            }
        }
    } else {
        // several: the other wavefronts hide the latency of a fetch at the
        // top of the row (measured faster than fetching a row ahead); the
        // wavefront priority follows the run's progress
        const int q1 = ya + (yb - ya) / 4, q2 = ya + (yb - ya) / 2, q3 = ya + 3 * (yb - ya) / 4;
#pragma unroll 1
        for (int y = ya; y < yb; ++y) {
            progress_priority(y, q1, q2, q3);
            fetch(y, pa);
            row(y, pa);
        }
    }
}

// One class of a batch in the column layout's radius <= 15 form, NV
// wavefronts per strip.  With several, thread 0 takes the next tile and
// hands it on through LDS; every tile passes barriers before its last
// row, so no wavefront can take a new tile while another still reads the
// previous handle.
template <int NW, int NV>
__device__ __forceinline__ void batch_column15(const BatchArgs& a, uint8_t* lds) {
    if constexpr (NV == 1) {
        for (;;) {
            const int32_t t = next_tile_wave(a.counter);
            if (t >= a.ntiles) break;
            const int i = job_of(a, t);
            const Job jb = a.jobs[i];
            tile_column15<NW, 1>(jb, t - a.first_tile[i], lds);
        }
    } else {
        __shared__ int32_t next;
        for (;;) {
            if (threadIdx.x == 0) next = (int32_t)atomicAdd(a.counter, 1u);
            lds_barrier();
            const int32_t t = __builtin_amdgcn_readfirstlane(next);
            if (t >= a.ntiles) break;
            const int i = job_of(a, t);
            const Job jb = a.jobs[i];
            tile_column15<NW, NV>(jb, t - a.first_tile[i], lds);
        }
    }
}

// One class of a batch in the column layout.
template <int NT>
__device__ __forceinline__ void batch_column(const BatchArgs& a, uint8_t* lds) {
    for (;;) {
        const int32_t t = next_tile_wave(a.counter);
        if (t >= a.ntiles) break;
        const int i = job_of(a, t);
        const Job jb = a.jobs[i];
        tile_column<NT>(jb, t - a.first_tile[i], lds);
    }
}

}  // namespace dev
}  // namespace oilpaint_impl
