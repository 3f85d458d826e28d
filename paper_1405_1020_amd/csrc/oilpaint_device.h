// Device code of the oil-paint filter (gfx950), shared by the kernel
// translation units.
//
// The method (Section 4 of the paper: histogram-based oil paint, its serial
// listing; Section 5: the same body run row-parallel): for each output
// pixel, bin the pixels of its (2r+1)^2 window by intensity level, keep per
// level a pixel count and three channel sums, pick the most populated level
// (lowest on ties) and output that level's channel sums divided by its count.
//
// How it is laid out on the GPU (the paper rebuilds the whole window for
// every pixel; none of the structure below is in the paper):
//   * A workgroup computes one tile: 64 (or fewer) output columns by a run of
//     output rows per wavefront.  Lane l owns column x0 + l and slides its
//     window histogram down the run: moving one row down removes the leaving
//     window row and adds the entering one, 2(2r+1) bin updates instead of a
//     (2r+1)^2 rebuild.
//   * Histograms live in LDS, one 64-bit word per level packing the count
//     and the three channel sums (F18: count:10 | three 18-bit sums for r
//     <= 15; F16: count:8 | three 16-bit sums for r <= 7), bins interleaved
//     across lanes (bin k of lane l at k*512 + l*8) so that every lane stays
//     on its own bank whatever level it touches.  No field can carry into
//     the next: each stays within its range.  Pixels outside the image get a
//     spare level that the mode search never scans, so the window needs no
//     clipping logic.
//   * STREAM layout (the default for r <= 15, L <= 64): one wavefront per
//     strip, or four sharing it (tile_stream_split); only the 2r+4 image rows
//     around the window are staged, in a ring, as 4-byte words {c0, c1, c2,
//     level} or (STREAM8) as 8-byte ready bin increments; a run's first
//     window comes either from direct updates or from column histograms.
//   * PACKED layout: the whole tile plus its r-pixel halo staged once, shared
//     by several wavefronts.
//   * COLUMN layout (r up to 255, oilpaint_column.h): column histograms and
//     per-level prefix sums across the strip; the work per row does not grow
//     with r.
//   * WIDE layout (anything else): 32-bit counts and sums, pixels read from
//     device memory.
//   * The mode search takes the maximum of (count << shift) | (C - level)
//     for a constant C above every level: the most populated level, the
//     lowest index among ties.
//   * The divisions are exact (div_exact here, div_exact32 in oilpaint_column.h).
#pragma once

#include <type_traits>

#include "oilpaint_internal.h"

namespace oilpaint_impl {
namespace dev {

// The tile of this workgroup in a plain launch (one workgroup per tile,
// tiles numbered strip by strip along each run of rows, run after run).
// The dispatcher deals workgroups to the GPU's eight XCDs in turn (workgroup
// b to XCD b mod 8), and each XCD has its own L2: in blockIdx order a
// strip's neighbours, which read the same halo columns and cache lines,
// would sit on other XCDs and fetch those lines again.  Here the tiles go
// to the XCDs in chunks of kXcdChunk neighbours, chunk c to XCD c mod 8, so
// that neighbours share an L2 while every XCD still takes tiles from all
// over the image (contiguous eighths measured slower where tile costs
// vary).  A bijection on 0 .. gridDim.x - 1 (the last, partial round of
// chunks keeps blockIdx order), so results do not depend on how workgroups
// are really dealt.
constexpr int kXcds = 8;
constexpr int kXcdChunk = 4;
__device__ __forceinline__ int xcd_tile() {
    const int n = (int)gridDim.x, b = (int)blockIdx.x;
    const int full = n - n % (kXcds * kXcdChunk);
    if (b >= full) return b;
    const int x = b % kXcds, i = b / kXcds;
    return ((i / kXcdChunk) * kXcds + x) * kXcdChunk + i % kXcdChunk;
}

// Products of operands below 2^24: the masks let the compiler use the
// full-rate 24-bit multiplies (v_mul_u32_u24, v_mul_hi_u32_u24) instead of
// the quarter-rate 32-bit ones.  mul24 is exact while the product is below
// 2^32, mulhi24 gives bits 32..47 of the 48-bit product.
__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) { return (a & 0xFFFFFFu) * (b & 0xFFFFFFu); }
__device__ __forceinline__ uint32_t mulhi24(uint32_t a, uint32_t b) {
    return (uint32_t)(((uint64_t)(a & 0xFFFFFFu) * (uint64_t)(b & 0xFFFFFFu)) >> 32);
}

// floor(s / n) for 1 <= n <= 961 and s <= 255 n, without a divide: with rn
// the hardware reciprocal of n (v_rcp_f32, within 1 ulp), the float estimate
// s * rn is within 1e-4 of s/n (s < 2^18, relative error of the reciprocal
// and the product a few ulp), and s/n lies at least 1/961 below the next
// integer, so truncating the estimate gives floor(s/n) or one less; the
// integer checks correct either way.
__device__ __forceinline__ float rcp_approx(uint32_t n) { return __builtin_amdgcn_rcpf((float)n); }
__device__ __forceinline__ uint32_t div_exact(uint32_t s, uint32_t n, float rn) {
    uint32_t q = (uint32_t)((float)s * rn);  // q, n < 2^18: 24-bit products
    q += (mul24(q + 1u, n) <= s) ? 1u : 0u;
    q -= (mul24(q, n) > s) ? 1u : 0u;
    return q;
}

// Intensity level of a pixel with channel sum s (Section 4 listing, level
// step).  Default reading: ((s / 3) * L) / 256, truncating, with
// s / 3 == (s * 43691) >> 17 for s <= 765.  Paper form: floor(s * L / 765)
// (equal to the listing's double expression for every s <= 765, L <= 256),
// with floor(x / 765) == mulhi(x, 5614337) for x <= 765 * 256.  Every
// operand is below 2^24 (s <= 765, L <= 256), so 24-bit products serve.
__device__ __forceinline__ uint32_t level_of(uint32_t s, uint32_t L, bool paper) {
    if (paper) return mulhi24(mul24(s, L), 5614337u);
    return mul24(mul24(s, 43691u) >> 17, L) >> 8;
}

// Image pointers as global-address-space pointers, so loads and stores are
// global_* instructions (flat ones would also count against the LDS wait
// counter and serialize with the histogram traffic).
typedef const __attribute__((address_space(1))) uint8_t* gsrc_t;
typedef __attribute__((address_space(1))) uint8_t* gdst_t;
__device__ __forceinline__ gsrc_t gsrc(const uint8_t* p) { return (gsrc_t)p; }
__device__ __forceinline__ gdst_t gdst(uint8_t* p) { return (gdst_t)p; }

// Compiler-only ordering point for LDS traffic shared between the lanes of
// one wavefront: the hardware already executes a wavefront's LDS operations
// in order, so no wait is needed, only that the compiler keep program order.
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

template <typename T>
__device__ __forceinline__ void lds_add(T* p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void lds_sub(T* p, T v) {
    __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LDS words addressed by their 32-bit LDS offset.
typedef __attribute__((address_space(3))) uint64_t lds_u64;
__device__ __forceinline__ uint32_t lds_offset(const uint8_t* p) {
    return (uint32_t)(size_t)(const __attribute__((address_space(3))) uint8_t*)p;
}
__device__ __forceinline__ lds_u64* lds_word(uint32_t off) { return (lds_u64*)(size_t)off; }
__device__ __forceinline__ void lds_add(lds_u64* p, uint64_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_sub(lds_u64* p, uint64_t v) {
    __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// 64-bit packed bin increment for a staged word {c0, c1, c2, level}.
__device__ __forceinline__ uint64_t packed_value(uint32_t w) {
    const uint32_t lo = (w & 0xFFu) | (((w >> 8) & 0xFFu) << 18);
    const uint32_t hi = (((w >> 16) & 0xFFu) << 4) | (1u << 22);
    return ((uint64_t)hi << 32) | lo;
}

// Bin formats of the streamed layout (one 64-bit word per level):
//   F18: count:10 @54 | sum2:18 @36 | sum1:18 @18 | sum0:18 @0  -- windows
//        up to 31 x 31 (count <= 961, sums <= 245,055)
//   F16: count:8 @48 | sum2:16 @32 | sum1:16 @16 | sum0:16 @0   -- windows
//        up to 15 x 15 (count <= 225, sums <= 57,375); byte-aligned fields,
//        so the increment of a staged word {c0, c1, c2, level} is two byte
//        permutes.
template <bool F16>
struct BinFmt;

template <>
struct BinFmt<false> {
    static constexpr uint32_t kCountMask = 0xFFC00000u;  // count bits in the high word
    static constexpr int kCountShift = 22;
    static __device__ __forceinline__ uint64_t inc(uint32_t w) { return packed_value(w); }
    static __device__ __forceinline__ void sums(uint64_t b, uint32_t& s0, uint32_t& s1, uint32_t& s2) {
        const uint32_t lo = (uint32_t)b, hi = (uint32_t)(b >> 32);
        s0 = lo & 0x3FFFFu;
        s1 = (lo >> 18) | ((hi & 0xFu) << 14);
        s2 = (hi >> 4) & 0x3FFFFu;
    }
};

template <>
struct BinFmt<true> {
    static constexpr uint32_t kCountMask = 0x00FF0000u;
    static constexpr int kCountShift = 16;
    static __device__ __forceinline__ uint64_t inc(uint32_t w) {
        const uint32_t lo = __builtin_amdgcn_perm(0u, w, 0x0C010C00u);  // c0 | c1 << 16
        const uint32_t hi = __builtin_amdgcn_perm(1u, w, 0x0C040C02u);  // c2 | 1 << 16
        return ((uint64_t)hi << 32) | lo;
    }
    static __device__ __forceinline__ void sums(uint64_t b, uint32_t& s0, uint32_t& s1, uint32_t& s2) {
        const uint32_t lo = (uint32_t)b, hi = (uint32_t)(b >> 32);
        s0 = lo & 0xFFFFu;
        s1 = lo >> 16;
        s2 = hi & 0xFFFFu;
    }
};

struct TileGeom {
    int x0, y0, yend;   // first column, first and one-past-last output row
    int tw, th;         // staged columns and rows (tile + halo)
};

__device__ __forceinline__ TileGeom tile_geom(const Job& j, int tile) {
    TileGeom g;
    const int tx = tile % j.tiles_x;
    const int ty = tile / j.tiles_x;
    g.x0 = tx * j.lanes;
    g.y0 = j.row_begin + ty * j.waves * j.rows;
    g.yend = min(g.y0 + j.waves * j.rows, j.row_end);
    g.tw = j.lanes + 2 * j.radius;
    g.th = (g.yend - g.y0) + 2 * j.radius;
    return g;
}

// ---------------------------------------------------------------------------
// PACKED layout
// ---------------------------------------------------------------------------

// Staged word of an in-image pixel.
__device__ __forceinline__ uint32_t staged_word(uint32_t c0, uint32_t c1, uint32_t c2, const Job& j) {
    uint32_t lev = level_of(c0 + c1 + c2, (uint32_t)j.levels, j.paper != 0);
    if (lev >= (uint32_t)j.levels) lev = (uint32_t)j.white;  // paper form: pure white
    return c0 | (c1 << 8) | (c2 << 16) | (lev << 24);
}

// Stage the tile and its r-pixel halo into LDS.  Every thread of the
// workgroup takes part; pixels are visited in chunks of 8 per thread so that
// 24 byte loads are in flight before any is used.  TW is the staged width
// when known at compile time (0: g.tw).  The caller synchronizes.
template <int TW = 0>
__device__ __forceinline__ void stage_packed(const Job& j, const TileGeom& g, uint32_t* tw32) {
    constexpr int CH = 8;
    const int r = j.radius;
    const int tw = TW ? TW : g.tw;
    const int npx = tw * g.th;
    const int nthr = blockDim.x;
    const uint32_t trash_word = (uint32_t)j.trash << 24;
    for (int base = threadIdx.x; base < npx; base += CH * nthr) {
        uint32_t c[CH][3];
        bool in[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int p = base + i * nthr;
            const int row = p / tw;
            const int col = p - row * tw;
            const int gy = g.y0 - r + row;
            const int gx = g.x0 - r + col;
            in[i] = p < npx && gy >= 0 && gy < j.height && gx >= 0 && gx < j.width;
            c[i][0] = c[i][1] = c[i][2] = 0;
            if (in[i]) {
                gsrc_t q = gsrc(j.src) + (size_t)gy * (size_t)j.stride + 3 * gx;
                c[i][0] = q[0];
                c[i][1] = q[1];
                c[i][2] = q[2];
            }
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int p = base + i * nthr;
            if (p < npx) tw32[p] = in[i] ? staged_word(c[i][0], c[i][1], c[i][2], j) : trash_word;
        }
    }
}

// Output of one pixel from its winning bin word (packed layout).
__device__ __forceinline__ void store_packed(const Job& j, int x, int y, uint32_t n, uint64_t b) {
    bool store = x < j.width;
    if (j.paper) store = store && n > 0 && x >= j.radius && x < j.width - j.radius && y >= j.radius &&
                         y < j.height - j.radius;
    if (!store) return;
    const uint32_t lo = (uint32_t)b, hi = (uint32_t)(b >> 32);
    const uint32_t s0 = lo & 0x3FFFFu;
    const uint32_t s1 = (lo >> 18) | ((hi & 0xFu) << 14);
    const uint32_t s2 = (hi >> 4) & 0x3FFFFu;
    const float rn = rcp_approx(n);
    gdst_t o = gdst(j.dst) + (size_t)y * (size_t)j.dst_stride + 3 * x;
    o[0] = (uint8_t)div_exact(s0, n, rn);
    o[1] = (uint8_t)div_exact(s1, n, rn);
    o[2] = (uint8_t)div_exact(s2, n, rn);
}

// The three output bytes of a pixel from its winning bin word, packed as
// c0 | c1 << 8 | c2 << 16.
template <bool F16>
__device__ __forceinline__ uint32_t finalize_packed(uint32_t n, uint64_t b) {
    uint32_t s0, s1, s2;
    BinFmt<F16>::sums(b, s0, s1, s2);
    const uint32_t nn = n ? n : 1u;
    const float rn = rcp_approx(nn);
    return div_exact(s0, nn, rn) | (div_exact(s1, nn, rn) << 8) | (div_exact(s2, nn, rn) << 16);
}

// Mode search over bins 0 .. scan-1 of one lane (scan a multiple of 8, at
// most SB): the reads are issued by mode_load, in groups of eight, as full
// 64-bit words (whole 8-byte slots keep the 64 lanes on distinct banks; a
// read of the high halves alone would pair lanes on a bank), and reduced by
// mode_reduce to the key (count << kCountShift) | (63 - level), whose
// maximum is the most populated level, the lowest among equals.
template <int SB>
struct ModeBins {
    uint64_t v[SB];
};

template <int SB>
__device__ __forceinline__ void mode_load(ModeBins<SB>& m, const uint8_t* hl, int scan) {
#pragma unroll
    for (int g = 0; g < SB / 8; ++g)
        if (g * 8 < scan) {
#pragma unroll
            for (int i = 0; i < 8; ++i) m.v[g * 8 + i] = *reinterpret_cast<const uint64_t*>(hl + (g * 8 + i) * 512);
        }
}

template <int SB, bool F16>
__device__ __forceinline__ uint32_t mode_reduce(const ModeBins<SB>& m, int scan) {
    static_assert(SB <= 64, "level index must fit 6 bits");
    constexpr uint32_t M = BinFmt<F16>::kCountMask;
    uint32_t best = 0;
#pragma unroll
    for (int g = 0; g < SB / 8; ++g)
        if (g * 8 < scan) {
#pragma unroll
            for (int i = 0; i < 8; ++i) asm volatile("" ::"v"((uint32_t)m.v[g * 8 + i]));  // keep whole-word reads
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                const uint32_t k = (uint32_t)(g * 8 + i);
                best = max(best, max(((uint32_t)(m.v[k] >> 32) & M) | (63u - k),
                                     ((uint32_t)(m.v[k + 1] >> 32) & M) | (62u - k)));
            }
        }
    return best;
}

// Store one output row of a 64-column strip.  A full strip goes through a
// 192-byte LDS row buffer and leaves as 48 dword stores; a partial strip (or
// the paper form, which writes only part of a row) stores per pixel.
__device__ __forceinline__ void store_row(const Job& j, int x0, int y, uint32_t n, uint32_t px, uint8_t* obuf) {
    const int lane = threadIdx.x & 63;
    const int x = x0 + lane;
    gdst_t row = gdst(j.dst) + (size_t)y * (size_t)j.dst_stride;
    if (x0 + 64 <= j.width && !j.paper) {
        obuf[3 * lane] = (uint8_t)px;
        obuf[3 * lane + 1] = (uint8_t)(px >> 8);
        obuf[3 * lane + 2] = (uint8_t)(px >> 16);
        lds_order();
        if (lane < 48) {
            const uint32_t w = reinterpret_cast<const uint32_t*>(obuf)[lane];
            *reinterpret_cast<__attribute__((address_space(1))) uint32_t*>(row + 3 * x0 + 4 * lane) = w;
        }
        lds_order();
        return;
    }
    bool store = x < j.width;
    if (j.paper) store = store && n > 0 && x >= j.radius && x < j.width - j.radius && y >= j.radius &&
                         y < j.height - j.radius;
    if (store) {
        row[3 * x] = (uint8_t)px;
        row[3 * x + 1] = (uint8_t)(px >> 8);
        row[3 * x + 2] = (uint8_t)(px >> 16);
    }
}

// Any radius <= 15, lane count and level count: runtime loops.
__device__ __forceinline__ void tile_packed(const Job& j, int tile, uint8_t* lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = j.waves;
    const int r = j.radius;
    const TileGeom g = tile_geom(j, tile);
    uint32_t* tw32 = reinterpret_cast<uint32_t*>(lds);
    stage_packed(j, g, tw32);
    __syncthreads();

    const int yw0 = g.y0 + wave * j.rows;
    if (wave >= nw || lane >= j.lanes || yw0 >= g.yend) return;
    const int yw1 = min(yw0 + j.rows, g.yend);
    const size_t tile_bytes = ((size_t)g.tw * (size_t)(nw * j.rows + 2 * r) * 4 + 15) & ~(size_t)15;
    const uint32_t binstride = (uint32_t)j.lanes * 8u;
    uint8_t* hl = lds + tile_bytes + (size_t)wave * j.bins * binstride + lane * 8;
    for (int k = 0; k < j.bins; ++k) *reinterpret_cast<uint64_t*>(hl + k * binstride) = 0;

    const int x = g.x0 + lane;
    const int span = 2 * r + 1;
    const uint32_t* t = tw32 + (yw0 - g.y0) * g.tw + lane;
    for (int dy = 0; dy < span; ++dy, t += g.tw)
        for (int dx = 0; dx < span; ++dx) {
            const uint32_t w = t[dx];
            lds_add(reinterpret_cast<uint64_t*>(hl + (w >> 24) * binstride), packed_value(w));
        }
    for (int y = yw0; y < yw1; ++y) {
        if (y > yw0) {
            // leaving image row y-1-r is staged row y-1-y0; entering row y+r is y+2r-y0
            const uint32_t* to = tw32 + (y - 1 - g.y0) * g.tw + lane;
            const uint32_t* tn = tw32 + (y + 2 * r - g.y0) * g.tw + lane;
            for (int dx = 0; dx < span; ++dx) {
                const uint32_t wo = to[dx];
                const uint32_t wn = tn[dx];
                lds_sub(reinterpret_cast<uint64_t*>(hl + (wo >> 24) * binstride), packed_value(wo));
                lds_add(reinterpret_cast<uint64_t*>(hl + (wn >> 24) * binstride), packed_value(wn));
            }
        }
        uint32_t best = 0;
        for (int k = 0; k < j.scan; ++k) {
            const uint32_t hi = (uint32_t)(*reinterpret_cast<const uint64_t*>(hl + k * binstride) >> 32);
            best = max(best, (hi & 0xFFC00000u) | (255u - (uint32_t)k));
        }
        const uint32_t kbest = 255u - (best & 0xFFu);
        store_packed(j, x, y, best >> 22, *reinterpret_cast<const uint64_t*>(hl + kbest * binstride));
    }
}

// Fast path: 64 lanes, a compile-time radius R <= 15 and at most 64 scanned
// levels (the level count rounded up to a multiple of 8; the extra bins stay
// empty and the trash bin sits after them).  Ordering within a lane's loop:
//   atomics of step y -> loads of step y+1's words -> mode-search reads of
//   row y+1 -> (consume) row y's winning bin, divide, store,
// so every LDS round trip overlaps other LDS traffic of the same wavefront.
template <int R, int SB>
__device__ __forceinline__ void tile_packed_fast(const Job& j, int tile, uint8_t* lds) {
    constexpr int SPAN = 2 * R + 1;
    constexpr int TW = 64 + 2 * R;
    constexpr uint32_t BS = 64u * 8u;  // bin stride
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = j.waves;
    const int scan = j.scan;  // multiple of 8, <= SB
    const TileGeom g = tile_geom(j, tile);
    uint32_t* tw32 = reinterpret_cast<uint32_t*>(lds);
    stage_packed<TW>(j, g, tw32);
    __syncthreads();

    const int yw0 = g.y0 + wave * j.rows;
    if (wave >= nw || yw0 >= g.yend) return;
    const int yw1 = min(yw0 + j.rows, g.yend);
    const size_t tile_bytes = ((size_t)TW * (size_t)(nw * j.rows + 2 * R) * 4 + 15) & ~(size_t)15;
    uint8_t* hl = lds + tile_bytes + (size_t)wave * j.bins * BS + lane * 8;
    for (int k = 0; k < j.bins; ++k) *reinterpret_cast<uint64_t*>(hl + k * BS) = 0;
    const int x = g.x0 + lane;

    // first window, one staged row at a time, the next row's words loaded
    // before the current row's atomics
    const uint32_t* t = tw32 + (yw0 - g.y0) * TW + lane;
    uint32_t w[SPAN];
#pragma unroll
    for (int i = 0; i < SPAN; ++i) w[i] = t[i];
#pragma unroll 1
    for (int dy = 0; dy < SPAN; ++dy) {
        uint32_t cur[SPAN];
#pragma unroll
        for (int i = 0; i < SPAN; ++i) cur[i] = w[i];
        t += TW;
        if (dy + 1 < SPAN) {
#pragma unroll
            for (int i = 0; i < SPAN; ++i) w[i] = t[i];
        }
#pragma unroll
        for (int i = 0; i < SPAN; ++i)
            lds_add(reinterpret_cast<uint64_t*>(hl + (cur[i] >> 24) * BS), packed_value(cur[i]));
    }

    // words of the step yw0 -> yw0+1
    uint32_t wo[SPAN], wn[SPAN];
    if (yw0 + 1 < yw1) {
        const uint32_t* to = tw32 + (yw0 - g.y0) * TW + lane;
        const uint32_t* tn = tw32 + (yw0 + 1 + 2 * R - g.y0) * TW + lane;
#pragma unroll
        for (int i = 0; i < SPAN; ++i) {
            wo[i] = to[i];
            wn[i] = tn[i];
        }
    }
    // mode-search reads of row yw0 (high words: count and sum2 bits)
    uint32_t hb[SB];
#pragma unroll
    for (int k = 0; k < SB; ++k)
        if (k < scan) hb[k] = (uint32_t)(*reinterpret_cast<const uint64_t*>(hl + k * BS) >> 32);

#pragma unroll 1
    for (int y = yw0; y < yw1; ++y) {
        // reduce row y's keys
        uint32_t best = 0;
#pragma unroll
        for (int k = 0; k < SB; k += 2)
            if (k < scan)
                best = max(best, max((hb[k] & 0xFFC00000u) | (255u - (uint32_t)k),
                                     (hb[k + 1] & 0xFFC00000u) | (254u - (uint32_t)k)));
        const uint32_t kbest = 255u - (best & 0xFFu);
        const uint64_t win = *reinterpret_cast<const uint64_t*>(hl + kbest * BS);
        if (y + 1 < yw1) {
            // step y -> y+1
#pragma unroll
            for (int i = 0; i < SPAN; ++i) {
                lds_sub(reinterpret_cast<uint64_t*>(hl + (wo[i] >> 24) * BS), packed_value(wo[i]));
                lds_add(reinterpret_cast<uint64_t*>(hl + (wn[i] >> 24) * BS), packed_value(wn[i]));
            }
            if (y + 2 < yw1) {
                // step y+1 -> y+2 removes image row y+1-R (staged row y+1-y0)
                // and adds image row y+2+R (staged row y+2+2R-y0)
                const uint32_t* to = tw32 + (y + 1 - g.y0) * TW + lane;
                const uint32_t* tn = tw32 + (y + 2 + 2 * R - g.y0) * TW + lane;
#pragma unroll
                for (int i = 0; i < SPAN; ++i) {
                    wo[i] = to[i];
                    wn[i] = tn[i];
                }
            }
#pragma unroll
            for (int k = 0; k < SB; ++k)
                if (k < scan) hb[k] = (uint32_t)(*reinterpret_cast<const uint64_t*>(hl + k * BS) >> 32);
        }
        store_packed(j, x, y, best >> 22, win);
    }
}

// ---------------------------------------------------------------------------
// WIDE layout: 32-bit count and sums in two 64-bit words per level
// (A = count | sum0 << 32, B = sum1 | sum2 << 32); pixels read from memory.
// ---------------------------------------------------------------------------
struct WidePix {
    uint32_t lev;
    uint64_t a, b;
};

__device__ __forceinline__ WidePix wide_pixel(const Job& j, int gx, int gy) {
    WidePix p;
    if (gx >= 0 && gx < j.width && gy >= 0 && gy < j.height) {
        gsrc_t q = gsrc(j.src) + (size_t)gy * (size_t)j.stride + 3 * gx;
        const uint32_t c0 = q[0], c1 = q[1], c2 = q[2];
        p.lev = level_of(c0 + c1 + c2, (uint32_t)j.levels, j.paper != 0);
        if (p.lev >= (uint32_t)j.levels) p.lev = (uint32_t)j.white;
        p.a = 1ull | ((uint64_t)c0 << 32);
        p.b = (uint64_t)c1 | ((uint64_t)c2 << 32);
    } else {
        p.lev = (uint32_t)j.trash;
        p.a = 0;
        p.b = 0;
    }
    return p;
}

__device__ __forceinline__ void tile_wide(const Job& j, int tile, uint8_t* lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = j.radius;
    const TileGeom g = tile_geom(j, tile);
    const int yw0 = g.y0 + wave * j.rows;
    if (wave >= j.waves || lane >= j.lanes || yw0 >= g.yend) return;
    const int yw1 = min(yw0 + j.rows, g.yend);
    const uint32_t binstride = (uint32_t)j.lanes * 8u;
    uint8_t* ha = lds + (size_t)wave * 2 * j.bins * binstride + lane * 8;
    uint8_t* hb = ha + (size_t)j.bins * binstride;
    for (int k = 0; k < j.bins; ++k) {
        *reinterpret_cast<uint64_t*>(ha + k * binstride) = 0;
        *reinterpret_cast<uint64_t*>(hb + k * binstride) = 0;
    }
    const int x = g.x0 + lane;
    const int span = 2 * r + 1;
    for (int dy = 0; dy < span; ++dy) {
        for (int dx = 0; dx < span; ++dx) {
            const WidePix p = wide_pixel(j, x - r + dx, yw0 - r + dy);
            lds_add(reinterpret_cast<uint64_t*>(ha + p.lev * binstride), p.a);
            lds_add(reinterpret_cast<uint64_t*>(hb + p.lev * binstride), p.b);
        }
    }
    for (int y = yw0; y < yw1; ++y) {
        if (y > yw0) {
            for (int dx = 0; dx < span; ++dx) {
                const WidePix po = wide_pixel(j, x - r + dx, y - 1 - r);
                const WidePix pn = wide_pixel(j, x - r + dx, y + r);
                lds_sub(reinterpret_cast<uint64_t*>(ha + po.lev * binstride), po.a);
                lds_sub(reinterpret_cast<uint64_t*>(hb + po.lev * binstride), po.b);
                lds_add(reinterpret_cast<uint64_t*>(ha + pn.lev * binstride), pn.a);
                lds_add(reinterpret_cast<uint64_t*>(hb + pn.lev * binstride), pn.b);
            }
        }
        uint32_t bestc = 0, bestk = 0;
        for (int k = 0; k < j.scan; ++k) {
            const uint32_t c = (uint32_t)*reinterpret_cast<const uint64_t*>(ha + k * binstride);
            if (c > bestc) {
                bestc = c;
                bestk = (uint32_t)k;
            }
        }
        const uint64_t a = *reinterpret_cast<const uint64_t*>(ha + bestk * binstride);
        const uint64_t b = *reinterpret_cast<const uint64_t*>(hb + bestk * binstride);
        const uint32_t n = (uint32_t)a;
        bool store = x < j.width;
        if (j.paper) store = store && n > 0 && x >= r && x < j.width - r && y >= r && y < j.height - r;
        if (store && n > 0) {
            // floor of the correctly rounded double quotient is exact here:
            // s < 2^32 and n < 2^25, so s/n is at least 1/n away from the
            // next integer, far more than the rounding error.
            const double dn = (double)n;
            gdst_t o = gdst(j.dst) + (size_t)y * (size_t)j.dst_stride + 3 * x;
            o[0] = (uint8_t)(uint32_t)((double)(uint32_t)(a >> 32) / dn);
            o[1] = (uint8_t)(uint32_t)((double)(uint32_t)b / dn);
            o[2] = (uint8_t)(uint32_t)((double)(uint32_t)(b >> 32) / dn);
        }
    }
}

// STREAM layout, one wavefront per workgroup (tile_stream; the four-wavefront
// form is tile_stream_split below): 64 output columns, a run of `rows`
// output rows.  Only the 2r+4 image rows around the window are
// staged, in a ring, so the LDS a workgroup needs is its histogram plus a
// few KB: several wavefronts fit on a CU and runs can be long.  Image rows
// are fetched two rows ahead into registers.
//   LDS: [histogram: bins x 64 lanes x 8 B]
//        [ring: (2R+4) rows x (64+2R) entries -- or, while a run's first
//         window is built from column histograms, those]
//        [output row buffer: 192 B]
//   Ring slot of image row g: (g - (ya - R)) mod (2R+4).
// Ring rows beyond the 2r+1 of a window: the entering row and the two rows
// fetched ahead.
constexpr int kStreamRingExtra = 4;

// (a << 9) + b as one instruction.  Written out because the compiler turns
// (x >> s) << 9 into a shift and a mask, and then needs a third instruction
// for the add.
__device__ __forceinline__ uint32_t shl9_add(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, 9, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Ring entries.  Each window update needs a pixel's bin increment and its
// level; the entry is what makes both cheap for the bin format in use.
//   4 bytes (F16 bins, and F18 bins with 64 scanned levels): the staged word
//     {c0, c1, c2, level}.
//   8 bytes (F18 bins, at most 32 scanned levels): the increment itself,
//     count bit 54 set, with the level in bits 55..63 -- the count field's
//     upper bits, which one pixel's increment leaves zero; an update masks
//     them off (1 instruction) instead of assembling 18-bit fields.
template <bool W8>
struct RingFmt;

template <>
struct RingFmt<false> {
    using T = uint32_t;
    static __device__ __forceinline__ T entry(uint32_t c0, uint32_t c1, uint32_t c2, const Job& j) {
        return staged_word(c0, c1, c2, j);
    }
    static __device__ __forceinline__ T outside(const Job& j) { return (uint32_t)j.trash << 24; }
    static __device__ __forceinline__ uint32_t bin(T e) { return e >> 24; }
    static __device__ __forceinline__ uint32_t bin_field(T e) { return e >> 24; }
    template <bool F16>
    static __device__ __forceinline__ uint64_t inc(T e) { return BinFmt<F16>::inc(e); }
};

template <>
struct RingFmt<true> {
    using T = uint64_t;
    static __device__ __forceinline__ T entry(uint32_t c0, uint32_t c1, uint32_t c2, const Job& j) {
        uint32_t lev = level_of(c0 + c1 + c2, (uint32_t)j.levels, j.paper != 0);
        if (lev >= (uint32_t)j.levels) lev = (uint32_t)j.white;  // paper form: pure white
        const uint32_t lo = c0 | (c1 << 18);
        const uint32_t hi = (c2 << 4) | (1u << 22) | (lev << 23);
        return ((uint64_t)hi << 32) | lo;
    }
    static __device__ __forceinline__ T outside(const Job& j) {
        return (uint64_t)((1u << 22) | ((uint32_t)j.trash << 23)) << 32;
    }
    static __device__ __forceinline__ uint32_t bin(T e) { return (uint32_t)(e >> 55); }
    static __device__ __forceinline__ uint32_t bin_field(T e) { return (uint32_t)(e >> 55); }
    template <bool F16>
    static __device__ __forceinline__ uint64_t inc(T e) {
        static_assert(!F16, "8-byte entries carry F18 increments");
        return e & 0x007FFFFFFFFFFFFFull;
    }
};

struct RowBytes {
    uint32_t a0, a1, a2, b0, b1, b2;  // pixels at columns lane and lane + 64
    bool ina, inb;                    // real pixels (else: outside the image)
};

// Bytes of image row gy at columns x0-R+lane and x0-R+lane+64.  The loads
// are unconditional -- coordinates are clamped into the image and a flag
// records whether the pixel is real -- so that no branch surrounds them and
// the wait for their data can be placed exactly, two steps later.
template <int R>
__device__ __forceinline__ void stream_load_row(const Job& j, int x0, int gy, RowBytes& rb) {
    const int lane = threadIdx.x & 63;
    const bool row_in = gy >= 0 && gy < j.height;
    const int gxa = x0 - R + lane;
    const int gxb = gxa + 64;
    const int gyc = min(max(gy, 0), j.height - 1);
    const int xa = min(max(gxa, 0), j.width - 1);
    const int xb = min(gxb, j.width - 1);
    gsrc_t row = gsrc(j.src) + (size_t)gyc * (size_t)j.stride;
    rb.a0 = row[3 * xa];
    rb.a1 = row[3 * xa + 1];
    rb.a2 = row[3 * xa + 2];
    rb.ina = row_in && gxa >= 0 && gxa < j.width;
    if (R > 0) {
        rb.b0 = row[3 * xb];
        rb.b1 = row[3 * xb + 1];
        rb.b2 = row[3 * xb + 2];
        rb.inb = row_in && lane < 2 * R && gxb < j.width;
    }
}

template <int R, bool W8>
__device__ __forceinline__ void stream_write_row(const Job& j, typename RingFmt<W8>::T* slot, const RowBytes& rb) {
    using RF = RingFmt<W8>;
    const int lane = threadIdx.x & 63;
    const typename RF::T out = RF::outside(j);
    slot[lane] = rb.ina ? RF::entry(rb.a0, rb.a1, rb.a2, j) : out;
    if (R > 0 && lane < 2 * R) slot[lane + 64] = rb.inb ? RF::entry(rb.b0, rb.b1, rb.b2, j) : out;
}

// Image pixel p of the (64+2R)-wide block whose top-left pixel is
// (x0 - R, y0 - R): its entry (outside pixels get the trash level), loaded
// with clamped coordinates so that the loads need no branch.
template <int R, bool W8>
struct PixelAt {
    static constexpr int TW = 64 + 2 * R;
    int row, col;
    uint32_t c0, c1, c2;
    bool in;
    __device__ __forceinline__ void load(const Job& j, int x0, int y0, int p) {
        row = p / TW;
        col = p - row * TW;
        const int gy = y0 - R + row;
        const int gx = x0 - R + col;
        in = gy >= 0 && gy < j.height && gx >= 0 && gx < j.width;
        const int gyc = min(max(gy, 0), j.height - 1);
        const int gxc = min(max(gx, 0), j.width - 1);
        gsrc_t q = gsrc(j.src) + (size_t)gyc * (size_t)j.stride + 3 * gxc;
        c0 = q[0];
        c1 = q[1];
        c2 = q[2];
    }
    __device__ __forceinline__ typename RingFmt<W8>::T entry(const Job& j) const {
        return in ? RingFmt<W8>::entry(c0, c1, c2, j) : RingFmt<W8>::outside(j);
    }
};

// Stage rows y0-R .. y0-R+nrows-1 of the strip (64+2R columns) into the
// ring, slot k holding row y0-R+k, by the NT threads of the workgroup;
// sixteen pixels per thread in flight (one wavefront per CU SIMD leaves
// little else to hide the memory latency).
template <int R, bool W8, int NT = 64>
__device__ __forceinline__ void stage_ring(const Job& j, int x0, int y0, int nrows, typename RingFmt<W8>::T* ring) {
    constexpr int CH = 16;
    constexpr int TW = 64 + 2 * R;
    const int t = NT == 64 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
    const int npx = TW * nrows;
    for (int base = t; base < npx; base += CH * NT) {
        PixelAt<R, W8> px[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) px[i].load(j, x0, y0, min(base + i * NT, npx - 1));
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (base + i * NT < npx) ring[base + i * NT] = px[i].entry(j);
    }
}

// Radius 1 in the streamed layout (one wavefront, more than eight scanned
// levels): a 3 x 3 window holds at most nine levels, so the mode is found in
// registers -- a window pixel's
// count is the number of window pixels on its level, the largest count wins
// and the lowest level among equal counts -- and no histogram is kept.  The
// workgroup's LDS is the ring and the output row buffer only.  The window's
// staged words slide down in registers; each output row reads one ring row,
// issued before the row's mode is computed.  Levels at or above L (the
// paper form's white level, pixels outside the image) are never chosen.
__device__ __forceinline__ uint32_t direct9_pixel(const uint32_t (&v)[9], uint32_t levels, uint32_t& n) {
    uint32_t lev[9], cnt[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        lev[i] = v[i] >> 24;
        cnt[i] = 1;
    }
#pragma unroll
    for (int i = 1; i < 9; ++i)
#pragma unroll
        for (int k = 0; k < i; ++k) {
            const uint32_t eq = lev[i] == lev[k] ? 1u : 0u;
            cnt[i] += eq;
            cnt[k] += eq;
        }
    uint32_t best = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) best = max(best, lev[i] < levels ? (cnt[i] << 8) | (255u - lev[i]) : 0u);
    n = best >> 8;
    const uint32_t kb = 255u - (best & 255u);
    uint32_t s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (n > 0 && lev[i] == kb) {
            s0 += v[i] & 0xFFu;
            s1 += (v[i] >> 8) & 0xFFu;
            s2 += (v[i] >> 16) & 0xFFu;
        }
    const uint32_t nn = n ? n : 1u;
    const float rn = rcp_approx(nn);
    return div_exact(s0, nn, rn) | (div_exact(s1, nn, rn) << 8) | (div_exact(s2, nn, rn) << 16);
}

__device__ __forceinline__ void tile_direct1(const Job& j, int unit, uint8_t* lds) {
    constexpr int R = 1;
    constexpr int TW = 64 + 2 * R;
    constexpr int RB = kStreamRingExtra + 2 * R;  // ring rows
    const int lane = threadIdx.x & 63;
    const int tx = unit % j.tiles_x;
    const int ty = unit / j.tiles_x;
    const int x0 = tx * 64;
    const int ya = j.row_begin + ty * j.rows;
    const int yb = min(ya + j.rows, j.row_end);
    uint32_t* ring = reinterpret_cast<uint32_t*>(lds);
    uint8_t* obuf = lds + stream_ring_bytes(j);
    auto slot = [&](int g) { return ring + ((g - (ya - R)) % RB) * TW; };
    stage_ring<R, false>(j, x0, ya, 2 * R + 2, ring);
    lds_order();
    RowBytes q0, q1;
    stream_load_row<R>(j, x0, ya + 2 + R, q0);
    stream_load_row<R>(j, x0, ya + 3 + R, q1);
    // window rows ya-1, ya, ya+1 (slots 0 .. 2), words of columns lane .. lane+2
    uint32_t w[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) w[3 * r + c] = ring[r * TW + lane + c];
    auto row = [&](int y) {
        uint32_t nw[3] = {0u, 0u, 0u};
        if (y + 1 < yb) {
            const uint32_t* s = slot(y + 2) + lane;  // the row entering the next window
#pragma unroll
            for (int c = 0; c < 3; ++c) nw[c] = s[c];
        }
        uint32_t n;
        const uint32_t px = direct9_pixel(w, (uint32_t)j.levels, n);
        store_row(j, x0, y, n, px, obuf);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            w[c] = w[3 + c];
            w[3 + c] = w[6 + c];
            w[6 + c] = nw[c];
        }
    };
    // Two output rows per iteration; at the top rows y+3 and y+4 (fetched an
    // iteration earlier) enter the ring, into the slots of rows y-3 and y-2.
    int y = ya;
#pragma unroll 1
    for (; y < yb; y += 2) {
        if (y + 2 < yb) stream_write_row<R, false>(j, slot(y + 2 + R), q0);
        if (y + 3 < yb) stream_write_row<R, false>(j, slot(y + 3 + R), q1);
        lds_order();
        if (y + 4 < yb) stream_load_row<R>(j, x0, y + 4 + R, q0);
        if (y + 5 < yb) stream_load_row<R>(j, x0, y + 5 + R, q1);
        row(y);
        if (y + 1 < yb) row(y + 1);
    }
}

// Sum of the 2R+1 column entries col[0 .. 2R] (packed bin words; each field's
// total stays in range), as four independent chains: the additions of one
// chain wait on each other, so a single chain of 2R+1 would be latency-bound.
template <int R>
__device__ __forceinline__ uint64_t window_column_sum(const uint64_t* col) {
    constexpr int SPAN = 2 * R + 1;
    uint64_t a[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < SPAN; ++i) a[i & 3] += col[i];
    return (a[0] + a[1]) + (a[2] + a[3]);
}

// W8: 8-byte ring entries (OILPAINT_HIST_STREAM8: radius >= 8, SB = 32).
template <int R, int SB, bool W8>
__device__ __forceinline__ void tile_stream(const Job& j, int unit, uint8_t* lds) {
    if constexpr (R == 1 && !W8) {
        if (j.scan > 8) {  // eight bins scan faster than nine-way compares
            tile_direct1(j, unit, lds);
            return;
        }
    }
    static_assert(!W8 || (R >= 8 && SB == 32), "8-byte entries: F18 bins, at most 32 scanned levels");
    constexpr int SPAN = 2 * R + 1;
    constexpr int TW = 64 + 2 * R;
    constexpr int RB = kStreamRingExtra + 2 * R;  // ring rows
    constexpr uint32_t BS = 64u * 8u;
    constexpr bool F16 = R <= 7;
    using Fmt = BinFmt<F16>;
    using RF = RingFmt<W8>;
    using T = typename RF::T;
    const int lane = threadIdx.x & 63;
    const int scan = j.scan;
    const int tx = unit % j.tiles_x;
    const int ty = unit / j.tiles_x;
    const int x0 = tx * 64;
    const int ya = j.row_begin + ty * j.rows;
    const int yb = min(ya + j.rows, j.row_end);
    uint8_t* hl = lds + lane * 8;
    // bin row of an entry for this lane: level * 512 + lane * 8 (as an LDS
    // offset, so that the shift-add is the whole address computation)
    const uint32_t lane_off = lds_offset(hl);
    auto bin_ptr = [&](T e) { return lds_word(shl9_add(RF::bin_field(e), lane_off)); };
    uint8_t* region = lds + (size_t)j.bins * BS;
    T* ring = reinterpret_cast<T*>(region);
    uint8_t* obuf = region + stream_ring_bytes(j);  // one output row, 192 bytes
    auto slot = [&](int g) { return ring + ((g - (ya - R)) % RB) * TW; };

    if (j.colfirst) {
        // First window from column histograms, built in the ring region
        // before the ring is staged: row k of column c at colh + k*CW + c*8,
        // levels >= scan (paper white, outside pixels) in a sink row.  The
        // (64+2R) x (2R+1) window pixels are read from the image, spread
        // over the lanes (no two lanes of one instruction share a column).
        constexpr int CW = TW * 8;
        constexpr int NP = SPAN * TW;
        constexpr int CH = 12;
        uint8_t* colh = region;
        const int n16 = (scan + 1) * CW / 16;
        for (int e = lane; e < n16; e += 64) *reinterpret_cast<uint4*>(colh + e * 16) = make_uint4(0u, 0u, 0u, 0u);
        lds_order();
        for (int base = lane; base < NP; base += CH * 64) {
            PixelAt<R, W8> px[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) px[i].load(j, x0, ya, min(base + i * 64, NP - 1));
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const T e = px[i].entry(j);
                const uint32_t k = min(RF::bin(e), (uint32_t)scan);
                if (base + i * 64 < NP)
                    lds_add(reinterpret_cast<uint64_t*>(colh + k * CW + px[i].col * 8), RF::template inc<F16>(e));
            }
        }
        lds_order();
#pragma unroll 1
        for (int k = 0; k < scan; ++k) {
            const uint64_t* col = reinterpret_cast<const uint64_t*>(colh + k * CW) + lane;
            *reinterpret_cast<uint64_t*>(hl + k * BS) = window_column_sum<R>(col);
        }
    } else {
        for (int k = 0; k < j.bins; ++k) *reinterpret_cast<uint64_t*>(hl + k * BS) = 0;
    }
    // the ring (rows ya-R .. ya+R+1, slots 0 .. 2R+1) replaces the column
    // histograms; it is read across lanes: keep every read after every
    // write (one wavefront, and LDS executes its operations in issue order)
    lds_order();
    stage_ring<R, W8>(j, x0, ya, 2 * R + 2, ring);
    lds_order();
    // rows ya+2+R and ya+3+R are fetched now and staged at the top of the
    // first loop iteration
    RowBytes q0, q1;
    stream_load_row<R>(j, x0, ya + 2 + R, q0);
    stream_load_row<R>(j, x0, ya + 3 + R, q1);

    if (!j.colfirst) {
        // first window: slots 0 .. 2R
        const T* t = ring + lane;
        T w[SPAN];
#pragma unroll
        for (int i = 0; i < SPAN; ++i) w[i] = t[i];
#pragma unroll 1
        for (int dy = 0; dy < SPAN; ++dy) {
            T cur[SPAN];
#pragma unroll
            for (int i = 0; i < SPAN; ++i) cur[i] = w[i];
            t += TW;
            if (dy + 1 < SPAN) {
#pragma unroll
                for (int i = 0; i < SPAN; ++i) w[i] = t[i];
            }
#pragma unroll
            for (int i = 0; i < SPAN; ++i)
                lds_add(bin_ptr(cur[i]), RF::template inc<F16>(cur[i]));
        }
    }
    // entries of the step ya -> ya+1: leaving row ya-R, entering row ya+1+R
    T wo[SPAN], wn[SPAN];
    {
        const T* so = slot(ya - R) + lane;
        const T* sn = slot(ya + 1 + R) + lane;
#pragma unroll
        for (int i = 0; i < SPAN; ++i) {
            wo[i] = so[i];
            wn[i] = sn[i];
        }
    }
    ModeBins<SB> mb;
    mode_load<SB>(mb, hl, scan);

    // One output row y, then the step y -> y+1 and the entries of the next step.
    auto row_step = [&](int y, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        const uint32_t best = mode_reduce<SB, F16>(mb, scan);
        const uint32_t kbest = 63u - (best & 63u);
        const uint32_t n = best >> Fmt::kCountShift;
        const uint64_t win = *reinterpret_cast<const uint64_t*>(hl + kbest * BS);
        if (FULL || y + 1 < yb) {
#pragma unroll
            for (int i = 0; i < SPAN; ++i) {
                lds_sub(bin_ptr(wo[i]), RF::template inc<F16>(wo[i]));
                lds_add(bin_ptr(wn[i]), RF::template inc<F16>(wn[i]));
            }
            if (FULL || y + 2 < yb) {
                // step y+1 -> y+2 removes row y+1-R and adds row y+2+R
                const T* so = slot(y + 1 - R) + lane;
                const T* sn = slot(y + 2 + R) + lane;
#pragma unroll
                for (int i = 0; i < SPAN; ++i) {
                    wo[i] = so[i];
                    wn[i] = sn[i];
                }
            }
            mode_load<SB>(mb, hl, scan);
        }
        store_row(j, x0, y, n, finalize_packed<F16>(n, win), obuf);
    };
    // Two output rows per iteration.  At the top, rows y+2+R and y+3+R
    // (fetched one iteration earlier) enter the ring -- into the slots of rows
    // y-R-2 and y-R-1, which no window needs any more -- and rows y+4+R and
    // y+5+R are fetched for the next iteration.
    using Full = std::true_type;
    using Tail = std::false_type;
    int y = ya;
#pragma unroll 1
    for (; y + 5 < yb; y += 2) {
        stream_write_row<R, W8>(j, slot(y + 2 + R), q0);
        stream_write_row<R, W8>(j, slot(y + 3 + R), q1);
        lds_order();
        stream_load_row<R>(j, x0, y + 4 + R, q0);
        stream_load_row<R>(j, x0, y + 5 + R, q1);
        row_step(y, Full{});
        row_step(y + 1, Full{});
    }
#pragma unroll 1
    for (; y < yb; y += 2) {
        if (y + 2 < yb) stream_write_row<R, W8>(j, slot(y + 2 + R), q0);
        if (y + 3 < yb) stream_write_row<R, W8>(j, slot(y + 3 + R), q1);
        lds_order();
        if (y + 4 < yb) stream_load_row<R>(j, x0, y + 4 + R, q0);
        if (y + 5 < yb) stream_load_row<R>(j, x0, y + 5 + R, q1);
        row_step(y, Tail{});
        if (y + 1 < yb) row_step(y + 1, Tail{});
    }
}

// Persistent batch kernels: the next tile of a class's queue, taken by the
// workgroup's first lane (one wavefront per workgroup) and broadcast.  The
// compiler barrier keeps the previous tile's LDS accesses before it; one
// wavefront's LDS operations execute in issue order.
__device__ __forceinline__ int32_t next_tile_wave(uint32_t* counter) {
    lds_order();
    uint32_t t = 0;
    if ((threadIdx.x & 63) == 0) t = atomicAdd(counter, 1u);
    return (int32_t)__builtin_amdgcn_readfirstlane(t);
}

// Job holding queue index t (uniform): the last i with first_tile[i] <= t.
__device__ __forceinline__ int job_of(const BatchArgs& a, int32_t t) {
    int lo = 0, hi = a.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.first_tile[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One class of a batch in the streamed layout (radius R, scan bucket SB,
// ring entry size).
template <int R, int SB, bool W8>
__device__ __forceinline__ void batch_stream(const BatchArgs& a, uint8_t* lds) {
    for (;;) {
        const int32_t t = next_tile_wave(a.counter);
        if (t >= a.ntiles) break;
        const int i = job_of(a, t);
        const Job jb = a.jobs[i];
        tile_stream<R, SB, W8>(jb, t - a.first_tile[i], lds);
    }
}

// ---------------------------------------------------------------------------
// The streamed layout worked by four wavefronts per strip
// ---------------------------------------------------------------------------
// The strip, the run of rows, the histogram and the ring of tile_stream<R,
// SB, W8>, shared by kSplitWaves wavefronts.  Wavefront w makes the updates
// of window columns w*C .. w*C+C-1 (C = ceil((2r+1)/4)) of every row step and
// scans bins w*MB .. w*MB+MB-1 (the host pads the scanned levels to 4*MB with
// bins no pixel reaches).  Two workgroup barriers per output row: after the
// updates (the window is complete) and after the scans (every wavefront's
// best level -- its key and bin word -- is in LDS).  Then one wavefront,
// rotating, combines the four and stores the row while all of them go on
// with the next row step.  Each wavefront does a quarter of the work, and a
// CU holds four times the wavefronts at the same LDS footprint, which hides
// the LDS latency that one wavefront per strip leaves exposed.
//   LDS: [histogram: bins x 64 lanes x 8 B][ring region][output row: 192 B]
//        [keys: 64 lanes x 4 x 4 B][bin words: 4 x 64 lanes x 8 B]

// Wavefronts per SIMD the plain four-wavefront kernels are compiled for (the
// second launch bound): five workgroups of four per CU, which the LDS of a
// 4-byte ring at r = 15 and 20 levels allows, need at most 96 registers per
// lane; one register more would leave four resident.
constexpr int kSplitMinWaves = 5;

// Workgroup barrier for LDS traffic: waits for this wavefront's LDS
// operations only (global loads fetched ahead stay in flight), then meets
// the other wavefronts.  Every wavefront of the workgroup reaches every one.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Wavefront priority from a run's progress: the fewer rows done, the higher.
// The workgroups sharing a CU start together; left to the hardware, which
// favours the oldest wavefronts, the first ones finish well ahead of the last
// and the CU ends with too few wavefronts to hide the LDS latency.  With this
// they move together.  q1 < q2 < q3 are the quarter points of the run.
__device__ __forceinline__ void progress_priority(int done, int q1, int q2, int q3) {
    if (done < q1)
        __builtin_amdgcn_s_setprio(3);
    else if (done < q2)
        __builtin_amdgcn_s_setprio(2);
    else if (done < q3)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

// One output row y of the four-wavefront forms: wait for the window (first
// barrier), scan this wavefront's block of mb bins (MB, or at most MB with
// RT) for its best key, publish the key and the winning bin word, wait for
// the other wavefronts (second barrier), and let one wavefront, rotating by
// row, combine the four and store the row.  With four bins or more the scan
// keeps only the key and reads the winning word back: the window does not
// change before the second barrier.
template <int MB, bool RT, bool F16>
__device__ __forceinline__ void split_mode_row(const Job& j, int x0, int y, int ya, int w, int mb, uint8_t* hl,
                                               uint32_t* keys, uint64_t* words, uint8_t* obuf) {
    constexpr int NW = kSplitWaves;
    constexpr uint32_t BS = 64u * 8u;
    using Fmt = BinFmt<F16>;
    constexpr uint32_t M = Fmt::kCountMask;
    const int lane = threadIdx.x & 63;
    lds_barrier();  // window(y) complete
    uint64_t v[MB];
    const uint8_t* hb = hl + (size_t)(w * mb) * BS;
#pragma unroll
    for (int i = 0; i < MB; ++i)
        if (!RT || i < mb) v[i] = *reinterpret_cast<const uint64_t*>(hb + i * BS);
    uint32_t best = 0;
    uint64_t bw = 0;
    if constexpr (MB >= 4) {
        // whole-word reads: a read of the count halves alone (every other
        // dword) would meet a two-way bank conflict
#pragma unroll
        for (int i = 0; i < MB; ++i)
            if (!RT || i < mb) asm volatile("" ::"v"((uint32_t)v[i]));
#pragma unroll
        for (int i = 0; i < MB; ++i)
            if (!RT || i < mb) best = max(best, ((uint32_t)(v[i] >> 32) & M) | (uint32_t)(63 - w * mb - i));
        bw = *reinterpret_cast<const uint64_t*>(hl + (63u - (best & 63u)) * BS);
    } else {
#pragma unroll
        for (int i = 0; i < MB; ++i)
            if (!RT || i < mb) {
                const uint32_t key = ((uint32_t)(v[i] >> 32) & M) | (uint32_t)(63 - w * mb - i);
                if (key > best) {
                    best = key;
                    bw = v[i];
                }
            }
    }
    keys[lane * NW + w] = best;
    words[w * 64 + lane] = bw;
    lds_barrier();  // every wavefront's best is in LDS; the window may change
    if (w == ((y - ya) & (NW - 1))) {
        const uint4 kk = *reinterpret_cast<const uint4*>(keys + lane * NW);
        // the largest key (keys of different wavefronts differ in level)
        uint32_t top = kk.x, ww = 0;
        if (kk.y > top) top = kk.y, ww = 1;
        if (kk.z > top) top = kk.z, ww = 2;
        if (kk.w > top) top = kk.w, ww = 3;
        const uint64_t win = words[ww * 64 + lane];
        const uint32_t n = top >> Fmt::kCountShift;
        store_row(j, x0, y, n, finalize_packed<F16>(n, win), obuf);
    }
}

// MB: bins per wavefront, or with RT their maximum, the count being
// j.scan / kSplitWaves (the persistent batch kernels, one per radius and
// level bucket).
template <int R, int MB, bool W8, bool RT = false>
__device__ __forceinline__ void tile_stream_split(const Job& j, int unit, uint8_t* lds) {
    static_assert(R >= 0 && R <= 15 && MB >= 1 && kSplitWaves * MB <= 64, "level index must fit 6 bits");
    static_assert(!W8 || (R >= 8 && kSplitWaves * MB <= 32), "8-byte entries: F18 bins, at most 32 scanned levels");
    constexpr int NW = kSplitWaves;
    constexpr int NT = 64 * NW;
    constexpr int SPAN = 2 * R + 1;
    constexpr int TW = 64 + 2 * R;
    constexpr int RB = kStreamRingExtra + 2 * R;
    constexpr int C = (SPAN + NW - 1) / NW;      // window columns per wavefront
    constexpr int CMIN = SPAN - (NW - 1) * C;    // those of the last wavefront
    constexpr uint32_t BS = 64u * 8u;
    constexpr bool F16 = R <= 7;
    using RF = RingFmt<W8>;
    using T = typename RF::T;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int c0 = w * C;
    const int scan = j.scan;
    const int mb = RT ? scan / NW : MB;  // bins this wavefront scans
    const int tx = unit % j.tiles_x;
    const int ty = unit / j.tiles_x;
    const int x0 = tx * 64;
    const int ya = j.row_begin + ty * j.rows;
    const int yb = min(ya + j.rows, j.row_end);
    uint8_t* hl = lds + lane * 8;
    const uint32_t lane_off = lds_offset(hl);
    auto bin_ptr = [&](T e) { return lds_word(shl9_add(RF::bin_field(e), lane_off)); };
    uint8_t* region = lds + (size_t)j.bins * BS;
    T* ring = reinterpret_cast<T*>(region);
    uint8_t* obuf = region + stream_ring_bytes(j);
    uint32_t* keys = reinterpret_cast<uint32_t*>(obuf + 192);                    // [lane][w]
    uint64_t* words = reinterpret_cast<uint64_t*>(obuf + 192 + 64 * NW * 4);     // [w][lane]
    auto slot = [&](int g) { return ring + ((g - (ya - R)) % RB) * TW; };
    auto mine = [&](int c) { return c < CMIN || c0 + c < SPAN; };  // uniform

    {
        // One load round for the run's first 2R+2 ring rows (ya-R .. ya+R+1),
        // spread over all NT threads.  Their entries stay in registers while
        // the first window is built -- from column histograms of the 2R+1
        // window rows among them, in the ring region (as in tile_stream) --
        // and then enter the ring.
        constexpr int NS = (2 * R + 2) * TW;
        constexpr int CH = (NS + NT - 1) / NT;
        constexpr int CW = TW * 8;
        constexpr int NP = SPAN * TW;
        const int t = (int)threadIdx.x;
        T ent[CH];
        {
            PixelAt<R, W8> px[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) px[i].load(j, x0, ya, min(t + i * NT, NS - 1));
            // while the loads are in flight: clear the column histograms, or
            // the histogram that direct updates will fill
            if (j.colfirst) {
                const int n16 = (scan + 1) * CW / 16;
                for (int e = t; e < n16; e += NT)
                    *reinterpret_cast<uint4*>(region + e * 16) = make_uint4(0u, 0u, 0u, 0u);
            } else {
                for (int k = w; k < j.bins; k += NW) *reinterpret_cast<uint64_t*>(hl + k * BS) = 0;
            }
#pragma unroll
            for (int i = 0; i < CH; ++i) ent[i] = px[i].entry(j);
        }
        lds_barrier();
        if (j.colfirst) {
            uint8_t* colh = region;
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int p = t + i * NT;
                const uint32_t k = min(RF::bin(ent[i]), (uint32_t)scan);
                if (p < NP)
                    lds_add(reinterpret_cast<uint64_t*>(colh + k * CW + (p % TW) * 8), RF::template inc<F16>(ent[i]));
            }
            lds_barrier();
#pragma unroll 1
            for (int k = w; k < scan; k += NW) {
                const uint64_t* col = reinterpret_cast<const uint64_t*>(colh + k * CW) + lane;
                *reinterpret_cast<uint64_t*>(hl + k * BS) = window_column_sum<R>(col);
            }
            // the ring replaces the column histograms
            lds_barrier();
        }
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (t + i * NT < NS) ring[t + i * NT] = ent[i];
    }
    lds_barrier();
    // rows ya+2+R (wavefront 0) and ya+3+R (wavefront 1) are fetched now and
    // staged at the top of the first loop iteration
    RowBytes q;
    if (w < 2) stream_load_row<R>(j, x0, ya + 2 + R + w, q);

    if (!j.colfirst) {
        // first window: this wavefront's columns of slots 0 .. 2R
        const T* t = ring + lane + c0;
#pragma unroll 1
        for (int dy = 0; dy < SPAN; ++dy) {
            T cur[C];
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (mine(c)) cur[c] = t[c];
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (mine(c)) lds_add(bin_ptr(cur[c]), RF::template inc<F16>(cur[c]));
            t += TW;
        }
    }
    // entries of the step ya -> ya+1: leaving row ya-R, entering row ya+1+R
    T wo[C], wn[C];
    {
        const T* so = slot(ya - R) + lane + c0;
        const T* sn = slot(ya + 1 + R) + lane + c0;
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (mine(c)) {
                wo[c] = so[c];
                wn[c] = sn[c];
            }
    }

    // Output row y, then the step y -> y+1 and the entries of the next step.
    auto row_step = [&](int y, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        split_mode_row<MB, RT, F16>(j, x0, y, ya, w, mb, hl, keys, words, obuf);
        if (FULL || y + 1 < yb) {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (mine(c)) {
                    lds_sub(bin_ptr(wo[c]), RF::template inc<F16>(wo[c]));
                    lds_add(bin_ptr(wn[c]), RF::template inc<F16>(wn[c]));
                }
            if (FULL || y + 2 < yb) {
                // step y+1 -> y+2 removes row y+1-R and adds row y+2+R
                const T* so = slot(y + 1 - R) + lane + c0;
                const T* sn = slot(y + 2 + R) + lane + c0;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (mine(c)) {
                        wo[c] = so[c];
                        wn[c] = sn[c];
                    }
            }
        }
    };
    // Two output rows per iteration.  At the top, rows y+2+R and y+3+R
    // (fetched one iteration earlier by wavefronts 0 and 1) enter the ring --
    // into the slots of rows y-R-2 and y-R-1, which no window needs any more
    // -- and rows y+4+R and y+5+R are fetched.  The barriers of the two rows
    // order the ring writes before every read of them.
    using Full = std::true_type;
    using Tail = std::false_type;
    const int q1 = ya + (yb - ya) / 4, q2 = ya + (yb - ya) / 2, q3 = ya + 3 * (yb - ya) / 4;
    int y = ya;
#pragma unroll 1
    for (; y + 5 < yb; y += 2) {
        progress_priority(y, q1, q2, q3);
        if (w < 2) {
            stream_write_row<R, W8>(j, slot(y + 2 + R + w), q);
            stream_load_row<R>(j, x0, y + 4 + R + w, q);
        }
        row_step(y, Full{});
        row_step(y + 1, Full{});
    }
#pragma unroll 1
    for (; y < yb; y += 2) {
        if (w < 2) {
            if (y + 2 + w < yb) stream_write_row<R, W8>(j, slot(y + 2 + R + w), q);
            if (y + 4 + w < yb) stream_load_row<R>(j, x0, y + 4 + R + w, q);
        }
        row_step(y, Tail{});
        if (y + 1 < yb) row_step(y + 1, Tail{});
    }
}

// The four-wavefront form with 8-byte entries (ready bin increments: an
// update is 3 instructions instead of the 4-byte word's 7) keeps no ring of
// window rows, which at 8 bytes would not leave five workgroups per CU.  The
// first window comes from column histograms of the run's first 2r+2 rows,
// built from registers; afterwards each row step needs only its leaving and
// its entering row.  They sit in kSplitRows8 row slots: per pair of output
// rows the two entering rows (slots 2p, 2p+1) and the two leaving rows (slots
// 4+2p, 5+2p), p the pair's parity, one row per wavefront, fetched from the
// image one pair ahead (a leaving row comes from the image again: it was
// read 2r+1 rows earlier and sits in L2).
//   LDS: [histogram: bins x 64 lanes x 8 B]
//        [column histograms, then the row slots: kSplitRows8 x (64+2r) x 8 B]
//        [output row: 192 B][keys: 64 lanes x 4 x 4 B][bin words: 4 x 64 x 8 B]
template <int R, int MB, bool RT = false>
__device__ __forceinline__ void tile_stream_split8(const Job& j, int unit, uint8_t* lds) {
    static_assert(R >= 8 && R <= 15 && MB >= 1 && kSplitWaves * MB <= 32, "F18 bins, at most 32 scanned levels");
    constexpr int NW = kSplitWaves;
    constexpr int NT = 64 * NW;
    constexpr int SPAN = 2 * R + 1;
    constexpr int TW = 64 + 2 * R;
    constexpr int C = (SPAN + NW - 1) / NW;
    constexpr int CMIN = SPAN - (NW - 1) * C;
    constexpr uint32_t BS = 64u * 8u;
    using RF = RingFmt<true>;
    using T = uint64_t;
    const int lane = threadIdx.x & 63;
    const int t = (int)threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int c0 = w * C;
    const int scan = j.scan;
    const int mb = RT ? scan / NW : MB;
    const int tx = unit % j.tiles_x;
    const int ty = unit / j.tiles_x;
    const int x0 = tx * 64;
    const int ya = j.row_begin + ty * j.rows;
    const int yb = min(ya + j.rows, j.row_end);
    uint8_t* hl = lds + lane * 8;
    const uint32_t lane_off = lds_offset(hl);
    auto bin_ptr = [&](T e) { return lds_word(shl9_add(RF::bin_field(e), lane_off)); };
    uint8_t* region = lds + (size_t)j.bins * BS;
    T* rows8 = reinterpret_cast<T*>(region);
    uint8_t* obuf = region + stream_ring_bytes(j);
    uint32_t* keys = reinterpret_cast<uint32_t*>(obuf + 192);
    uint64_t* words = reinterpret_cast<uint64_t*>(obuf + 192 + 64 * NW * 4);
    auto mine = [&](int c) { return c < CMIN || c0 + c < SPAN; };
    // the image row each wavefront stages for the pair of output rows y, y+1:
    // entering y+2+R, y+3+R (wavefronts 0, 1), leaving y+1-R, y+2-R (2, 3)
    auto staged_row = [&](int y) { return w < 2 ? y + 2 + R + w : y + 1 - R + (w - 2); };
    auto slot_of = [&](int p) { return rows8 + (size_t)((w < 2 ? 0 : 4) + 2 * p + (w & 1)) * TW; };

    {
        // first window from column histograms of rows ya-R .. ya+R (one load
        // round for rows ya-R .. ya+R+1 over all threads, as in
        // tile_stream_split); rows ya-R and ya+1+R, the leaving and entering
        // rows of the first step, then go to slots 6 and 2 (parity 1, first
        // rewritten by the second pair)
        constexpr int NS = (2 * R + 2) * TW;
        constexpr int CH = (NS + NT - 1) / NT;
        constexpr int CW = TW * 8;
        constexpr int NP = SPAN * TW;
        T ent[CH];
        {
            PixelAt<R, true> px[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) px[i].load(j, x0, ya, min(t + i * NT, NS - 1));
            const int n16 = (scan + 1) * CW / 16;
            for (int e = t; e < n16; e += NT) *reinterpret_cast<uint4*>(region + e * 16) = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
            for (int i = 0; i < CH; ++i) ent[i] = px[i].entry(j);
        }
        lds_barrier();
        uint8_t* colh = region;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int p = t + i * NT;
            const uint32_t k = min(RF::bin(ent[i]), (uint32_t)scan);
            if (p < NP) lds_add(reinterpret_cast<uint64_t*>(colh + k * CW + (p % TW) * 8), RF::template inc<false>(ent[i]));
        }
        lds_barrier();
#pragma unroll 1
        for (int k = w; k < scan; k += NW) {
            const uint64_t* col = reinterpret_cast<const uint64_t*>(colh + k * CW) + lane;
            *reinterpret_cast<uint64_t*>(hl + k * BS) = window_column_sum<R>(col);
        }
        lds_barrier();  // the row slots replace the column histograms
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int p = t + i * NT;
            if (p < NS) {
                const int row = p / TW, col = p - row * TW;
                if (row == 0) rows8[6 * TW + col] = ent[i];
                if (row == 2 * R + 1) rows8[2 * TW + col] = ent[i];
            }
        }
    }
    RowBytes q;
    stream_load_row<R>(j, x0, staged_row(ya), q);
    lds_barrier();
    T wo[C], wn[C];
    {
        const T* so = rows8 + 6 * TW + lane + c0;
        const T* sn = rows8 + 2 * TW + lane + c0;
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (mine(c)) {
                wo[c] = so[c];
                wn[c] = sn[c];
            }
    }

    // Output row y (k = 0 or 1 within its pair, p the pair's parity), then the
    // step y -> y+1 and the entries of the next step.
    auto row_step = [&](int y, int p, int k) {
        split_mode_row<MB, RT, false>(j, x0, y, ya, w, mb, hl, keys, words, obuf);
        if (y + 1 < yb) {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (mine(c)) {
                    lds_sub(bin_ptr(wo[c]), RF::template inc<false>(wo[c]));
                    lds_add(bin_ptr(wn[c]), RF::template inc<false>(wn[c]));
                }
            if (y + 2 < yb) {
                // step y+1 -> y+2: leaving row y+1-R (slot 4+2p+k), entering
                // row y+2+R (slot 2p+k)
                const T* so = rows8 + (size_t)(4 + 2 * p + k) * TW + lane + c0;
                const T* sn = rows8 + (size_t)(2 * p + k) * TW + lane + c0;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (mine(c)) {
                        wo[c] = so[c];
                        wn[c] = sn[c];
                    }
            }
        }
    };
    const int q1 = ya + (yb - ya) / 4, q2 = ya + (yb - ya) / 2, q3 = ya + 3 * (yb - ya) / 4;
    int y = ya;
#pragma unroll 1
    for (int it = 0; y < yb; y += 2, ++it) {
        const int p = it & 1;
        progress_priority(y, q1, q2, q3);
        // this pair's rows enter their slots (the same parity's slots were last
        // read two pairs ago, before the barriers since); the next pair's are
        // fetched
        if (y + 2 + (w & 1) < yb) stream_write_row<R, true>(j, slot_of(p), q);
        if (y + 4 + (w & 1) < yb) stream_load_row<R>(j, x0, staged_row(y + 2), q);
        row_step(y, p, 0);
        if (y + 1 < yb) row_step(y + 1, p, 1);
    }
}

// Persistent batch form: the next tile of the class's queue, taken by the
// workgroup's first thread and handed to all four wavefronts through LDS.
// The barrier after the hand-over also orders the previous tile's last LDS
// accesses before the next tile's first ones; the next hand-over comes only
// after every wavefront has read this one (the tile's own barriers lie
// between).
template <int R, int MB, bool W8>
__device__ __forceinline__ void batch_stream_split(const BatchArgs& a, uint8_t* lds) {
    __shared__ int32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = (int32_t)atomicAdd(a.counter, 1u);
        lds_barrier();
        const int32_t t = __builtin_amdgcn_readfirstlane(next);
        if (t >= a.ntiles) break;
        const int i = job_of(a, t);
        const Job jb = a.jobs[i];
        if constexpr (W8)
            tile_stream_split8<R, MB, true>(jb, t - a.first_tile[i], lds);
        else
            tile_stream_split<R, MB, false, true>(jb, t - a.first_tile[i], lds);
    }
}

}  // namespace dev
}  // namespace oilpaint_impl
