// gfx950 kernels of the oil-paint filter.
//
// The method (Section 4 of the paper: histogram-based oil paint, its serial
// listing; Section 5: the same body run row-parallel): for each output
// pixel, bin the pixels of its (2r+1)^2 window by intensity level, keep per
// level a pixel count and three channel sums, pick the most populated level
// (lowest on ties) and output that level's channel sums divided by its count.
//
// How it is laid out on the GPU (the paper rebuilds the whole window for
// every pixel; none of the structure below is in the paper):
//   * A workgroup computes one tile: `lanes` output columns by
//     waves * rows output rows.  Lane l of wavefront w owns column x0 + l and
//     output rows [y0 + w*rows, y0 + (w+1)*rows).
//   * PACKED layout: the tile plus an r-pixel halo is staged once into LDS,
//     one 32-bit word per pixel {c0, c1, c2, level}; the level is computed
//     once per staged pixel.  Pixels outside the image get a spare level
//     (the "trash" bin) that the mode search never scans, so the window needs
//     no clipping logic.  Each lane keeps its window histogram in LDS, one
//     64-bit word per level (count:10 | sum2:18 | sum1:18 | sum0:18), bins
//     interleaved across lanes (bin k of lane l at k*lanes*8 + l*8), which
//     keeps every lane on its own bank whatever level it touches.  Moving
//     one row down removes the leaving row and adds the entering row of the
//     window: 2(2r+1) 64-bit LDS atomics instead of a (2r+1)^2 rebuild.
//     No field can carry into the next: each stays within its range.
//   * The mode search scans the lane's bins with the key
//     (count << 22) | (255 - level), whose maximum is the most populated
//     level with the lowest index among ties.
//   * The division is exact (see div_exact).
//   * WIDE layout (windows wider than 31 or more than 255 levels): two
//     64-bit words per level with 32-bit count and sums, pixels read from
//     device memory.
#include "oilpaint_internal.h"

namespace oilpaint_impl {
namespace {

// floor(s / n) for 1 <= n <= 961 and s <= 255 n, without a divide: the float
// estimate s * (1/n) is within 1e-4 of s/n (s < 2^18, relative error of the
// reciprocal and the product a few ulp), and s/n lies at least 1/961 below
// the next integer, so truncating the estimate gives floor(s/n) or one less;
// the integer checks correct either way.
__device__ __forceinline__ uint32_t div_exact(uint32_t s, uint32_t n, float rn) {
    uint32_t q = (uint32_t)((float)s * rn);
    q += ((q + 1u) * n <= s) ? 1u : 0u;
    q -= (q * n > s) ? 1u : 0u;
    return q;
}

// Intensity level of a pixel with channel sum s (Section 4 listing, level
// step).  Default reading: ((s / 3) * L) / 256, truncating, with
// s / 3 == (s * 43691) >> 17 for s <= 765.  Paper form: floor(s * L / 765)
// (equal to the listing's double expression for every s <= 765, L <= 256),
// with floor(x / 765) == mulhi(x, 5614337) for x <= 765 * 256.
__device__ __forceinline__ uint32_t level_of(uint32_t s, uint32_t L, bool paper) {
    if (paper) return __umulhi(s * L, 5614337u);
    return (((s * 43691u) >> 17) * L) >> 8;
}

// Image pointers as global-address-space pointers, so loads and stores are
// global_* instructions (flat ones would also count against the LDS wait
// counter and serialize with the histogram traffic).
typedef const __attribute__((address_space(1))) uint8_t* gsrc_t;
typedef __attribute__((address_space(1))) uint8_t* gdst_t;
__device__ __forceinline__ gsrc_t gsrc(const uint8_t* p) { return (gsrc_t)p; }
__device__ __forceinline__ gdst_t gdst(uint8_t* p) { return (gdst_t)p; }

template <typename T>
__device__ __forceinline__ void lds_add(T* p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void lds_sub(T* p, T v) {
    __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// 64-bit packed bin increment for a staged word {c0, c1, c2, level}.
__device__ __forceinline__ uint64_t packed_value(uint32_t w) {
    const uint32_t lo = (w & 0xFFu) | (((w >> 8) & 0xFFu) << 18);
    const uint32_t hi = (((w >> 16) & 0xFFu) << 4) | (1u << 22);
    return ((uint64_t)hi << 32) | lo;
}

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
    const float rn = __frcp_rn((float)n);
    gdst_t o = gdst(j.dst) + (size_t)y * (size_t)j.dst_stride + 3 * x;
    o[0] = (uint8_t)div_exact(s0, n, rn);
    o[1] = (uint8_t)div_exact(s1, n, rn);
    o[2] = (uint8_t)div_exact(s2, n, rn);
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

// Batch form: every layout in one kernel, selected per tile.
__device__ __forceinline__ void run_tile(const Job& j, int tile, uint8_t* lds) {
    if (j.hist == OILPAINT_HIST_WIDE) {
        tile_wide(j, tile, lds);
        return;
    }
    if (j.fast) {
        const bool small = j.scan <= 32;
        switch (j.radius) {
#define OILPAINT_FAST_CASE(R)                                              \
    case R:                                                                \
        if (small)                                                         \
            tile_packed_fast<R, 32>(j, tile, lds);                         \
        else                                                               \
            tile_packed_fast<R, 64>(j, tile, lds);                         \
        return;
            OILPAINT_FAST_CASE(0) OILPAINT_FAST_CASE(1) OILPAINT_FAST_CASE(2) OILPAINT_FAST_CASE(3)
            OILPAINT_FAST_CASE(4) OILPAINT_FAST_CASE(5) OILPAINT_FAST_CASE(6) OILPAINT_FAST_CASE(7)
            OILPAINT_FAST_CASE(8) OILPAINT_FAST_CASE(9) OILPAINT_FAST_CASE(10) OILPAINT_FAST_CASE(11)
            OILPAINT_FAST_CASE(12) OILPAINT_FAST_CASE(13) OILPAINT_FAST_CASE(14) OILPAINT_FAST_CASE(15)
#undef OILPAINT_FAST_CASE
            default: break;
        }
    }
    tile_packed(j, tile, lds);
}

// One workgroup per tile, generic layouts (at most 8 wavefronts, so that a
// lane may hold up to 256 registers).
__global__ __launch_bounds__(512) void k_plain(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    if (j.hist == OILPAINT_HIST_WIDE)
        tile_wide(j, blockIdx.x, lds);
    else
        tile_packed(j, blockIdx.x, lds);
}

// One workgroup per tile, fast path for one (radius, scan bucket): each
// instantiation gets the registers its own radius needs.
template <int R, int SB>
__global__ __launch_bounds__(512) void k_plain_fast(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_packed_fast<R, SB>(j, blockIdx.x, lds);
}

// Persistent: workgroups pull tiles from a counter until the queue is empty.
__global__ __launch_bounds__(256) void k_batch(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ int32_t s_tile;
    for (;;) {
        __syncthreads();  // the previous tile's LDS reads are done
        if (threadIdx.x == 0) s_tile = (int32_t)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int32_t t = __builtin_amdgcn_readfirstlane(s_tile);
        if (t >= a.ntiles) break;
        // job holding queue index t: last i with first_tile[i] <= t
        int lo = 0, hi = a.njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.first_tile[mid] <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const Job jb = a.jobs[lo];
        run_tile(jb, t - a.first_tile[lo], lds);
    }
}

__global__ void k_reset(uint32_t* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

}  // namespace

// Allow dynamic LDS above the default 64 KB once per kernel: the device's
// per-workgroup LDS minus what the kernel declares statically.
static hipError_t allow_lds(const void* kernel, size_t lds, int& done) {
    if (lds <= 65536 || __atomic_load_n(&done, __ATOMIC_ACQUIRE)) return hipSuccess;
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return note_hip("hipGetDevice", e);
    const DeviceInfo d = device_info(device);
    hipFuncAttributes fa;
    e = hipFuncGetAttributes(&fa, kernel);
    if (e != hipSuccess) return note_hip("hipFuncGetAttributes", e);
    const size_t total = d.ok ? d.lds_per_block : 65536;
    const int dyn = (int)(total > fa.sharedSizeBytes ? total - fa.sharedSizeBytes : 0);
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (e != hipSuccess) return note_hip("hipFuncSetAttribute", e);
    __atomic_store_n(&done, 1, __ATOMIC_RELEASE);
    return hipSuccess;
}

namespace {
typedef void (*PlainKernel)(Job);

// Fast kernels by [radius][scan bucket 16 / 32 / 64].
#define OILPAINT_FAST_ROW(R) {k_plain_fast<R, 16>, k_plain_fast<R, 32>, k_plain_fast<R, 64>}
const PlainKernel kFast[kPackedMaxRadius + 1][3] = {
    OILPAINT_FAST_ROW(0),  OILPAINT_FAST_ROW(1),  OILPAINT_FAST_ROW(2),  OILPAINT_FAST_ROW(3),
    OILPAINT_FAST_ROW(4),  OILPAINT_FAST_ROW(5),  OILPAINT_FAST_ROW(6),  OILPAINT_FAST_ROW(7),
    OILPAINT_FAST_ROW(8),  OILPAINT_FAST_ROW(9),  OILPAINT_FAST_ROW(10), OILPAINT_FAST_ROW(11),
    OILPAINT_FAST_ROW(12), OILPAINT_FAST_ROW(13), OILPAINT_FAST_ROW(14), OILPAINT_FAST_ROW(15)};
#undef OILPAINT_FAST_ROW
int g_fast_lds_done[kPackedMaxRadius + 1][3];
int g_plain_lds_done;
}  // namespace

hipError_t launch_plain(const Job& j, int waves, size_t lds, hipStream_t stream) {
    const int tiles = j.tiles_x * j.tiles_y;
    if (tiles <= 0) return hipSuccess;
    PlainKernel k = k_plain;
    int* done = &g_plain_lds_done;
    if (j.fast && j.radius >= 0 && j.radius <= kPackedMaxRadius && j.scan <= 64) {
        const int b = j.scan <= 16 ? 0 : j.scan <= 32 ? 1 : 2;
        k = kFast[j.radius][b];
        done = &g_fast_lds_done[j.radius][b];
    }
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(k), lds, *done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(tiles), dim3(64 * waves), lds, stream, j);
    return note_hip("k_plain launch", hipGetLastError());
}

hipError_t launch_batch(const BatchArgs& a, int waves, size_t lds, int grid, hipStream_t stream) {
    static int lds_done = 0;
    if (a.ntiles <= 0) return hipSuccess;
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(k_batch), lds, lds_done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(64 * waves), lds, stream, a);
    return note_hip("k_batch launch", hipGetLastError());
}

hipError_t launch_reset_counter(uint32_t* counter, hipStream_t stream) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, counter);
    return note_hip("k_reset launch", hipGetLastError());
}

int batch_grid(int device, int waves, size_t lds) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_batch), 64 * waves,
                                                     lds) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    const DeviceInfo d = device_info(device);
    return per_cu * (d.cus > 0 ? d.cus : 1);
}

}  // namespace oilpaint_impl
