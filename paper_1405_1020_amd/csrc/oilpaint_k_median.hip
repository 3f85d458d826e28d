// Windowed median of one channel: the second filter of the oil paint's class
// (a per-window histogram of pixel values queried per output pixel; the
// paper's conclusions name this class of image filters).  For every output
// pixel, the lower median -- the element of rank floor((n-1)/2) of the n
// channel values in its (2r+1) x (2r+1) window clipped to the image -- into
// a one-channel image.
//
// Layout (the oil paint's streamed layout with another histogram): one
// wavefront per workgroup, 64 output columns, a run of rows; the 2r+3 image
// rows around the window sit in a ring of 16-bit channel values (256 marks a
// pixel outside the image).  Each lane keeps a two-level count histogram of
// its window in LDS: fine counts of the 256 values and coarse counts of 16
// bins of 16 values, CB-bit counts packed 32/CB to a word (8-bit for
// windows up to 15 x 15, else 16-bit), one sink word per level for outside
// pixels.  Word w of lane l sits at w*256 + l*4.  Moving one row down
// updates both levels for the leaving and the entering window row; the
// median is found by a cumulative scan of the coarse counts to the bin
// holding the rank, then of that bin's 16 fine counts.  A step's ring values
// are read into registers before its first update (reads placed after the
// atomics could not be moved ahead of them, and each would wait for every
// atomic before it): the next step's values at the end of each step, a
// whole window row at a time for the first window.
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int R>
struct MedianFmt {
    static constexpr int CB = R <= 7 ? 8 : 16;            // bits per count
    static constexpr int PER = 32 / CB;                   // counts per word
    static constexpr uint32_t MASK = (1u << CB) - 1u;
    static constexpr int FW = 256 / PER + 1;              // fine words, sink included
    static constexpr int CW = 16 / PER + 1;               // coarse words, sink included
    static constexpr int NW = FW + CW;
    static constexpr int SPAN = 2 * R + 1;
    static constexpr int TW = 64 + 2 * R;
    static constexpr int RB = 2 * R + 3;                  // ring rows
};

// Channel value of image pixel (gx, gy), or 256 outside the image; the load
// is unconditional (clamped coordinates).
__device__ __forceinline__ uint32_t median_value(const MedianJob& j, int gx, int gy) {
    const bool in = gx >= 0 && gx < j.width && gy >= 0 && gy < j.height;
    const int gxc = min(max(gx, 0), j.width - 1);
    const int gyc = min(max(gy, 0), j.height - 1);
    const uint32_t v = gsrc(j.src)[(size_t)gyc * (size_t)j.src_stride + (size_t)gxc * j.channels + j.channel];
    return in ? v : 256u;
}

template <int R>
__device__ __forceinline__ void median_update(uint8_t* lds, uint32_t lane4, uint32_t v, bool add) {
    using F = MedianFmt<R>;
    const uint32_t fw = v / F::PER, fs = (v % F::PER) * F::CB;
    const uint32_t cbin = v >> 4;
    const uint32_t cw = F::FW + cbin / F::PER, cs = (cbin % F::PER) * F::CB;
    uint32_t* pf = reinterpret_cast<uint32_t*>(lds + fw * 256u + lane4);
    uint32_t* pc = reinterpret_cast<uint32_t*>(lds + cw * 256u + lane4);
    if (add) {
        lds_add(pf, 1u << fs);
        lds_add(pc, 1u << cs);
    } else {
        lds_sub(pf, 1u << fs);
        lds_sub(pc, 1u << cs);
    }
}

template <int R>
__global__ __launch_bounds__(64) void k_median(MedianJob j) {
    using F = MedianFmt<R>;
    extern __shared__ __align__(16) uint8_t lds[];
    const int lane = threadIdx.x & 63;
    const uint32_t lane4 = (uint32_t)lane * 4u;
    const int unit = xcd_tile();
    const int tx = unit % j.tiles_x;
    const int ty = unit / j.tiles_x;
    const int x0 = tx * 64;
    const int ya = ty * j.rows;
    const int yb = min(ya + j.rows, j.height);
    uint16_t* ring = reinterpret_cast<uint16_t*>(lds + F::NW * 256);
    auto slot = [&](int g) { return ring + ((g - (ya - R)) % F::RB) * F::TW; };

    // histogram cleared, rows ya-R .. ya+R+1 staged (ring slots 0 .. 2R+1)
    for (int w = 0; w < F::NW; ++w) *reinterpret_cast<uint32_t*>(lds + w * 256 + lane4) = 0u;
    for (int p = lane; p < (2 * R + 2) * F::TW; p += 64) {
        const int row = p / F::TW, col = p - row * F::TW;
        ring[p] = (uint16_t)median_value(j, x0 - R + col, ya - R + row);
    }
    lds_order();
    // the row fetched ahead: ya+2+R
    uint32_t qa = median_value(j, x0 - R + lane, ya + 2 + R);
    uint32_t qb = R > 0 ? median_value(j, x0 - R + lane + 64, ya + 2 + R) : 256u;
    // first window: slots 0 .. 2R, one row of values in registers ahead of
    // the row being added
    {
        uint32_t nxt[F::SPAN];
#pragma unroll
        for (int i = 0; i < F::SPAN; ++i) nxt[i] = ring[lane + i];
#pragma unroll 1
        for (int dy = 0; dy < F::SPAN; ++dy) {
            uint32_t cur[F::SPAN];
#pragma unroll
            for (int i = 0; i < F::SPAN; ++i) cur[i] = nxt[i];
            if (dy + 1 < F::SPAN) {
                const uint16_t* t = ring + (dy + 1) * F::TW + lane;
#pragma unroll
                for (int i = 0; i < F::SPAN; ++i) nxt[i] = t[i];
            }
#pragma unroll
            for (int i = 0; i < F::SPAN; ++i) median_update<R>(lds, lane4, cur[i], true);
        }
    }
    // values of the step ya -> ya+1: leaving row ya-R, entering row ya+1+R
    uint32_t vo[F::SPAN], vn[F::SPAN];
    {
        const uint16_t* so = slot(ya - R) + lane;
        const uint16_t* sn = slot(ya + 1 + R) + lane;
#pragma unroll
        for (int i = 0; i < F::SPAN; ++i) {
            vo[i] = so[i];
            vn[i] = sn[i];
        }
    }
    const int x = x0 + lane;
    const int cols_in = min(x + R, j.width - 1) - max(x - R, 0) + 1;
#pragma unroll 1
    for (int y = ya; y < yb; ++y) {
        // the row fetched ahead enters the ring (slot of row y-R-1, which no
        // window needs any more); the next one is fetched
        if (y + 2 + R < yb + R + 1) {
            uint16_t* s = slot(y + 2 + R);
            s[lane] = (uint16_t)qa;
            if (lane < 2 * R) s[lane + 64] = (uint16_t)qb;
            qa = median_value(j, x0 - R + lane, y + 3 + R);
            if (R > 0) qb = median_value(j, x0 - R + lane + 64, y + 3 + R);
        }
        lds_order();
        // the lower median: rank floor((n-1)/2) of the n window values
        const int rows_in = min(y + R, j.height - 1) - max(y - R, 0) + 1;
        const uint32_t rank = (uint32_t)(rows_in * cols_in - 1) / 2u;
        uint32_t cum = 0, before = 0, b = 0;
#pragma unroll
        for (int w = 0; w < 16 / F::PER; ++w) {
            const uint32_t word = *reinterpret_cast<const uint32_t*>(lds + (F::FW + w) * 256 + lane4);
#pragma unroll
            for (int k = 0; k < F::PER; ++k) {
                cum += (word >> (k * F::CB)) & F::MASK;
                const bool below = cum <= rank;
                b += below ? 1u : 0u;
                before = below ? cum : before;
            }
        }
        const uint8_t* fine = lds + b * (16u / F::PER) * 256u + lane4;
        cum = before;
        uint32_t v = 0;
#pragma unroll
        for (int w = 0; w < 16 / F::PER; ++w) {
            const uint32_t word = *reinterpret_cast<const uint32_t*>(fine + w * 256);
#pragma unroll
            for (int k = 0; k < F::PER; ++k) {
                cum += (word >> (k * F::CB)) & F::MASK;
                v += cum <= rank ? 1u : 0u;
            }
        }
        if (x < j.width) gdst(j.dst)[(size_t)y * (size_t)j.dst_stride + x] = (uint8_t)(16u * b + v);
        // step y -> y+1: row y-R leaves, row y+1+R enters; then the values
        // of the step y+1 -> y+2 (rows y+1-R and y+2+R, the latter staged at
        // the top of this iteration)
        if (y + 1 < yb) {
#pragma unroll
            for (int i = 0; i < F::SPAN; ++i) {
                median_update<R>(lds, lane4, vo[i], false);
                median_update<R>(lds, lane4, vn[i], true);
            }
            if (y + 2 < yb) {
                const uint16_t* so = slot(y + 1 - R) + lane;
                const uint16_t* sn = slot(y + 2 + R) + lane;
#pragma unroll
                for (int i = 0; i < F::SPAN; ++i) {
                    vo[i] = so[i];
                    vn[i] = sn[i];
                }
            }
        }
    }
}

// Four wavefronts per strip: the same histogram and ring shared by a
// 256-thread workgroup.  Wavefront w makes the updates of window columns
// w*C .. w*C+C-1 (C = ceil((2r+1)/4)) of every row step, so a strip keeps
// four times the LDS operations in flight (one wavefront may have at most
// fifteen outstanding, and a row step of the one-wavefront form holds
// 4(2r+1) atomics); one wavefront, rotating by row, answers the row's
// queries between two workgroup barriers: after the updates (the window is
// complete) and after the queries (the window may change).
template <int R>
__global__ __launch_bounds__(256) void k_median4(MedianJob j) {
    using F = MedianFmt<R>;
    constexpr int NV = 4;                         // wavefronts
    constexpr int C = (F::SPAN + NV - 1) / NV;    // window columns per wavefront
    constexpr int CMIN = F::SPAN - (NV - 1) * C;  // those of the last wavefront
    constexpr int NS = (2 * R + 2) * F::TW;       // staged values
    constexpr int CH = (NS + 64 * NV - 1) / (64 * NV);
    extern __shared__ __align__(16) uint8_t lds[];
    const int lane = threadIdx.x & 63;
    const int t = (int)threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int c0 = w * C;
    auto mine = [&](int c) { return c < CMIN || c0 + c < F::SPAN; };  // uniform
    const uint32_t lane4 = (uint32_t)lane * 4u;
    const int unit = xcd_tile();
    const int tx = unit % j.tiles_x;
    const int ty = unit / j.tiles_x;
    const int x0 = tx * 64;
    const int ya = ty * j.rows;
    const int yb = min(ya + j.rows, j.height);
    uint16_t* ring = reinterpret_cast<uint16_t*>(lds + F::NW * 256);
    auto slot = [&](int g) { return ring + ((g - (ya - R)) % F::RB) * F::TW; };

    // histogram cleared, rows ya-R .. ya+R+1 staged (ring slots 0 .. 2R+1)
    // in one load round over all threads
    {
        uint32_t v[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int p = min(t + i * 64 * NV, NS - 1);
            const int row = p / F::TW, col = p - row * F::TW;
            v[i] = median_value(j, x0 - R + col, ya - R + row);
        }
        for (int wd = w; wd < F::NW; wd += NV) *reinterpret_cast<uint32_t*>(lds + wd * 256 + lane4) = 0u;
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (t + i * 64 * NV < NS) ring[t + i * 64 * NV] = (uint16_t)v[i];
    }
    lds_barrier();
    // the row fetched ahead (wavefront 0): ya+2+R
    uint32_t qa = 256u, qb = 256u;
    if (w == 0) {
        qa = median_value(j, x0 - R + lane, ya + 2 + R);
        if (R > 0) qb = median_value(j, x0 - R + lane + 64, ya + 2 + R);
    }
    // first window: this wavefront's columns of slots 0 .. 2R
#pragma unroll 1
    for (int dy = 0; dy < F::SPAN; ++dy) {
        const uint16_t* r0 = ring + dy * F::TW + lane + c0;
        uint32_t cur[C];
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (mine(c)) cur[c] = r0[c];
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (mine(c)) median_update<R>(lds, lane4, cur[c], true);
    }
    // values of the step ya -> ya+1: leaving row ya-R, entering row ya+1+R
    uint32_t vo[C], vn[C];
    {
        const uint16_t* so = slot(ya - R) + lane + c0;
        const uint16_t* sn = slot(ya + 1 + R) + lane + c0;
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (mine(c)) {
                vo[c] = so[c];
                vn[c] = sn[c];
            }
    }
    const int x = x0 + lane;
    const int cols_in = min(x + R, j.width - 1) - max(x - R, 0) + 1;
    const int q1 = ya + (yb - ya) / 4, q2 = ya + (yb - ya) / 2, q3 = ya + 3 * (yb - ya) / 4;
#pragma unroll 1
    for (int y = ya; y < yb; ++y) {
        progress_priority(y, q1, q2, q3);
        // the row fetched ahead enters the ring (slot of row y-R-1, which no
        // window needs any more); the next one is fetched
        if (w == 0 && y + 1 < yb) {
            uint16_t* s = slot(y + 2 + R);
            s[lane] = (uint16_t)qa;
            if (lane < 2 * R) s[lane + 64] = (uint16_t)qb;
            qa = median_value(j, x0 - R + lane, y + 3 + R);
            if (R > 0) qb = median_value(j, x0 - R + lane + 64, y + 3 + R);
        }
        lds_barrier();  // window y complete, ring row y+2+R staged
        if (w == ((y - ya) & (NV - 1))) {
            // the lower median: rank floor((n-1)/2) of the n window values
            const int rows_in = min(y + R, j.height - 1) - max(y - R, 0) + 1;
            const uint32_t rank = (uint32_t)(rows_in * cols_in - 1) / 2u;
            uint32_t cum = 0, before = 0, b = 0;
#pragma unroll
            for (int wd = 0; wd < 16 / F::PER; ++wd) {
                const uint32_t word = *reinterpret_cast<const uint32_t*>(lds + (F::FW + wd) * 256 + lane4);
#pragma unroll
                for (int k = 0; k < F::PER; ++k) {
                    cum += (word >> (k * F::CB)) & F::MASK;
                    const bool below = cum <= rank;
                    b += below ? 1u : 0u;
                    before = below ? cum : before;
                }
            }
            const uint8_t* fine = lds + b * (16u / F::PER) * 256u + lane4;
            cum = before;
            uint32_t v = 0;
#pragma unroll
            for (int wd = 0; wd < 16 / F::PER; ++wd) {
                const uint32_t word = *reinterpret_cast<const uint32_t*>(fine + wd * 256);
#pragma unroll
                for (int k = 0; k < F::PER; ++k) {
                    cum += (word >> (k * F::CB)) & F::MASK;
                    v += cum <= rank ? 1u : 0u;
                }
            }
            if (x < j.width) gdst(j.dst)[(size_t)y * (size_t)j.dst_stride + x] = (uint8_t)(16u * b + v);
        }
        lds_barrier();  // the queries are answered; the window may change
        if (y + 1 < yb) {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (mine(c)) {
                    median_update<R>(lds, lane4, vo[c], false);
                    median_update<R>(lds, lane4, vn[c], true);
                }
            if (y + 2 < yb) {
                const uint16_t* so = slot(y + 1 - R) + lane + c0;
                const uint16_t* sn = slot(y + 2 + R) + lane + c0;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (mine(c)) {
                        vo[c] = so[c];
                        vn[c] = sn[c];
                    }
            }
        }
    }
}

}  // namespace

// By radius.
const MedianKernel kMedian[kMedianMaxRadius + 1] = {
    k_median<0>, k_median<1>, k_median<2>,  k_median<3>,  k_median<4>,  k_median<5>,  k_median<6>,  k_median<7>,
    k_median<8>, k_median<9>, k_median<10>, k_median<11>, k_median<12>, k_median<13>, k_median<14>, k_median<15>};
const MedianKernel kMedian4[kMedianMaxRadius + 1] = {
    k_median4<0>, k_median4<1>, k_median4<2>,  k_median4<3>,  k_median4<4>,  k_median4<5>,
    k_median4<6>, k_median4<7>, k_median4<8>,  k_median4<9>,  k_median4<10>, k_median4<11>,
    k_median4<12>, k_median4<13>, k_median4<14>, k_median4<15>};

size_t median_lds_bytes(int radius) {
    const int cb = radius <= 7 ? 8 : 16;
    const int per = 32 / cb;
    const int nw = 256 / per + 1 + 16 / per + 1;
    return (size_t)nw * 256 + (size_t)(2 * radius + 3) * (64 + 2 * radius) * 2;
}

}  // namespace oilpaint_impl
