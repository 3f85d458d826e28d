// Windowed median of one channel with column histograms (radius up to 127):
// the oil paint's column layout (tile_column) applied to the median, so that
// the work per output row does not grow with the radius (after Perreault and
// Hebert, "Median filtering in constant time", 2007).
//
// One wavefront per workgroup, 64 output columns, a run of rows.  For each
// of the 64+2r columns of the strip, LDS holds the histogram of its 2r+1
// window rows in two levels: 256 fine counts and 16 coarse counts (bins of
// 16 values), one byte each (a column holds at most 255 pixels), four to a
// 32-bit word; word k of column c at (k * TW + c) * 4, so that the lanes of
// an instruction, one column each, touch consecutive words.  Pixels outside
// the image are counted nowhere: a window's pixel count n comes from its
// clipped extent.  Per output row:
//   pass 1: the coarse counts are widened to two 16-bit fields per word and
//     prefix-summed across the strip (a wavefront scan per 64 columns); a
//     lane's window count of each coarse bin is the difference of two prefix
//     words (32-bit sums wrap, but each field's window total is below 2^16,
//     so the difference is exact field by field).  The coarse bin holding
//     rank floor((n-1)/2) follows from a cumulative scan of its 16 counts;
//   pass 2: the same for the 16 fine counts of that coarse bin, one set of
//     prefix sums per distinct coarse bin in the wavefront (neighbouring
//     pixels mostly share it);
//   then every column histogram loses its leaving pixel and gains its
//   entering one.
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

// Inclusive prefix sum over the 64 lanes of a wavefront (every lane active).
__device__ __forceinline__ uint32_t scan64(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

constexpr int kFineWords = 64;   // 256 one-byte counts
constexpr int kCoarseWords = 4;  // 16 one-byte counts

// Channel value of pixel (gx, gy), and whether it lies in the image (the
// load is unconditional: clamped coordinates).
__device__ __forceinline__ uint32_t mc_value(const MedianJob& j, int gx, int gy, bool& in) {
    in = gx >= 0 && gx < j.width && gy >= 0 && gy < j.height;
    const int gxc = min(max(gx, 0), j.width - 1);
    const int gyc = min(max(gy, 0), j.height - 1);
    return gsrc(j.src)[(size_t)gyc * (size_t)j.src_stride + (size_t)gxc * j.channels + j.channel];
}

// Add (sign +1) or remove (sign -1) value v in column c's histograms.
__device__ __forceinline__ void mc_update(uint8_t* lds, int TW, int c, uint32_t v, bool add) {
    uint32_t* fw = reinterpret_cast<uint32_t*>(lds) + (size_t)(v >> 2) * TW + c;
    uint32_t* cw = reinterpret_cast<uint32_t*>(lds) + (size_t)(kFineWords + (v >> 6)) * TW + c;
    const uint32_t fi = 1u << (8 * (v & 3u)), ci = 1u << (8 * ((v >> 4) & 3u));
    if (add) {
        __hip_atomic_fetch_add(fw, fi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(cw, ci, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        __hip_atomic_fetch_sub(fw, fi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_sub(cw, ci, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// Prefix sums across the strip of the 16 one-byte counts in words
// base .. base+3 of every column, widened to 16-bit fields (word i: counts
// 2i and 2i+1), into P (TW + 1 entries of 8 words; entry 0 stays 0).
template <int NT>
__device__ __forceinline__ void mc_prefix(const uint8_t* lds, int TW, int base, uint32_t* P) {
    const int lane = threadIdx.x & 63;
    uint32_t carry[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = lane + 64 * t;
        uint32_t s[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t w = c < TW ? reinterpret_cast<const uint32_t*>(lds)[(size_t)(base + i) * TW + c] : 0u;
            s[2 * i] = __builtin_amdgcn_perm(0u, w, 0x0C010C00u);      // counts 4i, 4i+1
            s[2 * i + 1] = __builtin_amdgcn_perm(0u, w, 0x0C030C02u);  // counts 4i+2, 4i+3
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] = scan64(s[i]) + carry[i];
        if (c < TW) {
            uint4* e = reinterpret_cast<uint4*>(P + (size_t)(c + 1) * 8);
            e[0] = make_uint4(s[0], s[1], s[2], s[3]);
            e[1] = make_uint4(s[4], s[5], s[6], s[7]);
        }
        if (t + 1 < NT) {
#pragma unroll
            for (int i = 0; i < 8; ++i) carry[i] = (uint32_t)__builtin_amdgcn_readlane((int)s[i], 63);
        }
    }
}

// A lane's window counts of the 16 bins: prefix at column lane + 2R + 1 minus
// prefix at column lane; then the number of bins whose running count stays at
// or below `rank` (the bin holding it) and the count before that bin.
__device__ __forceinline__ uint32_t mc_locate(const uint32_t* P, int lane, int R, uint32_t rank, uint32_t& before) {
    const uint4* hi = reinterpret_cast<const uint4*>(P + (size_t)(lane + 2 * R + 1) * 8);
    const uint4* lo = reinterpret_cast<const uint4*>(P + (size_t)lane * 8);
    const uint4 h0 = hi[0], h1 = hi[1], l0 = lo[0], l1 = lo[1];
    const uint32_t d[8] = {h0.x - l0.x, h0.y - l0.y, h0.z - l0.z, h0.w - l0.w,
                           h1.x - l1.x, h1.y - l1.y, h1.z - l1.z, h1.w - l1.w};
    uint32_t cum = before, b = 0, at = before;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            cum += (d[i] >> (16 * k)) & 0xFFFFu;
            const bool below = cum <= rank;
            b += below ? 1u : 0u;
            at = below ? cum : at;
        }
    }
    before = at;
    return b;
}

template <int NT>
__global__ __launch_bounds__(64) void k_median_column(MedianJob j) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int R = j.radius;
    const int TW = 64 + 2 * R;
    const int lane = threadIdx.x & 63;
    const int unit = xcd_tile();
    const int tx = unit % j.tiles_x;
    const int ty = unit / j.tiles_x;
    const int x0 = tx * 64;
    const int ya = ty * j.rows;
    const int yb = min(ya + j.rows, j.height);
    const size_t hist_bytes = ((size_t)(kFineWords + kCoarseWords) * TW * 4 + 15) & ~(size_t)15;
    uint32_t* P = reinterpret_cast<uint32_t*>(lds + hist_bytes);
    {
        const int n16 = (int)(hist_bytes / 16);
        for (int e = lane; e < n16; e += 64) reinterpret_cast<uint4*>(lds)[e] = make_uint4(0u, 0u, 0u, 0u);
        if (lane < 2) reinterpret_cast<uint4*>(P)[lane] = make_uint4(0u, 0u, 0u, 0u);
    }
    lds_order();
    // column histograms of rows ya-R .. ya+R
#pragma unroll 1
    for (int gy = ya - R; gy <= ya + R; ++gy) {
        uint32_t v[NT];
        bool in[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) v[t] = mc_value(j, x0 - R + lane + 64 * t, gy, in[t]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = lane + 64 * t;
            if (c < TW && in[t]) mc_update(lds, TW, c, v[t], true);
        }
    }
    lds_order();
    const int x = x0 + lane;
    const int cols_in = min(x + R, j.width - 1) - max(x - R, 0) + 1;
#pragma unroll 1
    for (int y = ya; y < yb; ++y) {
        // the step's pixels, fetched now and applied after the row
        const bool step = y + 1 < yb;
        uint32_t vo[NT], vn[NT];
        bool io[NT], inn[NT];
        if (step) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                vo[t] = mc_value(j, x0 - R + lane + 64 * t, y - R, io[t]);
                vn[t] = mc_value(j, x0 - R + lane + 64 * t, y + 1 + R, inn[t]);
            }
        }
        // the lower median: rank floor((n-1)/2) of the n window values
        const int rows_in = min(y + R, j.height - 1) - max(y - R, 0) + 1;
        const uint32_t rank = (uint32_t)(rows_in * cols_in - 1) / 2u;
        mc_prefix<NT>(lds, TW, kFineWords, P);
        lds_order();
        uint32_t before = 0;
        const uint32_t cb = mc_locate(P, lane, R, rank, before);
        lds_order();
        uint32_t val = 0;
        uint64_t pending = __ballot(x < j.width);
        while (pending) {
            const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)cb, (int)__builtin_ctzll(pending));
            mc_prefix<NT>(lds, TW, (int)(4 * k), P);
            lds_order();
            const bool mine = x < j.width && cb == k;
            if (mine) {
                uint32_t bf = before;
                val = 16u * k + mc_locate(P, lane, R, rank, bf);
            }
            pending &= ~__ballot(mine);
            lds_order();
        }
        if (x < j.width) gdst(j.dst)[(size_t)y * (size_t)j.dst_stride + x] = (uint8_t)val;
        if (step) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int c = lane + 64 * t;
                if (c < TW) {
                    if (io[t]) mc_update(lds, TW, c, vo[t], false);
                    if (inn[t]) mc_update(lds, TW, c, vn[t], true);
                }
            }
            lds_order();
        }
    }
}

}  // namespace

// By 64-column chunks of the strip with its halo, ceil((64 + 2r) / 64) - 1.
const MedianKernel kMedianColumn[kMedianColumnChunks] = {k_median_column<1>, k_median_column<2>, k_median_column<3>,
                                                         k_median_column<4>, k_median_column<5>};

size_t median_column_lds_bytes(int radius) {
    const size_t tw = 64 + 2 * (size_t)radius;
    return (((size_t)(kFineWords + kCoarseWords) * tw * 4 + 15) & ~(size_t)15) + (tw + 1) * 32;
}

}  // namespace oilpaint_impl
