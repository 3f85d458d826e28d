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
//   * A workgroup of NW wavefronts computes one tile: `lanes` output columns
//     by NW * rows output rows.  Lane l of wavefront w owns column x0 + l and
//     output rows [y0 + w*rows, y0 + (w+1)*rows).
//   * PACKED layout: the tile plus an r-pixel halo is staged once into LDS,
//     one 32-bit word per pixel {c0, c1, c2, level}; the level is computed
//     once per staged pixel.  Pixels outside the image get a spare level
//     (the "trash" bin) whose bin is never scanned, so the window needs no
//     clipping logic.  Each lane keeps its window histogram in LDS, one
//     64-bit word per level (count:10 | sum2:18 | sum1:18 | sum0:18), bins
//     interleaved across lanes (bin k of lane l at k*lanes*8 + l*8), which
//     keeps every lane on its own bank whatever level it touches.  Moving
//     one row down removes the leaving row and adds the entering row of the
//     window: 2(2r+1) 64-bit LDS atomics instead of a (2r+1)^2 rebuild.
//     No field can carry into the next: each stays within its range.
//   * The mode search scans the lane's bins with the key
//     (count << 22) | (255 - level), whose maximum is the most populated
//     level with the lowest index among ties.
//   * The division is exact: q = mulhi(s, ceil(2^32 / n)) for n <= 961 and
//     s <= 255 n.
//   * WIDE layout (windows wider than 31 or L = 256): two 64-bit words per
//     level with 32-bit count and sums, pixels read from device memory.
#include "oilpaint_internal.h"

namespace oilpaint_impl {
namespace {

struct MagicTable {
    uint32_t v[1024];
};

constexpr MagicTable make_magic() {
    MagicTable t{};
    for (uint32_t n = 2; n < 1024; ++n) t.v[n] = (uint32_t)((0x100000000ull + n - 1) / n);
    return t;
}

// ceil(2^32 / n), n = 2..1023; entries 0 and 1 are unused (0).
__constant__ MagicTable kMagic = make_magic();

__device__ __forceinline__ uint32_t div_packed(uint32_t s, uint32_t n) {
    return n == 1 ? s : __umulhi(s, kMagic.v[n & 1023u]);
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
    const int nw = j.waves;
    TileGeom g;
    const int tx = tile % j.tiles_x;
    const int ty = tile / j.tiles_x;
    g.x0 = tx * j.lanes;
    g.y0 = j.row_begin + ty * nw * j.rows;
    g.yend = min(g.y0 + nw * j.rows, j.row_end);
    g.tw = j.lanes + 2 * j.radius;
    g.th = (g.yend - g.y0) + 2 * j.radius;
    return g;
}

// ---------------------------------------------------------------------------
// PACKED layout
// ---------------------------------------------------------------------------
__device__ void tile_packed(const Job& j, int tile, uint8_t* lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwb = blockDim.x >> 6;  // wavefronts that stage
    const int nw = j.waves;           // wavefronts that compute
    const int r = j.radius;
    const uint32_t L = (uint32_t)j.levels;
    const bool paper = j.paper != 0;
    const uint32_t nscan = L;                     // levels the mode search scans
    const uint32_t trash = L + (paper ? 1u : 0u); // bin for pixels outside the image
    const TileGeom g = tile_geom(j, tile);

    // ---- stage tile + halo into LDS, one word per pixel -------------------
    uint32_t* tw32 = reinterpret_cast<uint32_t*>(lds);
    const uint32_t trash_word = trash << 24;
    for (int row = wave; row < g.th; row += nwb) {
        const int gy = g.y0 - r + row;
        uint32_t* trow = tw32 + row * g.tw;
        const bool row_in = gy >= 0 && gy < j.height;
        const uint8_t* srow = j.src + (row_in ? (size_t)gy * (size_t)j.stride : 0);
        for (int col = lane; col < g.tw; col += 64) {
            const int gx = g.x0 - r + col;
            uint32_t w = trash_word;
            if (row_in && gx >= 0 && gx < j.width) {
                const uint8_t* p = srow + 3 * gx;
                const uint32_t c0 = p[0], c1 = p[1], c2 = p[2];
                w = c0 | (c1 << 8) | (c2 << 16) | (level_of(c0 + c1 + c2, L, paper) << 24);
            }
            trow[col] = w;
        }
    }
    __syncthreads();

    // ---- per-lane sliding histogram --------------------------------------
    const int yw0 = g.y0 + wave * j.rows;
    if (wave < nw && lane < j.lanes && yw0 < g.yend) {
        const int yw1 = min(yw0 + j.rows, g.yend);
        const size_t tile_bytes = ((size_t)g.tw * (size_t)(nw * j.rows + 2 * r) * 4 + 15) & ~(size_t)15;
        const uint32_t nbins = trash + 1;
        const uint32_t binstride = (uint32_t)j.lanes * 8u;
        uint8_t* hl = lds + tile_bytes + (size_t)wave * nbins * binstride + lane * 8;
        for (uint32_t k = 0; k < nbins; ++k) *reinterpret_cast<uint64_t*>(hl + k * binstride) = 0;

        const int x = g.x0 + lane;
        const int span = 2 * r + 1;
        // first window: staged rows (yw0 - y0) .. +2r, columns lane .. lane + 2r
        {
            const uint32_t* t = tw32 + (yw0 - g.y0) * g.tw + lane;
            for (int dy = 0; dy < span; ++dy, t += g.tw) {
                for (int dx = 0; dx < span; ++dx) {
                    const uint32_t w = t[dx];
                    lds_add(reinterpret_cast<uint64_t*>(hl + (w >> 24) * binstride), packed_value(w));
                }
            }
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
            // mode search over levels 0 .. nscan-1
            uint32_t best = 0;
            for (uint32_t k = 0; k < nscan; ++k) {
                const uint64_t b = *reinterpret_cast<const uint64_t*>(hl + k * binstride);
                const uint32_t hi = (uint32_t)(b >> 32);
                best = max(best, (hi & 0xFFC00000u) | (255u - k));
            }
            const uint32_t n = best >> 22;
            const uint32_t kbest = 255u - (best & 0xFFu);
            const uint64_t b = *reinterpret_cast<const uint64_t*>(hl + kbest * binstride);
            const uint32_t lo = (uint32_t)b, hi = (uint32_t)(b >> 32);
            const uint32_t s0 = lo & 0x3FFFFu;
            const uint32_t s1 = (lo >> 18) | ((hi & 0xFu) << 14);
            const uint32_t s2 = (hi >> 4) & 0x3FFFFu;
            bool store = x < j.width;
            if (paper) store = store && n > 0 && x >= r && x < j.width - r && y >= r && y < j.height - r;
            if (store) {
                uint8_t* o = j.dst + (size_t)y * (size_t)j.dst_stride + 3 * x;
                o[0] = (uint8_t)div_packed(s0, n);
                o[1] = (uint8_t)div_packed(s1, n);
                o[2] = (uint8_t)div_packed(s2, n);
            }
        }
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

__device__ __forceinline__ WidePix wide_pixel(const Job& j, int gx, int gy, uint32_t L, bool paper,
                                              uint32_t trash) {
    WidePix p;
    if (gx >= 0 && gx < j.width && gy >= 0 && gy < j.height) {
        const uint8_t* q = j.src + (size_t)gy * (size_t)j.stride + 3 * gx;
        const uint32_t c0 = q[0], c1 = q[1], c2 = q[2];
        p.lev = level_of(c0 + c1 + c2, L, paper);
        p.a = 1ull | ((uint64_t)c0 << 32);
        p.b = (uint64_t)c1 | ((uint64_t)c2 << 32);
    } else {
        p.lev = trash;
        p.a = 0;
        p.b = 0;
    }
    return p;
}

__device__ void tile_wide(const Job& j, int tile, uint8_t* lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = j.radius;
    const uint32_t L = (uint32_t)j.levels;
    const bool paper = j.paper != 0;
    const uint32_t trash = L + (paper ? 1u : 0u);
    const TileGeom g = tile_geom(j, tile);
    const int yw0 = g.y0 + wave * j.rows;
    if (wave >= j.waves || lane >= j.lanes || yw0 >= g.yend) return;
    const int yw1 = min(yw0 + j.rows, g.yend);
    const uint32_t nbins = trash + 1;
    const uint32_t binstride = (uint32_t)j.lanes * 8u;
    uint8_t* ha = lds + (size_t)wave * 2 * nbins * binstride + lane * 8;
    uint8_t* hb = ha + nbins * binstride;
    for (uint32_t k = 0; k < nbins; ++k) {
        *reinterpret_cast<uint64_t*>(ha + k * binstride) = 0;
        *reinterpret_cast<uint64_t*>(hb + k * binstride) = 0;
    }
    const int x = g.x0 + lane;
    const int span = 2 * r + 1;
    for (int dy = 0; dy < span; ++dy) {
        for (int dx = 0; dx < span; ++dx) {
            const WidePix p = wide_pixel(j, x - r + dx, yw0 - r + dy, L, paper, trash);
            lds_add(reinterpret_cast<uint64_t*>(ha + p.lev * binstride), p.a);
            lds_add(reinterpret_cast<uint64_t*>(hb + p.lev * binstride), p.b);
        }
    }
    for (int y = yw0; y < yw1; ++y) {
        if (y > yw0) {
            for (int dx = 0; dx < span; ++dx) {
                const WidePix po = wide_pixel(j, x - r + dx, y - 1 - r, L, paper, trash);
                const WidePix pn = wide_pixel(j, x - r + dx, y + r, L, paper, trash);
                lds_sub(reinterpret_cast<uint64_t*>(ha + po.lev * binstride), po.a);
                lds_sub(reinterpret_cast<uint64_t*>(hb + po.lev * binstride), po.b);
                lds_add(reinterpret_cast<uint64_t*>(ha + pn.lev * binstride), pn.a);
                lds_add(reinterpret_cast<uint64_t*>(hb + pn.lev * binstride), pn.b);
            }
        }
        uint32_t bestc = 0, bestk = 0;
        for (uint32_t k = 0; k < L; ++k) {
            const uint32_t c = (uint32_t)*reinterpret_cast<const uint64_t*>(ha + k * binstride);
            if (c > bestc) {
                bestc = c;
                bestk = k;
            }
        }
        const uint64_t a = *reinterpret_cast<const uint64_t*>(ha + bestk * binstride);
        const uint64_t b = *reinterpret_cast<const uint64_t*>(hb + bestk * binstride);
        const uint32_t n = (uint32_t)a;
        bool store = x < j.width;
        if (paper) store = store && n > 0 && x >= r && x < j.width - r && y >= r && y < j.height - r;
        if (store && n > 0) {
            // floor of the correctly rounded double quotient is exact here:
            // s < 2^32 and n < 2^25, so s/n is at least 1/n away from the
            // next integer, far more than the rounding error.
            const double dn = (double)n;
            uint8_t* o = j.dst + (size_t)y * (size_t)j.dst_stride + 3 * x;
            o[0] = (uint8_t)(uint32_t)((double)(uint32_t)(a >> 32) / dn);
            o[1] = (uint8_t)(uint32_t)((double)(uint32_t)b / dn);
            o[2] = (uint8_t)(uint32_t)((double)(uint32_t)(b >> 32) / dn);
        }
    }
}

__device__ __forceinline__ void run_tile(const Job& j, int tile, uint8_t* lds) {
    if (j.hist == OILPAINT_HIST_WIDE)
        tile_wide(j, tile, lds);
    else
        tile_packed(j, tile, lds);
}

// One workgroup per tile.
__global__ __launch_bounds__(1024) void k_plain(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    run_tile(j, blockIdx.x, lds);
}

// Persistent: workgroups pull tiles from a counter until the queue is empty.
__global__ __launch_bounds__(1024) void k_batch(BatchArgs a) {
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
        run_tile(a.jobs[lo], t - a.first_tile[lo], lds);
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

hipError_t launch_plain(const Job& j, int waves, size_t lds, hipStream_t stream) {
    static int lds_done = 0;
    const int tiles = j.tiles_x * j.tiles_y;
    if (tiles <= 0) return hipSuccess;
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(k_plain), lds, lds_done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_plain, dim3(tiles), dim3(64 * waves), lds, stream, j);
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
        per_cu < 1)
        per_cu = 1;
    const DeviceInfo d = device_info(device);
    return per_cu * (d.cus > 0 ? d.cus : 1);
}

}  // namespace oilpaint_impl
