// Register-resident histograms (OILPAINT_HIST_REGS): the per-level count and
// channel sums of Section 4's listing kept by each lane in its own registers,
// one packed 64-bit word per level (the streamed layout's F16 bin word:
// radius <= 7), for at most 16 levels.  A register cannot be addressed by a
// data-dependent level, so a window update adds the pixel's increment to
// every bin under a per-bin mask of "level == bin" (four VALU instructions
// per bin): the LDS atomics of the streamed layout become VALU work, and the
// workgroup's LDS is the ring of staged rows only.  One wavefront per strip
// of 64 output columns, a run of `rows` output rows, the rows sliding down
// as in the streamed layout (tile_stream).
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int LB>
struct RegHist {
    uint64_t h[LB];

    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int b = 0; b < LB; ++b) h[b] = 0;
    }
    // A staged word {c0, c1, c2, level}: levels >= LB (outside pixels, the
    // paper form's white level) match no bin.
    __device__ __forceinline__ void add(uint32_t e) {
        const uint32_t k = e >> 24;
        const uint64_t inc = BinFmt<true>::inc(e);
#pragma unroll
        for (int b = 0; b < LB; ++b) h[b] += k == (uint32_t)b ? inc : 0ull;
    }
    __device__ __forceinline__ void step(uint32_t out, uint32_t in) {
        const uint32_t ko = out >> 24, ki = in >> 24;
        const uint64_t io = BinFmt<true>::inc(out), ii = BinFmt<true>::inc(in);
#pragma unroll
        for (int b = 0; b < LB; ++b) h[b] = h[b] + (ki == (uint32_t)b ? ii : 0ull) - (ko == (uint32_t)b ? io : 0ull);
    }
    // Most populated of the first `scan` bins, lowest level on ties: the
    // count and the winning bin word.
    __device__ __forceinline__ uint32_t mode(uint64_t& win) const {
        constexpr uint32_t M = BinFmt<true>::kCountMask;
        uint32_t best = 0;
        win = 0;
#pragma unroll
        for (int b = 0; b < LB; ++b) {
            const uint32_t key = ((uint32_t)(h[b] >> 32) & M) | (uint32_t)(63 - b);
            if (key > best) {
                best = key;
                win = h[b];
            }
        }
        return best >> BinFmt<true>::kCountShift;
    }
};

template <int R, int LB>
__device__ __forceinline__ void tile_regs(const Job& j, int unit, uint8_t* lds) {
    static_assert(R <= 7, "F16 bin words: windows up to 15 x 15");
    constexpr int SPAN = 2 * R + 1;
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

    RegHist<LB> hist;
    hist.clear();
#pragma unroll 1
    for (int dy = 0; dy < SPAN; ++dy) {
        const uint32_t* t = ring + dy * TW + lane;
        uint32_t w[SPAN];
#pragma unroll
        for (int i = 0; i < SPAN; ++i) w[i] = t[i];
#pragma unroll
        for (int i = 0; i < SPAN; ++i) hist.add(w[i]);
    }
    auto row_step = [&](int y) {
        uint64_t win;
        const uint32_t n = hist.mode(win);
        if (y + 1 < yb) {
            // step y -> y+1: row y-R leaves, row y+1+R enters
            const uint32_t* so = slot(y - R) + lane;
            const uint32_t* sn = slot(y + 1 + R) + lane;
            uint32_t wo[SPAN], wn[SPAN];
#pragma unroll
            for (int i = 0; i < SPAN; ++i) {
                wo[i] = so[i];
                wn[i] = sn[i];
            }
#pragma unroll
            for (int i = 0; i < SPAN; ++i) hist.step(wo[i], wn[i]);
        }
        store_row(j, x0, y, n, finalize_packed<true>(n, win), obuf);
    };
    // Two output rows per iteration; at the top rows y+2+R and y+3+R (fetched
    // an iteration earlier) enter the ring, into the slots of rows y-R-2 and
    // y-R-1, and the next two rows are fetched.
    int y = ya;
#pragma unroll 1
    for (; y < yb; y += 2) {
        if (y + 2 < yb) stream_write_row<R, false>(j, slot(y + 2 + R), q0);
        if (y + 3 < yb) stream_write_row<R, false>(j, slot(y + 3 + R), q1);
        lds_order();
        if (y + 4 < yb) stream_load_row<R>(j, x0, y + 4 + R, q0);
        if (y + 5 < yb) stream_load_row<R>(j, x0, y + 5 + R, q1);
        row_step(y);
        if (y + 1 < yb) row_step(y + 1);
    }
}

template <int R, int LB>
__global__ __launch_bounds__(64) void k_plain_regs(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_regs<R, LB>(j, xcd_tile(), lds);
}

}  // namespace

#define OILPAINT_REGS_ROW(R) {k_plain_regs<R, 8>, k_plain_regs<R, 16>}

// By [radius][levels <= 8 ? 0 : 1].
const PlainKernel kRegs[8][2] = {OILPAINT_REGS_ROW(0), OILPAINT_REGS_ROW(1), OILPAINT_REGS_ROW(2),
                                 OILPAINT_REGS_ROW(3), OILPAINT_REGS_ROW(4), OILPAINT_REGS_ROW(5),
                                 OILPAINT_REGS_ROW(6), OILPAINT_REGS_ROW(7)};

#undef OILPAINT_REGS_ROW

}  // namespace oilpaint_impl
