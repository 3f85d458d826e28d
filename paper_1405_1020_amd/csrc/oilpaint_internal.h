// Internal declarations shared by the kernels and the host side of
// liboilpaint.so.  Nothing here is part of the public ABI (include/oilpaint.h).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "oilpaint.h"

namespace oilpaint_impl {

// Largest effective radius of the packed layout: a 31 x 31 window holds 961
// pixels, which fits the 10-bit count field, and 255 * 961 fits 18 bits.
constexpr int kPackedMaxRadius = 15;
// Largest effective radius of the wide layout: 255 * 4103^2 < 2^32.
constexpr int kWideMaxRadius = 2051;
// Largest effective radius of the column layout: a column of 2r+1 pixels
// keeps its count in 13 bits and its sums in 17, and a strip with its halo
// spans at most kColumnChunks wavefront widths.
constexpr int kColumnMaxRadius = 255;
constexpr int kColumnChunks = 9;
inline int column_chunks(int radius) { return (64 + 2 * radius + 63) / 64; }
// The column layout's form for radius <= 15 and at most 64 levels
// (tile_column15): column entries in the F18 bin word, level rows of
// kColumn15Stride columns, and per column its level counts three to a
// 32-bit word (column15_words(levels) words, bucketed: 3, 7, 11, 22).
constexpr int kColumn15Stride = 94;  // 64 + 2 * 15
constexpr int kColumn15Buckets = 4;
constexpr int kColumn15MaxLevels = 64;
inline int column15_bucket(int levels) { return levels <= 9 ? 0 : levels <= 21 ? 1 : levels <= 33 ? 2 : 3; }
inline int column15_words(int levels) {
    constexpr int kWords[kColumn15Buckets] = {3, 7, 11, 22};
    return kWords[column15_bucket(levels)];
}
// [column histograms: one row per level][count words][a key per
// wavefront][a partial word per wavefront but one][row buffer]: at r <= 15,
// 20 levels and four wavefronts 20,424 bytes, eight workgroups per CU
inline size_t column15_lds_bytes(int levels, int waves) {
    return (size_t)levels * kColumn15Stride * 8 + (size_t)column15_words(levels) * kColumn15Stride * 4 +
           (size_t)waves * 64 * 4 + (size_t)(waves - 1) * 64 * 8 + 192;
}
// Wavefronts per strip of the radius <= 15 form: 1, 2 or 4 (index 0, 1, 2).
inline int column15_wave_index(int waves) { return waves == 1 ? 0 : waves == 2 ? 1 : waves == 4 ? 2 : -1; }
// The same form for radius 16..31 (tile_column15's WIDE form, plain
// launches with two or four wavefronts per strip; one wavefront keeps the
// generic column form): level rows of kColumn31Stride columns, two 16-bit
// counts per word (column31_words(levels) words, bucketed: 4, 10, 16, 32).
constexpr int kColumn31Stride = 126;  // 64 + 2 * 31
constexpr int kColumn31MinRadius = 16;
constexpr int kColumn31MaxRadius = 31;
inline int column31_bucket(int levels) { return levels <= 8 ? 0 : levels <= 20 ? 1 : levels <= 32 ? 2 : 3; }
inline int column31_words(int levels) {
    constexpr int kWords[kColumn15Buckets] = {4, 10, 16, 32};
    return kWords[column31_bucket(levels)];
}
// [column histograms][count words][keys][partial word pairs][row buffer]
inline size_t column31_lds_bytes(int levels, int waves) {
    return (size_t)levels * kColumn31Stride * 8 + (size_t)column31_words(levels) * kColumn31Stride * 4 +
           (size_t)waves * 64 * 4 + (size_t)(waves - 1) * 64 * 16 + 192;
}
// Largest window pixel count the packed layout's division table covers.
constexpr int kPackedMaxCount = 961;

// One image, or a band of its output rows, as the kernels see it.  The
// launch shape (rows, lanes, hist) is resolved on the host.
struct Job {
    const uint8_t* src;
    uint8_t* dst;
    int32_t width, height;
    int32_t stride;     // src row stride, bytes
    int32_t dst_stride; // dst row stride, bytes
    int32_t radius;     // effective radius (clamped to max(width, height) - 1)
    int32_t levels;
    int32_t row_begin, row_end;
    int32_t paper;      // 1: literal listing semantics (OILPAINT_FLAG_PAPER)
    int32_t rows;       // output rows per lane
    int32_t lanes;      // active lanes per wavefront (output columns per tile)
    int32_t hist;       // OILPAINT_HIST_*
    int32_t tiles_x;    // tiles across the image
    int32_t tiles_y;    // tiles down the row band
    int32_t waves;      // wavefronts per tile that compute (<= the workgroup's)
    // histogram layout, decided on the host (set_layout)
    int32_t fast;       // 1: compile-time-radius path (PACKED, 64 lanes, scan <= 64)
    int32_t scan;       // bins the mode search scans (levels, or levels rounded up to 8)
    int32_t white;      // bin of the paper form's extra pure-white level
    int32_t trash;      // bin of pixels outside the image
    int32_t bins;       // bins per lane
    int32_t colfirst;   // streamed layout: first window built from column histograms
};

// Work-queue form of a batch: jobs[] in queue order, first_tile[i] the
// queue index of job i's first tile, first_tile[njobs] the total.
struct BatchArgs {
    const Job* jobs;
    const int32_t* first_tile;
    int32_t njobs;
    int32_t ntiles;
    uint32_t* counter;   // tile counter, reset to 0 before every launch
};

// On-chip bytes one workgroup needs for job `j` (its `waves` computing
// wavefronts).
size_t lds_bytes(const Job& j);

// Fill the histogram-layout fields of `j` from its shape (hist, lanes,
// radius, levels, paper): the levels 0..L-1 first -- rounded up to a multiple
// of 8 empty bins on the fast path -- then the paper form's white level,
// then the bin for pixels outside the image.
__host__ __device__ inline bool is_stream(int hist) { return hist == OILPAINT_HIST_STREAM || hist == OILPAINT_HIST_STREAM8; }

// Streamed layout worked by several wavefronts per strip (OILPAINT_HIST_STREAM
// or OILPAINT_HIST_STREAM8 with waves == kSplitWaves): the wavefronts share
// one histogram and one ring, each making a quarter of every row step's
// updates and scanning a block of split_bins(L) bins; the scanned levels are
// padded to kSplitWaves blocks with bins no pixel reaches.  Rows per tile are
// the run of every wavefront (not multiplied by the wavefront count).
constexpr int kSplitWaves = 4;
__host__ __device__ inline bool is_split(const Job& j) { return is_stream(j.hist) && j.waves == kSplitWaves; }
// Whether a column-layout job takes the radius <= 15 form.
inline bool column15(const Job& j) {
    return j.radius >= 0 && j.radius <= kPackedMaxRadius && j.levels >= 1 && j.levels <= kColumn15MaxLevels;
}
// Whether a column-layout job takes the radius 16..31 form.
inline bool column31(const Job& j) {
    return j.radius >= kColumn31MinRadius && j.radius <= kColumn31MaxRadius && j.levels >= 1 &&
           j.levels <= kColumn15MaxLevels && (j.waves == 2 || j.waves == 4);
}
inline int split_bins(int levels) {
    return levels <= 8 ? 2 : levels <= 16 ? 4 : levels <= 20 ? 5 : levels <= 32 ? 8 : 16;
}
inline int split_bucket(int bins) {
    return bins == 2 ? 0 : bins == 4 ? 1 : bins == 5 ? 2 : bins == 8 ? 3 : bins == 16 ? 4 : -1;
}
// LDS of the per-wavefront mode-search results: a 4-byte key per lane and
// wavefront, and the winning 8-byte bin word per lane and wavefront.
constexpr size_t kSplitPartBytes = (size_t)kSplitWaves * 64 * 12;
// With 8-byte entries the four-wavefront form keeps no ring of window rows:
// row slots for two row steps' entering and leaving rows, double-buffered
// (the first window always comes from column histograms).
constexpr int kSplitRows8 = 8;

// Streamed layout: bytes of the ring of (2r+4) rows of 64+2r entries (8 bytes
// each for OILPAINT_HIST_STREAM8, else 4), and of the column histograms a
// run's first window may be built from (scan + 1 rows of 64+2r 8-byte
// entries), which take the ring's place while they live.
__host__ __device__ inline size_t stream_ring_only_bytes(const Job& j) {
    if (is_split(j) && j.hist == OILPAINT_HIST_STREAM8)  // kSplitRows8 rows, 8-byte entries
        return (size_t)kSplitRows8 * (64 + 2 * (size_t)j.radius) * 8;
    return (2 * (size_t)j.radius + 4) * (64 + 2 * (size_t)j.radius) * (j.hist == OILPAINT_HIST_STREAM8 ? 8 : 4);
}
__host__ __device__ inline size_t stream_colh_bytes(const Job& j) {
    return (size_t)(j.scan + 1) * (64 + 2 * (size_t)j.radius) * 8;
}

//
// The streamed layout builds a run's first window either directly --
// (2r+1)^2 bin updates per lane -- or from column histograms: per column of
// the strip a histogram of its 2r+1 window rows (the (64+2r)(2r+1) pixels
// spread over the 64 lanes), then per level the sum of 2r+1 neighbouring
// columns.  The second costs ~(2r+1) reads per scanned level instead of
// ~(2r+1) updates per window row.  It is used when the window is wide for
// the level count, and only when the column histograms fit in the ring's
// place or the runs are short enough (at most 4(2r+1) rows) for the first
// window to matter more than the larger on-chip footprint.
inline void set_layout(Job& j) {
    if (j.hist == OILPAINT_HIST_REGS) {
        // registers hold bins 0 .. scan-1 (levels rounded up to 8 or 16); the
        // paper form's white level and outside pixels match no register
        j.fast = 0;
        j.scan = j.levels <= 8 ? 8 : 16;
        j.white = j.scan;
        j.trash = j.scan + (j.paper ? 1 : 0);
        j.bins = j.trash + 1;
        j.colfirst = 0;
        return;
    }
    if (j.hist == OILPAINT_HIST_COLUMN) {
        // levels 0 .. L-1, then one sink row for outside pixels and the
        // paper form's white level
        j.fast = 0;
        j.scan = j.levels;
        j.white = j.trash = j.levels;
        j.bins = j.levels + 1;
        j.colfirst = 0;
        return;
    }
    j.fast = ((j.hist == OILPAINT_HIST_PACKED || is_stream(j.hist)) && j.lanes == 64 &&
              j.radius <= kPackedMaxRadius && j.levels <= 64) ? 1 : 0;
    j.scan = j.fast ? (j.levels + 7) / 8 * 8 : j.levels;
    if (is_split(j) && j.levels <= 64) j.scan = kSplitWaves * split_bins(j.levels);
    j.white = j.scan;
    j.trash = j.scan + (j.paper ? 1 : 0);
    j.bins = j.trash + 1;
    j.colfirst = 0;
    if (is_stream(j.hist) && (2 * j.radius + 1) * 10 >= 4 * j.scan + 20)
        j.colfirst = (stream_colh_bytes(j) <= stream_ring_only_bytes(j) || j.rows <= 4 * (2 * j.radius + 1)) ? 1 : 0;
    if (is_split(j) && j.hist == OILPAINT_HIST_STREAM8) j.colfirst = 1;  // no ring of window rows
}

// Streamed layout: bytes of the ring region (the ring, or while they live
// the first window's column histograms).
__host__ __device__ inline size_t stream_ring_bytes(const Job& j) {
    const size_t ring = stream_ring_only_bytes(j);
    const size_t cols = j.colfirst ? stream_colh_bytes(j) : 0;
    const size_t b = ring > cols ? ring : cols;
    return (b + 15) & ~(size_t)15;
}

// Per-radius kernels (oilpaint_k_fast_*.hip, oilpaint_k_stream_*.hip):
// [radius - 0 or 8][scan bucket].
typedef void (*PlainKernel)(Job);
extern const PlainKernel kFast_lo[8][3];
extern const PlainKernel kFast_hi[8][3];
extern const PlainKernel kStream_lo[8][2];
extern const PlainKernel kStream_hi[8][2];
// Streamed kernels with 8-byte ring entries (OILPAINT_HIST_STREAM8),
// [radius - 8], levels <= 32.
extern const PlainKernel kStream8[8];
// The streamed kernels worked by kSplitWaves wavefronts per strip
// (oilpaint_k_split*.hip): [radius - 8 or 0][split_bucket(bins per
// wavefront)], 8-byte entries up to 8 bins per wavefront, 4-byte up to 16.
extern const PlainKernel kStream8Split[8][4];
extern const PlainKernel kStreamSplit_lo[8][5];
extern const PlainKernel kStreamSplit_hi[8][5];
// Register-histogram kernels (oilpaint_k_regs.hip): [radius][levels <= 8 ? 0 : 1].
extern const PlainKernel kRegs[8][2];
constexpr int kRegsMaxRadius = 7;
constexpr int kRegsMaxLevels = 16;

// Persistent batch kernels of the streamed layout (oilpaint_k_batch_*.hip),
// indexed like kStream_*.
typedef void (*BatchKernel)(BatchArgs);
extern const BatchKernel kBatchStream_lo[8][2];
extern const BatchKernel kBatchStream_hi[8][2];
extern const BatchKernel kBatchStream8[8];
// Persistent batch forms of the four-wavefront streamed kernels
// (oilpaint_k_split*.hip): [radius - 0 or 8][level bucket: up to 32, up to
// 64 levels], and [radius - 8] for 8-byte entries.
extern const BatchKernel kBatchSplit_lo[8][2];
extern const BatchKernel kBatchSplit_hi[8][2];
extern const BatchKernel kBatchSplit8[8];
// Column-layout kernels (oilpaint_k_column.hip), [chunks - 1].
extern const PlainKernel kColumn[kColumnChunks];
extern const BatchKernel kBatchColumn[kColumnChunks];
// Its radius <= 15 form, [column15_wave_index(waves)][column15_bucket(levels)];
// batch forms with one and with four wavefronts per strip.
extern const PlainKernel kColumn15[3][kColumn15Buckets];
// Its radius 16..31 form, [waves == 4][column31_bucket(levels)].
extern const PlainKernel kColumn31[2][kColumn15Buckets];
extern const BatchKernel kBatchColumn15[kColumn15Buckets];
extern const BatchKernel kBatchColumn15x4[kColumn15Buckets];

// Kernel class of a batch job: 2 * radius + scan bucket (0: scan <= 32,
// 1: scan <= 64) for the streamed layout, 32 + radius - 8 for its 8-byte
// form, 40 + chunks - 1 for the column layout (radius above 15 or more than
// 64 levels), 49 + column15_bucket(levels) for its radius <= 15 form and
// 53 + the same for that form with four wavefronts per strip, then the same
// for the
// four-wavefront streamed layouts (from kSplitClass: 2 * radius + bucket,
// then 32 + radius - 8), and kGenericClass for every other job (generic
// tile-staged and wide layouts, one kernel for all).  A batch launches one
// persistent kernel per class present, of batch_waves(class) wavefronts per
// workgroup.
constexpr int kStream8Class = 2 * (kPackedMaxRadius + 1);
constexpr int kColumnClass = kStream8Class + 8;
constexpr int kColumn15Class = kColumnClass + kColumnChunks;
constexpr int kColumn15x4Class = kColumn15Class + kColumn15Buckets;
constexpr int kSplitClass = kColumn15x4Class + kColumn15Buckets;
constexpr int kGenericClass = kSplitClass + kStream8Class + 8;
constexpr int kBatchClasses = kGenericClass + 1;
inline int batch_class(const Job& j) {
    const int split = is_split(j) ? kSplitClass : 0;
    if (j.hist == OILPAINT_HIST_STREAM && j.radius >= 0 && j.radius <= kPackedMaxRadius && j.scan <= 64)
        return split + 2 * j.radius + (j.scan <= 32 ? 0 : 1);
    if (j.hist == OILPAINT_HIST_STREAM8 && j.radius >= 8 && j.radius <= kPackedMaxRadius && j.scan <= 32)
        return split + kStream8Class + j.radius - 8;
    if (j.hist == OILPAINT_HIST_COLUMN && column15(j))
        return (j.waves == 4 ? kColumn15x4Class : kColumn15Class) + column15_bucket(j.levels);
    if (j.hist == OILPAINT_HIST_COLUMN && j.radius >= 0 && j.radius <= kColumnMaxRadius)
        return kColumnClass + column_chunks(j.radius) - 1;
    return kGenericClass;
}
inline int batch_waves(int cls) {
    if (cls >= kColumn15x4Class && cls < kColumn15x4Class + kColumn15Buckets) return 4;
    return cls >= kSplitClass && cls < kGenericClass ? kSplitWaves : 1;
}
// Output rows of one tile: a run per wavefront, except in the streamed and
// column layouts, whose wavefronts share one run.
inline int runs_per_tile(int hist, int waves) { return is_stream(hist) || hist == OILPAINT_HIST_COLUMN ? 1 : waves; }

// Windowed median of one channel (oilpaint_k_median.hip): one image, one
// wavefront per workgroup of 64 output columns by `rows` output rows.
constexpr int kMedianMaxRadius = 15;
struct MedianJob {
    const uint8_t* src;
    uint8_t* dst;
    int32_t width, height;
    int32_t src_stride, dst_stride;  // bytes
    int32_t channels, channel;       // interleaved channels of src, the one filtered
    int32_t radius;                  // effective radius
    int32_t rows, tiles_x, tiles_y;
};
typedef void (*MedianKernel)(MedianJob);
extern const MedianKernel kMedian[kMedianMaxRadius + 1];
// The same worked by four wavefronts per strip (256-thread workgroups).
extern const MedianKernel kMedian4[kMedianMaxRadius + 1];
// Whether a radius uses the four-wavefront form: measured per radius on
// 1920x1080 (one channel), where it was the faster of the two.
inline bool median_split(int radius) {
    constexpr bool kSplit[kMedianMaxRadius + 1] = {false, false, true, true, true, false, true, false,
                                                   true,  true,  true, true, true, true,  true, true};
    return radius >= 0 && radius <= kMedianMaxRadius && kSplit[radius];
}
size_t median_lds_bytes(int radius);
// The column-histogram form (oilpaint_k_median_column.hip): any radius up to
// 127, by 64-column chunks of the strip with its halo, minus one.
constexpr int kMedianColumnMaxRadius = 127;
constexpr int kMedianColumnChunks = 5;
extern const MedianKernel kMedianColumn[kMedianColumnChunks];
size_t median_column_lds_bytes(int radius);

// Kernel launches (oilpaint_kernels.hip).  Each returns a hipError_t.
hipError_t launch_plain(const Job& j, int waves, size_t lds, hipStream_t stream);
hipError_t launch_batch(const BatchArgs& a, int cls, int waves, size_t lds, int grid, hipStream_t stream);
// Clear n counters, stride_words apart (a kernel, so that a captured graph
// holds no memset node).
hipError_t launch_reset_counters(uint32_t* counters, int n, int stride_words, hipStream_t stream);
// Photo-like test image (3-byte pixels, `width` per row) for the tuner.
hipError_t launch_fill(uint8_t* p, size_t n, int width, hipStream_t stream);

// Record a failed HIP call (text readable through oilpaint_last_error) and
// clear the runtime's sticky last-error state.  Returns `e`.
hipError_t note_hip(const char* where, hipError_t e);
// Record an error text (readable through oilpaint_last_error).
void note_error(const char* text);

// Device facts, cached per device.
struct DeviceInfo {
    int cus;
    size_t lds_per_block;
    int ok;
};
DeviceInfo device_info(int device);

// Most workgroups of class `cls`'s persistent kernel that can be resident at
// once.
int batch_grid(int device, int cls, int waves, size_t lds);

}  // namespace oilpaint_impl
