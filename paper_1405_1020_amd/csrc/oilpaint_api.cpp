// Host side of liboilpaint.so: argument validation, launch-shape choice and
// the single-image entry points of include/oilpaint.h.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>

#include "oilpaint_internal.h"

namespace oilpaint_impl {

namespace {
thread_local char g_last_error[256] = "";
}

void note_error(const char* text) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", text); }

hipError_t note_hip(const char* where, hipError_t e) {
    if (e != hipSuccess) {
        std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
        (void)hipGetLastError();
    }
    return e;
}

// ---------------------------------------------------------------------------
// Device facts
// ---------------------------------------------------------------------------
DeviceInfo device_info(int device) {
    static std::mutex mu;
    static std::map<int, DeviceInfo> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(device);
    if (it != cache.end()) return it->second;
    DeviceInfo d{0, 0, 0};
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) == hipSuccess) {
        d.cus = p.multiProcessorCount;
        d.lds_per_block = p.sharedMemPerBlock;
        d.ok = 1;
    }
    cache[device] = d;
    return d;
}

size_t lds_bytes(const Job& j) {
    const int waves = j.waves;
    const size_t nb = (size_t)j.bins;
    const size_t lanes = (size_t)j.lanes;
    if (j.hist == OILPAINT_HIST_WIDE) return (size_t)waves * 2 * nb * lanes * 8;
    if (j.hist == OILPAINT_HIST_REGS) return stream_ring_bytes(j) + 192;
    if (is_stream(j.hist)) {
        // radius 1 with one wavefront and more than 8 scanned levels keeps its
        // window in registers (no histogram: tile_direct1)
        if (j.hist == OILPAINT_HIST_STREAM && j.waves == 1 && j.radius == 1 && j.scan > 8)
            return stream_ring_bytes(j) + 192;
        return nb * 64 * 8 + stream_ring_bytes(j) + 192 + (is_split(j) ? kSplitPartBytes : 0);
    }
    if (j.hist == OILPAINT_HIST_COLUMN) {
        if (column15(j)) return column15_lds_bytes(j.levels, j.waves);
        if (column31(j)) return column31_lds_bytes(j.levels, j.waves);
        const size_t tw = 64 + 2 * (size_t)j.radius;
        return ((nb * tw * 8 + 15) & ~(size_t)15) + (tw + 1) * 16 + 192;
    }
    const size_t tw = lanes + 2 * (size_t)j.radius;
    const size_t th = (size_t)waves * (size_t)j.rows + 2 * (size_t)j.radius;
    const size_t tile = (tw * th * 4 + 15) & ~(size_t)15;
    return tile + (size_t)waves * nb * lanes * 8;
}

namespace {

// Static LDS the kernels declare besides the dynamic block, with slack.
constexpr size_t kStaticLds = 256;

int effective_radius(int width, int height, int radius) {
    const int span = std::max(width, height) - 1;
    return std::min(radius, std::max(span, 0));
}

bool ranges_overlap(const uint8_t* a, size_t alen, const uint8_t* b, size_t blen) {
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + blen && pb < pa + alen;
}

std::mutex g_tune_mu;
std::map<std::pair<int, int>, oilpaint_variant> g_tuned;

bool packed_ok(int reff, int levels, bool paper) {
    return reff <= kPackedMaxRadius && levels + (paper ? 1 : 0) <= 255;
}

}  // namespace

// The checks of oilpaint_validate with separate src and dst strides.
int validate2(const uint8_t* src, int sstride, const uint8_t* dst, int dstride, int width, int height, int radius,
              int levels) {
    if (!src || !dst) return OILPAINT_ERR_NULL;
    if (width < 0 || height < 0 || radius < 0 || radius > 65535) return OILPAINT_ERR_ARG;
    if (levels < 1 || levels > 256) return OILPAINT_ERR_ARG;
    if (width > INT_MAX / 3) return OILPAINT_ERR_ARG;
    if (sstride < 3 * width || dstride < 3 * width) return OILPAINT_ERR_ARG;
    if (width == 0 || height == 0) return OILPAINT_OK;
    const size_t sspan = (size_t)(height - 1) * (size_t)sstride + 3 * (size_t)width;
    const size_t dspan = (size_t)(height - 1) * (size_t)dstride + 3 * (size_t)width;
    if ((uintptr_t)src + sspan < (uintptr_t)src || (uintptr_t)dst + dspan < (uintptr_t)dst) return OILPAINT_ERR_ARG;
    if (ranges_overlap(src, sspan, dst, dspan)) return OILPAINT_ERR_OVERLAP;
    return OILPAINT_OK;
}

// Rows per lane for a variant whose rows are 0: about per_cu workgroups per
// CU over the job's row band (long runs amortise the (2r+1)^2 first window,
// short runs give more workgroups), 2 .. 1024.  Small images get short runs:
// a GPU left half idle costs more than the extra first windows (640x480,
// r = 5, L = 20: 12.1 us at 8 rows, 10.6 at 4).
int auto_rows(const Job& j, const oilpaint_variant& v, int device) {
    const DeviceInfo d = device_info(device);
    const long cus = d.ok ? d.cus : 256;
    const long strips = (j.width + v.lanes - 1) / v.lanes;
    const long band = j.row_end - j.row_begin;
    const long want = (long)std::max(v.per_cu, 1) * cus;
    const long runs = runs_per_tile(v.hist, v.waves);
    long rows = (strips * band + want * runs - 1) / (want * runs);
    return (int)std::max(2L, std::min(rows, 1024L));
}

// Fill the launch-shape fields of `j` from `v`.  With v.rows == 0 the rows
// are derived from v.per_cu and halved while the on-chip footprint does not
// fit.  Returns OK or UNSUPPORTED.
int apply_variant(Job& j, const oilpaint_variant& v, int device) {
    if (v.rows < 0 || v.rows > 4096 || v.waves < 1 || v.waves > 8) return OILPAINT_ERR_UNSUPPORTED;
    if (v.rows == 0 && (v.per_cu < 1 || v.per_cu > 64)) return OILPAINT_ERR_UNSUPPORTED;
    if (v.lanes != 64 && v.lanes != 32 && v.lanes != 16) return OILPAINT_ERR_UNSUPPORTED;
    if (v.hist == OILPAINT_HIST_PACKED) {
        if (!packed_ok(j.radius, j.levels, j.paper != 0)) return OILPAINT_ERR_UNSUPPORTED;
    } else if (v.hist == OILPAINT_HIST_STREAM) {
        if (j.radius > kPackedMaxRadius || j.levels > 64 || v.lanes != 64 || (v.waves != 1 && v.waves != kSplitWaves))
            return OILPAINT_ERR_UNSUPPORTED;
    } else if (v.hist == OILPAINT_HIST_STREAM8) {
        if (j.radius < 8 || j.radius > kPackedMaxRadius || j.levels > 32 || v.lanes != 64 ||
            (v.waves != 1 && v.waves != kSplitWaves))
            return OILPAINT_ERR_UNSUPPORTED;
    } else if (v.hist == OILPAINT_HIST_COLUMN) {
        // several wavefronts per strip in the radius <= 15 form only
        Job jw = j;
        jw.waves = v.waves;
        const bool ok_waves = v.waves == 1 || (column15(j) && column15_wave_index(v.waves) >= 0) || column31(jw);
        if (j.radius > kColumnMaxRadius || !ok_waves || v.lanes != 64) return OILPAINT_ERR_UNSUPPORTED;
    } else if (v.hist == OILPAINT_HIST_WIDE) {
        if (j.radius > kWideMaxRadius) return OILPAINT_ERR_UNSUPPORTED;
    } else if (v.hist == OILPAINT_HIST_REGS) {
        if (j.radius > kRegsMaxRadius || j.levels > kRegsMaxLevels || v.lanes != 64 || v.waves != 1)
            return OILPAINT_ERR_UNSUPPORTED;
    } else {
        return OILPAINT_ERR_UNSUPPORTED;
    }
    j.rows = v.rows ? v.rows : auto_rows(j, v, device);
    j.lanes = v.lanes;
    j.hist = v.hist;
    j.waves = v.waves;
    set_layout(j);
    const DeviceInfo d = device_info(device);
    const size_t limit = d.ok ? d.lds_per_block : 65536;
    // the column-histogram first window is an optimisation: dropped first
    // when the footprint does not fit
    if (j.colfirst && !(is_split(j) && j.hist == OILPAINT_HIST_STREAM8) && lds_bytes(j) + kStaticLds > limit)
        j.colfirst = 0;
    while (lds_bytes(j) + kStaticLds > limit) {
        if (v.rows != 0 || j.rows == 1 || (is_split(j) && j.hist == OILPAINT_HIST_STREAM8))
            return OILPAINT_ERR_UNSUPPORTED;
        j.rows = std::max(1, j.rows / 2);
        set_layout(j);
        j.colfirst = 0;
    }
    const int band = j.row_end - j.row_begin;
    j.tiles_x = (j.width + j.lanes - 1) / j.lanes;
    const long per_tile = (long)runs_per_tile(v.hist, v.waves) * j.rows;
    j.tiles_y = (int)((band + per_tile - 1) / per_tile);
    return OILPAINT_OK;
}

// The built-in launch shape (before any tuning result): streamed rows when
// the window and level count allow it -- four wavefronts per strip, about
// four workgroups per CU, for radius 7 and up or more than 32 levels, else
// one wavefront, about eight per CU; for radii 16..255 column histograms,
// about two workgroups per CU, when they fit on chip; otherwise tiles of
// four wavefronts, about two per CU, or the wide layout; shrunk until the
// on-chip footprint fits.
oilpaint_variant default_variant(int width, int height, int reff, int levels, bool paper, int device) {
    oilpaint_variant v;
    v.rows = 0;
    v.lanes = 64;
    if (reff <= kPackedMaxRadius && levels <= 64) {
        const bool split = reff >= 7 || levels > 32;
        v.waves = split ? kSplitWaves : 1;
        v.hist = OILPAINT_HIST_STREAM;
        v.per_cu = split ? 4 : 8;
        return v;
    }
    if (reff > kPackedMaxRadius && reff <= kColumnMaxRadius) {
        // column histograms when they fit on chip
        v.waves = 1;
        v.hist = OILPAINT_HIST_COLUMN;
        v.per_cu = 2;
        Job t{};
        t.width = width;
        t.height = height;
        t.radius = reff;
        t.levels = levels;
        t.paper = paper ? 1 : 0;
        t.row_begin = 0;
        t.row_end = height;
        if (apply_variant(t, v, device) == OILPAINT_OK) return v;
    }
    v.waves = 4;
    v.per_cu = 2;
    v.hist = packed_ok(reff, levels, paper) ? OILPAINT_HIST_PACKED : OILPAINT_HIST_WIDE;
    if (v.hist == OILPAINT_HIST_WIDE) v.rows = 16;
    Job j{};
    j.width = width;
    j.height = height;
    j.radius = reff;
    j.levels = levels;
    j.paper = paper ? 1 : 0;
    j.row_begin = 0;
    j.row_end = height;
    for (;;) {
        Job t = j;
        if (apply_variant(t, v, device) == OILPAINT_OK) break;
        if (v.waves > 1)
            v.waves >>= 1;
        else if (v.lanes > 16)
            v.lanes >>= 1;
        else
            break;
    }
    return v;
}

oilpaint_variant choose_variant(int width, int height, int reff, int levels, bool paper, int device) {
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find({reff, levels});
        if (it != g_tuned.end() && !paper) return it->second;
    }
    return default_variant(width, height, reff, levels, paper, device);
}

// Validate a descriptor and build its Job (shape from `v`, or the library's
// choice when v is NULL).  Pure host work apart from device facts.
int make_job(const oilpaint_desc& d, const oilpaint_variant* v, int device, Job& j, bool& empty) {
    const int dst_stride = d.dst_stride ? d.dst_stride : d.stride;
    const int st = validate2(d.src, d.stride, d.dst, dst_stride, d.width, d.height, d.radius, d.levels);
    if (st != OILPAINT_OK) return st;
    if ((d.flags & ~OILPAINT_FLAG_PAPER) || d.reserved != 0) return OILPAINT_ERR_ARG;
    int rb = d.row_begin, re = d.row_end;
    if (rb == 0 && re == 0) re = d.height;
    if (rb < 0 || re < rb || re > d.height) return OILPAINT_ERR_ARG;
    empty = d.width == 0 || d.height == 0 || rb == re;
    std::memset(&j, 0, sizeof(j));
    j.src = d.src;
    j.dst = d.dst;
    j.width = d.width;
    j.height = d.height;
    j.stride = d.stride;
    j.dst_stride = dst_stride;
    j.radius = effective_radius(d.width, d.height, d.radius);
    j.levels = d.levels;
    j.row_begin = rb;
    j.row_end = re;
    j.paper = (d.flags & OILPAINT_FLAG_PAPER) ? 1 : 0;
    if (j.radius > kWideMaxRadius) return OILPAINT_ERR_UNSUPPORTED;
    // The listing's form writes only [r, W-r) x [r, H-r) with the radius as
    // given: nothing at all when 2r >= W or 2r >= H (clamping the radius
    // first would open an interior there).
    if (j.paper && (2 * (int64_t)d.radius >= d.width || 2 * (int64_t)d.radius >= d.height)) empty = true;
    if (empty) return OILPAINT_OK;
    const oilpaint_variant use =
        v ? *v : choose_variant(d.width, d.height, j.radius, d.levels, j.paper != 0, device);
    return apply_variant(j, use, device);
}

// Device-accessibility check of one pointer (ERR_NOT_DEVICE if host-only).
int check_device_ptr(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return OILPAINT_ERR_NOT_DEVICE;
    }
    if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) return OILPAINT_OK;
    if (a.type == hipMemoryTypeHost && a.devicePointer != nullptr) return OILPAINT_OK;  // mapped pinned
    return OILPAINT_ERR_NOT_DEVICE;
}

}  // namespace oilpaint_impl

using namespace oilpaint_impl;

extern "C" {

int oilpaint_version(void) { return OILPAINT_ABI_VERSION; }

const char* oilpaint_last_error(void) { return g_last_error; }

const char* oilpaint_strerror(int status) {
    switch (status) {
        case OILPAINT_OK: return "ok";
        case OILPAINT_ERR_NULL: return "null pointer";
        case OILPAINT_ERR_ARG: return "invalid argument (size, radius, levels, stride or row range)";
        case OILPAINT_ERR_OVERLAP: return "source and destination overlap";
        case OILPAINT_ERR_NOT_DEVICE: return "pointer is not device memory";
        case OILPAINT_ERR_HIP: return "HIP runtime error";
        case OILPAINT_ERR_NOMEM: return "out of memory";
        case OILPAINT_ERR_FULL: return "queue full";
        case OILPAINT_ERR_UNSUPPORTED: return "unsupported combination";
        default: return "unknown status";
    }
}

int oilpaint_validate(const uint8_t* src, const uint8_t* dst, int width, int height, int stride, int radius,
                      int levels) {
    return validate2(src, stride, dst, stride, width, height, radius, levels);
}

static int launch_desc(const oilpaint_desc& d, const oilpaint_variant* v, hipStream_t stream) {
    int device = 0;
    if (note_hip("hipGetDevice", hipGetDevice(&device)) != hipSuccess) return OILPAINT_ERR_HIP;
    Job j;
    bool empty = false;
    int st = make_job(d, v, device, j, empty);
    if (st != OILPAINT_OK || empty) return st;
    if ((st = check_device_ptr(d.src)) != OILPAINT_OK) return st;
    if ((st = check_device_ptr(d.dst)) != OILPAINT_OK) return st;
    const size_t lds = lds_bytes(j);
    if (launch_plain(j, j.waves, lds, stream) != hipSuccess) return OILPAINT_ERR_HIP;
    return OILPAINT_OK;
}

static int launch_one(const uint8_t* src, uint8_t* dst, int width, int height, int stride, int radius, int levels,
                      const oilpaint_variant* v, hipStream_t stream) {
    oilpaint_desc d{};
    d.src = src;
    d.dst = dst;
    d.width = width;
    d.height = height;
    d.stride = stride;
    d.radius = radius;
    d.levels = levels;
    return launch_desc(d, v, stream);
}

}  // extern "C"

namespace oilpaint_impl {
namespace {

std::mutex g_median_mu;
int g_median_kind[kMedianColumnMaxRadius + 1];  // installed kinds (0: the built-in choice)

// The built-in choice: radius <= 15 one or four wavefronts per strip (as
// measured per radius, median_split), above it the column form.
int median_default_kind(int reff) {
    if (reff <= kMedianMaxRadius) return median_split(reff) ? OILPAINT_MEDIAN_FOUR : OILPAINT_MEDIAN_ONE;
    return OILPAINT_MEDIAN_COLUMN;
}

bool median_kind_ok(int kind, int reff) {
    if (kind == OILPAINT_MEDIAN_ONE || kind == OILPAINT_MEDIAN_FOUR) return reff <= kMedianMaxRadius;
    if (kind == OILPAINT_MEDIAN_COLUMN) return reff <= kMedianColumnMaxRadius;
    return false;
}

int median_chosen_kind(int reff) {
    if (reff > kMedianColumnMaxRadius) return 0;
    std::lock_guard<std::mutex> lock(g_median_mu);
    const int k = g_median_kind[reff];
    return k ? k : median_default_kind(reff);
}

int median_launch(const uint8_t* src, int src_stride, int channels, int channel, uint8_t* dst, int dst_stride,
                  int width, int height, int radius, int kind, hipStream_t stream) {
    if (!src || !dst) return OILPAINT_ERR_NULL;
    if (width < 0 || height < 0 || radius < 0 || channels < 1 || channels > 4 || channel < 0 ||
        channel >= channels)
        return OILPAINT_ERR_ARG;
    if (kind < OILPAINT_MEDIAN_AUTO || kind > OILPAINT_MEDIAN_COLUMN) return OILPAINT_ERR_ARG;
    if ((int64_t)src_stride < (int64_t)channels * width || dst_stride < width) return OILPAINT_ERR_ARG;
    if (width == 0 || height == 0) return OILPAINT_OK;
    const size_t slen = (size_t)src_stride * (size_t)(height - 1) + (size_t)channels * (size_t)width;
    const size_t dlen = (size_t)dst_stride * (size_t)(height - 1) + (size_t)width;
    if (ranges_overlap(src, slen, dst, dlen)) return OILPAINT_ERR_OVERLAP;
    const int reff = effective_radius(width, height, radius);
    if (kind == OILPAINT_MEDIAN_AUTO) kind = median_chosen_kind(reff);
    if (kind == 0 || !median_kind_ok(kind, reff)) return OILPAINT_ERR_UNSUPPORTED;
    int st = check_device_ptr(src);
    if (st == OILPAINT_OK) st = check_device_ptr(dst);
    if (st != OILPAINT_OK) return st;
    int device = 0;
    if (note_hip("hipGetDevice", hipGetDevice(&device)) != hipSuccess) return OILPAINT_ERR_HIP;
    const DeviceInfo d = device_info(device);
    MedianJob j;
    j.src = src;
    j.dst = dst;
    j.width = width;
    j.height = height;
    j.src_stride = src_stride;
    j.dst_stride = dst_stride;
    j.channels = channels;
    j.channel = channel;
    j.radius = reff;
    // as many workgroups per CU as are resident at once (the kernel's
    // occupancy at this LDS size, at most 8), so that the whole grid runs in
    // one wave and runs are as long as that allows: 8 .. 1024 rows (the
    // column form's run start, 2r+1 rows of two atomics per column, costs
    // less than one of its output rows)
    MedianKernel kern;
    int threads = 64;
    size_t lds;
    if (kind == OILPAINT_MEDIAN_COLUMN) {
        const int nt = (64 + 2 * reff + 63) / 64;
        kern = kMedianColumn[nt - 1];
        lds = median_column_lds_bytes(reff);
        static int done[kMedianColumnChunks];
        if (lds > 65536 && !__atomic_load_n(&done[nt - 1], __ATOMIC_ACQUIRE)) {
            hipFuncAttributes fa;
            if (note_hip("hipFuncGetAttributes", hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern))) !=
                hipSuccess)
                return OILPAINT_ERR_HIP;
            const size_t total = d.ok ? d.lds_per_block : 65536;
            if (lds + fa.sharedSizeBytes > total) return OILPAINT_ERR_UNSUPPORTED;
            if (note_hip("hipFuncSetAttribute",
                         hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(total - fa.sharedSizeBytes))) != hipSuccess)
                return OILPAINT_ERR_HIP;
            __atomic_store_n(&done[nt - 1], 1, __ATOMIC_RELEASE);
        }
    } else {
        const bool split = kind == OILPAINT_MEDIAN_FOUR;
        kern = split ? kMedian4[reff] : kMedian[reff];
        threads = split ? 256 : 64;
        lds = median_lds_bytes(reff);
    }
    const long strips = (width + 63) / 64;
    int fit = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, reinterpret_cast<const void*>(kern), threads, lds) !=
            hipSuccess ||
        fit < 1) {
        (void)hipGetLastError();
        fit = (int)std::max<size_t>(1, (d.ok ? d.lds_per_block : 65536) / lds);
    }
    const long want = std::max(1L, std::min((long)fit, 8L)) * (d.ok ? d.cus : 256);
    j.rows = (int)std::max(8L, std::min((strips * height + want - 1) / want, 1024L));
    j.tiles_x = (int)strips;
    j.tiles_y = (height + j.rows - 1) / j.rows;
    hipLaunchKernelGGL(kern, dim3(j.tiles_x * j.tiles_y), dim3(threads), lds, stream, j);
    return note_hip("median launch", hipGetLastError()) == hipSuccess ? OILPAINT_OK : OILPAINT_ERR_HIP;
}

}  // namespace
}  // namespace oilpaint_impl

extern "C" {

int oilpaint_median_async(const uint8_t* src, int src_stride, int channels, int channel, uint8_t* dst,
                          int dst_stride, int width, int height, int radius, void* stream) {
    return median_launch(src, src_stride, channels, channel, dst, dst_stride, width, height, radius,
                         OILPAINT_MEDIAN_AUTO, (hipStream_t)stream);
}

int oilpaint_median_async_kind(const uint8_t* src, int src_stride, int channels, int channel, uint8_t* dst,
                               int dst_stride, int width, int height, int radius, int kind, void* stream) {
    return median_launch(src, src_stride, channels, channel, dst, dst_stride, width, height, radius, kind,
                         (hipStream_t)stream);
}

int oilpaint_median_set_kind(int radius, int kind) {
    if (radius < 0 || radius > kMedianColumnMaxRadius || kind < OILPAINT_MEDIAN_AUTO || kind > OILPAINT_MEDIAN_COLUMN)
        return OILPAINT_ERR_ARG;
    if (kind != OILPAINT_MEDIAN_AUTO && !median_kind_ok(kind, radius)) return OILPAINT_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_median_mu);
    g_median_kind[radius] = kind;
    return OILPAINT_OK;
}

int oilpaint_median_pick_kind(int radius) {
    if (radius < 0) return OILPAINT_ERR_ARG;
    const int k = median_chosen_kind(radius);
    return k ? k : OILPAINT_ERR_UNSUPPORTED;
}

int oilpaint_median(const uint8_t* src, int src_stride, int channels, int channel, uint8_t* dst, int dst_stride,
                    int width, int height, int radius) {
    const int st = oilpaint_median_async(src, src_stride, channels, channel, dst, dst_stride, width, height,
                                         radius, nullptr);
    if (st != OILPAINT_OK) return st;
    return note_hip("hipStreamSynchronize", hipStreamSynchronize(nullptr)) == hipSuccess ? OILPAINT_OK
                                                                                          : OILPAINT_ERR_HIP;
}

int oilpaint_run(const oilpaint_desc* desc, void* stream) {
    if (!desc) return OILPAINT_ERR_NULL;
    return launch_desc(*desc, nullptr, (hipStream_t)stream);
}

int oilpaint_async(const uint8_t* src, uint8_t* dst, int width, int height, int stride, int radius, int levels,
                   void* stream) {
    return launch_one(src, dst, width, height, stride, radius, levels, nullptr, (hipStream_t)stream);
}

int oilpaint_async_variant(const uint8_t* src, uint8_t* dst, int width, int height, int stride, int radius,
                           int levels, const oilpaint_variant* v, void* stream) {
    if (!v) return OILPAINT_ERR_NULL;
    return launch_one(src, dst, width, height, stride, radius, levels, v, (hipStream_t)stream);
}

int oilpaint(const uint8_t* src, uint8_t* dst, int width, int height, int stride, int radius, int levels) {
    const int st = launch_one(src, dst, width, height, stride, radius, levels, nullptr, nullptr);
    if (st != OILPAINT_OK) return st;
    if (note_hip("hipStreamSynchronize", hipStreamSynchronize(nullptr)) != hipSuccess) return OILPAINT_ERR_HIP;
    return OILPAINT_OK;
}

int oilpaint_tune(int width, int height, int radius, int levels, const oilpaint_variant* cands, int n, int reps,
                  void* stream_, float* ms_out) {
    if (!cands || !ms_out) return OILPAINT_ERR_NULL;
    if (width < 1 || height < 1 || width > (1 << 16) || height > (1 << 16) || radius < 0 || radius > 65535 ||
        levels < 1 || levels > 256 || n < 1 || reps < 1)
        return OILPAINT_ERR_ARG;
    hipStream_t stream = (hipStream_t)stream_;
    const size_t bytes = (size_t)width * (size_t)height * 3;
    uint8_t* src = nullptr;
    uint8_t* dst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = OILPAINT_OK;
    if (hipMalloc(&src, bytes) != hipSuccess || hipMalloc(&dst, bytes) != hipSuccess) {
        (void)hipGetLastError();
        st = OILPAINT_ERR_NOMEM;
    }
    if (st == OILPAINT_OK && (note_hip("hipEventCreate", hipEventCreate(&e0)) != hipSuccess ||
                              note_hip("hipEventCreate", hipEventCreate(&e1)) != hipSuccess))
        st = OILPAINT_ERR_HIP;
    if (st == OILPAINT_OK && launch_fill(src, bytes, width, stream) != hipSuccess) st = OILPAINT_ERR_HIP;
    for (int i = 0; st == OILPAINT_OK && i < n; ++i) {
        ms_out[i] = -1.0f;
        const int s0 = oilpaint_async_variant(src, dst, width, height, 3 * width, radius, levels, &cands[i], stream);
        if (s0 == OILPAINT_ERR_UNSUPPORTED) continue;
        if (s0 != OILPAINT_OK) {
            st = s0;
            break;
        }
        if (note_hip("hipEventRecord", hipEventRecord(e0, stream)) != hipSuccess) {
            st = OILPAINT_ERR_HIP;
            break;
        }
        for (int r = 0; r < reps && st == OILPAINT_OK; ++r)
            st = oilpaint_async_variant(src, dst, width, height, 3 * width, radius, levels, &cands[i], stream);
        if (st != OILPAINT_OK) break;
        float ms = 0.0f;
        if (note_hip("hipEventRecord", hipEventRecord(e1, stream)) != hipSuccess ||
            note_hip("hipEventSynchronize", hipEventSynchronize(e1)) != hipSuccess ||
            note_hip("hipEventElapsedTime", hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
            st = OILPAINT_ERR_HIP;
            break;
        }
        ms_out[i] = ms / (float)reps;
    }
    if (stream) (void)hipStreamSynchronize(stream);
    else (void)hipDeviceSynchronize();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    return st;
}

int oilpaint_pick_variant(int width, int height, int radius, int levels, oilpaint_variant* out) {
    if (!out) return OILPAINT_ERR_NULL;
    if (width < 0 || height < 0 || radius < 0 || radius > 65535 || levels < 1 || levels > 256)
        return OILPAINT_ERR_ARG;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) device = 0;
    const int reff = effective_radius(width, height, radius);
    oilpaint_variant v = choose_variant(width, height, reff, levels, false, device);
    if (width > 0 && height > 0) {
        // report the rows this image would get
        Job j{};
        j.width = width;
        j.height = height;
        j.radius = reff;
        j.levels = levels;
        j.row_begin = 0;
        j.row_end = height;
        if (apply_variant(j, v, device) == OILPAINT_OK) v.rows = j.rows;
    }
    *out = v;
    return OILPAINT_OK;
}

int oilpaint_set_variant(int radius, int levels, const oilpaint_variant* v) {
    if (!v) return OILPAINT_ERR_NULL;
    if (radius < 0 || radius > 65535 || levels < 1 || levels > 256) return OILPAINT_ERR_ARG;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) device = 0;
    Job j{};
    j.width = 1 << 20;
    j.height = 1 << 20;
    j.radius = radius;
    j.levels = levels;
    j.row_begin = 0;
    j.row_end = 1;
    const int st = apply_variant(j, *v, device);
    if (st != OILPAINT_OK) return st;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[{radius, levels}] = *v;
    return OILPAINT_OK;
}

int oilpaint_clear_variants(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned.clear();
    return OILPAINT_OK;
}

}  // extern "C"
