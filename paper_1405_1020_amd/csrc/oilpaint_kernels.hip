// Generic and persistent kernels of the oil-paint filter and their launch
// helpers; the per-radius kernels live in oilpaint_k_fast_*.hip and
// oilpaint_k_stream_*.hip.
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

// One workgroup per tile, generic layouts (at most 8 wavefronts, so that a
// lane may hold up to 256 registers).
__global__ __launch_bounds__(512) void k_plain(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    if (j.hist == OILPAINT_HIST_WIDE)
        tile_wide(j, xcd_tile(), lds);
    else
        tile_packed(j, xcd_tile(), lds);
}

// Persistent, the generic class of a batch (tile-staged and wide layouts):
// workgroups pull tiles from a counter until the queue is empty.  The
// streamed classes have kernels of their own (oilpaint_k_batch_*.hip).
__global__ __launch_bounds__(64) void k_batch(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ int32_t s_tile;
    for (;;) {
        __syncthreads();  // the previous tile's LDS reads are done
        if (threadIdx.x == 0) s_tile = (int32_t)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int32_t t = __builtin_amdgcn_readfirstlane(s_tile);
        if (t >= a.ntiles) break;
        const int i = job_of(a, t);
        const Job jb = a.jobs[i];
        if (jb.hist == OILPAINT_HIST_WIDE)
            tile_wide(jb, t - a.first_tile[i], lds);
        else
            tile_packed(jb, t - a.first_tile[i], lds);
    }
}

// A photo-like test image for timing launch shapes: per channel a smooth
// diagonal ramp with a slow ripple, plus small pseudo-random noise (a 32-bit
// integer hash of the byte index); `width` pixels of 3 bytes per row.
__global__ void k_fill(uint8_t* p, size_t n, int width) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 2654435761u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        const size_t px = i / 3;
        const uint32_t c = (uint32_t)(i - 3 * px);
        const uint32_t x = (uint32_t)(px % (size_t)width), y = (uint32_t)(px / (size_t)width);
        const uint32_t ramp = (x / 7 + y / 5 + 60 * c) + ((x / 97 + y / 61) & 3) * 23;
        p[i] = (uint8_t)((ramp & 255) ^ (h & 7));
    }
}

__global__ void k_reset(uint32_t* counters, int n, int stride_words) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[(size_t)i * stride_words] = 0u;
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
int g_fast_lds_done[kPackedMaxRadius + 1][3];
int g_stream_lds_done[kPackedMaxRadius + 1][2];
int g_stream8_lds_done[8];
int g_split_lds_done[8][4];
int g_split4_lds_done[kPackedMaxRadius + 1][5];
int g_column_lds_done[kColumnChunks];
int g_column15_lds_done[3][kColumn15Buckets];
int g_column31_lds_done[2][kColumn15Buckets];
int g_plain_lds_done;
int g_regs_lds_done;
int g_batch_lds_done[kBatchClasses];

BatchKernel batch_kernel(int cls) {
    if (cls < 0 || cls >= kGenericClass) return k_batch;
    if (cls >= kSplitClass) {
        const int c = cls - kSplitClass;
        if (c >= kStream8Class) return kBatchSplit8[c - kStream8Class];
        const int r = c >> 1, b = c & 1;
        return r <= 7 ? kBatchSplit_lo[r][b] : kBatchSplit_hi[r - 8][b];
    }
    if (cls >= kColumn15x4Class) return kBatchColumn15x4[cls - kColumn15x4Class];
    if (cls >= kColumn15Class) return kBatchColumn15[cls - kColumn15Class];
    if (cls >= kColumnClass) return kBatchColumn[cls - kColumnClass];
    if (cls >= kStream8Class) return kBatchStream8[cls - kStream8Class];
    const int r = cls >> 1, b = cls & 1;
    return r <= 7 ? kBatchStream_lo[r][b] : kBatchStream_hi[r - 8][b];
}
}  // namespace

hipError_t launch_plain(const Job& j, int waves, size_t lds, hipStream_t stream) {
    const int tiles = j.tiles_x * j.tiles_y;
    if (tiles <= 0) return hipSuccess;
    PlainKernel k = k_plain;
    int* done = &g_plain_lds_done;
    if (j.hist == OILPAINT_HIST_COLUMN) {
        if (j.radius < 0 || j.radius > kColumnMaxRadius || waves != j.waves) return hipErrorInvalidValue;
        if (column15(j)) {
            const int b = column15_bucket(j.levels), wi = column15_wave_index(waves);
            if (wi < 0) return hipErrorInvalidValue;
            k = kColumn15[wi][b];
            done = &g_column15_lds_done[wi][b];
        } else if (column31(j)) {
            const int b = column31_bucket(j.levels), wi = j.waves == 4 ? 1 : 0;
            if (waves != j.waves) return hipErrorInvalidValue;
            k = kColumn31[wi][b];
            done = &g_column31_lds_done[wi][b];
        } else {
            if (waves != 1) return hipErrorInvalidValue;
            const int nt = column_chunks(j.radius);
            k = kColumn[nt - 1];
            done = &g_column_lds_done[nt - 1];
        }
    } else if (j.hist == OILPAINT_HIST_STREAM && waves == kSplitWaves) {
        const int b = j.scan % kSplitWaves == 0 ? split_bucket(j.scan / kSplitWaves) : -1;
        if (j.radius < 0 || j.radius > kPackedMaxRadius || b < 0 || j.waves != kSplitWaves) return hipErrorInvalidValue;
        k = j.radius <= 7 ? kStreamSplit_lo[j.radius][b] : kStreamSplit_hi[j.radius - 8][b];
        done = &g_split4_lds_done[j.radius][b];
    } else if (j.hist == OILPAINT_HIST_REGS) {
        if (j.radius < 0 || j.radius > kRegsMaxRadius || j.levels > kRegsMaxLevels || waves != 1)
            return hipErrorInvalidValue;
        k = kRegs[j.radius][j.levels <= 8 ? 0 : 1];
        done = &g_regs_lds_done;
    } else if (j.hist == OILPAINT_HIST_STREAM8 && waves == kSplitWaves) {
        const int b = j.scan % kSplitWaves == 0 ? split_bucket(j.scan / kSplitWaves) : -1;
        if (j.radius < 8 || j.radius > kPackedMaxRadius || b < 0 || b > 3 || j.waves != kSplitWaves)
            return hipErrorInvalidValue;
        k = kStream8Split[j.radius - 8][b];
        done = &g_split_lds_done[j.radius - 8][b];
    } else if (j.hist == OILPAINT_HIST_STREAM8) {
        if (j.radius < 8 || j.radius > kPackedMaxRadius || j.scan > 32 || waves != 1) return hipErrorInvalidValue;
        k = kStream8[j.radius - 8];
        done = &g_stream8_lds_done[j.radius - 8];
    } else if (j.hist == OILPAINT_HIST_STREAM) {
        if (j.radius < 0 || j.radius > kPackedMaxRadius || j.scan > 64 || waves != 1) return hipErrorInvalidValue;
        const int b = j.scan <= 32 ? 0 : 1;
        k = j.radius <= 7 ? kStream_lo[j.radius][b] : kStream_hi[j.radius - 8][b];
        done = &g_stream_lds_done[j.radius][b];
    } else if (j.fast && j.radius >= 0 && j.radius <= kPackedMaxRadius && j.scan <= 64) {
        const int b = j.scan <= 16 ? 0 : j.scan <= 32 ? 1 : 2;
        k = j.radius <= 7 ? kFast_lo[j.radius][b] : kFast_hi[j.radius - 8][b];
        done = &g_fast_lds_done[j.radius][b];
    }
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(k), lds, *done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(tiles), dim3(64 * waves), lds, stream, j);
    return note_hip("k_plain launch", hipGetLastError());
}

hipError_t launch_batch(const BatchArgs& a, int cls, int waves, size_t lds, int grid, hipStream_t stream) {
    if (a.ntiles <= 0) return hipSuccess;
    if (cls < 0 || cls >= kBatchClasses || waves != batch_waves(cls)) return hipErrorInvalidValue;
    const BatchKernel k = batch_kernel(cls);
    const hipError_t e = allow_lds(reinterpret_cast<const void*>(k), lds, g_batch_lds_done[cls]);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * waves), lds, stream, a);
    return note_hip("batch kernel launch", hipGetLastError());
}

hipError_t launch_fill(uint8_t* p, size_t n, int width, hipStream_t stream) {
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, stream, p, n, width > 0 ? width : 1);
    return note_hip("k_fill launch", hipGetLastError());
}

hipError_t launch_reset_counters(uint32_t* counters, int n, int stride_words, hipStream_t stream) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, counters, n, stride_words);
    return note_hip("k_reset launch", hipGetLastError());
}

int batch_grid(int device, int cls, int waves, size_t lds) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(batch_kernel(cls)),
                                                     64 * waves, lds) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    const DeviceInfo d = device_info(device);
    return per_cu * (d.cus > 0 ? d.cus : 1);
}

}  // namespace oilpaint_impl
