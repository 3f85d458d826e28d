// LDS instruction-rate probe.  Not part of the filter: it measures, on the GPU
// at hand, how many LDS bytes (reads) or 64-lane 64-bit atomic adds a CU
// completes per shader clock, the rates the filter's LDS work is priced
// against in its roofline.
#include "oilpaint_device.h"

namespace oilpaint_impl {
int check_device_ptr(const void* p);
namespace {

constexpr int kProbeRows = 64;               // rows of 64 eight-byte words
constexpr int kProbeWords = kProbeRows * 64;  // 32 KB per workgroup
constexpr int kProbeUnroll = 16;

// Each of the four wavefronts issues iters x 16 LDS instructions of one kind:
//   OILPAINT_PROBE_READ64: 8-byte reads (the compiler may pair two rows into
//                          one instruction; bytes are what is counted)
//   OILPAINT_PROBE_ADD64:  64-bit atomic adds of 1, result unused
//   OILPAINT_PROBE_READ32: 4-byte reads
// Lane l of an instruction touches word l of a row, so the 64 lanes cover 64
// consecutive words (no bank conflicts); the row moves with the iteration
// and the wavefront.  Between two barriers, wavefront 0 reads the shader
// clock (s_memtime) and the 100 MHz real-time counter (s_memrealtime).
template <int KIND>
__global__ __launch_bounds__(256) void k_lds_probe(int iters, uint64_t* clocks) {
    __shared__ uint64_t w[kProbeWords];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kProbeWords; i += 256) w[i] = (uint64_t)i * 0x9E3779B97F4A7C15ull;
    __syncthreads();
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    uint64_t acc = 0;
    uint32_t acc32 = 0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kProbeUnroll; ++k) {
            const int row = (it + k + wave * kProbeUnroll) & (kProbeRows - 1);
            const int idx = row * 64 + lane;
            if (KIND == OILPAINT_PROBE_READ64) {
                acc ^= w[idx];
            } else if (KIND == OILPAINT_PROBE_ADD64) {
                __hip_atomic_fetch_add(&w[idx], (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
                acc32 ^= reinterpret_cast<const uint32_t*>(w)[row * 128 + lane];
            }
        }
    }
    __syncthreads();
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
        uint64_t* c = clocks + 4 * (size_t)blockIdx.x;
        c[0] = t0;
        c[1] = t1;
        c[2] = r0;
        c[3] = r1;
    }
    // keep the reads (and the atomics' words) alive: a store no launch takes
    const uint64_t keep = acc ^ acc32 ^ w[(lane * 7) & (kProbeWords - 1)];
    if (keep == 0x5a5a5a5a5a5a5a5aull && iters < 0) clocks[4 * (size_t)blockIdx.x] = keep;
}

}  // namespace
}  // namespace oilpaint_impl

using namespace oilpaint_impl;

extern "C" int oilpaint_lds_probe(int kind, int iters, int per_cu, uint64_t* clocks, int max_workgroups,
                                  int* workgroups, void* stream) {
    if (!clocks || !workgroups) return OILPAINT_ERR_NULL;
    if (iters < 1 || iters > (1 << 20) || per_cu < 1 || per_cu > 4) return OILPAINT_ERR_ARG;
    if (kind != OILPAINT_PROBE_READ64 && kind != OILPAINT_PROBE_ADD64 && kind != OILPAINT_PROBE_READ32)
        return OILPAINT_ERR_ARG;
    int device = 0;
    if (note_hip("hipGetDevice", hipGetDevice(&device)) != hipSuccess) return OILPAINT_ERR_HIP;
    const DeviceInfo d = device_info(device);
    if (!d.ok) return OILPAINT_ERR_HIP;
    const int grid = per_cu * d.cus;
    *workgroups = grid;
    if (grid > max_workgroups) return OILPAINT_ERR_ARG;
    const int st = check_device_ptr(clocks);
    if (st != OILPAINT_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    if (kind == OILPAINT_PROBE_READ64)
        hipLaunchKernelGGL(k_lds_probe<OILPAINT_PROBE_READ64>, dim3(grid), dim3(256), 0, s, iters, clocks);
    else if (kind == OILPAINT_PROBE_ADD64)
        hipLaunchKernelGGL(k_lds_probe<OILPAINT_PROBE_ADD64>, dim3(grid), dim3(256), 0, s, iters, clocks);
    else
        hipLaunchKernelGGL(k_lds_probe<OILPAINT_PROBE_READ32>, dim3(grid), dim3(256), 0, s, iters, clocks);
    return note_hip("k_lds_probe launch", hipGetLastError()) == hipSuccess ? OILPAINT_OK : OILPAINT_ERR_HIP;
}
