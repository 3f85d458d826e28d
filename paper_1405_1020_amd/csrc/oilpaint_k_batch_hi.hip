// Persistent batch kernels of the streamed layout, radius 8..15: one kernel
// per (radius, scan bucket), each with the registers and LDS of its own
// class only.
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int R, int SB>
__global__ __launch_bounds__(64) void k_batch_stream(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    batch_stream<R, SB, false>(a, lds);
}

}  // namespace

// Kernels for radius 8..15 by [radius - 8][scan bucket 32 / 64].
const BatchKernel kBatchStream_hi[8][2] = {
    {k_batch_stream<8, 32>, k_batch_stream<8, 64>},
    {k_batch_stream<9, 32>, k_batch_stream<9, 64>},
    {k_batch_stream<10, 32>, k_batch_stream<10, 64>},
    {k_batch_stream<11, 32>, k_batch_stream<11, 64>},
    {k_batch_stream<12, 32>, k_batch_stream<12, 64>},
    {k_batch_stream<13, 32>, k_batch_stream<13, 64>},
    {k_batch_stream<14, 32>, k_batch_stream<14, 64>},
    {k_batch_stream<15, 32>, k_batch_stream<15, 64>}};

}  // namespace oilpaint_impl
