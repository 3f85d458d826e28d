// Persistent batch kernels of the streamed layout, radius 0..7: one kernel
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

// Kernels for radius 0..7 by [radius - 0][scan bucket 32 / 64].
const BatchKernel kBatchStream_lo[8][2] = {
    {k_batch_stream<0, 32>, k_batch_stream<0, 64>},
    {k_batch_stream<1, 32>, k_batch_stream<1, 64>},
    {k_batch_stream<2, 32>, k_batch_stream<2, 64>},
    {k_batch_stream<3, 32>, k_batch_stream<3, 64>},
    {k_batch_stream<4, 32>, k_batch_stream<4, 64>},
    {k_batch_stream<5, 32>, k_batch_stream<5, 64>},
    {k_batch_stream<6, 32>, k_batch_stream<6, 64>},
    {k_batch_stream<7, 32>, k_batch_stream<7, 64>}};

}  // namespace oilpaint_impl
