// Streamed-row kernels, radius 8..15.
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

// One wavefront per workgroup, streamed rows.
template <int R, int SB>
__global__ __launch_bounds__(64) void k_plain_stream(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_stream<R, SB, false>(j, xcd_tile(), lds);
}


}  // namespace

// Kernels for radius 8..15 by [radius - 8][scan bucket 32 / 64].
const PlainKernel kStream_hi[8][2] = {
    {k_plain_stream<8, 32>, k_plain_stream<8, 64>},
    {k_plain_stream<9, 32>, k_plain_stream<9, 64>},
    {k_plain_stream<10, 32>, k_plain_stream<10, 64>},
    {k_plain_stream<11, 32>, k_plain_stream<11, 64>},
    {k_plain_stream<12, 32>, k_plain_stream<12, 64>},
    {k_plain_stream<13, 32>, k_plain_stream<13, 64>},
    {k_plain_stream<14, 32>, k_plain_stream<14, 64>},
    {k_plain_stream<15, 32>, k_plain_stream<15, 64>}};

}  // namespace oilpaint_impl
