// Streamed-row kernels, radius 0..7.
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

// Kernels for radius 0..7 by [radius - 0][scan bucket 32 / 64].
const PlainKernel kStream_lo[8][2] = {
    {k_plain_stream<0, 32>, k_plain_stream<0, 64>},
    {k_plain_stream<1, 32>, k_plain_stream<1, 64>},
    {k_plain_stream<2, 32>, k_plain_stream<2, 64>},
    {k_plain_stream<3, 32>, k_plain_stream<3, 64>},
    {k_plain_stream<4, 32>, k_plain_stream<4, 64>},
    {k_plain_stream<5, 32>, k_plain_stream<5, 64>},
    {k_plain_stream<6, 32>, k_plain_stream<6, 64>},
    {k_plain_stream<7, 32>, k_plain_stream<7, 64>}};

}  // namespace oilpaint_impl
