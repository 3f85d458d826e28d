// Tile-staged fast kernels, radius 0..7.
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

// One workgroup per tile, fast path for one (radius, scan bucket): each
// instantiation gets the registers its own radius needs.
template <int R, int SB>
__global__ __launch_bounds__(512) void k_plain_fast(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_packed_fast<R, SB>(j, xcd_tile(), lds);
}


}  // namespace

// Kernels for radius 0..7 by [radius - 0][scan bucket 16 / 32 / 64].
const PlainKernel kFast_lo[8][3] = {
    {k_plain_fast<0, 16>, k_plain_fast<0, 32>, k_plain_fast<0, 64>},
    {k_plain_fast<1, 16>, k_plain_fast<1, 32>, k_plain_fast<1, 64>},
    {k_plain_fast<2, 16>, k_plain_fast<2, 32>, k_plain_fast<2, 64>},
    {k_plain_fast<3, 16>, k_plain_fast<3, 32>, k_plain_fast<3, 64>},
    {k_plain_fast<4, 16>, k_plain_fast<4, 32>, k_plain_fast<4, 64>},
    {k_plain_fast<5, 16>, k_plain_fast<5, 32>, k_plain_fast<5, 64>},
    {k_plain_fast<6, 16>, k_plain_fast<6, 32>, k_plain_fast<6, 64>},
    {k_plain_fast<7, 16>, k_plain_fast<7, 32>, k_plain_fast<7, 64>}};

}  // namespace oilpaint_impl
