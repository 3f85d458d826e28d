// Tile-staged fast kernels, radius 8..15.
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

// Kernels for radius 8..15 by [radius - 8][scan bucket 16 / 32 / 64].
const PlainKernel kFast_hi[8][3] = {
    {k_plain_fast<8, 16>, k_plain_fast<8, 32>, k_plain_fast<8, 64>},
    {k_plain_fast<9, 16>, k_plain_fast<9, 32>, k_plain_fast<9, 64>},
    {k_plain_fast<10, 16>, k_plain_fast<10, 32>, k_plain_fast<10, 64>},
    {k_plain_fast<11, 16>, k_plain_fast<11, 32>, k_plain_fast<11, 64>},
    {k_plain_fast<12, 16>, k_plain_fast<12, 32>, k_plain_fast<12, 64>},
    {k_plain_fast<13, 16>, k_plain_fast<13, 32>, k_plain_fast<13, 64>},
    {k_plain_fast<14, 16>, k_plain_fast<14, 32>, k_plain_fast<14, 64>},
    {k_plain_fast<15, 16>, k_plain_fast<15, 32>, k_plain_fast<15, 64>}};

}  // namespace oilpaint_impl
