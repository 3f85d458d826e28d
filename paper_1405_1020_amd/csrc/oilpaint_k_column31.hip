// Column-layout kernels for radius 16..31 (OILPAINT_HIST_COLUMN, two or four
// wavefronts per strip): the radius <= 15 form's count words and pass 2 with
// 16-bit window counts and 20-bit window sums (tile_column15's WIDE form).
#include "oilpaint_column.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int NW, int NV>
__global__ __launch_bounds__(64 * NV) void k_plain_column31(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_column15<NW, NV, true>(j, xcd_tile(), lds);
}

}  // namespace

// By [waves == 4][column31_bucket(levels)]: 4, 10, 16 or 32 count words.
const PlainKernel kColumn31[2][kColumn15Buckets] = {
    {k_plain_column31<4, 2>, k_plain_column31<10, 2>, k_plain_column31<16, 2>, k_plain_column31<32, 2>},
    {k_plain_column31<4, 4>, k_plain_column31<10, 4>, k_plain_column31<16, 4>, k_plain_column31<32, 4>}};

}  // namespace oilpaint_impl
