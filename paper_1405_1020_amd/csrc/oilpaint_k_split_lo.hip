// Streamed-row kernels (4-byte ring entries) worked by four wavefronts per
// strip (OILPAINT_HIST_STREAM, waves 4), radius 0..7, by the number of bins
// each wavefront's mode search scans.
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int R, int MB>
__global__ __launch_bounds__(64 * kSplitWaves) void k_plain_split(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_stream_split<R, MB, false>(j, blockIdx.x, lds);
}

}  // namespace

#define OILPAINT_SPLIT_ROW(R) \
    {k_plain_split<R, 2>, k_plain_split<R, 4>, k_plain_split<R, 5>, k_plain_split<R, 8>, k_plain_split<R, 16>}

// By [radius - 0][split_bucket(bins per wavefront)]: 2, 4, 5, 8, 16 bins.
const PlainKernel kStreamSplit_lo[8][5] = {
    OILPAINT_SPLIT_ROW(0), OILPAINT_SPLIT_ROW(1), OILPAINT_SPLIT_ROW(2), OILPAINT_SPLIT_ROW(3),
    OILPAINT_SPLIT_ROW(4), OILPAINT_SPLIT_ROW(5), OILPAINT_SPLIT_ROW(6), OILPAINT_SPLIT_ROW(7)};

#undef OILPAINT_SPLIT_ROW

}  // namespace oilpaint_impl
