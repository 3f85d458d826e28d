// Streamed-row kernels (4-byte ring entries) worked by four wavefronts per
// strip (OILPAINT_HIST_STREAM, waves 4), radius 8..15, by the number of bins
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

// By [radius - 8][split_bucket(bins per wavefront)]: 2, 4, 5, 8, 16 bins.
const PlainKernel kStreamSplit_hi[8][5] = {
    OILPAINT_SPLIT_ROW(8), OILPAINT_SPLIT_ROW(9), OILPAINT_SPLIT_ROW(10), OILPAINT_SPLIT_ROW(11),
    OILPAINT_SPLIT_ROW(12), OILPAINT_SPLIT_ROW(13), OILPAINT_SPLIT_ROW(14), OILPAINT_SPLIT_ROW(15)};

#undef OILPAINT_SPLIT_ROW

}  // namespace oilpaint_impl
