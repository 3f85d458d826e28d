// Streamed-row kernels (4-byte ring entries) worked by four wavefronts per
// strip (OILPAINT_HIST_STREAM, waves 4), radius 0..7: plain kernels by the
// number of bins each wavefront's mode search scans, and the persistent batch
// form by level bucket (up to 8 or 16 bins per wavefront, the count from the
// job).
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int R, int MB>
__global__ __launch_bounds__(64 * kSplitWaves, kSplitMinWaves) void k_plain_split(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_stream_split<R, MB, false>(j, xcd_tile(), lds);
}

template <int R, int MB>
__global__ __launch_bounds__(64 * kSplitWaves) void k_batch_split(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    batch_stream_split<R, MB, false>(a, lds);
}

}  // namespace

#define OILPAINT_SPLIT_ROW(R) \
    {k_plain_split<R, 2>, k_plain_split<R, 4>, k_plain_split<R, 5>, k_plain_split<R, 8>, k_plain_split<R, 16>}

// By [radius - 0][split_bucket(bins per wavefront)]: 2, 4, 5, 8, 16 bins.
const PlainKernel kStreamSplit_lo[8][5] = {
    OILPAINT_SPLIT_ROW(0), OILPAINT_SPLIT_ROW(1), OILPAINT_SPLIT_ROW(2), OILPAINT_SPLIT_ROW(3),
    OILPAINT_SPLIT_ROW(4), OILPAINT_SPLIT_ROW(5), OILPAINT_SPLIT_ROW(6), OILPAINT_SPLIT_ROW(7)};

#undef OILPAINT_SPLIT_ROW

// By [radius - 0][level bucket: up to 32, up to 64 levels].
const BatchKernel kBatchSplit_lo[8][2] = {{k_batch_split<0, 8>, k_batch_split<0, 16>}, {k_batch_split<1, 8>, k_batch_split<1, 16>}, {k_batch_split<2, 8>, k_batch_split<2, 16>}, {k_batch_split<3, 8>, k_batch_split<3, 16>}, {k_batch_split<4, 8>, k_batch_split<4, 16>}, {k_batch_split<5, 8>, k_batch_split<5, 16>}, {k_batch_split<6, 8>, k_batch_split<6, 16>}, {k_batch_split<7, 8>, k_batch_split<7, 16>}};

}  // namespace oilpaint_impl
