// Streamed-row kernels (4-byte ring entries) worked by four wavefronts per
// strip (OILPAINT_HIST_STREAM, waves 4), radius 8..15: plain kernels by the
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

// By [radius - 8][split_bucket(bins per wavefront)]: 2, 4, 5, 8, 16 bins.
const PlainKernel kStreamSplit_hi[8][5] = {
    OILPAINT_SPLIT_ROW(8), OILPAINT_SPLIT_ROW(9), OILPAINT_SPLIT_ROW(10), OILPAINT_SPLIT_ROW(11),
    OILPAINT_SPLIT_ROW(12), OILPAINT_SPLIT_ROW(13), OILPAINT_SPLIT_ROW(14), OILPAINT_SPLIT_ROW(15)};

#undef OILPAINT_SPLIT_ROW

// By [radius - 8][level bucket: up to 32, up to 64 levels].
const BatchKernel kBatchSplit_hi[8][2] = {{k_batch_split<8, 8>, k_batch_split<8, 16>}, {k_batch_split<9, 8>, k_batch_split<9, 16>}, {k_batch_split<10, 8>, k_batch_split<10, 16>}, {k_batch_split<11, 8>, k_batch_split<11, 16>}, {k_batch_split<12, 8>, k_batch_split<12, 16>}, {k_batch_split<13, 8>, k_batch_split<13, 16>}, {k_batch_split<14, 8>, k_batch_split<14, 16>}, {k_batch_split<15, 8>, k_batch_split<15, 16>}};

}  // namespace oilpaint_impl
