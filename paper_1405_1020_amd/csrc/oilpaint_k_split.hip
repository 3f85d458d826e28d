// Streamed-row kernels with 8-byte ring entries worked by four wavefronts per
// strip (OILPAINT_HIST_STREAM8, waves 4), radius 8..15: plain kernels by the
// number of bins each wavefront's mode search scans, and the persistent
// batch form (up to 8 bins per wavefront, the count from the job).
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int R, int MB>
__global__ __launch_bounds__(64 * kSplitWaves, kSplitMinWaves) void k_plain_split8(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_stream_split8<R, MB>(j, xcd_tile(), lds);
}

template <int R>
__global__ __launch_bounds__(64 * kSplitWaves) void k_batch_split8(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    batch_stream_split<R, 8, true>(a, lds);
}

}  // namespace

#define OILPAINT_SPLIT_ROW(R) {k_plain_split8<R, 2>, k_plain_split8<R, 4>, k_plain_split8<R, 5>, k_plain_split8<R, 8>}

// By [radius - 8][split_bucket(bins per wavefront)]: 2, 4, 5, 8 bins.
const PlainKernel kStream8Split[8][4] = {OILPAINT_SPLIT_ROW(8),  OILPAINT_SPLIT_ROW(9),  OILPAINT_SPLIT_ROW(10),
                                         OILPAINT_SPLIT_ROW(11), OILPAINT_SPLIT_ROW(12), OILPAINT_SPLIT_ROW(13),
                                         OILPAINT_SPLIT_ROW(14), OILPAINT_SPLIT_ROW(15)};

#undef OILPAINT_SPLIT_ROW

// By [radius - 8].
const BatchKernel kBatchSplit8[8] = {k_batch_split8<8>,  k_batch_split8<9>,  k_batch_split8<10>, k_batch_split8<11>,
                                     k_batch_split8<12>, k_batch_split8<13>, k_batch_split8<14>, k_batch_split8<15>};

}  // namespace oilpaint_impl
