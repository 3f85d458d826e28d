// Column-layout kernels (OILPAINT_HIST_COLUMN), plain and persistent batch
// forms, by the number of 64-column chunks of a strip with its halo
// (1..9: radius up to 255).
#include "oilpaint_column.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int NT>
__global__ __launch_bounds__(64) void k_plain_column(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_column<NT>(j, blockIdx.x, lds);
}

template <int NT>
__global__ __launch_bounds__(64) void k_batch_column(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    batch_column<NT>(a, lds);
}

}  // namespace

// By [chunks - 1].
const PlainKernel kColumn[kColumnChunks] = {k_plain_column<1>, k_plain_column<2>, k_plain_column<3>,
                                            k_plain_column<4>, k_plain_column<5>, k_plain_column<6>,
                                            k_plain_column<7>, k_plain_column<8>, k_plain_column<9>};
const BatchKernel kBatchColumn[kColumnChunks] = {k_batch_column<1>, k_batch_column<2>, k_batch_column<3>,
                                                 k_batch_column<4>, k_batch_column<5>, k_batch_column<6>,
                                                 k_batch_column<7>, k_batch_column<8>, k_batch_column<9>};

}  // namespace oilpaint_impl
