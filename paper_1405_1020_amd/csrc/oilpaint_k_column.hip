// Column-layout kernels (OILPAINT_HIST_COLUMN), plain and persistent batch
// forms, by the number of 64-column chunks of a strip with its halo
// (1..9: radius up to 255), and the radius <= 15 form by prefix words.
#include "oilpaint_column.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int NT>
__global__ __launch_bounds__(64) void k_plain_column(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_column<NT>(j, xcd_tile(), lds);
}

template <int NT>
__global__ __launch_bounds__(64) void k_batch_column(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    batch_column<NT>(a, lds);
}

template <int NW, int NV>
__global__ __launch_bounds__(64 * NV) void k_plain_column15(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_column15<NW, NV>(j, xcd_tile(), lds);
}

template <int NW>
__global__ __launch_bounds__(64) void k_batch_column15(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    batch_column15<NW, 1>(a, lds);
}

template <int NW>
__global__ __launch_bounds__(256) void k_batch_column15x4(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    batch_column15<NW, 4>(a, lds);
}

}  // namespace

// By [column15_wave_index(waves)][column15_bucket(levels)].
const PlainKernel kColumn15[3][kColumn15Buckets] = {
    {k_plain_column15<3, 1>, k_plain_column15<7, 1>, k_plain_column15<11, 1>, k_plain_column15<22, 1>},
    {k_plain_column15<3, 2>, k_plain_column15<7, 2>, k_plain_column15<11, 2>, k_plain_column15<22, 2>},
    {k_plain_column15<3, 4>, k_plain_column15<7, 4>, k_plain_column15<11, 4>, k_plain_column15<22, 4>}};
// By [column15_bucket(levels)].
const BatchKernel kBatchColumn15[kColumn15Buckets] = {k_batch_column15<3>, k_batch_column15<7>,
                                                      k_batch_column15<11>, k_batch_column15<22>};
const BatchKernel kBatchColumn15x4[kColumn15Buckets] = {k_batch_column15x4<3>, k_batch_column15x4<7>,
                                                        k_batch_column15x4<11>, k_batch_column15x4<22>};

// By [chunks - 1].
const PlainKernel kColumn[kColumnChunks] = {k_plain_column<1>, k_plain_column<2>, k_plain_column<3>,
                                            k_plain_column<4>, k_plain_column<5>, k_plain_column<6>,
                                            k_plain_column<7>, k_plain_column<8>, k_plain_column<9>};
const BatchKernel kBatchColumn[kColumnChunks] = {k_batch_column<1>, k_batch_column<2>, k_batch_column<3>,
                                                 k_batch_column<4>, k_batch_column<5>, k_batch_column<6>,
                                                 k_batch_column<7>, k_batch_column<8>, k_batch_column<9>};

}  // namespace oilpaint_impl
