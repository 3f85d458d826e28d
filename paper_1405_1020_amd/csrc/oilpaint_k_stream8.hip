// Streamed-row kernels with 8-byte ring entries (OILPAINT_HIST_STREAM8),
// radius 8..15, at most 32 scanned levels: plain and persistent batch forms.
#include "oilpaint_device.h"

namespace oilpaint_impl {
using namespace dev;
namespace {

template <int R>
__global__ __launch_bounds__(64) void k_plain_stream8(Job j) {
    extern __shared__ __align__(16) uint8_t lds[];
    tile_stream<R, 32, true>(j, xcd_tile(), lds);
}

template <int R>
__global__ __launch_bounds__(64) void k_batch_stream8(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    batch_stream<R, 32, true>(a, lds);
}

}  // namespace

// By [radius - 8].
const PlainKernel kStream8[8] = {k_plain_stream8<8>,  k_plain_stream8<9>,  k_plain_stream8<10>, k_plain_stream8<11>,
                                 k_plain_stream8<12>, k_plain_stream8<13>, k_plain_stream8<14>, k_plain_stream8<15>};
const BatchKernel kBatchStream8[8] = {k_batch_stream8<8>,  k_batch_stream8<9>,  k_batch_stream8<10>,
                                      k_batch_stream8<11>, k_batch_stream8<12>, k_batch_stream8<13>,
                                      k_batch_stream8<14>, k_batch_stream8<15>};

}  // namespace oilpaint_impl
