// Internal interface between the JPEG host code (oilpaint_jpeg.cpp: marker
// syntax, Huffman coding, buffers) and its kernels (oilpaint_k_jpeg.hip:
// dequantization and inverse DCT, colour, forward DCT and quantization).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace oilpaint_impl {

constexpr int kJpegMaxComps = 3;

// Inverse DCT of every block of every component: coefficients (int16,
// natural order, 64 per block, each component's blocks in raster order over
// its block grid) -> 8-bit samples.  Component c's blocks are
// [first[c], first[c+1]) of the flattened list; its grid is bw[c] blocks
// wide; samples outside [0, limit_w) x [0, limit_h) are not written.
struct JpegIdctArgs {
    const int16_t* coef;
    uint8_t* plane[kJpegMaxComps];
    int32_t stride[kJpegMaxComps];
    int32_t bw[kJpegMaxComps];
    int32_t limit_w[kJpegMaxComps];
    int32_t limit_h[kJpegMaxComps];
    int32_t first[kJpegMaxComps + 1];
    uint16_t q[kJpegMaxComps][64];  // natural order
};

// Component samples -> interleaved RGB (JFIF), chroma replicated: the sample
// of component c under output pixel (x, y) is (x h[c] / hmax, y v[c] / vmax).
struct JpegColorArgs {
    const uint8_t* plane[kJpegMaxComps];
    int32_t stride[kJpegMaxComps];
    int32_t h[kJpegMaxComps], v[kJpegMaxComps];
    int32_t hmax, vmax, ncomp;
    int32_t width, height;
    uint8_t* dst;
    int32_t dst_stride;
};

// RGB -> Y, Cb, Cr planes over the MCU-padded grid (the image extended by
// repeating its last column and row); chroma averaged over fh x fv luma
// samples (rounded half up).  Y plane ymcu_w x ymcu_h, chroma planes
// (ymcu_w / fh) x (ymcu_h / fv).
struct JpegRgbArgs {
    const uint8_t* src;
    int32_t stride, width, height;
    int32_t ymcu_w, ymcu_h, fh, fv;
    uint8_t* plane[kJpegMaxComps];
    int32_t pstride[kJpegMaxComps];
};

// Forward DCT of (sample - 128) and quantization (nearest, halves away from
// zero) of every block; same block numbering as JpegIdctArgs.
struct JpegFdctArgs {
    const uint8_t* plane[kJpegMaxComps];
    int32_t stride[kJpegMaxComps];
    int32_t bw[kJpegMaxComps];
    int32_t first[kJpegMaxComps + 1];
    uint16_t q[kJpegMaxComps][64];
    int16_t* coef;
};

hipError_t launch_jpeg_idct(const JpegIdctArgs& a, hipStream_t stream);
hipError_t launch_jpeg_color(const JpegColorArgs& a, hipStream_t stream);
hipError_t launch_jpeg_rgb(const JpegRgbArgs& a, hipStream_t stream);
hipError_t launch_jpeg_fdct(const JpegFdctArgs& a, hipStream_t stream);

}  // namespace oilpaint_impl
