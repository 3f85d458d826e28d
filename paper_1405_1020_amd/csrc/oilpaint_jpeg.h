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

// The encoder's one interleaved scan, block by block (T.81 A.2.3): block t
// is block j = t mod bpm of MCU t / bpm, MCUs in raster order, mcux per row.
// Block j of an MCU belongs to component comp[j], at (dx[j], dy[j]) in the
// MCU's h[c] x v[c] blocks of that component; prev[j] is the index in the
// MCU of the previous block of the same component (-1 for the first, whose
// DC predictor is the previous MCU's block last[c]); tab[c] selects the
// Huffman tables (0 luminance, 1 chrominance).
constexpr int kJpegMaxMcuBlocks = 10;
struct JpegScanMap {
    int64_t blocks;
    int32_t bpm, mcux;
    int32_t comp[kJpegMaxMcuBlocks], dx[kJpegMaxMcuBlocks], dy[kJpegMaxMcuBlocks], prev[kJpegMaxMcuBlocks];
    int32_t last[kJpegMaxComps], h[kJpegMaxComps], v[kJpegMaxComps], bw[kJpegMaxComps], first[kJpegMaxComps];
    int32_t tab[kJpegMaxComps];
};

// Huffman coding on the device (oilpaint_k_huff.hip).
//   launch_huff_stats: symbol counts of the scan added to freq[4][256] (DC
//     luminance, DC chrominance, AC luminance, AC chrominance); `cus`
//     workgroups at most.
//   launch_huff_code: with tabs[4][256] = size << 16 | code of each symbol,
//     the bits of every block (bits[blocks]), their exclusive prefix sums
//     (offset[blocks], using tiles[huff_scan_tiles(blocks)], total bits in
//     *total) and the stream itself ORed into `words` (zeroed beforehand,
//     ceil(total / 32) + 1 words; bit 0 the most significant of word 0).
//   launch_huff_stuff: the nbits-bit stream, its last byte padded with one
//     bits, with a zero byte after every 0xFF into `out` (room for twice its
//     bytes); *ff_total receives the number of 0xFF bytes (tiles as above,
//     huff_scan_tiles of the byte count).
int64_t huff_scan_tiles(int64_t n);
hipError_t launch_huff_stats(const JpegScanMap& m, const int16_t* coef, unsigned long long* freq, int cus,
                             hipStream_t stream);
hipError_t launch_huff_code(const JpegScanMap& m, const int16_t* coef, const uint32_t* tabs, uint32_t* bits,
                            uint64_t* offset, uint64_t* tiles, uint64_t* total, uint32_t* words,
                            hipStream_t stream);
hipError_t launch_huff_stuff(const uint32_t* words, uint64_t nbits, uint64_t* tiles, uint64_t* ff_total,
                             uint8_t* out, hipStream_t stream);

hipError_t launch_jpeg_idct(const JpegIdctArgs& a, hipStream_t stream);
hipError_t launch_jpeg_color(const JpegColorArgs& a, hipStream_t stream);
hipError_t launch_jpeg_rgb(const JpegRgbArgs& a, hipStream_t stream);
hipError_t launch_jpeg_fdct(const JpegFdctArgs& a, hipStream_t stream);

}  // namespace oilpaint_impl
