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
//     ceil(total / 32) + 1 words; bit 0 the most significant of word 0);
//     `cus` sizes the grids.
//   launch_huff_stuff: the nbits-bit stream, its last byte padded with one
//     bits, with a zero byte after every 0xFF into `out` (room for twice its
//     bytes); *ff_total receives the number of 0xFF bytes (tiles as above,
//     huff_scan_tiles of the byte count).
int64_t huff_scan_tiles(int64_t n);
hipError_t launch_huff_stats(const JpegScanMap& m, const int16_t* coef, unsigned long long* freq, int cus,
                             hipStream_t stream);
hipError_t launch_huff_code(const JpegScanMap& m, const int16_t* coef, const uint32_t* tabs, uint32_t* bits,
                            uint64_t* offset, uint64_t* tiles, uint64_t* total, uint32_t* words, int cus,
                            hipStream_t stream);
hipError_t launch_huff_stuff(const uint32_t* words, uint64_t nbits, uint64_t* tiles, uint64_t* ff_total,
                             uint8_t* out, hipStream_t stream);

// Exclusive prefix sums of n 32-bit values into 64-bit `out` (tiles:
// huff_scan_tiles(n) entries; *total receives the sum).
hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint64_t* tiles, uint64_t* total, uint64_t* out,
                                 hipStream_t stream);

// Huffman decoding on the device (oilpaint_k_huffdec.hip).  The host takes
// the stuffed zero bytes and the RST markers out of a scan's entropy-coded
// data (T.81 B.1.1.5, E.1.4) and cuts each restart interval's bits into
// subsequences of equal length; a subsequence decodes the symbols that
// start in it.  Where its decoding really starts -- the bit, the block of the
// MCU, the coefficient -- is where its predecessor's decoding crosses into it,
// known only by decoding everything before.  So each subsequence is first
// decoded from every guess of a track: its first bit, any block j of the MCU,
// coefficient 0 or 1 (a block's DC, or its first AC symbol).  Decodings that
// meet in one state stay together, and Huffman codes resynchronize: the true
// decoding usually coincides with one of the tracks at the checkpoint (the
// first symbol boundary kJpegCheckBits into the subsequence).  A link pass
// decodes from every track's exit state to the next subsequence's checkpoint
// and names the track met there; the host follows the links from each
// interval's known start (decoding itself the rare subsequence whose true
// decoding meets no track) and hands every subsequence its true start state
// and first block; the last pass decodes and writes the coefficients.  The
// subsequence length is chosen per scan from its length (auto_sub_bits)
// unless oilpaint_jpeg_set_subsequence_bits fixes it.
constexpr int kJpegCheckBits = 256;  // the checkpoint, at most half the subsequence length

// One table for decoding (T.81 C, F.2.2.3): codes up to kJpegFastBits bits
// by lookup, longer ones by the largest code of each length.  (At 9 bits the
// lanes of a wavefront met a longer code in 71 % of the steps on a
// 1920x1080 photo-like image at quality 90, at 11 bits in 17 %.)
constexpr int kJpegFastBits = 11;
struct JpegHuffTable {
    uint16_t fast[1 << kJpegFastBits];  // (length << 8) | value by the leading bits; 0: the code is longer
    int32_t maxcode[18];  // largest code of each length, -1 for none
    int32_t valoff[17];   // value index = code + valoff[length]
    uint8_t vals[256];
};

// A subsequence: the symbols starting in bits [begin, end) of the scan's
// data; its restart interval `seg` ends at bit seg_end (bits from there on
// read as 0).  flags: 1 the interval's first subsequence, 2 its last.
struct JpegSub {
    uint64_t begin, end, seg_end;
    int32_t seg, flags;
};

// A restart interval: its blocks [first_block, end_block) in scan order,
// its first subsequence.
struct JpegSeg {
    int64_t first_block, end_block;
    int32_t first_sub, pad;
};

// One scan for decoding.  Block t of the scan (MCUs in raster order, mcux
// per row, bpm blocks each) is block j = t mod bpm of its MCU: component
// comp[j] (a frame component), at (dx[j], dy[j]) in that MCU's h x v blocks
// of it, decoded with DC table dct[j] and AC table act[j] (0..3).  For an
// interleaved scan h, v are the sampling factors; a scan of one component
// has MCUs of one block (h = v = 1) over that component's own block grid.
// Scan component k (0..ns-1) has nb[k] blocks per MCU starting at off[k].
// Tracks: 2 x bpm per subsequence, track u starting at block u / 2,
// coefficient u % 2.
struct JpegDecScan {
    const uint32_t* words;  // the scan's data as 32-bit words, the first bit the most significant of words[0]
    const JpegHuffTable* tables;  // DC 0-3, then AC 0-3
    const JpegSub* subs;
    const JpegSeg* segs;
    int16_t* coef;          // natural order, the frame's layout
    uint32_t* dcdiff;       // per scan block: DC difference + kJpegDcBias
    int64_t blocks, mcus, nwords;  // nwords: readable words (the data and 16 zero bytes)
    int32_t nsub, bpm, mcux, restart, ns, check_bits;
    uint32_t dsel, asel;    // the DC and AC table of MCU block j in bits 2j, 2j + 1
    int32_t comp[kJpegMaxMcuBlocks], dx[kJpegMaxMcuBlocks], dy[kJpegMaxMcuBlocks];
    int32_t dct[kJpegMaxMcuBlocks], act[kJpegMaxMcuBlocks];
    int32_t nb[kJpegMaxComps], off[kJpegMaxComps];
    int32_t h[kJpegMaxComps], v[kJpegMaxComps], bw[kJpegMaxComps], first[kJpegMaxComps];
};
constexpr uint32_t kJpegDcBias = 2048;  // DC differences lie in [-2047, 2047]

// Decoder states are packed as bit << 16 | block of the MCU << 8 | coefficient.
// A track of subsequence i: its state at the checkpoint and at its exit (the
// first symbol boundary at or past the subsequence's end), the blocks it
// completes before the checkpoint and between checkpoint and exit.
struct JpegTrack {
    uint64_t check, exit;
    uint32_t pre, post;
};
// A link from track u of subsequence i: the track of subsequence i + 1 met
// at its checkpoint (kJpegNoTrack: none), the blocks completed on the way.
struct JpegLink {
    uint32_t next, blocks;
};
constexpr uint32_t kJpegNoTrack = 0xFFFFFFFFu;
// What the host hands the decode pass, two parts per subsequence: the true
// state and block where a part starts, the bit where it stops (it decodes the
// symbols starting before `stop`); kJpegStopAtBlocks: until its restart
// interval's blocks are complete (an interval's last subsequence); block -1:
// nothing (the second part of a subsequence decoded whole by its first).
// A subsequence whose true decoding meets track u splits at the checkpoint,
// the second part starting from the track's state there.
struct JpegEntry {
    uint64_t state;
    int64_t block;
    uint64_t stop;
};
constexpr uint64_t kJpegStopAtBlocks = ~0ull;

// Tracks and links of every subsequence (2 x bpm each); sub_bits: the
// subsequences' length (at most kJpegMaxSubBits); tracks_done, if not null,
// is recorded on `stream` once the tracks are written (before the links).
constexpr int kJpegMaxSubBits = 16384;
hipError_t launch_huff_tracks(const JpegDecScan& s, int sub_bits, JpegTrack* tracks, JpegLink* links,
                              hipEvent_t tracks_done, hipStream_t stream);
// The decoding from the entries: coefficients into coef, DC differences
// into dcdiff, a malformed code flagged in *malformed; then the DC prefix
// sums per component and restart interval into coef (dcseq / dcsum: per
// scan block; tiles and total for their prefix sums).
hipError_t launch_huff_decode(const JpegDecScan& s, int sub_bits, const JpegEntry* entries, uint32_t* malformed,
                              uint64_t* tiles, uint64_t* total, uint32_t* dcseq, uint64_t* dcsum, hipStream_t stream);

hipError_t launch_jpeg_idct(const JpegIdctArgs& a, hipStream_t stream);
hipError_t launch_jpeg_color(const JpegColorArgs& a, hipStream_t stream);
hipError_t launch_jpeg_rgb(const JpegRgbArgs& a, hipStream_t stream);
hipError_t launch_jpeg_fdct(const JpegFdctArgs& a, hipStream_t stream);

}  // namespace oilpaint_impl
