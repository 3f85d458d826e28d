// Huffman decoding of baseline JPEG scans on the GPU (T.81 F.2.2: DC
// differences and run/size symbols, codes by the DECODE procedure of
// F.2.2.3), parallel over subsequences of the entropy-coded data.
//
// The data is a sequence of variable-length codes, so where a symbol starts
// is known only by decoding everything before it.  Each subsequence decodes
// the symbols that start within its bits, from a start state it does not
// know.  The tracks pass decodes every subsequence from 2 x bpm guesses (its
// first bit; any block of the MCU; its DC, or its first AC symbol), one
// thread each, recording each track's state at the checkpoint and at the
// exit.  The links pass decodes from every track's exit into the next
// subsequence up to its checkpoint and looks the state up among that
// subsequence's tracks.  The host follows the links from each restart
// interval's known start and returns the true start state and first block
// of every subsequence; the decode pass then decodes each subsequence once
// more from there, writing the coefficients.  DC values are prefix sums of
// the differences per component within each restart interval.
//
// A workgroup stages the bits its threads read (its subsequences and what
// follows them, byte-swapped words) in LDS with the Huffman tables: the
// threads of a wavefront decode different positions, so reads from device
// memory would stall the whole wavefront for whichever lane needs a word.
#include <algorithm>

#include "oilpaint_internal.h"
#include "oilpaint_jpeg.h"

namespace oilpaint_impl {
namespace {

// Zig-zag order (T.81 Figure A.6): the natural index of the k-th coefficient.
__constant__ uint8_t kZzDec[64] = {0,  1,  8,  16, 9,  2,  3,  10, 17, 24, 32, 25, 18, 11, 4,  5,
                                   12, 19, 26, 33, 40, 48, 41, 34, 27, 20, 13, 6,  7,  14, 21, 28,
                                   35, 42, 49, 56, 57, 50, 43, 36, 29, 22, 15, 23, 30, 37, 44, 51,
                                   58, 59, 52, 45, 38, 31, 39, 46, 53, 60, 61, 54, 47, 55, 62, 63};

constexpr int kTables = 8;                // DC 0-3, AC 0-3
constexpr int kTableWords = kTables * (int)sizeof(JpegHuffTable) / 4;
constexpr int kStageMarginBits = 192;     // past the last subsequence: checkpoint overrun and the reader's window
constexpr int kStageBudgetBits = 196608;  // staged subsequence bits per workgroup (24 KB; with the tables under 64 KB)

// Subsequences per workgroup for `per` threads each.
__host__ __device__ inline int group_subs(int per, int sub_bits) {
    const int by_threads = 256 / per;
    const int by_lds = kStageBudgetBits / sub_bits;
    return by_threads < by_lds ? by_threads : by_lds;
}
__host__ __device__ inline int stage_words(int group, int sub_bits, int check_bits) {
    return (int)(((int64_t)group * sub_bits + check_bits + kStageMarginBits) / 32) + 4;
}

// Copy the tables and the words [w0, w0 + n) of the data (byte-swapped;
// clamped to the readable words) into LDS.  Every thread calls it, with 256
// threads per workgroup.  Each round issues its loads before its stores, with
// indices clamped so that no branch stands between them, so that a round
// costs one memory latency rather than one per load.
static_assert(kTableWords % 4 == 0, "tables in 16-byte units");
__device__ __forceinline__ void stage(const JpegDecScan& s, uint32_t* lds_tables, uint32_t* lds_words, int64_t w0,
                                      int n) {
    constexpr int kT16 = kTableWords / 4;
    constexpr int kR = 5;
    const uint4* src = reinterpret_cast<const uint4*>(s.tables);
    uint4* dst = reinterpret_cast<uint4*>(lds_tables);
    const int t = (int)threadIdx.x;
    for (int base = 0; base < kT16; base += 256 * kR) {
        uint4 v0 = src[min(base + t, kT16 - 1)], v1 = src[min(base + t + 256, kT16 - 1)],
              v2 = src[min(base + t + 512, kT16 - 1)], v3 = src[min(base + t + 768, kT16 - 1)],
              v4 = src[min(base + t + 1024, kT16 - 1)];
        if (base + t < kT16) dst[base + t] = v0;
        if (base + t + 256 < kT16) dst[base + t + 256] = v1;
        if (base + t + 512 < kT16) dst[base + t + 512] = v2;
        if (base + t + 768 < kT16) dst[base + t + 768] = v3;
        if (base + t + 1024 < kT16) dst[base + t + 1024] = v4;
    }
    constexpr int kW = 8;
    const int64_t last = s.nwords - 1;
    for (int base = 0; base < n; base += 256 * kW) {
        uint32_t wv[kW];
#pragma unroll
        for (int r = 0; r < kW; ++r) {
            const int64_t g = w0 + base + t + 256 * r;
            wv[r] = s.words[g < last ? g : last];
        }
#pragma unroll
        for (int r = 0; r < kW; ++r) {
            const int i = base + t + 256 * r;
            if (i < n) lds_words[i] = w0 + i < s.nwords ? __builtin_bswap32(wv[r]) : 0u;
        }
    }
    __syncthreads();
}

// The codes longer than kJpegFastBits, up to 16 bits (T.81 F.2.2.3, DECODE):
// (length << 8) | value of the code that begins the 16 bits `top`, 0 if none
// does.
__device__ __forceinline__ uint32_t slow_code(const JpegHuffTable& t, uint32_t top) {
    for (uint32_t l = kJpegFastBits + 1; l <= 16; ++l) {
        const int32_t code = (int32_t)(top >> (16 - l));
        if (code <= t.maxcode[l]) return l << 8 | t.vals[(code + t.valoff[l]) & 255];
    }
    return 0u;
}

// Value of the t-bit magnitude v (T.81 F.2.2.1, EXTEND).
__device__ __forceinline__ int extend(uint32_t v, uint32_t t) {
    return (t && v < (1u << (t - 1))) ? (int)v - (1 << t) + 1 : (int)v;
}

// A decoding in progress over a workgroup's staged words: the position of
// the next symbol (bits from the staged region's first bit), the block of the
// MCU, the next coefficient of that block (0: its DC), and a window of three
// words in registers at `base`.  Bits at or past `end` (the restart
// interval's end) read as 0.  A symbol moves the position by at most 27 bits,
// so one step of the window per symbol suffices.
struct Dec {
    const uint32_t* w;
    uint32_t p, end, base, j, z;
    uint32_t a, b, c;
    __device__ __forceinline__ void init(const uint32_t* staged, uint64_t w0bit, uint64_t state, uint64_t seg_end) {
        w = staged;
        p = (uint32_t)((state >> 16) - w0bit);
        const uint64_t e = seg_end - w0bit;
        end = e < 0xFFFFFFFFull ? (uint32_t)e : 0xFFFFFFFFu;
        j = (uint32_t)(state >> 8) & 255u;
        z = (uint32_t)state & 255u;
        base = p & ~31u;
        a = b = c = 0u;
        if (p < end) {
            const uint32_t k = base >> 5;
            a = w[k];
            b = w[k + 1];
            c = w[k + 2];
        }
    }
    __device__ __forceinline__ uint64_t state(uint64_t w0bit) const {
        return ((uint64_t)p + w0bit) << 16 | (uint64_t)j << 8 | z;
    }
    __device__ __forceinline__ uint32_t peek32() {
        if (p >= end) return 0u;
        if (p - base >= 32) {
            a = b;
            b = c;
            base += 32;
            c = w[(base >> 5) + 2];
        }
        const uint32_t sh = p - base;
        uint32_t v = sh ? (a << sh) | (b >> (32 - sh)) : a;
        if (end - p < 32) v &= 0xFFFFFFFFu << (32 - (end - p));
        return v;
    }
};

// Where the decode pass writes: the DC difference of scan block t and the
// coefficients of its block, the MCU (mx, my) followed block by block.
struct Out {
    int64_t t;
    int32_t mx, my;
    int16_t* blk;
};

// Per MCU block j, in LDS for the decode pass: its component's first block,
// its grid's width and the block's position (h * mx + dx, v * my + dy).
struct BlockGeo {
    int32_t first, bw, h, v, dx, dy;
};

__device__ __forceinline__ int16_t* block_at(const JpegDecScan& s, const BlockGeo* geo, const Out& o, uint32_t j) {
    const BlockGeo& g = geo[j];
    const int64_t bx = (int64_t)o.mx * g.h + g.dx, by = (int64_t)o.my * g.v + g.dy;
    return s.coef + ((size_t)g.first + (size_t)by * (size_t)g.bw + (size_t)bx) * 64;
}

// Decode one symbol.  WRITE: store the DC difference of block o.t, or the
// coefficient into o.blk.  A code that matches no table entry, or a value
// T.81 does not allow there (a DC category above 11, an AC size above 10, a
// run past the block's end), returns false and moves one bit on.  A
// completed block moves to the MCU's next block and counts in `done`.  The
// cases are selects rather than branches: the lanes of a wavefront decode
// different symbols.
template <bool WRITE>
__device__ __forceinline__ bool step(const JpegDecScan& s, const JpegHuffTable* tl, const uint8_t* zz, Dec& d,
                                     const Out& o, uint32_t& done) {
    const uint32_t v = d.peek32();
    const bool dc = d.z == 0;
    const uint32_t sel = dc ? s.dsel : s.asel;
    const JpegHuffTable& t = tl[(dc ? 0u : 4u) + ((sel >> (2 * d.j)) & 3u)];
    uint32_t e = t.fast[v >> (32 - kJpegFastBits)];
    if (e == 0) e = slow_code(t, v >> 16);
    const uint32_t len = e >> 8, sym = e & 255u;
    const uint32_t r = sym >> 4, sz = sym & 15u;
    const bool ok = e != 0 && (dc ? sym <= 11 : (sz == 0 || (d.z + r <= 63 && sz <= 10)));
    const uint32_t nmag = ok ? (dc ? sym : sz) : 0u;
    if (WRITE && ok) {
        const int val = extend(nmag ? (v << len) >> (32 - nmag) : 0u, nmag);
        if (dc)
            s.dcdiff[o.t] = (uint32_t)(val + (int)kJpegDcBias);
        else if (sz)
            o.blk[zz[d.z + r]] = (int16_t)val;
    }
    const uint32_t znew = dc ? 1u : (sz ? d.z + r + 1 : (r == 15 ? d.z + 16 : 64u));
    d.p += ok ? len + nmag : 1u;
    d.z = ok ? znew : d.z;
    if (d.z >= 64) {
        d.z = 0;
        d.j = d.j + 1 == (uint32_t)s.bpm ? 0u : d.j + 1;
        ++done;
    }
    return ok;
}

// Run the decoding until its position reaches `until` (relative), counting
// the blocks it completes (every symbol takes at least one bit).
__device__ __forceinline__ uint32_t run_until(const JpegDecScan& s, const JpegHuffTable* tl, Dec& d,
                                              uint32_t until) {
    uint32_t done = 0;
    Out o;
    while (d.p < until) (void)step<false>(s, tl, nullptr, d, o, done);
    return done;
}

__device__ __forceinline__ int64_t group_first_word(const JpegDecScan& s, int i0) {
    return (int64_t)(s.subs[i0].begin >> 5);
}

// Track u of subsequence i: `group` subsequences per workgroup, 2 x bpm
// threads each.
__global__ __launch_bounds__(256) void k_huff_tracks(JpegDecScan s, int group, int nstage, JpegTrack* tracks) {
    extern __shared__ __align__(16) uint32_t lds[];
    JpegHuffTable* tl = reinterpret_cast<JpegHuffTable*>(lds);
    uint32_t* words = lds + kTableWords;
    const int nt = 2 * s.bpm;
    const int i0 = blockIdx.x * group;
    const int64_t w0 = group_first_word(s, i0);
    stage(s, lds, words, w0, nstage);
    const int g = threadIdx.x / nt, u = threadIdx.x - g * nt;
    const int i = i0 + g;
    if (g >= group || i >= s.nsub) return;
    const JpegSub sub = s.subs[i];
    const uint64_t w0bit = (uint64_t)w0 * 32;
    Dec d;
    d.init(words, w0bit, sub.begin << 16 | (uint64_t)(u >> 1) << 8 | (uint64_t)(u & 1), sub.seg_end);
    JpegTrack t;
    t.pre = run_until(s, tl, d, (uint32_t)(sub.begin + (uint64_t)s.check_bits - w0bit));
    t.check = d.state(w0bit);
    t.post = run_until(s, tl, d, (uint32_t)(sub.end - w0bit));
    t.exit = d.state(w0bit);
    tracks[(int64_t)i * nt + u] = t;
}

// Link from track u of subsequence i into subsequence i + 1 (of the same
// restart interval); the same grouping as the tracks.
__global__ __launch_bounds__(256) void k_huff_links(JpegDecScan s, int group, int nstage, const JpegTrack* tracks,
                                                    JpegLink* links) {
    extern __shared__ __align__(16) uint32_t lds[];
    JpegHuffTable* tl = reinterpret_cast<JpegHuffTable*>(lds);
    uint32_t* words = lds + kTableWords;
    const int nt = 2 * s.bpm;
    const int i0 = blockIdx.x * group;
    const int64_t w0 = group_first_word(s, i0);
    stage(s, lds, words, w0, nstage);
    const int g = threadIdx.x / nt, u = threadIdx.x - g * nt;
    const int i = i0 + g;
    if (g >= group || i >= s.nsub) return;
    const int64_t idx = (int64_t)i * nt + u;
    JpegLink l;
    l.next = kJpegNoTrack;
    l.blocks = 0;
    if (!(s.subs[i].flags & 2)) {
        const JpegSub nx = s.subs[i + 1];
        const uint64_t w0bit = (uint64_t)w0 * 32;
        Dec d;
        d.init(words, w0bit, tracks[idx].exit, nx.seg_end);
        l.blocks = run_until(s, tl, d, (uint32_t)(nx.begin + (uint64_t)s.check_bits - w0bit));
        const uint64_t e = d.state(w0bit);
        const JpegTrack* next = tracks + (int64_t)(i + 1) * nt;
        for (int v = 0; v < nt; ++v)
            if (next[v].check == e) {
                l.next = (uint32_t)v;
                break;
            }
    }
    links[idx] = l;
}

// The decoding proper: two threads per subsequence (its two parts), `group`
// subsequences per workgroup, each part from its true start state and block.
// An interval's last subsequence decodes until the interval's blocks are
// complete, reading zero bits past its data as a truncated interval does.
__global__ __launch_bounds__(256) void k_huff_decode(JpegDecScan s, int group, int nstage, const JpegEntry* entries,
                                                     uint32_t* malformed) {
    extern __shared__ __align__(16) uint32_t lds[];
    JpegHuffTable* tl = reinterpret_cast<JpegHuffTable*>(lds);
    BlockGeo* geo = reinterpret_cast<BlockGeo*>(lds + kTableWords);
    uint8_t* zz = reinterpret_cast<uint8_t*>(geo + kJpegMaxMcuBlocks);
    uint32_t* words = reinterpret_cast<uint32_t*>(zz + 64);
    const int i0 = blockIdx.x * group;
    const int64_t w0 = group_first_word(s, i0);
    if (threadIdx.x < (unsigned)s.bpm) {
        const int j = threadIdx.x, c = s.comp[j];
        geo[j].first = s.first[c];
        geo[j].bw = s.bw[c];
        geo[j].h = s.h[c];
        geo[j].v = s.v[c];
        geo[j].dx = s.dx[j];
        geo[j].dy = s.dy[j];
    }
    if (threadIdx.x < 64) zz[threadIdx.x] = kZzDec[threadIdx.x];
    stage(s, lds, words, w0, nstage);
    const int i = i0 + (int)(threadIdx.x >> 1);
    if ((int)(threadIdx.x >> 1) >= group || i >= s.nsub) return;
    const JpegEntry en = entries[2 * (int64_t)i + (threadIdx.x & 1)];
    if (en.block < 0) return;
    const JpegSub sub = s.subs[i];
    const JpegSeg seg = s.segs[sub.seg];
    const bool to_blocks = en.stop == kJpegStopAtBlocks;
    const uint64_t w0bit = (uint64_t)w0 * 32;
    Dec d;
    d.init(words, w0bit, en.state, sub.seg_end);
    const uint32_t stop = to_blocks ? 0xFFFFFFFFu : (uint32_t)(en.stop - w0bit);
    Out o;
    o.t = en.block;
    {
        const uint32_t mcu = (uint32_t)(o.t / s.bpm);
        o.mx = (int32_t)(mcu % (uint32_t)s.mcux);
        o.my = (int32_t)(mcu / (uint32_t)s.mcux);
    }
    o.blk = o.t < seg.end_block ? block_at(s, geo, o, d.j) : nullptr;
    // the part's bits, or the symbols of the interval's remaining blocks (at
    // most 64 each) past the subsequence's own bits
    const uint32_t lim = to_blocks ? (uint32_t)(sub.end - w0bit) : stop;
    uint64_t budget = (d.p < lim ? lim - d.p : 0) + 64;
    if (to_blocks && o.t < seg.end_block) budget += 65 * (uint64_t)(seg.end_block - o.t);
    uint32_t done = 0;
    while (o.t < seg.end_block && d.p < stop) {
        if (budget-- == 0 || !step<true>(s, tl, zz, d, o, done)) {
            atomicOr(malformed, 1u);
            return;
        }
        if (d.z == 0) {  // the block is complete; d.j is the next block of the MCU
            ++o.t;
            if (d.j == 0 && ++o.mx == s.mcux) {
                o.mx = 0;
                ++o.my;
            }
            o.blk = o.t < seg.end_block ? block_at(s, geo, o, d.j) : nullptr;
        }
    }
}

// Scan component k's DC differences in its own order: element e of k (its
// e-th block in scan order) at g = mcus x off[k] + e.
__device__ __forceinline__ int comp_of_element(const JpegDecScan& s, int64_t g) {
    int k = 0;
    while (k + 1 < s.ns && g >= s.mcus * s.off[k + 1]) ++k;
    return k;
}
__device__ __forceinline__ int64_t scan_block_of(const JpegDecScan& s, int k, int64_t e) {
    return (e / s.nb[k]) * s.bpm + s.off[k] + e % s.nb[k];
}

__global__ __launch_bounds__(256) void k_dc_gather(JpegDecScan s, uint32_t* seq) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= s.blocks) return;
    const int k = comp_of_element(s, g);
    seq[g] = s.dcdiff[scan_block_of(s, k, g - s.mcus * s.off[k])];
}

// DC of every block: its component's differences summed from the start of
// its restart interval (x: exclusive prefix sums of seq, biased values).
__global__ __launch_bounds__(256) void k_dc_finish(JpegDecScan s, const uint32_t* seq, const uint64_t* x) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= s.blocks) return;
    const int k = comp_of_element(s, g);
    const int64_t e = g - s.mcus * s.off[k];
    const int64_t mcu = e / s.nb[k];
    const int64_t m0 = s.restart ? mcu / s.restart * s.restart : 0;
    const int64_t g0 = s.mcus * s.off[k] + m0 * s.nb[k];
    const int64_t sum = (int64_t)(x[g] + seq[g] - x[g0]) - (int64_t)kJpegDcBias * (g - g0 + 1);
    const int64_t t = scan_block_of(s, k, e);
    const int64_t m = t / s.bpm;
    const int j = (int)(t - m * s.bpm), c = s.comp[j];
    const int64_t bx = (m % s.mcux) * s.h[c] + s.dx[j], by = (m / s.mcux) * s.v[c] + s.dy[j];
    s.coef[((size_t)s.first[c] + (size_t)by * (size_t)s.bw[c] + (size_t)bx) * 64] = (int16_t)sum;
}

}  // namespace

hipError_t launch_huff_tracks(const JpegDecScan& s, int sub_bits, JpegTrack* tracks, JpegLink* links,
                              hipEvent_t tracks_done, hipStream_t stream) {
    if (s.nsub <= 0) return hipSuccess;
    const int nt = 2 * s.bpm;
    const int group = group_subs(nt, sub_bits);
    const int nstage = stage_words(group, sub_bits, s.check_bits);
    const size_t lds = (size_t)(kTableWords + nstage) * 4;
    const dim3 g((unsigned)((s.nsub + group - 1) / group));
    hipLaunchKernelGGL(k_huff_tracks, g, dim3(256), lds, stream, s, group, nstage, tracks);
    if (tracks_done && note_hip("hipEventRecord", hipEventRecord(tracks_done, stream)) != hipSuccess)
        return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_huff_links, g, dim3(256), lds, stream, s, group, nstage, (const JpegTrack*)tracks, links);
    return note_hip("k_huff_links launch", hipGetLastError());
}

hipError_t launch_huff_decode(const JpegDecScan& s, int sub_bits, const JpegEntry* entries, uint32_t* malformed,
                              uint64_t* tiles, uint64_t* total, uint32_t* dcseq, uint64_t* dcsum, hipStream_t stream) {
    if (s.nsub <= 0 || s.blocks <= 0) return hipSuccess;
    // one wavefront of parts per workgroup, spread over more CUs (four per
    // workgroup: 90.5 us at 1920x1080, one: 77.2)
    const int group = std::min(group_subs(2, sub_bits), 32);
    const int nstage = stage_words(group, sub_bits, 0);
    const size_t lds = (size_t)kTableWords * 4 + kJpegMaxMcuBlocks * sizeof(BlockGeo) + 64 + (size_t)nstage * 4;
    hipLaunchKernelGGL(k_huff_decode, dim3((unsigned)((s.nsub + group - 1) / group)), dim3(256), lds, stream, s, group,
                       nstage, entries, malformed);
    const dim3 g((unsigned)((s.blocks + 255) / 256));
    hipLaunchKernelGGL(k_dc_gather, g, dim3(256), 0, stream, s, dcseq);
    if (launch_exclusive_scan(dcseq, s.blocks, tiles, total, dcsum, stream) != hipSuccess)
        return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_dc_finish, g, dim3(256), 0, stream, s, (const uint32_t*)dcseq, (const uint64_t*)dcsum);
    return note_hip("k_dc_finish launch", hipGetLastError());
}

}  // namespace oilpaint_impl
