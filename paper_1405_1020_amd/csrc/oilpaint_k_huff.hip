// Huffman coding of the encoder's scan on the GPU (T.81 F.1.2: DC
// differences and run/size symbols of the zig-zag coefficients, codes from
// tables fitted to the image per K.2; B.1.1.5: a zero byte after every 0xFF
// of the entropy-coded data).  The host fits the tables between the
// statistics pass and the coding passes; everything per block runs here.
//
// A wavefront works one 8 x 8 block at a time, lane k holding the k-th
// coefficient of the zig-zag sequence, over a grid sized to the GPU (each
// wavefront loads its next block while it codes the current one): the
// nonzero AC coefficients come from one ballot; lane k
// finds the zero run before it from the highest set bit below k, so every
// symbol of the block is known at once.  A lane's bits (its ZRL codes, its
// run/size code and its magnitude; lane 0: the DC code and magnitude) are
// placed by a prefix sum over the lanes, the block's own start by a prefix
// sum over the blocks, and written into 32-bit words (the first bit of the
// stream the most significant bit of word 0) with OR atomics, since a word
// may hold the tail of one code and the head of the next.  Byte stuffing is
// a count of 0xFF bytes per tile, a prefix sum and a scatter.
#include <algorithm>

#include "oilpaint_internal.h"
#include "oilpaint_jpeg.h"

namespace oilpaint_impl {
namespace {

// Zig-zag order (T.81 Figure A.6): the natural index of the k-th coefficient.
__constant__ uint8_t kZz[64] = {0,  1,  8,  16, 9,  2,  3,  10, 17, 24, 32, 25, 18, 11, 4,  5,
                                12, 19, 26, 33, 40, 48, 41, 34, 27, 20, 13, 6,  7,  14, 21, 28,
                                35, 42, 49, 56, 57, 50, 43, 36, 29, 22, 15, 23, 30, 37, 44, 51,
                                58, 59, 52, 45, 38, 31, 39, 46, 53, 60, 61, 54, 47, 55, 62, 63};

constexpr int kScanTile = 4096;  // elements per tile of the prefix sums (256 threads x 16)

// Size category of a DC difference or AC value (T.81 F.1.2.1.1): the bit
// length of |v|.
__device__ __forceinline__ uint32_t category(int v) {
    const uint32_t a = (uint32_t)(v < 0 ? -v : v);
    return a ? 32u - (uint32_t)__clz((int)a) : 0u;
}

// Magnitude bits of v in category s: v itself, or v - 1 for negative v (its
// low s bits), T.81 F.1.2.1.1.
__device__ __forceinline__ uint32_t magnitude(int v, uint32_t s) {
    return s ? ((uint32_t)(v < 0 ? v - 1 : v) & ((1u << s) - 1u)) : 0u;
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
template <typename T>
__device__ __forceinline__ T wave_scan(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// The same for 32-bit values with DPP row shifts and broadcasts (no LDS
// round trips).  Every lane must be active.
__device__ __forceinline__ uint32_t wave_scan32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// Exclusive prefix sum over the 256 threads of a workgroup (four
// wavefronts); `tot` receives the workgroup's sum.  Every thread calls it.
template <typename T>
__device__ __forceinline__ T group_scan(T v, T* lds4, T& tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const T inc = wave_scan(v);
    if (lane == 63) lds4[w] = inc;
    __syncthreads();
    T before = 0;
    tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const T s = lds4[i];
        before += i < w ? s : (T)0;
        tot += s;
    }
    __syncthreads();
    return before + inc - v;
}

// The block at position t of the scan: its coefficients and those of the
// previous block of the same component (the DC predictor), or nullptr for
// the component's first block.
struct BlockRef {
    const int16_t* coef;
    const int16_t* pred;
    int tab;
};

__device__ __forceinline__ BlockRef block_at(const JpegScanMap& m, const int16_t* coef, int64_t t) {
    const int64_t mcu = t / m.bpm;
    const int j = (int)(t - mcu * m.bpm);
    const int c = m.comp[j];
    auto index = [&](int64_t mc, int jj) {
        const int64_t mx = mc % m.mcux, my = mc / m.mcux;
        const int64_t bx = mx * m.h[c] + m.dx[jj], by = my * m.v[c] + m.dy[jj];
        return (int64_t)m.first[c] + by * m.bw[c] + bx;
    };
    BlockRef r;
    r.coef = coef + (size_t)index(mcu, j) * 64;
    r.tab = m.tab[c];
    if (m.prev[j] >= 0)
        r.pred = coef + (size_t)index(mcu, m.prev[j]) * 64;
    else if (mcu > 0)
        r.pred = coef + (size_t)index(mcu - 1, m.last[c]) * 64;
    else
        r.pred = nullptr;
    return r;
}

// What a lane needs of block t: its zig-zag coefficient (natural index zz),
// the DC predictor (0 for the component's first block) and the table set.
struct BlockVals {
    int v, pred, tab;
};

__device__ __forceinline__ BlockVals load_block(const JpegScanMap& m, const int16_t* coef, int64_t t, int zz) {
    const BlockRef b = block_at(m, coef, t);
    BlockVals r;
    r.v = b.coef[zz];
    r.pred = b.pred ? (int)b.pred[0] : 0;
    r.tab = b.tab;
    return r;
}

// The symbols of one block, lane k for zig-zag position k:
//   lane 0: the DC category `cat` (of the difference `val`), and whether the
//     block ends with an EOB (its last AC coefficient is 0);
//   lane k >= 1 with a nonzero coefficient: `zrl` ZRL codes, then the
//     run/size symbol `sym` and the value's category `cat`.
struct LaneSym {
    int val;
    uint32_t cat, sym, zrl;
    bool live, eob;
};

__device__ __forceinline__ LaneSym lane_symbols(const BlockVals& b) {
    const int k = threadIdx.x & 63;
    LaneSym s;
    const int v = b.v;
    const uint64_t nz = __ballot(k > 0 && v != 0);
    if (k == 0) {
        s.val = v - b.pred;
        s.cat = category(s.val);
        s.sym = s.cat;
        s.zrl = 0;
        s.live = true;
        s.eob = (nz >> 63) == 0;
    } else {
        const uint64_t below = nz & ((1ull << k) - 1ull);
        const int prev = below ? 63 - __clzll((long long)below) : 0;
        const uint32_t run = (uint32_t)(k - prev - 1);
        s.val = v;
        s.cat = category(v);
        s.sym = (run & 15u) << 4 | s.cat;
        s.zrl = run >> 4;
        s.live = v != 0;
        s.eob = false;
    }
    return s;
}

// Symbol statistics: a persistent grid, one wavefront per block in turn,
// counts in LDS (DC luminance, DC chrominance, AC luminance, AC
// chrominance: 256 each), added to the device totals at the end.
__global__ __launch_bounds__(1024) void k_huff_stats(JpegScanMap m, const int16_t* coef,
                                                     unsigned long long* freq) {
    __shared__ uint32_t h[4 * 256];
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int zz = kZz[lane];
    const int waves = blockDim.x >> 6;
    const int64_t stride = (int64_t)gridDim.x * waves;
    int64_t t = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6);
    BlockVals next{};
    if (t < m.blocks) next = load_block(m, coef, t, zz);
    for (; t < m.blocks; t += stride) {
        const BlockVals b = next;
        if (t + stride < m.blocks) next = load_block(m, coef, t + stride, zz);
        const LaneSym s = lane_symbols(b);
        uint32_t* dc = h + b.tab * 256;
        uint32_t* ac = h + (2 + b.tab) * 256;
        if (lane == 0) {
            atomicAdd(dc + s.cat, 1u);
            if (s.eob) atomicAdd(ac + 0x00, 1u);
        } else if (s.live) {
            if (s.zrl) atomicAdd(ac + 0xF0, s.zrl);
            atomicAdd(ac + s.sym, 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x)
        if (h[i]) atomicAdd(freq + i, (unsigned long long)h[i]);
}

// The code tables (size << 16 | code per symbol; 0-3 as above) into LDS.
__device__ __forceinline__ void load_tables(const uint32_t* tabs, uint32_t* lds) {
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) lds[i] = tabs[i];
    __syncthreads();
}

// Bits a lane contributes (lane 0: its DC code and magnitude, not the EOB).
__device__ __forceinline__ uint32_t lane_bits(const LaneSym& s, const uint32_t* dc, const uint32_t* ac) {
    const int lane = threadIdx.x & 63;
    if (lane == 0) return (dc[s.cat] >> 16) + s.cat;
    if (!s.live) return 0;
    return s.zrl * (ac[0xF0] >> 16) + (ac[s.sym] >> 16) + s.cat;
}

// Bits of every block.
__global__ __launch_bounds__(256) void k_huff_bits(JpegScanMap m, const int16_t* coef, const uint32_t* tabs,
                                                   uint32_t* bits) {
    __shared__ uint32_t tl[4 * 256];
    load_tables(tabs, tl);
    const int lane = threadIdx.x & 63;
    const int zz = kZz[lane];
    const int64_t stride = (int64_t)gridDim.x * 4;
    int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    BlockVals next{};
    if (t < m.blocks) next = load_block(m, coef, t, zz);
    for (; t < m.blocks; t += stride) {
        const BlockVals b = next;
        if (t + stride < m.blocks) next = load_block(m, coef, t + stride, zz);
        const LaneSym s = lane_symbols(b);
        const uint32_t* dc = tl + b.tab * 256;
        const uint32_t* ac = tl + (2 + b.tab) * 256;
        uint32_t n = lane_bits(s, dc, ac);
        if (lane == 0 && s.eob) n += ac[0x00] >> 16;
        n = wave_scan32(n);
        if (lane == 63) bits[t] = n;
    }
}

// OR `len` (<= 32) bits of `val` into the stream at bit `pos`.
__device__ __forceinline__ void put_bits(uint32_t* words, uint64_t pos, uint32_t val, uint32_t len) {
    if (len == 0) return;
    const uint64_t w = pos >> 5;
    const uint32_t b = (uint32_t)(pos & 31);
    const uint64_t v = (uint64_t)(val & (len == 32 ? 0xFFFFFFFFu : ((1u << len) - 1u))) << (64 - b - len);
    const uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
    if (hi) atomicOr(words + w, hi);
    if (lo) atomicOr(words + w + 1, lo);
}

// The bits of every block at its offset (exclusive prefix sum of the block
// sizes).
__global__ __launch_bounds__(256) void k_huff_write(JpegScanMap m, const int16_t* coef, const uint32_t* tabs,
                                                    const uint64_t* offset, uint32_t* words) {
    __shared__ uint32_t tl[4 * 256];
    load_tables(tabs, tl);
    const int lane = threadIdx.x & 63;
    const int zz = kZz[lane];
    const int64_t stride = (int64_t)gridDim.x * 4;
    int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    BlockVals next{};
    uint64_t next_off = 0;
    if (t < m.blocks) {
        next = load_block(m, coef, t, zz);
        next_off = offset[t];
    }
    for (; t < m.blocks; t += stride) {
        const BlockVals b = next;
        const uint64_t off = next_off;
        if (t + stride < m.blocks) {
            next = load_block(m, coef, t + stride, zz);
            next_off = offset[t + stride];
        }
        const LaneSym s = lane_symbols(b);
        const uint32_t* dc = tl + b.tab * 256;
        const uint32_t* ac = tl + (2 + b.tab) * 256;
        const uint32_t n = lane_bits(s, dc, ac);
        const uint32_t inc = wave_scan32(n);
        uint64_t pos = off + (inc - n);
        if (lane == 0) {
            const uint32_t e = dc[s.cat];
            put_bits(words, pos, (e & 0xFFFFu) << s.cat | magnitude(s.val, s.cat), (e >> 16) + s.cat);
        }
        const uint32_t body = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);  // the block's bits before its EOB
        if (lane == 0 && s.eob) {
            const uint32_t e = ac[0x00];
            put_bits(words, off + body, e & 0xFFFFu, e >> 16);
        }
        if (lane > 0 && s.live) {
            const uint32_t z = ac[0xF0];
            for (uint32_t i = 0; i < s.zrl; ++i) {
                put_bits(words, pos, z & 0xFFFFu, z >> 16);
                pos += z >> 16;
            }
            const uint32_t e = ac[s.sym];
            put_bits(words, pos, (e & 0xFFFFu) << s.cat | magnitude(s.val, s.cat), (e >> 16) + s.cat);
        }
    }
}

// Byte i of the stream (total bits `nbits`; the last byte padded with one
// bits, T.81 F.1.2.3).
__device__ __forceinline__ uint32_t stream_byte(const uint32_t* words, uint64_t nbits, uint64_t i) {
    uint32_t byte = (words[i >> 2] >> (24 - 8 * (uint32_t)(i & 3))) & 0xFFu;
    const uint64_t nbytes = (nbits + 7) >> 3;
    if (i + 1 == nbytes && (nbits & 7)) byte |= 0xFFu >> (nbits & 7);
    return byte;
}

// 0xFF bytes per tile of kScanTile bytes.
__global__ __launch_bounds__(256) void k_ff_count(const uint32_t* words, uint64_t nbits, uint64_t* tiles) {
    __shared__ uint32_t s4[4];
    const uint64_t nbytes = (nbits + 7) >> 3;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * 16;
    uint32_t n = 0;
    for (int i = 0; i < 16; ++i)
        if (base + i < nbytes) n += stream_byte(words, nbits, base + i) == 0xFFu;
    uint32_t tot;
    (void)group_scan(n, s4, tot);
    if (threadIdx.x == 0) tiles[blockIdx.x] = tot;
}

// The stuffed stream: byte i at i + (0xFF bytes before it), a zero after
// every 0xFF.
__global__ __launch_bounds__(256) void k_ff_scatter(const uint32_t* words, uint64_t nbits, const uint64_t* tiles,
                                                    uint8_t* out) {
    __shared__ uint32_t s4[4];
    const uint64_t nbytes = (nbits + 7) >> 3;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * 16;
    uint32_t by[16];
    uint32_t n = 0;
    for (int i = 0; i < 16; ++i) {
        by[i] = base + i < nbytes ? stream_byte(words, nbits, base + i) : 0u;
        n += base + i < nbytes && by[i] == 0xFFu;
    }
    uint32_t tot;
    uint64_t o = base + tiles[blockIdx.x] + group_scan(n, s4, tot);
    for (int i = 0; i < 16; ++i) {
        if (base + i >= nbytes) break;
        out[o++] = (uint8_t)by[i];
        if (by[i] == 0xFFu) out[o++] = 0;
    }
}

// Prefix sums of n 32-bit values into 64-bit offsets, in three passes:
// tile sums, an exclusive scan of the tile sums (one workgroup), and the
// scan within each tile.
__global__ __launch_bounds__(256) void k_tile_sums(const uint32_t* in, int64_t n, uint64_t* tiles) {
    __shared__ uint64_t s4[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * 16;
    uint64_t v = 0;
    for (int i = 0; i < 16; ++i)
        if (base + i < n) v += in[base + i];
    uint64_t tot;
    (void)group_scan(v, s4, tot);
    if (threadIdx.x == 0) tiles[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_tiles(uint64_t* tiles, int64_t n, uint64_t* total) {
    __shared__ uint64_t s4[4];
    uint64_t carry = 0;
    for (int64_t b = 0; b < n; b += 256) {
        const int64_t i = b + threadIdx.x;
        const uint64_t v = i < n ? tiles[i] : 0;
        uint64_t tot;
        const uint64_t ex = group_scan(v, s4, tot);
        if (i < n) tiles[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void k_tile_scan(const uint32_t* in, int64_t n, const uint64_t* tiles,
                                                   uint64_t* out) {
    __shared__ uint64_t s4[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * 16;
    uint32_t v[16];
    uint64_t sum = 0;
    for (int i = 0; i < 16; ++i) {
        v[i] = base + i < n ? in[base + i] : 0u;
        sum += v[i];
    }
    uint64_t tot;
    uint64_t o = tiles[blockIdx.x] + group_scan(sum, s4, tot);
    for (int i = 0; i < 16; ++i) {
        if (base + i >= n) break;
        out[base + i] = o;
        o += v[i];
    }
}

int64_t tiles_of(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

}  // namespace

int64_t huff_scan_tiles(int64_t n) { return tiles_of(n); }

hipError_t launch_huff_stats(const JpegScanMap& m, const int16_t* coef, unsigned long long* freq, int cus,
                             hipStream_t stream) {
    if (m.blocks <= 0) return hipSuccess;
    const int64_t want = (m.blocks + 63) / 64;  // at least 4 blocks per wavefront
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)std::max(cus, 1)));
    hipLaunchKernelGGL(k_huff_stats, dim3(grid), dim3(1024), 0, stream, m, coef, freq);
    return note_hip("k_huff_stats launch", hipGetLastError());
}

hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint64_t* tiles, uint64_t* total, uint64_t* out,
                                 hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t nt = tiles_of(n);
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nt), dim3(256), 0, stream, in, n, tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(256), 0, stream, tiles, nt, total);
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)nt), dim3(256), 0, stream, in, n, tiles, out);
    return note_hip("k_tile_scan launch", hipGetLastError());
}

hipError_t launch_huff_code(const JpegScanMap& m, const int16_t* coef, const uint32_t* tabs, uint32_t* bits,
                            uint64_t* offset, uint64_t* tiles, uint64_t* total, uint32_t* words, int cus,
                            hipStream_t stream) {
    if (m.blocks <= 0) return hipSuccess;
    // eight workgroups of four wavefronts per CU, each wavefront a few blocks
    const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((m.blocks + 3) / 4, 8 * (int64_t)std::max(cus, 1))));
    hipLaunchKernelGGL(k_huff_bits, g, dim3(256), 0, stream, m, coef, tabs, bits);
    if (launch_exclusive_scan(bits, m.blocks, tiles, total, offset, stream) != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_huff_write, g, dim3(256), 0, stream, m, coef, tabs, offset, words);
    return note_hip("k_huff_write launch", hipGetLastError());
}

hipError_t launch_huff_stuff(const uint32_t* words, uint64_t nbits, uint64_t* tiles, uint64_t* ff_total,
                             uint8_t* out, hipStream_t stream) {
    const int64_t nbytes = (int64_t)((nbits + 7) >> 3);
    if (nbytes <= 0) return hipSuccess;
    const int64_t nt = tiles_of(nbytes);
    hipLaunchKernelGGL(k_ff_count, dim3((unsigned)nt), dim3(256), 0, stream, words, nbits, tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(256), 0, stream, tiles, nt, ff_total);
    hipLaunchKernelGGL(k_ff_scatter, dim3((unsigned)nt), dim3(256), 0, stream, words, nbits, tiles, out);
    return note_hip("k_ff_scatter launch", hipGetLastError());
}

}  // namespace oilpaint_impl
