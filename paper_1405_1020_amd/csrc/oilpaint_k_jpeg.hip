// Device steps of the JPEG codec around the filter: dequantization and the
// 8 x 8 inverse DCT (T.81 A.3.3, A.3.5), JFIF colour conversion with chroma
// replication (decode); JFIF colour conversion with chroma averaging, the
// forward DCT and quantization (T.81 A.3.3, A.3.4) (encode).  Eight lanes
// per 8 x 8 block, eight blocks per wavefront: a lane transforms one row of
// its block in registers, the rows meet through LDS, and the lane then
// transforms one column; colour conversion one lane per pixel.  Huffman
// decoding runs in oilpaint_k_huffdec.hip, the encoder's Huffman coding in
// oilpaint_k_huff.hip.
#include "oilpaint_internal.h"
#include "oilpaint_jpeg.h"

namespace oilpaint_impl {
namespace {

// cos(m pi / 16) / sqrt(2), m = 0..8.
constexpr float kCosR2[9] = {
    0.70710678118654752f, 0.69351992266107906f, 0.65328148243818826f, 0.58794459036236287f,
    0.50000000000000000f, 0.39284747919355110f, 0.27059805007309849f, 0.13794968964147150f,
    0.0f};

// sqrt(2) x C(u)/2 x cos((2x+1) u pi / 16): exactly 1/2 for u = 0 and +-1/2
// for u = 4, so that blocks whose exact transform is rational (flat blocks,
// the u, v in {0, 4} terms) come out exact in fp32; the transform is this
// basis applied twice, then halved.  Evaluated at compile time: the loops
// below are unrolled, so every basis value is an immediate operand.
constexpr float basis(int u, int x) {
    if (u == 0) return 0.5f;
    const int m = ((2 * x + 1) * u) & 31;
    if (m <= 8) return kCosR2[m];
    if (m <= 16) return -kCosR2[16 - m];
    if (m <= 24) return -kCosR2[m - 16];
    return kCosR2[32 - m];
}

__device__ __forceinline__ int comp_of(const int32_t* first, int b) {
    int c = 0;
    while (c + 1 < kJpegMaxComps && b >= first[c + 1]) ++c;
    return c;
}

// Workgroup: four wavefronts of eight blocks; lane = (block, i): row i in the
// first pass, column i in the second.  The rows' results go through LDS
// (rows of 9 floats: a column read touches eight banks); each wavefront
// works its own blocks, so program order keeps its LDS accesses in order.
constexpr int kDctBlocksPerGroup = 32;
constexpr int kDctPitch = 9;

// Inverse: t[v][x] = sum_u S[v][u] B[u][x] (row v), s[y][x] = sum_v B[v][y]
// t[v][x] (column x), each sum accumulated in index order; sample =
// floor(clamp(s / 2 + 128.5)).
__global__ __launch_bounds__(256) void k_jpeg_idct(JpegIdctArgs a) {
    __shared__ float s_t[kDctBlocksPerGroup][8 * kDctPitch];
    const int lane = threadIdx.x & 63;
    const int lb = (int)(threadIdx.x >> 3);  // block within the workgroup
    const int i = lane & 7;
    const int total = a.first[kJpegMaxComps];
    const int b = blockIdx.x * kDctBlocksPerGroup + lb;
    const bool live = b < total;
    const int c = live ? comp_of(a.first, b) : 0;
    float* t = s_t[lb];
    {
        float S[8];
        if (live) {
            const uint4 raw = *reinterpret_cast<const uint4*>(a.coef + (size_t)b * 64 + i * 8);
            const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int coef = (int)(int16_t)(w[u >> 1] >> (16 * (u & 1)));
                S[u] = (float)(coef * (int)a.q[c][i * 8 + u]);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) S[u] = 0.f;
        }
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            float acc = 0.f;
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = fmaf(S[u], basis(u, x), acc);
            t[i * kDctPitch + x] = acc;
        }
    }
    asm volatile("" ::: "memory");
    float tv[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) tv[v] = t[v * kDctPitch + i];
    if (!live) return;
    const int k = b - a.first[c];
    const int by = k / a.bw[c], bx = k - by * a.bw[c];
    const int x = bx * 8 + i;
    if (x >= a.limit_w[c]) return;
#pragma unroll
    for (int yy = 0; yy < 8; ++yy) {
        float s = 0.f;
#pragma unroll
        for (int v = 0; v < 8; ++v) s = fmaf(basis(v, yy), tv[v], s);
        const int y = by * 8 + yy;
        const int val = (int)floorf(fminf(fmaxf(s * 0.5f + 128.5f, 0.f), 255.f));
        if (y < a.limit_h[c]) a.plane[c][(size_t)y * a.stride[c] + x] = (uint8_t)val;
    }
}

// R = Y + 1.402 Cr', G = Y - 0.344136 Cb' - 0.714136 Cr', B = Y + 1.772 Cb'
// (Cb' = Cb - 128, Cr' = Cr - 128) in integers scaled by 10^6, rounded half
// up: every numerator is offset by 256 x 10^6 to stay positive, so integer
// division floors.
__global__ __launch_bounds__(256) void k_jpeg_color(JpegColorArgs a) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= a.width) return;
    const int Y = a.plane[0][(size_t)(y * a.v[0] / a.vmax) * a.stride[0] + x * a.h[0] / a.hmax];
    uint8_t* d = a.dst + (size_t)y * a.dst_stride + 3 * x;
    if (a.ncomp == 1) {
        d[0] = d[1] = d[2] = (uint8_t)Y;
        return;
    }
    const int cb = (int)a.plane[1][(size_t)(y * a.v[1] / a.vmax) * a.stride[1] + x * a.h[1] / a.hmax] - 128;
    const int cr = (int)a.plane[2][(size_t)(y * a.v[2] / a.vmax) * a.stride[2] + x * a.h[2] / a.hmax] - 128;
    constexpr int M = 1000000, OFF = 256 * M;
    const int R = Y + (1402000 * cr + M / 2 + OFF) / M - 256;
    const int G = Y + (-344136 * cb - 714136 * cr + M / 2 + OFF) / M - 256;
    const int B = Y + (1772000 * cb + M / 2 + OFF) / M - 256;
    d[0] = (uint8_t)min(255, max(0, R));
    d[1] = (uint8_t)min(255, max(0, G));
    d[2] = (uint8_t)min(255, max(0, B));
}

// One lane per chroma sample: its fh x fv luma-grid pixels (the image's last
// column and row repeated beyond its edge) give fh x fv Y samples and one
// averaged Cb and Cr.  Y = 0.299 R + 0.587 G + 0.114 B, Cb = -0.168736 R -
// 0.331264 G + 0.5 B + 128, Cr = 0.5 R - 0.418688 G - 0.081312 B + 128, in
// integers scaled by 10^6 (every numerator is non-negative), rounded half up.
__global__ __launch_bounds__(256) void k_jpeg_rgb(JpegRgbArgs a) {
    const int cw = a.ymcu_w / a.fh;
    const int cx = blockIdx.x * 256 + threadIdx.x;
    const int cy = blockIdx.y;
    if (cx >= cw) return;
    constexpr int M = 1000000;
    int scb = 0, scr = 0;
    for (int j = 0; j < a.fv; ++j) {
        const int y = cy * a.fv + j;
        const int sy = min(y, a.height - 1);
        for (int i = 0; i < a.fh; ++i) {
            const int x = cx * a.fh + i;
            const int sx = min(x, a.width - 1);
            const uint8_t* p = a.src + (size_t)sy * a.stride + 3 * sx;
            const int R = p[0], G = p[1], B = p[2];
            const int Y = (299000 * R + 587000 * G + 114000 * B + M / 2) / M;
            const int Cb = min(255, (-168736 * R - 331264 * G + 500000 * B + 128 * M + M / 2) / M);
            const int Cr = min(255, (500000 * R - 418688 * G - 81312 * B + 128 * M + M / 2) / M);
            a.plane[0][(size_t)y * a.pstride[0] + x] = (uint8_t)min(255, Y);
            scb += Cb;
            scr += Cr;
        }
    }
    const int n = a.fh * a.fv;
    a.plane[1][(size_t)cy * a.pstride[1] + cx] = (uint8_t)((scb + n / 2) / n);
    a.plane[2][(size_t)cy * a.pstride[2] + cx] = (uint8_t)((scr + n / 2) / n);
}

// Forward: t[y][u] = sum_x s[y][x] B[u][x] (row y), S[v][u] = sum_y B[v][y]
// t[y][u] (column u), each sum accumulated in index order; quantized
// coefficient = round half away from zero of S / 2 / Q.
__global__ __launch_bounds__(256) void k_jpeg_fdct(JpegFdctArgs a) {
    __shared__ float s_t[kDctBlocksPerGroup][8 * kDctPitch];
    const int lane = threadIdx.x & 63;
    const int lb = (int)(threadIdx.x >> 3);
    const int i = lane & 7;
    const int total = a.first[kJpegMaxComps];
    const int b = blockIdx.x * kDctBlocksPerGroup + lb;
    const bool live = b < total;
    const int c = live ? comp_of(a.first, b) : 0;
    float* t = s_t[lb];
    {
        float sm[8];
        if (live) {
            const int k = b - a.first[c];
            const int by = k / a.bw[c], bx = k - by * a.bw[c];
            const uint8_t* row = a.plane[c] + (size_t)(by * 8 + i) * a.stride[c] + bx * 8;
#pragma unroll
            for (int x = 0; x < 8; ++x) sm[x] = (float)((int)row[x] - 128);
        } else {
#pragma unroll
            for (int x = 0; x < 8; ++x) sm[x] = 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            float acc = 0.f;
#pragma unroll
            for (int x = 0; x < 8; ++x) acc = fmaf(sm[x], basis(u, x), acc);
            t[i * kDctPitch + u] = acc;
        }
    }
    asm volatile("" ::: "memory");
    float ty[8];
#pragma unroll
    for (int y = 0; y < 8; ++y) ty[y] = t[y * kDctPitch + i];
    if (!live) return;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        float S = 0.f;
#pragma unroll
        for (int y = 0; y < 8; ++y) S = fmaf(basis(v, y), ty[y], S);
        const float q = S * 0.5f / (float)a.q[c][v * 8 + i];
        const float m = floorf(fabsf(q) + 0.5f);
        a.coef[(size_t)b * 64 + v * 8 + i] = (int16_t)(q < 0.f ? -m : m);
    }
}

}  // namespace

hipError_t launch_jpeg_idct(const JpegIdctArgs& a, hipStream_t stream) {
    const int total = a.first[kJpegMaxComps];
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jpeg_idct, dim3((total + kDctBlocksPerGroup - 1) / kDctBlocksPerGroup), dim3(256), 0,
                       stream, a);
    return note_hip("k_jpeg_idct launch", hipGetLastError());
}

hipError_t launch_jpeg_color(const JpegColorArgs& a, hipStream_t stream) {
    if (a.width <= 0 || a.height <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jpeg_color, dim3((a.width + 255) / 256, a.height), dim3(256), 0, stream, a);
    return note_hip("k_jpeg_color launch", hipGetLastError());
}

hipError_t launch_jpeg_rgb(const JpegRgbArgs& a, hipStream_t stream) {
    const int cw = a.ymcu_w / a.fh, ch = a.ymcu_h / a.fv;
    if (cw <= 0 || ch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jpeg_rgb, dim3((cw + 255) / 256, ch), dim3(256), 0, stream, a);
    return note_hip("k_jpeg_rgb launch", hipGetLastError());
}

hipError_t launch_jpeg_fdct(const JpegFdctArgs& a, hipStream_t stream) {
    const int total = a.first[kJpegMaxComps];
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jpeg_fdct, dim3((total + kDctBlocksPerGroup - 1) / kDctBlocksPerGroup), dim3(256), 0,
                       stream, a);
    return note_hip("k_jpeg_fdct launch", hipGetLastError());
}

}  // namespace oilpaint_impl
