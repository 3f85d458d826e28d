// Device steps of the JPEG codec around the filter: dequantization and the
// 8 x 8 inverse DCT (T.81 A.3.3, A.3.5), JFIF colour conversion with chroma
// replication (decode); JFIF colour conversion with chroma averaging, the
// forward DCT and quantization (T.81 A.3.3, A.3.4) (encode).  One wavefront
// per 8 x 8 block (lane = one sample or coefficient), separable passes through
// LDS; colour conversion one lane per pixel.  Entropy decoding runs on the
// host (oilpaint_jpeg.cpp), the encoder's Huffman coding in
// oilpaint_k_huff.hip.
#include "oilpaint_internal.h"
#include "oilpaint_jpeg.h"

namespace oilpaint_impl {
namespace {

// cos(m pi / 16) / sqrt(2), m = 0..8.
__constant__ float kCosR2[9] = {
    0.70710678118654752f, 0.69351992266107906f, 0.65328148243818826f, 0.58794459036236287f,
    0.50000000000000000f, 0.39284747919355110f, 0.27059805007309849f, 0.13794968964147150f,
    0.0f};

// sqrt(2) x C(u)/2 x cos((2x+1) u pi / 16): exactly 1/2 for u = 0 and +-1/2
// for u = 4, so that blocks whose exact transform is rational (flat blocks,
// the u, v in {0, 4} terms) come out exact in fp32; the transform is this
// basis applied twice, then halved.
__device__ __forceinline__ float basis(int u, int x) {
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

// Four blocks per workgroup, one per wavefront.
__global__ __launch_bounds__(256) void k_jpeg_idct(JpegIdctArgs a) {
    __shared__ float s_coef[4][64];
    __shared__ float s_tmp[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int total = a.first[kJpegMaxComps];
    const int b = blockIdx.x * 4 + wave;
    const bool live = b < total;
    const int c = live ? comp_of(a.first, b) : 0;
    const int r = lane >> 3, col = lane & 7;
    if (live) s_coef[wave][lane] = (float)((int)a.coef[(size_t)b * 64 + lane] * (int)a.q[c][lane]);
    __syncthreads();
    // rows: t[v][x] = sum_u S[v][u] B[u][x]   (lane = (v, x))
    float t = 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) t = fmaf(s_coef[wave][r * 8 + u], basis(u, col), t);
    s_tmp[wave][lane] = t;
    __syncthreads();
    // columns: s[y][x] = sum_v B[v][y] t[v][x]   (lane = (y, x))
    float s = 0.f;
#pragma unroll
    for (int v = 0; v < 8; ++v) s = fmaf(basis(v, r), s_tmp[wave][v * 8 + col], s);
    if (!live) return;
    const int v = (int)floorf(fminf(fmaxf(s * 0.5f + 128.5f, 0.f), 255.f));
    const int k = b - a.first[c];
    const int by = k / a.bw[c], bx = k - by * a.bw[c];
    const int y = by * 8 + r, x = bx * 8 + col;
    if (x < a.limit_w[c] && y < a.limit_h[c])
        a.plane[c][(size_t)y * a.stride[c] + x] = (uint8_t)v;
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

__global__ __launch_bounds__(256) void k_jpeg_fdct(JpegFdctArgs a) {
    __shared__ float s_smp[4][64];
    __shared__ float s_tmp[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int total = a.first[kJpegMaxComps];
    const int b = blockIdx.x * 4 + wave;
    const bool live = b < total;
    const int c = live ? comp_of(a.first, b) : 0;
    const int r = lane >> 3, col = lane & 7;
    if (live) {
        const int k = b - a.first[c];
        const int by = k / a.bw[c], bx = k - by * a.bw[c];
        s_smp[wave][lane] = (float)((int)a.plane[c][(size_t)(by * 8 + r) * a.stride[c] + bx * 8 + col] - 128);
    }
    __syncthreads();
    // rows: t[y][u] = sum_x s[y][x] B[u][x]   (lane = (y, u))
    float t = 0.f;
#pragma unroll
    for (int x = 0; x < 8; ++x) t = fmaf(s_smp[wave][r * 8 + x], basis(col, x), t);
    s_tmp[wave][lane] = t;
    __syncthreads();
    // columns: S[v][u] = sum_y B[v][y] t[y][u]   (lane = (v, u))
    float S = 0.f;
#pragma unroll
    for (int y = 0; y < 8; ++y) S = fmaf(basis(r, y), s_tmp[wave][y * 8 + col], S);
    if (!live) return;
    const float q = S * 0.5f / (float)a.q[c][lane];
    const float m = floorf(fabsf(q) + 0.5f);
    a.coef[(size_t)b * 64 + lane] = (int16_t)(q < 0.f ? -m : m);
}

}  // namespace

hipError_t launch_jpeg_idct(const JpegIdctArgs& a, hipStream_t stream) {
    const int total = a.first[kJpegMaxComps];
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jpeg_idct, dim3((total + 3) / 4), dim3(256), 0, stream, a);
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
    hipLaunchKernelGGL(k_jpeg_fdct, dim3((total + 3) / 4), dim3(256), 0, stream, a);
    return note_hip("k_jpeg_fdct launch", hipGetLastError());
}

}  // namespace oilpaint_impl
