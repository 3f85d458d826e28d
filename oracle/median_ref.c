/*
 * median_ref.c -- plain CPU oracle for the windowed median filter, the
 * second filter of the same class as the oil paint (a per-window histogram
 * of pixel values, queried per output pixel; the paper's conclusions name
 * this class of image filters).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never calls it
 * and shares no code, header or table with it.
 *
 * What it computes, for a `channels`-interleaved 8-bit image and one channel
 * index `ch`:
 *
 *   for every output pixel (x, y):
 *     * V = the values src[yy][xx][ch] over the (2r+1) x (2r+1) window
 *       centred on (x, y), clipped to the image; n = |V| >= 1;
 *     * the output is the lower median of V: its element of rank
 *       floor((n - 1) / 2) in increasing order (0-based);
 *     * dst is a one-channel image (one byte per pixel, its own row stride;
 *       bytes [width, dst_stride) of a row are not written).
 *
 * The definition is written out directly: a 256-count histogram of the
 * window, then the smallest value whose cumulative count exceeds the rank.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    const uint8_t *src;
    uint8_t *dst;
    int width, height, src_stride, dst_stride, channels, ch, radius;
    int row_begin, row_end;
} median_job;

static void median_pixel(const median_job *j, int x, int y)
{
    unsigned count[256];
    int yy, xx, v;
    unsigned n = 0, rank, cum = 0;
    const int y0 = y - j->radius < 0 ? 0 : y - j->radius;
    const int y1 = y + j->radius > j->height - 1 ? j->height - 1 : y + j->radius;
    const int x0 = x - j->radius < 0 ? 0 : x - j->radius;
    const int x1 = x + j->radius > j->width - 1 ? j->width - 1 : x + j->radius;
    for (v = 0; v < 256; ++v) count[v] = 0;
    for (yy = y0; yy <= y1; ++yy)
        for (xx = x0; xx <= x1; ++xx) {
            ++count[j->src[(long)yy * j->src_stride + (long)xx * j->channels + j->ch]];
            ++n;
        }
    rank = (n - 1) / 2;
    for (v = 0; v < 256; ++v) {
        cum += count[v];
        if (cum > rank) {
            j->dst[(long)y * j->dst_stride + x] = (uint8_t)v;
            return;
        }
    }
    abort(); /* n >= 1, so some value holds the rank */
}

static void *median_rows(void *arg)
{
    const median_job *j = (const median_job *)arg;
    int y, x;
    for (y = j->row_begin; y < j->row_end; ++y)
        for (x = 0; x < j->width; ++x) median_pixel(j, x, y);
    return NULL;
}

/* Returns 0, -1 for a NULL pointer, -2 for an invalid size or channel. */
int median_ref(const uint8_t *src, uint8_t *dst, int width, int height, int src_stride, int dst_stride,
               int channels, int ch, int radius, int nthreads)
{
    pthread_t tids[256];
    median_job jobs[256];
    int t;
    if (!src || !dst) return -1;
    if (width < 0 || height < 0 || radius < 0 || channels < 1 || channels > 4 || ch < 0 || ch >= channels)
        return -2;
    if ((long)src_stride < (long)channels * width || dst_stride < width) return -2;
    if (width == 0 || height == 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > height) nthreads = height;
    for (t = 0; t < nthreads; ++t) {
        jobs[t].src = src;
        jobs[t].dst = dst;
        jobs[t].width = width;
        jobs[t].height = height;
        jobs[t].src_stride = src_stride;
        jobs[t].dst_stride = dst_stride;
        jobs[t].channels = channels;
        jobs[t].ch = ch;
        jobs[t].radius = radius;
        jobs[t].row_begin = (int)((long)height * t / nthreads);
        jobs[t].row_end = (int)((long)height * (t + 1) / nthreads);
    }
    if (nthreads == 1) {
        median_rows(&jobs[0]);
        return 0;
    }
    for (t = 0; t < nthreads; ++t)
        if (pthread_create(&tids[t], NULL, median_rows, &jobs[t]) != 0) {
            int u;
            for (u = t; u < nthreads; ++u) median_rows(&jobs[u]);
            nthreads = t;
            break;
        }
    for (t = 0; t < nthreads; ++t) pthread_join(tids[t], NULL);
    return 0;
}
