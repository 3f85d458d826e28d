/* The C oracles under gcc's sanitizers (tests/test_host_sanitizers.py builds
 * this with AddressSanitizer and UndefinedBehaviorSanitizer, and again with
 * ThreadSanitizer): the filter in both forms and the median on small images
 * of every shape class -- single pixels, rows, columns, windows wider than
 * the image, padded strides -- single- and multi-threaded.  Besides the
 * sanitizers' own reports it checks what holds at any size: radius 0 gives
 * the image back (a one-pixel window is its own mode, mean and median), the
 * thread count never changes the result, and padding bytes are never
 * written. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oilpaint_ref(const uint8_t *src, uint8_t *dst, int width, int height, int stride, int radius, int levels,
                 int nthreads);
int oilpaint_ref_paper(const uint8_t *src, uint8_t *dst, int width, int height, int stride, int radius, int levels,
                       int nthreads);
int median_ref(const uint8_t *src, uint8_t *dst, int width, int height, int src_stride, int dst_stride,
               int channels, int ch, int radius, int nthreads);

static int failures = 0;
#define EXPECT(c)                                                                  \
    do {                                                                           \
        if (!(c)) {                                                                \
            fprintf(stderr, "%s:%d: failed: %s\n", __FILE__, __LINE__, #c);        \
            ++failures;                                                            \
        }                                                                          \
    } while (0)

static uint64_t rng = 0x243F6A8885A308D3ull;
static uint32_t next_u32(void)
{
    rng ^= rng >> 12;
    rng ^= rng << 25;
    rng ^= rng >> 27;
    return (uint32_t)((rng * 0x2545F4914F6CDD1Dull) >> 32);
}

/* One (w, h, stride) shape: every radius in radii, a few level counts, both
 * filter forms and the median on each channel. */
static void shape(int w, int h, int pad, int threads)
{
    static const int radii[] = {0, 1, 2, 3, 5, 9};
    static const int levels[] = {1, 2, 20, 64, 256};
    const int stride = 3 * w + pad;
    const size_t bytes = (size_t)stride * (size_t)h;
    uint8_t *src = malloc(bytes ? bytes : 1), *a = malloc(bytes ? bytes : 1), *b = malloc(bytes ? bytes : 1);
    size_t i;
    unsigned ri, li;
    int y, x, c;
    for (i = 0; i < bytes; ++i) src[i] = (uint8_t)next_u32();
    for (ri = 0; ri < sizeof(radii) / sizeof(radii[0]); ++ri)
        for (li = 0; li < sizeof(levels) / sizeof(levels[0]); ++li) {
            const int r = radii[ri], L = levels[li];
            int paper;
            for (paper = 0; paper < 2; ++paper) {
                int (*f)(const uint8_t *, uint8_t *, int, int, int, int, int, int) =
                    paper ? oilpaint_ref_paper : oilpaint_ref;
                memset(a, 0xCD, bytes);
                memset(b, 0xCD, bytes);
                EXPECT(f(src, a, w, h, stride, r, L, 1) == 0);
                EXPECT(f(src, b, w, h, stride, r, L, threads) == 0);
                EXPECT(memcmp(a, b, bytes) == 0);
                for (y = 0; y < h; ++y)
                    for (x = 3 * w; x < stride; ++x) EXPECT(a[(size_t)y * stride + x] == 0xCD);
                if (r == 0 && !paper)
                    for (y = 0; y < h; ++y) EXPECT(memcmp(a + (size_t)y * stride, src + (size_t)y * stride, 3 * (size_t)w) == 0);
            }
        }
    for (ri = 0; ri < sizeof(radii) / sizeof(radii[0]); ++ri)
        for (c = 0; c < 3; ++c) {
            const int r = radii[ri];
            const int dstride = w + pad;
            const size_t db = (size_t)dstride * (size_t)h;
            uint8_t *m1 = malloc(db ? db : 1), *m2 = malloc(db ? db : 1);
            memset(m1, 0xCD, db);
            memset(m2, 0xCD, db);
            EXPECT(median_ref(src, m1, w, h, stride, dstride, 3, c, r, 1) == 0);
            EXPECT(median_ref(src, m2, w, h, stride, dstride, 3, c, r, threads) == 0);
            EXPECT(memcmp(m1, m2, db) == 0);
            for (y = 0; y < h; ++y) {
                for (x = w; x < dstride; ++x) EXPECT(m1[(size_t)y * dstride + x] == 0xCD);
                if (r == 0)
                    for (x = 0; x < w; ++x) EXPECT(m1[(size_t)y * dstride + x] == src[(size_t)y * stride + 3 * x + c]);
            }
            free(m1);
            free(m2);
        }
    free(src);
    free(a);
    free(b);
}

int main(int argc, char **argv)
{
    static const int shapes[][3] = {{1, 1, 0}, {1, 7, 1}, {7, 1, 0}, {2, 2, 5}, {3, 11, 0}, {17, 5, 3},
                                    {31, 29, 0}, {64, 9, 2}, {70, 40, 7}};
    const int threads = argc > 1 ? atoi(argv[1]) : 4;
    unsigned k;
    uint8_t one[3] = {1, 2, 3}, out[3];
    /* argument checks */
    EXPECT(oilpaint_ref(NULL, out, 1, 1, 3, 0, 20, 1) != 0);
    EXPECT(oilpaint_ref(one, out, -1, 1, 3, 0, 20, 1) != 0);
    EXPECT(oilpaint_ref(one, out, 1, 1, 3, 0, 0, 1) != 0);
    EXPECT(median_ref(one, out, 1, 1, 3, 1, 3, 3, 0, 1) != 0);
    /* empty images */
    EXPECT(oilpaint_ref(one, out, 0, 0, 0, 2, 20, threads) == 0);
    EXPECT(median_ref(one, out, 0, 5, 0, 0, 3, 0, 2, threads) == 0);
    for (k = 0; k < sizeof(shapes) / sizeof(shapes[0]); ++k) shape(shapes[k][0], shapes[k][1], shapes[k][2], threads);
    printf("%d failures\n", failures);
    return failures ? 1 : 0;
}
