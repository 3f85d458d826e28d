/*
 * oilpaint.h -- C-ABI of liboilpaint.so, the gfx950 (MI355X) oil-paint filter.
 *
 * The operation (Mukherjee, "Study on performance improvement of oil paint
 * image filter algorithm using parallel pattern library", Section 4: the
 * histogram-based algorithm, its interface ApplyOilPaintOnBuffer and its
 * serial listing; Section 5 keeps the same interface for the parallel form):
 *
 *   For every output pixel (x, y) of an interleaved 8-bit, 3-channel image,
 *   each pixel of the (2r+1) x (2r+1) window around (x, y) is given the
 *   intensity level  k = ((c0 + c1 + c2) / 3) * L / 256  (unsigned integer
 *   arithmetic, truncating, left to right; k in [0, L)).  Per level the
 *   number of window pixels and the three channel sums are kept.  The level
 *   holding the most pixels is chosen -- the lowest level when several hold
 *   the same largest number -- and each output channel is that level's
 *   channel sum divided by its pixel count, truncated.
 *
 *   The window is clipped to the image: near the border only its in-image
 *   pixels take part, and every pixel of the image is written.  (The paper's
 *   listing processes only the interior [r, W-r) x [r, H-r); that literal
 *   form is OILPAINT_FLAG_PAPER below.)  The result is a unique byte array:
 *   it is bit-exact, with no tolerance.
 *
 * Conventions shared by every entry point:
 *   - Images are `height` rows of `width` pixels; a pixel is 3 bytes
 *     (c0, c1, c2), and row y starts at byte y * stride.  In the
 *     single-image calls one `stride` (bytes, >= 3 * width) serves src and
 *     dst; descriptors (oilpaint_desc) may give dst its own stride.  Bytes
 *     [3*width, stride) of a row are neither read nor written.  Channel order
 *     does not matter: the filter commutes with any permutation of the three
 *     channels.
 *   - src and dst are device pointers (hipMalloc'd, or any memory the
 *     current device can access) owned by the caller; the library keeps no
 *     reference to them after the work completes.  src and dst must not
 *     overlap (the filter is not in-place, as in the paper, whose caller
 *     allocates a separate output buffer).
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  *_async calls only enqueue work.
 *   - Every call returns an int status: OILPAINT_OK (0) or a negative
 *     OILPAINT_ERR_* code.  On any error nothing is enqueued and dst is left
 *     untouched.  An image with width == 0 or height == 0 is a no-op that
 *     returns OILPAINT_OK once the pointers and sizes are valid.
 *   - radius: 0 <= r <= 65535.  Any r >= max(width, height) - 1 behaves as
 *     that value (every window already holds the whole image); an image whose
 *     effective radius exceeds 2051 returns OILPAINT_ERR_UNSUPPORTED (the
 *     32-bit window sums could overflow).  levels: 1 <= L <= 256.
 *   - The library is thread-safe for calls on different streams; calls that
 *     share an oilpaint_plan or oilpaint_queue must be serialised by the
 *     caller.
 */
#ifndef OILPAINT_H
#define OILPAINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OILPAINT_ABI_VERSION 1

/* Status codes. */
#define OILPAINT_OK              0
#define OILPAINT_ERR_NULL       -1  /* a required pointer is NULL (the paper's E_FAIL case) */
#define OILPAINT_ERR_ARG        -2  /* a size, radius, level count, stride or row range is invalid */
#define OILPAINT_ERR_OVERLAP    -3  /* src and dst byte ranges overlap */
#define OILPAINT_ERR_NOT_DEVICE -4  /* src or dst is not memory the current device can access */
#define OILPAINT_ERR_HIP        -5  /* a HIP runtime call failed */
#define OILPAINT_ERR_NOMEM      -6  /* the library could not allocate its own scratch */
#define OILPAINT_ERR_FULL       -7  /* an oilpaint_queue has no free slot */
#define OILPAINT_ERR_UNSUPPORTED -8 /* a combination the library does not handle (see each call) */

/* Flags (oilpaint_desc.flags). */
#define OILPAINT_FLAG_PAPER 1u  /* the paper's listing taken literally: level
                                   ((c0+c1+c2) * L / 3.0) / 255 truncated, which
                                   has L+1 levels of which the last (pure white)
                                   is never chosen; only the interior
                                   [r, W-r) x [r, H-r) is written; a pixel whose
                                   scanned levels are all empty is not written */

/* Library version (OILPAINT_ABI_VERSION). */
int oilpaint_version(void);

/* Static text for a status code; never NULL. */
const char *oilpaint_strerror(int status);

/* Text of the last HIP runtime failure seen by the library on the calling
 * thread ("" if none): the call that failed and HIP's message.  Valid until
 * the thread's next library call. */
const char *oilpaint_last_error(void);

/* Pure host-side argument check, no HIP call and no GPU needed: the checks
 * every entry point runs first.  Returns OILPAINT_OK, ERR_NULL, ERR_ARG or
 * ERR_OVERLAP (byte ranges [p, p + (height-1)*stride + 3*width) of src and
 * dst intersect). */
int oilpaint_validate(const uint8_t *src, const uint8_t *dst, int width, int height, int stride,
                      int radius, int levels);

/* Filter one image and wait for it: enqueue on the default stream, then
 * synchronize that stream (Section 4 interface: input buffer, size, level
 * count, radius, output buffer). */
int oilpaint(const uint8_t *src, uint8_t *dst, int width, int height, int stride, int radius,
             int levels);

/* Filter one image asynchronously on `stream` with the launch shape the
 * library picks for (radius, levels) -- its built-in choice or the one
 * installed by oilpaint_set_variant. */
int oilpaint_async(const uint8_t *src, uint8_t *dst, int width, int height, int stride,
                   int radius, int levels, void *stream);

/* ---------------------------------------------------------------------------
 * Launch shapes ("variants").  A tile of the image is computed by one
 * workgroup of `waves` wavefronts of 64 lanes; each lane owns one output
 * column and slides its window histogram down `rows` output rows.  `hist`
 * selects the per-lane histogram layout:
 *   OILPAINT_HIST_PACKED  one 64-bit word per level (count:10 | three
 *                         18-bit channel sums), the tile and its halo staged
 *                         on chip; windows up to 31 x 31 (radius <= 15) and
 *                         levels <= 255 (<= 254 with OILPAINT_FLAG_PAPER)
 *   OILPAINT_HIST_STREAM  the PACKED bins with only the 2r+2 image rows the
 *                         windows span kept on chip, fetched as the run
 *                         advances; 64 lanes, radius <= 15, levels <= 64;
 *                         waves = 1 (one wavefront per strip) or 4 (four
 *                         wavefronts share a strip, as described for
 *                         OILPAINT_HIST_STREAM8)
 *   OILPAINT_HIST_WIDE    32-bit count and sums, pixels read from device
 *                         memory; any level count and radius up to 2051
 *   OILPAINT_HIST_STREAM8 OILPAINT_HIST_STREAM whose on-chip rows hold each
 *                         pixel's ready-made bin increment (8 bytes instead
 *                         of 4): fewer instructions per window update, twice
 *                         the row storage; radius 8..15, levels <= 32.
 *                         waves = 1: one wavefront per strip; waves = 4: four
 *                         wavefronts share one strip's histogram and rows,
 *                         each making a quarter of every row step's updates
 *                         and of the mode search (a CU then holds four times
 *                         the wavefronts at about the same on-chip
 *                         footprint); `rows` is then the run of the whole
 *                         workgroup.  Batches and plans run these jobs with
 *                         waves = 1.
 *   OILPAINT_HIST_COLUMN  per-column histograms of the window rows; each
 *                         lane's window is the difference of two per-level
 *                         prefix sums across the strip, so the work per
 *                         output row does not grow with the radius (column
 *                         histograms after Perreault and Hebert, "Median
 *                         filtering in constant time", 2007); 64 lanes,
 *                         radius <= 255, any level count whose (levels + 1)
 *                         x (64 + 2 radius) 8-byte column histograms fit on
 *                         chip; one wavefront per workgroup, or, for radius
 *                         <= 15 and at most 64 levels, 1, 2 or 4 wavefronts
 *                         sharing the strip (runs as in STREAM: waves x 64
 *                         threads work one run of `rows` output rows), and
 *                         for radius 16..31 and at most 64 levels 2 or 4
 *                         (the same count-word form with wider fields).
 *                         Batches and plans run such jobs with 4 wavefronts
 *                         from radius 7 to 15; below it in the streamed
 *                         layout (with waves = 1 in the paper form); above
 *                         it with one wavefront.
 *   OILPAINT_HIST_REGS    the PACKED bin word of every level in each lane's
 *                         own registers instead of LDS (the listing's
 *                         per-level arrays per thread): a window update adds
 *                         the pixel's increment to every bin under a mask
 *                         "level == bin" (a register cannot be addressed by
 *                         the level), so LDS atomics become VALU work; the
 *                         rows are streamed as in STREAM.  64 lanes, one
 *                         wavefront, radius <= 7, levels <= 16.  Batches and
 *                         plans run such jobs in the streamed layout.
 * ------------------------------------------------------------------------- */
#define OILPAINT_HIST_PACKED  0
#define OILPAINT_HIST_STREAM  1
#define OILPAINT_HIST_WIDE    2
#define OILPAINT_HIST_STREAM8 3
#define OILPAINT_HIST_COLUMN  4
#define OILPAINT_HIST_REGS    5

typedef struct oilpaint_variant {
    int32_t rows;   /* output rows per lane, >= 1; 0: derived from per_cu */
    int32_t waves;  /* wavefronts per workgroup, 1..8 */
    int32_t hist;   /* OILPAINT_HIST_* */
    int32_t lanes;  /* active lanes (= output columns) per wavefront: 64, 32 or 16 */
    int32_t per_cu; /* with rows = 0: rows are chosen so that an image yields about
                       per_cu workgroups per compute unit (1..64), 2 .. 1024 rows,
                       then halved while the on-chip footprint does not fit */
} oilpaint_variant;

/* The variant oilpaint_async would use for (radius, levels) and an image of
 * the given size, with `rows` resolved for that size.  Returns OK or
 * ERR_ARG / ERR_NULL. */
int oilpaint_pick_variant(int width, int height, int radius, int levels, oilpaint_variant *out);

/* Install `v` as the choice for (radius, levels) (the autotuner's result).
 * Returns ERR_UNSUPPORTED if v cannot run (radius, levels) -- for example a
 * PACKED layout for a window wider than 31, or a shape whose on-chip memory
 * exceeds the device's. */
int oilpaint_set_variant(int radius, int levels, const oilpaint_variant *v);

/* Forget every installed choice. */
int oilpaint_clear_variants(void);

/* Filter one image with an explicit variant (for tuning and tests). */
int oilpaint_async_variant(const uint8_t *src, uint8_t *dst, int width, int height, int stride,
                           int radius, int levels, const oilpaint_variant *v, void *stream);

/* Time n candidate variants for (radius, levels) on a width x height image
 * that the library allocates and fills with a fixed photo-like pattern
 * (smooth ramps with small noise: the column layout's cost depends on how
 * many distinct modes neighbouring pixels have, and photographs have few).
 * Each candidate is run once untimed,
 * then `reps` times between HIP events on `stream`; ms_out[i] receives its
 * average milliseconds per launch, or -1 if it cannot run (radius, levels).
 * Synchronizes `stream`.  Returns OK, ERR_NULL, ERR_ARG, ERR_NOMEM or
 * ERR_HIP.  The autotuner (paper_1405_1020_amd/tune.py) installs the winner
 * with oilpaint_set_variant. */
int oilpaint_tune(int width, int height, int radius, int levels, const oilpaint_variant *candidates,
                  int n, int reps, void *stream, float *ms_out);

/* ---------------------------------------------------------------------------
 * Batches: many images of uneven size, radius and level count in ONE
 * persistent launch over a flattened tile queue.
 * ------------------------------------------------------------------------- */
typedef struct oilpaint_desc {
    const uint8_t *src;    /* device pointer, image as above */
    uint8_t *dst;          /* device pointer, disjoint from src */
    int32_t width, height;
    int32_t stride;        /* row stride of src in bytes (>= 3 * width) */
    int32_t dst_stride;    /* row stride of dst in bytes; 0 means `stride` */
    int32_t radius, levels;
    int32_t row_begin;     /* compute output rows [row_begin, row_end) only; */
    int32_t row_end;       /* row_begin = row_end = 0 selects every row      */
    uint32_t flags;        /* OILPAINT_FLAG_* */
    uint32_t reserved;     /* must be 0 */
} oilpaint_desc;

/* Filter one descriptor asynchronously on `stream` with the plain kernel
 * (one workgroup per tile, the library's launch shape).  Unlike
 * oilpaint_async it takes separate src and dst strides -- for example a
 * crop of a larger resident image written to a dense output -- a row band
 * and flags.  Validation as oilpaint_batch for one item. */
int oilpaint_run(const oilpaint_desc *desc, void *stream);

/* Validate all n descriptors (all or nothing: on error *bad_index, if not
 * NULL, receives the first failing index and nothing is enqueued), then
 * enqueue the persistent launch on `stream` that computes every image.  The
 * images are grouped into kernel classes (streamed layout: one class per
 * radius and level bucket; every other layout: one generic class); each
 * class is one persistent kernel over its own flattened tile queue, sized
 * by its own registers and LDS, and the classes run concurrently on up to
 * four streams forked from and joined back into `stream`.  The descriptor
 * array is copied; it may be reused when the call returns. */
int oilpaint_batch(const oilpaint_desc *descs, int n, void *stream, int *bad_index);

/* oilpaint_batch for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same validation, kernels and results as oilpaint_batch, but the batch's
 * argument block (a counter per kernel class, the classes' tile prefix sums
 * and the job descriptors: 256 + 16 per class + 4 (n + classes) + 104 n bytes
 * or so) lives in a static device array of OILPAINT_NOALLOC_SCRATCH_BYTES
 * that each GPU the library runs on holds until the process ends, and the
 * call makes no hipMalloc, hipFree or other allocating call (its first call
 * on a device takes the array's address there and creates the side streams
 * the classes run on).  A batch whose block does not fit returns ERR_ARG
 * (text in oilpaint_last_error) and enqueues nothing.  The block is
 * uploaded from pageable host memory, so the call returns once the upload
 * is done.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (on different streams, or from several threads without
 * ordering) race; calls on one stream are ordered. */
#define OILPAINT_NOALLOC_SCRATCH_BYTES (1 << 20)
int oilpaint_batch_noalloc(const oilpaint_desc *descs, int n, void *stream, int *bad_index);

/* A batch plan: the descriptors are validated and laid out once (tile queues
 * in device memory, ordered by estimated cost) and the launch -- a counter
 * reset kernel, then the classes' persistent kernels as parallel graph
 * branches -- is captured in a hipGraph that oilpaint_plan_launch replays.  Replays compute the same descriptors; the
 * caller may change the CONTENTS of the src images between replays. */
typedef struct oilpaint_plan oilpaint_plan;
int oilpaint_plan_create(const oilpaint_desc *descs, int n, void *stream, oilpaint_plan **out,
                         int *bad_index);
int oilpaint_plan_launch(oilpaint_plan *plan, void *stream);
/* Number of tiles and of workgroups over all classes' persistent kernels. */
int oilpaint_plan_info(const oilpaint_plan *plan, int *tiles, int *workgroups);
int oilpaint_plan_destroy(oilpaint_plan *plan);

/* ---------------------------------------------------------------------------
 * Windowed median of one channel: the second filter of the oil paint's class
 * (a per-window histogram of pixel values queried per output pixel; the
 * paper's conclusions name this class of filters).  For every pixel, the
 * lower median -- the element of rank floor((n-1)/2), 0-based, of the n
 * values of channel `channel` in its (2r+1) x (2r+1) window clipped to the
 * image -- is written to a one-channel image.
 * ------------------------------------------------------------------------- */

/* src: `channels` (1..4) interleaved 8-bit channels per pixel, rows
 * src_stride bytes apart (>= channels * width); dst: one byte per pixel, rows
 * dst_stride bytes apart (>= width); bytes [width, dst_stride) of a dst row
 * are not written.  Device pointers, disjoint.  Effective radius (the radius
 * clamped to max(width, height) - 1) at most 127, else ERR_UNSUPPORTED.
 * Enqueues on `stream`; errors as oilpaint_async (ERR_NULL, ERR_ARG for a
 * size, stride or channel, ERR_OVERLAP, ERR_NOT_DEVICE, ERR_HIP).  The
 * kernel form is the one installed for the radius (oilpaint_median_set_kind)
 * or else the built-in choice (one or four wavefronts per strip up to radius
 * 15, column histograms above). */
int oilpaint_median_async(const uint8_t *src, int src_stride, int channels, int channel, uint8_t *dst,
                          int dst_stride, int width, int height, int radius, void *stream);
/* Kernel forms of the median:
 *   OILPAINT_MEDIAN_ONE     two-level count histogram per lane in LDS, rows
 *                           sliding down, one wavefront per 64-column strip
 *                           (radius <= 15);
 *   OILPAINT_MEDIAN_FOUR    the same worked by four wavefronts per strip
 *                           (radius <= 15);
 *   OILPAINT_MEDIAN_COLUMN  one-byte fine and coarse histograms of every
 *                           column's window rows; each lane's window counts
 *                           are differences of prefix sums across the strip,
 *                           so the work per row does not grow with the radius
 *                           (radius <= 127).
 * OILPAINT_MEDIAN_AUTO selects the installed or built-in form. */
#define OILPAINT_MEDIAN_AUTO   0
#define OILPAINT_MEDIAN_ONE    1
#define OILPAINT_MEDIAN_FOUR   2
#define OILPAINT_MEDIAN_COLUMN 3
/* oilpaint_median_async with an explicit form (ERR_UNSUPPORTED where the form
 * does not cover the effective radius). */
int oilpaint_median_async_kind(const uint8_t *src, int src_stride, int channels, int channel, uint8_t *dst,
                               int dst_stride, int width, int height, int radius, int kind, void *stream);
/* Install the form used for `radius` (0..127) from now on (the tuner's
 * choice); OILPAINT_MEDIAN_AUTO restores the built-in one. */
int oilpaint_median_set_kind(int radius, int kind);
/* The form oilpaint_median_async uses for an effective radius, or
 * ERR_UNSUPPORTED. */
int oilpaint_median_pick_kind(int radius);
/* The same on the default stream, then wait for it. */
int oilpaint_median(const uint8_t *src, int src_stride, int channels, int channel, uint8_t *dst,
                    int dst_stride, int width, int height, int radius);

/* ---------------------------------------------------------------------------
 * Continuous batching.  A queue accepts filter requests at any time; each
 * oilpaint_queue_step (also run by push, poll and completed) packs the small
 * requests that are waiting -- new requests and the unfinished rows of
 * running ones, an equal share of the launch's pixels each, in whole tile
 * rows -- into one batch launch, keeping at most four launches in flight, so
 * that requests that arrive while others are on the GPU share the next
 * launch with them.  Launches run on the queue's side streams and do not
 * wait for each other: the next launch's kernels start while the previous
 * one's last tiles finish.  A launch covers `step_pixels` output pixels, or
 * a quarter of the waiting small-request pixels when that is more (at most
 * 64 x step_pixels).  A request of at least 4 Mi output pixels, and a lone
 * request with nothing in flight, is launched whole with the plain kernel
 * and its own launch shape; while small requests wait, at most every other
 * launch is such a large request.
 * ------------------------------------------------------------------------- */
typedef struct oilpaint_queue oilpaint_queue;

/* capacity: most requests held at once (pending or running).  step_pixels:
 * work per launch (output pixels, >= 1; 0 picks a default).  The queue uses
 * its own non-blocking stream on the current device. */
int oilpaint_queue_create(int capacity, int64_t step_pixels, oilpaint_queue **out);
/* Append one request.  *ticket receives its id.  ERR_FULL if `capacity`
 * requests are already held; a descriptor error (as oilpaint_run) is
 * returned at once and the request is not queued.  The descriptor is
 * copied; the images must stay valid until the request is reported
 * complete.  A launch holding rows of a request that fails to be enqueued
 * fails that request: it is reported complete with the error as its status
 * (poll, completed), once no kernel of it can still write its dst, and the
 * queue goes on with the others. */
int oilpaint_queue_push(oilpaint_queue *q, const oilpaint_desc *desc, uint64_t *ticket);
/* Make progress without blocking; returns the number of launches enqueued. */
int oilpaint_queue_step(oilpaint_queue *q);
/* 1 if the request's output is complete (its bytes are in dst and visible
 * to later work on any stream), 0 if not yet, the request's error code if it
 * failed (see push), ERR_ARG for an unknown ticket.  Once poll has returned
 * 1 or a request's error for a ticket the queue forgets it. */
int oilpaint_queue_poll(oilpaint_queue *q, uint64_t ticket);
/* Tickets of requests completed since they were last reported (by poll or
 * by this call), in completion order: at most `max` are written to
 * `tickets`, and those are forgotten.  If `status` is not NULL, status[i]
 * receives OILPAINT_OK or the error of a failed request.  Returns the number
 * written, or an error code.  One call replaces a poll per request. */
int oilpaint_queue_completed(oilpaint_queue *q, uint64_t *tickets, int *status, int max);
/* Block until every pushed request is complete (or failed). */
int oilpaint_queue_drain(oilpaint_queue *q);
/* Failure injection for tests of the error path: the queue's next `n`
 * launches are treated as failed before anything is enqueued (their
 * requests fail with ERR_HIP).  No kernel runs for them. */
int oilpaint_queue_fail_next(oilpaint_queue *q, int n);
/* The queue's control stream (hipStream_t as void*), which carries the
 * uploads and counter resets; the filter kernels run on side streams.  Use
 * poll or completed to learn that a request's output is ready. */
void *oilpaint_queue_stream(oilpaint_queue *q);
int oilpaint_queue_destroy(oilpaint_queue *q);

/* ---------------------------------------------------------------------------
 * JPEG decode and encode around the filter.  The paper's program reads a JPEG
 * file, filters its pixels and writes a JPEG file, timing decode, filter and
 * encode apart (Section 3: its decoder, its encoder and the file driver);
 * here the per-sample steps run on the GPU, so a decoded image is filtered
 * where it lies and the filtered image is encoded from there.
 *
 * Format: baseline sequential DCT-based JPEG (ITU-T T.81 | ISO/IEC 10918-1;
 * SOF0 or SOF1, Huffman coding, 8-bit samples and 8-bit quantization tables),
 * one or three components with sampling factors 1..4, restart intervals,
 * interleaved or per-component scans, in JFIF's YCbCr colour space.
 * Progressive, lossless, hierarchical and arithmetic-coded files return
 * ERR_UNSUPPORTED; malformed ones ERR_ARG.
 *
 * What is computed (the same definitions as the test oracle):
 *   decode: Huffman decoding (F.2.2) on the GPU, parallel over subsequences
 *     of the entropy-coded data: each is decoded from every guess of where
 *     its decoding starts, the guesses meet the true decoding at a
 *     checkpoint (Huffman codes resynchronize), and the host follows the
 *     links between subsequences to hand each its true start (the host also
 *     strips the byte stuffing and RST markers and plans the subsequences);
 *     on the GPU too, dequantization (A.3.5) and the 8 x 8 inverse DCT (A.3.3) in fp32, each
 *     sample + 128 rounded half up and clamped to [0, 255]; each chroma sample
 *     replicated over the Hmax/H x Vmax/V pixels it covers; JFIF YCbCr -> RGB
 *     (R = Y + 1.402 Cr', G = Y - 0.344136 Cb' - 0.714136 Cr', B = Y + 1.772
 *     Cb', Cb' = Cb - 128, Cr' = Cr - 128) evaluated exactly in integers,
 *     rounded half up, clamped; one component gives R = G = B = Y.
 *   encode: the image extended to whole MCUs by repeating its last column and
 *     row; JFIF RGB -> YCbCr exactly in integers, rounded half up; each chroma
 *     sample the mean of the pixels it covers, rounded half up; the 8 x 8
 *     forward DCT (A.3.3) of sample - 128 in fp32 and quantization to the
 *     nearest integer, halves away from zero (A.3.4), on the GPU; Huffman
 *     coding (F.1.2) with tables fitted to the image (K.2): the symbol
 *     statistics, the codes, their placement and the byte stuffing (B.1.1.5)
 *     on the GPU, the table fitting and the headers on the host.
 *     Quantization tables: T.81 Tables K.1 and K.2 scaled by quality
 *     (1..100; 50 keeps them, q < 50 scales by 5000/q %, q >= 50 by 200-2q %,
 *     each entry rounded and kept in [1, 255]).  Subsampling 0, 1, 2: 4:4:4,
 *     4:2:2, 4:2:0 (Y sampled 1x1, 2x1, 2x2; Cb and Cr 1x1).
 *   An fp32 inverse or forward DCT value that lies within about 2^-18 x the
 *   block's sum of |coefficients| (or |samples - 128|) of a rounding
 *   boundary may round the other way than the exact transform would.
 *
 * Coefficient layout (host buffers below and the device buffers inside):
 * int16, natural (row-major) order, 64 per block; component c's block (bx,
 * by) of its MCU-padded grid at (first_block[c] + by * blocks_w[c] + bx) x 64.
 * ------------------------------------------------------------------------- */
typedef struct oilpaint_jpeg_info {
    int32_t width, height, components;
    int32_t h_samp[3], v_samp[3];          /* sampling factors */
    int32_t comp_width[3], comp_height[3]; /* samples of each component */
    int32_t blocks_w[3], blocks_h[3];      /* its MCU-padded block grid */
    int32_t first_block[3];                /* its first block in the coefficient layout */
    int64_t blocks;                        /* blocks of all components */
    int32_t restart_interval, scans;
} oilpaint_jpeg_info;

/* Parse a JPEG file's headers (host memory; pure host work). */
int oilpaint_jpeg_header(const uint8_t *data, size_t len, oilpaint_jpeg_info *info);
/* Entropy-decode every scan into host memory `coef` (the layout above;
 * blocks no scan covers are 0).  *count receives the number of
 * coefficients; ERR_NOMEM (nothing written) if capacity is smaller.  Pure
 * host work. */
int oilpaint_jpeg_coefficients(const uint8_t *data, size_t len, int16_t *coef, size_t capacity, size_t *count);
/* Decode a JPEG file (host memory) into dst, interleaved RGB on the device
 * (rows dst_stride >= 3 x width bytes apart; bytes past 3 x width are not
 * written).  The call waits on `stream` for the Huffman decoding (to report
 * a malformed stream as ERR_ARG); the inverse DCT and colour kernels are
 * left enqueued on it.  *host_ms, if not NULL, receives the host time of
 * parsing, stripping the markers and planning the subsequences.  The
 * library keeps the coefficient and sample buffers per device (grown as
 * needed); a call waits for the previous call's work on them.  The
 * coefficients are those oilpaint_jpeg_coefficients gives. */
int oilpaint_jpeg_decode(const uint8_t *data, size_t len, uint8_t *dst, int dst_stride, void *stream,
                         double *host_ms);
/* The same without colour conversion: each component's own samples
 * (comp_width x comp_height) into planes[c] (device memory, rows strides[c]
 * >= comp_width bytes apart). */
int oilpaint_jpeg_decode_planes(const uint8_t *data, size_t len, uint8_t *const *planes, const int *strides,
                                void *stream, double *host_ms);
/* Length in bits of the subsequences the device's Huffman decoding splits
 * the data into, 64 .. 16384, or 0 (the default): chosen per scan, about
 * 0.35 x the square root of its data bits in multiples of 64 within
 * 128 .. 1024 (ERR_ARG otherwise).  Shorter ones give more threads, each
 * with less to decode, and more links to follow.  Process-wide. */
int oilpaint_jpeg_set_subsequence_bits(int bits);
/* Encode width x height interleaved RGB (device memory, rows `stride` bytes
 * apart) as a JFIF file into `out` (host memory).  *out_len receives the
 * file's length; ERR_NOMEM if it exceeds `capacity` (out untouched).  The
 * kernels and the downloads run on `stream`, which the call synchronizes
 * (twice: for the symbol counts and for the coded stream); *host_ms, if not
 * NULL, receives the host time of fitting the tables and writing the
 * headers.  The same coefficients give the same bytes as
 * oilpaint_jpeg_write. */
int oilpaint_jpeg_encode(const uint8_t *src, int width, int height, int stride, int quality, int subsampling,
                         uint8_t *out, size_t capacity, size_t *out_len, void *stream, double *host_ms);
/* A capacity always large enough for oilpaint_jpeg_encode of that size. */
size_t oilpaint_jpeg_encode_bound(int width, int height);
/* The frame oilpaint_jpeg_encode writes for these arguments (its block
 * layout). */
int oilpaint_jpeg_encode_info(int width, int height, int quality, int subsampling, oilpaint_jpeg_info *info);
/* The encoder's host half: entropy-code quantized coefficients (host memory,
 * the layout of oilpaint_jpeg_encode_info's frame) into a JFIF file.  Pure
 * host work. */
int oilpaint_jpeg_write(const int16_t *coef, int width, int height, int quality, int subsampling, uint8_t *out,
                        size_t capacity, size_t *out_len);

/* ---------------------------------------------------------------------------
 * LDS rate probe (measurement, not part of the filter).  The filter's sliding
 * window is bound by LDS instruction throughput (its bin updates are 64-bit
 * LDS atomics, its mode search reads bins from LDS); this probe measures the
 * rates its roofline is priced against on the GPU at hand.
 * ------------------------------------------------------------------------- */
#define OILPAINT_PROBE_READ64 0 /* 8-byte LDS reads, 64 consecutive words per instruction */
#define OILPAINT_PROBE_ADD64 1  /* 64-bit LDS atomic adds, result unused */
#define OILPAINT_PROBE_READ32 2 /* 4-byte LDS reads */

/* Enqueue on `stream` a kernel of per_cu (1..4) workgroups of 256 lanes per
 * CU, each holding 32 KB of LDS; each of its four wavefronts issues iters x 16
 * 64-lane LDS operations of kind `kind` (OILPAINT_PROBE_*) on distinct
 * words.  Workgroup w writes, from its first wavefront between two barriers
 * around the loop, the shader clock (s_memtime) at start and end and the
 * 100 MHz real-time counter at start and end to clocks[4w .. 4w+3] (device
 * memory, at least 4 x max_workgroups uint64).  *workgroups receives the
 * grid size (per_cu x CUs); ERR_ARG if it exceeds max_workgroups or an
 * argument is out of range, ERR_NOT_DEVICE if clocks is not device memory. */
int oilpaint_lds_probe(int kind, int iters, int per_cu, uint64_t *clocks, int max_workgroups, int *workgroups,
                       void *stream);

#ifdef __cplusplus
}
#endif

#endif /* OILPAINT_H */
