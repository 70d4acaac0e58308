/*
 * conv_sep5.h -- C ABI of the width-5 separable image convolution library
 * (libconvsep5.so) for AMD Instinct MI355X (gfx950).
 *
 * The operation (arXiv 1711.09791, Section 1, Eq. 1 with the separable kernel
 * K[i][j] = k_i k_j defined right after it):
 *
 *     B[p][y][x] = sum_{i=-2..2} sum_{j=-2..2} A[p][y+i][x+j] * k[i+2] * k[j+2]
 *
 * for every plane p and every pixel whose 5x5 neighbourhood lies inside the
 * image (2 <= y < rows-2, 2 <= x < cols-2; Section 5 starts the convolution at
 * pixel (2,2) and ignores the edges).  Every other output pixel (the 2-pixel
 * frame) is written as +0.0.  The form is a correlation: k[0] weights the
 * neighbour at offset -2 (the tap order of the paper's listings in
 * Sections 5.3 and 5.4).  Images smaller than 5 in either dimension have no
 * interior and come out all zeros.
 *
 * Arithmetic: FP32 accumulation in every storage type.  The horizontal and the
 * vertical 5-tap filters are each one multiply followed by four fused
 * multiply-adds in tap order k[0]..k[4].  The two-pass and the fused one-pass
 * forms perform the same operations on the same values, so their outputs are
 * bitwise identical; so are the batched, graph-replayed and served results
 * for the same image and taps.  The direct 25-tap mode (the paper's
 * single-pass arithmetic, Section 5.2, Eq. 2 / Eq. 3) rounds K[a][b] once
 * to FP32 on the host, runs a 5-term FMA chain per kernel row and adds the
 * five row partials pairwise.
 *
 * Conventions shared by every entry point:
 *  - Device pointers are plain HIP device addresses (for example the data
 *    pointer of a torch tensor); the caller owns them and keeps them alive
 *    until the stream work completes (or, for the server, until poll reports
 *    the ticket done).  Host arrays (taps, descriptors) are copied before the
 *    call returns.
 *  - Calls only enqueue work on the given stream (NULL = the default stream of
 *    the current device); nothing synchronises except conv_serve_destroy and
 *    the tuner.  All work runs on the device current at call time.
 *  - Arguments are validated before any HIP call.  Errors are returned as a
 *    conv_status; a thread-local message is available from conv_last_error().
 *    No C++ exception crosses this boundary.
 */
#ifndef CONV_SEP5_H
#define CONV_SEP5_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CONV_OK = 0,
    CONV_EINVAL = -1,    /* bad argument (null pointer, bad shape, dtype, mode) */
    CONV_EALIAS = -2,    /* input and output (or workspace) byte ranges overlap */
    CONV_ENOMEM = -3,    /* allocation failed / request larger than a budget   */
    CONV_EHIP = -4,      /* a HIP runtime call or kernel launch failed          */
    CONV_EAGAIN = -5,    /* serving: the ticket is still pending                */
    CONV_ENOTFOUND = -6  /* serving: unknown (or already reported) ticket       */
} conv_status;

/* Storage type of the input and output image.  Accumulation is FP32 always. */
typedef enum { CONV_F32 = 0, CONV_F16 = 1, CONV_BF16 = 2 } conv_dtype;

/*
 * Image descriptor (the paper's planes/rows/cols image record, Section 5.3,
 * with planar [plane][row][col] storage, Section 5.2 Eq. 2, and the flat
 * index p*rows*cols + r*cols + c of Section 5.4 generalised by strides).
 * Element (p, y, x) lives at base + p*plane_stride + y*pitch + x, counted in
 * elements of `dtype`.  The same layout applies to the input and the output.
 *   planes       >= 0 (3 colour planes in the paper's workload)
 *   rows, cols   >= 0 (any of planes/rows/cols == 0 means "nothing to do")
 *   pitch        elements between rows; 0 means cols; otherwise >= cols
 *   plane_stride elements between planes; 0 means rows*pitch; otherwise
 *                either >= (rows-1)*pitch + cols (planar), or >= cols with
 *                (planes-1)*plane_stride + cols <= pitch: the planes' rows
 *                side by side in one row (the row-interleaved "3R x C"
 *                layout of Section 6).  Each plane keeps its own border.
 *                1 with 2..4 planes: planes interleaved per pixel (packed
 *                HWC, e.g. RGB): element (p, y, x) at y*pitch + x*planes + p,
 *                pitch >= cols*planes (0 means cols*planes).  Each channel is
 *                convolved on its own with its own border, bitwise as in the
 *                planar layout.  Taken by conv_sep5_1pass and conv_sep5_2pass
 *                (the two-pass workspace then holds HWC rows); the other
 *                entry points return CONV_EINVAL for it.
 * The fast path needs 16-byte aligned base pointers and cols, pitch and
 * plane_stride (HWC: cols*planes and pitch) that are multiples of
 * 16/sizeof(element); other layouts run a slower element-wise path with
 * identical results.  Rows that start on a 128-byte line run fastest (each
 * wave reads and writes 1 KB of a row): a pitch of a multiple of 128 bytes
 * gives that for every row.
 */
typedef struct {
    int32_t planes;
    int32_t rows;
    int32_t cols;
    int32_t dtype;        /* conv_dtype */
    int64_t pitch;
    int64_t plane_stride;
} conv_image;

/* conv_sep5_1pass modes. */
enum {
    CONV_1PASS_FUSED = 0,    /* row-filtered intermediate kept in registers */
    CONV_1PASS_DIRECT25 = 1  /* 25 multiply-adds per pixel (Eq. 2 / Eq. 3)  */
};

/*
 * Two-pass form (Section 5.1, "two-pass algorithm"; Section 5.3 and 5.4
 * listings): a row kernel filters every row of every plane horizontally into
 * the FP32 workspace `d_tmp`, then a column kernel filters it vertically into
 * `d_out`.  The two kernels are ordered on `stream` (the analogue of the
 * barrier between the passes).
 *   d_in, d_out  device images described by *img; d_out == d_in is allowed
 *                (the paper's in-place two-pass, Section 7) -- any other
 *                partial overlap is CONV_EALIAS.
 *   d_tmp        FP32 workspace of planes*rows*cols floats, dense
 *                [plane][row][col]; must not overlap d_in or d_out.  NULL
 *                makes the library take stream-ordered memory for it
 *                (hipMallocAsync / hipFreeAsync on `stream`).
 *   k            5 FP32 taps (host array).
 */
conv_status conv_sep5_2pass(const void *d_in, void *d_out, float *d_tmp,
                            const float k[5], const conv_image *img,
                            hipStream_t stream);

/*
 * Two-pass form with the intermediate stored as tmp_dtype.  The paper's
 * auxiliary array (Section 7) is float, which CONV_F32 gives (identical to
 * conv_sep5_2pass).  CONV_F16 / CONV_BF16 keep it in 16 bits: each row-filter
 * value is computed in FP32 as in the FP32 form and rounded once to the
 * 16-bit format (round to nearest even) before the column pass reads it.
 * That halves the intermediate's bytes (2 + 2 instead of 4 + 4 per
 * plane-pixel) but adds one rounding per intermediate value: the result is
 * not bitwise equal to the FP32 form.  Its definition is the two-pass sum with
 * each intermediate rounded once; the deviation of one FP32 row chain near a
 * 16-bit rounding midpoint can move that intermediate by one 16-bit unit.
 *   d_in, d_out  as conv_sep5_2pass (d_out == d_in allowed)
 *   d_tmp        workspace of planes*rows*cols values of tmp_dtype, dense
 *                [plane][row][col]; must not overlap d_in or d_out; NULL:
 *                stream-ordered library memory
 *   k            5 FP32 taps (host array)
 *   tmp_dtype    CONV_F32, CONV_F16 or CONV_BF16; pixel-interleaved images
 *                (plane_stride 1) take CONV_F32 only (else CONV_EINVAL)
 * Launches run with one wave per workgroup and the configured rows per tile
 * and XCD order.
 */
conv_status conv_sep5_2pass_ex(const void *d_in, void *d_out, void *d_tmp,
                               const float k[5], const conv_image *img,
                               int32_t tmp_dtype, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the two-pass
 * form of conv_sep5_2pass_ex with its intermediate held in a static device
 * array of the library, CONV_NOALLOC_SCRATCH_BYTES (128 MiB) per GPU, which a
 * GPU holds from the library's first use on it until the process ends.  The
 * call allocates nothing (no hipMalloc, hipMallocAsync, hipFree or allocating
 * library routine) and computes exactly what conv_sep5_2pass_ex computes with
 * a caller's workspace, bitwise.
 *   d_in, d_out, k, img  as conv_sep5_2pass_ex (d_out == d_in allowed)
 *   tmp_dtype    CONV_F32, CONV_F16 or CONV_BF16, as conv_sep5_2pass_ex
 * An intermediate larger than the array (planes*rows*cols*4 bytes for
 * CONV_F32, *2 for the 16-bit types; 128 MiB holds 3 x 3840 x 2160 in FP32)
 * is CONV_ENOMEM, checked before any HIP call.  Every call on one GPU uses
 * that GPU's one array, and the array keeps the last call's contents (the row
 * pass writes every value the column pass reads, so nothing is cleared):
 * calls ordered on one stream are safe; calls that can overlap on one GPU
 * (different streams, or threads without stream ordering between them) race
 * on the array and give wrong results.
 */
#define CONV_NOALLOC_SCRATCH_BYTES (128ull << 20)
conv_status conv_sep5_2pass_noalloc(const void *d_in, void *d_out, const float k[5],
                                    const conv_image *img, int32_t tmp_dtype,
                                    hipStream_t stream);

/*
 * Single-pass form (Section 5.1 and Section 7, "single-pass without
 * copy-back": the result is written once to a separate output).  One kernel;
 * mode CONV_1PASS_FUSED keeps the row-filtered rows in registers, mode
 * CONV_1PASS_DIRECT25 evaluates the 25-term sum of Eq. 2.
 *   d_in, d_out  device images described by *img.  d_out == d_in selects the
 *                paper's single-pass WITH copy-back (Section 5.2, Section 7):
 *                the result goes to stream-ordered scratch (hipMallocAsync /
 *                hipFreeAsync on `stream`) and a copy kernel writes it over
 *                the input -- 16 B per plane-pixel instead of 8.  Any other
 *                overlap is CONV_EALIAS.
 *   k            5 FP32 taps (host array).
 */
conv_status conv_sep5_1pass(const void *d_in, void *d_out, const float k[5],
                            const conv_image *img, int mode,
                            hipStream_t stream);

/*
 * Image copy: every element of the image described by *img is copied from
 * d_in to d_out (same layout), by the streaming tile kernel that performs the
 * copy-back step of the single pass with copy-back (Section 7: the result
 * built in B is copied back into A).  It moves the same bytes per
 * plane-pixel as a fused single pass without the filter, so it is also the
 * achievable-bandwidth reference for the convolution kernels.
 *   d_in, d_out  device images; d_out == d_in does nothing; any other
 *                overlap is CONV_EALIAS.
 */
conv_status conv_image_copy(const void *d_in, void *d_out, const conv_image *img,
                            hipStream_t stream);

/*
 * Many images of different sizes in ONE kernel launch (the device-side
 * counterpart of the paper's task agglomeration over planes, Section 6): one
 * workgroup per tile by default, a persistent grid when the batch tile
 * configuration asks for one (persist_wgs_per_cu > 0).  All images must share one dtype; each has its own taps.
 *   n            number of images (>= 0; 0 enqueues nothing)
 *   d_in, d_out  host arrays of n device pointers
 *   k            host array of n*5 FP32 taps (image i uses k[5i .. 5i+4])
 *   imgs         host array of n descriptors
 *   mode         CONV_1PASS_FUSED or CONV_1PASS_DIRECT25
 * Each output must not overlap its own input or any other image's output.
 * Up to 16 images, the per-image descriptors ride in the kernel argument;
 * a larger batch stages its descriptor table through a library-owned pinned
 * ring, copied to device memory on `stream`.
 */
conv_status conv_sep5_batch(int32_t n, const void *const *d_in,
                            void *const *d_out, const float *k,
                            const conv_image *imgs, int mode,
                            hipStream_t stream);

/*
 * A batch bound once to fixed buffers and replayed as a captured hipGraph.
 * plan_create validates like conv_sep5_batch, uploads the descriptor table to
 * library-owned device memory and captures the launch; plan_launch replays
 * the graph on `stream`; plan_destroy frees the plan (the caller must make
 * sure no replay is still running).
 */
typedef struct conv_plan conv_plan;
conv_status conv_batch_plan_create(int32_t n, const void *const *d_in,
                                   void *const *d_out, const float *k,
                                   const conv_image *imgs, int mode,
                                   conv_plan **plan);
conv_status conv_batch_plan_launch(conv_plan *plan, hipStream_t stream);
conv_status conv_batch_plan_destroy(conv_plan *plan);

/*
 * Any odd width n = 2r+1, 1 <= n <= CONV_MAX_WIDTH (the paper fixes n = 5;
 * Section 5.1 weighs the O(n) work per pixel of the separable passes against
 * the O(n^2) of the direct sum, which these entry points let a caller measure
 * at every width).  Same image descriptor, storage types and conventions as
 * the width-5 entry points; the frame of r pixels is written as +0.0 and an
 * image smaller than n in either dimension comes out all zeros.
 * Arithmetic: each 1-D filter is one multiply and n-1 fused multiply-adds in
 * tap order; the direct form runs an n-term FMA chain per kernel row and adds
 * the n row partials pairwise (the first half of every split is the largest
 * power of two below its length).  At n = 5 this is exactly the arithmetic of
 * conv_sep5_1pass / conv_sep5_2pass, and the results are bitwise equal.
 * Returns CONV_EINVAL for an even n or n outside 1..CONV_MAX_WIDTH.
 */
#define CONV_MAX_WIDTH 9

/*
 * Width-n separable single pass (Eq. 1 with K = k k^T).  mode
 * CONV_1PASS_FUSED keeps the row-filtered rows in registers; mode
 * CONV_1PASS_DIRECT25 evaluates the n*n-term sum with K[a][b] = k[a]*k[b]
 * rounded once to FP32 on the host.  d_out == d_in runs the single pass with
 * copy-back, as in conv_sep5_1pass.
 *   k   n FP32 taps (host array); k[0] weights the neighbour at offset -r.
 */
conv_status conv_sepn_1pass(const void *d_in, void *d_out, const float *k,
                            int32_t n, const conv_image *img, int mode,
                            hipStream_t stream);

/*
 * Width-n two-pass form (Section 5.1): row kernel into the FP32 workspace
 * d_tmp (planes*rows*cols floats, or NULL for stream-ordered scratch), then
 * column kernel into d_out.  Aliasing rules as conv_sep5_2pass.
 */
conv_status conv_sepn_2pass(const void *d_in, void *d_out, float *d_tmp,
                            const float *k, int32_t n, const conv_image *img,
                            hipStream_t stream);

/*
 * Direct width-n convolution with a full, not necessarily separable kernel
 * (Eq. 1 as written, before the separable restriction that follows it):
 *   B[p][y][x] = sum_{a=0..n-1} sum_{b=0..n-1} A[p][y+a-r][x+b-r] * K[a*n+b]
 *   K   n*n FP32 weights, row-major (host array).
 * d_out == d_in runs with copy-back.
 */
conv_status conv_2d_direct(const void *d_in, void *d_out, const float *K,
                           int32_t n, const conv_image *img,
                           hipStream_t stream);

/*
 * One Gaussian-pyramid level: blur with the width-5 separable kernel, then
 * keep every second row and column.  The paper names image scaling as the
 * step of its stereo-matching application next to the convolution (Section
 * 1) without defining it; this is the blur-then-decimate reading:
 *     out[p][yo][xo] = B[p][2*yo][2*xo],  0 <= yo < ceil(rows/2),
 *                                         0 <= xo < ceil(cols/2)
 * with B the convolution of conv_sep5_1pass (same FMA chains, zero frame), so
 * the result equals conv_sep5_1pass's output at the sampled pixels bitwise.
 * One fused kernel: the input is read once and only the sampled outputs are
 * computed and written (1 + 1/4 of the image's bytes).
 *   d_in, in_img    input image (any layout accepted by conv_image)
 *   d_out, out_img  output image: same dtype and planes, rows = ceil(rows/2),
 *                   cols = ceil(cols/2), its own pitch and plane_stride;
 *                   must not overlap the input (CONV_EALIAS)
 *   k               5 FP32 taps (host array)
 */
conv_status conv_pyr_down(const void *d_in, const conv_image *in_img,
                          void *d_out, const conv_image *out_img,
                          const float k[5], hipStream_t stream);

/*
 * Tile configuration (the autotuner's search space).  Results never depend on
 * it: every configuration gives bitwise identical output.
 *   rows_per_tile  output rows a wavefront walks down per tile (4..4096)
 *   waves_per_wg   wavefronts per workgroup, each on its own column strip
 *                  (1, 2 or 4)
 *   persist_wgs_per_cu  batch kernel: resident workgroups per compute unit
 *                  (1..32), the persistent grid being this times the CU
 *                  count; 0: one workgroup per tile (up to 2^20 of them)
 *   xcd_slabs      0: workgroups take tiles in launch order, so the resident
 *                  waves sweep the image (or batch) as one compact window;
 *                  1: each of the 8 XCDs takes one contiguous slab of tiles
 *                  (full rows), so horizontal halos stay in that XCD's L2;
 *                  c in 2..4096: the XCDs take turns on chunks of c full
 *                  band rows (batch kernel: of 8c consecutive tiles), so
 *                  horizontal halos and all but one band boundary per chunk
 *                  stay in one L2
 *   pack_tail      fused (and FP32 direct25) launches with one wave per
 *                  workgroup and 4- or 8-row bands, aligned images: a last
 *                  column strip of at most a half (quarter) of a wave's width
 *                  is taken by one wave for 2 (4) bands at once.
 *                  0: when the launch has more tiles than the GPU holds at
 *                  once (16 per compute unit); 1: always; -1: never
 */
typedef struct {
    int32_t rows_per_tile;
    int32_t waves_per_wg;
    int32_t persist_wgs_per_cu;
    int32_t xcd_slabs;
    int32_t pack_tail;
} conv_tile_cfg;

/*
 * kind: 0 = single-image kernels (fused 1pass, 2pass, image copy), 1 = batch
 * kernel, 2 = single-image direct 25-tap kernel (CONV_1PASS_DIRECT25, which
 * is bound by its vector ALU work rather than by memory; its 16-bit defaults
 * are 16-row bands).
 * get/set address the default configuration of (dtype, kind).  set also
 * drops what the tuner installed for (dtype, kind), so an explicit
 * configuration applies to every workload size.
 */
conv_status conv_get_tile_cfg(int32_t dtype, int32_t kind, conv_tile_cfg *cfg);
conv_status conv_set_tile_cfg(int32_t dtype, int32_t kind, const conv_tile_cfg *cfg);

/*
 * The configuration a call of (dtype, kind) whose input plus output bytes
 * (summed over a batch) are footprint_bytes runs with: the tuner's choice for
 * that size class if one is installed (*tuned = 1), else the default
 * (*tuned = 0; tuned may be NULL).  Size classes: <= 64 MiB, <= 256 MiB (the
 * GPU's last-level cache), <= 1 GiB, larger.
 */
conv_status conv_get_tile_cfg_for(int32_t dtype, int32_t kind, uint64_t footprint_bytes,
                                  conv_tile_cfg *cfg, int32_t *tuned);

/*
 * Autotuner (the paper points to auto-tuning for performance portability,
 * Section 3.2): times every candidate configuration of `kind` on the given
 * workload with HIP events (`reps` timed launches each, after one warm-up),
 * installs the fastest for the workload's storage type, kind and size class
 * and returns it in *best, with its median time per launch in *best_ms.
 * kind 0 tunes on image 0 alone (fused 1pass), kind 2 on image 0 alone
 * (direct 25-tap 1pass), kind 1 on the whole batch.
 * Synchronises `stream`.  Calls of other size classes keep their own choice.
 * The launches reuse the same buffers, so a workload whose input and output
 * fit the GPU's 256 MB last-level cache is timed with a warm cache (where
 * other tile orders win than for images streamed from HBM).
 * If the environment variable CONV_TUNE_CACHE names a file, every installed
 * choice is written to it after the run (conv_tune_save).
 */
conv_status conv_tune(int32_t kind, int32_t n, const void *const *d_in,
                      void *const *d_out, const float *k,
                      const conv_image *imgs, int32_t reps,
                      hipStream_t stream, conv_tile_cfg *best, float *best_ms);

/*
 * Tuner cache.  save writes every installed tuner choice to `path` as JSON
 * ({"format": "convsep5-tune-1", "entries": [{"dtype", "kind", "size_class",
 * the five conv_tile_cfg fields, "ms"}, ...]}), replacing the file
 * atomically.  load reads such a file and installs its entries (all or
 * nothing: a malformed file or an out-of-range entry is CONV_EINVAL and
 * changes nothing; a missing file is CONV_ENOTFOUND).  The file named by
 * CONV_TUNE_CACHE, if any, is loaded at the library's first use.
 */
conv_status conv_tune_save(const char *path);
conv_status conv_tune_load(const char *path);

/* ---------------------------------------------------------------------------
 * Continuous-batching server.  A scheduler thread admits submitted requests in
 * arrival order while a slot is free and their HBM footprint (input + output
 * bytes) fits the budget, packs the requests admitted together into one
 * launch on the next idle stream (the batch kernel; a lone request runs the
 * single-image kernel), and retires requests when a one-lane kernel that the
 * stream runs after the launch has written the launch's token into its
 * completion word (pinned host memory).  Requests that arrive while others run
 * are admitted into the next launch, on another stream, so their work overlaps
 * on the device.
 * Each result is bitwise identical to a lone conv_sep5_1pass (fused) call.
 * The queue is host memory (request descriptors); the images stay in device
 * memory throughout.
 * Ordering: requests whose buffers overlap run in submission order.  A
 * request that reads bytes an earlier, not yet completed request writes, or
 * writes bytes such a request reads or writes (a chained pair: B's input is
 * A's output; a shared output), is not admitted until that earlier request
 * has completed, and never shares its launch; admission waits for it (later
 * requests queue behind it).  A request's own input and output must not
 * overlap (CONV_EALIAS at submit).
 */
typedef struct {
    uint64_t hbm_budget_bytes; /* max sum of footprints in flight (> 0)      */
    int32_t max_slots;         /* max requests in flight (>= 1)              */
    int32_t n_streams;         /* launch streams (1..16)                     */
    int32_t max_batch;         /* max requests per launch (>= 1)             */
    int32_t device;            /* HIP device ordinal (-1: current device)    */
    uint64_t max_batch_bytes;  /* max footprint per launch (0: no limit); a
                                  request larger than this runs alone      */
    int32_t producer_wait;     /* 1: order each launch after the submitters'
                                  streams (an event per submit, see
                                  conv_serve_submit); 0: the caller promises
                                  every input is complete when it submits  */
    int32_t queue_only;        /* 0: a submit that finds nothing queued and
                                  a stream idle launches its request itself
                                  (the scheduler retires it) while submits
                                  are sparse (the running mean gap and the
                                  gap before this submit >= 8 us, about one
                                  launch's enqueue time); dense arrivals go
                                  to the scheduler, which batches them;
                                  1: every launch is made by the scheduler */
    int32_t launch_depth;      /* launches in flight per stream (0..4; 0 and
                                  1: one, the next group is admitted when it
                                  completes; 2..4: a group may also be
                                  queued behind a running launch, so the
                                  stream starts it without a host round
                                  trip)                                     */
} conv_serve_cfg;

typedef struct {
    uint64_t submit_ns;  /* host CLOCK_MONOTONIC at submit                    */
    uint64_t admit_ns;   /* when it was admitted into a launch                */
    uint64_t launch_ns;  /* when that launch was enqueued                     */
    uint64_t done_ns;    /* when the scheduler saw the launch's event done    */
    int32_t batch_size;  /* requests in its launch                            */
    int32_t stream;      /* index of the stream it ran on                     */
} conv_req_times;

typedef struct conv_server conv_server;

conv_status conv_serve_create(const conv_serve_cfg *cfg, conv_server **srv);
/* Non-blocking (it never waits for the GPU; with queue_only = 0 it may
 * enqueue the request's launch itself, see conv_serve_cfg).  d_in/d_out:
 * device image (FP32/FP16/BF16) as in
 * conv_sep5_1pass; k: 5 host taps.  `stream` is the caller's producer stream
 * (NULL: the default stream): with producer_wait = 1, work enqueued on it
 * before this call -- the writes that fill d_in, say -- completes before the
 * request's kernel starts (an event is recorded on it here and waited on by
 * the launch); with producer_wait = 0 it is ignored.  Footprint
 * larger than the budget -> CONV_ENOMEM; bad arguments -> CONV_EINVAL /
 * CONV_EALIAS.  *ticket > 0. */
conv_status conv_serve_submit(conv_server *srv, const void *d_in, void *d_out,
                              const float k[5], const conv_image *img,
                              hipStream_t stream, uint64_t *ticket);
/* CONV_OK: done (times filled if t != NULL; the ticket is then forgotten);
 * CONV_EAGAIN: pending; CONV_ENOTFOUND: unknown ticket; CONV_EHIP: its launch
 * failed. */
conv_status conv_serve_poll(conv_server *srv, uint64_t ticket,
                            conv_req_times *t);
/* Blocks until every submitted request has completed. */
conv_status conv_serve_drain(conv_server *srv);

/* Counters since creation (for tests and benchmarks). */
typedef struct {
    uint64_t submitted;           /* accepted submissions                     */
    uint64_t completed;           /* requests whose launch finished           */
    uint64_t failed;              /* requests whose launch failed             */
    uint64_t launches;            /* launches enqueued                        */
    uint64_t max_bytes_in_flight; /* high-water mark of admitted footprints   */
    int32_t max_slots_in_flight;  /* high-water mark of admitted requests     */
    int32_t max_batch;            /* largest launch                           */
    int32_t max_streams_busy;     /* most launches in flight at once          */
    int32_t direct_launches;      /* launches a submit made itself (of
                                     `launches`; counts to 2^31 - 1)          */
} conv_serve_stats;
conv_status conv_serve_get_stats(conv_server *srv, conv_serve_stats *stats);
/* Drains, stops the scheduler and frees the server. */
conv_status conv_serve_destroy(conv_server *srv);

/* Thread-local description of the last error of this thread ("" if none). */
const char *conv_last_error(void);

/* Library version string. */
const char *conv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CONV_SEP5_H */
