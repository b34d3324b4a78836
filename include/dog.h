/*
 * dog.h - C ABI of the MI355X (gfx950) Difference-of-Gaussians blob detector.
 *
 * The method is the DoG blob detector of arXiv:2010.08486 ("Towards Online
 * Steering of Flame Spray Pyrolysis Nanoparticle Synthesis"):
 *   - scale space L(x, y, sigma) = g(sigma) * I                  (Sec. 3)
 *   - a ladder of standard deviations sigma_i, here geometric:
 *     k = floor(ln(sigma_max/sigma_min)/ln(sigma_ratio)) + 1 DoG planes,
 *     sigma_i = sigma_min * sigma_ratio^i, i = 0..k               (Sec. 4, Eq. 1
 *                                                                  in geometric form)
 *   - Gaussian kernels sampled out to radius floor(truncate*sigma + 0.5),
 *     normalised to sum 1, reflect (half-sample symmetric) borders (Sec. 4.1)
 *   - D_i = sigma_i * (L_i - L_{i+1})                              (Sec. 4, Eq. 2-3;
 *     sign chosen so bright blobs give positive maxima)
 *   - a voxel (i, y, x) is a blob iff D_i(y, x) equals the maximum of its
 *     3x3x3 neighbourhood over (x, y, scale) (neighbours outside the cube
 *     ignored, every tied voxel kept) and D_i(y, x) > threshold (strict)
 *                                                                 (Sec. 4 local-maximum
 *                                                                  heuristic, Sec. 4.1 Thresh)
 *   - blob radius sqrt(2)*sigma_i (Sec. 3); overlap pruning (Sec. 4.1): for
 *     blobs in (y, x, scale) order, pairs whose disk intersection exceeds
 *     `overlap` times the smaller disk's area lose the blob with the smaller
 *     sigma (the later one on a tie).  overlap >= 1 disables pruning.
 *
 * Conventions for every entry point:
 *   - Return value: DOG_OK (0) or a negative DOG_E* code.  On error nothing
 *     is returned through output pointers (they are set to NULL / 0) and
 *     dog_last_error() describes the failure (thread-local string).
 *   - Images are fp32, row-major, `height` rows of `width` pixels, rows
 *     `row_stride` elements apart (row_stride >= width).  Pixels must be
 *     finite.  1 <= height, width <= 32768, height * row_stride < 2^29 and
 *     width * (height + 63) < 2^29 (every plane stays below 2 GiB).
 *   - Blob lists are sorted by (y, x, scale), allocated with malloc by the
 *     library and released with dog_blobs_free().
 *   - Streams are hipStream_t values passed as void*; the sequence is
 *     issued on that stream, after the work already queued there (NULL = the
 *     null stream).  Entry points that return results (blob lists, limits,
 *     planes) return after those results are complete; the two that only
 *     queue work return at once and say so below: dog_detect_device_async,
 *     and dog_preprocess when limits_out is NULL.
 */
#ifndef DOG_H
#define DOG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DOG_OK 0
#define DOG_EINVAL (-1)   /* invalid argument                                  */
#define DOG_ENOMEM (-2)   /* footprint exceeds the HBM budget / allocation failed */
#define DOG_EDEVICE (-3)  /* HIP runtime error (message in dog_last_error)      */
#define DOG_EBUSY (-4)    /* server queue full, or context awaiting finish      */
#define DOG_EAGAIN (-5)   /* server result not ready yet                        */
#define DOG_ENOTFOUND (-6)/* unknown server ticket                              */

/* One detected blob.  y = row, x = column (0-based, the pixel of the DoG
 * maximum); scale = ladder index i (0..k-1); sigma = sigma_i (the lower
 * sigma of the pair, Sec. 4 Eq. 3); response = D_i(y, x) as computed in fp32;
 * the blob radius is sqrt(2)*sigma (Sec. 3). */
typedef struct {
    int32_t y;
    int32_t x;
    int32_t scale;
    float sigma;
    float response;
} dog_blob;

/* Detector hyper-parameters (Sec. 4: min_sigma, max_sigma, n_bin; Sec. 4.1:
 * truncate, threshold default 0.1, overlap default 0.5).  truncate == 0
 * selects 4.0.  Valid: 0 < sigma_min <= sigma_max, finite threshold,
 * 0 <= overlap <= 1, truncate >= 0, at most 63 DoG planes, and
 *   ladder 0 (geometric): sigma_ratio > 1; sigma_i = sigma_min sigma_ratio^i,
 *     k = floor(ln(sigma_max/sigma_min)/ln(sigma_ratio)) + 1 DoG planes;
 *   ladder 1 (arithmetic, Sec. 4 Eq. 1): n_bin >= 1; the n_bin + 1 sigmas
 *     sigma_min + i (sigma_max - sigma_min)/n_bin, i = 0..n_bin, k = n_bin
 *     (sigma_ratio is not used).
 * coalesce 0: of two blobs overlapping more than `overlap`, the one with the
 * smaller sigma is removed; 1: it is coalesced into the other, whose sigma
 * becomes the mean of the two (Sec. 4.1, averaging the radius) and is what
 * later pairs see.  reserved must be 0.  All-zero new fields give the
 * geometric ladder with pruning. */
typedef struct {
    double sigma_min;
    double sigma_max;
    double sigma_ratio;
    double threshold;
    double overlap;
    double truncate;
    int32_t ladder;
    int32_t n_bin;
    int32_t coalesce;
    int32_t reserved;
} dog_params;

/* A frame of a batch or a server request.  on_device = 1: `data` is a device
 * pointer on the context's GPU; 0: a host pointer (copied into the context's
 * pinned staging, then to the device); 2: a pinned host pointer (page-locked,
 * e.g. from hipHostMalloc), copied to the device by DMA with no staging copy. */
typedef struct {
    const float* data;
    int64_t height;
    int64_t width;
    int64_t row_stride;
    int32_t on_device;
    int32_t reserved;
} dog_frame;

/* Per-frame result of a batch or a server request. */
typedef struct {
    dog_blob* blobs;     /* malloc'd, sorted; release with dog_blobs_free   */
    int64_t count;       /* blobs after pruning                            */
    int64_t raw_count;   /* local maxima above threshold, before pruning   */
    int32_t status;      /* DOG_OK or a DOG_E* code for this frame         */
    int32_t reserved;
    int64_t t_arrive_ns; /* server only: submit time (CLOCK_MONOTONIC ns)  */
    int64_t t_done_ns;   /* server only: time the blob list was ready      */
} dog_result;

typedef struct dog_context dog_context;
typedef struct dog_server dog_server;

/* ------------------------------------------------------------ one frame */

/* Whole detector on a HOST image, on device 0 through a library-owned
 * context (created on first use, kept until process exit; calls are
 * serialised).  The image is borrowed for the duration of the call.
 * *blobs_out receives a malloc'd array of *count_out blobs (NULL if 0). */
int dog_detect(const float* image, int64_t height, int64_t width, int64_t row_stride,
               double sigma_min, double sigma_max, double sigma_ratio, double threshold,
               double overlap, dog_blob** blobs_out, int64_t* count_out);

/* Release a blob array returned by the library (NULL is allowed). */
void dog_blobs_free(dog_blob* blobs);

/* Host step on its own: sort blobs[0..n) by (y, x, scale) and apply the
 * overlap pruning above in place (coalescing when params->coalesce is 1),
 * with sigma taken as the FP64 ladder value of each blob's scale index under
 * `params` (the fp32 sigma field is ignored and rewritten; with coalescing
 * it receives the survivor's final sigma).  *n_out receives the surviving
 * count. */
int dog_prune(const dog_params* params, dog_blob* blobs, int64_t n, int64_t* n_out);

/* The overlap step and the radius histogram on the GPU (Sec. 4.1: pruning
 * or coalescing overlapping blobs and histogramming their radii, steps the
 * paper notes could move to the GPU).  d_blobs: n blobs in DEVICE memory on
 * the context's GPU, in any order (their sigma field is ignored; each blob
 * takes the FP64 ladder sigma of its scale index under `params`).  One
 * workgroup sorts them by (y, x, scale) and prunes exactly as dog_prune
 * does (the same visits in the same order, coalescing when
 * params->coalesce is 1), then histograms the survivors as
 * dog_radius_histogram does.  *blobs_out receives the survivors (malloc'd,
 * sorted, sigma = ladder sigma or coalesced mean), *count_out their number,
 * hist_out (host, k int64, may be NULL) the histogram.  Work is queued on
 * `stream` after what is already there; the call returns when the results
 * are on the host.  A list of more blobs (or touching pairs) than one
 * workgroup holds (4096 blobs and 8192 pairs where a workgroup may use
 * 128 KB of LDS) is pruned by the same steps on the host, with the same
 * result.  Errors: DOG_EINVAL (NULL pointers, bad parameters, a blob with
 * y or x outside [0, 32768) or a scale outside the ladder), DOG_EBUSY,
 * device errors. */
int dog_prune_device(dog_context* ctx, const dog_params* params, const dog_blob* d_blobs,
                     int64_t n, void* stream, dog_blob** blobs_out, int64_t* count_out,
                     int64_t* hist_out);

/* Radius histogram (Sec. 4.1: blobs are histogrammed with bin centres at
 * the detectable radii sqrt(2) sigma_i of the ladder's k DoG scales):
 * counts_out[0..k) receives, for each scale, the number of blobs[0..n)
 * whose radius sqrt(2) sigma (their sigma field, ladder values or coalesced
 * means) is nearest that scale's, the lower scale on a tie.  k as in
 * dog_plan_info.  DOG_EINVAL on NULL pointers, bad parameters or a
 * non-finite sigma. */
int dog_radius_histogram(const dog_params* params, const dog_blob* blobs, int64_t n,
                         int64_t* counts_out);

/* Description of the last error on the calling thread ("" if none). */
const char* dog_last_error(void);

/* Library and kernel version string. */
const char* dog_version(void);

/* ------------------------------------------------------------ contexts */

/* A context owns device workspace (scale-space planes, candidate buffer,
 * launch tables), pinned host staging and a stream on GPU `device`.
 * hbm_budget_bytes caps the device memory it allocates (0 = 90% of the free
 * memory at creation).  A context is not thread-safe. */
int dog_context_create(int device, uint64_t hbm_budget_bytes, dog_context** ctx);
void dog_context_destroy(dog_context* ctx);

/* The ladder these parameters produce: *k_out DoG planes, and (when the
 * arrays are non-NULL and cap >= k+1) the k+1 sigmas and kernel radii. */
int dog_plan_info(const dog_params* params, int32_t* k_out, double* sigmas_out,
                  int32_t* radii_out, int32_t cap);

/* Device bytes the context would need to hold a batch of n_frames frames of
 * the given shapes at these parameters (planes + tables + candidates). */
int dog_footprint(const dog_params* params, int32_t n_frames, const int64_t* heights,
                  const int64_t* widths, uint64_t* bytes_out);

/* Whole detector on a DEVICE image (d_image on the context's GPU, valid until
 * the call returns).  Work is issued on `stream` (hipStream_t, NULL = the
 * null stream); the call returns after the blob list is on the host. */
int dog_detect_device(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                      int64_t row_stride, const dog_params* params, void* stream,
                      dog_blob** blobs_out, int64_t* count_out);

/* dog_detect_device in two halves, so a caller can queue the next frame's
 * work, or do its own, while the host finishes this one (the device steps
 * of Sec. 4.1, then the host sort and its overlap pruning).
 * dog_detect_device_async queues the detector on `stream` (as above) and
 * returns without waiting; d_image must stay valid and unchanged until the
 * stream has passed the launch.  dog_detect_device_finish waits for it and
 * returns the pruned blob list exactly as dog_detect_device would.  One
 * launch per context at a time: until finish, every other call on the
 * context returns DOG_EBUSY (dog_context_destroy waits for the launch);
 * finish with nothing launched returns DOG_EINVAL.  Pipelining takes two
 * contexts, used in turn. */
int dog_detect_device_async(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                            int64_t row_stride, const dog_params* params, void* stream);
int dog_detect_device_finish(dog_context* ctx, dog_blob** blobs_out, int64_t* count_out);

/* Preprocessing (Sec. 4.1, the optional first step): Gaussian smoothing of
 * the device image (sigma smooth_sigma, radius floor(4 sigma + 0.5) <= 16,
 * normalised weights, half-sample reflection; 0 = no smoothing), then a
 * contrast stretch to [0, 1] that saturates the fraction `saturated` of the
 * pixels (the paper uses 0.0035), half at each end: with N pixels and
 * m = floor(saturated N / 2), lo and hi are the m-th smallest and m-th
 * largest smoothed values (exact order statistics of the fp32 smoothed
 * image), and d_out = clamp((S - lo)/(hi - lo), 0, 1), or 0 where hi == lo.
 * d_out (device, height x width, dense rows) receives the result and may
 * then go to dog_detect_device on the same stream; d_smoothed (device, same
 * shape, may be NULL) receives S.  Work is queued on `stream` as in
 * dog_detect_device; if limits_out (host, 2 floats) is non-NULL the call
 * waits and stores lo and hi there, else it returns without waiting.
 * d_image and the outputs must not overlap.  Successive calls on one
 * context share its scratch: a call on another stream waits on the device
 * for the previous one.  Errors: DOG_EINVAL (bad
 * pointer, shape, sigma or fraction; radius above 16), DOG_EBUSY (a launch
 * of dog_detect_device_async not finished), device errors. */
int dog_preprocess(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                   int64_t row_stride, double smooth_sigma, double saturated, float* d_out,
                   float* d_smoothed, float* limits_out, void* stream);

/* dog_preprocess for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with no context.  Its select state,
 * histograms and weights (about 265 KB) live in a static device array, one
 * per GPU, held until the process ends; the call allocates nothing
 * (no hipMalloc, hipFree, pinned or heap memory), uploads nothing and never
 * waits.  It runs on the calling thread's current device, on `stream` (a
 * stream of that device; NULL = the null stream): a fill kernel clears the
 * histograms and stores the weights, then the four preprocessing kernels.
 * d_image, d_out and d_smoothed as in dog_preprocess.  d_limits (device, 2
 * floats, may be NULL) receives lo and hi once the stream has passed the
 * call.  Calls that overlap on one GPU (other streams, other threads) share
 * the array and race: the caller orders them.  Limits: the image bounds of
 * every entry point (height * row_stride < 2^29) and a smoothing radius of
 * at most 16; beyond them DOG_EINVAL with a message.  Errors: DOG_EINVAL,
 * DOG_EDEVICE. */
int dog_preprocess_noalloc(const float* d_image, int64_t height, int64_t width,
                           int64_t row_stride, double smooth_sigma, double saturated,
                           float* d_out, float* d_smoothed, float* d_limits, void* stream);

/* Whole detector on n_frames frames of any sizes.  The frames are cut into
 * consecutive groups of at most dog_set_batch_grouping's pixel count (by
 * default 2^20, one 1024x1024 frame; a larger frame forms a group alone),
 * and each group is one launch sequence (three kernels over tile tables
 * built for it) on one of the context's lanes: child contexts with their own
 * streams and workspaces, so several groups run at once and each group's
 * planes stay close to the Infinity Cache between its kernels.  The lanes
 * start after the work queued on `stream`; the call returns when every
 * group is done.  With grouping 0, one frame group, or profiling on, the
 * batch is one launch sequence on `stream`.  Frames
 * larger than the budget allows together are processed in consecutive
 * launch sequences.  results[f] receives frame f's blob list; the return
 * value is DOG_OK if every frame succeeded, else the first frame error. */
int dog_detect_batch(dog_context* ctx, int32_t n_frames, const dog_frame* frames,
                     const dog_params* params, void* stream, dog_result* results);

/* Batch grouping of the context (see dog_detect_batch): groups of at most
 * max_group_pixels pixels (0: the whole batch, or each budget-sized chunk
 * of it, as one launch sequence) on `lanes` concurrent lanes (1..16; 1 runs
 * the groups one after another).  Default 2^20 pixels on 3 lanes (three
 * sequences of 2^20 pixels hold ~225 MB of planes).  Each lane
 * holds its own workspace, at most a quarter of the context's budget. */
int dog_set_batch_grouping(dog_context* ctx, int64_t max_group_pixels, int32_t lanes);

/* Release the blob arrays of n results (sets them to NULL). */
void dog_results_free(dog_result* results, int32_t n);

/* Intermediate planes of the same kernels for one device image, row-major
 * fp32 into caller-owned DEVICE buffers: L_out (k+1) x height x width
 * Gaussian planes, D_out k x height x width DoG planes (either may be NULL),
 * and *k_out = k.  Used by parity tests. */
int dog_debug_planes(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                     int64_t row_stride, const dog_params* params, float* L_out, float* D_out,
                     int32_t* k_out);

/* Unpruned candidate list (local maxima above threshold) of one device
 * image, sorted by (y, x, scale).  Used by parity tests. */
int dog_debug_candidates(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                         int64_t row_stride, const dog_params* params, dog_blob** blobs_out,
                         int64_t* count_out);

/* Kernel variant (tile geometry) selection.  Every variant computes bitwise
 * identical results (same taps, same summation order); they differ only in
 * speed.  dog_num_variants() variants exist; dog_variant_info describes one:
 * S outputs per lane, waves per workgroup, strips per wave, local-maximum
 * rows per wave.  dog_set_variant(ctx, v >= 0) pins variant v for every
 * launch of the context; v < 0 returns to automatic selection (the tuned
 * choice of the launch's dominant frame shape when one exists, see below,
 * else the built-in default). */
int dog_num_variants(void);
int dog_variant_info(int variant, int32_t* S, int32_t* waves, int32_t* strips, int32_t* nms_rows);
int dog_set_variant(dog_context* ctx, int variant);

/* Autotuner.  dog_autotune times, with the per-kernel event timing below,
 * one untimed launch then `reps` timed ones (reps = 0 means 5) of the device
 * image d_image (height x width floats, row_stride >= width elements apart,
 * on the context's device) per configuration: every variant with every plane
 * blurred directly; then, on frames whose sides are powers of two in
 * [64, 2048], that variant with the widest plane, the two widest, ... in the
 * transform domain (dog_set_dct); then, if a transform threshold won, every
 * variant again at that threshold.  The built-in default variant and the
 * direct blur each stand unless beaten by more than 2 %, so repeated tuning
 * gives the same choice.  It records the variant and the threshold for
 * frames of this shape and ladder, and writes the winning variant to
 * *variant_out and each variant's mean microseconds per frame (all kernels,
 * at the chosen threshold) to us_out[dog_num_variants()] (either may be
 * NULL).  Variants give bitwise the same results; the threshold changes the
 * planes it moves to the transform domain within the plane tolerance and is
 * applied per frame by the frame's own shape.  A launch whose dominant shape
 * (most pixels) was not tuned uses the variant of the tuned shape with the
 * same radii nearest in pixel count; an untuned shape is blurred directly.
 * The variant pinned with dog_set_variant and a threshold pinned with
 * dog_set_dct are restored afterwards (and, while pinned, used instead).
 * dog_autotune_save writes the choices as JSON to `path`; dog_autotune_load
 * adds those of a file written for the same architecture and kernel build
 * (a file of another build loads nothing and is not an error).
 * dog_autotune_choice reports the variant automatic selection would take for
 * one frame of the given shape, dog_autotune_transform the threshold (0: all
 * planes direct).  Errors: DOG_EINVAL (NULL pointer, bad shape or
 * parameters, unreadable or unwritable file), DOG_EBUSY (a launch of
 * dog_detect_device_async not finished), device errors. */
int dog_autotune(dog_context* ctx, const dog_params* params, const float* d_image, int64_t height,
                 int64_t width, int64_t row_stride, int32_t reps, int32_t* variant_out,
                 double* us_out);
int dog_autotune_save(dog_context* ctx, const char* path);
int dog_autotune_load(dog_context* ctx, const char* path);
int dog_autotune_choice(dog_context* ctx, const dog_params* params, int64_t height, int64_t width,
                        int32_t* variant_out);
int dog_autotune_transform(dog_context* ctx, const dog_params* params, int64_t height,
                           int64_t width, int32_t* min_taps_out);

/* Launch mode: on (default) = the launch sequence of a table layout (frame
 * table upload, the three kernels, candidate readback) is captured once into
 * a hipGraph and replayed while frame shapes, parameters and buffers stay the
 * same; off = the same operations are issued one by one on every call.
 * Results are identical in both modes. */
int dog_set_graph_mode(dog_context* ctx, int32_t on);

/* Per-kernel timing: when on, every launch sequence of the context records
 * HIP events around each of its three kernels (pass 1, pass 2, local
 * maxima) on the stream they run on; dog_kernel_times returns the summed
 * milliseconds of each kernel (ms_out[3]) and the number of sequences since
 * profiling was last switched on.  Timing adds three event records per
 * sequence and is off by default; while it is on the sequence is issued
 * directly rather than replayed as a graph (events inside a graph cannot be
 * timed), with the same kernels and arguments. */
int dog_set_profiling(dog_context* ctx, int32_t on);
int dog_kernel_times(dog_context* ctx, double* ms_out, int64_t* launches_out);
/* The same for every kernel of a sequence (cap >= 5): pass 1, pass 2, local
 * maxima, then the transform-domain blur's pass 1 and pass 2 (0 where the
 * sequences had no such work). */
int dog_kernel_times_all(dog_context* ctx, double* ms_out, int32_t cap, int64_t* launches_out);

/* Transform-domain blur (Sec. 4.1, the convolution taken through a fast
 * Fourier transform, whose cost does not grow with sigma): on frames whose
 * sides are powers of two in [64, 2048], ladder planes whose kernels have
 * at least min_taps taps (2 r + 1) are blurred, in each of the two
 * separable passes, as a product in the type-II cosine transform domain of
 * the lines, which is exact for the half-sample symmetric border: one
 * forward transform of the frame's columns serves every such plane in the
 * first pass, and each plane then costs one inverse transform per pass and
 * one forward one in the second (fp32 FFTs of the lines in LDS, FP64
 * transfer functions of the kernels rounded once to fp32).  The planes agree
 * with the direct blur within the detector's plane tolerance, not bit for
 * bit.  min_taps 0 blurs every plane directly; -1 (the default) takes the
 * threshold dog_autotune chose for each frame's shape (0 for shapes it has
 * not tuned).  A pass whose transform-domain lines all have one length of
 * 128 to 1024 runs them in the direct blur's launch (variants with room for
 * them in the ring), else in launches of their own.  DOG_EINVAL for
 * min_taps < -1. */
int dog_set_dct(dog_context* ctx, int32_t min_taps);


/* ------------------------------------------------------------ serving */

/* Serving loop: frames are submitted at any time; a dispatcher forms a
 * batch from whatever waits (at most max_batch_frames, and only while the
 * device footprint of all batches in flight stays within the admission
 * budget) and hands it to an idle slot.  Each slot owns a context and a
 * stream, so batches overlap on the device; a request that arrives while
 * others run joins the next batch as soon as a slot and memory are free.
 * Host frames are copied at submit into page-locked buffers the server
 * pools (up to 4 GiB; beyond that, pageable copies), from which the slot's
 * upload is a plain DMA.  Device frames (on_device = 1) are borrowed: the
 * caller keeps them valid and unchanged until the ticket's result is taken.
 * Results are the same as dog_detect on the frame alone. */
typedef struct {
    int32_t max_batch_frames;   /* frames per launch sequence (<= 0: 16)              */
    int32_t slots;              /* launch sequences in flight (<= 0: 3)               */
    int32_t queue_capacity;     /* waiting requests before DOG_EBUSY (<= 0: 4096)    */
    int32_t dry_run;            /* test hook: no GPU work; a batch takes
                                   dry_run_us_per_mpx per Mpixel and finds no blobs  */
    uint64_t hbm_budget_bytes;  /* admission budget (0: the slot context's budget)   */
    double max_wait_ms;         /* batching window (0: launch whatever waits)        */
    double dry_run_us_per_mpx;
    const char* tune_cache;     /* autotuner choices (dog_autotune_save) loaded into
                                   every slot context, or NULL                        */
    int64_t max_batch_pixels;   /* pixels per launch sequence (0: 2^20, one 1024x1024
                                   frame, so the planes of three slots' batches stay
                                   close to the 256 MB Infinity Cache between their
                                   kernels; < 0: no cap); a batch always takes at
                                   least one frame                                    */
} dog_server_opts;

typedef struct {
    int64_t submitted, completed, failed, rejected, queued, running, batches;
    double mean_batch_frames;
    double p50_ms, p99_ms, mean_ms, max_ms;   /* submit -> blob list ready          */
    double frames_per_s;                      /* completed / (last done - first submit) */
    /* Admission: a slot that runs a batch commits the device bytes its
     * workspace may reach for that batch (each buffer at least what it holds,
     * grown to the batch's planes and staged inputs, plus launch tables and
     * candidates), an idle slot what its workspace holds.  reserved = the
     * sum over the slots now; it never exceeds the budget, and each slot's
     * allocations are capped at its commit.  held = the bytes the slots'
     * workspaces actually hold after their last batches; peak over batch
     * completions. */
    uint64_t reserved_bytes, peak_reserved_bytes;
    uint64_t held_bytes, peak_held_bytes;
    int64_t admission_waits;   /* times the oldest waiting request did not fit */
} dog_stats;

/* Create a server on GPU `device` for fixed detector parameters.  A request
 * is rejected at submit (DOG_ENOMEM) when its frame alone would need more
 * than the budget: dog_footprint of that frame (its planes, the staged input
 * of a host frame, launch tables and candidates).  Idle slots keep their
 * workspaces between batches and release them when the oldest waiting
 * request would not fit otherwise. */
int dog_server_create(int device, const dog_params* params, const dog_server_opts* opts,
                      dog_server** out);
/* Queue a host frame (copied; the caller may reuse its buffer at once).
 * DOG_EBUSY: queue full; DOG_ENOMEM: the frame alone exceeds the budget. */
int dog_server_submit(dog_server* sv, const dog_frame* frame, uint64_t* ticket);
/* Result of a ticket: DOG_OK (moved into *out, with t_arrive_ns/t_done_ns),
 * DOG_EAGAIN (not done yet), DOG_ENOTFOUND (unknown or already taken). */
int dog_server_poll(dog_server* sv, uint64_t ticket, dog_result* out);
int dog_server_wait(dog_server* sv, uint64_t ticket, dog_result* out);
/* Block until every submitted request has completed. */
int dog_server_drain(dog_server* sv);
int dog_server_stats(dog_server* sv, dog_stats* out);
/* Finish running batches, drop queued requests and untaken results. */
void dog_server_destroy(dog_server* sv);

#ifdef __cplusplus
}
#endif

#endif /* DOG_H */
