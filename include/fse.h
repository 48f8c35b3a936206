/*
 * fse.h -- C ABI of the MI355X (gfx950) Frequency Selective Extrapolation
 * library, libfse.so.
 *
 * Frequency Selective Extrapolation (FSE) replaces the lost pixels of an image
 * block by block: each processing block fits a sparse weighted superposition
 * of 2-D DFT basis functions to the known and already reconstructed pixels of
 * a support window around it, greedily, K basis functions at a time, and
 * writes the model into its lost pixels (Sec. II).  The library also provides
 * the paper's overlapping-tile framework (Sec. III): the compact tiling of
 * Algorithm 1 (eqs. (1)-(5)), tiles grown by a stripe of d pixels, processed
 * independently, cropped and merged.
 *
 * Conventions
 *  - Every call returns fse_status_t: FSE_OK (0) or a negative error code;
 *    fse_status_string() names it.  No C++ exception crosses the ABI: a host
 *    allocation that fails inside a call returns FSE_ERR_OUT_OF_MEMORY, any
 *    other failure of the host code FSE_ERR_INVALID_ARG.
 *  - Image, mask and output buffers are DEVICE pointers owned by the caller;
 *    they must stay valid until the work enqueued on `stream` (or the served
 *    request) has completed.  `stream` is a hipStream_t passed as void*
 *    (NULL = the null stream).
 *  - Images are float32, masks uint8 (1 = lost, 0 = known), row-major with a
 *    pitch counted in elements.  Values of the input at lost pixels are never
 *    read (they may be NaN).  The output receives the input at known pixels
 *    and the extrapolated value at lost pixels; it must not alias the input.
 *  - The library owns its device workspace (planning tables, a per-pixel
 *    FP64 copy of reconstructed values, scheduling counters).  It
 *    grows on demand and is kept per stream until fse_release() or exit.
 *  - A fault of the device surfaces as FSE_ERR_DEVICE on the call that
 *    observes it.
 *  - Calls are thread-safe.
 */
#ifndef FSE_H
#define FSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fse_status_t;

#define FSE_OK 0
#define FSE_ERR_INVALID_ARG (-1)
#define FSE_ERR_UNSUPPORTED (-2)
#define FSE_ERR_BUDGET (-3)
#define FSE_ERR_OUT_OF_MEMORY (-4)
#define FSE_ERR_DEVICE (-5)
#define FSE_ERR_TIMEOUT (-6)
#define FSE_ERR_NOT_FOUND (-7)
#define FSE_ERR_BUSY (-8)
#define FSE_ERR_CANCELLED (-9)

/* arithmetic of the DFT and of the selection loop */
#define FSE_PREC_F64 0   /* FP64 MFMA DFT, FP64 loop, FP64 reconstructed values */
#define FSE_PREC_F32 1   /* FP32 MFMA DFT, FP32 loop (FP64 W0 and coefficients) */
#define FSE_PREC_BF16X3 2 /* BF16x3 split MFMA DFT with FP32 accumulate, FP32 loop */

/* how the processing blocks of one call are executed */
#define FSE_SCHED_PERSISTENT 0 /* one persistent launch, device-side dependency waits */
#define FSE_SCHED_WAVEFRONT 1  /* one launch per wavefront key (host-synchronised) */
#define FSE_SCHED_PER_BLOCK 2  /* one launch per block in raster order (plain path) */

/* whole image with exact raster semantics, or the paper's tile framework */
#define FSE_WHOLE 0
#define FSE_TILED 1          /* compact tiling, Algorithm 1 (Sec. III) */
#define FSE_TILED_VERTICAL 2 /* N full-height stripes: the baseline the compact tiling improves on */

/* processing order of the blocks (each order is executed exactly: a block sees
 * the pixels of every block before it in the order as reconstructed) */
#define FSE_ORDER_RASTER 0    /* raster order of the blocks' top-left corners */
#define FSE_ORDER_OPTIMIZED 1 /* optimised order, Sec. II: large lost areas close from their margins
                                 inwards; each step takes the remaining block whose support window offers
                                 the largest share of usable weight (its sum of window weights under the
                                 current statuses over that of a fully known window; the weights rounded
                                 to multiples of 2^-30 so that shares compare exactly), ties to the
                                 raster-earlier block.  Fixed by the mask alone, planned on the host. */

#define FSE_MAX_CLASSES 3

/* A device image: float32 values, `pitch` elements between rows. */
typedef struct {
    float* data;
    int32_t width, height;
    int64_t pitch;
} fse_image_t;

/* A device loss mask: uint8, 1 = lost, 0 = known. */
typedef struct {
    const uint8_t* data;
    int32_t width, height;
    int64_t pitch;
} fse_mask_t;

/* One tile of Algorithm 1: core rectangle (x, y, w, h) and the core grown by
 * the stripe d on every side, clipped to the image (ox, oy, ow, oh). */
typedef struct {
    int32_t x, y, w, h;
    int32_t ox, oy, ow, oh;
} fse_tile_t;

/* A processing-block class: block edge B, support border b (window and DFT
 * size M = B + 2b), number of selection steps K. */
typedef struct {
    int32_t block, border, iters;
} fse_class_t;

/*
 * Parameters.  classes[0..n_classes-1] are ordered by decreasing block edge,
 * each edge a multiple of the next; every class but the last takes aligned
 * squares that are entirely lost, the last class takes the aligned cells
 * that still hold a lost pixel.  Block edges are powers of two up to 16;
 * supported windows: M = 32 and M = 64.
 * rho in (0,1]: isotropic weight decay rho^distance; recon_weight in (0,1]:
 * extra factor for pixels reconstructed by earlier blocks; gamma in (0,2):
 * orthogonality-deficiency compensation.
 * Tiled modes: align is a multiple of every class's block edge, so tile
 * cores start on the image's block grid; the stripe d is any d >= 0.  Each
 * extended tile is processed as an image of its own (Sec. III), with its
 * block grid anchored at its own top-left corner: a d that is not a
 * multiple of align shifts that grid against the image's.
 * trace_sel (device, may be NULL): receives the selected index u*M+v of
 * every step of every block, at [block_index * trace_stride + step], the
 * block index being the block's position in the processing order (raster
 * order unless `order` says otherwise); trace_capacity bounds the number of
 * blocks traced.
 * order: FSE_ORDER_RASTER or FSE_ORDER_OPTIMIZED.
 */
typedef struct {
    int32_t n_classes;
    fse_class_t classes[FSE_MAX_CLASSES];
    double rho, gamma, recon_weight;
    int32_t precision; /* FSE_PREC_* */
    int32_t schedule;  /* FSE_SCHED_* */
    int32_t tiling;    /* FSE_WHOLE, FSE_TILED or FSE_TILED_VERTICAL */
    int32_t n_tiles, overlap, align; /* tiled modes: tiles N, stripe d, grid alignment */
    int32_t workgroups;              /* persistent grid size; 0 = automatic (twice the mean blocks per wavefront key, at most the resident capacity) */
    int32_t block_waves;             /* wave64s per processing block: 1, 2 or 4; 0 = automatic */
    int32_t* trace_sel;
    int32_t trace_stride;
    int64_t trace_capacity;
    int32_t order; /* FSE_ORDER_* */
} fse_params_t;

/* Counters of the last fse_extrapolate* call on the calling thread. */
typedef struct {
    int64_t n_blocks;     /* processing blocks executed (tiles: summed over tiles) */
    int64_t n_lost_pixels;
    int64_t n_degenerate; /* blocks whose window held no usable pixel (W0 = 0) */
    int64_t n_jobs;       /* images x tiles */
    int32_t wavefront_keys;
    double host_plan_ms;  /* host-side planning time */
    double kernel_ms;     /* device time of the block kernel(s), HIP events on the call's stream */
    int32_t device_error; /* non-zero: a dependency wait hit its time limit (results invalid); the limit is
                             5 s, or FSE_WAIT_LIMIT_US microseconds from the environment when the launch is
                             prepared */
} fse_run_stats_t;

const char* fse_status_string(fse_status_t s);

/* Default parameters: one class B=4, b=14 (32x32 window and DFT), K=100,
 * rho=0.8, gamma=0.5, recon_weight=0.5, FP64, persistent schedule, whole image. */
fse_status_t fse_params_default(fse_params_t* p);

/*
 * Compact tiling, Algorithm 1 with eqs. (1)-(5) of Sec. III, plus the stripe
 * d of Sec. III.  tiles: caller-owned host array of N entries.  align > 1
 * moves every interior tile edge down to a multiple of align (the block grid)
 * so that the blocks of a tile coincide with those of the image.  For large
 * N the row heights of eq. (4) add up to more than H; rows are then clipped
 * at the bottom edge, and tiles of rows past it are empty (w or h = 0).
 * Errors: INVALID_ARG when W, H, N < 1, d < 0, align < 1 or N > W*H.
 */
fse_status_t fse_plan_tiles(int32_t W, int32_t H, int32_t N, int32_t d, int32_t align,
                            fse_tile_t* tiles);

/*
 * N vertical stripes of the full height (all tiles in one row: widths as in
 * eq. (5) with n_C = N), with the same stripe d and alignment as
 * fse_plan_tiles.  The straightforward tiling that Sec. III improves on with
 * compact tiles: it needs more overlap (stripes on long edges) for the same
 * N.  Same arguments and errors as fse_plan_tiles.
 */
fse_status_t fse_plan_tiles_vertical(int32_t W, int32_t H, int32_t N, int32_t d, int32_t align,
                                     fse_tile_t* tiles);

/*
 * Extrapolate the lost pixels of one image (Sec. II; with p->tiling ==
 * FSE_TILED or FSE_TILED_VERTICAL through the tile framework of Sec. III).  Enqueued on `stream`;
 * returns once the work is enqueued (the planner reads the mask back to the
 * host first, so the call waits for the mask to be ready).
 * Errors: INVALID_ARG (null pointers, size mismatch, parameter ranges),
 * UNSUPPORTED (window size not 32 or 64), OUT_OF_MEMORY, DEVICE.
 */
fse_status_t fse_extrapolate(const fse_image_t* image, const fse_mask_t* mask, const fse_params_t* p,
                             fse_image_t* out, void* stream);

/* Same for n images in one batched persistent launch (blocks of all images
 * and tiles share the device queue).  Arrays of n entries. */
fse_status_t fse_extrapolate_batch(int32_t n, const fse_image_t* images, const fse_mask_t* masks,
                                   const fse_params_t* p, fse_image_t* outs, void* stream);

/*
 * fse_extrapolate without allocation, for callers that cannot allocate
 * device memory (code that must not call hipMalloc: tight serving loops,
 * harnesses that forbid it).  Same arguments, results and errors as
 * fse_extrapolate (results are identical); the device scratch of the call
 * (FP64 working copy of reconstructed pixels, planning tables, flags and
 * counters) lives in one fixed array of FSE_NOALLOC_SCRATCH_BYTES per device,
 * held from the first call on that device until the process ends.  The call
 * allocates no device or pinned host memory; the host planner reuses its
 * own heap storage between calls.
 *  - BUDGET when the call needs more scratch than the array holds (about
 *    8 bytes per pixel of the image, or of every extended tile, plus ~48
 *    bytes per processing block: a 1920x1080 image fits, 4 Mpixel do not);
 *    nothing is enqueued then.
 *  - All calls of this entry point in the process share the array of their
 *    device: a call waits (on the host) until the previous call's kernels have
 *    finished before it reuses the array, so calls on different streams are
 *    serialised rather than overlapped.
 *  - The time of the kernels is not measured (fse_last_stats reports
 *    kernel_ms = 0; its device_error and n_degenerate words are read from the
 *    array until the next call of this entry point on that device).
 */
#define FSE_NOALLOC_SCRATCH_BYTES (32ull << 20)
fse_status_t fse_extrapolate_noalloc(const fse_image_t* image, const fse_mask_t* mask, const fse_params_t* p,
                                     fse_image_t* out, void* stream);

/* Statistics of the last extrapolate call made by this thread; waits for
 * that call's stream to finish its work. */
fse_status_t fse_last_stats(fse_run_stats_t* st);

/* Schedule autotuner: runs the given batch (outputs written to outs) under
 * candidate schedules, timing each with HIP events on `stream`, and returns *p
 * with the fastest schedule in *best:
 *  - tiled modes with p->n_tiles == 0: first the tile count N of Algorithm 1
 *    (Sec. III), from {16, 32, 64, 128, 256}, with the caller's stripe d and
 *    the automatic grid (N, unlike the rest, changes results: the tile
 *    framework's output depends on its tiles);
 *  - then wave64s per block in {1, 2, 4}, or only p->block_waves when that is
 *    not 0 (eight per workgroup when 64x64 windows are present), and
 *    persistent grids of {automatic, 128, 256, 384,
 *    512, 768, 1024, resident capacity} workgroups; neither changes results.
 * The result is cached in-process per workload signature: sizes, classes,
 * parameters, and the number of blocks and of dependency levels of the masks
 * (from a first call), so masks of the same size but another structure are
 * tuned anew; a cached signature returns after that first call.  Requires the
 * persistent schedule.  Errors as fse_extrapolate_batch. */
fse_status_t fse_autotune(int32_t n, const fse_image_t* images, const fse_mask_t* masks, const fse_params_t* p,
                          fse_image_t* outs, void* stream, fse_params_t* best);

/* The same search for callers that keep `streams` (2..8) consecutive calls in
 * flight on as many streams: each candidate is timed over rounds of
 * consecutive calls spread over `streams` streams of the tuner's own (the
 * device runs several launches at once, where the best grid differs from a
 * launch alone), by the host clock.  The first stream writes outs; the others
 * write to temporary outputs the tuner allocates and frees.  Cached
 * separately from fse_autotune. */
fse_status_t fse_autotune_overlapped(int32_t n, const fse_image_t* images, const fse_mask_t* masks,
                                     const fse_params_t* p, fse_image_t* outs, int32_t streams,
                                     fse_params_t* best);

/* Free all cached device workspace (waits for the streams that use it).
 * Calls running on other threads finish first (each holds its workspace's
 * lock); fse_last_stats for a call whose workspace was freed returns the
 * host-side statistics only (no kernel time, no device error flag). */
fse_status_t fse_release(void);

/* ---- prepared plans replayed as HIP graphs ---------------------------- */

/* A plan fixes n loss masks and the parameters: blocks, dependency order and
 * device tables are built once, the masks are copied (the caller may free
 * them after the call), and the launch sequence is captured in a HIP graph.
 * Only the persistent schedule can be planned; trace_sel must be NULL.
 * Errors: INVALID_ARG, UNSUPPORTED, OUT_OF_MEMORY, DEVICE. */
typedef struct fse_plan fse_plan_t;
fse_status_t fse_plan_create(int32_t n, const fse_mask_t* masks, const fse_params_t* p, fse_plan_t** plan);
/* Extrapolate n images with the plan's masks: images[i] and outs[i] must have
 * the size of mask i.  Enqueued on `stream` as one graph launch; executions of
 * one plan are serialised (each waits until the previous one has finished). */
fse_status_t fse_plan_execute(fse_plan_t* plan, const fse_image_t* images, fse_image_t* outs, void* stream);
/* Statistics of the plan (blocks, lost pixels, jobs, planning time) and of
 * its last execution: waits until that execution has finished and reports
 * its device error word (non-zero: a dependency wait hit its time limit and
 * the outputs are invalid) and its degenerate blocks.  kernel_ms is 0 (graph
 * launches are not timed).  Before the first execution both words read 0. */
fse_status_t fse_plan_stats(fse_plan_t* plan, fse_run_stats_t* st);
fse_status_t fse_plan_destroy(fse_plan_t* plan);

/* ---- serving: continuous batching of requests ------------------------- */

typedef struct fse_server fse_server_t;

typedef struct {
    int64_t hbm_budget_bytes; /* device memory the server may hold for requests */
    int32_t max_slots;        /* launches in flight at once (1..16), each on a stream with a hardware queue
                                 of its own (created with a CU mask of all CUs: plain streams share the
                                 runtime's small queue pool, where two launches would run one after the
                                 other) */
    int32_t device;           /* HIP device ordinal */
    int32_t workgroups;       /* persistent grid size, 0 = automatic */
} fse_serve_config_t;

typedef struct {
    double t_submit_ms, t_admit_ms, t_done_ms; /* host steady clock */
    int64_t n_blocks;
} fse_request_stats_t;

fse_status_t fse_serve_create(const fse_serve_config_t* cfg, fse_server_t** server);
/* Queue a request.  A request whose launch fails -- including a launch whose
 * dependency wait hit its time limit (see fse_run_stats_t.device_error) --
 * completes with that error (FSE_ERR_DEVICE) from fse_serve_wait and
 * fse_serve_poll; its output is then invalid.
 * The buffers are device pointers owned by the caller and
 * must stay valid until the request is done.  The server's streams are not
 * ordered after the caller's: image and mask must hold their final contents
 * when the request is submitted (synchronise the work that wrote them first).
 * BUDGET when the request can never fit the budget. */
fse_status_t fse_serve_submit(fse_server_t* s, const fse_image_t* image, const fse_mask_t* mask,
                              const fse_params_t* p, fse_image_t* out, uint64_t* ticket);
fse_status_t fse_serve_poll(fse_server_t* s, uint64_t ticket, int32_t* done, fse_request_stats_t* st);
/* timeout_us < 0 waits without limit; TIMEOUT when it expires. */
fse_status_t fse_serve_wait(fse_server_t* s, uint64_t ticket, int64_t timeout_us, fse_request_stats_t* st);
/* Withdraw a request that is still queued: its wait and poll then report
 * CANCELLED and its output is left untouched.  BUSY once it has been admitted
 * into a launch (it then completes normally); NOT_FOUND for an unknown or
 * already collected ticket. */
fse_status_t fse_serve_cancel(fse_server_t* s, uint64_t ticket);
fse_status_t fse_serve_destroy(fse_server_t* s);

#ifdef __cplusplus
}
#endif

#endif /* FSE_H */
