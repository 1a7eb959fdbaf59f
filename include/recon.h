/*
 * recon.h - C ABI of the MI355X (gfx950) Fourier-slice insertion library.
 *
 * The library implements the data-parallel core of 3D Fourier reconstruction
 * as the paper states it in Sect. 5.3.1, Algorithm 1 ("3D reconstruction"):
 * zero-initialise a complex Fourier volume G and a weight volume W in GPU
 * memory, insert batches of 2D Fourier samples (slices) of arbitrary
 * orientation into G and W, and apply the weights W to G.  The insertion step
 * and its interpolation weights are described in Sect. 4.2 ("3D Fourier
 * Reconstruction"); the interpolation window used here is the Kaiser-Bessel
 * blob of radius a, taper alpha and order m, tabulated in squared distance.
 *
 * Conventions (all sizes in elements unless stated):
 *   h = n / 2.  The volume is the centered box {-h..h}^3, stored [z][y][x]
 *   with x fastest, index = coordinate + h; G is complex64 (interleaved
 *   float re, im), W is float32, V (output of recon_finalize) is complex64.
 *   A slice is the centered 2D DFT of a real projection image in Hermitian
 *   half-plane layout [row = ky + h][kx], kx in [0, h], complex64 (or a pair
 *   of 16-bit floats per component, see recon_slice_dtype).  Its full-plane
 *   value is F(k) for kx > 0 or (kx = 0 and ky >= 0), otherwise conj F(-k);
 *   stored entries with kx = 0, ky < 0 are never read.  Samples inserted are
 *   those with kx^2 + ky^2 < r_max^2.  An orientation is a quaternion
 *   (w, x, y, z), scalar first, normalised before use; sample k of a slice
 *   with rotation R sits at volume frequency R (kx, ky, 0)^T and adds
 *   b(d^2) F(k) to G and b(d^2) to W at every voxel within distance a.
 *
 * Memory: every device buffer is allocated by the caller and borrowed.
 * All work is enqueued on the context's HIP stream and is asynchronous with
 * respect to the host unless a function says otherwise; buffers passed to a
 * call must stay valid until the stream has passed that call.  Functions
 * return a recon_status; none throws across the ABI.  The text of the last
 * error of the calling thread is available from recon_last_error().
 * A context is not thread-safe: calls on one context must be serialised.
 */
#ifndef RECON_H
#define RECON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum recon_status {
    RECON_OK = 0,
    RECON_EINVAL = -1,   /* invalid argument (null pointer, size out of range) */
    RECON_ENOMEM = -2,   /* workspace too small, or host allocation failed */
    RECON_EDEVICE = -3,  /* HIP runtime error; text in recon_last_error() */
    RECON_ECONFIG = -4   /* kernel configuration not runnable on this device */
} recon_status;

/* Storage type of slice samples. */
typedef enum recon_slice_dtype {
    RECON_SLICE_C64 = 0,   /* complex64: float re, float im (8 bytes/sample) */
    RECON_SLICE_F16 = 1,   /* IEEE half re, im, times a per-slice FP32 scale */
    RECON_SLICE_BF16 = 2   /* bfloat16 re, im (no scale needed) */
} recon_slice_dtype;

/* Problem description.  Fill with recon_default_params() and override. */
typedef struct recon_params {
    int32_t n;            /* slice edge; even, 4 <= n <= 1024; volume (n+1)^3 */
    float blob_radius;    /* a, 1 <= a <= 2.95 (default 1.9) */
    float blob_alpha;     /* 0 <= alpha <= 60 (default 15); alpha = 0 needs m = 0 */
    int32_t blob_order;   /* m, 0 <= m <= 8 (default 0) */
    int32_t table_size;   /* N, 2 <= N <= 65536 (default 10000); 0: no table, weights on
                             the fly (needs a blob whose series converges within 72
                             terms: alpha up to about 60 for order 0) */
    int32_t table_lerp;   /* 1: linear interpolation in the table (default), 0: truncation */
    float r_max;          /* 0 < r_max <= n/2 (default n/2) */
    int32_t slice_dtype;  /* recon_slice_dtype (default RECON_SLICE_C64) */
    int32_t max_batch;    /* largest count passed to recon_insert_batch (default 1500) */
} recon_params;

/* Kernel variants of the insertion step. */
typedef enum recon_variant {
    RECON_VARIANT_AUTO = 0,    /* library choice (currently the slab gather) */
    RECON_VARIANT_NAIVE = 1,   /* one thread per voxel, every slice, global reads */
    RECON_VARIANT_BINNED = 2,  /* 4^3 tiles binned per wavefront, lane = voxel, global reads */
    RECON_VARIANT_SLAB = 3     /* 8^3 tiles, LDS-staged slice rectangle, slab-enumerated hits */
} recon_variant;

/* Tuning knobs of the insertion kernels (the paper's tuning-space idea,
 * Sect. 4.2 "3D Fourier Reconstruction" and Table 3: work-group size, work
 * mapping inside tiles of samples, weight source).  Zero in any field means
 * "library default".  Invalid combinations are rejected with RECON_ECONFIG. */
typedef struct recon_config {
    int32_t variant;          /* recon_variant */
    int32_t waves_per_block;  /* wavefronts per work-group: 1, 2, 4, 8, 12 or 16; the slab
                                 variant runs 4 or 8, or 11 (three waves per SIMD, window
                                 reads never preloaded; the default where it exists) for
                                 blob radii in [1.5, 2) with table interpolation */
    int32_t group;            /* slices staged per LDS group (binned): 1..16 */
    int32_t inner_chunk;      /* slices per inner FP32 partial sum: 1..256 (default 64 for
                                 the slab variant, 32 for the others) */
    int32_t split;            /* max slice-range splits of one tile (binned, slab): 1..64
                                 (default 32 for the slab variant, 16 for binned) */
    int32_t slab_flags;       /* slab variant, 4 | bits: bit 0 LDS float atomics for the
                                 accumulators, bit 1 issue all window reads before use
                                 (default 4 | 2; 4 with the 11-wave slab default) */
    int32_t cu_count;         /* work-groups of the persistent insertion kernels (slab,
                                 binned): 0 = one per compute unit of the device; set it to
                                 the number of CUs the context's stream may use when that
                                 stream is restricted to a subset (a CU-masked stream).
                                 Not a tuning knob: the tuner keeps the current value */
    int32_t weights;          /* recon_weights: interpolation weights from the table or
                                 evaluated on the fly (the slab variant then runs at most
                                 8 waves and has no window preload) */
    int32_t traversal;        /* recon_traversal bits: how the work maps to the tiles
                                 (default 0) */
    int32_t reserved[7];
} recon_config;

/* Traversal of the work (Sect. 4.2, "3D Fourier Reconstruction": the mapping
 * of work-items to the data inside tiles is a tuning option). */
typedef enum recon_traversal {
    /* slab variant: the lanes take a tile's columns (along the dominant axis
     * of the slice normal) with the second in-plane axis varying fastest;
     * without it, the first (axes in x, y, z order).  This reorders the hit
     * list, and so which hits fall into a slice's last round, where a window
     * sum may be split over 2 or 4 lanes: results change by FP32 rounding. */
    RECON_TRAVERSAL_COLUMNS_SECOND = 1,
    /* slab and binned variants: the work queue holds the tiles in spatial
     * (Morton) order within each of the plan's three cost tiers; without it,
     * items in decreasing estimated cost.  No result bit changes.  Batched
     * launches (recon_batch_*) keep the cost order. */
    RECON_TRAVERSAL_SPATIAL_QUEUE = 2
} recon_traversal;

/* Source of the interpolation weights (Sect. 4.2, "3D Fourier
 * Reconstruction": precomputed or computed on the fly).  The table holds
 * T[i] = b(i a^2/(N-1)) built in FP64 and is read by the rule of
 * recon_params.table_lerp; on the fly the kernels evaluate the blob itself,
 * b = s^m sum_j c_j s^j with s = 1 - d^2/a^2 and c_j from the power series of
 * I_m (terms until the rest is below 1e-10), by Horner's rule in FP32.  Both
 * agree with the exact blob to about 1e-7. */
typedef enum recon_weights {
    RECON_WEIGHTS_DEFAULT = 0,   /* the table if table_size > 0, else on the fly */
    RECON_WEIGHTS_TABLE = 1,
    RECON_WEIGHTS_OTF = 2
} recon_weights;

typedef struct recon_ctx recon_ctx;

/* Default parameters for slice edge n (a = 1.9, alpha = 15, m = 0,
 * N = 10000, lerp, r_max = n/2, complex64, max_batch = 1500). */
recon_status recon_default_params(int32_t n, recon_params *out);

/* Sizes in bytes of the caller-allocated buffers for these parameters:
 * G (complex64 (n+1)^3), W (float32 (n+1)^3) and the device workspace
 * (blob table, per-slice orientations, bins, partial sums, counters).
 * Any output pointer may be NULL. */
recon_status recon_query_sizes(const recon_params *p, size_t *g_bytes, size_t *w_bytes,
                               size_t *ws_bytes);

/* Algorithm 1, first two steps: validates p, builds the blob table on the
 * host in FP64 and uploads it (FP32) into the workspace, and zeroes G and W
 * on `stream` (a hipStream_t; NULL = the null stream).  d_G, d_W and d_ws
 * must be device memory of at least the sizes from recon_query_sizes, 256-byte
 * aligned, and must outlive the context.  This call synchronises `stream`
 * once before returning.  On success *out receives a new context. */
recon_status recon_init(const recon_params *p, void *d_G, void *d_W, void *d_ws,
                        size_t ws_bytes, void *stream, recon_ctx **out);

/* recon_init without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the workspace is a static device array
 * of the library, RECON_STATIC_WS_BYTES (192 MiB) on each device it runs on,
 * held until the process ends.  The call allocates no device memory; the
 * caller still passes G and W as for recon_init.  Every later call on the
 * context uses that array exactly as recon_init's contexts use d_ws, with the
 * same kernels and results.
 *
 * One context per device may hold the array at a time: a second
 * recon_init_static on a device whose array belongs to a live context fails
 * with RECON_EINVAL; recon_destroy releases it.  The array keeps the last
 * context's contents; recon_init_static clears what must start at zero (the
 * counters) and rewrites the table and the work plan.  Calls on the context
 * that overlap (other threads or streams) race, as on any context.
 * Parameters whose workspace (recon_query_sizes) exceeds the array fail with
 * RECON_ENOMEM before any device call; the library's defaults fit every box
 * up to n = 1024.  Otherwise the errors of recon_init. */
#define RECON_STATIC_WS_BYTES ((size_t)192 << 20)
recon_status recon_init_static(const recon_params *p, void *d_G, void *d_W, void *stream, recon_ctx **out);

/* Zeroes G and W again and clears the slice counters (asynchronous). */
recon_status recon_reset(recon_ctx *ctx);

/* Algorithm 1, insertion step (Sect. 4.2, "3D Fourier Reconstruction"):
 * inserts `count` slices into G and W.  d_slices: device [count][n][n/2+1]
 * samples of the context's slice_dtype.  d_scales: device float[count]
 * multiplying each slice (required for RECON_SLICE_F16, may be NULL
 * otherwise, meaning 1).  d_quats: device float[count][4] (w, x, y, z).
 * 0 <= count <= max_batch; count = 0 is a no-op.  A quaternion that is zero
 * or not finite makes its slice contribute nothing; such slices are counted
 * (recon_stats).  Only the half box x >= 0 of G and W is accumulated here;
 * recon_finalize completes the x < 0 half from Hermitian symmetry.
 * Arithmetic: weights and accumulation in FP32; each slice's rotation is
 * formed in double-float arithmetic and rounded once to FP32, and where
 * positions in table units are large (n/2 sqrt((N-1)/a^2) > 6800: n > 256
 * for the default blob) the slab kernel forms window offsets exactly (a grid
 * part of each scaled axis whose products with voxel coordinates are exact,
 * plus a remainder), so the FP32 position error does not grow with the
 * distance from the origin.
 * Accuracy: results agree with an FP64 evaluation of the same sums to
 * 1e-5 relative L2.  A sample whose squared distance lies within FP32
 * rounding of the cut-off a^2 may be counted or dropped differently; for
 * blobs whose edge weight b(a^2) is not small (alpha below about 8) such a
 * voxel differs by whole edge-weight samples, on a fraction of voxels below
 * 1e-4, and every other voxel meets the bar. */
recon_status recon_insert_batch(recon_ctx *ctx, const void *d_slices, const float *d_scales,
                                const float *d_quats, int32_t count);

/* Algorithm 1, last step ("apply weights W to G"): fills the x < 0 half of G
 * and W from their Hermitian mirror (G(-v) = conj G(v), W(-v) = W(v)) and
 * writes V = G / W (divided in FP64) where W > w_threshold, else 0, into the
 * caller's device buffer d_V (complex64 (n+1)^3; may be NULL to only mirror).
 * Non-destructive: more slices may be inserted afterwards. */
recon_status recon_finalize(recon_ctx *ctx, void *d_V, float w_threshold);

/* Selects insertion-kernel knobs (NULL restores the defaults).  Checks the
 * configuration against the device's limits; RECON_ECONFIG if infeasible. */
recon_status recon_set_config(recon_ctx *ctx, const recon_config *cfg);

/* Current (resolved) knobs. */
recon_status recon_get_config(const recon_ctx *ctx, recon_config *cfg);

/* Replaces the stream used for subsequent calls. */
recon_status recon_set_stream(recon_ctx *ctx, void *stream);

/* Timing hook for measurement: when start/stop are non-NULL hipEvent_t
 * handles, the next recon_insert_batch calls record `start` on the context's
 * stream immediately before the main insertion kernel and `stop` immediately
 * after it (prep and partial-sum kernels excluded); recon_batch_insert does
 * the same around its one insertion kernel with the events of its first
 * context.  NULL, NULL disables. */
recon_status recon_set_timing_events(recon_ctx *ctx, void *start, void *stop);

/* ---------------------------------------------------------------------
 * Batched insertion: several reconstructions (up to 8, any box sizes and
 * slice counts, same blob parameters, slice storage type and device) inserted by one
 * persistent launch of the slab kernel, whose work queue holds the tiles of
 * every reconstruction ordered by estimated cost.  recon_batch_insert only
 * enqueues kernels (no host synchronisation, no allocation, no copies), so a
 * caller may capture it in a HIP graph and replay it.  Work runs on the
 * first context's stream.  The launch takes the first context's
 * configuration at recon_batch_create when it is a slab-kernel one (set with
 * recon_set_config, or picked by the context's tuner), else the slab
 * kernel's single-context default for the shared blob (11 waves per
 * work-group for the 4 x 4 interpolated window, else 8), and exact window
 * geometry for every box when any box needs it (see recon_insert_batch).
 * --------------------------------------------------------------------- */
typedef struct recon_batch recon_batch;

/* Device workspace bytes the batch needs (its combined work plan). */
recon_status recon_batch_query_size(recon_ctx *const *ctxs, int32_t njobs, size_t *ws_bytes);

/* Builds the combined plan for the contexts and uploads it into d_ws
 * (256-byte aligned, at least the queried size; synchronises the first
 * context's stream once).  The contexts must outlive the batch. */
recon_status recon_batch_create(recon_ctx *const *ctxs, int32_t njobs, void *d_ws, size_t ws_bytes,
                                 recon_batch **out);

/* Inserts counts[j] slices into reconstruction j, for every j, in one
 * launch.  Per job: d_slices[j] (the context's slice storage type),
 * d_scales[j] (half storage only, else may be NULL; the array itself may be
 * NULL when no job needs scales), d_quats[j]; 0 <= counts[j] <= that
 * context's max_batch. */
recon_status recon_batch_insert(recon_batch *b, const void *const *d_slices, const float *const *d_scales,
                                const float *const *d_quats, const int32_t *counts);

void recon_batch_destroy(recon_batch *b);

/* ---------------------------------------------------------------------
 * Dynamic autotuning (Sect. 3.2, "Offline and Dynamic tuning", and its use
 * in Sect. 5.3: non-blocking tuning, where every tuning step performs real
 * work with a new configuration, here one recon_insert_batch call, and the
 * search continues with the fastest configuration once it stops).
 * The tuning space is the set of kernel configurations (recon_config) that
 * are runnable on the context's device.
 * --------------------------------------------------------------------- */
typedef struct recon_tune_opts {
    int32_t max_steps;          /* configurations to try; 0 = the whole space (or the
                                   whole candidate list) */
    int32_t reserved0;
    uint64_t seed;              /* seed of the random search order */
    double target_ns_per_slice; /* stop early once a configuration reaches this
                                   insertion time per slice, kernel and partial-sum
                                   reduction (0 = never) */
    int32_t order_count;        /* candidates: when order is not NULL, the search tries
                                   the tuning-space indices order[0..order_count-1] in
                                   that order (distinct, each in [0, space size)) instead
                                   of a random permutation of the whole space; a
                                   predictor's ranking, for example.  Host memory, read
                                   during recon_tune_begin only */
    int32_t reserved1;
    const int32_t *order;
    int32_t reserved[4];
} recon_tune_opts;

typedef struct recon_tune_info {
    int32_t active;             /* 1 while steps remain */
    int32_t steps_done;         /* configurations measured so far */
    int32_t space_size;         /* configurations in the tuning space */
    int32_t best_index;         /* index of the fastest measured (-1 if none) */
    double best_ns_per_slice;   /* its insertion time per slice (kernel and partial-sum reduction) */
    double mean_ns_per_slice;   /* mean over the measured configurations */
    recon_config best;          /* the fastest measured configuration */
} recon_tune_info;

/* Number of configurations in the tuning space, and the index-th of them
 * (in a fixed enumeration order). */
recon_status recon_tune_space_size(const recon_ctx *ctx, int32_t *size);
recon_status recon_tune_space_config(const recon_ctx *ctx, int32_t index, recon_config *out);

/* Starts a random search (or a search over the given candidates): the next
 * recon_insert_batch calls each run one untried configuration, timed with
 * events around the whole insertion (the insertion kernel and the ordered
 * reduction of its partial sums, whose cost grows with the split knob).
 * Measuring a step waits for the previous step's kernel (tuning steps are
 * not overlapped, as in the paper's tuning phase).  After max_steps steps, or
 * when the target is met, the fastest configuration is selected and kept. */
recon_status recon_tune_begin(recon_ctx *ctx, const recon_tune_opts *opts);

/* Progress of the search (waits for a pending step's timing). */
recon_status recon_tune_get_info(recon_ctx *ctx, recon_tune_info *info);

/* Ends the search now and selects the fastest measured configuration. */
recon_status recon_tune_end(recon_ctx *ctx);

/* Amortization of dynamic tuning (Sect. 5.4).  Eq. 4: kernel invocations
 * n needed so that s tuning steps at average time t_avg, followed by
 * invocations at t_well, run at relative performance rp of always running
 * at t_well: n = rp s (t_avg / t_well - 1) / (1 - rp), for 0 < rp < 1.
 * Eq. 5: random-search steps s that find one of a fraction r of
 * well-performing configurations with probability p: s = log(1-p) / log(1-r). */
recon_status recon_tune_invocations(double rp, double s, double t_avg, double t_well, double *n);
recon_status recon_tune_steps(double r, double p, double *s);

/* ---------------------------------------------------------------------
 * Learned configuration predictor: a multilayer perceptron
 * n_in -> n_hidden -> n_hidden -> n_out (ReLU, softmax) mapping workload
 * features to scores over the tuning space, trained on the tuner's timings.
 * The paper names learning from collected tuning data as related and future
 * work (Sect. 2; Sect. 6).  Parameters are one device float buffer
 * W1[n_in][H], b1[H], W2[H][H], b2[H], W3[H][C], b3[C] (row-major, [in][out]).
 * Sizes: 1 <= n_in <= 64, 1 <= H <= 1024, 2 <= C <= 4096, 1 <= batch <= 65536.
 * --------------------------------------------------------------------- */
recon_status recon_mlp_sizes(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch,
                             size_t *param_floats, size_t *ws_bytes);

/* Inference: d_probs[batch][n_out] = softmax(MLP(d_x[batch][n_in])).
 * d_ws: device workspace of ws_bytes from recon_mlp_sizes. Asynchronous on `stream`. */
recon_status recon_mlp_forward(const float *d_params, int32_t n_in, int32_t n_hidden, int32_t n_out,
                               const float *d_x, int32_t batch, void *d_ws, float *d_probs, void *stream);

/* One gradient-descent step on the mean cross-entropy against target
 * distributions d_y[batch][n_out]: d_params -= lr * gradient.  Optional
 * outputs: d_loss (one float, the batch loss before the step) and d_grads
 * (the gradient, parameter layout).  lr = 0 only computes them. */
recon_status recon_mlp_train_step(float *d_params, int32_t n_in, int32_t n_hidden, int32_t n_out,
                                  const float *d_x, const float *d_y, int32_t batch, float lr,
                                  void *d_ws, float *d_loss, float *d_grads, void *stream);

/* Slices inserted so far and slices rejected for a bad quaternion.
 * Synchronises the context's stream. */
recon_status recon_stats(recon_ctx *ctx, uint64_t *slices_inserted, uint64_t *slices_rejected);

/* Releases the context (not the caller's buffers).  NULL is ignored. */
void recon_destroy(recon_ctx *ctx);

/* Last error text of the calling thread ("" if none). */
const char *recon_last_error(void);

/* Library version string. */
const char *recon_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RECON_H */
