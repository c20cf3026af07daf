/*
 * fcfc.h -- C ABI of the MI355X (gfx950) exact pair-counting library.
 *
 * The library counts pairs of 3-D points into separation histograms, the
 * kernel of every two-point correlation function estimator (DD, DR, RR):
 *   - separations s, (s, mu) or (s_perp, pi) as defined in Sect. 2.5 of
 *     Zhao, "Fast Correlation Function Calculator" (FCFC), with the line of
 *     sight e_z or the pair mid-point s1 + s2;
 *   - half-open bins [e_k, e_k+1) tested on squared edges (Sect. 3.2), with
 *     the index look-up table of Sect. 3.2.3 for the squared separation;
 *   - regular-grid cells (Sect. 2.1) pruned by the largest separation, and a
 *     periodic box handled by per-cell-pair wrap offsets (Sect. 3.1);
 *   - auto counts take each unordered pair once (Sect. 3.1), cross counts
 *     every ordered pair (i in catalogue 1, j in catalogue 2).
 * Counts are exact: FP32 separations on the vector ALUs, and every pair whose
 * FP32 value lies within a proven error band of a bin edge is re-evaluated
 * with the FP64 definition, so int64 counts equal those of an FP64 evaluation
 * of the definition bit for bit.  Weighted counts are exact sums of the FP64
 * products w_i*w_j rounded once to FP64.
 *
 * Conventions shared by every entry point:
 *   - Return value: FCFC_OK (0) or a negative fcfc_status; nothing aborts.
 *     fcfc_last_error() gives a thread-local text for the last failure.
 *   - Catalogue arrays are DEVICE pointers owned by the caller: positions
 *     N x 3 row-major float64, weights N float64 (or NULL).  The library
 *     never frees them and keeps no reference to them after the call that
 *     reads them returns; it copies what it needs into cell structures.
 *   - Histogram outputs are DEVICE pointers, row-major [n1][n2] (first
 *     dimension s or s_perp, second mu or pi; n2 = 1 for s), OVERWRITTEN.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Work
 *     is enqueued on it; calls return before the GPU finishes unless stated.
 *   - On an error detected on the host, nothing is enqueued and outputs are
 *     left untouched.
 *   - Plans and cell sets are immutable once built; concurrent counts on
 *     different streams may share them.
 */
#ifndef FCFC_H
#define FCFC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fcfc_status;
#define FCFC_OK 0
#define FCFC_EINVAL -1      /* bad argument (null pointer, unknown enum, bad size) */
#define FCFC_ENOMEM -2      /* device or host allocation failed */
#define FCFC_EBOX -3        /* a point lies outside [0,L) (periodic) or the plan's bounds (open) */
#define FCFC_ENONFINITE -4  /* NaN or Inf in positions or weights */
#define FCFC_ERANGE -5      /* s_max > L/2, too many bins for LDS, weight range too wide, ... */
#define FCFC_EEDGES -6      /* edges not strictly increasing, negative, mu edge > 1, non-uniform mu */
#define FCFC_EGRID -7       /* cell sets were not built on the same plan */
#define FCFC_EHIP -8        /* a HIP runtime call failed */
#define FCFC_EMODEL -9      /* scheduler model unusable (the analytic fallback is used) */
#define FCFC_ESTATE -10     /* call out of order (e.g. open box without bounds) */

/* separation binning (Sect. 2.5) */
#define FCFC_BIN_S 0         /* s */
#define FCFC_BIN_S_MU 1      /* (s, mu), mu = pi / s in [0,1] */
#define FCFC_BIN_SPERP_PI 2  /* (s_perp, pi) */

/* line of sight (Sect. 2.5) */
#define FCFC_LOS_Z 0         /* l = e_z (simulation boxes) */
#define FCFC_LOS_MIDPOINT 1  /* l = s1 + s2 (observed catalogues; open boxes only) */

/* work-list order (0, the default, is the heuristic) */
#define FCFC_ORDER_HEURISTIC 0   /* longest first by A points x B points */
#define FCFC_ORDER_BUILT 1       /* enumeration order (row by row) */
#define FCFC_ORDER_LEARNED 2     /* longest first by the attached cost model (else heuristic) */

typedef struct fcfc_plan_s *fcfc_plan_t;
typedef struct fcfc_cells_s *fcfc_cells_t;
typedef struct fcfc_batch_s *fcfc_batch_t;
typedef struct fcfc_model_s *fcfc_model_t;

/* A catalogue: device pointers owned by the caller. */
typedef struct {
    const double *xyz;  /* n x 3, row-major float64 */
    const double *w;    /* n float64 weights, or NULL */
    int64_t n;          /* 0 .. 2^31 points (FCFC_EINVAL beyond) */
} fcfc_catalog;

/* Tuning knobs; zero means "choose".  Counts never depend on them. */
typedef struct {
    int32_t cells_per_rmax;  /* k: cell side = r_prune / k, 1..8 */
    int32_t tile_points;     /* A points per wavefront tile: 64 or 128 */
    int32_t seg_cells;       /* consecutive A cells a tile may span, 1..32 (0: 32) */
    int32_t b_chunk;         /* max B points per work item, 256..2^19 (0: 16384) */
    int32_t hist_copies;     /* LDS histogram copies per workgroup: 1, 2 or 4 */
    int32_t order;           /* FCFC_ORDER_* */
    int32_t record_timing;   /* 1: record per-item GPU time (training data) */
    int32_t n_hint;          /* expected catalogue size, for automatic choices */
    int32_t lut_log2;        /* log2 of the look-up table length target, 10..15 */
    int32_t group_waves;     /* wavefronts per counting workgroup, 1..16 (0: as many as fit) */
    int32_t shard_count;     /* 0 or 1: the whole work list; G > 1: count one of G shards */
    int32_t shard_index;     /* the shard counted, 0..G-1: ordered items i with i % G == index */
    int32_t batch_chunk;     /* batches: work items per wavefront a workgroup takes at once, 1..1024 (0: 32) */
    int32_t flush_log2;      /* a wavefront empties the workgroup's LDS histograms into the outputs
                                once it has claimed 2^flush_log2 candidate pairs since it last did,
                                1..26 (0: 26); the bound that keeps the 32-bit LDS counters from
                                overflowing, lowered only to exercise that merge */
    int32_t tree_leaf;       /* 0: the regular grid of Sect. 2.1.  32..128: a balanced k-d tree
                                (Sect. 2.2) with leaves of at most this many points, counted
                                through a dual-tree work list (Sect. 3.1); open boxes only
                                (FCFC_EINVAL for a periodic plan).  Batches, triangle counts,
                                predictions and the learned order take grid plans only */
    int32_t reserved;
} fcfc_tuning;

/* Statistics of the last count on a plan (host copy; see fcfc_plan_stats). */
typedef struct {
    int64_t items;           /* work items (A tile x B row piece) */
    int64_t candidates;      /* pair separations evaluated in FP32 */
    int64_t rechecks;        /* pairs re-evaluated in FP64 near an edge */
    int64_t in_range;        /* pairs counted (sum of the histogram) */
    int64_t cells;           /* grid cells */
    int32_t grid[3];         /* cells per axis */
    int32_t cells_per_rmax;  /* k actually used */
    double cell_side;        /* cell side length */
    double kernel_ms;        /* duration of the counting kernel (HIP events) */
    double band_d2_rel;      /* widest FP32 error band, relative to its edge */
    int32_t lut_entries;     /* squared-separation look-up table length */
    int32_t wg_per_cu;       /* resident counting workgroups per CU */
    int32_t order_used;      /* FCFC_ORDER_* the work list actually ran in */
    int32_t group_waves;     /* wavefronts per counting workgroup */
    int64_t flushes;         /* LDS histogram merges made before the end of the launch (flush_log2) */
} fcfc_stats;

/*
 * fcfc_plan_create -- validate the bins and box and fix every host-side
 * choice: squared edges E_k = e_k*e_k (Sect. 3.2.1), the squared-separation
 * look-up table with its FP32 error bands (Sect. 3.2.3), the prune radius
 * (s_max, or sqrt(s_perp_max^2 + pi_max^2)), and, for a periodic box, the grid.
 *   kind     FCFC_BIN_*; los FCFC_LOS_* (ignored for FCFC_BIN_S).
 *   edges1   host array of n1+1 strictly increasing, non-negative s or s_perp edges.
 *   edges2   host array of n2+1 edges: mu edges k/n2 (k = 0..n2) for S_MU,
 *            pi edges for SPERP_PI; NULL and n2 = 0 for S.
 *   box_L    > 0: periodic cube [0,L)^3 (needs prune radius <= L/2); 0: open box.
 *   tune     NULL or knobs.
 * Errors: FCFC_EINVAL, FCFC_EEDGES, FCFC_ERANGE (prune radius > L/2, or the
 * histogram does not fit in LDS), FCFC_ENOMEM.  Host only; no GPU work.
 */
fcfc_status fcfc_plan_create(int32_t kind, int32_t los, const double *edges1, int32_t n1,
                             const double *edges2, int32_t n2, double box_L,
                             const fcfc_tuning *tune, fcfc_plan_t *out);

/*
 * fcfc_plan_fit_bounds -- open box: compute on the GPU the axis-aligned
 * bounding box of all given catalogues (the first pass of the grid build,
 * Sect. 2.1) and fix the grid over it.  Synchronises `stream` once.
 * Errors: FCFC_ESTATE (periodic plan or grid already fixed), FCFC_ENONFINITE,
 * FCFC_ERANGE (mid-point line of sight with the origin inside the box), FCFC_EHIP.
 */
fcfc_status fcfc_plan_fit_bounds(fcfc_plan_t plan, const fcfc_catalog *cats, int32_t ncat,
                                 void *stream);

/*
 * fcfc_plan_set_bounds -- open box: fix the grid over the given host box
 * lo[3]..hi[3] instead.  Errors: FCFC_ESTATE, FCFC_EINVAL, FCFC_ERANGE.
 */
fcfc_status fcfc_plan_set_bounds(fcfc_plan_t plan, const double lo[3], const double hi[3]);

/*
 * fcfc_build_cells -- validate a catalogue and build its cell list on the GPU
 * (Sect. 2.1: cell key per point, stable radix sort by key, cell offsets),
 * keeping cell-local FP32 coordinates for the distance kernel, FP64
 * coordinates for the edge recheck and sorted weights.  The result owns its
 * device memory (release with fcfc_cells_free).  Synchronises `stream` once
 * to read the validation flags.
 * Errors: FCFC_ESTATE (open plan without bounds), FCFC_ENONFINITE, FCFC_EBOX,
 * FCFC_EINVAL, FCFC_ENOMEM, FCFC_EHIP.
 */
fcfc_status fcfc_build_cells(fcfc_plan_t plan, const fcfc_catalog *cat, void *stream,
                             fcfc_cells_t *out);

/*
 * fcfc_count_pairs -- count pairs into histograms.
 *   c2 == NULL: auto count of c1 (each unordered pair once).
 *   d_counts:   device int64 [n1*n2], overwritten.
 *   d_wcounts:  device float64 [n1*n2] or NULL; requires weights in both
 *               cell sets.  Exact sum of w_i*w_j rounded once.
 * Builds the work list (A tile x B row pieces of the pruned stencil) on the
 * GPU, orders it, runs the persistent counting kernel and the final merge.
 * Synchronises `stream` once to size the work list.
 * Errors: FCFC_EGRID (cell sets from different plans), FCFC_EINVAL
 * (weights requested but missing), FCFC_ERANGE (weight dynamic range too
 * wide for exact accumulation, or a weighted histogram whose 16 bytes per
 * bin of exact accumulators do not fit the LDS next to the counts: about
 * 7,000 bins on MI355X), FCFC_ENOMEM, FCFC_EHIP.
 */
fcfc_status fcfc_count_pairs(fcfc_plan_t plan, fcfc_cells_t c1, fcfc_cells_t c2,
                             int64_t *d_counts, double *d_wcounts, void *stream);

/*
 * fcfc_count_pairs_noalloc -- fcfc_count_pairs for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same counts, bit for bit, with every
 * scratch buffer of the count (work list, counters, sort space, kernel
 * arguments, exact weighted accumulators) carved out of one library-owned
 * device array of fcfc_noalloc_scratch_bytes() bytes (64 MiB) per device,
 * which each device keeps until the process ends.  The caller still passes
 * the cell sets and the outputs; no hipMalloc, hipFree or allocating routine
 * is called.  Every call on a device shares that device's array and leaves
 * it holding its own contents (what must start at zero is cleared on the
 * stream first), so calls that overlap in time on one device race: serialise
 * them (one stream, or events).  Synchronises `stream` once to size the work
 * list, as fcfc_count_pairs does.  Per-item timings (record_timing) are not
 * recorded.  fcfc_plan_stats reports this count only on a plan that has
 * already run an allocating count (which made its statistics buffer);
 * otherwise it returns FCFC_ESTATE.
 * Errors: as fcfc_count_pairs, plus FCFC_ERANGE when the count's scratch
 * (about 100 bytes per work item plus the tables, tiles and row counts)
 * exceeds the array; the outputs are then untouched.
 */
fcfc_status fcfc_count_pairs_noalloc(fcfc_plan_t plan, fcfc_cells_t c1, fcfc_cells_t c2,
                                     int64_t *d_counts, double *d_wcounts, void *stream);
/* Bytes of the per-device scratch array of fcfc_count_pairs_noalloc. */
int64_t fcfc_noalloc_scratch_bytes(void);

/* Statistics of the last fcfc_count_pairs on this plan (synchronises the
 * stream that count ran on).  Errors: FCFC_EINVAL, FCFC_ESTATE. */
fcfc_status fcfc_plan_stats(fcfc_plan_t plan, fcfc_stats *out);

/*
 * fcfc_weight_scale -- the fixed-point scale of the exact weighted sums, on
 * the host (no GPU work).  The weighted counts add up the FP64 products of
 * weights exactly (the product w_i*w_j for a pair; fl(fl(a*b)*c) for a
 * triangle), as integers in units of 2^-S: every non-zero product is then an
 * integer below 2^62 after scaling by 2^S.  wmin1/wmin2 are the smallest
 * non-zero |w| of the two catalogues (0 if a catalogue has none), wmax1/wmax2
 * the largest |w|; nfactors is 2 (pairs) or 3 (triangles, which use wmin1
 * and wmax1 only).  *S receives the scale exponent.  fcfc_count_pairs,
 * fcfc_batch_create and fcfc_count_triplets apply exactly this rule to the
 * weights of their cell sets.
 * Errors: FCFC_EINVAL (null S, nfactors not 2 or 3, negative or non-finite
 * arguments); FCFC_ERANGE when the smallest product underflows (is zero or
 * subnormal), when 2^S would overflow, or when the largest product over the
 * smallest does not fit 2^62 / 2^53 (about 5e2 for pairs).
 */
fcfc_status fcfc_weight_scale(double wmin1, double wmax1, double wmin2, double wmax2, int32_t nfactors,
                              int32_t *S);

/*
 * fcfc_batch_create / fcfc_batch_run -- auto counts of many catalogues on one
 * plan in one pipeline: one cell build keyed by (catalogue, cell), one work
 * list, one persistent counting launch that writes ncat histograms
 * (d_counts: ncat x n1*n2 int64; d_wcounts likewise, or NULL).  Each
 * unordered pair of every catalogue is counted once, exactly as
 * fcfc_count_pairs does per catalogue.  Any plan works: periodic, or an open
 * box whose bounds are set (fcfc_plan_fit_bounds over every catalogue, or
 * fcfc_plan_set_bounds), with either line of sight.  fcfc_batch_create
 * validates the catalogues, sizes every buffer (synchronising `stream` once)
 * and keeps the catalogue pointers: they must stay valid and keep their sizes
 * for the life of the batch.  fcfc_batch_run enqueues the whole pipeline;
 * with use_graph it is captured into a HIP graph on the first run and
 * replayed afterwards.  The items of each catalogue (pair) run largest
 * first: by the heuristic cost (A points x B points), or, when the plan's
 * order is FCFC_ORDER_LEARNED and a model is attached (fcfc_plan_set_model),
 * by the model's predicted time, using a copy of the model taken here (later
 * training does not change the batch; a non-finite prediction sends the
 * whole list back to the heuristic key).  The order never changes a count.
 * Errors: FCFC_ESTATE (open plan without bounds), FCFC_EINVAL (mixed weights,
 * nulls), FCFC_EBOX, FCFC_ENONFINITE, FCFC_ERANGE, FCFC_ENOMEM, FCFC_EHIP.
 */
fcfc_status fcfc_batch_create(fcfc_plan_t plan, const fcfc_catalog *cats, int32_t ncat,
                              void *stream, fcfc_batch_t *out);
/*
 * fcfc_batch_create_pairs -- like fcfc_batch_create, for any list of
 * catalogue pairs: pairs[2q] = a, pairs[2q+1] = b (0 <= a, b < ncat).  a == b
 * is the auto count of catalogue a (unordered pairs, as fcfc_count_pairs with
 * c2 = NULL); a != b the cross count of every ordered pair (i in a, j in b).
 * This is the multi-tracer configuration of App. D (data, randoms and other
 * tracers counted against each other, e.g. DD, DR, RR) with one shared cell
 * build: fcfc_batch_run writes npairs histograms, d_counts[q * n1*n2 + bin]
 * for pair q, in one counting launch whose work items of all pairs share the
 * GPU (largest estimated pair first).  Weighted counts need weights in every
 * catalogue.  Errors as fcfc_batch_create, plus FCFC_EINVAL for npairs < 1,
 * npairs > 2^20 or a catalogue index outside [0, ncat).
 */
fcfc_status fcfc_batch_create_pairs(fcfc_plan_t plan, const fcfc_catalog *cats, int32_t ncat,
                                    const int32_t *pairs, int32_t npairs, void *stream,
                                    fcfc_batch_t *out);
fcfc_status fcfc_batch_run(fcfc_batch_t batch, int64_t *d_counts, double *d_wcounts,
                           int32_t use_graph, void *stream);
/*
 * fcfc_batch_check -- wait for `stream`, report the work items of the last
 * run and its GPU time in ms (HIP events around the pipeline), and return
 * FCFC_ERANGE if the work list outgrew the capacity sized at creation (the
 * catalogue contents changed since fcfc_batch_create; counts are then invalid).
 */
fcfc_status fcfc_batch_check(fcfc_batch_t batch, void* stream, uint32_t *n_items, float *ms);
/*
 * fcfc_batch_stats -- wait for `stream` and report the counting launch of the
 * last fcfc_batch_run: out[0] candidate pairs evaluated in FP32, out[1] pairs
 * re-evaluated in FP64, out[2] LDS histogram merges made before the end of
 * the launch (see fcfc_tuning.flush_log2).  Errors: FCFC_EINVAL (null
 * arguments), FCFC_EHIP.
 */
fcfc_status fcfc_batch_stats(fcfc_batch_t batch, void *stream, int64_t out[3]);
void fcfc_batch_free(fcfc_batch_t batch);

void fcfc_cells_free(fcfc_cells_t cells);
void fcfc_plan_free(fcfc_plan_t plan);

/* Number of points and grid cells of a cell set (host values). */
fcfc_status fcfc_cells_info(fcfc_cells_t cells, int64_t *n_points, int64_t *n_cells);

/*
 * Learned work-item cost model.  Not part of the paper's method, which
 * leaves better load balancing to future work (Sect. 4.2, 4.3 and 6): a small
 * multilayer perceptron, 4 -> 64 -> 64 -> 64 -> 1 FP32 with ReLU, that maps
 * the features of a work item to log2(1 + its counting time in GPU wall-clock
 * ticks).  Features, per item: log2(1 + A points), log2(1 + B points), the
 * transverse cell-row separation sqrt(dy^2 + dz^2) in cells, and cells per
 * prune radius.  Inputs and target are standardised with stored means and
 * standard deviations (norm[10]: x mean[4], x std[4], y mean, y std).
 * Parameters are one packed FP32 array of fcfc_model_nparams() values:
 * W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4.
 * The model orders work items and picks the cell size; it never changes
 * a count.  Forward, backward and the Adam update are GPU kernels.
 */
int32_t fcfc_model_nparams(void);
/* New model, He-uniform weights from `seed`, zero biases, identity norm. */
fcfc_status fcfc_model_create(uint64_t seed, fcfc_model_t *out);
void fcfc_model_free(fcfc_model_t model);
/* Host copies of the parameters and/or the normalisation (either may be NULL). */
fcfc_status fcfc_model_get(fcfc_model_t model, float *params, float *norm);
/* Replace parameters and/or normalisation (either may be NULL) and reset the
 * optimiser state.  Errors: FCFC_EINVAL (non-finite or non-positive scale). */
fcfc_status fcfc_model_set(fcfc_model_t model, const float *params, const float *norm);
/* d_out[i] = prediction for d_feat[i*4 .. i*4+3] (device arrays, m rows). */
fcfc_status fcfc_model_predict(fcfc_model_t model, const float *d_feat, int64_t m, float *d_out,
                               void *stream);
/* Gradient of 0.5 * sum (y - t)^2 over the m samples, in standardised units,
 * with respect to the packed parameters (host grad[nparams]); *loss gets the
 * loss.  Synchronises `stream`. */
fcfc_status fcfc_model_grad(fcfc_model_t model, const float *d_feat, const float *d_target, int64_t m,
                            float *grad, float *loss, void *stream);
/* Set the normalisation from the samples, then `epochs` passes of Adam
 * (beta 0.9 / 0.999, eps 1e-8) over minibatches of `batch` (>= 64) samples
 * shuffled with `seed`.  *final_loss: mean loss of the last epoch.
 * Errors: FCFC_EINVAL (m < 2, epochs < 1, batch < 64, lr <= 0). */
fcfc_status fcfc_model_train(fcfc_model_t model, const float *d_feat, const float *d_target, int64_t m,
                             int32_t epochs, int32_t batch, float lr, uint64_t seed, void *stream,
                             float *final_loss);
/* Versioned binary file (magic, parameter count, norm, parameters).
 * fcfc_model_load: FCFC_EMODEL for a missing, short or non-finite file. */
fcfc_status fcfc_model_save(fcfc_model_t model, const char *path);
fcfc_status fcfc_model_load(const char *path, fcfc_model_t *out);

/*
 * fcfc_plan_timings -- training data: features (d_feat, cap x 4) and
 * log2(1 + ticks) (d_logt, cap) of every work item of the last count run on
 * this plan with record_timing = 1.  *n gets the item count; with d_feat NULL
 * only *n is set.  Errors: FCFC_ESTATE (no recorded count), FCFC_EINVAL
 * (cap < *n).
 */
fcfc_status fcfc_plan_timings(fcfc_plan_t plan, float *d_feat, float *d_logt, int64_t cap, int64_t *n,
                              void *stream);
/* Attach a model (not owned; NULL detaches) used by FCFC_ORDER_LEARNED.
 * Without one, or if a prediction is not finite, the count runs in
 * FCFC_ORDER_HEURISTIC and fcfc_stats.order_used says so. */
fcfc_status fcfc_plan_set_model(fcfc_plan_t plan, fcfc_model_t model);
/*
 * fcfc_plan_predict -- build the work list of fcfc_count_pairs(plan, c1, c2)
 * without counting, and return the model's predicted counting time: the larger
 * of the summed predicted item times divided by the number of resident
 * wavefronts and the largest predicted item time, in ms (*pred_ms), and the
 * item count.  Synchronises `stream`.
 */
fcfc_status fcfc_plan_predict(fcfc_plan_t plan, fcfc_cells_t c1, fcfc_cells_t c2, fcfc_model_t model,
                              void *stream, double *pred_ms, int64_t *n_items);
/*
 * fcfc_choose_cells -- pick cells per prune radius k in 1..6 for counting
 * c1 (x c2, or auto with c2 NULL): for each k, a plan with the given bins,
 * box and tuning (cells_per_rmax = k) is made, the catalogues are gridded and
 * fcfc_plan_predict scores the work list; *best_k is the k with the lowest
 * predicted time, pred_ms[k-1] each prediction (NaN where a k is not
 * possible).  With model NULL, *best_k is the analytic choice (cell side such
 * that a cell holds about 24 points on average, App. B) and pred_ms is NaN.
 * Open boxes fit the bounds to the catalogues.  Errors: as fcfc_plan_create
 * and fcfc_build_cells.
 */
fcfc_status fcfc_choose_cells(fcfc_model_t model, int32_t kind, int32_t los, const double *edges1,
                              int32_t n1, const double *edges2, int32_t n2, double box_L,
                              const fcfc_tuning *tune, const fcfc_catalog *c1, const fcfc_catalog *c2,
                              void *stream, int32_t *best_k, double pred_ms[6]);

/*
 * fcfc_autotune -- pick the tuning knobs of a count by timing it.  Not part
 * of the paper, which studies the cell size by hand (Sect. 2.1, App. B).
 * Runs build + count (best of two, GPU events) on the given catalogues for:
 * the analytic tuning; the analytic k +- 1 and, with a model, the two cell
 * sizes it predicts fastest; then, from the fastest, 2 and 4 histogram
 * copies, the other tile width, look-up tables of 2^12 and 2^14 entries,
 * workgroups of 16, 14 and 12 wavefronts and, with a model, the learned work
 * order, keeping each change that is faster.  When the fastest cell size is
 * one only the model proposed, the same knobs are also searched from the
 * fastest of the analytic k and its neighbours, and the faster result kept:
 * a model only adds candidates to the search without it.  Settings that are not possible for these bins are
 * skipped.  With the learned order in *best, counts need the model attached
 * (fcfc_plan_set_model) to use it.
 *   base       NULL or knobs kept fixed (n_hint and the order are kept).
 *   weighted   1: time weighted counts (c1 and c2 need weights).
 *   cache_path NULL, or a text file of earlier results keyed by a signature
 *              (library version, device, bins, box, line of sight, weighting,
 *              catalogue sizes to a half-octave): a hit returns without any
 *              trial (*trials = 0); a miss tunes and appends a line.
 *   best       every knob set explicitly; *best_ms its time; *heuristic_ms
 *              the analytic tuning's time (NaN on a cache hit); *trials the
 *              configurations timed.  Counts never depend on the knobs.
 * Errors: as fcfc_plan_create, fcfc_build_cells and fcfc_count_pairs;
 * FCFC_EINVAL for null arguments or missing weights.
 */
fcfc_status fcfc_autotune(fcfc_model_t model, int32_t kind, int32_t los, const double *edges1,
                          int32_t n1, const double *edges2, int32_t n2, double box_L,
                          const fcfc_tuning *base, const fcfc_catalog *c1, const fcfc_catalog *c2,
                          int32_t weighted, const char *cache_path, void *stream, fcfc_tuning *best,
                          double *best_ms, double *heuristic_ms, int32_t *trials);

/*
 * fcfc_diag_transcendental -- measure, over every FP32 input in [2^-64, 2^64)
 * (a range holding every squared separation and |l|^2 the kernel can form),
 * the largest relative error of the hardware reciprocal square root and
 * reciprocal used for mu (Sect. 2.5) and the mid-point pi, against the FP64
 * value of the exact function.  *assumed gets the bound the FP32 error bands
 * are built with; the bands are sound only if both measured values stay below
 * it.  Synchronises `stream`.  Errors: FCFC_EINVAL, FCFC_EHIP.
 */
fcfc_status fcfc_diag_transcendental(double *rsq_max_rel, double *rcp_max_rel, double *assumed,
                                     void *stream);

/*
 * fcfc_plan_numerics -- the FP32 constants the counting kernel takes from a
 * plan: the grid its cell-local coordinates are relative to, the candidate
 * threshold, and the bands around bin edges inside which a pair is binned
 * again in FP64 (the single-precision evaluation of the separations of
 * Sect. 2.5 made exact, with the squared-edge bins of Sect. 3.2.1).  Host
 * only: needs no GPU, so that tests can replay the kernel's FP32 decisions.
 *   nx, ny, nz, cells_per_rmax, lo, side  the grid (lo = 0 in a periodic box)
 *   e_axis     bound on the FP32 error of one displacement component
 *   side32     FP32 cell side the kernel forms displacements with
 *   r2prune32  a pair is a candidate when its FP32 d2 is below this (every
 *              kind except (s_perp, pi) along z, which tests vmax of both tables)
 *   d2small    (s, mu): pairs with FP32 d2 below this are always rechecked
 *   mu_tolA, mu_tolC  (s, mu): a pair whose FP32 mu*n2 lies closer than
 *              mu_tolA * rsq(d2) + mu_tolC to an interior mu edge is rechecked
 *   trans_rel  relative error assumed for the hardware rsq and rcp
 *   has_big    the larger tables exist (fcfc_plan_table 2, 3)
 * Errors: FCFC_EINVAL (null), FCFC_ESTATE (open box before its bounds are set).
 */
typedef struct fcfc_numerics {
    int32_t nx, ny, nz, cells_per_rmax;
    double lo[3];
    double side;
    double e_axis;
    float side32, r2prune32, d2small, mu_tolA, mu_tolC, trans_rel;
    int32_t has_big;
    int32_t reserved;
} fcfc_numerics;
fcfc_status fcfc_plan_numerics(fcfc_plan_t plan, fcfc_numerics *out);

/*
 * fcfc_plan_table -- copy one of a plan's squared-separation look-up tables
 * (Sect. 3.2.3) with its bands.  which: 0 the first axis (s or s_perp), 1 the
 * second ((s_perp, pi): pi), 2 and 3 the same with more entries (when
 * has_big: twice as many for s and (s, mu), four times for (s_perp, pi)).
 * Host only.  Every output may be NULL.
 *   E          n+1 squared edges e_k * e_k in FP64 (n = bins of the axis)
 *   lo, hi     n+1 FP32 band ends: an FP32 value v < lo[k] stands for a
 *              squared separation below E[k], v >= hi[k] for one at or above
 *              it (lo = hi = 0 where E = 0)
 *   tab, cap   up to cap entries; entry j covers the FP32 values v with
 *              floor(v * scale) = j and holds their bin (>= 0), -1 (out of
 *              range), or -2 - k when the band of edge k is the first that
 *              meets the entry (the kernel then compares v with the bands)
 *   n_entries  the table length; scale a power of two; vmax = hi[n]
 * Errors: FCFC_EINVAL (null plan, unknown or absent table), FCFC_ESTATE
 * (open box before its bounds are set).
 */
fcfc_status fcfc_plan_table(fcfc_plan_t plan, int32_t which, double *E, float *lo, float *hi,
                            int16_t *tab, int64_t cap, int64_t *n_entries, float *scale, float *vmax);

/*
 * fcfc_diag_peaks -- roofline microbenchmarks on the current device, timed with
 * HIP events: FP32 FMA rate (one FMA per lane per instruction, no packed
 * math; TFLOP/s, 2 flops per FMA), conflict-free LDS ds_add_u32 and
 * ds_add_u64 rates (atomics per second, whole device) and a 1 GiB
 * device-to-device copy (GB/s, bytes read + written).  Any output may be
 * NULL.  Allocates about 2 GiB while it runs; synchronises `stream`.
 * Errors: FCFC_ENOMEM, FCFC_EHIP.
 */
fcfc_status fcfc_diag_peaks(double *fma_tflops, double *lds_u32_per_s, double *lds_u64_per_s,
                            double *copy_gbps, void *stream);

/*
 * Angular pair counts.  The method applies to points on the sky directly
 * (Sect. 3.1; angular statistics are the future work of Sect. 6): a sky
 * position is a unit vector, and the angle theta between two positions maps
 * one to one onto their chord 2 sin(theta / 2), so angular bins are chord
 * bins of the unit vectors, counted by the s path of this library.
 *
 * fcfc_radec_to_unit -- d_xyz[3i..3i+2] = (cos d cos a, cos d sin a, sin d)
 * for right ascension a = d_ra_deg[i] and declination d = d_dec_deg[i] in
 * degrees (device arrays of n values; d_xyz n x 3 row-major, written).  The
 * vectors are unit length to FP64 rounding.  Enqueued on `stream`; non-finite
 * angles give non-finite vectors, which fcfc_build_cells rejects.
 * Errors: FCFC_EINVAL (null arrays, n < 0).
 */
fcfc_status fcfc_radec_to_unit(const double *d_ra_deg, const double *d_dec_deg, int64_t n,
                               double *d_xyz, void *stream);
/*
 * fcfc_angular_plan -- a plan counting pairs of unit vectors in the angular
 * bins theta_deg[0..n] (host array, degrees, strictly increasing in [0, 180]):
 * an s plan (FCFC_BIN_S) over the chord edges c_k = 2 sin(theta_k / 2),
 * computed once in FP64, in an open box holding the unit sphere.  The
 * counted quantity is the chord of the FP64 unit vectors against these
 * edges (half-open bins of the squared chord, as every separation here); it
 * equals the angular bin except for pairs within rounding of an edge.
 * chord_out (host, n + 1 values, or NULL) receives the edges used.  Cells
 * are built and counted as with any plan (fcfc_build_cells, fcfc_count_pairs,
 * batches); positions must be unit vectors (any point outside [-1, 1]^3 is
 * FCFC_EBOX).  Errors: FCFC_EINVAL, FCFC_EEDGES (an edge outside [0, 180],
 * or chords not strictly increasing), and those of fcfc_plan_create.
 */
fcfc_status fcfc_angular_plan(const double *theta_deg, int32_t n, const fcfc_tuning *tune,
                              double *chord_out, fcfc_plan_t *out);

/*
 * fcfc_bin_squared -- the histogram update routine on its own (Sect. 3.2):
 * bins n squared separations d_s2[0..n) (device FP64, 8-byte aligned, read
 * only) into d_counts[0..n1) (device int64, overwritten) with the plan's
 * first-axis bins: value v counts in bin i when E_i <= v < E_{i+1}, where
 * E_i is the FP64 square of edge i.  NaN, negative values and values at or
 * above the top squared edge count nowhere; -0.0 counts as 0.  The look-up
 * table (2^lut_log2 entries, 2^14 by default) is built from the edges alone
 * on the first call and kept by the plan; its FP32 bands cover the rounding
 * of a value to FP32, and any value inside a band is compared in FP64, so
 * the counts are exact.  Any plan works, periodic or open, with or without
 * bounds.  Enqueued on `stream`; fcfc_plan_stats afterwards gives the values
 * (candidates), FP64 rechecks, values in range and the kernel time.
 * Errors: FCFC_EINVAL (null plan or counts, n < 0 or above 2^61, unaligned
 * values), FCFC_EEDGES (edges too close for FP32 bands), FCFC_ERANGE (the
 * bins and table do not fit the LDS), FCFC_EHIP.
 */
fcfc_status fcfc_bin_squared(fcfc_plan_t plan, const double *d_s2, int64_t n, int64_t *d_counts,
                             void *stream);

/*
 * fcfc_count_triplets -- exact triangle counts of one cell set, the
 * three-point extension of the pair counts (Sect. 6 lists three-point
 * statistics as future work).  Every set {i, j, k} of three distinct points
 * is counted once when each of its three sides s = |x_b - x_a| (Sect. 2.5;
 * per-axis minimum image in a periodic box) lies in [e_0, e_n) of the plan's
 * s edges.  Its bin is (a, b, c), the three side bins sorted so that
 * a <= b <= c, in d_counts: device int64 [n1][n1][n1] row-major, overwritten
 * (entries with a > b or b > c are zero).  Sides are evaluated in FP64, in
 * the operation order of the pair definition, and binned exactly.
 *   plan       an s plan (FCFC_BIN_S) with at most 32 bins; periodic or open.
 *   cells      built on that plan by fcfc_build_cells.
 *   d_wcounts  NULL, or device FP64 [n1][n1][n1] (overwritten) for weighted
 *              counts: a triangle weighs fl(fl(a*b)*c) for its three point
 *              weights sorted by value a <= b <= c; each bin is the exact sum
 *              of those products rounded once.  Needs a cell set built with
 *              weights, and (max |w| / min non-zero |w|)^3 below about 2^9.
 * Enqueued on `stream`; fcfc_plan_stats afterwards gives the side evaluations
 * (candidates), FP64 rechecks, triangles counted (in_range) and the kernel
 * time.  Errors: FCFC_EINVAL (null arguments, not an s plan, weighted counts
 * of an unweighted cell set), FCFC_EGRID (cells of another plan),
 * FCFC_ERANGE (more than 32 bins, the tables or weighted sums do not fit the
 * LDS, or the weight range is too wide), FCFC_EHIP.
 */
fcfc_status fcfc_count_triplets(fcfc_plan_t plan, fcfc_cells_t cells, int64_t *d_counts,
                                double *d_wcounts, void *stream);

/*
 * From pair counts to correlation functions (Sect. 1, App. D).  All arrays
 * are device FP64; counts enter as FP64 (exact below 2^53).
 *
 * fcfc_xi -- any linear estimator over normalised pair counts:
 *   xi[b] = (sum_t coef[t] X_t[b] / norm[t]) / (X_den[b] / norm[den]),
 * with nterms (1..8) histograms d_terms[t] (host array of device pointers)
 * and normalisations norm[t] > 0 (e.g. N_D (N_D - 1) / 2 for an auto DD,
 * N_D N_R for DR).  Landy-Szalay: (DD, DR, RR), coef (1, -2, 1), den 2;
 * Peebles-Hauser: (DD, RR), coef (1, -1), den 1; Szapudi-Szalay (cross):
 * (D1D2, D1R2, R1D2, R1R2), coef (1, -1, -1, 1), den 3.  A bin with a zero
 * denominator gets NaN.  Errors: FCFC_EINVAL.
 */
fcfc_status fcfc_xi(int32_t nterms, const double *const *d_terms, const double *coef,
                    const double *norm, int32_t den, int64_t nbins, double *d_xi, void *stream);
/*
 * fcfc_pair_norm -- the number of pairs behind a count, the normalisation of
 * the estimators (Sect. 1, App. D): n1 (n1 - 1) / 2 for an auto count of n1
 * points (n2 < 0), n1 n2 for a cross count; formed exactly in 128-bit
 * integers and rounded once to FP64.  Host only.  Weighted counts are
 * normalised by sums of weight products instead (pass them to fcfc_xi).
 * Errors: FCFC_EINVAL (null output, n1 < 0).
 */
fcfc_status fcfc_pair_norm(int64_t n1, int64_t n2, double *out);
/*
 * fcfc_landy_szalay -- the Landy-Szalay estimator of unweighted counts:
 * xi = (DD/nDD - 2 DR/nDR + RR/nRR) / (RR/nRR) per bin, with the pair
 * normalisations of fcfc_pair_norm (auto DD of n_d points, cross DR, auto RR
 * of n_r points).  d_dd, d_dr, d_rr: device FP64 [nbins] (counts, exact below
 * 2^53); d_xi: device FP64 [nbins], overwritten; NaN where RR is zero.
 * Errors: FCFC_EINVAL (null arrays, n_d or n_r below 2), FCFC_EHIP.
 */
fcfc_status fcfc_landy_szalay(const double *d_dd, const double *d_dr, const double *d_rr, int64_t n_d,
                              int64_t n_r, int64_t nbins, double *d_xi, void *stream);
/*
 * fcfc_analytic_rr -- the pair counts of a uniform periodic box for the plan's
 * bins: npairs * V_bin / L^3 (npairs = N (N - 1) / 2 for an auto count, or
 * ((sum w)^2 - sum w^2) / 2 weighted).  V_bin is the separation-space volume
 * of the bin: a spherical shell for s; the shell times dmu for (s, mu)
 * (line of sight z); a cylindrical annulus times 2 dpi for (s_perp, pi).
 * Writes n1*n2 values.  Errors: FCFC_ESTATE (open plan), FCFC_EINVAL.
 */
fcfc_status fcfc_analytic_rr(fcfc_plan_t plan, double npairs, double *d_rr, void *stream);
/*
 * fcfc_multipoles -- Legendre multipoles of xi(s, mu) held constant within
 * each mu bin: out[k*ns + i] = (2 l + 1) sum_j xi[i*nmu + j] * integral of
 * P_l over [mu_j, mu_j+1], l = ells[k] (0..64).  mu_edges: host, nmu + 1
 * values.  Errors: FCFC_EINVAL, FCFC_ENOMEM, FCFC_EHIP.
 */
fcfc_status fcfc_multipoles(const double *d_xi, int32_t ns, const double *mu_edges, int32_t nmu,
                            const int32_t *ells, int32_t nell, double *d_out, void *stream);
/*
 * fcfc_wp -- projected correlation function w_p(s_perp_i) = 2 sum_j
 * xi[i*npi + j] (pi_j+1 - pi_j) over all pi bins.  pi_edges: host, npi + 1
 * values.  Errors: FCFC_EINVAL, FCFC_ENOMEM, FCFC_EHIP.
 */
fcfc_status fcfc_wp(const double *d_xi, int32_t nsp, const double *pi_edges, int32_t npi,
                    double *d_out, void *stream);

const char *fcfc_status_str(fcfc_status s);
const char *fcfc_last_error(void);
int32_t fcfc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FCFC_H */
