/*
 * wo.h -- C ABI of the MI355X (gfx950) picking-plan evaluator.
 *
 * The library scores candidate plans for the order-picking subproblem of
 * arXiv 2110.13693 (section 5): a plan clusters product categories into
 * warehouse zones (Subproblem 3, placement by category) and fixes the
 * sequence in which orders are picked (Subproblem 5 and section 6, "in which
 * sequence the orders should be picked during a given time frame").  The
 * route objective is the sum of per-tour distances and the picking rate is a
 * function of it (Subproblem 2, Eq. (2): min sum d_i, delta = f(d)).
 *
 * Model (one instance = one single-block parallel-aisle warehouse):
 *   - locations l = 0 .. 2*N*S-1, aisle-major: aisle l / (2S), depth index
 *     (l mod 2S) / 2, side l mod 2; the depth of index j is j*pitch + pitch/2
 *     from the front cross aisle; the depot is the front of aisle 0;
 *   - zones are contiguous location ranges laid out in zone order, zone z as
 *     long as the category placed in it; inside a zone SKUs sit in ascending
 *     SKU id (id = popularity rank);
 *   - the order sequence is cut next-fit into tours of at most `capacity`
 *     items (orders are never split; a larger order is a tour of its own);
 *   - a tour's distance is its S-shape route:
 *       2*spacing*a_max + (k even ? k*L : (k-1)*L + 2*y_far),  L = S*pitch,
 *     k = number of aisles holding a pick, a_max the last of them, y_far the
 *     farthest pick depth in a_max;
 *   - D = sum over tours (int64 inside; the int32 output saturates at
 *     INT32_MAX); throughput = n_orders * window / (D / walk + t_item * items),
 *     evaluated in IEEE double without contraction and rounded once to float.
 *
 * Conventions.
 *   - Pointers named d_* are device pointers (HIP device memory, e.g. torch
 *     tensors' data_ptr()); other pointers are host pointers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls marked "async" only enqueue work on it; the caller keeps every
 *     d_* buffer alive until the stream has passed the call.
 *   - Every call returns a wo_status and never throws.  On failure
 *     wo_last_error() gives a message (thread-local, valid until the next call
 *     on the same thread).  Argument checks happen on the host before any
 *     work is enqueued; a failing call enqueues nothing.  HIP runtime errors
 *     return WO_E_DEVICE.
 *   - Handles are not thread-safe; a handle used from two threads at once
 *     returns WO_E_STATE for the second caller.
 *   - One stream per handle, or ordered streams: a handle keeps device state
 *     that its calls share and upload in their own stream (for
 *     wo_eval_plans: the plan map and the tables built from it, the queue
 *     tickets, the validation flag, the first-fit tour table).  A call on a
 *     stream other than the previous call's, while that call may still be
 *     running, returns WO_E_STATE and enqueues nothing when either call
 *     rewrites that state; when neither does, the library orders the new
 *     call after the previous one.  Replays of a captured graph are not seen
 *     by the handle: the caller orders them with its other calls.
 */
#ifndef WO_H
#define WO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WO_OK = 0,
    WO_E_INVAL = 1,        /* malformed argument (NULL, bad permutation, ...) */
    WO_E_RANGE = 2,        /* argument outside a supported size limit */
    WO_E_NOMEM = 3,        /* host or device allocation failed */
    WO_E_DEVICE = 4,       /* a HIP runtime call failed */
    WO_E_STATE = 5,        /* handle in use or in the wrong state */
    WO_E_UNSUPPORTED = 6   /* valid input this build does not handle */
} wo_status;

/* Size limits checked by wo_load_warehouse (WO_E_RANGE beyond them). */
#define WO_MAX_CATEGORIES 64        /* zone_of rows are 64 bytes */
#define WO_MAX_ORDERS 65535         /* order ids are uint16 */
#define WO_MAX_CAPACITY 32          /* items per tour */
#define WO_MAX_LOCATIONS (1 << 22)  /* 2*N*S */
#define WO_MAX_LINES (1 << 24)      /* order lines per instance */
#define WO_ZONE_PAD 0xFF

/* Short human-readable name of a status code (static string); any value
 * outside the enumeration gives "WO_E_UNKNOWN". */
const char *wo_status_str(int32_t s);

/* Message of the last failing call on this thread ("" if none). */
const char *wo_last_error(void);

/* ------------------------------------------------------------------ */
/* Warehouse instances                                                  */
/* ------------------------------------------------------------------ */

/* Host description of one instance.  All distances are integer decimetres.
 * Arrays are read during wo_load_warehouse only and may be freed after it. */
typedef struct {
    int32_t n_aisles;          /* N >= 1 */
    int32_t slots_per_side;    /* S >= 1; two sides per aisle */
    int32_t pitch_dm;          /* slot pitch, even, >= 2 */
    int32_t spacing_dm;        /* aisle centre-to-centre distance, >= 0 */
    int32_t capacity;          /* items per tour, 1 .. WO_MAX_CAPACITY */
    int32_t n_categories;      /* 1 .. WO_MAX_CATEGORIES */
    int32_t n_skus;            /* >= n_categories; sum of category sizes <= 2*N*S */
    const int32_t *sku_category;   /* [n_skus], each in [0, n_categories), every
                                      category non-empty */
    int32_t n_orders;          /* 1 .. WO_MAX_ORDERS */
    const int32_t *order_offsets;  /* [n_orders + 1], offsets[0] = 0, strictly
                                      increasing (every order has >= 1 line) */
    const int32_t *order_skus;     /* [order_offsets[n_orders]], each in [0, n_skus);
                                      one line = one item */
    double walk_dm_per_s;      /* walking speed, dm/s (> 0), e.g. 12.0 */
    double seconds_per_item;   /* picking time per item (>= 0), e.g. 10.0 */
    double window_s;           /* time window (> 0), e.g. 28800.0 */
    int32_t routing;           /* WO_ROUTE_*: route of every tour (0 = S-shape);
                                  the same for all instances of one load */
    int32_t batching;          /* WO_BATCH_*: how orders form tours (0 = next fit);
                                  the same for all instances of one load */
} wo_instance_desc;

/* Route of a tour (section 5, Subproblem 2 leaves the routing method open;
 * these are the standard policies of the order-picking literature, depot at
 * the front of aisle 0, L = slots_per_side * pitch_dm):
 *   WO_ROUTE_SSHAPE      every aisle with a pick is crossed entirely; with an
 *                        odd count the last one is entered and left from the
 *                        front;
 *   WO_ROUTE_RETURN      every aisle with a pick is entered from the front up
 *                        to its farthest pick and left the same way;
 *   WO_ROUTE_LARGEST_GAP the first and last aisles with picks are crossed;
 *                        every other one is entered from both cross aisles,
 *                        each time up to its largest gap (front to first pick,
 *                        between picks, last pick to back) and back; a single
 *                        aisle is a return route;
 *   WO_ROUTE_COMBINED    every aisle with a pick is visited once, in ascending
 *                        order, and either crossed or entered and left from
 *                        the cross aisle the picker is on, the choices that
 *                        make the walk shortest; the walk ends on the front
 *                        (crossing the last aisle if it is on the back);
 *   WO_ROUTE_OPTIMAL     the shortest closed walk from the depot through every
 *                        pick (the minimum route distance of the same passage),
 *                        exact for the single-block layout.
 * The routes other than S-shape keep every pick of a tour in an LDS row of
 * WO_MAX_PICK_SLOTS entries, sorted and walked per tour; an order of more
 * lines is a tour of its own (the capacity is at most WO_MAX_PICK_SLOTS) and
 * is sorted and walked apart, by the whole workgroup, from the order's own
 * line list.  Such an order may have up to WO_MAX_ROUTED_ORDER_LINES lines;
 * a longer one fails wo_load_warehouse with WO_E_UNSUPPORTED.  The optimal route computes
 * in 32-bit integers: 4 * spacing * (n_aisles + 2) + 4 * L * (n_aisles + 1)
 * must stay below 2^30 dm, else the load fails with WO_E_RANGE. */
enum { WO_ROUTE_SSHAPE = 0, WO_ROUTE_RETURN = 1, WO_ROUTE_LARGEST_GAP = 2, WO_ROUTE_OPTIMAL = 3,
       WO_ROUTE_COMBINED = 4 };

/* Batching of orders into tours (the paper cuts the order sequence greedily
 * into capacity-bounded tours, section 5, Subproblem 2 and section 6; these
 * are the two greedy rules of the order-batching literature):
 *   WO_BATCH_NEXT_FIT   an order joins the open tour if the items fit, else
 *                       it opens a new tour (tours are runs of the sequence);
 *   WO_BATCH_FIRST_FIT  an order joins the earliest-opened tour with room for
 *                       it, else it opens a new tour;
 *   WO_BATCH_SEED       seed batching: tours are built one at a time; a tour
 *                       starts from the order earliest in the sequence that
 *                       is in no tour yet, then, while any such order fits,
 *                       takes the one that adds the fewest aisles the tour
 *                       does not visit yet (ties: earlier in the sequence).
 *                       The tours depend on the slotting as well.
 * An order larger than the capacity is a tour of its own under all three.
 * First fit and seed batching take every route; the launch configuration
 * (wo_set_eval_config, wo_autotune_eval) does not apply to them.  Seed
 * batching keeps per-plan tables in LDS -- about 4 bytes per order, 2 per
 * line and 4 per aisle -- and takes orders that visit at most 1,023 aisles;
 * an instance beyond either limit fails at load with WO_E_UNSUPPORTED (the
 * paper-scale instance needs 38 KB). */
enum { WO_BATCH_NEXT_FIT = 0, WO_BATCH_FIRST_FIT = 1, WO_BATCH_SEED = 2 };
#define WO_MAX_PICK_SLOTS 32
#define WO_MAX_ROUTED_ORDER_LINES 8192

typedef struct wo_wh wo_wh;

/* Class-based storage (section 5, Subproblem 3: products are placed by how
 * often they are picked, with an unsupervised clustering such as K-means).
 * Clusters the n_skus SKUs into at most k (1 .. 64) categories by Lloyd's
 * K-means on pick frequency, the number of entries of d_order_skus naming
 * each SKU:
 *   - start: centroid c is the distinct frequency of rank
 *     floor((2c + 1) D / (2k)) among the D distinct frequencies;
 *   - a step assigns every SKU to its nearest centroid (exact rational
 *     arithmetic; a tie goes to the lower index) and moves each non-empty
 *     cluster's centroid to its members' mean; the iteration ends at the first
 *     assignment equal to the previous one or after max_iter (>= 1);
 *   - the non-empty clusters become categories 0 .. k_used - 1 by descending
 *     mean frequency (equal means: lower cluster first), so category 0 holds
 *     the fastest movers.
 * d_order_skus: device int32 [n_lines] (1 .. WO_MAX_LINES), each in
 * [0, n_skus); d_category: device int32 [n_skus], written.  *k_used and
 * *n_iter (assignments performed) are written when not NULL.  The result
 * can serve as a wo_instance_desc's sku_category.  Synchronous on `stream`;
 * it allocates and frees its own scratch, so it is not for graph capture.
 * WO_E_INVAL / WO_E_RANGE for bad arguments or an out-of-range SKU id. */
wo_status wo_kmeans_categories(const int32_t *d_order_skus, int64_t n_lines, int32_t n_skus, int32_t k,
                               int32_t max_iter, int32_t *d_category, int32_t *k_used, int32_t *n_iter,
                               void *stream);

/* K-means categories without allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The clustering and its arguments are those of
 * wo_kmeans_categories, with three differences:
 *   - asynchronous on `stream`: it enqueues kernels only (no allocation,
 *     memset or host synchronisation), so it may be captured into a graph;
 *     max_iter is in 1 .. WO_KMEANS_NOALLOC_MAX_ITER;
 *   - d_k_used and d_n_iter are device int32 pointers (each nullable) that
 *     receive the categories used and the assignments performed; an order
 *     line naming a SKU outside 0 .. n_skus - 1 sets *d_k_used to -1 (and
 *     d_category is then unspecified);
 *   - the scratch (4 n_skus + 8 (n_lines + 1) bytes plus the iteration state,
 *     each part rounded up to 256 bytes) lives in a static device array of
 *     WO_KMEANS_NOALLOC_SCRATCH bytes that every GPU the library runs on
 *     holds until the process ends; a larger need returns WO_E_RANGE before
 *     anything is enqueued.
 * All calls on one GPU share its array, and each call clears it first:
 * calls that overlap on one GPU (on different streams, or from several
 * threads) race, so the caller orders them. */
#define WO_KMEANS_NOALLOC_SCRATCH (8 << 20)
#define WO_KMEANS_NOALLOC_MAX_ITER 256
wo_status wo_kmeans_categories_noalloc(const int32_t *d_order_skus, int64_t n_lines, int32_t n_skus, int32_t k,
                                       int32_t max_iter, int32_t *d_category, int32_t *d_k_used,
                                       int32_t *d_n_iter, void *stream);

/* Load n_instances (>= 1) instances onto the current HIP device.
 * Validates every descriptor (WO_E_INVAL / WO_E_RANGE), packs per-line
 * records and order tables, copies them to device memory on `stream` and
 * synchronises it.  On success *out owns the device memory until
 * wo_free_warehouse.  Synchronous.
 * The next-fit evaluator keeps one tile of tour rows in LDS and passes over
 * the lines once per tile; a tile holds the expected tour count of the
 * instance with a margin (fewer where LDS runs out).  The environment
 * variable WO_TILE_TOURS=t (t >= 1) caps every instance's tile at t tours,
 * for measuring that choice. */
wo_status wo_load_warehouse(const wo_instance_desc *descs, int32_t n_instances,
                            void *stream, wo_wh **out);

/* Release an instance handle (NULL is a no-op).  Synchronises the device
 * before freeing so that no enqueued call still uses the memory. */
wo_status wo_free_warehouse(wo_wh *wh);

/* Number of orders / items of instance i (host-side lookup). */
wo_status wo_instance_info(const wo_wh *wh, int32_t i, int32_t *n_orders, int32_t *n_items,
                           int32_t *n_categories);

/* ------------------------------------------------------------------ */
/* Exact evaluation (the hot path)                                      */
/* ------------------------------------------------------------------ */

/* Evaluate n_plans plans exactly (async).
 *
 * plan_offsets: host int64[n_instances + 1], plan rows of instance i are
 *   [plan_offsets[i], plan_offsets[i+1]); plan_offsets[0] = 0 and
 *   plan_offsets[n_instances] = n_plans.  May be NULL when the handle holds a
 *   single instance.
 * d_zone_of: uint8[n_plans][64]; row p gives the zone of each category of its
 *   instance (a permutation of 0..C-1 in the first C bytes; the rest ignored).
 * d_order_seq: uint16, the plans' order sequences packed row after row:
 *   instance i's rows follow those of instance i-1, each row n_orders(i)
 *   entries, a permutation of 0..n_orders(i)-1.
 * d_dist: int32[n_plans] out, total S-shape distance (saturating).
 * d_orders_per_window: float[n_plans] out, may be NULL.
 *
 * Plan contents are not checked on the host (they live in device memory);
 * with the environment variable WO_VALIDATE=1 the kernel checks that every
 * row is a permutation and this call synchronises and returns WO_E_INVAL if
 * one is not.  Without it, a non-permutation row yields an unspecified value
 * for that row (never an out-of-bounds access). */
wo_status wo_eval_plans(wo_wh *wh, const int64_t *plan_offsets, int64_t n_plans,
                        const uint8_t *d_zone_of, const uint16_t *d_order_seq,
                        int32_t *d_dist, float *d_orders_per_window, void *stream);


/* Launch configuration of the evaluation kernel for a handle:
 *  - block_threads: threads per workgroup (64, 128, 256 or 512; one
 *    workgroup evaluates one plan at a time);
 *  - blocks_per_cu: workgroups per CU (0 = as many as registers and LDS
 *    allow);
 *  - queue: the work distribution (0 = grid stride over plan rows, 1 = a
 *    ticket queue over a work list that puts the plans of the most
 *    expensive instances first -- useful for uneven batches);
 *  - line_pass: the mapping of the aisle-set pass (S-shape; the other routes
 *    always take 0): 0 = the instance's lines in a fixed order, one per
 *    lane, each order's tour entry looked up in a table (default); 1 = one
 *    order per lane; 2 = the lines in sequence order, 64 consecutive ones
 *    per wave, so that the lines of a tour sit in adjacent lanes and its
 *    farthest location is one segmented wave maximum (instances with an
 *    order larger than the capacity take 0);
 *  - small_orders: plans of instances with at most this many orders (0 to
 *    1024) are evaluated in a launch of their own with 64-thread
 *    workgroups, and those with at most twice as many in one with
 *    128-thread workgroups, each sized by its instances' own LDS needs, so
 *    that many small plans run per CU; 0 = one launch for every instance.
 *    Default 1024.
 * `ms` is the measured time of one call when returned by the autotuner. */
typedef struct {
    int32_t block_threads;
    int32_t blocks_per_cu;
    int32_t queue;
    int32_t line_pass;   /* 0: one line per lane (default), 1: one order per lane, 2: sequence order */
    int32_t small_orders;
    float ms;
} wo_eval_config;

wo_status wo_set_eval_config(wo_wh *wh, const wo_eval_config *cfg);
wo_status wo_get_eval_config(const wo_wh *wh, wo_eval_config *cfg);

/* Autotuner: times wo_eval_plans on the given plans for every supported
 * configuration (best of `reps` runs each, after a warm-up), keeps the
 * fastest in the handle and returns it in best_out.  h_all (nullable)
 * receives up to *n_all timed configurations; *n_all is set to how many
 * were timed.  Synchronous; overwrites d_dist.  A first-fit handle has one
 * launch shape: its current configuration is timed once and kept. */
wo_status wo_autotune_eval(wo_wh *wh, const int64_t *plan_offsets, int64_t n_plans, const uint8_t *d_zone_of,
                           const uint16_t *d_order_seq, int32_t *d_dist, int32_t reps, void *stream,
                           wo_eval_config *best_out, wo_eval_config *h_all, int32_t *n_all);

/* Persistent autotune cache: a JSON file {"entries": [...]} whose entries
 * hold a key -- the device's architecture name ("arch", e.g. "gfx950"), its
 * compute units ("cus"), the handle's route and batching, and the buckets
 * ceil(log2(.)) of its instance count ("instances"), of its largest order
 * count ("orders") and of the call's plan count ("plans") -- and a launch
 * configuration ("block_threads", "blocks_per_cu", "queue", "line_pass",
 * "small_orders", and the measured "ms").
 *  - wo_autotune_eval stores its winner in the file named by the
 *    environment variable WO_TUNE_CACHE, if set (the tuned configuration is
 *    applied either way; a write failure is returned as WO_E_INVAL).
 *  - Until a configuration is chosen (wo_set_eval_config, wo_autotune_eval,
 *    wo_tune_cache_lookup), wo_eval_plans consults that file whenever the
 *    plan-count bucket differs from the previous call's and uses the
 *    matching entry, else the default configuration (also when the file is
 *    missing or malformed).
 *  - wo_tune_cache_store writes cfg (NULL: the handle's configuration) as
 *    the entry of the handle's key for n_plans plans, replacing one with the
 *    same key; the file is rewritten through a temporary file beside it.
 *  - wo_tune_cache_lookup applies the entry of the handle's key for n_plans
 *    plans if there is one (*found = 1) and chooses it; *found = 0 leaves the
 *    configuration as it is.  A missing file is an empty cache; a malformed
 *    one, or an entry with an invalid configuration, gives WO_E_INVAL.
 * Synchronous host calls; they touch no device memory. */
wo_status wo_tune_cache_store(wo_wh *wh, const char *path, int64_t n_plans, const wo_eval_config *cfg);
wo_status wo_tune_cache_lookup(wo_wh *wh, const char *path, int64_t n_plans, int32_t *found);

/* Graph capture: after one call with the same plan_offsets and n_plans (which
 * uploads the plan map and the work lists), wo_eval_plans enqueues kernels
 * only (ticket reset kernels and one or two evaluation launches) and may be
 * captured into a HIP graph and replayed; WO_VALIDATE must be unset while
 * capturing. */

/* ------------------------------------------------------------------ */
/* Learned surrogate and screening                                      */
/* ------------------------------------------------------------------ */
/* The paper's hybrid decision making (section 1, Figure 1) trains machine
 * learning models on simulated scenarios and lets them decide; here the
 * simulator is the exact evaluator above and the model predicts a plan's
 * total distance from its slotting alone:
 *   x = one-hot(zone_of) as a 64 x 64 matrix (row = category, column = zone;
 *       categories >= n_categories and padding give zero rows) = 4096 inputs,
 *   h1 = GELU(x W1 + b1) (1024), h2 = GELU(h1 W2 + b2) (256),
 *   y = h2 W3 + b3, prediction = y * std + mean,
 * GELU in its tanh form.  Products run on MFMA with bf16 operands (weights
 * and activations) and fp32 accumulation; fp32 master weights; Adam.
 *
 * Host parameter layout (float32, WO_SUR_PARAMS values): W1 [4096][1024]
 * (input-major: y = x W + b), b1 [1024], W2 [1024][256], b2 [256],
 * W3 [256], b3 [1]. */
#define WO_SUR_PARAMS 4457985
#define WO_SCREEN_MAX_KEEP 4096

typedef struct wo_sur wo_sur;

/* Create a surrogate on the current device for instances with n_categories
 * categories (zone bytes of categories >= n_categories are ignored).
 * h_init: host parameters in the layout above, or NULL for He-uniform
 * weights drawn from `seed` by a counter generator (zero biases).
 * Synchronous. */
wo_status wo_sur_create(int32_t n_categories, const float *h_init, uint64_t seed, void *stream,
                        wo_sur **out);

/* Release a surrogate (NULL is a no-op); synchronises the device first. */
wo_status wo_sur_free(wo_sur *s);

/* Target standardisation used for training and prediction.  Without a call,
 * wo_sur_train sets it to the mean and standard deviation of its targets. */
wo_status wo_sur_set_scale(wo_sur *s, double mean, double std);
wo_status wo_sur_get_scale(const wo_sur *s, double *mean, double *std);

/* Copy the fp32 parameters to host memory (WO_SUR_PARAMS floats, layout
 * above).  Synchronises the device. */
wo_status wo_sur_get_params(const wo_sur *s, float *h_out);

/* Forward and backward pass of one batch without an update: gradients of
 * L = mean_b (y_b - t_b)^2 with respect to every parameter, into host memory
 * in the parameter layout, and the loss.  n: multiple of 128, at most 4096;
 * d_zone_of uint8[n][64]; d_target float[n] (standardised).  Synchronous. */
wo_status wo_sur_gradients(wo_sur *s, int32_t n, const uint8_t *d_zone_of, const float *d_target,
                           float *h_grad, float *h_loss, void *stream);

/* Train on n (plan, exact distance) pairs: d_zone_of uint8[n][64],
 * d_dist int32[n] (e.g. from wo_eval_plans).  Mini-batch Adam (lr, beta
 * 0.9 / 0.999, eps 1e-8) over `epochs` shuffled passes (each epoch's
 * shuffle is a keyed pseudorandom permutation of the samples, keyed by `seed`
 * and the epoch, evaluated on the device); batch a multiple of 128 in
 * [128, 4096]; a last partial batch is dropped; n <= 2^31 - 1.  h_last_loss (nullable) receives the mean batch loss of the last
 * epoch.  Returns when the work is done (it synchronises the stream). */
wo_status wo_sur_train(wo_sur *s, int64_t n, const uint8_t *d_zone_of, const int32_t *d_dist,
                       int32_t epochs, int32_t batch, float lr, uint64_t seed, float *h_last_loss,
                       void *stream);

/* Predicted distances (de-standardised) of n plans into d_pred float[n]
 * (async). */
wo_status wo_sur_predict(wo_sur *s, int64_t n, const uint8_t *d_zone_of, float *d_pred, void *stream);

/* Checkpoint: parameters, Adam moments, step count and standardisation to a
 * file, and a new surrogate from such a file (bit-exact resume). */
wo_status wo_sur_save(const wo_sur *s, const char *path);
wo_status wo_sur_load(const char *path, void *stream, wo_sur **out);

/* Screen n_plans candidate slottings of instance `inst`: predict each with
 * the surrogate and write the indices of the `keep` smallest predictions,
 * ordered by (prediction, index), to d_keep_idx int32[keep] (async).
 * d_pred (nullable) receives all predictions.  keep <= WO_SCREEN_MAX_KEEP,
 * n_plans <= 2^24.  The exact evaluator has the last word: re-score the kept
 * plans with wo_eval_plans. */
wo_status wo_screen_plans(wo_wh *wh, int32_t inst, wo_sur *s, int64_t n_plans, const uint8_t *d_zone_of,
                          float *d_pred, int64_t keep, int32_t *d_keep_idx, void *stream);

/* ------------------------------------------------------------------ */
/* Genetic plan search                                                  */
/* ------------------------------------------------------------------ */
/* The paper's top-level optimiser organises the subsystem searches from the
 * CPU (section 5, Figure 10); here a genetic algorithm over whole plans runs
 * on the device and the host only asks for generations.  Random draws come
 * from the SplitMix64 finaliser (Steele, Lea & Flood 2014) over
 *   h = sm(sm(sm(seed + stream) ^ (generation << 32 | child)) ^ position),
 *   r32 = h >> 32,  streams 1 tournament, 2 zone coin, 3 zone partner,
 *   4 insert coin, 5 insert target;
 * a coin succeeds when r32 < mutation_threshold; a uniform integer in [0, m)
 * is (r32 * m) >> 32.
 *   Tournament: `tournament` draws from the population, winner = smallest
 *   (distance, index).  Zone swap: for each category c in turn, on success
 *   swap its zone with uniform other category.  Order insert: for each
 *   sequence position i = 0 .. n-1 in turn, on success move the element
 *   currently at i so that it ends at uniform position j.
 * Plain generation (no surrogate): child 0 = the best individual unchanged;
 * child b >= 1 = tournament winner (child id b) with both mutations; all are
 * evaluated exactly and replace the population.
 * Screened generation (with a surrogate): `candidates` children (child id b)
 * take a tournament winner's zones with the zone swap; the surrogate keeps
 * the `keep` best by (prediction, index) (wo_screen_plans); each kept
 * candidate then takes its parent's sequence with the order insert (child id
 * = candidate id), is evaluated exactly and replaces one of the `keep` worst
 * individuals (largest distance, ties by smaller index), in rank order.
 * Generations count from 0 across calls. */
typedef struct {
    int32_t population;            /* 2 .. 2^24 */
    int32_t tournament;            /* 1 .. 64, e.g. 4 */
    uint32_t mutation_threshold;   /* per-position success if r32 < this; 85899345 = 0.02 */
    int32_t candidates;            /* screened children per generation (0: plain only) */
    int32_t keep;                  /* survivors of the screen, <= WO_SCREEN_MAX_KEEP, < population */
    uint64_t seed;
} wo_search_params;

typedef struct wo_search wo_search;

/* Create a search over instance `inst` of wh from an initial population
 * (d_init_zone_of uint8[population][64], d_init_seq uint16[population][n]),
 * which is copied and evaluated exactly.  Synchronous. */
wo_status wo_search_create(wo_wh *wh, int32_t inst, const wo_search_params *params,
                           const uint8_t *d_init_zone_of, const uint16_t *d_init_seq, void *stream,
                           wo_search **out);

/* Release a search (NULL is a no-op); synchronises the device first. */
wo_status wo_search_free(wo_search *s);

/* Run n_generations generations (async): plain when sur is NULL, screened
 * otherwise (the search must have been created with candidates > 0). */
wo_status wo_search_step(wo_wh *wh, wo_search *s, wo_sur *sur, int32_t n_generations, void *stream);

/* Checkpoint of a search to a file: the population, its distances, the
 * parameters and the generation counter.  Random numbers are a function of
 * (seed, generation, child, position), so a search resumed with
 * wo_search_load continues bit-exactly.  Synchronous. */
wo_status wo_search_save(wo_search *s, const char *path, void *stream);

/* Resume a search saved by wo_search_save on instance `inst` of wh, which
 * must have the same order and category counts; the population is evaluated
 * again and its distances must equal the saved ones (else WO_E_INVAL, as for
 * a file that is not a search checkpoint).  Synchronous. */
wo_status wo_search_load(wo_wh *wh, int32_t inst, const char *path, void *stream, wo_search **out);

/* Best individual so far (each argument nullable): zone row (64 bytes),
 * sequence (n entries), distance, generations run.  Synchronous. */
wo_status wo_search_best(wo_search *s, uint8_t *h_zone_of, uint16_t *h_seq, int32_t *h_dist,
                         int32_t *h_generation, void *stream);

/* Copy the population (each argument nullable) to device buffers, and the
 * candidate ids kept by the last screened generation (int32[keep]).  Async. */
wo_status wo_search_population(wo_search *s, uint8_t *d_zone_of, uint16_t *d_seq, int32_t *d_dist,
                               int32_t *d_last_kept, void *stream);

/* ------------------------------------------------------------------ */
/* Aisle width design                                                   */
/* ------------------------------------------------------------------ */
/* Section 5, Subproblem 1, Eq. (1): maximise the share of the floor the
 * racks take, A_ind / A_max, with the width a between racks as the design
 * variable, subject to k * delta - a <= 0, where delta is the picking
 * frequency Subproblem 2 returns for the plan (Eq. (2): delta = f(d)).
 * Reading of the single-block geometry: each aisle is a corridor of width a
 * with a rack face of depth r on each side (neighbouring aisles' racks stand
 * back to back), so aisles are a + 2 r apart centre to centre; racks are
 * L = slots_per_side * pitch long; a cross aisle of width c runs along the
 * front and the back:
 *     A_ind / A_max = 2 r L / ((a + 2 r) (L + 2 c)),
 * falling with a.  delta is the evaluator's orders per window,
 * n_orders * window / (D / walk + t_item * items), and D grows with the
 * spacing, so the constraint holds from one width on and the optimum is the
 * smallest width in [min_width_dm, max_width_dm] that meets it.  k is the
 * width (dm) the flow of one order per window needs. */
#define WO_AISLE_MAX_WIDTHS 4096
typedef struct {
    int32_t rack_depth_dm;     /* r >= 1 */
    int32_t cross_aisle_dm;    /* c >= 0 */
    int32_t min_width_dm;      /* >= 1 */
    int32_t max_width_dm;      /* >= min; at most WO_AISLE_MAX_WIDTHS widths in the range */
    double k_dm;               /* >= 0 */
} wo_aisle_params;

typedef struct {
    int32_t width_dm;          /* the optimum a (max_width_dm when no width is feasible) */
    int32_t spacing_dm;        /* a + 2 r: the aisles' centre-to-centre distance */
    int32_t feasible;          /* 1 when k * delta <= a holds at width_dm */
    int32_t widths_evaluated;
    int32_t distance;          /* D of the plan at width_dm (int32, saturating) */
    double orders_per_window;  /* delta at width_dm, in IEEE double */
    double utilization;        /* A_ind / A_max at width_dm */
} wo_aisle_result;

/* Evaluates the plan of instance `inst` (d_zone_of: 64 bytes, d_order_seq:
 * n_orders uint16 on the device) at every whole-decimetre width of the range
 * in one launch of the exact evaluator, each copy of the plan with its own
 * spacing (the load's spacing_dm is not used), and returns the narrowest
 * width meeting the constraint, deciding each width in IEEE double from the
 * integer distance.  h_dist (host int32[max - min + 1], nullable) receives
 * D at every width.  The handle's route and batching apply; the optimal
 * route needs 4 (max + 2 r)(N + 2) + 4 L (N + 1) < 2^30 dm (else
 * WO_E_RANGE).  Synchronous; allocates its own buffers. */
wo_status wo_aisle_width(wo_wh *wh, int32_t inst, const uint8_t *d_zone_of, const uint16_t *d_order_seq,
                         const wo_aisle_params *params, int32_t *h_dist, void *stream, wo_aisle_result *out);

/* ------------------------------------------------------------------ */
/* Order categories (SVM)                                               */
/* ------------------------------------------------------------------ */
/* Section 5, subroutine 5: every order belongs to a category of orders; an
 * SVM (Cortes and Vapnik 1995) configures the categories from the outputs of
 * the subroutines before it and is refreshed continuously from a window of
 * the most recent orders, newer data replacing older.  Readings (the paper
 * gives no features, model or rule):
 *   - an order's features are the shares of its lines in each product
 *     category (e.g. the K-means classes of Subproblem 3):
 *     x[c] = (lines whose SKU is in category c) / (lines of the order);
 *   - one linear SVM per category of orders against the rest: hinge loss
 *     plus lambda / 2 times the squared norm of the weights, the bias being
 *     the weight of a constant feature 1;
 *   - training: full-batch subgradient steps over the window with the step
 *     sizes of Pegasos (Shalev-Shwartz et al. 2007), eta_t = 1 / (lambda t),
 *     t counting every step since creation;
 *   - an order takes the category of the largest score (ties: the lower).
 * All arithmetic is IEEE double, one operation at a time, every sum in a
 * fixed order (features by index, samples from the oldest), so results do
 * not depend on the launch shape.  Labels outside [0, n_classes) count as
 * negatives for every class. */
#define WO_SVM_MAX_FEATURES 64
#define WO_SVM_MAX_CLASSES 64
#define WO_SVM_MAX_WINDOW (1 << 22)

typedef struct wo_svm wo_svm;

/* Features of n_orders orders (async): d_order_offsets int32[n_orders + 1],
 * d_order_skus int32[n_lines], d_sku_category int32[n_skus] (each in
 * [0, n_features) to count), d_features double[n_orders][n_features] out.
 * Lines outside [0, n_lines), SKUs outside [0, n_skus) and categories outside
 * [0, n_features) count in the order's length only. */
wo_status wo_order_features(const int32_t *d_order_offsets, const int32_t *d_order_skus, int32_t n_orders,
                            int64_t n_lines, const int32_t *d_sku_category, int32_t n_skus, int32_t n_features,
                            double *d_features, void *stream);

/* An SVM over n_features (1 .. 64) features and n_classes (2 .. 64)
 * categories, refreshed from a window of the last `window` samples
 * (1 .. WO_SVM_MAX_WINDOW); weights start at zero.  Synchronous. */
wo_status wo_svm_create(int32_t n_features, int32_t n_classes, int32_t window, double lambda, void *stream,
                        wo_svm **out);
wo_status wo_svm_free(wo_svm *s);

/* Append n samples to the window (async): d_features double[n][F],
 * d_labels int32[n]; the window keeps the last `window` samples pushed. */
wo_status wo_svm_push(wo_svm *s, int64_t n, const double *d_features, const int32_t *d_labels, void *stream);

/* `iterations` subgradient steps on the window's samples from the current
 * weights (async); WO_E_STATE when the window is empty. */
wo_status wo_svm_train(wo_svm *s, int32_t iterations, void *stream);

/* Category of each of n samples into d_class int32[n] (async). */
wo_status wo_svm_predict(wo_svm *s, int64_t n, const double *d_features, int32_t *d_class, void *stream);

/* Weights (host double[n_classes][n_features + 1], bias last; nullable),
 * steps so far and samples in the window (each nullable).  Synchronous. */
wo_status wo_svm_get_weights(wo_svm *s, double *h_weights, int64_t *h_steps, int64_t *h_window_count,
                             void *stream);

/* ------------------------------------------------------------------ */
/* Diagnostics                                                          */
/* ------------------------------------------------------------------ */

/* Measured 32-bit integer VALU throughput of the current device, in
 * operations per second: the denominator of the evaluator's roofline
 * measured rather than derived from unit counts and clock.  Every lane of a
 * grid that fills every CU runs independent chains of 32-bit adds and
 * exclusive ors (one operation per lane per instruction); the best of `reps`
 * (1 .. 100) timed launches counts.  Synchronous; allocates a small output
 * buffer. */
wo_status wo_measure_int_peak(int32_t reps, double *ops_per_s, void *stream);

/* Measured peaks of the current device, the denominators of the rooflines
 * measured rather than taken from published figures: the integer VALU rate
 * as wo_measure_int_peak gives it; the LDS read bandwidth (every wave reads
 * 1 KB per instruction, without bank conflicts); the HBM read bandwidth (a
 * 1 GiB buffer read once with 16-byte loads); the dense BF16 MFMA rate
 * (four independent 32 x 32 x 16 products per wave); the L2 read bandwidth
 * (each XCD re-reads a 2 MB slice of its own, 64 times, with 16-byte loads;
 * workgroup b is taken to run on XCD b % 8).  Each is the best of
 * `reps` (1 .. 100) timed launches.  Synchronous; allocates 1 GiB and small
 * output buffers for the call. */
typedef struct {
    double int_ops_per_s;
    double lds_bytes_per_s;
    double hbm_read_bytes_per_s;
    double bf16_flops_per_s;
    double l2_read_bytes_per_s;
} wo_peaks;
wo_status wo_measure_peaks(int32_t reps, wo_peaks *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WO_H */
