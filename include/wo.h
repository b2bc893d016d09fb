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

/* Short human-readable name of a status code (static string). */
const char *wo_status_str(wo_status s);

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
} wo_instance_desc;

typedef struct wo_wh wo_wh;

/* Load n_instances (>= 1) instances onto the current HIP device.
 * Validates every descriptor (WO_E_INVAL / WO_E_RANGE), packs per-line
 * records and order tables, copies them to device memory on `stream` and
 * synchronises it.  On success *out owns the device memory until
 * wo_free_warehouse.  Synchronous. */
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

#ifdef __cplusplus
}
#endif

#endif /* WO_H */
