/*
 * wo_oracle.c -- plain, sequential CPU oracle for picking-plan evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * What it computes (arXiv 2110.13693, section 5, Subproblem 2, Eq. (2): the
 * route objective is a sum of per-route distances d_i, and the picking
 * frequency is a function delta = f(d) of that distance; Subproblem 3: product
 * placement by category; section 6: clustering categories and choosing the
 * order sequence within a time frame).  A plan is
 *   - zone_of[c]: the zone that category c occupies (a permutation of the
 *     categories), and
 *   - seq[i]: the order picked i-th (a permutation of the orders).
 * Evaluation, one plan, in the order the method states it:
 *   1. slot map: zones are contiguous location ranges laid out in zone order;
 *      zone z is exactly as long as the category it holds; inside a category
 *      the SKUs sit in ascending SKU id (id = popularity rank);
 *   2. location decode: location l lies in aisle l / (2S), at depth index
 *      (l mod 2S) / 2 (side = l mod 2 does not change the walk), depth
 *      coordinate y = j * pitch + pitch / 2 from the front cross aisle;
 *   3. tours: next-fit over seq -- an order joins the open tour if the tour's
 *      item count plus the order's stays <= capacity, otherwise it opens a new
 *      tour; an order is never split (an order larger than the capacity is a
 *      tour of its own); or, when the instance asks for it, first fit
 *      (orc_tours_first_fit below) or seed batching (orc_tours_seed below);
 *   4. route per tour, by one of the standard policies of the routing
 *      literature the paper builds on (de Koster et al. 2007), depot at the
 *      front of aisle 0, L = S * pitch:
 *      - S-shape (the default): every aisle holding a pick is traversed
 *        entirely, in ascending order; if the number k of such aisles is odd
 *        the last one is entered from the front and left the same way after
 *        its farthest pick;
 *        cost = 2 * spacing * a_max + (k even ? k * L : (k - 1) * L + 2 * y_far);
 *      - return: every aisle holding a pick is entered from the front up to
 *        its farthest pick and left the same way;
 *        cost = 2 * spacing * a_max + sum over those aisles of 2 * y_max;
 *      - largest gap: the first and the last aisle holding picks are
 *        traversed entirely (front to back, then back to front); every other
 *        such aisle is entered from the front and from the back, each time up
 *        to its largest gap and back, the largest gap being the longest of:
 *        front to first pick, between adjacent picks, last pick to back;
 *        cost = 2 * spacing * a_max + 2 * L + sum over the inner aisles of
 *        2 * (L - gap); with a single aisle it is the return route;
 *      - combined: every aisle holding a pick is visited once, in ascending
 *        order, and either crossed to the other cross aisle or entered and
 *        left from the cross aisle the picker is on, whichever choice makes
 *        the whole walk shortest (orc_combined_cost below);
 *      - optimal: the shortest closed walk from the depot through every pick
 *        (the paper's minimum route distance), by a dynamic programme over the
 *        aisles (orc_optimal_cost below states it);
 *   5. D = sum of tour costs (exact in int64; the int32 output saturates at
 *      INT32_MAX);
 *   6. throughput over the time window (delta = f(d)):
 *      T = D / walk_speed + seconds_per_item * items,
 *      orders_per_window = n_orders * window / T, evaluated in double and
 *      rounded once to float.
 */
#include <errno.h>
#include <limits.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_CAT 64
#define ORC_ZONE_PAD 0xFF

typedef struct {
    int32_t n_aisles, slots_per_side, pitch_dm, spacing_dm, capacity, n_categories;
    int32_t n_skus;
    const int32_t *sku_category;   /* [n_skus] */
    int32_t n_orders;
    const int32_t *order_offsets;  /* [n_orders + 1] */
    const int32_t *order_skus;     /* [order_offsets[n_orders]] */
    double walk_dm_per_s, seconds_per_item, window_s;
    int32_t routing;               /* ORC_ROUTE_* */
    int32_t batching;              /* ORC_BATCH_* */
} orc_instance;

enum { ORC_ROUTE_SSHAPE = 0, ORC_ROUTE_RETURN = 1, ORC_ROUTE_LARGEST_GAP = 2, ORC_ROUTE_OPTIMAL = 3,
       ORC_ROUTE_COMBINED = 4 };
enum { ORC_BATCH_NEXT_FIT = 0, ORC_BATCH_FIRST_FIT = 1, ORC_BATCH_SEED = 2 };

enum { ORC_OK = 0, ORC_E_INVAL = 1, ORC_E_NOMEM = 3 };

/* ------------------------------------------------------------------ */
/* step 1: slot map (Subproblem 3: placement grouped by category)      */
/* ------------------------------------------------------------------ */

/* loc_of_sku[s] for every SKU under zone assignment zone_of. */
int orc_locations(const orc_instance *w, const uint8_t *zone_of, int32_t *loc_of_sku)
{
    int C = w->n_categories;
    int64_t size[ORC_MAX_CAT] = {0};
    int64_t start[ORC_MAX_CAT];
    int cat_in_zone[ORC_MAX_CAT];
    int64_t next_rank[ORC_MAX_CAT] = {0};
    int c, z;
    int32_t s;

    if (C < 1 || C > ORC_MAX_CAT) return ORC_E_INVAL;
    for (z = 0; z < C; z++) cat_in_zone[z] = -1;
    for (c = 0; c < C; c++) {
        if (zone_of[c] >= C || cat_in_zone[zone_of[c]] != -1) return ORC_E_INVAL;
        cat_in_zone[zone_of[c]] = c;
    }
    for (s = 0; s < w->n_skus; s++) {
        int32_t cs = w->sku_category[s];
        if (cs < 0 || cs >= C) return ORC_E_INVAL;
        size[cs]++;
    }
    /* zones are laid out one after another in zone order */
    {
        int64_t acc = 0;
        for (z = 0; z < C; z++) {
            start[cat_in_zone[z]] = acc;
            acc += size[cat_in_zone[z]];
        }
        if (acc > 2LL * w->n_aisles * w->slots_per_side) return ORC_E_INVAL;
    }
    /* inside a zone: ascending SKU id */
    for (s = 0; s < w->n_skus; s++) {
        int32_t cs = w->sku_category[s];
        loc_of_sku[s] = (int32_t)(start[cs] + next_rank[cs]);
        next_rank[cs]++;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* step 2: location decode                                             */
/* ------------------------------------------------------------------ */

void orc_decode(const orc_instance *w, int32_t loc, int32_t *aisle, int32_t *y)
{
    int32_t per_aisle = 2 * w->slots_per_side;
    int32_t j = (loc % per_aisle) / 2;
    *aisle = loc / per_aisle;
    *y = j * w->pitch_dm + w->pitch_dm / 2;
}

/* ------------------------------------------------------------------ */
/* step 3: next-fit tours over the order sequence                      */
/* ------------------------------------------------------------------ */

/* tour_first[t] = position in seq of tour t's first order; tour_first[n_tours]
 * = n_orders.  tour_first must hold n_orders + 1 entries. */
int orc_tours(const orc_instance *w, const uint16_t *seq, int32_t *tour_first, int32_t *n_tours)
{
    int32_t i, t = 0;
    int64_t load = 0;
    for (i = 0; i < w->n_orders; i++) {
        int32_t o = seq[i];
        int64_t items;
        if (o >= w->n_orders) return ORC_E_INVAL;
        items = w->order_offsets[o + 1] - w->order_offsets[o];
        if (i == 0 || load + items > w->capacity) {
            tour_first[t++] = i;   /* open a new tour */
            load = 0;
        }
        load += items;
    }
    tour_first[t] = w->n_orders;
    *n_tours = t;
    return ORC_OK;
}

/* First fit, the other greedy order-batching rule of the literature: each
 * order, in sequence, joins the earliest-opened tour whose item count plus
 * the order's stays <= capacity; when no open tour has room it opens a new
 * one.  An order larger than the capacity therefore gets a tour of its own,
 * which nothing joins later.  tour_of[i] = tour of the order at position i,
 * tours numbered in opening order. */
int orc_tours_first_fit(const orc_instance *w, const uint16_t *seq, int32_t *tour_of, int32_t *n_tours)
{
    int32_t i, t, T = 0;
    int64_t *load = (int64_t *)malloc(sizeof(int64_t) * (size_t)w->n_orders);
    if (!load) return ORC_E_NOMEM;
    for (i = 0; i < w->n_orders; i++) {
        int32_t o = seq[i];
        int64_t items;
        if (o >= w->n_orders) { free(load); return ORC_E_INVAL; }
        items = w->order_offsets[o + 1] - w->order_offsets[o];
        for (t = 0; t < T; t++)
            if (load[t] + items <= w->capacity) break;
        if (t == T) load[T++] = 0;   /* open a new tour */
        load[t] += items;
        tour_of[i] = t;
    }
    free(load);
    *n_tours = T;
    return ORC_OK;
}

/* Seed batching, the third greedy rule of the order-batching literature
 * (seed algorithms; de Koster, Van der Poort and Wolters 1999): tours are
 * built one at a time.  A tour starts from a seed, the order earliest in the
 * sequence that is in no tour yet; then, while some such order fits (the
 * tour's item count plus the order's stays <= capacity), the one that adds
 * the fewest aisles the tour does not visit yet joins it, ties going to the
 * order earlier in the sequence.  An order's aisles are those of its lines'
 * locations under the plan's slotting (loc_of_sku).  An order larger than the
 * capacity never fits a tour it does not seed, and a tour it seeds takes
 * nothing else.  tour_of[i] = tour of the order at position i, tours numbered
 * in the order they are built. */
int orc_tours_seed(const orc_instance *w, const int32_t *loc_of_sku, const uint16_t *seq, int32_t *tour_of,
                   int32_t *n_tours)
{
    const int32_t n = w->n_orders, per_aisle = 2 * w->slots_per_side;
    int32_t i, T = 0;
    int32_t *visits = (int32_t *)malloc(sizeof(int32_t) * (size_t)w->n_aisles);   /* tour that last visited */
    int32_t *seen = (int32_t *)malloc(sizeof(int32_t) * (size_t)w->n_aisles);     /* order scan that saw it */
    int32_t stamp = 0;
    if (!visits || !seen) { free(visits); free(seen); return ORC_E_NOMEM; }
    for (i = 0; i < w->n_aisles; i++) visits[i] = -1, seen[i] = -1;
    for (i = 0; i < n; i++) {
        if (seq[i] >= n) { free(visits); free(seen); return ORC_E_INVAL; }
        tour_of[i] = -1;
    }
    for (;;) {
        int32_t s = -1, l;
        int64_t load;
        for (i = 0; i < n; i++)
            if (tour_of[i] < 0) { s = i; break; }
        if (s < 0) break;
        /* the seed */
        tour_of[s] = T;
        load = w->order_offsets[seq[s] + 1] - w->order_offsets[seq[s]];
        for (l = w->order_offsets[seq[s]]; l < w->order_offsets[seq[s] + 1]; l++)
            visits[loc_of_sku[w->order_skus[l]] / per_aisle] = T;
        for (;;) {
            int32_t best = -1, best_new = 0;
            for (i = 0; i < n; i++) {
                int32_t o = seq[i], fresh = 0;
                if (tour_of[i] >= 0) continue;
                if (load + (w->order_offsets[o + 1] - w->order_offsets[o]) > w->capacity) continue;
                /* distinct aisles of the order that the tour does not visit */
                stamp++;
                for (l = w->order_offsets[o]; l < w->order_offsets[o + 1]; l++) {
                    int32_t a = loc_of_sku[w->order_skus[l]] / per_aisle;
                    if (visits[a] != T && seen[a] != stamp) fresh++;
                    seen[a] = stamp;
                }
                if (best < 0 || fresh < best_new) best = i, best_new = fresh;
            }
            if (best < 0) break;
            tour_of[best] = T;
            load += w->order_offsets[seq[best] + 1] - w->order_offsets[seq[best]];
            for (l = w->order_offsets[seq[best]]; l < w->order_offsets[seq[best] + 1]; l++)
                visits[loc_of_sku[w->order_skus[l]] / per_aisle] = T;
        }
        T++;
    }
    free(visits); free(seen);
    *n_tours = T;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* step 4: S-shape cost of one tour, given its pick locations          */
/* ------------------------------------------------------------------ */

int64_t orc_sshape_cost(const orc_instance *w, const int32_t *locs, int32_t n)
{
    int64_t L = (int64_t)w->slots_per_side * w->pitch_dm;
    char *visited;
    int32_t i, k = 0, a_max = -1, y_far = 0;
    int64_t cost;

    if (n <= 0) return 0;
    visited = (char *)calloc((size_t)w->n_aisles, 1);
    if (!visited) return -1;
    for (i = 0; i < n; i++) {
        int32_t a, y;
        orc_decode(w, locs[i], &a, &y);
        if (!visited[a]) { visited[a] = 1; k++; }
        if (a > a_max) { a_max = a; y_far = y; }
        else if (a == a_max && y > y_far) y_far = y;
    }
    free(visited);
    cost = 2LL * w->spacing_dm * a_max;
    if (k % 2 == 0) cost += (int64_t)k * L;
    else cost += (int64_t)(k - 1) * L + 2LL * y_far;
    return cost;
}

/* Return and largest gap need every pick's depth per aisle: the picks are
 * decoded and sorted by (aisle, depth), then each aisle is one run. */
typedef struct { int32_t a, y; } orc_pick;

static int orc_pick_cmp(const void *p, const void *q)
{
    const orc_pick *x = (const orc_pick *)p, *z = (const orc_pick *)q;
    if (x->a != z->a) return x->a < z->a ? -1 : 1;
    return x->y < z->y ? -1 : (x->y > z->y);
}

static orc_pick *orc_sorted_picks(const orc_instance *w, const int32_t *locs, int32_t n)
{
    int32_t i;
    orc_pick *pk = (orc_pick *)malloc(sizeof(orc_pick) * (size_t)n);
    if (!pk) return NULL;
    for (i = 0; i < n; i++) orc_decode(w, locs[i], &pk[i].a, &pk[i].y);
    qsort(pk, (size_t)n, sizeof(orc_pick), orc_pick_cmp);
    return pk;
}

int64_t orc_return_cost(const orc_instance *w, const int32_t *locs, int32_t n)
{
    int32_t i;
    int64_t cost;
    orc_pick *pk;
    if (n <= 0) return 0;
    pk = orc_sorted_picks(w, locs, n);
    if (!pk) return -1;
    cost = 2LL * w->spacing_dm * pk[n - 1].a;
    for (i = 0; i < n; i++)
        if (i == n - 1 || pk[i + 1].a != pk[i].a) cost += 2LL * pk[i].y;   /* farthest pick of its aisle */
    free(pk);
    return cost;
}

int64_t orc_largest_gap_cost(const orc_instance *w, const int32_t *locs, int32_t n)
{
    int64_t L = (int64_t)w->slots_per_side * w->pitch_dm;
    int32_t i, first, a_lo, a_hi;
    int64_t cost;
    orc_pick *pk;
    if (n <= 0) return 0;
    pk = orc_sorted_picks(w, locs, n);
    if (!pk) return -1;
    a_lo = pk[0].a;
    a_hi = pk[n - 1].a;
    if (a_lo == a_hi) {
        cost = 2LL * w->spacing_dm * a_hi + 2LL * pk[n - 1].y;
        free(pk);
        return cost;
    }
    cost = 2LL * w->spacing_dm * a_hi + 2 * L;
    for (first = 0; first < n; first = i) {
        int64_t gap;
        for (i = first; i < n && pk[i].a == pk[first].a; i++) {}
        if (pk[first].a == a_lo || pk[first].a == a_hi) continue;
        gap = pk[first].y;                                   /* front to first pick */
        if (L - pk[i - 1].y > gap) gap = L - pk[i - 1].y;    /* last pick to back */
        {
            int32_t j;
            for (j = first; j + 1 < i; j++)
                if (pk[j + 1].y - pk[j].y > gap) gap = pk[j + 1].y - pk[j].y;
        }
        cost += 2 * (L - gap);
    }
    free(pk);
    return cost;
}

/* Optimal route (the paper's minimum route distance, section 5, Subproblem 2,
 * found there by trying visiting orders).  In a single-block warehouse the
 * shortest closed walk from the depot through every pick is found exactly by
 * a dynamic programme over the aisles from left to right, in the manner of
 * Ratliff and Rosenthal (1983).  It is stated here from first principles:
 *
 *   A closed walk is a connected multigraph on the aisle graph in which every
 *   vertex has even degree; an edge is never needed more than twice.  The
 *   vertices are the two ends of every aisle (front f_j at y = 0, back b_j at
 *   y = L), the picks, and the depot (= f_0).  The programme decides, column
 *   by column, first the vertical edges inside aisle j, then the horizontal
 *   edges f_j-f_{j+1} and b_j-b_{j+1} (0, 1 or 2 copies each).  After a column
 *   only f_j and b_j can still gain edges, so a partial solution is described
 *   by: for each of f_j, b_j whether it is absent (no edge, not the depot),
 *   of even or of odd degree; whether the two lie in one component; and
 *   whether a component has been closed off (it can touch nothing to the
 *   right, so it must be the whole walk: the state DONE).
 *
 *   Inside an aisle with picks y_1 <= ... <= y_m, every pick needs even
 *   degree > 0, so the m + 1 segments (front-y_1, ..., y_m-back) all have the
 *   same multiplicity parity: either all are used once (a traversal, cost L,
 *   joining f_j and b_j) or each is used 0 or 2 times.  In the second case the
 *   doubled segments must reach the front or the back (a doubled run touching
 *   neither is a component that can never join the rest), so exactly one
 *   segment is left out (cost 2 (L - that segment), picks below it hang on
 *   f_j, picks above it on b_j) or none (cost 2 L, joining f_j and b_j).  An
 *   aisle without picks may also be left empty.
 *
 *   A horizontal edge from an absent vertex would be a dead end that can be
 *   removed, so it is not generated.  The walk never needs a column right of
 *   the last aisle with picks, nor left of the depot's aisle 0. */
enum { ORC_ABSENT = 0, ORC_EVEN = 1, ORC_ODD = 2 };
#define ORC_NSTATE 19            /* (front, back, joined) + DONE */
#define ORC_DONE 18
#define ORC_INF ((int64_t)1 << 60)

static int orc_state(int f, int b, int joined) { return (f * 3 + b) * 2 + (f && b ? joined : 0); }

static int orc_add_degree(int st, int d)
{
    if (d == 0) return st;
    if (st == ORC_ABSENT) return (d & 1) ? ORC_ODD : ORC_EVEN;
    if (d & 1) return st == ORC_ODD ? ORC_EVEN : ORC_ODD;
    return st;
}

static void orc_relax(int64_t *cost, int s, int64_t c)
{
    if (c < cost[s]) cost[s] = c;
}

/* One vertical pattern of aisle j applied to state s (not DONE).
 * df, db: degree added at the front and back end; join: the pattern links
 * front and back; lo_f / hi_b: some picks hang on the front / back end only. */
static void orc_vertical(int64_t *out, int s, int64_t c, int df, int db, int join, int lo_f, int hi_b)
{
    int f = s / 6, b = (s / 2) % 3, joined = s & 1;
    int nf = orc_add_degree(f, df), nb = orc_add_degree(b, db);
    if (join) {
        joined = 1;                          /* the pattern is a path from f_j to b_j */
    } else {
        /* an end that was absent and gains edges starts a new component:
         * it is not joined to the other end */
        if ((lo_f && f == ORC_ABSENT) || (hi_b && b == ORC_ABSENT)) joined = 0;
    }
    orc_relax(out, orc_state(nf, nb, joined), c);
}

int64_t orc_optimal_cost(const orc_instance *w, const int32_t *locs, int32_t n)
{
    const int64_t L = (int64_t)w->slots_per_side * w->pitch_dm;
    const int64_t sp = w->spacing_dm;
    int64_t cur[ORC_NSTATE], nxt[ORC_NSTATE], best;
    int32_t i, j, first, a_max;
    orc_pick *pk;
    if (n <= 0) return 0;
    pk = orc_sorted_picks(w, locs, n);
    if (!pk) return -1;
    a_max = pk[n - 1].a;

    for (i = 0; i < ORC_NSTATE; i++) cur[i] = ORC_INF;
    cur[orc_state(ORC_EVEN, ORC_ABSENT, 0)] = 0;        /* the depot at f_0, no edge yet */
    first = 0;
    for (j = 0; j <= a_max; j++) {
        int32_t last = first, s, g;
        while (last < n && pk[last].a == j) last++;   /* picks of aisle j: [first, last) */
        /* vertical edges inside aisle j */
        for (i = 0; i < ORC_NSTATE; i++) nxt[i] = ORC_INF;
        for (s = 0; s < ORC_NSTATE; s++) {
            int64_t c = cur[s];
            if (c >= ORC_INF) continue;
            if (s == ORC_DONE) {                     /* nothing may be added any more */
                if (last == first) orc_relax(nxt, ORC_DONE, c);
                continue;
            }
            if (last == first) orc_vertical(nxt, s, c, 0, 0, 0, 0, 0);      /* left empty */
            orc_vertical(nxt, s, c + L, 1, 1, 1, 0, 0);                      /* traversed once */
            orc_vertical(nxt, s, c + 2 * L, 2, 2, 1, 0, 0);                  /* traversed twice */
            for (g = first; g <= last && last > first; g++) {
                /* leave out segment g: from y_{g-1} (front if g = first) to
                 * y_g (back if g = last); everything else doubled */
                int64_t lo = g == first ? 0 : pk[g - 1].y;
                int64_t hi = g == last ? L : pk[g].y;
                int has_lo = g > first, has_hi = g < last;
                orc_vertical(nxt, s, c + 2 * (L - (hi - lo)), has_lo ? 2 : 0, has_hi ? 2 : 0, 0,
                             has_lo, has_hi);
            }
        }
        memcpy(cur, nxt, sizeof cur);
        first = last;
        if (j == a_max) break;
        /* horizontal edges to column j + 1 */
        for (i = 0; i < ORC_NSTATE; i++) nxt[i] = ORC_INF;
        for (s = 0; s < ORC_NSTATE; s++) {
            int hf, hb, f = s / 6, b = (s / 2) % 3, joined = s & 1;
            int64_t c = cur[s];
            if (c >= ORC_INF) continue;
            if (s == ORC_DONE) { orc_relax(nxt, ORC_DONE, c); continue; }
            for (hf = 0; hf <= 2; hf++)
                for (hb = 0; hb <= 2; hb++) {
                    if ((f == ORC_ABSENT && hf) || (b == ORC_ABSENT && hb)) continue;
                    /* f_j and b_j are final now: even degree */
                    if (f != ORC_ABSENT && orc_add_degree(f, hf) != ORC_EVEN) continue;
                    if (b != ORC_ABSENT && orc_add_degree(b, hb) != ORC_EVEN) continue;
                    if (f && b && !joined) {
                        /* two components: each must continue to the right */
                        if (!hf || !hb) continue;
                    } else if (!hf && !hb) {
                        orc_relax(nxt, ORC_DONE, c);      /* the one component closes */
                        continue;
                    }
                    orc_relax(nxt, orc_state(orc_add_degree(ORC_ABSENT, hf), orc_add_degree(ORC_ABSENT, hb),
                                             joined || !(f && b)),
                              c + sp * (hf + hb));
                }
        }
        memcpy(cur, nxt, sizeof cur);
    }
    free(pk);
    /* the walk ends after aisle a_max: even ends, one component */
    best = cur[ORC_DONE];
    for (i = 0; i < ORC_NSTATE; i++) {
        int f = i / 6, b = (i / 2) % 3;
        if (i == ORC_DONE || f == ORC_ODD || b == ORC_ODD || (f == ORC_ABSENT && b == ORC_ABSENT)) continue;
        if (f && b && !(i & 1)) continue;
        if (cur[i] < best) best = cur[i];
    }
    return best;
}

/* Combined route (the combined heuristic of the routing literature the paper
 * builds on, which mixes S-shape crossings and return visits).  Reading: the
 * picker starts at the depot on the front cross aisle and visits the aisles
 * holding picks once each, in ascending order, moving along the cross aisle it
 * is on; in each it either crosses the aisle (L, ending on the other cross
 * aisle) or goes in from its own cross aisle to the farthest pick and back
 * (2 y_max from the front, 2 (L - y_min) from the back).  After the last aisle
 * it returns to the depot along the front, first crossing the last aisle if
 * it is on the back.  The choices are made by a programme over the aisles
 * with one state per cross aisle; S-shape and return are two of the choices,
 * so the route is never longer than either. */
int64_t orc_combined_cost(const orc_instance *w, const int32_t *locs, int32_t n)
{
    const int64_t L = (int64_t)w->slots_per_side * w->pitch_dm;
    const int64_t sp = w->spacing_dm;
    int64_t front = 0, back = -1;          /* best length so far ending on each cross aisle (-1: none) */
    int32_t i, first, prev = 0;
    orc_pick *pk;
    if (n <= 0) return 0;
    pk = orc_sorted_picks(w, locs, n);
    if (!pk) return -1;
    for (first = 0; first < n; first = i) {
        int32_t a = pk[first].a;
        int64_t ylo = pk[first].y, yhi, f2, b2, step;
        for (i = first; i < n && pk[i].a == a; i++) {}
        yhi = pk[i - 1].y;
        step = sp * (a - prev);
        prev = a;
        /* arrive along the same cross aisle, then return or cross */
        f2 = front + step + 2 * yhi;                            /* front, return */
        b2 = front + step + L;                                  /* front, crossed */
        if (back >= 0) {
            int64_t bb = back + step + 2 * (L - ylo);           /* back, return */
            int64_t bf = back + step + L;                       /* back, crossed */
            if (bb < b2) b2 = bb;
            if (bf < f2) f2 = bf;
        }
        front = f2;
        back = b2;
    }
    free(pk);
    /* home along the front; from the back, cross the last aisle first */
    {
        int64_t home_f = front + sp * prev, home_b = back + L + sp * prev;
        return home_f < home_b ? home_f : home_b;
    }
}

int64_t orc_tour_cost(const orc_instance *w, const int32_t *locs, int32_t n)
{
    switch (w->routing) {
    case ORC_ROUTE_RETURN: return orc_return_cost(w, locs, n);
    case ORC_ROUTE_LARGEST_GAP: return orc_largest_gap_cost(w, locs, n);
    case ORC_ROUTE_OPTIMAL: return orc_optimal_cost(w, locs, n);
    case ORC_ROUTE_COMBINED: return orc_combined_cost(w, locs, n);
    default: return orc_sshape_cost(w, locs, n);
    }
}

/* ------------------------------------------------------------------ */
/* steps 5-6: one whole plan                                           */
/* ------------------------------------------------------------------ */

static float orc_throughput(const orc_instance *w, int64_t D)
{
    double items = (double)w->order_offsets[w->n_orders];
    double T = (double)D / w->walk_dm_per_s + w->seconds_per_item * items;
    double r = ((double)w->n_orders * w->window_s) / T;
    return (float)r;
}

/* Scratch: loc_of_sku [n_skus], tour_first [n_orders+1], picks [max tour lines]. */
static int orc_eval_plan_ws(const orc_instance *w, const uint8_t *zone_of, const uint16_t *seq,
                            int32_t *loc_of_sku, int32_t *tour_first, int32_t *picks,
                            int64_t *dist_exact, int32_t *dist, float *thr)
{
    int32_t t, n_tours, i;
    int64_t D = 0;
    int rc = orc_locations(w, zone_of, loc_of_sku);
    if (rc) return rc;
    if (w->batching == ORC_BATCH_FIRST_FIT || w->batching == ORC_BATCH_SEED) {
        /* tour_first holds the tour of every position here; a tour's picks
         * are the lines of its orders */
        rc = w->batching == ORC_BATCH_SEED ? orc_tours_seed(w, loc_of_sku, seq, tour_first, &n_tours)
                                           : orc_tours_first_fit(w, seq, tour_first, &n_tours);
        if (rc) return rc;
        for (t = 0; t < n_tours; t++) {
            int32_t n = 0;
            int64_t c;
            for (i = 0; i < w->n_orders; i++) {
                int32_t o = seq[i], l;
                if (tour_first[i] != t) continue;
                for (l = w->order_offsets[o]; l < w->order_offsets[o + 1]; l++)
                    picks[n++] = loc_of_sku[w->order_skus[l]];
            }
            c = orc_tour_cost(w, picks, n);
            if (c < 0) return ORC_E_NOMEM;
            D += c;
        }
        goto done;
    }
    rc = orc_tours(w, seq, tour_first, &n_tours);
    if (rc) return rc;
    for (t = 0; t < n_tours; t++) {
        int32_t n = 0;
        for (i = tour_first[t]; i < tour_first[t + 1]; i++) {
            int32_t o = seq[i], l;
            for (l = w->order_offsets[o]; l < w->order_offsets[o + 1]; l++)
                picks[n++] = loc_of_sku[w->order_skus[l]];
        }
        {
            int64_t c = orc_tour_cost(w, picks, n);
            if (c < 0) return ORC_E_NOMEM;
            D += c;
        }
    }
done:
    if (dist_exact) *dist_exact = D;
    if (dist) *dist = D > INT32_MAX ? INT32_MAX : (int32_t)D;
    if (thr) *thr = orc_throughput(w, D);
    return ORC_OK;
}

static int orc_check_instance(const orc_instance *w)
{
    int32_t o, l;
    if (w->n_aisles < 1 || w->slots_per_side < 1 || w->pitch_dm < 2 || (w->pitch_dm & 1) ||
        w->spacing_dm < 0 || w->capacity < 1 || w->n_orders < 1 || w->n_orders > 65535 ||
        w->routing < ORC_ROUTE_SSHAPE || w->routing > ORC_ROUTE_COMBINED ||
        w->batching < ORC_BATCH_NEXT_FIT || w->batching > ORC_BATCH_SEED)
        return ORC_E_INVAL;
    if (w->order_offsets[0] != 0) return ORC_E_INVAL;
    for (o = 0; o < w->n_orders; o++)
        if (w->order_offsets[o + 1] <= w->order_offsets[o]) return ORC_E_INVAL;
    for (l = 0; l < w->order_offsets[w->n_orders]; l++)
        if (w->order_skus[l] < 0 || w->order_skus[l] >= w->n_skus) return ORC_E_INVAL;
    return ORC_OK;
}

static int32_t orc_max_order_lines(const orc_instance *w)
{
    int32_t o, m = 0;
    for (o = 0; o < w->n_orders; o++) {
        int32_t n = w->order_offsets[o + 1] - w->order_offsets[o];
        if (n > m) m = n;
    }
    return m;
}

int orc_eval_plan(const orc_instance *w, const uint8_t *zone_of, const uint16_t *seq,
                  int64_t *dist_exact, int32_t *dist, float *thr)
{
    int32_t *loc, *tf, *picks;
    int rc = orc_check_instance(w);
    if (rc) return rc;
    loc = (int32_t *)malloc(sizeof(int32_t) * (size_t)w->n_skus);
    tf = (int32_t *)malloc(sizeof(int32_t) * ((size_t)w->n_orders + 1));
    /* a tour holds at most max(capacity, largest order) lines */
    picks = (int32_t *)malloc(sizeof(int32_t) *
                              (size_t)(w->capacity + orc_max_order_lines(w) + 1));
    if (!loc || !tf || !picks) rc = ORC_E_NOMEM;
    else rc = orc_eval_plan_ws(w, zone_of, seq, loc, tf, picks, dist_exact, dist, thr);
    free(loc); free(tf); free(picks);
    return rc;
}

/* ------------------------------------------------------------------ */
/* many plans, optionally on several host threads (baseline timing)    */
/* ------------------------------------------------------------------ */

typedef struct {
    const orc_instance *w;
    const uint8_t *zone_of;     /* [n_plans][64] */
    const uint16_t *seq;        /* [n_plans][n_orders] */
    int32_t *dist;
    float *thr;
    int64_t n_plans;
    int64_t next;               /* shared counter */
    pthread_mutex_t mu;
    int rc;
} orc_job;

static void *orc_worker(void *arg)
{
    orc_job *j = (orc_job *)arg;
    const orc_instance *w = j->w;
    int32_t *loc = (int32_t *)malloc(sizeof(int32_t) * (size_t)w->n_skus);
    int32_t *tf = (int32_t *)malloc(sizeof(int32_t) * ((size_t)w->n_orders + 1));
    int32_t *picks = (int32_t *)malloc(sizeof(int32_t) *
                                       (size_t)(w->capacity + orc_max_order_lines(w) + 1));
    if (!loc || !tf || !picks) {
        pthread_mutex_lock(&j->mu); j->rc = ORC_E_NOMEM; pthread_mutex_unlock(&j->mu);
    } else {
        for (;;) {
            int64_t p;
            int rc;
            pthread_mutex_lock(&j->mu);
            p = j->next++;
            pthread_mutex_unlock(&j->mu);
            if (p >= j->n_plans) break;
            rc = orc_eval_plan_ws(w, j->zone_of + 64 * p, j->seq + (size_t)w->n_orders * p,
                                  loc, tf, picks, NULL, j->dist ? j->dist + p : NULL,
                                  j->thr ? j->thr + p : NULL);
            if (rc) { pthread_mutex_lock(&j->mu); j->rc = rc; pthread_mutex_unlock(&j->mu); }
        }
    }
    free(loc); free(tf); free(picks);
    return NULL;
}

int orc_eval_plans(const orc_instance *w, int64_t n_plans, const uint8_t *zone_of,
                   const uint16_t *seq, int32_t *dist, float *thr, int n_threads)
{
    orc_job job;
    pthread_t *th;
    int t, rc = orc_check_instance(w);
    if (rc) return rc;
    if (n_threads < 1) n_threads = 1;
    memset(&job, 0, sizeof job);
    job.w = w; job.zone_of = zone_of; job.seq = seq; job.dist = dist; job.thr = thr;
    job.n_plans = n_plans;
    pthread_mutex_init(&job.mu, NULL);
    th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    if (!th) return ORC_E_NOMEM;
    for (t = 0; t < n_threads; t++) pthread_create(&th[t], NULL, orc_worker, &job);
    for (t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&job.mu);
    return job.rc;
}

/* Scalar integer throughput of one core, for the CPU side of the roofline
 * that the benchmark reports beside the oracle's timing (not part of the
 * method): eight independent chains of one add and one exclusive or per
 * step.  Returns the operations performed; the chains' combination goes to
 * *sink so that nothing is folded away. */
int64_t orc_int_ops(int64_t steps, uint32_t seed, uint32_t *sink)
{
    uint32_t a0 = seed, a1 = seed ^ 1u, a2 = seed ^ 2u, a3 = seed ^ 3u;
    uint32_t a4 = seed ^ 4u, a5 = seed ^ 5u, a6 = seed ^ 6u, a7 = seed ^ 7u;
    const uint32_t c = seed | 1u, d = seed * 2654435761u;
    for (int64_t i = 0; i < steps; i++) {
        a0 = (a0 + c) ^ d;
        a1 = (a1 + c) ^ d;
        a2 = (a2 + c) ^ d;
        a3 = (a3 + c) ^ d;
        a4 = (a4 + c) ^ d;
        a5 = (a5 + c) ^ d;
        a6 = (a6 + c) ^ d;
        a7 = (a7 + c) ^ d;
    }
    *sink = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
    return steps * 16;
}
