/*
 * Runs the CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_sanitizers.py with gcc, host code only): small seeded
 * instances under every route and batching rule, the threaded and the single
 * plan evaluation (which must agree), and the route functions on edge inputs
 * (no pick, one pick, duplicates).  Exit status 0 when all agree.
 */
#include "../oracle/wo_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static uint32_t next_u32(void)
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(rng_state >> 33);
}

static uint32_t below(uint32_t m) { return (uint32_t)(((uint64_t)next_u32() * m) >> 32); }

static int check_instance(int routing, int batching, int n_aisles, int slots, int capacity, int n_orders)
{
    enum { CATS = 12 };
    const int n_skus = 2 * n_aisles * slots < 600 ? 2 * n_aisles * slots : 600;
    const int n_plans = 9;
    int32_t *cat = malloc(sizeof(int32_t) * (size_t)n_skus);
    int32_t *off = malloc(sizeof(int32_t) * (size_t)(n_orders + 1));
    int32_t *skus = malloc(sizeof(int32_t) * (size_t)n_orders * 8);
    uint8_t *zone = malloc((size_t)64 * n_plans);
    uint16_t *seq = malloc(sizeof(uint16_t) * (size_t)n_orders * n_plans);
    int32_t *d_many = malloc(sizeof(int32_t) * n_plans);
    float *t_many = malloc(sizeof(float) * n_plans);
    int i, p, rc = 0;
    orc_instance w;
    for (i = 0; i < n_skus; i++) cat[i] = i % CATS;
    off[0] = 0;
    for (i = 0; i < n_orders; i++) {
        int l, n = 1 + (int)below(capacity + 3 < 8 ? capacity + 3 : 8);
        for (l = 0; l < n; l++) skus[off[i] + l] = (int32_t)below((uint32_t)n_skus);
        off[i + 1] = off[i] + n;
    }
    for (p = 0; p < n_plans; p++) {
        uint8_t *z = zone + 64 * p;
        uint16_t *s = seq + (size_t)n_orders * p;
        memset(z, 0xFF, 64);
        for (i = 0; i < CATS; i++) z[i] = (uint8_t)i;
        for (i = CATS - 1; i > 0; i--) { int j = (int)below((uint32_t)i + 1); uint8_t x = z[i]; z[i] = z[j]; z[j] = x; }
        for (i = 0; i < n_orders; i++) s[i] = (uint16_t)i;
        for (i = n_orders - 1; i > 0; i--) { int j = (int)below((uint32_t)i + 1); uint16_t x = s[i]; s[i] = s[j]; s[j] = x; }
    }
    w.n_aisles = n_aisles; w.slots_per_side = slots; w.pitch_dm = 10; w.spacing_dm = 30; w.capacity = capacity;
    w.n_categories = CATS; w.n_skus = n_skus; w.sku_category = cat; w.n_orders = n_orders;
    w.order_offsets = off; w.order_skus = skus; w.walk_dm_per_s = 12.0; w.seconds_per_item = 10.0;
    w.window_s = 28800.0; w.routing = routing; w.batching = batching;
    if (orc_eval_plans(&w, n_plans, zone, seq, d_many, t_many, 3) != ORC_OK) rc = 1;
    for (p = 0; p < n_plans && !rc; p++) {
        int64_t de; int32_t d; float t;
        if (orc_eval_plan(&w, zone + 64 * p, seq + (size_t)n_orders * p, &de, &d, &t) != ORC_OK) rc = 2;
        else if (d != d_many[p] || t != t_many[p]) rc = 3;
    }
    free(cat); free(off); free(skus); free(zone); free(seq); free(d_many); free(t_many);
    return rc;
}

int main(void)
{
    int routing, batching, rc = 0;
    for (routing = 0; routing <= 4 && !rc; routing++)
        for (batching = 0; batching <= ORC_BATCH_SEED && !rc; batching++) {
            rc = check_instance(routing, batching, 10, 30, 5, 40);
            if (!rc) rc = check_instance(routing, batching, 1, 3, 1, 7);       /* one aisle, capacity 1 */
            if (!rc) rc = check_instance(routing, batching, 33, 2, 9, 64);     /* short aisles */
            if (rc) fprintf(stderr, "routing %d batching %d: code %d\n", routing, batching, rc);
        }
    {
        /* route functions on edge inputs */
        orc_instance w;
        int32_t cat[4] = {0, 0, 0, 0}, off[2] = {0, 1}, sk[1] = {0};
        int32_t locs[5] = {5, 5, 0, 59, 30};
        memset(&w, 0, sizeof w);
        w.n_aisles = 2; w.slots_per_side = 15; w.pitch_dm = 10; w.spacing_dm = 30; w.capacity = 5;
        w.n_categories = 1; w.n_skus = 4; w.sku_category = cat; w.n_orders = 1; w.order_offsets = off;
        w.order_skus = sk;
        if (orc_optimal_cost(&w, locs, 0) != 0 || orc_combined_cost(&w, locs, 0) != 0) rc = 4;
        if (orc_optimal_cost(&w, locs, 1) != orc_return_cost(&w, locs, 1)) rc = 5;
        if (orc_optimal_cost(&w, locs, 5) > orc_combined_cost(&w, locs, 5)) rc = 6;
        if (orc_combined_cost(&w, locs, 5) > orc_sshape_cost(&w, locs, 5)) rc = 7;
        if (rc) fprintf(stderr, "route edge inputs: code %d\n", rc);
    }
    return rc;
}
