// Host side of the C ABI declared in include/wo.h: argument checks, instance
// packing, device memory, launches.  Never throws across the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "wo_common.h"
#include "wo_internal.h"

using namespace wo;

// ----------------------------------------------------------------------------
// errors
// ----------------------------------------------------------------------------

static thread_local std::string g_err;

wo_status wo_fail(wo_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define fail wo_fail
#define HIP_TRY WO_HIP

extern "C" const char *wo_status_str(wo_status s)
{
    switch (s) {
    case WO_OK: return "WO_OK";
    case WO_E_INVAL: return "WO_E_INVAL";
    case WO_E_RANGE: return "WO_E_RANGE";
    case WO_E_NOMEM: return "WO_E_NOMEM";
    case WO_E_DEVICE: return "WO_E_DEVICE";
    case WO_E_STATE: return "WO_E_STATE";
    case WO_E_UNSUPPORTED: return "WO_E_UNSUPPORTED";
    }
    return "WO_E_UNKNOWN";
}

extern "C" const char *wo_last_error(void) { return g_err.c_str(); }

static bool env_flag(const char *name, const char *value)
{
    const char *v = getenv(name);
    return v && strcmp(v, value) == 0;
}

bool wo_fault_injected() { return env_flag("WO_FAULT_INJECT", "alloc"); }

static wo_status dev_alloc(void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(WO_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return WO_OK;
}

// ----------------------------------------------------------------------------
// handle
// ----------------------------------------------------------------------------

struct wo_wh {
    int32_t n_inst = 0;
    int device = 0;
    std::vector<InstDev> inst;          // host copies
    std::vector<uint32_t> lds;          // LDS bytes per instance
    uint32_t lds_max = 0;
    int cu_count = 0;
    void *d_pool = nullptr;             // line records | order sizes
    const uint2 *d_lines = nullptr;
    const uint8_t *d_cnt = nullptr;
    InstDev *d_inst = nullptr;
    int64_t *d_map = nullptr;           // plan_begin [n+1] | seq_base [n]
    int32_t *d_err = nullptr;
    std::vector<int64_t> map_cached;    // what d_map holds
    std::atomic<int> busy{0};
};

namespace {
struct Busy {
    std::atomic<int> *f;
    bool ok;
    explicit Busy(std::atomic<int> *flag) : f(flag)
    {
        int z = 0;
        ok = f->compare_exchange_strong(z, 1);
    }
    ~Busy()
    {
        if (ok) f->store(0);
    }
};
}  // namespace

// Choose ls = l << shift and magic with aisle(l) = mulhi_u24(ls, magic) for
// every location l < n_loc.  With magic = ceil(2^32 / (d << shift)) the error
// term is e = magic * (d << shift) - 2^32 < (d << shift), and the quotient is
// exact when (max ls) * e < 2^32 (standard multiply-by-reciprocal bound).
static bool pick_division(uint32_t d, uint32_t n_loc, uint32_t *shift, uint32_t *magic)
{
    for (uint32_t s = 0; s < 12; s++) {
        uint64_t ds = (uint64_t)d << s;
        uint64_t max_ls = (uint64_t)(n_loc - 1) << s;
        if (max_ls >= (1ull << 24)) break;
        uint64_t m = ((1ull << 32) + ds - 1) / ds;
        if (m >= (1ull << 24)) continue;
        uint64_t e = m * ds - (1ull << 32);
        if (max_ls * e >= (1ull << 32)) continue;
        *shift = s;
        *magic = (uint32_t)m;
        return true;
    }
    return false;
}

static wo_status check_desc(const wo_instance_desc &d, int idx)
{
    if (d.n_aisles < 1 || d.slots_per_side < 1)
        return fail(WO_E_INVAL, "instance %d: n_aisles and slots_per_side must be >= 1", idx);
    if (d.pitch_dm < 2 || (d.pitch_dm & 1))
        return fail(WO_E_INVAL, "instance %d: slot pitch must be even and >= 2 (got %d)", idx, d.pitch_dm);
    if (d.spacing_dm < 0) return fail(WO_E_INVAL, "instance %d: negative aisle spacing", idx);
    if (d.capacity < 1) return fail(WO_E_INVAL, "instance %d: capacity must be >= 1", idx);
    if (d.capacity > WO_MAX_CAPACITY)
        return fail(WO_E_RANGE, "instance %d: capacity %d > %d", idx, d.capacity, WO_MAX_CAPACITY);
    if (d.n_categories < 1) return fail(WO_E_INVAL, "instance %d: need >= 1 category", idx);
    if (d.n_categories > WO_MAX_CATEGORIES)
        return fail(WO_E_RANGE, "instance %d: %d categories > %d", idx, d.n_categories, WO_MAX_CATEGORIES);
    int64_t n_loc = 2ll * d.n_aisles * d.slots_per_side;
    if (n_loc > WO_MAX_LOCATIONS)
        return fail(WO_E_RANGE, "instance %d: %lld locations > %d", idx, (long long)n_loc, WO_MAX_LOCATIONS);
    if (d.n_orders < 1) return fail(WO_E_INVAL, "instance %d: need >= 1 order", idx);
    if (d.n_orders > WO_MAX_ORDERS)
        return fail(WO_E_RANGE, "instance %d: %d orders > %d", idx, d.n_orders, WO_MAX_ORDERS);
    if (d.n_skus < d.n_categories) return fail(WO_E_INVAL, "instance %d: fewer SKUs than categories", idx);
    if (d.n_skus > n_loc)
        return fail(WO_E_RANGE, "instance %d: %d SKUs do not fit %lld locations", idx, d.n_skus, (long long)n_loc);
    if (!d.sku_category || !d.order_offsets || !d.order_skus)
        return fail(WO_E_INVAL, "instance %d: NULL array", idx);
    if (!(d.walk_dm_per_s > 0) || !(d.seconds_per_item >= 0) || !(d.window_s > 0))
        return fail(WO_E_INVAL, "instance %d: walk speed and window must be > 0, item time >= 0", idx);
    std::vector<int32_t> size(d.n_categories, 0);
    for (int32_t s = 0; s < d.n_skus; s++) {
        int32_t c = d.sku_category[s];
        if (c < 0 || c >= d.n_categories)
            return fail(WO_E_INVAL, "instance %d: SKU %d has category %d out of range", idx, s, c);
        size[c]++;
    }
    for (int32_t c = 0; c < d.n_categories; c++)
        if (size[c] == 0) return fail(WO_E_INVAL, "instance %d: category %d is empty", idx, c);
    if (d.order_offsets[0] != 0) return fail(WO_E_INVAL, "instance %d: order_offsets[0] != 0", idx);
    for (int32_t o = 0; o < d.n_orders; o++)
        if (d.order_offsets[o + 1] <= d.order_offsets[o])
            return fail(WO_E_INVAL, "instance %d: order %d has no line", idx, o);
    int64_t lines = d.order_offsets[d.n_orders];
    if (lines > WO_MAX_LINES)
        return fail(WO_E_RANGE, "instance %d: %lld lines > %d", idx, (long long)lines, WO_MAX_LINES);
    for (int64_t l = 0; l < lines; l++)
        if (d.order_skus[l] < 0 || d.order_skus[l] >= d.n_skus)
            return fail(WO_E_INVAL, "instance %d: line %lld names SKU %d out of range", idx, (long long)l,
                        d.order_skus[l]);
    return WO_OK;
}

extern "C" wo_status wo_load_warehouse(const wo_instance_desc *descs, int32_t n_instances, void *stream,
                                       wo_wh **out)
{
    if (!out) return fail(WO_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!descs) return fail(WO_E_INVAL, "descs is NULL");
    if (n_instances < 1) return fail(WO_E_INVAL, "n_instances must be >= 1");
    for (int32_t i = 0; i < n_instances; i++) {
        wo_status s = check_desc(descs[i], i);
        if (s) return s;
    }

    // allocation fault injection for tests (WO_FAULT_INJECT=alloc); it fires
    // before any HIP call so that it also runs on a host without a GPU
    if (wo_fault_injected()) return fail(WO_E_NOMEM, "injected allocation failure");
    wo_wh *wh = new (std::nothrow) wo_wh;
    if (!wh) return fail(WO_E_NOMEM, "host allocation failed");
    std::unique_ptr<wo_wh, wo_status (*)(wo_wh *)> guard(wh, wo_free_warehouse);
    HIP_TRY(hipGetDevice(&wh->device));
    int lds_max = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, wh->device));
    HIP_TRY(hipDeviceGetAttribute(&wh->cu_count, hipDeviceAttributeMultiprocessorCount, wh->device));
    wh->lds_max = (uint32_t)std::min(lds_max, 160 * 1024);
    wh->n_inst = n_instances;
    wh->inst.resize(n_instances);
    wh->lds.resize(n_instances);

    // pooled host arrays
    std::vector<uint2> lines;
    std::vector<uint8_t> cnt;
    for (int32_t i = 0; i < n_instances; i++) {
        const wo_instance_desc &d = descs[i];
        InstDev &I = wh->inst[i];
        memset(&I, 0, sizeof I);
        uint32_t per_aisle = 2u * (uint32_t)d.slots_per_side;
        uint32_t n_loc = per_aisle * (uint32_t)d.n_aisles;
        if (!pick_division(per_aisle, n_loc, &I.shift, &I.magic))
            return fail(WO_E_UNSUPPORTED, "instance %d: no 24-bit reciprocal for %u locations per aisle", i,
                        per_aisle);
        I.n_aisles = d.n_aisles;
        I.words = (d.n_aisles + 31) / 32;
        I.capacity = d.capacity;
        I.n_cat = d.n_categories;
        I.n_orders = d.n_orders;
        I.n_lines = d.order_offsets[d.n_orders];
        I.d_s = per_aisle << I.shift;
        I.pitch = d.pitch_dm;
        I.spacing = d.spacing_dm;
        I.L = d.slots_per_side * d.pitch_dm;
        I.walk = d.walk_dm_per_s;
        I.t_item = d.seconds_per_item;
        I.window = d.window_s;

        // rank of each SKU inside its category, ascending SKU id
        std::vector<int32_t> rank(d.n_skus), next(d.n_categories, 0);
        for (int32_t c = 0; c < d.n_categories; c++) I.cat_size[c] = 0;
        for (int32_t s = 0; s < d.n_skus; s++) {
            int32_t c = d.sku_category[s];
            rank[s] = next[c]++;
            I.cat_size[c]++;
        }

        I.line_off = (int64_t)lines.size();
        I.cnt_off = (int64_t)cnt.size();
        int64_t units = 0;
        for (int32_t o = 0; o < d.n_orders; o++) {
            for (int32_t l = d.order_offsets[o]; l < d.order_offsets[o + 1]; l++) {
                int32_t s = d.order_skus[l];
                uint32_t c = (uint32_t)d.sku_category[s];
                lines.push_back(make_uint2(((uint32_t)rank[s] << I.shift) | ((4u * c) << 24), (uint32_t)o));
            }
            // an order larger than the capacity is a tour of its own whatever
            // its size, so sizes are clamped to capacity + 1 for the tour cut
            int32_t sz = d.order_offsets[o + 1] - d.order_offsets[o];
            int32_t u = std::min(sz, d.capacity + 1);
            cnt.push_back((uint8_t)u);
            units += u;
        }
        while (cnt.size() % 16) cnt.push_back(0);
        I.n_units = (int32_t)units;

        // Parallel next-fit: about (Q / mean order size) order starts fall in
        // a Q-item window, each a candidate entry of a segment; take as many
        // segments as the chase lanes allow, no shorter than 2Q items, and long
        // enough that a chain rarely needs more than the record slots.
        const double items = (double)I.n_lines;
        const double avg_len = items / d.n_orders;
        const double cand = std::max(1.0, std::min((double)d.capacity, d.capacity / avg_len));
        const double tour_items = std::max(1.0, d.capacity - 0.5 * (avg_len - 1.0));
        int g_lanes = 1 + (int)((0.7 * CHASE_LANES - 1.0) / cand);
        int g_len = (int)(items / (2.0 * d.capacity));
        int g = std::min(std::min(g_lanes, g_len), MAX_SEG);
        int g_recs = (int)std::ceil(items / (0.6 * CHASE_RECS * tour_items));
        bool short_segs = (double)I.n_units / std::max(g, 1) < 65535.0;  // chase records are 16-bit offsets
        I.n_seg = (g >= 2 && g >= g_recs && short_segs) ? g : 1;

        // tours per LDS tile: the expected tour count with margin (more tours
        // take another pass over the lines), never more than the orders
        int64_t t_cap = (int64_t)std::ceil(1.1 * items / tour_items) + 32;
        t_cap = std::min<int64_t>(t_cap, d.n_orders);
        t_cap = std::max<int64_t>(t_cap, 1);
        EvalLayout ly = eval_layout(d.n_orders, I.n_units, I.words, (int32_t)t_cap);
        while (ly.total > wh->lds_max && t_cap > 1) {
            t_cap = t_cap / 2;
            ly = eval_layout(d.n_orders, I.n_units, I.words, (int32_t)t_cap);
        }
        I.t_cap = (int32_t)t_cap;
        if (ly.total > wh->lds_max)
            return fail(WO_E_RANGE, "instance %d: needs %u bytes of LDS, device has %u", i, ly.total, wh->lds_max);
        wh->lds[i] = ly.total;
    }

    size_t b_lines = lines.size() * sizeof(uint2), b_cnt = cnt.size();
    size_t o_cnt = (b_lines + 255) & ~size_t(255);
    size_t bytes = o_cnt + b_cnt;
    wo_status st;
    if ((st = dev_alloc(&wh->d_pool, bytes))) return st;
    if ((st = dev_alloc((void **)&wh->d_inst, sizeof(InstDev) * n_instances))) return st;
    if ((st = dev_alloc((void **)&wh->d_map, sizeof(int64_t) * (2 * n_instances + 1)))) return st;
    if ((st = dev_alloc((void **)&wh->d_err, 64))) return st;
    wh->d_lines = (const uint2 *)wh->d_pool;
    wh->d_cnt = (const uint8_t *)wh->d_pool + o_cnt;
    hipStream_t s = (hipStream_t)stream;
    if (b_lines) HIP_TRY(hipMemcpyAsync(wh->d_pool, lines.data(), b_lines, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync((char *)wh->d_pool + o_cnt, cnt.data(), b_cnt, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(wh->d_inst, wh->inst.data(), sizeof(InstDev) * n_instances, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(wh->d_err, 0, 64, s));
    HIP_TRY(hipStreamSynchronize(s));
    wh->lds_max = *std::max_element(wh->lds.begin(), wh->lds.end());
    guard.release();
    *out = wh;
    return WO_OK;
}

extern "C" wo_status wo_free_warehouse(wo_wh *wh)
{
    if (!wh) return WO_OK;
    if (wh->d_pool || wh->d_inst || wh->d_map || wh->d_err) (void)hipDeviceSynchronize();
    if (wh->d_pool) (void)hipFree(wh->d_pool);
    if (wh->d_inst) (void)hipFree(wh->d_inst);
    if (wh->d_map) (void)hipFree(wh->d_map);
    if (wh->d_err) (void)hipFree(wh->d_err);
    delete wh;
    return WO_OK;
}

extern "C" wo_status wo_instance_info(const wo_wh *wh, int32_t i, int32_t *n_orders, int32_t *n_items,
                                      int32_t *n_categories)
{
    if (!wh) return fail(WO_E_INVAL, "handle is NULL");
    if (i < 0 || i >= wh->n_inst) return fail(WO_E_RANGE, "instance %d out of range", i);
    if (n_orders) *n_orders = wh->inst[i].n_orders;
    if (n_items) *n_items = wh->inst[i].n_lines;
    if (n_categories) *n_categories = wh->inst[i].n_cat;
    return WO_OK;
}

extern "C" wo_status wo_eval_plans(wo_wh *wh, const int64_t *plan_offsets, int64_t n_plans,
                                   const uint8_t *d_zone_of, const uint16_t *d_order_seq, int32_t *d_dist,
                                   float *d_orders_per_window, void *stream)
{
    if (!wh) return fail(WO_E_INVAL, "handle is NULL");
    Busy busy(&wh->busy);
    if (!busy.ok) return fail(WO_E_STATE, "handle is in use by another thread");
    if (n_plans < 0) return fail(WO_E_INVAL, "n_plans < 0");
    if (!plan_offsets && wh->n_inst != 1)
        return fail(WO_E_INVAL, "plan_offsets is required for a handle with %d instances", wh->n_inst);
    std::vector<int64_t> map(2 * wh->n_inst + 1);
    if (plan_offsets) {
        if (plan_offsets[0] != 0 || plan_offsets[wh->n_inst] != n_plans)
            return fail(WO_E_INVAL, "plan_offsets must start at 0 and end at n_plans");
        for (int32_t i = 0; i < wh->n_inst; i++)
            if (plan_offsets[i + 1] < plan_offsets[i]) return fail(WO_E_INVAL, "plan_offsets must not decrease");
        for (int32_t i = 0; i <= wh->n_inst; i++) map[i] = plan_offsets[i];
    } else {
        map[0] = 0;
        map[1] = n_plans;
    }
    int64_t base = 0;
    for (int32_t i = 0; i < wh->n_inst; i++) {
        map[wh->n_inst + 1 + i] = base;
        base += (map[i + 1] - map[i]) * (int64_t)wh->inst[i].n_orders;
    }
    if (n_plans == 0) return WO_OK;
    if (!d_zone_of || !d_order_seq || !d_dist) return fail(WO_E_INVAL, "NULL device buffer");
    hipStream_t s = (hipStream_t)stream;
    if (map != wh->map_cached) {
        HIP_TRY(hipMemcpyAsync(wh->d_map, map.data(), sizeof(int64_t) * map.size(), hipMemcpyHostToDevice, s));
        wh->map_cached = map;
    }
    const bool validate = env_flag("WO_VALIDATE", "1");
    if (validate) HIP_TRY(hipMemsetAsync(wh->d_err, 0, 4, s));

    EvalArgs a;
    a.inst = wh->d_inst;
    a.n_inst = wh->n_inst;
    a.n_plans = n_plans;
    a.plan_begin = wh->d_map;
    a.seq_base = wh->d_map + wh->n_inst + 1;
    a.lines = wh->d_lines;
    a.cnt = wh->d_cnt;
    a.zone_of = d_zone_of;
    a.seq = d_order_seq;
    a.dist = d_dist;
    a.thr = d_orders_per_window;
    a.err = wh->d_err;
    a.validate = validate ? 1 : 0;
    int per_cu = std::max(1, (int)((160u * 1024u) / std::max(1u, wh->lds_max)));
    int64_t grid = std::min<int64_t>(n_plans, (int64_t)wh->cu_count * per_cu);
    HIP_TRY(launch_eval(a, wh->lds_max, (int)grid, s));
    if (validate) {
        int32_t err = 0;
        HIP_TRY(hipMemcpyAsync(&err, wh->d_err, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (err) return fail(WO_E_INVAL, "a plan row is not a permutation (WO_VALIDATE=1)");
    }
    return WO_OK;
}

// Evaluate n_plans plans of one instance of the handle (rows packed with that
// instance's order count), for callers inside the library.  No argument
// checks beyond the handle's: the caller owns the buffers.
wo_status wo::eval_instance(wo_wh *wh, int32_t inst, int64_t n_plans, const uint8_t *d_zone_of,
                            const uint16_t *d_order_seq, int32_t *d_dist, float *d_thr, hipStream_t s)
{
    if (n_plans <= 0) return WO_OK;
    EvalArgs a;
    a.inst = wh->d_inst + inst;
    a.n_inst = 1;
    a.n_plans = n_plans;
    const int64_t *zero_map = (const int64_t *)((const char *)wh->d_err + 16);   // zeroed at load
    a.plan_begin = zero_map;
    a.seq_base = zero_map;
    a.lines = wh->d_lines;
    a.cnt = wh->d_cnt;
    a.zone_of = d_zone_of;
    a.seq = d_order_seq;
    a.dist = d_dist;
    a.thr = d_thr;
    a.err = wh->d_err;
    a.validate = 0;
    const uint32_t lds = wh->lds[inst];
    int per_cu = std::max(1, (int)((160u * 1024u) / std::max(1u, lds)));
    int64_t grid = std::min<int64_t>(n_plans, (int64_t)wh->cu_count * per_cu);
    HIP_TRY(launch_eval(a, lds, (int)grid, s));
    return WO_OK;
}

int32_t wo::instance_orders(const wo_wh *wh, int32_t inst) { return wh->inst[inst].n_orders; }
int32_t wo::instance_categories(const wo_wh *wh, int32_t inst) { return wh->inst[inst].n_cat; }
int32_t wo::instance_count(const wo_wh *wh) { return wh->n_inst; }
