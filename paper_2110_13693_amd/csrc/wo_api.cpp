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

extern "C" const char *wo_status_str(int32_t s)
{
    switch (s) {     // any integer: a value outside the enumeration is WO_E_UNKNOWN
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
    const uint32_t *d_grec = nullptr;
    const uint32_t *d_gbase = nullptr;
    const uint16_t *d_gord = nullptr;
    const uint32_t *d_ordoff = nullptr;
    const uint32_t *d_ordrec = nullptr;
    const uint32_t *d_big = nullptr;
    InstDev *d_inst = nullptr;
    int64_t *d_map = nullptr;           // plan_begin [n+1] | seq_base [n]
    int32_t *d_err = nullptr;
    std::vector<int64_t> map_cached;    // what d_map holds
    // launch configuration (wo_autotune_eval / wo_set_eval_config)
    int block = 256;
    int per_cu = 0;                     // 0: as many as LDS allows
    int queue = 0;                      // 1: ticket queue over the cost-ordered work list
    int main_mode = 0;                  // line pass: 0 one line per lane, 1 one order per lane, 2 sequence order
    int route = WO_ROUTE_SSHAPE;        // the route of every instance of the handle
    int batching = WO_BATCH_NEXT_FIT;   // the order batching of every instance of the handle
    std::vector<uint32_t> ff_lds;       // first fit: LDS of one plan of each instance
    uint32_t ff_lds_max = 0;
    uint16_t *d_ff_tour = nullptr;      // first fit: tour of every order, one slice per workgroup
    uint32_t *d_ff_queue = nullptr;     // first fit: open tours past the first 64, one slice per workgroup
    int64_t ff_stride = 0;              // entries per slice (largest order count + 1, rounded up)
    int ff_slots = 0;                   // slices: the most workgroups a first-fit launch may have
    int small_orders = 1024;            // instances up to this size get a launch of 64-thread workgroups
    std::string arch;                   // the device's architecture name, e.g. "gfx950"
    bool cfg_chosen = false;            // set by wo_set_eval_config, the autotuner or a cache lookup
    int cache_bucket = -1;              // plan-count bucket of the last lookup in the WO_TUNE_CACHE file
    // Work lists by launch class (0: the configured workgroups, 1: 64-thread
    // workgroups for instances of at most small_orders orders, 2: 128-thread
    // workgroups for instances of at most twice that): plan rows, most
    // expensive instances first, and the LDS the class needs.
    struct WorkClass {
        int32_t *d_work = nullptr;
        int64_t cap = 0;
        std::vector<int32_t> host;      // what d_work holds (kept alive for the async upload)
        int64_t n = 0;
        uint32_t lds = 0;
    } wc[3];
    std::vector<int64_t> wc_map;        // plan map the work lists were built for
    int wc_small = -1;                  // small_orders the work lists were built for
    int32_t *d_pinst = nullptr;         // instance of each plan row (several instances only)
    int64_t pinst_cap = 0;
    std::vector<int32_t> pinst_host;
    std::vector<int64_t> pinst_map;     // plan map d_pinst was built for
    // The device state above is shared by every call on the handle.  A call
    // on a stream other than the previous call's may rewrite it only once
    // that call has finished: the previous call's completion is recorded in
    // last_done (outside graph capture).
    hipEvent_t last_done = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_last = false;
    bool last_wrote = false;            // the previous call rewrote shared state (its uploads run in its stream)
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
    if (d.routing < WO_ROUTE_SSHAPE || d.routing > WO_ROUTE_COMBINED)
        return fail(WO_E_INVAL, "instance %d: unknown routing %d", idx, d.routing);
    if (d.batching < WO_BATCH_NEXT_FIT || d.batching > WO_BATCH_SEED)
        return fail(WO_E_INVAL, "instance %d: unknown batching %d", idx, d.batching);
    if (d.capacity > WO_MAX_CAPACITY)
        return fail(WO_E_RANGE, "instance %d: capacity %d > %d", idx, d.capacity, WO_MAX_CAPACITY);
    if (d.n_categories < 1) return fail(WO_E_INVAL, "instance %d: need >= 1 category", idx);
    if (d.n_categories > WO_MAX_CATEGORIES)
        return fail(WO_E_RANGE, "instance %d: %d categories > %d", idx, d.n_categories, WO_MAX_CATEGORIES);
    int64_t n_loc = 2ll * d.n_aisles * d.slots_per_side;
    if (n_loc > WO_MAX_LOCATIONS)
        return fail(WO_E_RANGE, "instance %d: %lld locations > %d", idx, (long long)n_loc, WO_MAX_LOCATIONS);
    if (d.routing == WO_ROUTE_OPTIMAL) {
        // every class cost of the optimal route's programme, plus its
        // unreachable marker 2^30, must fit a signed 32-bit integer
        const int64_t L = (int64_t)d.slots_per_side * d.pitch_dm;
        const int64_t bound = 4ll * d.spacing_dm * (d.n_aisles + 2) + 4ll * L * (d.n_aisles + 1);
        if (bound >= (1ll << 30))
            return fail(WO_E_RANGE, "instance %d: warehouse too large for the optimal route's 32-bit "
                        "distances (%lld dm)", idx, (long long)bound);
    }
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
        if (descs[i].routing != descs[0].routing)
            return fail(WO_E_UNSUPPORTED, "instance %d: routing differs from instance 0's (one route per load)", i);
        if (descs[i].batching != descs[0].batching)
            return fail(WO_E_UNSUPPORTED, "instance %d: batching differs from instance 0's (one rule per load)", i);
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
    {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, wh->device));
        wh->arch = prop.gcnArchName;
        wh->arch = wh->arch.substr(0, wh->arch.find(':'));   // "gfx950:sramecc+:xnack-" -> "gfx950"
    }
    wh->lds_max = (uint32_t)std::min(lds_max, 160 * 1024) - 256;   // room for the kernels' static LDS
    wh->n_inst = n_instances;
    wh->route = descs[0].routing;
    wh->batching = descs[0].batching;
    wh->inst.resize(n_instances);
    wh->lds.resize(n_instances);
    wh->ff_lds.resize(n_instances);

    // pooled host arrays
    std::vector<uint2> lines;
    std::vector<uint8_t> cnt;
    std::vector<uint32_t> grec, gbase;
    std::vector<uint16_t> gord;
    std::vector<uint32_t> ordoff, ordrec;   // each order's line records
    std::vector<uint32_t> big;              // pick rows: the orders routed apart
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
        {
            // zones fill locations [0, n_skus), so only the aisles up to the
            // one holding location n_skus - 1 can be visited
            const int32_t used = (int32_t)(((uint32_t)std::max(d.n_skus, 1) - 1u) / per_aisle + 1u);
            I.words = (std::min(used, d.n_aisles) + 31) / 32;
        }
        I.route = d.routing;
        {
            // a tour holds at most max(capacity, largest order) lines; with
            // pick rows, the orders of more than MAX_PICK_SLOTS lines (each a
            // tour of its own, as the capacity is at most MAX_PICK_SLOTS) are
            // listed and routed apart, and the rows keep the others
            int32_t max_lines = 0, max_big = 0;
            I.big_off = (int64_t)big.size();
            I.n_big = 0;
            for (int32_t o = 0; o < d.n_orders; o++) {
                const int32_t len = d.order_offsets[o + 1] - d.order_offsets[o];
                if (d.routing != WO_ROUTE_SSHAPE && len > MAX_PICK_SLOTS) {
                    if (len > MAX_BIG_ORDER_LINES)
                        return fail(WO_E_UNSUPPORTED, "instance %d: order %d has %d lines; the routes other than "
                                    "S-shape take orders of at most %d", i, o, len, MAX_BIG_ORDER_LINES);
                    big.push_back((uint32_t)o);
                    I.n_big++;
                    max_big = std::max(max_big, len);
                } else {
                    max_lines = std::max(max_lines, len);
                }
            }
            I.big_np2 = 0;
            if (max_big) {
                I.big_np2 = 1;
                while (I.big_np2 < max_big) I.big_np2 <<= 1;
            }
            I.pick_slots = std::max(d.capacity, max_lines);
            I.row_b = (int32_t)(d.routing == WO_ROUTE_SSHAPE ? row_bytes(I.words) : pick_row_bytes(I.pick_slots));
        }
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

        // order sizes clamped to capacity + 1: an order larger than the
        // capacity is a tour of its own whatever its size
        I.cnt_off = (int64_t)cnt.size();
        int64_t units = 0;
        for (int32_t o = 0; o < d.n_orders; o++) {
            const int32_t u = std::min(d.order_offsets[o + 1] - d.order_offsets[o], d.capacity + 1);
            cnt.push_back((uint8_t)u);
            units += u;
        }
        // zeros for the dummy entry n and the sink entry n + 1, then padding
        while (cnt.size() < (size_t)I.cnt_off + cnt_bytes(d.n_orders)) cnt.push_back(0);
        I.n_units = (int32_t)units;
        I.min_size = d.capacity + 1;
        for (int32_t o = 0; o < d.n_orders; o++) I.min_size = std::min<int32_t>(I.min_size, cnt[(size_t)I.cnt_off + o]);
        I.n_skus = d.n_skus;
        // tours of next-fit over the orders in instance order: the orders are
        // exchangeable, so this is the tour count of a typical plan, whatever
        // the spread of order sizes
        int64_t tours_est = 0;
        {
            int64_t load = 0;
            for (int32_t o = 0; o < d.n_orders; o++) {
                const int64_t u = cnt[(size_t)I.cnt_off + o];
                if (tours_est == 0 || load + u > d.capacity) {
                    tours_est++;
                    load = u;
                } else {
                    load += u;
                }
            }
        }

        // groups of 64 orders by descending size, lines stored line-major
        {
            std::vector<int32_t> ord(d.n_orders);
            for (int32_t o = 0; o < d.n_orders; o++) ord[o] = o;
            auto len = [&](int32_t o) { return d.order_offsets[o + 1] - d.order_offsets[o]; };
            std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return len(x) > len(y); });
            I.n_grp = (d.n_orders + 63) / 64;
            I.grec_off = (int64_t)grec.size();
            I.gbase_off = (int64_t)gbase.size();
            I.gord_off = (int64_t)gord.size();
            uint32_t off = 0;
            for (int32_t g = 0; g < I.n_grp; g++) {
                gbase.push_back(off);
                const int32_t L = len(ord[64 * g]);
                for (int32_t k = 0; k < L; k++) {
                    for (int32_t j = 0; j < 64; j++) {
                        const int32_t q = 64 * g + j;
                        uint32_t r = 0;
                        if (q < d.n_orders) {
                            const int32_t o = ord[q];
                            const int32_t l = d.order_offsets[o] + (k < len(o) ? k : 0);
                            const int32_t sk = d.order_skus[l];
                            r = ((uint32_t)rank[sk] << I.shift) | ((4u * (uint32_t)d.sku_category[sk]) << 24);
                        }
                        grec.push_back(r);
                    }
                }
                off += (uint32_t)(64 * L);
                for (int32_t j = 0; j < 64; j++) {
                    const int32_t q = 64 * g + j;
                    gord.push_back(q < d.n_orders ? (uint16_t)ord[q] : (uint16_t)0xFFFF);
                }
            }
            gbase.push_back(off);
        }

        // Parallel next-fit: about (Q / mean order size) order starts fall in
        // a Q-unit window, each a candidate entry of a segment.  With 2^lg
        // opening records per chain, take the fewest segments whose chains
        // fit the estimated tours with margin, plus one; fewer if the chase
        // lanes or a minimum length of 2Q units do not allow them.  Longer
        // records are tried only when 32 do not fit; without any fit, plans
        // take the serial chain.
        const double avg_len = (double)units / d.n_orders;
        const double cand = std::max(1.0, std::min((double)d.capacity, d.capacity / avg_len));
        I.n_seg = 1;
        I.chase_log2 = 5;
        for (int lg = 5; lg <= MAX_CHASE_LOG2; lg++) {
            const int g_recs = (int)std::ceil((double)tours_est / (0.75 * (1 << lg)));
            const int g_lanes = 1 + (int)((0.85 * CHASE_LANES - 1.0) / cand);
            const int g_len = (int)((double)units / (2.0 * d.capacity));
            const int g = std::min(std::min(g_recs + 1, g_lanes), std::min(g_len, MAX_SEG));
            const bool short_segs = (double)I.n_units / std::max(g, 1) < 65535.0;   // 16-bit records
            if (g >= 2 && g >= g_recs && short_segs) {
                I.n_seg = g;
                I.chase_log2 = lg;
                break;
            }
        }
        // room for the expected chase lanes with margin, in whole waves
        {
            const double lanes = 1.0 + (I.n_seg - 1) * cand;
            int cl = ((int)std::ceil(1.3 * lanes + 16.0) + 63) / 64 * 64;
            I.chase_lanes = std::min(CHASE_LANES, std::max(64, cl));
        }

        // tours per LDS tile: the expected tour count with margin (more tours
        // take another pass over the lines), never more than the orders, and
        // few enough that a row's byte offset fits the 16-bit tour entries
        int64_t t_cap = (int64_t)std::ceil(1.04 * (double)tours_est) + 8;
        t_cap = std::min<int64_t>(t_cap, d.n_orders);
        t_cap = std::min<int64_t>(t_cap, 65535 / I.row_b - 1);
        if (const char *cap = getenv("WO_TILE_TOURS"))
            if (atoll(cap) >= 1) t_cap = std::min<int64_t>(t_cap, atoll(cap));
        t_cap = std::max<int64_t>(t_cap, 1);
        // the region of the rows also holds the sort of the largest listed order
        const int64_t t_big = ((int64_t)4 * I.big_np2 + I.row_b - 1) / I.row_b;
        t_cap = std::max(t_cap, t_big);
        EvalLayout ly = eval_layout(d.n_orders, I.n_units, (uint32_t)I.row_b, (int32_t)t_cap, I.chase_log2, I.chase_lanes);
        while (ly.total > wh->lds_max && t_cap > 1) {
            t_cap = t_cap / 2;
            ly = eval_layout(d.n_orders, I.n_units, (uint32_t)I.row_b, (int32_t)t_cap, I.chase_log2, I.chase_lanes);
        }
        I.t_cap = (int32_t)t_cap;
        if (ly.total > wh->lds_max || t_cap < t_big)
            return fail(WO_E_RANGE, "instance %d: needs %u bytes of LDS, device has %u", i,
                        std::max(ly.total, (uint32_t)(LDS_REGION + 4 * I.big_np2)), wh->lds_max);

        // line records; y is the LDS byte offset of the order's tour entry in
        // this instance's layout.  Padding records sit on the dummy entry
        // (order n), whose row is never summed.  In instance order the lines
        // are cut into groups of LINE_PAD = 64 lanes x 8 slots: lane j of a
        // group takes 8 consecutive lines (mostly of one or two orders), and
        // the group is stored slot-major so that each slot is one coalesced
        // 512-byte load for a wave.  Lanes of one slot so hold lines of
        // different orders and their row updates rarely share an address.
        I.line_off = (int64_t)lines.size();
        {
            std::vector<uint2> flat;
            flat.reserve((size_t)I.n_lines + LINE_PAD);
            for (int32_t o = 0; o < d.n_orders; o++) {
                for (int32_t l = d.order_offsets[o]; l < d.order_offsets[o + 1]; l++) {
                    const int32_t sk = d.order_skus[l];
                    const uint32_t c = (uint32_t)d.sku_category[sk];
                    flat.push_back(make_uint2(((uint32_t)rank[sk] << I.shift) | ((4u * c) << 24),
                                              ly.tour + 2u * (uint32_t)o));
                }
            }
            while (flat.size() % LINE_PAD) flat.push_back(make_uint2(0u, ly.tour + 2u * (uint32_t)d.n_orders));
            // bit 31 of y marks the first slot of a run of one order's lines
            // in a lane (the slot that reads the tour entry)
            for (size_t g = 0; g < flat.size(); g += LINE_PAD)
                for (int u = 0; u < LINE_SLOTS; u++)
                    for (int j = 0; j < 64; j++) {
                        const size_t k = g + (size_t)j * LINE_SLOTS + u;
                        uint2 r = flat[k];
                        if (u == 0 || flat[k - 1].y != r.y) r.y |= 0x80000000u;
                        lines.push_back(r);
                    }
        }
        I.n_lines_pad = (int32_t)(lines.size() - (size_t)I.line_off);
        wh->lds[i] = ly.total;
        wh->ff_lds[i] = std::max(ff_lds_bytes(d.routing, I.row_b), ff_rows_off() + 4u * (uint32_t)I.big_np2);
        {
            // each order's line records (seed batching, and the line pass in
            // sequence order)
            I.ordoff_off = (int64_t)ordoff.size();
            I.ordrec_off = (int64_t)ordrec.size();
            for (int32_t o = 0; o <= d.n_orders; o++) ordoff.push_back((uint32_t)d.order_offsets[o]);
            for (int32_t l = 0; l < d.order_offsets[d.n_orders]; l++) {
                const int32_t sk = d.order_skus[l];
                ordrec.push_back(((uint32_t)rank[sk] << I.shift) | ((4u * (uint32_t)d.sku_category[sk]) << 24));
            }
        }
        if (d.batching == WO_BATCH_SEED) {
            int32_t max_lines = 0;
            for (int32_t o = 0; o < d.n_orders; o++)
                max_lines = std::max(max_lines, d.order_offsets[o + 1] - d.order_offsets[o]);
            if (std::min(max_lines, d.n_aisles) > SEED_MAX_AISLES)
                return fail(WO_E_UNSUPPORTED, "instance %d: seed batching takes orders of at most %d aisles (an order "
                            "has %d lines over %d aisles)", i, SEED_MAX_AISLES, max_lines, d.n_aisles);
            const uint32_t need = seed_layout(d.n_orders, d.n_aisles, d.order_offsets[d.n_orders]).total;
            if (need > wh->lds_max)
                return fail(WO_E_UNSUPPORTED, "instance %d: seed batching needs %u bytes of LDS (about 4 per order, "
                            "2 per line and 4 per aisle), the device has %u", i, need, wh->lds_max);
            wh->ff_lds[i] = std::max(wh->ff_lds[i], need);
        }
    }

    size_t b_lines = lines.size() * sizeof(uint2), b_cnt = cnt.size();
    size_t o_cnt = (b_lines + 255) & ~size_t(255);
    size_t o_grec = (o_cnt + b_cnt + 255) & ~size_t(255);
    size_t o_gbase = (o_grec + grec.size() * 4 + 255) & ~size_t(255);
    size_t o_gord = (o_gbase + gbase.size() * 4 + 255) & ~size_t(255);
    size_t o_ordoff = (o_gord + gord.size() * 2 + 255) & ~size_t(255);
    size_t o_ordrec = (o_ordoff + ordoff.size() * 4 + 255) & ~size_t(255);
    size_t o_big = (o_ordrec + ordrec.size() * 4 + 255) & ~size_t(255);
    size_t bytes = o_big + big.size() * 4;
    wo_status st;
    if ((st = dev_alloc(&wh->d_pool, bytes))) return st;
    if ((st = dev_alloc((void **)&wh->d_inst, sizeof(InstDev) * n_instances))) return st;
    if ((st = dev_alloc((void **)&wh->d_map, sizeof(int64_t) * (2 * n_instances + 1)))) return st;
    if ((st = dev_alloc((void **)&wh->d_err, 64))) return st;
    // ordering between streams of this device only: no timing, no system-scope fence
    HIP_TRY(hipEventCreateWithFlags(&wh->last_done, hipEventDisableTiming | hipEventDisableSystemFence));
    wh->d_lines = (const uint2 *)wh->d_pool;
    wh->d_cnt = (const uint8_t *)wh->d_pool + o_cnt;
    wh->d_grec = (const uint32_t *)((const char *)wh->d_pool + o_grec);
    wh->d_gbase = (const uint32_t *)((const char *)wh->d_pool + o_gbase);
    wh->d_gord = (const uint16_t *)((const char *)wh->d_pool + o_gord);
    wh->d_ordoff = (const uint32_t *)((const char *)wh->d_pool + o_ordoff);
    wh->d_ordrec = (const uint32_t *)((const char *)wh->d_pool + o_ordrec);
    wh->d_big = (const uint32_t *)((const char *)wh->d_pool + o_big);
    hipStream_t s = (hipStream_t)stream;
    if (b_lines) HIP_TRY(hipMemcpyAsync(wh->d_pool, lines.data(), b_lines, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync((char *)wh->d_pool + o_cnt, cnt.data(), b_cnt, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync((char *)wh->d_pool + o_grec, grec.data(), grec.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync((char *)wh->d_pool + o_gbase, gbase.data(), gbase.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync((char *)wh->d_pool + o_gord, gord.data(), gord.size() * 2, hipMemcpyHostToDevice, s));
    if (!ordoff.empty())
        HIP_TRY(hipMemcpyAsync((char *)wh->d_pool + o_ordoff, ordoff.data(), ordoff.size() * 4, hipMemcpyHostToDevice, s));
    if (!ordrec.empty())
        HIP_TRY(hipMemcpyAsync((char *)wh->d_pool + o_ordrec, ordrec.data(), ordrec.size() * 4, hipMemcpyHostToDevice, s));
    if (!big.empty())
        HIP_TRY(hipMemcpyAsync((char *)wh->d_pool + o_big, big.data(), big.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(wh->d_inst, wh->inst.data(), sizeof(InstDev) * n_instances, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(wh->d_err, 0, 64, s));
    HIP_TRY(hipStreamSynchronize(s));
    wh->lds_max = *std::max_element(wh->lds.begin(), wh->lds.end());
    wh->ff_lds_max = *std::max_element(wh->ff_lds.begin(), wh->ff_lds.end());
    if (wh->batching != WO_BATCH_NEXT_FIT) {
        int32_t n_max = 0;
        for (int32_t i = 0; i < n_instances; i++) n_max = std::max(n_max, descs[i].n_orders);
        wh->ff_stride = ((int64_t)n_max + 1 + 63) & ~(int64_t)63;
        wh->ff_slots = wh->cu_count *
                       eval_ff_max_blocks_per_cu(wh->route, wh->batching == WO_BATCH_SEED,
                                                 *std::min_element(wh->ff_lds.begin(), wh->ff_lds.end()));
        if ((st = dev_alloc((void **)&wh->d_ff_tour, sizeof(uint16_t) * (size_t)wh->ff_stride * wh->ff_slots)))
            return st;
        if ((st = dev_alloc((void **)&wh->d_ff_queue, sizeof(uint32_t) * (size_t)wh->ff_stride * wh->ff_slots)))
            return st;
    }
    guard.release();
    *out = wh;
    return WO_OK;
}

extern "C" wo_status wo_free_warehouse(wo_wh *wh)
{
    if (!wh) return WO_OK;
    if (wh->d_pool || wh->d_inst || wh->d_map || wh->d_err || wh->d_ff_tour || wh->d_ff_queue) (void)hipDeviceSynchronize();
    if (wh->d_pool) (void)hipFree(wh->d_pool);
    if (wh->d_inst) (void)hipFree(wh->d_inst);
    if (wh->d_map) (void)hipFree(wh->d_map);
    if (wh->d_err) (void)hipFree(wh->d_err);
    for (auto &c : wh->wc)
        if (c.d_work) (void)hipFree(c.d_work);
    if (wh->d_pinst) (void)hipFree(wh->d_pinst);
    if (wh->d_ff_tour) (void)hipFree(wh->d_ff_tour);
    if (wh->d_ff_queue) (void)hipFree(wh->d_ff_queue);
    if (wh->last_done) (void)hipEventDestroy(wh->last_done);
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

// Blocks to launch: `per_cu` workgroups per CU (or as many as the LDS allows,
// at most 32 waves per CU), never more than there are plans.
static int launch_grid(const wo_wh *wh, int block, int per_cu_cfg, uint32_t lds, int64_t n_plans)
{
    const int fit = eval_max_blocks_per_cu(block, wh->route, lds, wh->main_mode);
    const int per_cu = per_cu_cfg > 0 ? std::min(per_cu_cfg, fit) : fit;
    return (int)std::min<int64_t>(n_plans, (int64_t)wh->cu_count * per_cu);
}

static int ff_grid(const wo_wh *wh, uint32_t lds, int64_t n_plans)
{
    const int64_t fit = (int64_t)wh->cu_count * eval_ff_max_blocks_per_cu(wh->route, wh->batching == WO_BATCH_SEED, lds);
    return (int)std::min<int64_t>(n_plans, std::min<int64_t>(fit, wh->ff_slots));   // one tour table slice each
}

static int launch_grid(const wo_wh *wh, uint32_t lds, int64_t n_plans)
{
    return launch_grid(wh, wh->block, wh->per_cu, lds, n_plans);
}

// Work lists by launch class, plans of the most expensive instances first
// (longest-processing-time order; cost ~ lines + 2 * orders per plan).  With
// small_orders > 0, instances of at most that many orders form class 1 and
// those of at most twice as many class 2.
static int class_of(const wo_wh *wh, int32_t i)
{
    const int n = wh->inst[i].n_orders, s = wh->small_orders;
    if (s <= 0) return 0;
    return n <= s ? 1 : (n <= 2 * s ? 2 : 0);
}
static const int class_block[3] = {0, 64, 128};   // 0: the configured block size

static wo_status prepare_work(wo_wh *wh, const std::vector<int64_t> &map, int64_t n_plans, hipStream_t s)
{
    if (map == wh->wc_map && wh->wc_small == wh->small_orders) return WO_OK;
    if (n_plans > INT32_MAX) return fail(WO_E_RANGE, "too many plans for the work lists");
    std::vector<int32_t> order(wh->n_inst);
    for (int32_t i = 0; i < wh->n_inst; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        const int64_t cx = (int64_t)wh->inst[x].n_lines + 2ll * wh->inst[x].n_orders;
        const int64_t cy = (int64_t)wh->inst[y].n_lines + 2ll * wh->inst[y].n_orders;
        return cx > cy;
    });
    for (int c = 0; c < 3; c++) {
        wo_wh::WorkClass &w = wh->wc[c];
        w.host.clear();
        w.lds = 0;
        for (int32_t i : order) {
            if (class_of(wh, i) != c) continue;
            for (int64_t p = map[i]; p < map[i + 1]; p++) w.host.push_back((int32_t)p);
            if (map[i + 1] > map[i]) w.lds = std::max(w.lds, wh->lds[i]);
        }
        w.n = (int64_t)w.host.size();
        if (w.n == 0) continue;
        if (w.cap < w.n) {
            if (w.d_work) (void)hipFree(w.d_work);
            w.d_work = nullptr;
            w.cap = 0;
            wo_status st = dev_alloc((void **)&w.d_work, sizeof(int32_t) * (size_t)w.n);
            if (st) return st;
            w.cap = w.n;
        }
        HIP_TRY(hipMemcpyAsync(w.d_work, w.host.data(), sizeof(int32_t) * (size_t)w.n, hipMemcpyHostToDevice, s));
    }
    wh->wc_map = map;
    wh->wc_small = wh->small_orders;
    return WO_OK;
}

namespace {
int log2_bucket(int64_t x);
wo_status tune_cache_lookup(wo_wh *wh, const char *path, int64_t n_plans, bool *found, bool chosen);
}  // namespace
static wo_status check_cfg(const wo_eval_config *cfg);
static void apply_cfg(wo_wh *wh, const wo_eval_config &c, bool chosen);

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
    const bool validate = env_flag("WO_VALIDATE", "1");
    // Unless the caller chose a configuration, a call whose plan count falls
    // in another bucket than the previous call's takes its configuration from
    // the WO_TUNE_CACHE file: the matching entry, else the defaults (also for
    // a file that cannot be read).
    if (!wh->cfg_chosen) {
        const char *cache = getenv("WO_TUNE_CACHE");
        const int b = log2_bucket(n_plans);
        if (cache && *cache && b != wh->cache_bucket) {
            wh->cache_bucket = b;
            bool found = false;
            if (tune_cache_lookup(wh, cache, n_plans, &found, false) != WO_OK || !found)
                apply_cfg(wh, wo_eval_config{256, 0, 0, 0, 1024, 0.f}, false);
        }
    }
    {
        // shared device state this call writes: the plan map and the tables
        // built from it, the queue tickets, the validation flag, the
        // first-fit tour table
        bool any_small = false;
        for (int32_t i = 0; i < wh->n_inst; i++) any_small |= class_of(wh, i) != 0 && map[i + 1] > map[i];
        const bool writes = map != wh->map_cached || (wh->n_inst > 1 && (map != wh->pinst_map || wh->pinst_cap < n_plans)) ||
                            ((any_small || wh->queue) && (map != wh->wc_map || wh->wc_small != wh->small_orders)) ||
                            wh->queue || validate || wh->batching != WO_BATCH_NEXT_FIT;
        // A call on another stream while the previous call may still run:
        // refused when it would rewrite state the previous call reads, or
        // read state whose upload the previous call enqueued on its own
        // stream; when both only read, it is ordered after the previous call
        // so that one event keeps marking the completion of every earlier
        // call.
        // (Under graph capture nothing here runs: an event query would
        // invalidate the capture, and a captured call runs only when its
        // graph is replayed, which the caller orders.)
        hipStreamCaptureStatus cap0 = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(s, &cap0));
        if (cap0 == hipStreamCaptureStatusNone && wh->has_last && s != wh->last_stream) {
            const hipError_t q = hipEventQuery(wh->last_done);
            if (q == hipErrorNotReady) {
                if (writes || wh->last_wrote)
                    return fail(WO_E_STATE, "the handle's previous call, on another stream, may still be running "
                                "and one of the two calls rewrites state the other reads; order the two streams "
                                "or use one stream");
                HIP_TRY(hipStreamWaitEvent(s, wh->last_done, 0));
            } else {
                (void)hipGetLastError();
            }
        }
        wh->last_wrote = writes;
    }
    if (map != wh->map_cached) {
        wh->map_cached = map;
        HIP_TRY(hipMemcpyAsync(wh->d_map, wh->map_cached.data(), sizeof(int64_t) * map.size(),
                               hipMemcpyHostToDevice, s));
    }
    // instance of every plan row, so that the kernel needs no search
    if (wh->n_inst > 1 && (map != wh->pinst_map || wh->pinst_cap < n_plans)) {
        if (n_plans > INT32_MAX) return fail(WO_E_RANGE, "too many plans");
        if (wh->pinst_cap < n_plans) {
            if (wh->d_pinst) (void)hipFree(wh->d_pinst);
            wh->d_pinst = nullptr;
            wh->pinst_cap = 0;
            wo_status st = dev_alloc((void **)&wh->d_pinst, sizeof(int32_t) * (size_t)n_plans);
            if (st) return st;
            wh->pinst_cap = n_plans;
        }
        wh->pinst_host.resize((size_t)n_plans);
        for (int32_t i = 0; i < wh->n_inst; i++)
            for (int64_t p = map[i]; p < map[i + 1]; p++) wh->pinst_host[(size_t)p] = i;
        HIP_TRY(hipMemcpyAsync(wh->d_pinst, wh->pinst_host.data(), sizeof(int32_t) * (size_t)n_plans,
                               hipMemcpyHostToDevice, s));
        wh->pinst_map = map;
    }
    if (validate) HIP_TRY(hipMemsetAsync(wh->d_err, 0, 4, s));

    EvalArgs a;
    a.inst = wh->d_inst;
    a.n_inst = wh->n_inst;
    a.n_plans = n_plans;
    a.plan_begin = wh->d_map;
    a.seq_base = wh->d_map + wh->n_inst + 1;
    a.plan_inst = wh->n_inst > 1 ? wh->d_pinst : nullptr;
    a.lines = wh->d_lines;
    a.cnt = wh->d_cnt;
    a.grec = wh->d_grec;
    a.gbase = wh->d_gbase;
    a.gord = wh->d_gord;
    a.ordoff = wh->d_ordoff;
    a.ordrec = wh->d_ordrec;
    a.big = wh->d_big;
    a.main_mode = wh->route == WO_ROUTE_SSHAPE ? wh->main_mode : 0;   // pick rows: line per lane only
    a.zone_of = d_zone_of;
    a.seq = d_order_seq;
    a.dist = d_dist;
    a.thr = d_orders_per_window;
    a.err = wh->d_err;
    a.validate = validate ? 1 : 0;
    a.queue = 0;
    a.chunk = 1;
    a.queue_ctr = (uint32_t *)((char *)wh->d_err + 48);
    a.work = nullptr;
    a.ff_tour = wh->d_ff_tour;
    a.ff_stride = wh->ff_stride;
    a.ff_queue = wh->d_ff_queue;
    a.plan_spacing = nullptr;
    bool any_small = false;
    for (int32_t i = 0; i < wh->n_inst; i++) any_small |= class_of(wh, i) != 0 && map[i + 1] > map[i];
    if (wh->batching != WO_BATCH_NEXT_FIT) {
        // first fit has a kernel of its own, one wavefront per plan; the
        // launch configuration above applies to next fit only
        HIP_TRY(launch_eval_ff(a, wh->ff_lds_max, ff_grid(wh, wh->ff_lds_max, n_plans), wh->route,
                               wh->batching == WO_BATCH_SEED, s));
    } else if (!any_small && !wh->queue) {
        // one launch, grid stride over the plan rows
        HIP_TRY(launch_eval(a, wh->lds_max, launch_grid(wh, wh->lds_max, n_plans), wh->block, wh->route, s));
    } else {
        // one launch per class over its work list: the configured workgroups
        // for the large instances, 64- and 128-thread ones for the small ones
        wo_status st = prepare_work(wh, map, n_plans, s);
        if (st) return st;
        for (int c = 0; c < 3; c++) {
            const wo_wh::WorkClass &w = wh->wc[c];
            if (w.n == 0) continue;
            EvalArgs ac = a;
            ac.n_plans = w.n;
            ac.work = w.d_work;
            ac.queue = wh->queue;
            ac.queue_ctr = (uint32_t *)((char *)wh->d_err + 48 + 4 * c);
            const int block = c ? class_block[c] : wh->block;
            const int per_cu = c ? 0 : wh->per_cu;
            const int grid = launch_grid(wh, block, per_cu, w.lds, w.n);
            // the small instances' plans go out in chunks of consecutive
            // work items, so that a workgroup mostly keeps its instance's
            // tables (grid stride: 2 per step; queue: 4 per ticket), where
            // every workgroup has many plans (with few, chunks would leave
            // workgroups idle)
            ac.chunk = (c && w.n >= (int64_t)grid * 8) ? (wh->queue ? 4 : 2) : 1;
            HIP_TRY(launch_eval(ac, w.lds, grid, block, wh->route, s));
        }
    }
    // the completion of this call, for the next call on another stream (not
    // under graph capture: a captured call runs only when its graph does)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap));
    if (cap == hipStreamCaptureStatusNone) {
        HIP_TRY(hipEventRecord(wh->last_done, s));
        wh->last_stream = s;
        wh->has_last = true;
    }
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
                            const uint16_t *d_order_seq, int32_t *d_dist, float *d_thr, hipStream_t s,
                            const int32_t *d_plan_spacing)
{
    if (n_plans <= 0) return WO_OK;
    EvalArgs a;
    a.inst = wh->d_inst + inst;
    a.n_inst = 1;
    a.n_plans = n_plans;
    const int64_t *zero_map = (const int64_t *)((const char *)wh->d_err + 16);   // zeroed at load
    a.plan_begin = zero_map;
    a.seq_base = zero_map;
    a.plan_inst = nullptr;
    a.lines = wh->d_lines;
    a.cnt = wh->d_cnt;
    a.grec = wh->d_grec;
    a.gbase = wh->d_gbase;
    a.gord = wh->d_gord;
    a.ordoff = wh->d_ordoff;
    a.ordrec = wh->d_ordrec;
    a.big = wh->d_big;
    a.main_mode = wh->route == WO_ROUTE_SSHAPE ? wh->main_mode : 0;   // pick rows: line per lane only
    a.zone_of = d_zone_of;
    a.seq = d_order_seq;
    a.dist = d_dist;
    a.thr = d_thr;
    a.err = wh->d_err;
    a.validate = 0;
    a.queue = 0;
    a.chunk = 1;
    a.queue_ctr = nullptr;
    a.work = nullptr;
    a.ff_tour = wh->d_ff_tour;
    a.ff_stride = wh->ff_stride;
    a.ff_queue = wh->d_ff_queue;
    a.plan_spacing = d_plan_spacing;
    if (wh->batching != WO_BATCH_NEXT_FIT) {
        const uint32_t lds = wh->ff_lds[inst];
        HIP_TRY(launch_eval_ff(a, lds, ff_grid(wh, lds, n_plans), wh->route, wh->batching == WO_BATCH_SEED, s));
        return WO_OK;
    }
    const uint32_t lds = wh->lds[inst];
    HIP_TRY(launch_eval(a, lds, launch_grid(wh, lds, n_plans), wh->block, wh->route, s));
    return WO_OK;
}

int32_t wo::instance_orders(const wo_wh *wh, int32_t inst) { return wh->inst[inst].n_orders; }
const InstDev &wo::instance_dev(const wo_wh *wh, int32_t inst) { return wh->inst[inst]; }
int32_t wo::instance_categories(const wo_wh *wh, int32_t inst) { return wh->inst[inst].n_cat; }
int32_t wo::instance_count(const wo_wh *wh) { return wh->n_inst; }

static wo_status check_cfg(const wo_eval_config *cfg)
{
    if (cfg->block_threads != 64 && cfg->block_threads != 128 && cfg->block_threads != 256 &&
        cfg->block_threads != 512)
        return fail(WO_E_INVAL, "block_threads must be 64, 128, 256 or 512");
    if (cfg->blocks_per_cu < 0 || cfg->blocks_per_cu > 32) return fail(WO_E_INVAL, "blocks_per_cu in [0, 32]");
    if (cfg->queue != 0 && cfg->queue != 1) return fail(WO_E_INVAL, "queue must be 0 or 1");
    if (cfg->line_pass < 0 || cfg->line_pass > 2) return fail(WO_E_INVAL, "line_pass must be 0, 1 or 2");
    if (cfg->small_orders < 0 || cfg->small_orders > 1024) return fail(WO_E_INVAL, "small_orders in [0, 1024]");
    return WO_OK;
}

// chosen: set by the caller (wo_set_eval_config, the autotuner, an explicit
// cache lookup), after which calls no longer consult the WO_TUNE_CACHE file
static void apply_cfg(wo_wh *wh, const wo_eval_config &c, bool chosen)
{
    wh->block = c.block_threads;
    wh->per_cu = c.blocks_per_cu;
    wh->queue = c.queue;
    wh->main_mode = c.line_pass;
    wh->small_orders = c.small_orders;
    if (chosen) wh->cfg_chosen = true;
}

extern "C" wo_status wo_set_eval_config(wo_wh *wh, const wo_eval_config *cfg)
{
    if (!wh || !cfg) return fail(WO_E_INVAL, "NULL argument");
    if (wo_status st = check_cfg(cfg)) return st;
    Busy busy(&wh->busy);
    if (!busy.ok) return fail(WO_E_STATE, "handle is in use by another thread");
    apply_cfg(wh, *cfg, true);
    return WO_OK;
}

extern "C" wo_status wo_get_eval_config(const wo_wh *wh, wo_eval_config *cfg)
{
    if (!wh || !cfg) return fail(WO_E_INVAL, "NULL argument");
    cfg->block_threads = wh->block;
    cfg->blocks_per_cu = wh->per_cu;
    cfg->queue = wh->queue;
    cfg->line_pass = wh->main_mode;
    cfg->small_orders = wh->small_orders;
    cfg->ms = 0.f;
    return WO_OK;
}

// ---- persistent autotune cache ------------------------------------------
// A JSON file {"entries": [{...}, ...]}; an entry holds its key -- "arch",
// "cus", "route", "batching", and the buckets "instances", "orders", "plans"
// (ceil(log2) of the instance count, the largest order count and the plan
// count) -- and the configuration: "block_threads", "blocks_per_cu",
// "queue", "line_pass", "small_orders", "ms".
namespace {

struct TuneEntry {
    std::string arch;
    int64_t v[13];   // cus route batching instances orders plans | block per_cu queue line_pass small_orders | ms*1e6 | -
};
const char *const kTuneKeys[12] = {"cus", "route", "batching", "instances", "orders", "plans", "block_threads",
                                   "blocks_per_cu", "queue", "line_pass", "small_orders", "ms"};

int log2_bucket(int64_t x)
{
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < x) b++;
    return b;
}

void tune_key(const wo_wh *wh, int64_t n_plans, TuneEntry *e)
{
    int32_t n_max = 0;
    for (const InstDev &I : wh->inst) n_max = std::max(n_max, I.n_orders);
    e->arch = wh->arch;
    e->v[0] = wh->cu_count;
    e->v[1] = wh->route;
    e->v[2] = wh->batching;
    e->v[3] = log2_bucket(wh->n_inst);
    e->v[4] = log2_bucket(n_max);
    e->v[5] = log2_bucket(n_plans);
}

bool same_key(const TuneEntry &a, const TuneEntry &b)
{
    if (a.arch != b.arch) return false;
    for (int k = 0; k < 6; k++)
        if (a.v[k] != b.v[k]) return false;
    return true;
}

// Reads every entry; a missing file is an empty cache.  Returns false (with
// the message set) on a file that is not such a JSON document.
bool read_tune_cache(const char *path, std::vector<TuneEntry> *out)
{
    out->clear();
    FILE *f = fopen(path, "rb");
    if (!f) return true;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    size_t p = text.find("\"entries\"");
    if (p == std::string::npos || (p = text.find('[', p)) == std::string::npos) {
        wo_fail(WO_E_INVAL, "tune cache %s: no \"entries\" array", path);
        return false;
    }
    p++;
    for (;;) {
        while (p < text.size() && (isspace((unsigned char)text[p]) || text[p] == ',')) p++;
        if (p < text.size() && text[p] == ']') return true;
        if (p >= text.size() || text[p] != '{') break;
        const size_t end = text.find('}', p);
        if (end == std::string::npos) break;
        const std::string obj = text.substr(p + 1, end - p - 1);
        TuneEntry e;
        bool have[12] = {false}, have_arch = false;
        size_t q = 0;
        for (;;) {
            const size_t k0 = obj.find('"', q);
            if (k0 == std::string::npos) break;
            const size_t k1 = obj.find('"', k0 + 1);
            const size_t colon = k1 == std::string::npos ? k1 : obj.find(':', k1);
            if (colon == std::string::npos) {
                wo_fail(WO_E_INVAL, "tune cache %s: malformed entry", path);
                return false;
            }
            const std::string key = obj.substr(k0 + 1, k1 - k0 - 1);
            size_t v = colon + 1;
            while (v < obj.size() && isspace((unsigned char)obj[v])) v++;
            if (v < obj.size() && obj[v] == '"') {
                const size_t v1 = obj.find('"', v + 1);
                if (v1 == std::string::npos) {
                    wo_fail(WO_E_INVAL, "tune cache %s: unterminated string", path);
                    return false;
                }
                if (key == "arch") {
                    e.arch = obj.substr(v + 1, v1 - v - 1);
                    have_arch = true;
                }
                q = v1 + 1;
            } else {
                char *stop = nullptr;
                const double x = strtod(obj.c_str() + v, &stop);
                if (stop == obj.c_str() + v) {
                    wo_fail(WO_E_INVAL, "tune cache %s: value of \"%s\" is not a number", path, key.c_str());
                    return false;
                }
                for (int k = 0; k < 12; k++)
                    if (key == kTuneKeys[k]) {
                        e.v[k] = k == 11 ? (int64_t)llround(x * 1e6) : (int64_t)llround(x);
                        have[k] = true;
                    }
                q = (size_t)(stop - obj.c_str());
            }
        }
        for (int k = 0; k < 12; k++)
            if (!have[k]) {
                wo_fail(WO_E_INVAL, "tune cache %s: an entry lacks \"%s\"", path, kTuneKeys[k]);
                return false;
            }
        if (!have_arch) {
            wo_fail(WO_E_INVAL, "tune cache %s: an entry lacks \"arch\"", path);
            return false;
        }
        out->push_back(e);
        p = end + 1;
    }
    wo_fail(WO_E_INVAL, "tune cache %s: malformed \"entries\" array", path);
    return false;
}

// Writes the entries to a temporary file beside `path`, then renames it.
bool write_tune_cache(const char *path, const std::vector<TuneEntry> &entries)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) {
        wo_fail(WO_E_INVAL, "tune cache %s: cannot write %s", path, tmp.c_str());
        return false;
    }
    fprintf(f, "{\"entries\": [");
    for (size_t i = 0; i < entries.size(); i++) {
        const TuneEntry &e = entries[i];
        fprintf(f, "%s\n  {\"arch\": \"%s\"", i ? "," : "", e.arch.c_str());
        for (int k = 0; k < 11; k++) fprintf(f, ", \"%s\": %lld", kTuneKeys[k], (long long)e.v[k]);
        fprintf(f, ", \"ms\": %.6f}", (double)e.v[11] * 1e-6);
    }
    fprintf(f, "\n]}\n");
    const bool ok = fflush(f) == 0;
    if (fclose(f) != 0 || !ok || rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        wo_fail(WO_E_INVAL, "tune cache %s: write failed", path);
        return false;
    }
    return true;
}

wo_status tune_cache_store(wo_wh *wh, const char *path, int64_t n_plans, const wo_eval_config &c)
{
    std::vector<TuneEntry> entries;
    if (!read_tune_cache(path, &entries)) return WO_E_INVAL;
    TuneEntry e;
    tune_key(wh, n_plans, &e);
    e.v[6] = c.block_threads;
    e.v[7] = c.blocks_per_cu;
    e.v[8] = c.queue;
    e.v[9] = c.line_pass;
    e.v[10] = c.small_orders;
    e.v[11] = (int64_t)llround((double)c.ms * 1e6);
    bool replaced = false;
    for (TuneEntry &x : entries)
        if (same_key(x, e)) {
            x = e;
            replaced = true;
        }
    if (!replaced) entries.push_back(e);
    return write_tune_cache(path, entries) ? WO_OK : WO_E_INVAL;
}

wo_status tune_cache_lookup(wo_wh *wh, const char *path, int64_t n_plans, bool *found, bool chosen)
{
    *found = false;
    std::vector<TuneEntry> entries;
    if (!read_tune_cache(path, &entries)) return WO_E_INVAL;
    TuneEntry key;
    tune_key(wh, n_plans, &key);
    for (const TuneEntry &e : entries)
        if (same_key(e, key)) {
            const wo_eval_config c{(int32_t)e.v[6], (int32_t)e.v[7], (int32_t)e.v[8], (int32_t)e.v[9],
                                   (int32_t)e.v[10], (float)((double)e.v[11] * 1e-6)};
            if (wo_status st = check_cfg(&c)) return st;
            apply_cfg(wh, c, chosen);
            *found = true;
        }
    return WO_OK;
}

}  // namespace

extern "C" wo_status wo_tune_cache_store(wo_wh *wh, const char *path, int64_t n_plans, const wo_eval_config *cfg)
{
    if (!wh || !path) return fail(WO_E_INVAL, "NULL argument");
    if (n_plans < 1) return fail(WO_E_INVAL, "n_plans must be >= 1");
    if (cfg)
        if (wo_status st = check_cfg(cfg)) return st;
    Busy busy(&wh->busy);
    if (!busy.ok) return fail(WO_E_STATE, "handle is in use by another thread");
    const wo_eval_config c = cfg ? *cfg : wo_eval_config{wh->block, wh->per_cu, wh->queue, wh->main_mode,
                                                         wh->small_orders, 0.f};
    return tune_cache_store(wh, path, n_plans, c);
}

extern "C" wo_status wo_tune_cache_lookup(wo_wh *wh, const char *path, int64_t n_plans, int32_t *found)
{
    if (!wh || !path || !found) return fail(WO_E_INVAL, "NULL argument");
    if (n_plans < 1) return fail(WO_E_INVAL, "n_plans must be >= 1");
    Busy busy(&wh->busy);
    if (!busy.ok) return fail(WO_E_STATE, "handle is in use by another thread");
    bool f = false;
    const wo_status st = tune_cache_lookup(wh, path, n_plans, &f, true);
    *found = f ? 1 : 0;
    return st;
}

extern "C" wo_status wo_autotune_eval(wo_wh *wh, const int64_t *plan_offsets, int64_t n_plans,
                                      const uint8_t *d_zone_of, const uint16_t *d_order_seq, int32_t *d_dist,
                                      int32_t reps, void *stream, wo_eval_config *best_out,
                                      wo_eval_config *h_all, int32_t *n_all)
{
    if (!wh) return fail(WO_E_INVAL, "handle is NULL");
    if (reps < 1) return fail(WO_E_INVAL, "reps must be >= 1");
    if (n_plans < 1) return fail(WO_E_INVAL, "need plans to time");
    hipStream_t s = (hipStream_t)stream;
    const wo_eval_config saved{wh->block, wh->per_cu, wh->queue, wh->main_mode, wh->small_orders, 0.f};
    const bool chosen0 = wh->cfg_chosen;
    wh->cfg_chosen = true;              // no cache lookup while configurations are timed
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    wo_eval_config best = saved;
    best.ms = 3.0e38f;
    int count = 0;
    wo_status st = WO_OK;
    auto apply = [&](const wo_eval_config &c) {
        wh->block = c.block_threads;
        wh->per_cu = c.blocks_per_cu;
        wh->queue = c.queue;
        wh->main_mode = c.line_pass;
        wh->small_orders = c.small_orders;
    };
    // time one configuration: a warm-up call (which also builds the work
    // lists outside the timed region), then the best of `reps`
    auto time_cfg = [&](wo_eval_config c) -> wo_status {
        apply(c);
        wo_status r = wo_eval_plans(wh, plan_offsets, n_plans, d_zone_of, d_order_seq, d_dist, nullptr, stream);
        if (r) return r;
        float ms_best = 3.0e38f;
        for (int k = 0; k < reps; k++) {
            if (hipEventRecord(e0, s) != hipSuccess) return fail(WO_E_DEVICE, "hipEventRecord failed");
            if ((r = wo_eval_plans(wh, plan_offsets, n_plans, d_zone_of, d_order_seq, d_dist, nullptr, stream)))
                return r;
            float ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                return fail(WO_E_DEVICE, "event timing failed");
            ms_best = std::min(ms_best, ms);
        }
        c.ms = ms_best;
        if (h_all && n_all && count < *n_all) h_all[count] = c;
        count++;
        if (ms_best < best.ms) best = c;
        return WO_OK;
    };
    const int blocks[4] = {64, 128, 256, 512};
    const int per_cus[8] = {1, 2, 3, 4, 6, 8, 12, 16};
    // first fit has one launch shape: time it once and keep the configuration
    const int n_blocks = wh->batching != WO_BATCH_NEXT_FIT ? 0 : 4;
    if (n_blocks == 0) st = time_cfg(saved);
    for (int bi = 0; bi < n_blocks && !st; bi++) {
        for (int pi = 0; pi < 8 && !st; pi++) {
            const int blk = blocks[bi], pc = per_cus[pi];
            for (int qm = 0; qm < 6 && !st; qm++) {
                if (wh->route != WO_ROUTE_SSHAPE && (qm >> 1)) continue;   // pick rows: line per lane only
                if (pc > eval_max_blocks_per_cu(blk, wh->route, wh->lds_max, qm >> 1)) continue;   // registers, LDS
                st = time_cfg(wo_eval_config{blk, pc, qm & 1, qm >> 1, saved.small_orders, 0.f});
            }
        }
    }
    // the small-instance launch on and off, with the best configuration
    bool any_small = false;
    for (int32_t i = 0; i < wh->n_inst && n_blocks; i++) any_small |= wh->inst[i].n_orders <= 1024;
    if (!st && any_small) {
        wo_eval_config c = best;
        c.small_orders = saved.small_orders > 0 ? 0 : 1024;
        st = time_cfg(c);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) {
        apply(saved);
        wh->cfg_chosen = chosen0;
        return st;
    }
    apply(best);
    if (best_out) *best_out = best;
    if (n_all) *n_all = count;
    const char *cache = getenv("WO_TUNE_CACHE");
    if (cache && *cache) return tune_cache_store(wh, cache, n_plans, best);
    return WO_OK;
}
