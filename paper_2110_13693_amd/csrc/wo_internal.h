// Internal types shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wo.h"

namespace wo {

// Device-side description of one loaded instance.  Location arithmetic runs
// in a scaled domain ls = l << shift so that the aisle of a location is one
// 24-bit multiply-high: aisle = mulhi_u24(ls, magic).  The host picks shift
// and magic per instance and proves the identity for every location.
struct InstDev {
    int32_t n_aisles;
    int32_t words;          // 32-bit words of a tour's aisle set: the aisles that hold SKUs, rounded up
    int32_t capacity;
    int32_t n_cat;
    int32_t n_orders;
    int32_t n_lines;        // = items (one line = one item)
    int32_t n_units;        // sum over orders of min(size, capacity + 1): the bitmap's span
    uint32_t magic;         // aisle = mulhi_u24(ls, magic)
    uint32_t shift;         // ls = l << shift
    uint32_t d_s;           // (2 * slots_per_side) << shift
    int32_t pitch;
    int32_t spacing;
    int32_t L;              // slots_per_side * pitch
    int32_t t_cap;          // tours per LDS tile
    int32_t n_seg;          // item-space segments chased in parallel (1 = serial chain)
    int32_t n_lines_pad;    // line records stored: n_lines rounded up to whole groups of LINE_PAD
    int32_t chase_log2;     // log2 of the opening records per chase lane
    int32_t chase_lanes;    // chase lanes the LDS layout holds (a multiple of 64, <= CHASE_LANES)
    int32_t min_size;       // smallest min(size, capacity + 1) over the orders: a room below it never fills
    int32_t route;          // WO_ROUTE_*
    int32_t pick_slots;     // routes other than S-shape: pick entries per tour row (<= MAX_PICK_SLOTS)
    int32_t row_b;          // bytes of one tour row in LDS
    // uint2 line records [n_lines_pad]: x = (rank << shift) | (4*cat) << 24,
    // y = LDS byte offset of the order's tour entry (2 * order + the tour
    // table's offset), with bit 31 set on the first of a lane's consecutive
    // slots that hold lines of one order; the padding records point at the
    // dummy entry of order n_orders, whose row absorbs them.  Stored in
    // groups of 64 x LINE_SLOTS,
    // slot-major (record u * 64 + j of a group is line j * LINE_SLOTS + u of
    // it in instance order).
    int64_t line_off;
    int64_t cnt_off;        // u8 per order: min(size, capacity + 1) [n_orders], zero-padded to 16 bytes past n_orders + 2
    // orders in groups of 64 by descending size (one order per lane): group g
    // holds lines [gbase[g], gbase[g+1]) of grec, line k of its lane j at
    // gbase[g] + 64 k + j (shorter orders repeat their first line); gord holds
    // the order id of each lane (0xFFFF: none)
    int64_t grec_off;       // u32 records, same packing as line_off's x
    int64_t gbase_off;      // u32 [n_grp + 1], relative to grec_off
    int64_t gord_off;       // u16 [64 * n_grp]
    int32_t n_grp;
    // order o's lines are ordrec[ordoff[o] .. ordoff[o + 1]) (same packing as
    // grec), both relative to the offsets below
    int64_t ordoff_off;     // u32 [n_orders + 1]
    int64_t ordrec_off;     // u32 [n_lines]
    // routes with pick rows: the orders with more than MAX_PICK_SLOTS lines
    // (each a tour of its own), evaluated apart from the pick rows
    int64_t big_off;        // u32 order ids [n_big] in the pooled list
    int32_t n_big;
    int32_t big_np2;        // the largest such order's line count rounded up to a power of two (0: none)
    int32_t n_skus;         // sum of the category sizes: a zone start never exceeds n_skus - size
    double walk;
    double t_item;
    double window;
    int32_t cat_size[WO_MAX_CATEGORIES];
};

struct EvalArgs {
    const InstDev *inst;    // device table [n_inst]
    int32_t n_inst;
    int64_t n_plans;
    const int64_t *plan_begin;  // device [n_inst + 1]: plan rows of instance i (unused if n_inst == 1)
    const int64_t *seq_base;    // device [n_inst]: element offset of instance i's first sequence row
    const int32_t *plan_inst;   // device [n_plans]: instance of each plan row (null: search plan_begin)
    const uint2 *lines;     // pooled arrays
    const uint8_t *cnt;
    const uint32_t *grec;
    const uint32_t *gbase;
    const uint16_t *gord;
    const uint32_t *ordoff;
    const uint32_t *ordrec;
    const uint32_t *big;    // orders beyond a pick row, per instance (InstDev::big_off)
    int32_t main_mode;      // 0: one line per lane, 1: one order per lane (groups), 2: sequence order
    const uint8_t *zone_of;
    const uint16_t *seq;
    int32_t *dist;
    float *thr;
    int32_t *err;           // device flag, validation mode
    int32_t validate;
    int32_t queue;          // 1: take plans from a ticket counter
    int32_t chunk;          // consecutive work items per grid-stride step or ticket (>= 1)
    uint32_t *queue_ctr;
    const int32_t *work;    // work item -> plan row (null: identity)
    uint16_t *ff_tour;      // first fit: tour of every order, ff_stride entries per workgroup
    int64_t ff_stride;
    uint32_t *ff_queue;     // first fit: open tours past the first 64, ff_stride entries per workgroup
    const int32_t *plan_spacing;   // device [n_plans]: aisle spacing of each plan row (null: the instance's)
};

// Parallel next-fit: lanes that chase candidate tour chains (at most
// CHASE_LANES; an instance holds room for chase_lanes of them); each records
// up to 2^chase_log2 openings (at most 2^MAX_CHASE_LOG2).
constexpr int CHASE_LANES = 256;
constexpr int MAX_CHASE_LOG2 = 6;
constexpr int MAX_SEG = 64;
// line records come in groups of 64 lanes x LINE_SLOTS consecutive lines,
// padded to whole groups, so that the line pass needs no bounds checks
constexpr int LINE_SLOTS = 8;
constexpr int LINE_PAD = 64 * LINE_SLOTS;
// fixed LDS offsets: the zone-start table, the work-queue ticket, then the
// region shared by the chase records and the per-tour rows (the kernel holds
// no static LDS, so these are the addresses the instructions see)
constexpr uint32_t LDS_ZS = 0;
constexpr uint32_t LDS_TICKET = 256;
constexpr uint32_t LDS_REGION = 272;

// LDS layout of one evaluation block for an instance; host and device use the
// same function so that the launch size, the line records' tour offsets and
// the kernel agree.  The zone starts (64 words) sit at offset 0 and the shared
// region at offset 272, so that the line pass addresses both with immediate
// offsets.  The region holds, in turn: the permutation-check bitmap
// (validation), the chase records, and the per-tour rows of one tile.  A row
// is 1 + words 32-bit words: the tour's farthest scaled location, then its
// aisle set (and a pad word when that count is even); a tile has t_cap rows
// plus one dummy row.
struct EvalLayout {
    uint32_t rec, nrec, nxt, cand;     // chase phase (inside the region)
    uint32_t red, misc, seg, cnt, tour, pref, B, P;
    uint32_t total;
};

__host__ __device__ inline uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

__host__ __device__ inline uint32_t bitmap_words(int32_t n_units) { return ((uint32_t)n_units >> 5) + 3u; }

// An S-shape row is the farthest location plus the aisle set; a return or
// largest-gap row is a pick count plus up to pick_slots scaled locations.
// Rows are padded to an odd word count so that rows of random tours spread
// over all 32 LDS banks.
constexpr int MAX_PICK_SLOTS = 32;
// a tour of several orders holds at most the capacity: an order longer than a
// pick row is always a tour of its own
static_assert(WO_MAX_CAPACITY <= MAX_PICK_SLOTS, "capacity beyond a pick row");
// routes other than S-shape: the most lines an order may have (its sort in LDS)
constexpr int MAX_BIG_ORDER_LINES = WO_MAX_ROUTED_ORDER_LINES;
__host__ __device__ inline uint32_t row_bytes(int32_t words) { return 4u * ((uint32_t)(words + 1) | 1u); }
__host__ __device__ inline uint32_t pick_row_bytes(int32_t slots) { return 4u * ((uint32_t)(slots + 1) | 1u); }

// First-fit batching runs in a kernel of its own, one wavefront per plan.
// LDS: the zone starts (64 words), then one tile of tour rows (192 S-shape
// rows, or 64 pick rows for the other routes); the tour of every order goes
// to a global table with one slice per workgroup of the launch, and open
// tours beyond the 64 a wavefront keeps in registers to a queue with one
// slice per workgroup.  Tours never outnumber orders.
__host__ __device__ constexpr int ff_tile(int route) { return route == WO_ROUTE_SSHAPE ? 192 : 64; }
__host__ __device__ inline uint32_t ff_rows_off() { return 256u; }

// bytes of the cnt table (order sizes, then zeros for the dummy and sink entries)
__host__ __device__ inline uint32_t cnt_bytes(int32_t n_orders) { return align16((uint32_t)n_orders + 2u); }
__host__ __device__ inline uint32_t ff_lds_bytes(int route, int32_t row_b)
{
    return ff_rows_off() + (uint32_t)ff_tile(route) * (uint32_t)row_b;
}

__host__ __device__ inline EvalLayout eval_layout(int32_t n_orders, int32_t n_units, uint32_t rb,
                                                  int32_t t_cap, int32_t chase_log2, int32_t chase_lanes)
{
    const uint32_t cl = (uint32_t)chase_lanes;
    EvalLayout L;
    const uint32_t n = (uint32_t)n_orders, nb = bitmap_words(n_units);
    uint32_t c = LDS_REGION;
    L.rec = c;   c = align16(c + (2u * cl << chase_log2));
    L.nrec = c;  c = align16(c + 4u * cl);
    L.nxt = c;   c = align16(c + 4u * cl);
    L.cand = c;  c = align16(c + 4u * cl);
    const uint32_t rows = align16(LDS_REGION + rb * (uint32_t)(t_cap + 1));
    const uint32_t seen = align16(LDS_REGION + 4u * ((n + 31) / 32));
    uint32_t b = c > rows ? c : rows;
    if (seen > b) b = seen;
    L.red = b;   b = align16(b + 2 * 16 * 4 + 8 * 8);   // two scan slots, one int64 reduction slot
    L.misc = b;  b = align16(b + 16 * 4);
    L.seg = b;   b = align16(b + 4 * 4 * (MAX_SEG + 1));   // lane_base | wbits | true_lane | seg start
    L.cnt = b;   b += cnt_bytes(n_orders);
    L.tour = b;  b = align16(b + 2 * (n + 2));            // + dummy entry n, sink entry n + 1
    L.pref = b;  b = align16(b + 4 * nb);               // order starts below each unit word
    L.B = b;     b = align16(b + 4 * nb);
    L.P = b;     b = align16(b + 4 * (n / 32 + 3));      // tour openings by sequence position
    L.total = b;
    return L;
}

// Seed batching builds its tours in LDS before the tile pass, in the space
// the tile's rows take afterwards: per sequence position a state word (new
// aisles of the order for the tour being built, bits 0-9; its aisle count,
// bits 10-19; its size, bits 20-27; bit 31 once it is in a tour); per aisle
// the end of its list of positions; the positions grouped by aisle (one entry
// per order and aisle it visits, at most one per line); the tour's aisle set.
// An order visits at most SEED_MAX_AISLES aisles.
constexpr int SEED_MAX_AISLES = 1023;
struct SeedLayout {
    uint32_t st, aend, apos, tbits, total;
};
__host__ __device__ inline SeedLayout seed_layout(int32_t n_orders, int32_t n_aisles, int32_t n_lines)
{
    SeedLayout L;
    uint32_t b = ff_rows_off();
    L.st = b;     b = (b + 4u * (uint32_t)n_orders + 15u) & ~15u;
    L.aend = b;   b += 4u * (uint32_t)n_aisles;
    L.tbits = b;  b += 4u * (((uint32_t)n_aisles + 31u) / 32u);
    L.apos = b;   b = (b + 2u * (uint32_t)n_lines + 15u) & ~15u;
    L.total = b;
    return L;
}

hipError_t launch_eval(const EvalArgs &a, uint32_t lds_bytes, int grid, int block, int route, hipStream_t s);
// workgroups of the evaluation kernel that fit one CU (registers and LDS)
int eval_max_blocks_per_cu(int block, int route, uint32_t lds_bytes, int line_pass = 0);
// First-fit batching: one 64-thread workgroup per plan.
hipError_t launch_eval_ff(const EvalArgs &a, uint32_t lds_bytes, int grid, int route, bool seed, hipStream_t s);
int eval_ff_max_blocks_per_cu(int route, bool seed, uint32_t lds_bytes);

// library-internal helpers over a loaded handle
wo_status eval_instance(wo_wh *wh, int32_t inst, int64_t n_plans, const uint8_t *d_zone_of,
                        const uint16_t *d_order_seq, int32_t *d_dist, float *d_thr, hipStream_t s,
                        const int32_t *d_plan_spacing = nullptr);
const InstDev &instance_dev(const wo_wh *wh, int32_t inst);
int32_t instance_orders(const wo_wh *wh, int32_t inst);
int32_t instance_categories(const wo_wh *wh, int32_t inst);
int32_t instance_count(const wo_wh *wh);

}  // namespace wo
