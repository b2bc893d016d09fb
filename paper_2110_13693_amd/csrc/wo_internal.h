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
    int32_t words;          // ceil(n_aisles / 32): 32-bit words of a tour's aisle set
    int32_t capacity;
    int32_t n_cat;
    int32_t n_orders;
    int32_t n_lines;        // = items (one line = one item)
    uint32_t magic;         // aisle = mulhi_u24(ls, magic)
    uint32_t shift;         // ls = l << shift
    uint32_t d_s;           // (2 * slots_per_side) << shift
    int32_t pitch;
    int32_t spacing;
    int32_t L;              // slots_per_side * pitch
    int32_t t_cap;          // tours per LDS tile
    int32_t pad0;
    int64_t rec_off;        // u32 line records [n_lines]:  (rank << shift) | (4*cat) << 24
    int64_t ooff_off;       // u32 order line offsets [n_orders + 1]
    int64_t lord_off;       // u16 order id of each line [n_lines]
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
    const uint32_t *rec;    // pooled arrays
    const uint32_t *ooff;
    const uint16_t *lord;
    const uint8_t *zone_of;
    const uint16_t *seq;
    int32_t *dist;
    float *thr;
    int32_t *err;           // device flag, validation mode
    int32_t validate;
};

// LDS layout of one evaluation block for an instance; host and device use the
// same function so that the launch size and the kernel agree.
struct EvalLayout {
    uint32_t zs, red, ctr, P, sq, e, tour, flag, mask, mx, total;
};

__host__ __device__ inline uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

__host__ __device__ inline EvalLayout eval_layout(int32_t n_orders, int32_t words, int32_t t_cap)
{
    EvalLayout L;
    uint32_t n = (uint32_t)n_orders, b = 0;
    L.zs = b;   b = align16(b + 64 * 4);
    L.red = b;  b = align16(b + 16 * 8);
    L.ctr = b;  b = align16(b + 16 * 4);
    L.P = b;    b = align16(b + 4 * (n + 1));
    L.sq = b;   b = align16(b + 2 * n);
    L.e = b;    b = align16(b + 2 * n);
    L.tour = b; b = align16(b + 2 * n);
    L.flag = b; b = align16(b + n);
    L.mask = b; b = align16(b + 4u * (uint32_t)words * (uint32_t)t_cap);
    L.mx = b;   b = align16(b + 4u * (uint32_t)t_cap);
    L.total = b;
    return L;
}

hipError_t launch_eval(const EvalArgs &a, uint32_t lds_bytes, int grid, hipStream_t s);

}  // namespace wo
