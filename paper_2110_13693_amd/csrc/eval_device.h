// Device helpers shared by the plan-evaluation kernels (eval.hip: next-fit
// batching; firstfit.hip: first-fit and seed batching): wave scans, location
// arithmetic, the time-window rate, the instance of a plan row, and the route
// of one tour from its picks (section 5, Subproblem 2).
#pragma once

#include "wo_internal.h"

namespace wo {

// Inclusive prefix sum over the 64 lanes of a wave (all lanes active): shifts
// by 1, 2, 4, 8 inside each row of 16 lanes, then the row totals carried by
// the row broadcasts of lanes 15 and 31.
static __device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);   // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return x;
}

// Smallest value over the 64 lanes of a wave (all lanes active), the same
// shifts and broadcasts; every lane gets it.
static __device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x111, 0xF, 0xF, false));   // row_shr:1
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x112, 0xF, 0xF, false));   // row_shr:2
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x114, 0xF, 0xF, false));   // row_shr:4
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x118, 0xF, 0xF, false));   // row_shr:8
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));   // row_bcast:15
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));   // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

static __device__ __forceinline__ uint32_t mulhi24(uint32_t x, uint32_t m)
{
    return (uint32_t)(((uint64_t)(x & 0xFFFFFFu) * (uint64_t)(m & 0xFFFFFFu)) >> 32);
}

static __device__ __forceinline__ float window_throughput(int64_t D, const InstDev &I)
{
    // T = D / walk + t_item * items; orders * window / T: IEEE double, one
    // operation at a time (no multiply-add contraction), rounded once
#pragma clang fp contract(off)
    const double q = (double)D / I.walk;
    const double u = I.t_item * (double)I.n_lines;
    const double T = q + u;
    const double r = ((double)I.n_orders * I.window) / T;
    return (float)r;
}

// Instance of plan row p: from the per-plan table when there is one, else the
// last instance whose first row is <= p.
static __device__ __forceinline__ int instance_of(const EvalArgs &A, int64_t p)
{
    if (A.n_inst <= 1) return 0;
    if (A.plan_inst) return A.plan_inst[p];
    int lo = 0, hi = A.n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.plan_begin[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Ascending bitonic sort of 32 words held in registers (straight-line min/max).
static __device__ __forceinline__ void sort32(uint32_t (&v)[MAX_PICK_SLOTS])
{
#pragma unroll
    for (int k = 2; k <= MAX_PICK_SLOTS; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < MAX_PICK_SLOTS; i++) {
                const int l = i ^ j;
                if (l > i) {
                    const uint32_t a = v[i], b = v[l];
                    const bool up = (i & k) == 0;
                    v[i] = up ? min(a, b) : max(a, b);
                    v[l] = up ? max(a, b) : min(a, b);
                }
            }
}

// Optimal route of one tour (the minimum route distance of section 5,
// Subproblem 2) in the manner of Ratliff and Rosenthal: a programme over the
// aisles holding picks, left to right.  A partial walk is in one of five
// classes at the two ends (front f, back b) of the last aisle decided:
//   O1: f and b of odd degree, one component;
//   F : only f in the walk (even degree);
//   B : only b in the walk (even degree);
//   E1: f and b of even degree, one component;
//   E2: f and b of even degree, two components.
// A tour's distances are bounded at load so that every class cost, including
// the unreachable value OPT_INF plus any sum of additions, stays below 2^31.
#define OPT_INF 0x40000000
struct OptClasses { int32_t o1, f, b, e1, e2; };

// Carry the classes over r >= 1 steps along the cross aisles to the next
// aisle with picks (r - 1 aisles without picks in between).  One step costs
// 2w in O1, F and B (one edge each way, or both on one side) and 4w in E1 and
// E2.  In the aisles passed, a class may change by a crossing (cost L) or a
// double crossing (2 L); the cheapest such change is taken as early as it
// lowers the step cost and as late as it raises it, which gives these forms.
static __device__ __forceinline__ void opt_run(OptClasses &s, int32_t r, int32_t w, int32_t L)
{
    const int32_t a = 2 * w;
    const int32_t ar = a * r, ar1 = ar + a, ar2 = ar1 + a;
    const int32_t m_fbe = min(min(s.f, s.b), s.e1);
    OptClasses n;
    n.o1 = s.o1 + ar;
    n.f = min(s.f, s.e1) + ar;            // E1 drops its back end
    n.b = min(s.b, s.e1) + ar;
    n.e1 = s.e1 + 2 * ar;
    n.e2 = s.e2 + 2 * ar;
    if (r >= 2) {                         // an aisle without picks lies in between
        n.o1 = min(n.o1, min(m_fbe + ar, s.e2 + ar1) + L);
        n.f = min(n.f, min(min(s.o1 + ar + L, s.b + ar + 2 * L), s.e2 + ar1 + 2 * L));
        n.b = min(n.b, min(min(s.o1 + ar + L, s.f + ar + 2 * L), s.e2 + ar1 + 2 * L));
        n.e1 = min(n.e1, min(min(s.o1 + ar1 + L, m_fbe + ar1 + 2 * L), s.e2 + ar2 + 2 * L));
    }
    s = n;
}

// The aisle's own edges: a crossing (L), a double crossing (2 L), in from the
// front to the last pick (cF), in from the back to the first pick (cB), or in
// from both sides leaving out the largest gap between two picks (cG; 2 L when
// the aisle has a single pick, which never beats cF or cB then).
static __device__ __forceinline__ void opt_aisle(OptClasses &s, int32_t L, int32_t cF, int32_t cB, int32_t cG)
{
    const int32_t cmin = min(min(cF, cB), cG);
    const int32_t m_even = min(min(s.f, s.b), min(s.e1, s.e2));
    OptClasses n;
    n.o1 = min(s.o1 + cmin, m_even + L);
    n.f = s.f + cF;
    n.b = s.b + cB;
    n.e1 = min(min(s.o1 + L, s.e1 + cmin), m_even + 2 * L);
    n.e2 = min(min(s.f + min(cB, cG), s.b + min(cF, cG)), s.e2 + cmin);
    s = n;
}

// Walk of one tour for the return, largest-gap, combined or optimal route,
// fed the tour's picks one at a time sorted by scaled location, i.e. by
// aisle and then depth (section 5, Subproblem 2).  The first pick starts the
// walk, each further one is a step, and cost() closes it.
template <int ROUTE>
struct PickWalk {
    const InstDev &I;
    uint32_t magic;
    int32_t spacing;
    uint32_t ca, a_lo;                // current aisle, first aisle
    // optimal: the five classes, the last aisle decided, first and last
    // depth in the current aisle and its largest gap (-1: one pick)
    OptClasses s;
    uint32_t done;
    int32_t ylo, yhi, gap;
    // combined: the best walks ending on the front and on the back
    int64_t front, back;
    // return / largest gap: previous depth in the aisle (front: 0), largest
    // gap so far in it, and the sum over closed aisles
    int32_t py, g;
    int64_t sum;

    __device__ __forceinline__ int32_t depth(uint32_t ls, uint32_t a) const
    {
        return (int32_t)((ls - a * I.d_s) >> (I.shift + 1)) * I.pitch + I.pitch / 2;
    }

    __device__ __forceinline__ PickWalk(const InstDev &inst, int32_t sp, uint32_t m, uint32_t first)
        : I(inst), magic(m), spacing(sp)
    {
        const int32_t L = I.L;
        ca = mulhi24(first, magic);
        a_lo = ca;
        const int32_t y = depth(first, ca);
        if (ROUTE == WO_ROUTE_OPTIMAL) {
            // start: the depot at the front of aisle 0; if aisle 0 holds no
            // pick it may still be crossed once or twice
            s = {a_lo ? L : OPT_INF, 0, OPT_INF, a_lo ? 2 * L : OPT_INF, OPT_INF};
            done = 0;
            ylo = y;
            yhi = y;
            gap = -1;
        } else if (ROUTE == WO_ROUTE_COMBINED) {
            front = 0;
            back = (int64_t)1 << 60;      // the back is not reachable yet
            done = 0;
            ylo = y;
            yhi = y;
        } else {
            sum = 0;
            g = y;
            py = y;
        }
    }

    __device__ __forceinline__ void step(uint32_t ls)
    {
        const int32_t L = I.L;
        const uint32_t a = mulhi24(ls, magic);
        const int32_t y = depth(ls, a);
        if (ROUTE == WO_ROUTE_OPTIMAL) {
            if (a != ca) {                // aisle ca is complete
                if (ca != done) opt_run(s, (int32_t)(ca - done), spacing, L);
                opt_aisle(s, L, 2 * yhi, 2 * (L - ylo), gap >= 0 ? 2 * (L - gap) : 2 * L);
                done = ca;
                ca = a;
                ylo = y;
                gap = -1;
            } else {
                gap = max(gap, y - yhi);
            }
            yhi = y;
        } else if (ROUTE == WO_ROUTE_COMBINED) {
            // each aisle with picks crossed or entered and left from the
            // cross aisle the picker is on, best choice by one length per
            // cross aisle
            if (a != ca) {
                const int64_t st = (int64_t)spacing * (int64_t)(ca - done);
                const int64_t f2 = min(front + 2ll * yhi, back + L), b2 = min(front + L, back + 2ll * L - 2ll * ylo);
                front = f2 + st;
                back = b2 + st;
                done = ca;
                ca = a;
                ylo = y;
            }
            yhi = y;
        } else {
            if (a != ca) {                // close aisle ca
                if (ROUTE == WO_ROUTE_RETURN) {
                    sum += py;
                } else {
                    g = max(g, L - py);
                    if (ca != a_lo) sum += L - g;
                }
                ca = a;
                py = 0;
                g = 0;
            }
            g = max(g, y - py);
            py = y;
        }
    }

    __device__ __forceinline__ int64_t cost()
    {
        const int32_t L = I.L;
        if (ROUTE == WO_ROUTE_OPTIMAL) {
            if (ca != done) opt_run(s, (int32_t)(ca - done), spacing, L);
            opt_aisle(s, L, 2 * yhi, 2 * (L - ylo), gap >= 0 ? 2 * (L - gap) : 2 * L);
            return (int64_t)min(min(s.f, s.b), s.e1);   // even ends, one component
        }
        if (ROUTE == WO_ROUTE_COMBINED) {
            // the walk ends on the front (crossing the last aisle from the back)
            const int64_t st = (int64_t)spacing * (int64_t)(ca - done);
            const int64_t f2 = min(front + 2ll * yhi, back + L), b2 = min(front + L, back + 2ll * L - 2ll * ylo);
            return min(f2, b2 + L) + st + (int64_t)spacing * (int64_t)ca;
        }
        const int64_t horiz = 2ll * spacing * ca;    // ca is the farthest aisle now
        if (ROUTE == WO_ROUTE_RETURN) return horiz + 2 * (sum + py);
        if (ca == a_lo) return horiz + 2ll * py;     // one aisle: the return route
        return horiz + 2ll * L + 2 * sum;
    }
};

// Route cost of one tour from its np (1 .. MAX_PICK_SLOTS) sorted picks in
// registers.
template <int ROUTE>
static __device__ __forceinline__ int64_t pick_route_cost(const uint32_t (&v)[MAX_PICK_SLOTS], uint32_t np, int32_t spacing,
                                                          const InstDev &I, uint32_t magic)
{
    PickWalk<ROUTE> w(I, spacing, magic, v[0]);
#pragma unroll
    for (int i = 1; i < MAX_PICK_SLOTS; i++)
        if ((uint32_t)i < np) w.step(v[i]);
    return w.cost();
}

// Route costs of the instance's orders with more lines than a pick row keeps
// (each a tour of its own, since the capacity is at most MAX_PICK_SLOTS), for
// one plan: the workgroup's NT threads stage an order's scaled locations in
// LDS (`scr`, at least 4 * I.big_np2 bytes, free for the call; zs the zone
// starts), sort them (bitonic, padded with all ones), and thread 0 walks
// them.  Returns the sum on thread 0 and 0 elsewhere; every thread must call.
template <int ROUTE, int NT>
static __device__ int64_t big_orders_cost(const EvalArgs &A, const InstDev &I, const uint32_t *zs, uint32_t *scr,
                                          int32_t spacing)
{
    const int tid = threadIdx.x;
    const uint32_t *big = A.big + I.big_off;
    const uint32_t *ordoff = A.ordoff + I.ordoff_off;
    const uint32_t *ordrec = A.ordrec + I.ordrec_off;
    int64_t acc = 0;
    for (int b = 0; b < I.n_big; b++) {
        const uint32_t o = big[b];
        const uint32_t r0 = ordoff[o];
        const uint32_t m2 = min(1u << (32 - __builtin_clz(max(ordoff[o + 1] - r0, 2u) - 1u)), (uint32_t)I.big_np2);
        const uint32_t m = min(ordoff[o + 1] - r0, m2);
        __syncthreads();                 // scr is free (earlier use, previous order)
        for (uint32_t i = tid; i < m2; i += NT) {
            const uint32_t r = i < m ? ordrec[r0 + i] : 0u;
            scr[i] = i < m ? r + zs[r >> 26] : 0xFFFFFFFFu;
        }
        for (uint32_t k = 2; k <= m2; k <<= 1)
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                __syncthreads();
                for (uint32_t i = tid; i < m2; i += NT) {
                    const uint32_t l = i ^ j;
                    if (l > i) {
                        const uint32_t x = scr[i], y = scr[l];
                        const bool up = (i & k) == 0;
                        if ((x > y) == up) {
                            scr[i] = y;
                            scr[l] = x;
                        }
                    }
                }
            }
        __syncthreads();
        if (tid == 0) {
            PickWalk<ROUTE> w(I, spacing, I.magic, scr[0]);
            for (uint32_t i = 1; i < m; i++) w.step(scr[i]);
            acc += w.cost();
        }
    }
    __syncthreads();                     // scr is free again
    return acc;
}

}  // namespace wo
