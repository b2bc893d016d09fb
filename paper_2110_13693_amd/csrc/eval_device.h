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

// Return, largest-gap, combined or optimal route of one tour from its np >= 1 picks,
// sorted by scaled location, i.e. by aisle and then depth (section 5,
// Subproblem 2).
template <int ROUTE>
static __device__ __forceinline__ int64_t pick_route_cost(const uint32_t (&v)[MAX_PICK_SLOTS], uint32_t np, int32_t spacing,
                                                          const InstDev &I, uint32_t magic)
{
    const int32_t L = I.L;
    uint32_t ca = mulhi24(v[0], magic);               // current aisle
    const uint32_t a_lo = ca;
    if (ROUTE == WO_ROUTE_OPTIMAL) {
        // start: the depot at the front of aisle 0; if aisle 0 holds no pick
        // it may still be crossed once or twice
        OptClasses s = {a_lo ? L : OPT_INF, 0, OPT_INF, a_lo ? 2 * L : OPT_INF, OPT_INF};
        uint32_t done = 0;                            // the last aisle decided
        int32_t ylo = 0, yhi = 0, gap = -1;           // first and last depth, largest gap (-1: one pick)
#pragma unroll
        for (int i = 0; i < MAX_PICK_SLOTS; i++) {
            if ((uint32_t)i < np) {
                const uint32_t a = mulhi24(v[i], magic);
                const int32_t y = (int32_t)((v[i] - a * I.d_s) >> (I.shift + 1)) * I.pitch + I.pitch / 2;
                if (i == 0) {
                    ylo = y;
                } else if (a != ca) {                 // aisle ca is complete
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
            }
        }
        if (ca != done) opt_run(s, (int32_t)(ca - done), spacing, L);
        opt_aisle(s, L, 2 * yhi, 2 * (L - ylo), gap >= 0 ? 2 * (L - gap) : 2 * L);
        return (int64_t)min(min(s.f, s.b), s.e1);     // even ends, one component
    }
    if (ROUTE == WO_ROUTE_COMBINED) {
        // each aisle with picks crossed or entered and left from the cross
        // aisle the picker is on, best choice by one length per cross aisle;
        // the walk ends on the front (crossing the last aisle from the back)
        const int64_t W = spacing, L2 = 2ll * L;
        int64_t front = 0, back = (int64_t)1 << 60;   // the back is not reachable yet
        uint32_t done = 0;
        int32_t ylo = 0, yhi = 0;
#pragma unroll
        for (int i = 0; i < MAX_PICK_SLOTS; i++) {
            if ((uint32_t)i < np) {
                const uint32_t a = mulhi24(v[i], magic);
                const int32_t y = (int32_t)((v[i] - a * I.d_s) >> (I.shift + 1)) * I.pitch + I.pitch / 2;
                if (i == 0) {
                    ylo = y;
                } else if (a != ca) {                 // aisle ca is complete
                    const int64_t step = W * (int64_t)(ca - done);
                    const int64_t f2 = min(front + 2ll * yhi, back + L), b2 = min(front + L, back + L2 - 2ll * ylo);
                    front = f2 + step;
                    back = b2 + step;
                    done = ca;
                    ca = a;
                    ylo = y;
                }
                yhi = y;
            }
        }
        const int64_t step = W * (int64_t)(ca - done);
        const int64_t f2 = min(front + 2ll * yhi, back + L), b2 = min(front + L, back + L2 - 2ll * ylo);
        return min(f2, b2 + L) + step + W * (int64_t)ca;
    }
    int32_t py = 0;                                   // previous depth in the aisle (front: 0)
    int32_t g = 0;                                    // largest gap so far in the aisle
    int64_t sum = 0;                                  // return: farthest depths; gap: inner L - gap
#pragma unroll
    for (int i = 0; i < MAX_PICK_SLOTS; i++) {
        if ((uint32_t)i < np) {
            const uint32_t a = mulhi24(v[i], magic);
            const int32_t y = (int32_t)((v[i] - a * I.d_s) >> (I.shift + 1)) * I.pitch + I.pitch / 2;
            if (a != ca) {                            // close aisle ca
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
    const int64_t horiz = 2ll * spacing * ca;       // ca is the farthest aisle now
    if (ROUTE == WO_ROUTE_RETURN) return horiz + 2 * (sum + py);
    if (ca == a_lo) return horiz + 2ll * py;           // one aisle: the return route
    return horiz + 2ll * L + 2 * sum;
}

}  // namespace wo
