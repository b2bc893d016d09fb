// First-fit order batching (see eval_ff_kernel below), for every route.
#include "eval_device.h"

namespace wo {

// Largest value over the wavefront (DPP row shifts and broadcasts, as in
// wave_incl_scan; lanes without a source keep their own value).
static __device__ __forceinline__ int32_t wave_max_i32(int32_t v)
{
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x111, 0xF, 0xF, false));   // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x112, 0xF, 0xF, false));   // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x114, 0xF, 0xF, false));   // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x118, 0xF, 0xF, false));   // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xA, 0xF, false));   // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xC, 0xF, false));   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Plans under first-fit order batching (the other greedy batching rule of the
// order-picking literature beside next fit; section 5, Subproblem 2 leaves
// the batching of orders into tours open), for each route.  One wavefront
// evaluates one plan:
//   1. zone starts: each category's start is the total size of the
//      categories in lower zones (one pass over the categories per lane);
//   2. first fit, order by order in sequence: lane l keeps the free room of
//      tours l, 64 + l, 128 + l, ... in registers (a byte each), and lane c
//      an upper bound of the largest room among tours 64c .. 64c + 63.  The
//      groups whose bound admits the order are tried in turn: one register
//      of the group and a ballot find its first tour with room; a group
//      without one gets its exact largest room as its new bound.  Every order
//      has an item, so an empty room never fits;
//   3. tiles of tours: for the S-shape route, every line of an order in the
//      tile sets its aisle bit in the tour's LDS row and the order raises the
//      tour's farthest location, then one lane per tour takes the closed
//      form; for the other routes every line record appends its location to
//      its tour's pick row, then one lane per tour sorts the picks and walks
//      them as the next-fit kernel does;
//   4. the wave's sum, saturated to int32, and the rate over the window.
template <int ROUTE>
__global__ __launch_bounds__(64) void eval_ff_kernel(EvalArgs A)
{
    constexpr int TILE = ff_tile(ROUTE);
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    for (int64_t p = blockIdx.x; p < A.n_plans; p += gridDim.x) {
        const int ii = instance_of(A, p);
        const InstDev &I = A.inst[ii];
        const int n = I.n_orders;
        const int C = I.n_cat;
        const int32_t Q = I.capacity;
        const int32_t wsp = A.plan_spacing ? A.plan_spacing[p] : I.spacing;   // aisle spacing of this plan
        const int64_t row = p - (A.n_inst > 1 ? A.plan_begin[ii] : 0);
        const uint16_t *seq = A.seq + A.seq_base[ii] + row * (int64_t)n;
        const uint8_t *cnt = A.cnt + I.cnt_off;
        uint32_t *zs = (uint32_t *)smem;
        uint16_t *tour_of = A.ff_tour + (int64_t)blockIdx.x * A.ff_stride;   // this workgroup's slice
        uint32_t *rows = (uint32_t *)(smem + ff_rows_off());
        const uint32_t RW = (uint32_t)I.row_b / 4u;
        int bad = 0;

        // ---- 1. zone starts ---------------------------------------------
        {
            const uint32_t zc = lane < C ? (uint32_t)A.zone_of[p * 64 + lane] : 0xFFu;
            const uint32_t sz = lane < C ? (uint32_t)I.cat_size[lane] : 0u;
            uint32_t start = 0;
            for (int c = 0; c < C; c++) {
                const uint32_t zo = (uint32_t)__shfl((int)zc, c, 64);
                start += zo < zc ? (uint32_t)I.cat_size[c] : 0u;
            }
            // a malformed row cannot move a category off the warehouse
            start = min(start, (uint32_t)I.n_skus - sz);
            zs[lane] = (start << I.shift) - ((uint32_t)(4 * lane) << 24);
            if (A.validate) {
                uint64_t m = (lane < C && zc < 64u) ? (1ull << zc) : 0ull;
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) m |= __shfl_xor(m, d, 64);
                const uint64_t want = (C == 64) ? ~0ull : ((1ull << C) - 1ull);
                if (m != want) bad = 1;
            }
        }
        for (int o = lane; o <= n; o += 64) tour_of[o] = 0xFFFFu;   // no tour yet; entry n: padding
        if (A.validate) {
            // every order exactly once: mark them in the tour table, which
            // is then reset
            __syncthreads();
            for (int i = lane; i < n; i += 64) {
                const uint32_t o = seq[i];
                if (o < (uint32_t)n) tour_of[o] = 0; else bad = 1;
            }
            __syncthreads();
            for (int o = lane; o < n; o += 64) {
                bad |= tour_of[o] != 0;
                tour_of[o] = 0xFFFFu;
            }
        }
        __syncthreads();

        // ---- 2. first fit -------------------------------------------------
        // a chain of dependent steps: it issues ahead of other plans' tiles
        __builtin_amdgcn_s_setprio(2);
        int T = 0;                         // tours opened (uniform)
        int32_t gmax = 0;                  // lane c: >= the largest room in tours 64c..64c+63
        uint32_t R[FF_MAX_ORDERS / 256];   // byte b of R[q]: room of tour 64 (4q + b) + lane
#pragma unroll
        for (int q = 0; q < FF_MAX_ORDERS / 256; q++) R[q] = 0u;
        for (int i0 = 0; i0 < n; i0 += 64) {
            const int i = i0 + lane;
            const uint32_t o_l = i < n ? min((uint32_t)seq[i], (uint32_t)n) : (uint32_t)n;
            // min(size, Q + 1); 0 for an id out of range, which then joins
            // some tour without taking room and is left out below
            const uint32_t s_l = cnt[o_l];
            const int m = __builtin_amdgcn_readfirstlane(min(64, n - i0));   // uniform: a scalar loop bound
            int t_l = 0;                               // lane j: tour of position i0 + j
            for (int j = 0; j < m; j++) {
                const int32_t sz = __builtin_amdgcn_readlane((int)s_l, j);
                int c = -1, k = 0;                     // group and lane of the tour found
                uint64_t g = __ballot(gmax >= sz);     // none for an order larger than Q
                if (g) {
                    // the first group whose bound admits the order: usually it has room
                    int cg = __builtin_ctzll(g);
                    int32_t r = (int32_t)((R[cg >> 2] >> (8u * (uint32_t)(cg & 3))) & 0xFFu);
                    uint64_t f = __ballot(r >= sz);
                    while (!f) {                       // the bound was stale (uniform)
                        const int32_t mx = wave_max_i32(r);
                        if (lane == cg) gmax = mx;
                        g &= g - 1;
                        if (!g) break;
                        cg = __builtin_ctzll(g);
                        r = (int32_t)((R[cg >> 2] >> (8u * (uint32_t)(cg & 3))) & 0xFFu);
                        f = __ballot(r >= sz);
                    }
                    if (f) {
                        c = cg;
                        k = __builtin_ctzll(f);
                    }
                }
                int t;
                if (c >= 0) {                          // the order joins tour 64c + k
                    t = 64 * c + k;
                    // every lane takes part (no divergent update of the register array)
                    R[c >> 2] -= lane == k ? (uint32_t)sz << (8u * (uint32_t)(c & 3)) : 0u;
                } else {                               // no open tour has room
                    t = T;
                    const int32_t r0 = sz <= Q ? Q - sz : 0;   // a larger order rides alone
                    const int cn = T >> 6;
                    R[cn >> 2] |= lane == (T & 63) ? (uint32_t)r0 << (8u * (uint32_t)(cn & 3)) : 0u;
                    if (lane == cn) gmax = max(gmax, r0);
                    T++;
                }
                t_l = lane == j ? t : t_l;
            }
            // read after the tile loop's barrier
            if (i < n && o_l < (uint32_t)n) tour_of[o_l] = (uint16_t)t_l;
        }

        __builtin_amdgcn_s_setprio(0);

        // ---- 3. tiles of tours -----------------------------------------------
        int64_t acc = 0;
        for (int t0 = 0; t0 < T; t0 += TILE) {
            for (uint32_t k = lane; k < TILE * RW; k += 64) rows[k] = 0u;
            __syncthreads();
            if (ROUTE == WO_ROUTE_SSHAPE) {
                // aisle sets and farthest locations, one order per lane from
                // the groups of 64 orders of like size: an order outside the
                // tile loads none of its lines
                const uint32_t *grec = A.grec + I.grec_off;
                const uint32_t *gbase = A.gbase + I.gbase_off;
                const uint16_t *gord = A.gord + I.gord_off;
                for (int g = 0; g < I.n_grp; g++) {
                    const uint32_t o = gord[64 * g + lane];            // 0xFFFF: no order
                    const uint32_t b0 = gbase[g];
                    const uint32_t len = (gbase[g + 1] - b0) >> 6;     // lines of the group's longest order
                    const uint32_t t = (o < (uint32_t)n ? (uint32_t)tour_of[o] : 0xFFFFu) - (uint32_t)t0;
                    if (t >= (uint32_t)TILE) continue;
                    uint32_t far = 0;
                    for (uint32_t k = 0; k < len; k += 4) {
                        uint32_t x[4];
#pragma unroll
                        for (int q = 0; q < 4; q++)                     // shorter orders repeat their first line
                            x[q] = grec[b0 + 64u * min(k + (uint32_t)q, len - 1u) + (uint32_t)lane];
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            const uint32_t ls = x[q] + zs[x[q] >> 26];
                            const uint32_t a = mulhi24(ls, I.magic);
                            atomicOr(&rows[t * RW + 1u + (a >> 5)], 1u << (a & 31u));
                            far = max(far, ls);
                        }
                    }
                    atomicMax(&rows[t * RW], far);
                }
            } else {
                // pick rows: every line exactly once, from the instance's line
                // records, which name their order by its entry in the
                // next-fit kernel's tour table (the padding records name
                // order n)
                const uint32_t nf_tour = eval_layout(n, I.n_units, (uint32_t)I.row_b, I.t_cap, I.chase_log2,
                                                     I.chase_lanes).tour;
                const uint2 *lines = A.lines + I.line_off;
                for (int r = lane; r < I.n_lines_pad; r += 64) {
                    const uint2 rec = lines[r];
                    const uint32_t o = ((rec.y & 0x7FFFFFFFu) - nf_tour) >> 1;
                    const uint32_t t = (o < (uint32_t)n ? (uint32_t)tour_of[o] : 0xFFFFu) - (uint32_t)t0;
                    if (t >= (uint32_t)TILE) continue;
                    const uint32_t ls = rec.x + zs[rec.x >> 26];
                    const uint32_t e = atomicAdd(&rows[t * RW], 1u);
                    rows[t * RW + 1u + min(e, (uint32_t)I.pick_slots - 1u)] = ls;
                }
            }
            __syncthreads();
            for (int tt = lane; tt < TILE && t0 + tt < T; tt += 64) {
                const uint32_t *rw = rows + (uint32_t)tt * RW;
                if (ROUTE == WO_ROUTE_SSHAPE) {
                    const uint32_t ls = rw[0];
                    int k = 0;
                    for (int w = 0; w < I.words; w++) k += __popc(rw[1 + w]);
                    const uint32_t a = mulhi24(ls, I.magic);
                    const int64_t y = (int64_t)((ls - a * I.d_s) >> (I.shift + 1)) * I.pitch + I.pitch / 2;
                    acc += 2ll * wsp * a + ((k & 1) ? (int64_t)(k - 1) * I.L + 2 * y : (int64_t)k * I.L);
                } else {
                    const uint32_t np = min(rw[0], (uint32_t)I.pick_slots);
                    if (np == 0) continue;                  // only a malformed row leaves a tour empty
                    uint32_t v[MAX_PICK_SLOTS];
#pragma unroll
                    for (int i = 0; i < MAX_PICK_SLOTS; i++) v[i] = (uint32_t)i < np ? rw[1 + i] : 0xFFFFFFFFu;
                    sort32(v);
                    acc += pick_route_cost<ROUTE>(v, np, wsp, I, I.magic);
                }
            }
            __syncthreads();
        }

        // ---- 4. sum and rate -----------------------------------------------
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
        if (A.validate && bad) atomicOr(A.err, 1);
        if (lane == 0) {
            A.dist[p] = acc > 2147483647ll ? 2147483647 : (int32_t)acc;
            if (A.thr) A.thr[p] = window_throughput(acc, I);
        }
        __syncthreads();
    }
}

template <int ROUTE>
static hipError_t launch_eval_ff_r(const EvalArgs &a, uint32_t lds_bytes, int grid, hipStream_t s)
{
    static uint32_t attr_bytes = 0;
    if (lds_bytes > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)eval_ff_kernel<ROUTE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        attr_bytes = lds_bytes;
    }
    hipLaunchKernelGGL(eval_ff_kernel<ROUTE>, dim3(grid), dim3(64), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_eval_ff(const EvalArgs &a, uint32_t lds_bytes, int grid, int route, hipStream_t s)
{
    switch (route) {
    case WO_ROUTE_SSHAPE: return launch_eval_ff_r<WO_ROUTE_SSHAPE>(a, lds_bytes, grid, s);
    case WO_ROUTE_RETURN: return launch_eval_ff_r<WO_ROUTE_RETURN>(a, lds_bytes, grid, s);
    case WO_ROUTE_LARGEST_GAP: return launch_eval_ff_r<WO_ROUTE_LARGEST_GAP>(a, lds_bytes, grid, s);
    case WO_ROUTE_OPTIMAL: return launch_eval_ff_r<WO_ROUTE_OPTIMAL>(a, lds_bytes, grid, s);
    case WO_ROUTE_COMBINED: return launch_eval_ff_r<WO_ROUTE_COMBINED>(a, lds_bytes, grid, s);
    }
    return hipErrorInvalidValue;
}

template <int ROUTE>
static int ff_max_blocks_r(uint32_t lds_bytes)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, eval_ff_kernel<ROUTE>, 64, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

int eval_ff_max_blocks_per_cu(int route, uint32_t lds_bytes)
{
    switch (route) {
    case WO_ROUTE_RETURN: return ff_max_blocks_r<WO_ROUTE_RETURN>(lds_bytes);
    case WO_ROUTE_LARGEST_GAP: return ff_max_blocks_r<WO_ROUTE_LARGEST_GAP>(lds_bytes);
    case WO_ROUTE_OPTIMAL: return ff_max_blocks_r<WO_ROUTE_OPTIMAL>(lds_bytes);
    case WO_ROUTE_COMBINED: return ff_max_blocks_r<WO_ROUTE_COMBINED>(lds_bytes);
    }
    return ff_max_blocks_r<WO_ROUTE_SSHAPE>(lds_bytes);
}

}  // namespace wo
