// First-fit order batching (see eval_ff_kernel below), for every route.
#include "eval_device.h"

namespace wo {

// x with lane l (uniform) set to v (uniform): v_writelane
extern "C" __device__ int wo_writelane_i32(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
static __device__ __forceinline__ uint32_t set_lane(uint32_t x, uint32_t v, int l)
{
    return (uint32_t)wo_writelane_i32((int)v, l, (int)x);
}

// Plans under first-fit or seed order batching (the other greedy batching
// rules of the order-picking literature beside next fit; section 5,
// Subproblem 2 leaves the batching of orders into tours open), for each
// route.  One wavefront evaluates one plan:
//   1. zone starts: each category's start is the total size of the
//      categories in lower zones (one pass over the categories per lane);
//   2. first fit, order by order in sequence, over the open tours only (a
//      tour whose room falls below the instance's smallest order can never
//      take another one).  Lane j keeps the j-th tour in opening order and
//      its room, so one ballot finds the earliest tour with room; full tours
//      leave the lanes only when the lanes run out.  The open tours stay few
//      (first fit keeps filling the earliest ones), but any beyond 64 wait,
//      in order, in a queue in global memory that is searched, 64 at a time,
//      when no lane has room, and refills the lanes;
//   2'. or seed batching: per position the order's size, aisle count and
//      "new aisles" (for the tour being built) in one word, and per aisle the positions
//      of the orders visiting it, all in LDS.  A tour starts from the
//      earliest position in no tour; each order that joins it marks its
//      aisles in the tour's set, and every order visiting an aisle new to
//      the tour loses one new aisle (an atomic decrement per order and
//      aisle); then one wave-wide minimum over (new aisles, position) of the
//      orders that fit picks the next one;
//   3. tiles of tours: for the S-shape route, every line of an order in the
//      tile sets its aisle bit in the tour's LDS row and the order raises the
//      tour's farthest location, then one lane per tour takes the closed
//      form; for the other routes every line record appends its location to
//      its tour's pick row, then one lane per tour sorts the picks and walks
//      them as the next-fit kernel does;
//   4. the wave's sum, saturated to int32, and the rate over the window.
template <int ROUTE, bool SEED>
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

        // ---- 2. tours ------------------------------------------------------
        // a chain of dependent steps: it issues ahead of other plans' tiles
        __builtin_amdgcn_s_setprio(2);
        int T = 0;                                      // tours opened (uniform)
        if constexpr (SEED) {
            // seed batching
            const int NA = I.n_aisles;
            const SeedLayout L = seed_layout(n, NA, I.n_lines);
            // per position: new aisles (bits 0-9), the order's aisles (10-19),
            // its size (20-27), in a tour (bit 31)
            uint32_t *st = (uint32_t *)(smem + L.st);
            uint32_t *aend = (uint32_t *)(smem + L.aend);  // end of each aisle's list of positions
            uint32_t *tbits = (uint32_t *)(smem + L.tbits);
            uint16_t *apos = (uint16_t *)(smem + L.apos);
            const uint32_t *oo = A.ordoff + I.ordoff_off;
            const uint32_t *orr = A.ordrec + I.ordrec_off;
            const uint32_t magic = I.magic;
            auto aisle_of = [&](uint32_t rec) { return mulhi24(rec + zs[rec >> 26], magic); };
            // each distinct aisle of order o's lines, once
            auto for_aisles = [&](uint32_t o, auto f) {
                const uint32_t l0 = oo[o], l1 = oo[o + 1];
                for (uint32_t l = l0; l < l1; l++) {
                    const uint32_t a = aisle_of(orr[l]);
                    bool dup = false;
                    for (uint32_t m = l0; m < l && !dup; m++) dup = aisle_of(orr[m]) == a;
                    if (!dup) f(a);
                }
            };
            for (int a = lane; a < NA; a += 64) aend[a] = 0u;
            __syncthreads();
            // per position: the order's size and aisle count; per aisle: its orders
            for (int q = lane; q < n; q += 64) {
                const uint32_t o = min((uint32_t)seq[q], (uint32_t)(n - 1));
                uint32_t k = 0;
                for_aisles(o, [&](uint32_t a) {
                    k++;
                    atomicAdd(&aend[a], 1u);
                });
                st[q] = k | (k << 10) | ((uint32_t)cnt[o] << 20);
            }
            __syncthreads();
            {
                uint32_t carry = 0;                          // starts of the lists (exclusive scan)
                for (int a0 = 0; a0 < NA; a0 += 64) {
                    const int a = a0 + lane;
                    const uint32_t c = a < NA ? aend[a] : 0u;
                    const uint32_t inc = wave_incl_scan(c) + carry;
                    if (a < NA) aend[a] = inc - c;
                    carry = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
                }
            }
            __syncthreads();
            for (int q = lane; q < n; q += 64) {               // each start advances to its list's end
                const uint32_t o = min((uint32_t)seq[q], (uint32_t)(n - 1));
                // (a malformed sequence, with an order twice, could hold more
                // entries than the table: they are dropped)
                for_aisles(o, [&](uint32_t a) {
                    const uint32_t e = atomicAdd(&aend[a], 1u);
                    if (e < (uint32_t)I.n_lines) apos[e] = (uint16_t)q;
                });
            }
            __syncthreads();
            int next = 0;                                    // positions before it are all in tours (uniform)
            for (;;) {
                // the seed: the earliest position in no tour
                int s = -1;
                for (int b = next; b < n; b += 64) {
                    const uint64_t m = __ballot(b + lane < n && !(st[min(b + lane, n - 1)] >> 31));
                    if (m) {
                        s = b + (int)__builtin_ctzll(m);
                        break;
                    }
                }
                if (s < 0) break;
                next = s;
                // a new tour: every aisle of every later order is new to it
                // (four consecutive positions per lane and access)
                for (int r0 = next & ~3; r0 < n; r0 += 256) {
                    const int i0 = r0 + 4 * lane;
                    if (i0 + 4 <= n) {
                        uint4 w = *(const uint4 *)(st + i0);
                        w.x = (w.x & ~0x3FFu) | ((w.x >> 10) & 0x3FFu);
                        w.y = (w.y & ~0x3FFu) | ((w.y >> 10) & 0x3FFu);
                        w.z = (w.z & ~0x3FFu) | ((w.z >> 10) & 0x3FFu);
                        w.w = (w.w & ~0x3FFu) | ((w.w >> 10) & 0x3FFu);
                        *(uint4 *)(st + i0) = w;
                    } else {
                        for (int q = i0; q < n; q++) st[q] = (st[q] & ~0x3FFu) | ((st[q] >> 10) & 0x3FFu);
                    }
                }
                for (int w = lane; w < (NA + 31) / 32; w += 64) tbits[w] = 0u;
                __syncthreads();
                uint32_t load = 0;
                int q = s;                                   // the order joining the tour (uniform)
                for (;;) {
                    const uint32_t o = min((uint32_t)seq[q], (uint32_t)(n - 1));
                    if (lane == 0) {
                        st[q] |= 1u << 31;
                        tour_of[o] = (uint16_t)T;
                    }
                    load += (st[q] >> 20) & 0xFFu;
                    // each aisle it adds: every order visiting that aisle has
                    // one new aisle fewer.  The order's lines, 64 at a time,
                    // one per lane; a line counts if no earlier line of the
                    // order has its aisle and the tour does not visit it yet.
                    const uint32_t l0 = oo[o], l1 = oo[o + 1];
                    for (uint32_t c0 = l0; c0 < l1; c0 += 64) {
                        const uint32_t l = c0 + lane;
                        const uint32_t a = l < l1 ? aisle_of(orr[l]) : 0xFFFFFFFFu;
                        bool fresh = l < l1 && !((tbits[min(a, (uint32_t)NA - 1u) >> 5] >> (a & 31u)) & 1u);
                        const uint32_t m_c = min(64u, l1 - c0);
                        for (uint32_t i = 0; i < m_c; i++)           // earlier lines of this chunk
                            fresh = fresh && !(i < (uint32_t)lane && (uint32_t)__builtin_amdgcn_readlane((int)a, (int)i) == a);
                        for (uint32_t m = l0; m < c0 && fresh; m++)  // earlier chunks (orders of more than 64 lines)
                            fresh = aisle_of(orr[m]) != a;
                        uint64_t nm = __ballot(fresh);
                        while (nm) {
                            const int j = (int)__builtin_ctzll(nm);
                            nm &= nm - 1ull;
                            const uint32_t aj = (uint32_t)__builtin_amdgcn_readlane((int)a, j);
                            if (lane == 0) tbits[aj >> 5] |= 1u << (aj & 31u);
                            const uint32_t e1 = min(aend[aj], (uint32_t)I.n_lines);
                            for (uint32_t e = (aj ? aend[aj - 1] : 0u) + lane; e < e1; e += 64) {
                                const uint32_t r = apos[e];
                                if ((int)r >= next && (int)r < n) atomicSub(&st[r], 1u);
                            }
                        }
                    }
                    __syncthreads();
                    // the order that fits with the fewest new aisles, the earliest of them
                    // (four consecutive positions per lane and read, branch-free;
                    // positions before `next` are all in tours)
                    uint32_t best = 0xFFFFFFFFu;
                    for (int r0 = next & ~3; r0 < n; r0 += 256) {
                        const int i0 = r0 + 4 * lane;
                        const uint4 w4 = i0 < n ? *(const uint4 *)(st + i0) : make_uint4(~0u, ~0u, ~0u, ~0u);
                        const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                        for (int u = 0; u < 4; u++) {
                            const uint32_t i = (uint32_t)(i0 + u);
                            const bool ok = i < (uint32_t)n && (int32_t)w[u] >= 0 &&
                                            load + ((w[u] >> 20) & 0xFFu) <= (uint32_t)Q;
                            best = min(best, ok ? (((w[u] & 0x3FFu) << 16) | i) : 0xFFFFFFFFu);
                        }
                    }
                    best = wave_min_u32(best);
                    if (best == 0xFFFFFFFFu) break;
                    q = (int)(best & 0xFFFFu);
                }
                T++;
            }
        } else {
            // ---- 2. first fit -------------------------------------------------
            const uint32_t mins = (uint32_t)__builtin_amdgcn_readfirstlane(I.min_size);   // a room below it never takes an order
            // Lanes [0, k) hold tours in opening order with their rooms, lanes
            // past k room 0.  A tour whose room falls below mins stays in its
            // lane until the lanes run out (no order fits it, so a ballot never
            // picks it); open tours opened after the lanes' wait in the queue
            // [qh, qt), in order, whenever it is not empty.
            int k = 0;                                      // uniform
            uint32_t room = 0, tour = 0;
            uint32_t *queue = A.ff_queue + (int64_t)blockIdx.x * A.ff_stride;
            int qh = 0, qt = 0;                             // uniform
            // the full tours leave the lanes (the others move down, in order),
            // then the freed lanes take the queue's open tours, in order
            auto compact = [&]() {
                const uint64_t live = __ballot(room >= mins);
                const uint32_t nlive = (uint32_t)__builtin_popcountll(live);
                const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(live >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)live, 0u));
                // a permutation: open tours to lanes [0, nlive), the rest after them
                const uint32_t dst = ((live >> lane) & 1ull) ? below : nlive + (uint32_t)lane - below;
                const uint32_t rr = (uint32_t)__builtin_amdgcn_ds_permute((int)(dst << 2), (int)room);
                const uint32_t tt = (uint32_t)__builtin_amdgcn_ds_permute((int)(dst << 2), (int)tour);
                room = (uint32_t)lane < nlive ? rr : 0u;
                tour = tt;
                k = (int)nlive;
                while (k < 64 && qh < qt) {
                    const uint32_t e = qh + lane < qt ? queue[qh + lane] : 0u;
                    uint64_t lv = __ballot((e >> 16) >= mins);
                    int taken = 0;
                    while (lv && k < 64) {
                        const int f = __builtin_ctzll(lv);
                        const uint32_t ef = (uint32_t)__builtin_amdgcn_readlane((int)e, f);
                        room = set_lane(room, ef >> 16, k);
                        tour = set_lane(tour, ef & 0xFFFFu, k);
                        k++;
                        taken = f + 1;
                        lv &= lv - 1ull;
                    }
                    qh = k < 64 ? min(qh + 64, qt) : qh + taken;
                }
            };
            for (int i0 = 0; i0 < n; i0 += 64) {
                const int i = i0 + lane;
                const uint32_t o_l = i < n ? min((uint32_t)seq[i], (uint32_t)n) : (uint32_t)n;
                // min(size, Q + 1); an id out of range (a malformed row, whose
                // result is unspecified) counts as one item and is left out below
                const uint32_t s_l = max((uint32_t)cnt[o_l], 1u);
                const int m = __builtin_amdgcn_readfirstlane(min(64, n - i0));   // uniform: a scalar loop bound
                uint32_t t_l = 0;                               // lane j: tour of position i0 + j
    #pragma unroll 2
                for (int j = 0; j < m; j++) {
                    const uint32_t sz = (uint32_t)__builtin_amdgcn_readlane((int)s_l, j);
                    // no order (of at least one item) fits room 0 or a room below mins
                    const uint64_t hit = __ballot(room >= sz);
                    uint32_t t = 0;
                    if (hit) {                                   // the earliest tour in the lanes with room
                        const int f = __builtin_ctzll(hit);
                        t = (uint32_t)__builtin_amdgcn_readlane((int)tour, f);
                        room = set_lane(room, (uint32_t)__builtin_amdgcn_readlane((int)room, f) - sz, f);
                    } else {
                        bool found = false;
                        // the queued tours, in order, 64 at a time
                        for (int b = qh; b < qt && !found; b += 64) {
                            const uint32_t e = b + lane < qt ? queue[b + lane] : 0u;
                            const uint64_t h = __ballot((e >> 16) >= sz);
                            if (h) {
                                const int f = __builtin_ctzll(h);
                                const uint32_t ef = (uint32_t)__builtin_amdgcn_readlane((int)e, f);
                                t = ef & 0xFFFFu;
                                if (lane == 0) queue[b + f] = (((ef >> 16) - sz) << 16) | t;
                                found = true;
                            }
                        }
                        if (!found) {                            // no open tour has room: a new one
                            t = (uint32_t)T++;
                            const uint32_t r0 = sz <= (uint32_t)Q ? (uint32_t)Q - sz : 0u;   // a larger order rides alone
                            if (r0 >= mins) {
                                if (k == 64) compact();
                                if (k < 64 && qh == qt) {
                                    room = set_lane(room, r0, k);
                                    tour = set_lane(tour, t, k);
                                    k++;
                                } else {
                                    if (lane == 0) queue[qt] = (r0 << 16) | t;
                                    qt++;
                                }
                            }
                        }
                        __threadfence_block();                   // queue stores before later loads of them
                    }
                    t_l = set_lane(t_l, t, j);
                }
                // read after the tile loop's barrier
                if (i < n && o_l < (uint32_t)n) tour_of[o_l] = (uint16_t)t_l;
            }
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
                    const uint32_t np = rw[0];
                    if (np == 0) continue;                  // only a malformed row leaves a tour empty
                    if (np > (uint32_t)I.pick_slots) continue;   // an order routed apart (below)
                    uint32_t v[MAX_PICK_SLOTS];
#pragma unroll
                    for (int i = 0; i < MAX_PICK_SLOTS; i++) v[i] = (uint32_t)i < np ? rw[1 + i] : 0xFFFFFFFFu;
                    sort32(v);
                    acc += pick_route_cost<ROUTE>(v, np, wsp, I, I.magic);
                }
            }
            __syncthreads();
        }
        // orders longer than a pick row, each a tour of its own
        if (ROUTE != WO_ROUTE_SSHAPE && I.n_big > 0) acc += big_orders_cost<ROUTE, 64>(A, I, zs, rows, wsp);

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

template <int ROUTE, bool SEED>
static hipError_t launch_eval_ff_r(const EvalArgs &a, uint32_t lds_bytes, int grid, hipStream_t s)
{
    static uint32_t attr_bytes = 0;
    if (lds_bytes > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)eval_ff_kernel<ROUTE, SEED>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        attr_bytes = lds_bytes;
    }
    hipLaunchKernelGGL((eval_ff_kernel<ROUTE, SEED>), dim3(grid), dim3(64), lds_bytes, s, a);
    return hipGetLastError();
}

template <bool SEED>
static hipError_t launch_eval_ff_s(const EvalArgs &a, uint32_t lds_bytes, int grid, int route, hipStream_t s)
{
    switch (route) {
    case WO_ROUTE_SSHAPE: return launch_eval_ff_r<WO_ROUTE_SSHAPE, SEED>(a, lds_bytes, grid, s);
    case WO_ROUTE_RETURN: return launch_eval_ff_r<WO_ROUTE_RETURN, SEED>(a, lds_bytes, grid, s);
    case WO_ROUTE_LARGEST_GAP: return launch_eval_ff_r<WO_ROUTE_LARGEST_GAP, SEED>(a, lds_bytes, grid, s);
    case WO_ROUTE_OPTIMAL: return launch_eval_ff_r<WO_ROUTE_OPTIMAL, SEED>(a, lds_bytes, grid, s);
    case WO_ROUTE_COMBINED: return launch_eval_ff_r<WO_ROUTE_COMBINED, SEED>(a, lds_bytes, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_eval_ff(const EvalArgs &a, uint32_t lds_bytes, int grid, int route, bool seed, hipStream_t s)
{
    return seed ? launch_eval_ff_s<true>(a, lds_bytes, grid, route, s)
                : launch_eval_ff_s<false>(a, lds_bytes, grid, route, s);
}

template <int ROUTE, bool SEED>
static int ff_max_blocks_r(uint32_t lds_bytes)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, eval_ff_kernel<ROUTE, SEED>, 64, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

template <bool SEED>
static int ff_max_blocks_s(int route, uint32_t lds_bytes)
{
    switch (route) {
    case WO_ROUTE_RETURN: return ff_max_blocks_r<WO_ROUTE_RETURN, SEED>(lds_bytes);
    case WO_ROUTE_LARGEST_GAP: return ff_max_blocks_r<WO_ROUTE_LARGEST_GAP, SEED>(lds_bytes);
    case WO_ROUTE_OPTIMAL: return ff_max_blocks_r<WO_ROUTE_OPTIMAL, SEED>(lds_bytes);
    case WO_ROUTE_COMBINED: return ff_max_blocks_r<WO_ROUTE_COMBINED, SEED>(lds_bytes);
    }
    return ff_max_blocks_r<WO_ROUTE_SSHAPE, SEED>(lds_bytes);
}

int eval_ff_max_blocks_per_cu(int route, bool seed, uint32_t lds_bytes)
{
    return seed ? ff_max_blocks_s<true>(route, lds_bytes) : ff_max_blocks_s<false>(route, lds_bytes);
}

}  // namespace wo
