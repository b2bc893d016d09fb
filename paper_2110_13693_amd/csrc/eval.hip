// Exact plan evaluation on gfx950: slot map, next-fit tours, S-shape distance,
// time-window throughput (arXiv 2110.13693, section 5, Subproblems 2 and 3,
// Eq. (2); section 6).  One workgroup evaluates one plan at a time and walks
// the plans with a grid stride; several workgroups share a CU so that one's
// latency-bound phases overlap the others' work.
//
// Per plan:
//   1. zone starts: start[c] = sum of the sizes of categories placed in a
//      lower zone; kept in LDS pre-shifted so that a line's scaled location
//      is one add: ls = rec + zs[rec >> 26];
//   2. a bitmap B over "units" of the sequence: bit P[i] is set where the
//      i-th order of the sequence starts, P being the prefix sum of the order
//      sizes clamped to Q + 1 (an order larger than Q is a tour of its own
//      whatever its exact size), plus a sentinel bit at the total;
//   3. next-fit: a tour opened at unit x ends after the last order that
//      starts within (x, x + Q]; so the next tour opens at
//      E(x) = highest set bit of B in (x, x + Q] (a 64-bit window of B).
//      Tours open on the orbit of 0 under E.  The orbit is found in
//      parallel: the unit range is cut into segments, and for each segment
//      every order start that can be the first tour opened in it (those
//      within Q units of its start) is chased to the segment end; the true
//      entries are then linked segment after segment;
//   4. tour ids: the rank of each opening position among the order starts is
//      the sequence position of the tour's first order; a block scan over
//      these flags gives every order its tour id;
//   5. every order line (in instance order, coalesced) sets its aisle bit in
//      its tour's aisle set (ds_or) and raises its tour's farthest location
//      (ds_max) -- the largest location of a tour is, at once, the last
//      aisle visited and the farthest depth in it;
//   6. per tour: k = popcount of the aisle set, S-shape closed form; the
//      block sums the tours in int64.
#include "wo_internal.h"

namespace wo {

static __device__ __forceinline__ uint32_t mulhi24(uint32_t x, uint32_t m)
{
    return (uint32_t)(((uint64_t)(x & 0xFFFFFFu) * (uint64_t)(m & 0xFFFFFFu)) >> 32);
}

static __device__ __forceinline__ uint32_t ffbh(uint32_t x)   // leading zeros, 32 for 0
{
    return x ? (uint32_t)__builtin_clz(x) : 32u;
}

template <int BLOCK>
static __device__ __forceinline__ int block_excl_scan(int v, int *scratch, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) scratch[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / 64; i++) {
        int s = scratch[i];
        off += (i < w) ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

template <int BLOCK>
static __device__ __forceinline__ int64_t block_sum64(int64_t v, int64_t *scratch)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / 64; i++) t += scratch[i];
    __syncthreads();
    return t;
}

static __device__ __forceinline__ float window_throughput(int64_t D, const InstDev &I)
{
    // T = D / walk + t_item * items; orders * window / T, IEEE double, no contraction
    double T = __dadd_rn(__ddiv_rn((double)D, I.walk), __dmul_rn(I.t_item, (double)I.n_lines));
    double r = __ddiv_rn(__dmul_rn((double)I.n_orders, I.window), T);
    return __double2float_rn(r);
}

// Bits [x, x + 32) of bitmap B (B holds at least (x >> 5) + 2 words).
static __device__ __forceinline__ uint32_t bits_at(const uint32_t *B, uint32_t x)
{
    const uint32_t w = x >> 5;
    return __builtin_amdgcn_alignbit(B[w + 1], B[w], x & 31u);
}

// Next tour opening after a tour opened at unit x (no order larger than Q).
static __device__ __forceinline__ uint32_t next_open(const uint32_t *B, uint32_t x, uint32_t maskQ)
{
    const uint32_t win = bits_at(B, x + 1) & maskQ;
    return x + 32u - ffbh(win);        // x + 1 + highest set bit
}

// Number of order starts below unit x = sequence position of the order at x.
static __device__ __forceinline__ uint32_t rank_of(const uint32_t *B, const uint32_t *prefB, uint32_t x)
{
    const uint32_t w = x >> 5;
    return prefB[w] + __popc(B[w] & ((1u << (x & 31u)) - 1u));
}

// Bits [lo, hi) of bitmap F, counted.
static __device__ __forceinline__ int count_range(const uint32_t *F, int lo, int hi)
{
    int c = 0;
    while (lo < hi) {
        const int w = lo >> 5;
        const int lim = min(hi, (w + 1) << 5);
        const int len = lim - lo;
        const uint32_t m = (len == 32 ? 0xFFFFFFFFu : ((1u << len) - 1u)) << (lo & 31);
        c += __popc(F[w] & m);
        lo = lim;
    }
    return c;
}

// Instance of plan row p: the last one whose first row is <= p.
static __device__ __forceinline__ int instance_of(const EvalArgs &A, int64_t p)
{
    if (A.n_inst <= 1) return 0;
    int lo = 0, hi = A.n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.plan_begin[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void eval_plans_kernel(EvalArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_next;
    constexpr int SEQ_CHUNK = 4096 / BLOCK;  // sequence positions per thread kept in registers
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    int loaded = -1;                        // instance whose count table sits in LDS

    // work items: a grid stride, or a queue (atomic ticket) over a work order
    // that puts the most expensive plans first
    int64_t item = blockIdx.x;
    if (A.queue) {
        if (tid == 0) s_next = atomicAdd(A.queue_ctr, 1u);
        __syncthreads();
        item = s_next;
        __syncthreads();
    }
    // the next plan's sequence chunk and zone row, loaded while the current
    // plan's line pass runs
    bool have_pf = false;                   // uniform
    uint32_t sv_pf[SEQ_CHUNK / 2];          // two 16-bit order ids per register
    uint32_t zc_pf = 0xFFu;
    while (item < A.n_plans) {
        if (A.queue && tid == 0) s_next = atomicAdd(A.queue_ctr, 1u);   // ticket of the next plan
        const int64_t p = A.work ? (int64_t)A.work[item] : item;
        const int ii = instance_of(A, p);
        const InstDev &I = A.inst[ii];
        const int n = I.n_orders;
        const int C = I.n_cat;
        const uint32_t Q = (uint32_t)I.capacity;
        const uint32_t maskQ = Q >= 32u ? 0xFFFFFFFFu : ((1u << Q) - 1u);
        const uint32_t n_units = (uint32_t)I.n_units;
        const int64_t row = p - (A.n_inst > 1 ? A.plan_begin[ii] : 0);
        const uint16_t *seq = A.seq + A.seq_base[ii] + row * (int64_t)n;
        const uint2 *lines = A.lines + I.line_off;
        const EvalLayout Ly = eval_layout(n, I.n_units, I.words, I.t_cap);
        uint32_t *zs = (uint32_t *)(smem + Ly.zs);
        int64_t *red = (int64_t *)(smem + Ly.red);
        int *misc = (int *)(smem + Ly.misc);
        uint32_t *lane_base = (uint32_t *)(smem + Ly.seg);
        uint32_t *wbits = lane_base + (MAX_SEG + 1);
        uint32_t *true_lane = wbits + (MAX_SEG + 1);
        uint32_t *segs = true_lane + (MAX_SEG + 1);
        uint8_t *cnt = (uint8_t *)(smem + Ly.cnt);
        uint32_t *F = (uint32_t *)(smem + Ly.F);
        uint16_t *tour = (uint16_t *)(smem + Ly.tour);
        uint32_t *B = (uint32_t *)(smem + Ly.B);
        uint32_t *prefB = (uint32_t *)(smem + Ly.prefB);
        uint16_t *crec = (uint16_t *)(smem + Ly.rec);
        uint32_t *cnrec = (uint32_t *)(smem + Ly.nrec);
        uint32_t *cnxt = (uint32_t *)(smem + Ly.nxt);
        uint32_t *mask = (uint32_t *)(smem + Ly.mask);
        uint32_t *mx = (uint32_t *)(smem + Ly.mx);
        const uint32_t nB = bitmap_words(I.n_units);
        const int nF = (n + 31) / 32 + 1;
        int bad = 0;

        // ---- staging: count table, cleared bitmaps ------------------------
        if (ii != loaded) {
            const uint4 *src = (const uint4 *)(A.cnt + I.cnt_off);
            uint4 *dst = (uint4 *)cnt;
            for (int k = tid; k < (n + 15) / 16; k += BLOCK) dst[k] = src[k];
            loaded = ii;
        }
        for (uint32_t w = tid; w < nB; w += BLOCK) B[w] = 0;
        for (int w = tid; w < nF; w += BLOCK) F[w] = 0;
        if (tid < 16) misc[tid] = 0;

        // ---- 1. zone starts (wave 0) -------------------------------------
        if (tid < 64) {
            const uint32_t zc = have_pf ? zc_pf : ((lane < C) ? (uint32_t)A.zone_of[p * 64 + lane] : 0xFFu);
            const uint32_t sz = (lane < C) ? (uint32_t)I.cat_size[lane] : 0u;
            uint32_t start = 0;
            for (int c2 = 0; c2 < C; c2++) {
                const uint32_t z2 = (uint32_t)__builtin_amdgcn_readlane((int)zc, c2);
                const uint32_t s2 = (uint32_t)__builtin_amdgcn_readlane((int)sz, c2);
                start += (z2 < zc) ? s2 : 0u;
            }
            zs[lane] = (start << I.shift) - ((uint32_t)(4 * lane) << 24);
            if (A.validate) {
                uint64_t m = (lane < C && zc < 64u) ? (1ull << zc) : 0ull;
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) m |= __shfl_xor(m, d, 64);
                const uint64_t want = (C == 64) ? ~0ull : ((1ull << C) - 1ull);
                if (lane == 0 && m != want) bad = 1;
            }
        }

        // ---- 2. unit bitmap of order starts --------------------------------
        const int ch = (n + BLOCK - 1) / BLOCK;
        const int b0 = min(n, tid * ch), b1 = min(n, b0 + ch);
        const bool one_piece = ch <= SEQ_CHUNK;          // uniform
        uint32_t svp[SEQ_CHUNK / 2];                    // the chunk's order ids, two per register
        if (one_piece) {
#pragma unroll
            for (int k = 0; k < SEQ_CHUNK; k++) {
                const int i = b0 + k;
                uint32_t o = (i < b1) ? (have_pf ? ((sv_pf[k >> 1] >> (16 * (k & 1))) & 0xFFFFu) : (uint32_t)seq[i]) : 0u;
                if (o >= (uint32_t)n) { bad = 1; o = (uint32_t)(n - 1); }
                if (k & 1) svp[k >> 1] |= o << 16; else svp[k >> 1] = o;
            }
        }
#define SV(k) ((svp[(k) >> 1] >> (16 * ((k) & 1))) & 0xFFFFu)
        __syncthreads();                                 // count table, zeroed bitmaps
        const int64_t next_item = A.queue ? (int64_t)s_next : item + (int64_t)gridDim.x;
        int local = 0, big = 0;
        if (one_piece) {
#pragma unroll
            for (int k = 0; k < SEQ_CHUNK; k++) {
                if (b0 + k < b1) {
                    const int c = cnt[SV(k)];
                    local += c;
                    big |= c > (int)Q;
                }
            }
        } else {
            for (int i = b0; i < b1; i++) {
                uint32_t o = seq[i];
                if (o >= (uint32_t)n) { bad = 1; o = (uint32_t)(n - 1); }
                const int c = cnt[o];
                local += c;
                big |= c > (int)Q;
            }
        }
        int total_units;
        uint32_t run = (uint32_t)block_excl_scan<BLOCK>(local, (int *)red, &total_units);
        {
            uint32_t cur = run >> 5, acc = 0;
            if (one_piece) {
#pragma unroll
                for (int k = 0; k < SEQ_CHUNK; k++) {
                    if (b0 + k < b1) {
                        const uint32_t w = run >> 5;
                        if (w != cur) { atomicOr(&B[cur], acc); acc = 0; cur = w; }
                        acc |= 1u << (run & 31u);
                        run += cnt[SV(k)];
                    }
                }
            } else {
                for (int i = b0; i < b1; i++) {
                    uint32_t o = seq[i];
                    if (o >= (uint32_t)n) o = (uint32_t)(n - 1);
                    const uint32_t w = run >> 5;
                    if (w != cur) { atomicOr(&B[cur], acc); acc = 0; cur = w; }
                    acc |= 1u << (run & 31u);
                    run += cnt[o];
                }
            }
            if (acc) atomicOr(&B[cur], acc);
        }
        if (tid == 0) atomicOr(&B[n_units >> 5], 1u << (n_units & 31u));   // sentinel
        if (big) misc[0] = 1;
        if (A.validate) {
            // permutation check: mark every order once (bitmap in the region)
            uint32_t *seen = (uint32_t *)(smem + Ly.region);
            for (int w = tid; w < (n + 31) / 32; w += BLOCK) seen[w] = 0;
            __syncthreads();
            for (int i = tid; i < n; i += BLOCK) {
                const uint32_t o = seq[i];
                if (o >= (uint32_t)n) continue;
                const uint32_t old = atomicOr(&seen[o >> 5], 1u << (o & 31));
                if (old & (1u << (o & 31))) bad = 1;
            }
        }
        __syncthreads();
        {   // prefix popcounts of B (word granularity)
            const int wch = ((int)nB + BLOCK - 1) / BLOCK;
            const int w0 = min((int)nB, tid * wch), w1 = min((int)nB, w0 + wch);
            int c = 0;
            for (int w = w0; w < w1; w++) c += __popc(B[w]);
            int tot;
            int r = block_excl_scan<BLOCK>(c, (int *)red, &tot);
            for (int w = w0; w < w1; w++) {
                prefB[w] = (uint32_t)r;
                r += __popc(B[w]);
            }
        }

        // ---- 3. segments and their candidate entries (wave 0) ------------
        int G = (misc[0] || I.n_seg <= 1) ? 1 : I.n_seg;   // uniform
        if (G > 1 && tid < 64) {
            const int g = lane;
            const uint32_t s_g = (uint32_t)(((uint64_t)g * n_units) / (uint32_t)G);
            uint32_t c = 0, wb = 0;
            if (g == 0) {
                c = 1;
            } else if (g < G) {
                const uint32_t lim = n_units - s_g;   // candidates are order starts < n_units
                wb = bits_at(B, s_g) & maskQ;
                if (lim < 32u) wb &= (1u << lim) - 1u;
                c = __popc(wb);
            }
            uint32_t inc = c;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t t = __shfl_up(inc, d, 64);
                if (lane >= d) inc += t;
            }
            lane_base[g] = inc - c;
            wbits[g] = wb;
            segs[g] = g <= G ? s_g : n_units;
            if (g == 63) misc[1] = (int)inc;          // total chase lanes
        }
        if (G > 1 && tid == 0) segs[G] = n_units;
        __syncthreads();
        if (G > 1 && misc[1] > CHASE_LANES) G = 1;    // uniform

        // ---- 4. chase ------------------------------------------------------
        if (G > 1) {
            const int L_tot = misc[1];
            for (int l = tid; l < L_tot; l += BLOCK) {
                int lo = 0, hi = G - 1;                  // segment of lane l
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((int)lane_base[mid] <= l) lo = mid; else hi = mid - 1;
                }
                const int g = lo;
                const uint32_t s_g = segs[g];
                const uint32_t s_e = segs[g + 1];
                uint32_t x = s_g;
                if (g > 0) {
                    uint32_t wb = wbits[g];
                    for (int k = l - (int)lane_base[g]; k > 0; k--) wb &= wb - 1u;
                    x = s_g + (uint32_t)__builtin_ctz(wb);
                }
                uint16_t *r = crec + l * CHASE_RECS;
                uint32_t nr = 0;
                r[nr++] = (uint16_t)(x - s_g);
                for (;;) {
                    x = next_open(B, x, maskQ);
                    if (x >= s_e) break;
                    if (nr == CHASE_RECS) { misc[2] = 1; break; }
                    r[nr++] = (uint16_t)(x - s_g);
                }
                cnrec[l] = nr;
                // the lane of the next segment whose candidate is this exit
                uint32_t nx = 0xFFFFFFFFu;
                if (g + 1 < G) {
                    const uint32_t off = x - s_e;
                    const uint32_t wb = wbits[g + 1];
                    if (off < 32u && ((wb >> off) & 1u))
                        nx = lane_base[g + 1] + __popc(wb & ((1u << off) - 1u));
                }
                cnxt[l] = nx;
            }
            __syncthreads();
            // ---- link the true entries, segment after segment ------------
            if (tid == 0 && !misc[2]) {
                uint32_t l = 0;
                for (int g = 0; g < G; g++) {
                    true_lane[g] = l;
                    if (g + 1 < G) {
                        l = cnxt[l];
                        if (l == 0xFFFFFFFFu) { misc[2] = 1; break; }
                    }
                }
            }
            __syncthreads();
            if (!misc[2]) {
                for (int idx = tid; idx < G * CHASE_RECS; idx += BLOCK) {
                    const int g = idx / CHASE_RECS, k = idx % CHASE_RECS;
                    const uint32_t l = true_lane[g];
                    if ((uint32_t)k < cnrec[l]) {
                        const uint32_t x = segs[g] + crec[l * CHASE_RECS + k];
                        const uint32_t i = rank_of(B, prefB, x);
                        atomicOr(&F[i >> 5], 1u << (i & 31u));
                    }
                }
            } else {
                G = 1;                                   // fall back to the serial chain
            }
        }
        if (G == 1) {
            // serial chain (also handles orders larger than the capacity)
            if (tid == 0) {
                uint32_t x = 0;
                while (x < n_units) {
                    const uint32_t i = rank_of(B, prefB, x);
                    F[i >> 5] |= 1u << (i & 31u);
                    const uint32_t win = bits_at(B, x + 1) & maskQ;
                    if (win) {
                        x = x + 32u - ffbh(win);
                    } else {                             // an order larger than Q: its own tour
                        uint32_t y = x + 1;
                        while (!((B[y >> 5] >> (y & 31u)) & 1u)) y++;
                        x = y;
                    }
                }
            }
        }
        __syncthreads();

        // ---- tour id of every order --------------------------------------
        int n_tours;
        int trun = block_excl_scan<BLOCK>(count_range(F, b0, b1), (int *)red, &n_tours) - 1;
        if (one_piece) {
#pragma unroll
            for (int k = 0; k < SEQ_CHUNK; k++) {
                const int i = b0 + k;
                if (i < b1) {
                    trun += (F[i >> 5] >> (i & 31)) & 1u;
                    tour[SV(k)] = (uint16_t)trun;
                }
            }
        } else {
            for (int i = b0; i < b1; i++) {
                uint32_t o = seq[i];
                if (o >= (uint32_t)n) o = (uint32_t)(n - 1);
                trun += (F[i >> 5] >> (i & 31)) & 1u;
                tour[o] = (uint16_t)trun;
            }
        }
        __syncthreads();

        // ---- prefetch of the next plan's inputs ---------------------------
        have_pf = false;
        if (next_item < A.n_plans) {
            const int64_t pn = A.work ? (int64_t)A.work[next_item] : next_item;
            const int iin = instance_of(A, pn);
            const InstDev &In = A.inst[iin];
            const int nn = In.n_orders;
            const int chn = (nn + BLOCK - 1) / BLOCK;
            if (chn <= SEQ_CHUNK) {                      // uniform
                const uint16_t *seqn = A.seq + A.seq_base[iin] + (pn - (A.n_inst > 1 ? A.plan_begin[iin] : 0)) * (int64_t)nn;
                const int c0 = min(nn, tid * chn), c1 = min(nn, c0 + chn);
#pragma unroll
                for (int k = 0; k < SEQ_CHUNK; k += 2) {
                    const uint32_t lo = (c0 + k < c1) ? (uint32_t)seqn[c0 + k] : 0u;
                    const uint32_t hi = (c0 + k + 1 < c1) ? (uint32_t)seqn[c0 + k + 1] : 0u;
                    sv_pf[k >> 1] = lo | (hi << 16);
                }
                zc_pf = (tid < 64 && lane < In.n_cat) ? (uint32_t)A.zone_of[pn * 64 + lane] : 0xFFu;
                have_pf = true;
            }
        }

        // ---- 5./6. aisle sets and S-shape per tour tile ------------------
        const int W = I.words;
        const int T = I.t_cap;
        const uint32_t magic = I.magic;
        const int n_lines = I.n_lines;
        int64_t acc = 0;
        for (int t0 = 0; t0 < n_tours; t0 += T) {
            for (int k = tid; k < W * T; k += BLOCK) mask[k] = 0;
            for (int k = tid; k < T; k += BLOCK) mx[k] = 0;
            __syncthreads();
            if (A.main_mode == 0) {
                // one line per lane, 8 coalesced loads in flight per thread
                constexpr int U = 8;
                for (int q0 = tid; q0 < n_lines; q0 += U * BLOCK) {
                    uint2 v[U];
#pragma unroll
                    for (int u = 0; u < U; u++) {
                        const int q = q0 + u * BLOCK;
                        v[u] = (q < n_lines) ? lines[q] : make_uint2(0u, 0xFFFFFFFFu);
                    }
#pragma unroll
                    for (int u = 0; u < U; u++) {
                        if (v[u].y != 0xFFFFFFFFu) {
                            const uint32_t t = (uint32_t)tour[v[u].y] - (uint32_t)t0;
                            if (t < (uint32_t)T) {
                                const uint32_t r = v[u].x;
                                const uint32_t ls = r + zs[r >> 26];
                                const uint32_t a = mulhi24(ls, magic);
                                atomicOr(&mask[(a >> 5) * T + t], 1u << (a & 31));
                                atomicMax(&mx[t], ls);
                            }
                        }
                    }
                }
            } else {
                // one order per lane: its tour looked up once, its farthest
                // location kept in a register, the zone start of each line
                // taken from the wave's copy of the table by lane permute.
                // The next group's order ids and first 8 line records are
                // loaded while the current group is processed.
                constexpr int PF = 8;
                const int zsv = (int)zs[lane];
                const uint32_t *grec = A.grec + I.grec_off;
                const uint32_t *gbase = A.gbase + I.gbase_off;
                const uint16_t *gord = A.gord + I.gord_off;
                const int gstep = BLOCK / 64;
                int g = tid >> 6;
                uint32_t o_n = 0xFFFFu, b_n = 0, L_n = 0, r_n[PF];
                if (g < I.n_grp) {
                    o_n = gord[g * 64 + lane];
                    b_n = gbase[g];
                    L_n = (gbase[g + 1] - b_n) >> 6;
#pragma unroll
                    for (int u = 0; u < PF; u++) r_n[u] = (uint32_t)u < L_n ? grec[b_n + u * 64 + lane] : 0u;
                }
                while (g < I.n_grp) {
                    const uint32_t o = o_n, b0g = b_n, L = L_n;
                    uint32_t r[PF];
#pragma unroll
                    for (int u = 0; u < PF; u++) r[u] = r_n[u];
                    const int gn = g + gstep;
                    if (gn < I.n_grp) {
                        o_n = gord[gn * 64 + lane];
                        b_n = gbase[gn];
                        L_n = (gbase[gn + 1] - b_n) >> 6;
#pragma unroll
                        for (int u = 0; u < PF; u++) r_n[u] = (uint32_t)u < L_n ? grec[b_n + u * 64 + lane] : 0u;
                    }
                    const uint32_t t = (o != 0xFFFFu) ? (uint32_t)tour[o] - (uint32_t)t0 : 0xFFFFFFFFu;
                    const bool active = t < (uint32_t)T;
                    uint32_t far = 0;
#pragma unroll
                    for (int u = 0; u < PF; u++) {
                        if ((uint32_t)u < L) {
                            const uint32_t ls = r[u] + (uint32_t)__builtin_amdgcn_ds_bpermute((int)(r[u] >> 24), zsv);
                            const uint32_t a = mulhi24(ls, magic);
                            if (active) atomicOr(&mask[(a >> 5) * T + t], 1u << (a & 31));
                            far = max(far, ls);
                        }
                    }
                    for (uint32_t kk = PF; kk < L; kk++) {     // long orders
                        const uint32_t rr = grec[b0g + kk * 64 + lane];
                        const uint32_t ls = rr + (uint32_t)__builtin_amdgcn_ds_bpermute((int)(rr >> 24), zsv);
                        const uint32_t a = mulhi24(ls, magic);
                        if (active) atomicOr(&mask[(a >> 5) * T + t], 1u << (a & 31));
                        far = max(far, ls);
                    }
                    if (active) atomicMax(&mx[t], far);
                    g = gn;
                }
            }
            __syncthreads();
            const int nt = min(T, n_tours - t0);
            for (int t = tid; t < nt; t += BLOCK) {
                int k = 0;
                for (int w = 0; w < W; w++) k += __popc(mask[w * T + t]);
                const uint32_t ls = mx[t];
                const uint32_t a = mulhi24(ls, magic);
                const uint32_t j = (ls - a * I.d_s) >> (I.shift + 1);
                const int64_t y = (int64_t)j * I.pitch + I.pitch / 2;
                int64_t cost = 2ll * I.spacing * a;
                cost += (k & 1) ? (int64_t)(k - 1) * I.L + 2 * y : (int64_t)k * I.L;
                acc += cost;
            }
            __syncthreads();
        }
        const int64_t D = block_sum64<BLOCK>(acc, red);
        if (A.validate && bad) atomicOr(A.err, 1);
        if (tid == 0) {
            A.dist[p] = D > 2147483647ll ? 2147483647 : (int32_t)D;
            if (A.thr) A.thr[p] = window_throughput(D, I);
        }
        __syncthreads();
        item = next_item;
    }
}

// Reset of the work-queue ticket (a kernel, so that it can sit in a graph).
__global__ void reset_ticket_kernel(uint32_t *ctr) { *ctr = 0u; }

template <int BLOCK>
static hipError_t launch_eval_t(const EvalArgs &a, uint32_t lds_bytes, int grid, hipStream_t s)
{
    // raise the dynamic LDS limit to what this launch needs (the kernel also
    // holds a few bytes of static LDS, so the whole 160 KB cannot be asked for)
    static uint32_t attr_bytes = 0;
    if (lds_bytes > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)eval_plans_kernel<BLOCK>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        attr_bytes = lds_bytes;
    }
    if (a.queue) hipLaunchKernelGGL(reset_ticket_kernel, dim3(1), dim3(1), 0, s, a.queue_ctr);
    hipLaunchKernelGGL(eval_plans_kernel<BLOCK>, dim3(grid), dim3(BLOCK), lds_bytes, s, a);
    return hipGetLastError();
}

template <int BLOCK>
static int max_blocks_t(uint32_t lds_bytes)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, eval_plans_kernel<BLOCK>, BLOCK, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

int eval_max_blocks_per_cu(int block, uint32_t lds_bytes)
{
    switch (block) {
    case 128: return max_blocks_t<128>(lds_bytes);
    case 256: return max_blocks_t<256>(lds_bytes);
    case 512: return max_blocks_t<512>(lds_bytes);
    }
    return 1;
}

hipError_t launch_eval(const EvalArgs &a, uint32_t lds_bytes, int grid, int block, hipStream_t s)
{
    switch (block) {
    case 128: return launch_eval_t<128>(a, lds_bytes, grid, s);
    case 256: return launch_eval_t<256>(a, lds_bytes, grid, s);
    case 512: return launch_eval_t<512>(a, lds_bytes, grid, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace wo
