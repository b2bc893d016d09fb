// Exact plan evaluation on gfx950: slot map, next-fit tours, S-shape distance,
// time-window throughput (arXiv 2110.13693, section 5, Subproblems 2 and 3,
// Eq. (2); section 6).  One workgroup evaluates one plan at a time and walks
// the plans with a grid stride (or a ticket queue); several workgroups share a
// CU so that one's latency-bound phases overlap the others' work.
//
// Per plan:
//   1. zone starts: start[c] = sum of the sizes of categories placed in a
//      lower zone -- the sizes are permuted into zone order across the lanes
//      of one wave, scanned, and permuted back; kept in LDS pre-shifted so
//      that a line's scaled location is one add: ls = rec + zs[rec >> 24]
//      (each wave keeps the table in registers and reads it by lane permute);
//   2. a bitmap B over "units" of the sequence: bit P[i] is set where the
//      i-th order of the sequence starts, P being the prefix sum of the order
//      sizes clamped to Q + 1 (an order larger than Q is a tour of its own
//      whatever its exact size), plus a sentinel bit at the total;
//   3. next-fit: a tour opened at unit x ends after the last order that
//      starts within (x, x + Q]; so the next tour opens at
//      E(x) = highest set bit of B in (x, x + Q] (a 32-bit window of B).
//      Tours open on the orbit of 0 under E.  The orbit is found in
//      parallel: the unit range is cut into segments, and for each segment
//      every order start that can be the first tour opened in it (those
//      within Q units of its start) is chased to the segment end; the true
//      entries are then linked segment after segment and their openings
//      marked, by sequence position, in a bitmap P (the position of the
//      order starting at unit x is the count of set bits of B below x);
//   4. tour ids: a thread's opening flags are P at its positions; a block
//      scan over their counts numbers the tours, and every order's entry in
//      the tour table receives the byte offset of its tour's LDS row;
//   5. every order line (instance order, coalesced) sets its aisle bit in
//      its tour's row (ds_or) and raises the row's farthest location
//      (ds_max, once per run of an order's lines) -- the largest location
//      of a tour is, at once, the last aisle visited and the farthest depth
//      in it;
//   6. per tour: k = popcount of the aisle set, S-shape closed form; the
//      block sums the tours in int64.
// Tours beyond one tile of rows are handled in further passes over the lines.
// The return, largest-gap, optimal and combined routes (ROUTE = 1 .. 4)
// share steps 1-4; their rows hold each tour's picks instead (step 5 appends the line's
// scaled location), and step 6 sorts a tour's picks by (aisle, depth) and
// walks them once (eval_device.h).  First-fit batching has a kernel of its
// own (firstfit.hip).
#include "eval_device.h"

namespace wo {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

static __device__ __forceinline__ uint32_t ffbh(uint32_t x)   // leading zeros, 32 for 0
{
    return x ? (uint32_t)__builtin_clz(x) : 32u;
}

// both 16-bit halves of a limited to those of b
static __device__ __forceinline__ uint32_t min_u16x2(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t,
                              __builtin_elementwise_min(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
}

// Exclusive block scan with one barrier.  `slot` holds BLOCK / 64 words and
// must not be reused before the block has passed another barrier.
template <int BLOCK>
static __device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *slot, uint32_t *total)
{
    const uint32_t inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) slot[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / 64; i++) {
        const uint32_t s = slot[i];
        off += (i < w) ? s : 0u;
        tot += s;
    }
    *total = tot;
    return off + inc - v;
}

// Block sum of 64-bit values with one barrier (the wave sums by DPP on the
// two halves, carried by 64-bit adds).
template <int BLOCK>
static __device__ __forceinline__ int64_t block_sum64(int64_t v, int64_t *slot)
{
    uint64_t x = (uint64_t)v;
#define WO_DPP64(ctrl, rmask)                                                                                   \
    x += ((uint64_t)(uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), ctrl, rmask, 0xF, false) \
          << 32) |                                                                                              \
         (uint64_t)(uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, ctrl, rmask, 0xF, false)
    WO_DPP64(0x111, 0xF);
    WO_DPP64(0x112, 0xF);
    WO_DPP64(0x114, 0xF);
    WO_DPP64(0x118, 0xF);
    WO_DPP64(0x142, 0xA);
    WO_DPP64(0x143, 0xC);
#undef WO_DPP64
    if ((threadIdx.x & 63) == 63) slot[threadIdx.x >> 6] = (int64_t)x;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / 64; i++) t += slot[i];
    return t;
}

// LDS by absolute address.  The kernel declares no static LDS, so its dynamic
// LDS starts at address 0 and a layout offset is the address itself; the line
// pass uses these so that a table offset held in a register needs no base add.
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
static __device__ __forceinline__ lds_u32 *lds32(uint32_t a) { return (lds_u32 *)(size_t)a; }
static __device__ __forceinline__ lds_u16 *lds16(uint32_t a) { return (lds_u16 *)(size_t)a; }

// Byte address of the word holding bit x of a bitmap at LDS address base
// (uniform): a shift and one shift-add, which the compiler would otherwise
// turn into shift, mask and add.
static __device__ __forceinline__ uint32_t word_addr(uint32_t base, uint32_t x)
{
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, 2, %2" : "=v"(r) : "v"(x >> 5), "s"(base));
    return r;
}

// Bits [x, x + 32) of bitmap B (B holds at least (x >> 5) + 2 words).
static __device__ __forceinline__ uint32_t bits_at(const uint32_t *B, uint32_t x)
{
    const uint32_t w = x >> 5;
    return __builtin_amdgcn_alignbit(B[w + 1], B[w], x & 31u);
}

// Leading zeros of a word by v_ffbh_u32, which gives all ones for 0.
static __device__ __forceinline__ uint32_t ffbh_raw(uint32_t x)
{
    uint32_t r;
    asm("v_ffbh_u32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// One chase step in terms of y = x + 1, for a tour opened at unit x: the
// next opening E(x) is x + 1 + the highest set bit of the window (x, x + Q]
// of the bitmap at LDS address B, and the result is E(x) + 1.  With no order
// larger than Q the window holds the next order start (or the sentinel); an
// empty window would move y by 33, never back.
static __device__ __forceinline__ uint32_t next_open1(uint32_t B, uint32_t y, uint32_t maskQ)
{
    const uint32_t a = word_addr(B, y);
    const uint32_t win = __builtin_amdgcn_alignbit(*lds32(a + 4u), *lds32(a), y) & maskQ;
    return y + 32u - ffbh_raw(win);
}

// The order ids of sequence positions [0, nv) of `s`, two per 32-bit word.
// A full, 16-byte aligned chunk is loaded as it is and the function returns
// true: the caller clamps it to n - 1 (with min_u16x2) when it uses it, so
// that a prefetch does not wait for its data.  Otherwise the ids are clamped
// here and positions nv .. CH - 1 get the sink id n + 1 (size 0).
template <int CH>
static __device__ __forceinline__ bool load_chunk(const uint16_t *s, int nv, uint32_t n, uint4 *out)
{
    if (nv == CH && (((uintptr_t)s) & 15u) == 0) {
#pragma unroll
        for (int j = 0; j < CH / 8; j++) out[j] = ((const uint4 *)s)[j];
        return true;
    }
    const uint32_t lim = n - 1u, sink = n + 1u;
    uint32_t w[CH / 2];
#pragma unroll
    for (int k = 0; k < CH; k += 2) {
        const uint32_t lo = (k < nv) ? min((uint32_t)s[k], lim) : sink;
        const uint32_t hi = (k + 1 < nv) ? min((uint32_t)s[k + 1], lim) : sink;
        w[k >> 1] = lo | (hi << 16);
    }
#pragma unroll
    for (int j = 0; j < CH / 8; j++) out[j] = make_uint4(w[4 * j], w[4 * j + 1], w[4 * j + 2], w[4 * j + 3]);
    return false;
}

template <int BLOCK, int ROUTE, bool SEQ_PASS>
__global__ __launch_bounds__(BLOCK, ROUTE == WO_ROUTE_SSHAPE ? 4 : 2) void eval_plans_kernel(EvalArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t &s_next = *(uint32_t *)(smem + LDS_TICKET);
    constexpr int SEQ_CHUNK = BLOCK >= 256 ? 4096 / BLOCK : 16;   // sequence positions per thread in registers
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    int loaded = -1;                        // instance whose tables sit in LDS

    // work items: a grid stride, or a queue (atomic ticket) over a work order
    // that puts the most expensive plans first; either hands out chunks of
    // A.chunk consecutive items (a work list keeps an instance's plans
    // together, so a chunk mostly stages its instance once)
    const int64_t seq_base0 = A.seq_base[0];
    const int64_t K = A.chunk;
    int64_t item = (int64_t)blockIdx.x * K;
    if (A.queue) {
        if (tid == 0) s_next = atomicAdd(A.queue_ctr, 1u);
        __syncthreads();
        item = (int64_t)s_next * K;
        __syncthreads();
    }
    // the next plan's sequence chunk and zone row, loaded while the current
    // plan's line pass runs
    bool have_pf = false;                   // uniform
    bool pf_raw = false;                    // sv_pf still needs clamping
    uint4 sv_pf[SEQ_CHUNK / 8];             // two 16-bit order ids per 32-bit word
    uint32_t zc_pf = 0xFFu;
    while (item < A.n_plans) {
        const bool chunk_end = (item + 1) % K == 0;    // uniform
        if (A.queue && chunk_end && tid == 0) s_next = atomicAdd(A.queue_ctr, 1u);   // ticket of the next chunk
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
        const EvalLayout Ly = eval_layout(n, I.n_units, (uint32_t)I.row_b, I.t_cap, I.chase_log2, I.chase_lanes);
        uint32_t *zs = (uint32_t *)(smem + LDS_ZS);
        uint32_t *scan_a = (uint32_t *)(smem + Ly.red);
        uint32_t *scan_b = scan_a + 16;
        int64_t *sum_slot = (int64_t *)(smem + Ly.red + 128);
        int *misc = (int *)(smem + Ly.misc);
        uint32_t *lane_base = (uint32_t *)(smem + Ly.seg);
        uint32_t *wbits = lane_base + (MAX_SEG + 1);
        uint32_t *true_lane = wbits + (MAX_SEG + 1);
        uint32_t *segs = true_lane + (MAX_SEG + 1);
        uint8_t *cnt = (uint8_t *)(smem + Ly.cnt);
        uint16_t *tour = (uint16_t *)(smem + Ly.tour);
        uint32_t *B = (uint32_t *)(smem + Ly.B);
        uint32_t *P = (uint32_t *)(smem + Ly.P);
        uint32_t *pref = (uint32_t *)(smem + Ly.pref);
        uint16_t *crec = (uint16_t *)(smem + Ly.rec);
        uint32_t *cnrec = (uint32_t *)(smem + Ly.nrec);
        uint32_t *cnxt = (uint32_t *)(smem + Ly.nxt);
        uint32_t *cand = (uint32_t *)(smem + Ly.cand);
        const int T = I.t_cap;
        const uint32_t RB = (uint32_t)I.row_b;
        const uint32_t dummy = (uint32_t)T * RB;          // byte offset of the dummy row
        int bad = 0;

        // ---- staging: per-instance tables, cleared bitmaps -----------------
        if (ii != loaded) {
            const uint4 *src = (const uint4 *)(A.cnt + I.cnt_off);
            uint4 *dst = (uint4 *)cnt;
            for (int k = tid; k < (int)(cnt_bytes(n) / 16); k += BLOCK) dst[k] = src[k];
            // every tour entry starts at the dummy row, so that an entry a
            // malformed sequence leaves unwritten still points inside the tile
            for (int k = tid; k < n + 2; k += BLOCK) tour[k] = (uint16_t)dummy;
            if (tid < 64) {
                // segment starts, fixed by the instance's unit total (a plan
                // whose total differs is not evaluated); 32-bit products since
                // the total is below 2^22
                const uint32_t G0 = (uint32_t)max(I.n_seg, 1), nu = n_units;
                segs[lane] = (uint32_t)lane < G0 ? (uint32_t)lane * nu / G0 : nu;
                if (lane == 0) segs[MAX_SEG] = nu;
            }
            loaded = ii;
        }
        {
            uint4 *bf = (uint4 *)B;
            const int nbf = (int)((Ly.total - Ly.B) / 16);
            for (int k = tid; k < nbf; k += BLOCK) bf[k] = make_uint4(0u, 0u, 0u, 0u);
        }
        if (tid < 16) misc[tid] = 0;

        // The phases up to the tour numbering are chains of dependent steps
        // and barriers; the aisle pass is throughput work.  Waves in the
        // former issue first, so that a CU's workgroups in their aisle pass
        // fill the gaps of those in the serial phases rather than delay them.
        __builtin_amdgcn_s_setprio(2);

        // ---- 1. zone starts (wave 0) -------------------------------------
        if (tid < 64) {
            const uint32_t zc = have_pf ? zc_pf : ((lane < C) ? (uint32_t)A.zone_of[p * 64 + lane] : 0xFFu);
            const uint32_t sz = (lane < C) ? (uint32_t)I.cat_size[lane] : 0u;
            // lanes past C send a zero size to their own lane, so a valid row
            // fills every lane exactly once
            const uint32_t zl = (lane < C) ? (zc & 63u) : (uint32_t)lane;
            const uint32_t by_zone = (uint32_t)__builtin_amdgcn_ds_permute((int)(zl << 2), (int)sz);
            const uint32_t incl = wave_incl_scan(by_zone);
            uint32_t start = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(zl << 2), (int)(incl - by_zone));
            // a malformed row cannot move a category off the warehouse
            start = min(start, (uint32_t)I.n_skus - sz);
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
        const int nv = b1 - b0;
        const bool one_piece = ch <= SEQ_CHUNK;          // uniform
        uint32_t svp[SEQ_CHUNK / 2];                    // the chunk's order ids, two per register
        uint32_t csp[SEQ_CHUNK / 4];                    // their clamped sizes (<= 33), four per register
        if (one_piece) {
            bool raw;
            uint4 ld[SEQ_CHUNK / 8];
            if (have_pf) {
                raw = pf_raw;
#pragma unroll
                for (int j = 0; j < SEQ_CHUNK / 8; j++) ld[j] = sv_pf[j];
            } else {
                raw = load_chunk<SEQ_CHUNK>(seq + b0, nv, (uint32_t)n, ld);
            }
#pragma unroll
            for (int j = 0; j < SEQ_CHUNK / 8; j++) {
                svp[4 * j + 0] = ld[j].x;
                svp[4 * j + 1] = ld[j].y;
                svp[4 * j + 2] = ld[j].z;
                svp[4 * j + 3] = ld[j].w;
            }
            if (raw) {
                const uint32_t lim2 = (uint32_t)(n - 1) * 0x10001u;
#pragma unroll
                for (int k = 0; k < SEQ_CHUNK / 2; k++) svp[k] = min_u16x2(svp[k], lim2);
            }
        }
        have_pf = false;
#define SV(k) ((svp[(k) >> 1] >> (16 * ((k) & 1))) & 0xFFFFu)
#define CS(k) ((csp[(k) >> 2] >> (8 * ((k) & 3))) & 0xFFu)
        __syncthreads();                                 // tables, zeroed bitmaps, zone starts
        const int64_t next_item = !chunk_end ? item + 1
                                  : A.queue ? (int64_t)s_next * K
                                            : item + 1 + (int64_t)(gridDim.x - 1) * K;
        uint32_t local = 0, cmax = 0;
        if (one_piece) {
#pragma unroll
            for (int k = 0; k < SEQ_CHUNK; k++) {
                const uint32_t c = cnt[SV(k)];
                if (k % 4 == 0) csp[k / 4] = c; else csp[k / 4] |= c << (8 * (k % 4));
                local += c;
                cmax = max(cmax, c);
            }
        } else {
            for (int i = b0; i < b1; i++) {
                const uint32_t c = cnt[min((uint32_t)seq[i], (uint32_t)(n - 1))];
                local += c;
                cmax = max(cmax, c);
            }
        }
        uint32_t total_units;
        const uint32_t run0 = block_excl_scan<BLOCK>(local, scan_a, &total_units);
        // a malformed sequence can change the unit total; such a plan is not
        // evaluated (its result is unspecified) and no bitmap is written
        const bool units_ok = total_units == n_units;   // uniform
        if (A.validate) {
            // permutation check: mark every order once (bitmap in the region)
            uint32_t *seen = (uint32_t *)(smem + LDS_REGION);
            for (int w = tid; w < (n + 31) / 32; w += BLOCK) seen[w] = 0;
            __syncthreads();
            for (int i = tid; i < n; i += BLOCK) {
                const uint32_t o = seq[i];
                if (o >= (uint32_t)n) { bad = 1; continue; }
                const uint32_t old = atomicOr(&seen[o >> 5], 1u << (o & 31));
                if (old & (1u << (o & 31))) bad = 1;
            }
            if (!units_ok) bad = 1;
        }
        int64_t acc = 0;
        if (units_ok) {
            if (one_piece) {
                // positions past the chunk have size 0 and set the next
                // chunk's first bit (or the sentinel) again
                uint32_t run = run0;
#pragma unroll
                for (int k = 0; k < SEQ_CHUNK; k++) {
                    __hip_atomic_fetch_or(lds32(word_addr(Ly.B, run)), 1u << (run & 31u), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
                    run += CS(k);
                }
            } else {
                uint32_t run = run0;
                for (int i = b0; i < b1; i++) {
                    atomicOr(&B[run >> 5], 1u << (run & 31u));
                    run += cnt[min((uint32_t)seq[i], (uint32_t)(n - 1))];
                }
            }
            if (tid == 0) atomicOr(&B[n_units >> 5], 1u << (n_units & 31u));   // sentinel
            if (cmax > Q) misc[0] = 1;
            __syncthreads();

            // order starts per unit word, for the position of an opening unit
            const uint32_t nbw = bitmap_words((int32_t)n_units);
            const uint32_t wpt = (nbw + BLOCK - 1) / BLOCK;
            const uint32_t w0 = min(nbw, (uint32_t)tid * wpt), w1 = min(nbw, w0 + wpt);
            uint32_t pc = 0;
            for (uint32_t w = w0; w < w1; w++) pc += __popc(B[w]);

            // ---- 3. segments and their candidate entries (wave 0) --------
            const bool any_big = misc[0] != 0;         // uniform: an order larger than Q
            int G = (any_big || I.n_seg <= 1) ? 1 : I.n_seg;   // uniform
            if (G > 1 && tid < 64) {
                const int g = lane;
                const uint32_t s_g = segs[g];
                uint32_t wb = 0;
                if (g == 0) {
                    wb = 1u;                          // the tour opened at unit 0
                } else if (g < G) {
                    const uint32_t lim = n_units - s_g;   // candidates are order starts < n_units
                    wb = bits_at(B, s_g) & maskQ;
                    if (lim < 32u) wb &= (1u << lim) - 1u;
                }
                const uint32_t c = __popc(wb);
                const uint32_t inc = wave_incl_scan(c);
                const uint32_t base = inc - c;
                const uint32_t lanes = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
                lane_base[g] = base;
                wbits[g] = wb;
                if (lanes <= (uint32_t)I.chase_lanes) {
                    uint32_t m = wb, idx = base;
                    while (m) {
                        cand[idx++] = ((uint32_t)g << 26) | (s_g + (uint32_t)__builtin_ctz(m));
                        m &= m - 1u;
                    }
                }
                if (g == 0) misc[1] = (int)lanes;
            }
            {
                // the scan's barrier also publishes the segment tables
                uint32_t n_starts;
                uint32_t base = block_excl_scan<BLOCK>(pc, scan_a, &n_starts);
                for (uint32_t w = w0; w < w1; w++) {
                    pref[w] = base;
                    base += __popc(B[w]);
                }
            }
            // position in the sequence of the order that starts at unit x
            auto pos_of = [&](uint32_t x) -> uint32_t {
                const uint32_t w = x >> 5;
                return pref[w] + __popc(B[w] & ~(0xFFFFFFFFu << (x & 31u)));
            };
            if (G > 1 && misc[1] > I.chase_lanes) G = 1;  // uniform

            // ---- 4. chase ---------------------------------------------------
            const int CR2 = I.chase_log2;
            if (G > 1) {
                const int L_tot = misc[1];
                for (int l = tid; l < L_tot; l += BLOCK) {
                    const uint32_t cv = cand[l];
                    const int g = (int)(cv >> 26);
                    uint32_t x = cv & 0x3FFFFFFu;
                    const uint32_t s_g = segs[g];
                    const uint32_t s_e = segs[g + 1];
                    // one loop exit; records past the last slot overwrite it
                    // and send the plan to the serial chain
                    const uint32_t rb = Ly.rec + ((uint32_t)l << (CR2 + 1));
                    const uint32_t rl = rb + (2u << CR2) - 2u;
                    const uint32_t s_g1 = s_g + 1u, s_e1 = s_e + 1u;
                    uint32_t ra = rb, y = x + 1u;
                    do {
                        *lds16(min(ra, rl)) = (uint16_t)(y - s_g1);
                        ra += 2u;
                        y = next_open1(Ly.B, y, maskQ);
                    } while (y < s_e1);
                    x = y - 1u;
                    cnrec[l] = (ra - rb) >> 1;            // more than 2^CR2: records lost
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
                // ---- link the true entries, segment after segment --------
                // (wave 0 holds every chase lane's exit in registers and
                // follows the links with lane reads)
                if (tid < 64 && !misc[2]) {
                    const int L_tot = misc[1];
                    uint32_t c[CHASE_LANES / 64];
#pragma unroll
                    for (int j = 0; j < CHASE_LANES / 64; j++)
                        c[j] = (lane + 64 * j < L_tot) ? cnxt[lane + 64 * j] : 0xFFFFFFFFu;
                    uint32_t l = 0, tl = 0;
                    bool ok = true;
                    for (int g = 0; g < G; g++) {
                        if (lane == g) tl = l;
                        if (g + 1 < G) {
                            const uint32_t j = l >> 6;
                            uint32_t v = c[0];
#pragma unroll
                            for (int jj = 1; jj < CHASE_LANES / 64; jj++) v = (j == (uint32_t)jj) ? c[jj] : v;
                            l = (uint32_t)__builtin_amdgcn_readlane((int)v, (int)(l & 63u));
                            if (l == 0xFFFFFFFFu) { ok = false; break; }
                        }
                    }
                    if (lane < G) true_lane[lane] = tl;
                    // only a true chain's lost records matter
                    const bool lost = lane < G && cnrec[tl] > (1u << CR2);
                    if ((!ok || __ballot(lost) != 0) && lane == 0) misc[2] = 1;
                }
                __syncthreads();
                if (!misc[2]) {
                    for (int idx = tid; idx < (G << CR2); idx += BLOCK) {
                        const int g = idx >> CR2, k = idx & ((1 << CR2) - 1);
                        const uint32_t l = true_lane[g];
                        if ((uint32_t)k < cnrec[l]) {
                            const uint32_t r = pos_of(segs[g] + crec[(l << CR2) + k]);
                            atomicOr(&P[r >> 5], 1u << (r & 31u));
                        }
                    }
                } else {
                    G = 1;                               // fall back to the serial chain
                }
            }
            if (G == 1) {
                // serial chain (also handles orders larger than the capacity)
                __syncthreads();                         // the start counts
                if (tid == 0) {
                    uint32_t x = 0;
                    while (x < n_units) {
                        const uint32_t r = pos_of(x);
                        P[r >> 5] |= 1u << (r & 31u);
                        const uint32_t win = bits_at(B, x + 1) & maskQ;
                        if (win) {
                            x = x + 32u - ffbh(win);
                        } else {                         // an order larger than Q: its own tour
                            uint32_t y = x + 1;
                            while (!((B[y >> 5] >> (y & 31u)) & 1u)) y++;
                            x = y;
                        }
                    }
                }
            }
            __syncthreads();

            // ---- tour ids; tour entries for the first tile -------------------
            uint32_t opm = 0;                            // bit k: position b0 + k opens a tour
            uint32_t n_open = 0;
            if (one_piece) {
                opm = bits_at(P, (uint32_t)b0) & ~(0xFFFFFFFFu << nv);   // nv <= 16
                n_open = __popc(opm);
            } else {
                for (int i = b0; i < b1; i += 32) {
                    const int m = min(32, b1 - i);
                    const uint32_t bits = bits_at(P, (uint32_t)i);
                    n_open += __popc(m == 32 ? bits : bits & ~(0xFFFFFFFFu << m));
                }
            }
            // the rows of the tile are free once the flags are set
            {
                uint4 *rows = (uint4 *)(smem + LDS_REGION);
                const int nr4 = (int)((RB * (uint32_t)(T + 1) + 15u) / 16u);
                for (int k = tid; k < nr4; k += BLOCK) rows[k] = make_uint4(0u, 0u, 0u, 0u);
            }
            uint32_t n_tours;
            const uint32_t first_tour = block_excl_scan<BLOCK>(n_open, scan_b, &n_tours);
            // entry of the order at a position: its tour's row, or the dummy
            // row for tours outside the tile [t0, t0 + T)
            // (later tiles re-derive the tour ids from the sequence in memory)
            auto write_entries = [&](uint32_t t0, bool from_regs) {
                uint32_t t = first_tour - 1u;            // wraps; a store always follows an opening
                if (from_regs) {                         // first tile (t0 = 0): the row offset
                    uint32_t tr = t * RB;                // t * RB, below dummy = T * RB iff t < T
#pragma unroll
                    for (int k = 0; k < SEQ_CHUNK; k++) {
                        tr += ((opm >> k) & 1u) * RB;
                        tour[SV(k)] = (uint16_t)min(tr, dummy);
                    }
                } else {
                    for (int i = b0; i < b1; i++) {
                        const uint32_t o = min((uint32_t)seq[i], (uint32_t)(n - 1));
                        t += (P[i >> 5] >> (i & 31)) & 1u;
                        const uint32_t rel = t - t0;
                        tour[o] = (uint16_t)(rel < (uint32_t)T ? rel * RB : dummy);
                    }
                }
            };
            // line pass in sequence order: every unit is a line (no order
            // larger than Q); tours come from the openings counted per word
            // of P, with no tour table
            const int mm = (ROUTE == WO_ROUTE_SSHAPE && SEQ_PASS && !any_big) ? 2 : (A.main_mode == 1 ? 1 : 0);
            if (SEQ_PASS && mm == 2) {
                uint32_t *pp = (uint32_t *)tour;         // the tour table is not used
                const uint32_t npw = ((uint32_t)n + 31u) / 32u;
                const uint32_t ppt = (npw + BLOCK - 1) / BLOCK;
                const uint32_t q0 = min(npw, (uint32_t)tid * ppt), q1 = min(npw, q0 + ppt);
                uint32_t c = 0;
                for (uint32_t w = q0; w < q1; w++) c += __popc(P[w]);
                uint32_t tot;
                uint32_t base = block_excl_scan<BLOCK>(c, scan_a, &tot);
                for (uint32_t w = q0; w < q1; w++) {
                    pp[w] = base;
                    base += __popc(P[w]);
                }
            } else {
                write_entries(0u, one_piece);
            }
            __syncthreads();

            // ---- prefetch of the next plan's inputs -----------------------
            if (next_item < A.n_plans) {
                const int64_t pn = A.work ? (int64_t)A.work[next_item] : next_item;
                // one instance: the next plan's row follows from this plan's
                // sizes with no table loads
                const bool same = A.n_inst <= 1;
                const int iin = same ? ii : instance_of(A, pn);
                const InstDev &In = A.inst[iin];
                const int nn = same ? n : In.n_orders;
                const int cn = same ? C : In.n_cat;
                const int chn = (nn + BLOCK - 1) / BLOCK;
                if (chn <= SEQ_CHUNK) {                  // uniform
                    const uint16_t *seqn = same ? A.seq + seq_base0 + pn * (int64_t)nn
                                                : A.seq + A.seq_base[iin] + (pn - A.plan_begin[iin]) * (int64_t)nn;
                    const int c0 = min(nn, tid * chn), c1 = min(nn, c0 + chn);
                    pf_raw = load_chunk<SEQ_CHUNK>(seqn + c0, c1 - c0, (uint32_t)nn, sv_pf);
                    zc_pf = (tid < 64 && lane < cn) ? (uint32_t)A.zone_of[pn * 64 + lane] : 0xFFu;
                    have_pf = true;
                }
            }

            __builtin_amdgcn_s_setprio(0);

            // ---- 5./6. aisle sets and S-shape per tour tile ------------------
            const uint32_t magic = I.magic;
            const int32_t wsp = A.plan_spacing ? A.plan_spacing[p] : I.spacing;   // aisle spacing of this plan
            for (uint32_t t0 = 0; t0 < n_tours; t0 += (uint32_t)T) {
                if (t0 > 0) {
                    __syncthreads();                     // the previous tile's rows are read
                    if (!(SEQ_PASS && mm == 2)) write_entries(t0, false);
                    uint4 *rows = (uint4 *)(smem + LDS_REGION);
                    const int nr4 = (int)((RB * (uint32_t)(T + 1) + 15u) / 16u);
                    for (int k = tid; k < nr4; k += BLOCK) rows[k] = make_uint4(0u, 0u, 0u, 0u);
                    __syncthreads();
                }
                if (ROUTE == WO_ROUTE_SSHAPE && SEQ_PASS && mm == 2) {
                    // each wave takes 64 consecutive units (lines) of the
                    // sequence: a line finds its order from the unit bitmap,
                    // its record in the order's line list, its tour from the
                    // opening flags; the farthest location of each tour's
                    // lanes is one segmented max across the wave (tours are
                    // contiguous), raised once per tour and wave
                    const uint32_t *ordoff = A.ordoff + I.ordoff_off;
                    const uint32_t *ordrec = A.ordrec + I.ordrec_off;
                    const uint32_t *pp = (const uint32_t *)tour;
                    const int zsv = (int)zs[lane];
                    for (uint32_t c0 = (uint32_t)(tid >> 6) * 64u; c0 < n_units; c0 += (uint32_t)BLOCK) {
                        const uint32_t su = c0 + (uint32_t)lane;
                        const bool act = su < n_units;
                        uint32_t rec = 0, tr = 0xFFFFFFFFu;
                        if (act) {
                            const uint32_t w = su >> 5;
                            const uint32_t hi = B[w] & (0xFFFFFFFFu >> (31u - (su & 31u)));
                            uint32_t start, cle;
                            if (hi) {
                                start = (w << 5) + 31u - (uint32_t)__builtin_clz(hi);
                                cle = pref[w] + __popc(hi);
                            } else {                     // the order began in the word below (size <= Q <= 32)
                                const uint32_t lo = w ? B[w - 1] : 1u;
                                start = ((w - 1u) << 5) + 31u - ffbh(lo);
                                cle = pref[w];
                            }
                            const uint32_t pos = min(cle - 1u, (uint32_t)(n - 1));
                            const uint32_t o = min((uint32_t)seq[pos], (uint32_t)(n - 1));
                            const uint32_t j = min(su - start, ordoff[o + 1] - ordoff[o] - 1u);
                            rec = ordrec[ordoff[o] + j];
                            const uint32_t pw = pos >> 5;
                            const uint32_t t = pp[pw] + __popc(P[pw] & (0xFFFFFFFFu >> (31u - (pos & 31u)))) - 1u;
                            const uint32_t rel = t - t0;
                            tr = rel < (uint32_t)T ? rel * RB : dummy;
                        }
                        const uint32_t ls = rec + (uint32_t)__builtin_amdgcn_ds_bpermute((int)(rec >> 24), zsv);
                        if (act) {
                            const uint32_t a = mulhi24(ls, magic);
                            __hip_atomic_fetch_or(lds32(LDS_REGION + 4u + tr + ((a >> 5) << 2)), 1u << (a & 31u),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        // segments of equal tour rows: heads by ballot, max by
                        // shifted lane reads within each segment
                        const uint32_t prev = (uint32_t)__shfl_up((int)tr, 1, 64);
                        const uint64_t heads = __ballot(lane == 0 || prev != tr);
                        const int seg0 = 63 - __builtin_clzll(heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull)));
                        uint32_t m = act ? ls : 0u;
#pragma unroll
                        for (int d = 1; d < 64; d <<= 1) {
                            const uint32_t x = (uint32_t)__shfl_up((int)m, d, 64);
                            if (lane - d >= seg0) m = max(m, x);
                        }
                        const bool last = lane == 63 || ((heads >> (lane + 1)) & 1ull);
                        if (act && last)
                            __hip_atomic_fetch_max(lds32(LDS_REGION + tr), m, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                } else if (ROUTE != WO_ROUTE_SSHAPE || mm == 0) {
                    // each wave takes whole groups of 64 lanes x 8 line slots
                    constexpr int U = LINE_SLOTS;
                    constexpr int NW = BLOCK / 64;
                    const int zsv = (int)zs[lane];
                    const uint2 *lines = A.lines + I.line_off + lane;
                    const int n_grp8 = I.n_lines_pad / LINE_PAD;
                    for (int gi = tid >> 6; gi < n_grp8; gi += NW) {   // uniform per wave
                        uint2 v[U];
                        uint32_t tb[U], zv[U];
#pragma unroll
                        for (int u = 0; u < U; u++) v[u] = lines[gi * LINE_PAD + u * 64];
                        // all table reads of the group before its atomics.
                        // Every slot reads its order's tour entry (reading it
                        // only at the first slot of a run takes a branch per
                        // slot, which costs more); a lane's slots hold
                        // consecutive lines, so an order's farthest location
                        // is raised once per run (bit 31 of y marks the first
                        // slot of a run)
                        bool first[U];
#pragma unroll
                        for (int u = 0; u < U; u++) {
                            first[u] = u == 0 || (int32_t)v[u].y < 0;
                            tb[u] = *lds16(v[u].y & 0x7FFFFFFFu);
                            zv[u] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(v[u].x >> 24), zsv);
                        }
                        if (ROUTE != WO_ROUTE_SSHAPE) {
                            // pick rows: take the next entry of the tour's row
                            // (the dummy row's count runs past its entries,
                            // which then share its last one)
                            const uint32_t last = (uint32_t)I.pick_slots - 1u;
#pragma unroll
                            for (int u = 0; u < U; u++) {
                                const uint32_t e = __hip_atomic_fetch_add(lds32(LDS_REGION + tb[u]), 1u, __ATOMIC_RELAXED,
                                                                          __HIP_MEMORY_SCOPE_WORKGROUP);
                                *lds32(LDS_REGION + 4u + tb[u] + (min(e, last) << 2)) = v[u].x + zv[u];
                            }
                            continue;
                        }
                        uint32_t far = 0;
#pragma unroll
                        for (int u = 0; u < U; u++) {
                            const uint32_t ls = v[u].x + zv[u];
                            const uint32_t a = mulhi24(ls, magic);
                            __hip_atomic_fetch_or(lds32(LDS_REGION + 4u + tb[u] + ((a >> 5) << 2)), 1u << (a & 31u),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            far = max(far, ls);
                            if (u == U - 1 || first[u + 1]) {
                                __hip_atomic_fetch_max(lds32(LDS_REGION + tb[u]), far, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                                far = 0;
                            }
                        }
                    }
                } else {
                    // one order per lane: its row looked up once, its farthest
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
                            for (int u = 0; u < PF; u++)
                                r_n[u] = (uint32_t)u < L_n ? grec[b_n + u * 64 + lane] : 0u;
                        }
                        const uint32_t tb = (o != 0xFFFFu) ? (uint32_t)tour[o] : dummy;
                        uint32_t far = 0;
#pragma unroll
                        for (int u = 0; u < PF; u++) {
                            if ((uint32_t)u < L) {
                                const uint32_t ls =
                                    r[u] + (uint32_t)__builtin_amdgcn_ds_bpermute((int)(r[u] >> 24), zsv);
                                const uint32_t a = mulhi24(ls, magic);
                                __hip_atomic_fetch_or(lds32(LDS_REGION + 4u + tb + ((a >> 5) << 2)), 1u << (a & 31u),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                                far = max(far, ls);
                            }
                        }
                        for (uint32_t kk = PF; kk < L; kk++) {     // long orders
                            const uint32_t rr = grec[b0g + kk * 64 + lane];
                            const uint32_t ls = rr + (uint32_t)__builtin_amdgcn_ds_bpermute((int)(rr >> 24), zsv);
                            const uint32_t a = mulhi24(ls, magic);
                            __hip_atomic_fetch_or(lds32(LDS_REGION + 4u + tb + ((a >> 5) << 2)), 1u << (a & 31u),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            far = max(far, ls);
                        }
                        __hip_atomic_fetch_max(lds32(LDS_REGION + tb), far, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        g = gn;
                    }
                }
                __syncthreads();
                const int nt = (int)min((uint32_t)T, n_tours - t0);
                if (ROUTE != WO_ROUTE_SSHAPE) {
                    for (int t = tid; t < nt; t += BLOCK) {
                        const uint32_t *rw = (const uint32_t *)(smem + LDS_REGION + (uint32_t)t * RB);
                        const uint32_t np = rw[0];                 // >= 1: a tour has picks
                        if (np > (uint32_t)I.pick_slots) continue; // an order routed apart (below)
                        uint32_t v[MAX_PICK_SLOTS];
#pragma unroll
                        for (int i = 0; i < MAX_PICK_SLOTS; i++) v[i] = (uint32_t)i < np ? rw[1 + i] : 0xFFFFFFFFu;
                        sort32(v);
                        acc += pick_route_cost<ROUTE>(v, np, wsp, I, magic);
                    }
                    continue;
                }
                const int W = I.words;
                for (int t = tid; t < nt; t += BLOCK) {
                    const uint32_t *rw = (const uint32_t *)(smem + LDS_REGION + (uint32_t)t * RB);
                    const uint32_t ls = rw[0];
                    int k = 0, w = 0;
                    for (; w + 4 <= W; w += 4)
                        k += __popc(rw[1 + w]) + __popc(rw[2 + w]) + __popc(rw[3 + w]) + __popc(rw[4 + w]);
                    for (; w < W; w++) k += __popc(rw[1 + w]);
                    const uint32_t a = mulhi24(ls, magic);
                    const uint32_t j = (ls - a * I.d_s) >> (I.shift + 1);
                    const int64_t y = (int64_t)j * I.pitch + I.pitch / 2;
                    int64_t cost = 2ll * wsp * a;
                    cost += (k & 1) ? (int64_t)(k - 1) * I.L + 2 * y : (int64_t)k * I.L;
                    acc += cost;
                }
            }
            // orders longer than a pick row, each a tour of its own
            if (ROUTE != WO_ROUTE_SSHAPE && I.n_big > 0)   // uniform
                acc += big_orders_cost<ROUTE, BLOCK>(A, I, zs, (uint32_t *)(smem + LDS_REGION), wsp);
        }
#undef SV
#undef CS
        __builtin_amdgcn_s_setprio(0);                 // also for a plan that was not evaluated
        const int64_t D = block_sum64<BLOCK>(acc, sum_slot);
        if (A.validate && bad) atomicOr(A.err, 1);
        if (tid == 0) {
            const int64_t Dv = units_ok ? D : (int64_t)2147483647;
            A.dist[p] = Dv > 2147483647ll ? 2147483647 : (int32_t)Dv;
            if (A.thr) A.thr[p] = window_throughput(Dv, I);
        }
        item = next_item;
    }
}

// Reset of the work-queue ticket (a kernel, so that it can sit in a graph).
__global__ void reset_ticket_kernel(uint32_t *ctr) { *ctr = 0u; }

template <int BLOCK, int ROUTE, bool SEQ_PASS>
static hipError_t launch_eval_t(const EvalArgs &a, uint32_t lds_bytes, int grid, hipStream_t s)
{
    // raise the dynamic LDS limit to what this launch needs
    static uint32_t attr_bytes = 0;
    if (lds_bytes > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)eval_plans_kernel<BLOCK, ROUTE, SEQ_PASS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        attr_bytes = lds_bytes;
    }
    if (a.queue) hipLaunchKernelGGL(reset_ticket_kernel, dim3(1), dim3(1), 0, s, a.queue_ctr);
    hipLaunchKernelGGL((eval_plans_kernel<BLOCK, ROUTE, SEQ_PASS>), dim3(grid), dim3(BLOCK), lds_bytes, s, a);
    return hipGetLastError();
}

template <int BLOCK, int ROUTE, bool SEQ_PASS>
static int max_blocks_t(uint32_t lds_bytes)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, eval_plans_kernel<BLOCK, ROUTE, SEQ_PASS>, BLOCK, lds_bytes) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

template <int ROUTE, bool SEQ_PASS = false>
static int max_blocks_r(int block, uint32_t lds_bytes)
{
    switch (block) {
    case 64: return max_blocks_t<64, ROUTE, SEQ_PASS>(lds_bytes);
    case 128: return max_blocks_t<128, ROUTE, SEQ_PASS>(lds_bytes);
    case 256: return max_blocks_t<256, ROUTE, SEQ_PASS>(lds_bytes);
    case 512: return max_blocks_t<512, ROUTE, SEQ_PASS>(lds_bytes);
    }
    return 1;
}

int eval_max_blocks_per_cu(int block, int route, uint32_t lds_bytes, int line_pass)
{
    if (route == WO_ROUTE_SSHAPE && line_pass == 2) return max_blocks_r<WO_ROUTE_SSHAPE, true>(block, lds_bytes);
    switch (route) {
    case WO_ROUTE_RETURN: return max_blocks_r<WO_ROUTE_RETURN>(block, lds_bytes);
    case WO_ROUTE_LARGEST_GAP: return max_blocks_r<WO_ROUTE_LARGEST_GAP>(block, lds_bytes);
    case WO_ROUTE_OPTIMAL: return max_blocks_r<WO_ROUTE_OPTIMAL>(block, lds_bytes);
    case WO_ROUTE_COMBINED: return max_blocks_r<WO_ROUTE_COMBINED>(block, lds_bytes);
    }
    return max_blocks_r<WO_ROUTE_SSHAPE>(block, lds_bytes);
}

template <int ROUTE, bool SEQ_PASS = false>
static hipError_t launch_eval_r(const EvalArgs &a, uint32_t lds_bytes, int grid, int block, hipStream_t s)
{
    switch (block) {
    case 64: return launch_eval_t<64, ROUTE, SEQ_PASS>(a, lds_bytes, grid, s);
    case 128: return launch_eval_t<128, ROUTE, SEQ_PASS>(a, lds_bytes, grid, s);
    case 256: return launch_eval_t<256, ROUTE, SEQ_PASS>(a, lds_bytes, grid, s);
    case 512: return launch_eval_t<512, ROUTE, SEQ_PASS>(a, lds_bytes, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_eval(const EvalArgs &a, uint32_t lds_bytes, int grid, int block, int route, hipStream_t s)
{
    switch (route) {
    case WO_ROUTE_SSHAPE:
        // the line pass in sequence order is an instantiation of its own, so
        // that the default one carries none of its code
        if (a.main_mode == 2) return launch_eval_r<WO_ROUTE_SSHAPE, true>(a, lds_bytes, grid, block, s);
        return launch_eval_r<WO_ROUTE_SSHAPE>(a, lds_bytes, grid, block, s);
    case WO_ROUTE_RETURN: return launch_eval_r<WO_ROUTE_RETURN>(a, lds_bytes, grid, block, s);
    case WO_ROUTE_LARGEST_GAP: return launch_eval_r<WO_ROUTE_LARGEST_GAP>(a, lds_bytes, grid, block, s);
    case WO_ROUTE_OPTIMAL: return launch_eval_r<WO_ROUTE_OPTIMAL>(a, lds_bytes, grid, block, s);
    case WO_ROUTE_COMBINED: return launch_eval_r<WO_ROUTE_COMBINED>(a, lds_bytes, grid, block, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace wo
