// Exact plan evaluation on gfx950: slot map, next-fit tours, S-shape distance,
// time-window throughput (arXiv 2110.13693, section 5, Subproblems 2 and 3,
// Eq. (2); section 6).  One workgroup evaluates one plan at a time and walks
// the plans with a grid stride.
//
// Per plan:
//   1. zone starts: start[c] = sum of the sizes of categories placed in a
//      lower zone; kept in LDS pre-shifted so that a line's scaled location
//      is one add: ls = rec + zs[rec >> 24 / 4];
//   2. the order sequence is staged in LDS with its item prefix sums P;
//   3. next-fit: e(i) = one past the last order of a tour opened at position
//      i = the largest m with P[m] - P[i] <= Q (at least i + 1); tours start
//      on the orbit of 0 under e; each order gets its tour id;
//   4. every order line (in instance order, coalesced) sets its aisle bit in
//      its tour's aisle set (ds_or) and raises its tour's farthest location
//      (ds_max) -- the largest location of a tour is, at once, the last
//      aisle visited and the farthest depth in it;
//   5. per tour: k = popcount of the aisle set, S-shape closed form; the
//      block sums the tours in int64.
#include "wo_internal.h"

namespace wo {

static __device__ __forceinline__ uint32_t mulhi24(uint32_t x, uint32_t m)
{
    return (uint32_t)(((uint64_t)(x & 0xFFFFFFu) * (uint64_t)(m & 0xFFFFFFu)) >> 32);
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

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void eval_plans_kernel(EvalArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;

    for (int64_t p = blockIdx.x; p < A.n_plans; p += gridDim.x) {
        int ii = 0;
        if (A.n_inst > 1) {
            int lo = 0, hi = A.n_inst - 1;   // last instance whose first row <= p
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (A.plan_begin[mid] <= p) lo = mid; else hi = mid - 1;
            }
            ii = lo;
        }
        const InstDev &I = A.inst[ii];
        const int n = I.n_orders;
        const int C = I.n_cat;
        const uint32_t Q = (uint32_t)I.capacity;
        const int64_t row = p - (A.n_inst > 1 ? A.plan_begin[ii] : 0);
        const uint16_t *seq = A.seq + A.seq_base[ii] + row * (int64_t)n;
        const uint32_t *rec = A.rec + I.rec_off;
        const uint32_t *ooff = A.ooff + I.ooff_off;
        const uint16_t *lord = A.lord + I.lord_off;
        const EvalLayout Ly = eval_layout(n, I.words, I.t_cap);
        uint32_t *zs = (uint32_t *)(smem + Ly.zs);
        int64_t *red = (int64_t *)(smem + Ly.red);
        uint32_t *P = (uint32_t *)(smem + Ly.P);
        uint16_t *sq = (uint16_t *)(smem + Ly.sq);
        uint16_t *e = (uint16_t *)(smem + Ly.e);
        uint16_t *tour = (uint16_t *)(smem + Ly.tour);
        uint8_t *flag = (uint8_t *)(smem + Ly.flag);
        uint32_t *mask = (uint32_t *)(smem + Ly.mask);
        uint32_t *mx = (uint32_t *)(smem + Ly.mx);
        int bad = 0;

        // ---- 1. zone starts (wave 0) -------------------------------------
        if (tid < 64) {
            uint32_t zc = (lane < C) ? (uint32_t)A.zone_of[p * 64 + lane] : 0xFFu;
            uint32_t start = 0;
            for (int c2 = 0; c2 < C; c2++) {
                uint32_t z2 = (uint32_t)__shfl((int)zc, c2, 64);
                start += (z2 < zc) ? (uint32_t)I.cat_size[c2] : 0u;
            }
            zs[lane] = (start << I.shift) - ((uint32_t)(4 * lane) << 24);
            if (A.validate) {
                uint64_t m = (lane < C && zc < 64u) ? (1ull << zc) : 0ull;
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) m |= __shfl_xor(m, d, 64);
                uint64_t want = (C == 64) ? ~0ull : ((1ull << C) - 1ull);
                if (lane == 0 && m != want) bad = 1;
            }
        }

        // ---- 2. sequence, item prefix sums -------------------------------
        const int ch = (n + BLOCK - 1) / BLOCK;
        const int b0 = min(n, tid * ch), b1 = min(n, b0 + ch);
        int local = 0;
        for (int i = b0; i < b1; i++) {
            uint32_t o = seq[i];
            if (o >= (uint32_t)n) { bad = 1; o = (uint32_t)(n - 1); }
            sq[i] = (uint16_t)o;
            flag[i] = 0;
            local += (int)(ooff[o + 1] - ooff[o]);
        }
        int total_items;
        int run = block_excl_scan<BLOCK>(local, (int *)red, &total_items);
        for (int i = b0; i < b1; i++) {
            P[i] = (uint32_t)run;
            uint32_t o = sq[i];
            run += (int)(ooff[o + 1] - ooff[o]);
        }
        if (tid == 0) P[n] = (uint32_t)total_items;
        if (A.validate) {
            // permutation check: mark every order once (bitmap in the mask area)
            uint32_t *seen = mask;
            for (int w = tid; w < (n + 31) / 32; w += BLOCK) seen[w] = 0;
            __syncthreads();
            for (int i = tid; i < n; i += BLOCK) {
                uint32_t o = sq[i];
                uint32_t old = atomicOr(&seen[o >> 5], 1u << (o & 31));
                if (old & (1u << (o & 31))) bad = 1;
            }
        }
        __syncthreads();

        // ---- 3. next-fit tours -------------------------------------------
        for (int i = tid; i < n; i += BLOCK) {
            const uint32_t target = P[i] + Q;
            int m = i + 1;
            if (P[i + 1] <= target) {
                int lo = i + 1, hi = min(n, i + (int)Q);   // P[lo] <= target
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (P[mid] <= target) lo = mid; else hi = mid - 1;
                }
                m = lo;
            }
            e[i] = (uint16_t)m;
        }
        __syncthreads();
        if (tid == 0) {
            int x = 0;
            while (x < n) { flag[x] = 1; x = e[x]; }
        }
        __syncthreads();
        int cnt = 0;
        for (int i = b0; i < b1; i++) cnt += flag[i];
        int n_tours;
        int tid_run = block_excl_scan<BLOCK>(cnt, (int *)red, &n_tours) - 1;
        for (int i = b0; i < b1; i++) {
            tid_run += flag[i];
            tour[sq[i]] = (uint16_t)tid_run;
        }
        __syncthreads();

        // ---- 4./5. aisle sets and S-shape per tour tile ------------------
        const int W = I.words;
        const int T = I.t_cap;
        const uint32_t magic = I.magic;
        int64_t acc = 0;
        for (int t0 = 0; t0 < n_tours; t0 += T) {
            for (int k = tid; k < W * T; k += BLOCK) mask[k] = 0;
            for (int k = tid; k < T; k += BLOCK) mx[k] = 0;
            __syncthreads();
            for (int q = tid; q < I.n_lines; q += BLOCK) {
                const uint32_t t = (uint32_t)tour[lord[q]] - (uint32_t)t0;
                if (t < (uint32_t)T) {
                    const uint32_t r = rec[q];
                    const uint32_t ls = r + zs[r >> 26];
                    const uint32_t a = mulhi24(ls, magic);
                    atomicOr(&mask[(a >> 5) * T + t], 1u << (a & 31));
                    atomicMax(&mx[t], ls);
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
    }
}

hipError_t launch_eval(const EvalArgs &a, uint32_t lds_bytes, int grid, hipStream_t s)
{
    constexpr int BLOCK = 256;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)eval_plans_kernel<BLOCK>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(eval_plans_kernel<BLOCK>, dim3(grid), dim3(BLOCK), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace wo
