// Genetic plan search on gfx950 (the top-level optimiser of the paper's SDO,
// section 5, organising the clustering and sequencing searches of section 6).
//
// Random numbers come from a counter generator: the SplitMix64 finaliser
// (Steele, Lea & Flood 2014) over (seed, stream, generation, child, position),
// so every draw is recomputable anywhere.  Operators:
//   - tournament: `tsize` uniform draws from the population, winner = the
//     smallest (distance, index);
//   - zone swap: for each category position c in turn, with probability
//     thr / 2^32, swap its zone with a uniformly chosen other position;
//   - order insert: for each sequence position i = 0 .. n-1 in turn, with the
//     same probability, move the element currently at i so that it ends at a
//     uniform position j;
//   - uniform integers in [0, m): (r32 * m) >> 32.
#include "wo_internal.h"
#include "wo_search.h"

namespace wo {

static __device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static __device__ __forceinline__ uint32_t draw(uint64_t seed, uint32_t stream, uint32_t gen, uint32_t child,
                                                uint32_t pos)
{
    uint64_t h = splitmix64(seed + stream);
    h = splitmix64(h ^ (((uint64_t)gen << 32) | child));
    h = splitmix64(h ^ (uint64_t)pos);
    return (uint32_t)(h >> 32);
}

static __device__ __forceinline__ uint32_t uniform(uint32_t r, uint32_t m)
{
    return (uint32_t)(((uint64_t)r * m) >> 32);
}

static __device__ int tournament(const int32_t *dist, int P, int tsize, uint64_t seed, uint32_t gen, uint32_t child)
{
    int best = -1;
    int32_t bd = 0;
    for (int k = 0; k < tsize; k++) {
        const int i = (int)uniform(draw(seed, RS_TOURNAMENT, gen, child, (uint32_t)k), (uint32_t)P);
        const int32_t d = dist[i];
        if (best < 0 || d < bd || (d == bd && i < best)) {
            best = i;
            bd = d;
        }
    }
    return best;
}

static __device__ void mutate_zones(uint8_t *z, int C, uint32_t thr, uint64_t seed, uint32_t gen, uint32_t child)
{
    if (C < 2) return;
    for (int c = 0; c < C; c++) {
        if (draw(seed, RS_ZONE_COIN, gen, child, (uint32_t)c) < thr) {
            uint32_t j = uniform(draw(seed, RS_ZONE_PARTNER, gen, child, (uint32_t)c), (uint32_t)(C - 1));
            if ((int)j >= c) j++;
            const uint8_t t = z[c];
            z[c] = z[j];
            z[j] = t;
        }
    }
}

// Index of the best individual (smallest distance, then index).  One block.
__global__ __launch_bounds__(1024) void argmin_kernel(const int32_t *dist, int P, int32_t *out)
{
    __shared__ unsigned long long best[1024];
    unsigned long long b = ~0ull;
    for (int i = threadIdx.x; i < P; i += 1024) {
        const unsigned long long k = ((unsigned long long)(uint32_t)(dist[i] ^ 0x80000000) << 32) | (uint32_t)i;
        b = k < b ? k : b;
    }
    best[threadIdx.x] = b;
    __syncthreads();
    for (int s = 512; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s && best[threadIdx.x + s] < best[threadIdx.x]) best[threadIdx.x] = best[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (int32_t)(best[0] & 0xFFFFFFFFull);
}

// Screened arm: candidate slottings (tournament winner's zones, mutated).
__global__ __launch_bounds__(256) void candidates_kernel(CandArgs a)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= a.K) return;
    const int par = tournament(a.pd, a.P, a.tsize, a.seed, a.gen, (uint32_t)b);
    uint8_t z[64];
    for (int c = 0; c < 64; c++) z[c] = a.pz[(int64_t)par * 64 + c];
    mutate_zones(z, a.C, a.thr, a.seed, a.gen, (uint32_t)b);
    for (int c = 0; c < 64; c++) a.cand_zone[(int64_t)b * 64 + c] = z[c];
    a.cand_parent[b] = par;
}

// One workgroup per child: choose the parent, copy, mutate zones and sequence.
__global__ __launch_bounds__(256) void breed_kernel(BreedArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *buf = (uint16_t *)smem;                                    // n
    uint32_t *moves = (uint32_t *)(smem + ((2 * a.n + 15) & ~15));       // n / 32 + 1 words
    __shared__ int s_parent;
    __shared__ uint32_t s_cid;
    const int c = blockIdx.x, tid = threadIdx.x;
    const int n = a.n;
    if (tid == 0) {
        int par;
        uint32_t cid;
        bool elite = false;
        if (a.mode == 0) {
            cid = (uint32_t)c;
            if (c == 0) {
                par = a.best[0];
                elite = true;
            } else {
                par = tournament(a.pd, a.P, a.tsize, a.seed, a.gen, cid);
            }
        } else {
            cid = (uint32_t)a.kept[c];
            par = a.cand_parent[cid];
        }
        uint8_t z[64];
        for (int k = 0; k < 64; k++)
            z[k] = a.mode == 0 ? a.pz[(int64_t)par * 64 + k] : a.cand_zone[(int64_t)cid * 64 + k];
        if (a.mode == 0 && !elite) mutate_zones(z, a.C, a.thr, a.seed, a.gen, cid);
        for (int k = 0; k < 64; k++) a.cz[(int64_t)c * 64 + k] = z[k];
        s_parent = elite ? -1 - par : par;
        s_cid = cid;
    }
    const int nw = n / 32 + 1;
    for (int w = tid; w < nw; w += 256) moves[w] = 0;
    __syncthreads();
    const bool elite = s_parent < 0;
    const int par = elite ? -1 - s_parent : s_parent;
    const uint32_t cid = s_cid;
    const uint16_t *src = a.ps + (int64_t)par * n;
    for (int i = tid; i < n; i += 256) buf[i] = src[i];
    if (!elite) {
        for (int i = tid; i < n; i += 256)
            if (draw(a.seed, RS_INSERT_COIN, a.gen, cid, (uint32_t)i) < a.thr) atomicOr(&moves[i >> 5], 1u << (i & 31));
    }
    __syncthreads();
    if (!elite) {
        // positions with a move, in increasing order; each move shifts the
        // range between i and j by one (chunks in a safe order, all reads of a
        // chunk before its writes)
        for (int w = 0; w < nw; w++) {
            uint32_t bits = moves[w];
            while (bits) {
                const int i = w * 32 + __builtin_ctz(bits);
                bits &= bits - 1u;
                const int j = (int)uniform(draw(a.seed, RS_INSERT_TARGET, a.gen, cid, (uint32_t)i), (uint32_t)n);
                if (j == i) continue;
                const uint16_t v = buf[i];
                __syncthreads();
                if (j > i) {            // buf[i..j-1] = buf[i+1..j]
                    for (int base = i; base < j; base += 256 * 8) {
                        uint16_t t[8];
#pragma unroll
                        for (int q = 0; q < 8; q++) {
                            const int k = base + q * 256 + tid;
                            t[q] = k < j ? buf[k + 1] : 0;
                        }
                        __syncthreads();
#pragma unroll
                        for (int q = 0; q < 8; q++) {
                            const int k = base + q * 256 + tid;
                            if (k < j) buf[k] = t[q];
                        }
                        __syncthreads();
                    }
                } else {                // buf[j+1..i] = buf[j..i-1], from the top down
                    for (int top = i; top > j; top -= 256 * 8) {
                        uint16_t t[8];
#pragma unroll
                        for (int q = 0; q < 8; q++) {
                            const int k = top - q * 256 - tid;
                            t[q] = k > j ? buf[k - 1] : 0;
                        }
                        __syncthreads();
#pragma unroll
                        for (int q = 0; q < 8; q++) {
                            const int k = top - q * 256 - tid;
                            if (k > j) buf[k] = t[q];
                        }
                        __syncthreads();
                    }
                }
                if (tid == 0) buf[j] = v;
                __syncthreads();
            }
        }
    }
    uint16_t *dst = a.cs + (int64_t)c * n;
    for (int i = tid; i < n; i += 256) dst[i] = buf[i];
}

// Screened arm: the evaluated children replace the worst individuals.
__global__ __launch_bounds__(256) void replace_kernel(ReplaceArgs a)
{
    const int r = blockIdx.x;
    const int dst = a.worst[r];
    for (int k = threadIdx.x; k < 64; k += 256) a.pz[(int64_t)dst * 64 + k] = a.cz[(int64_t)r * 64 + k];
    for (int k = threadIdx.x; k < a.n; k += 256) a.ps[(int64_t)dst * a.n + k] = a.cs[(int64_t)r * a.n + k];
    if (threadIdx.x == 0) a.pd[dst] = a.cd[r];
}

hipError_t launch_argmin(const int32_t *dist, int P, int32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(argmin_kernel, dim3(1), dim3(1024), 0, s, dist, P, out);
    return hipGetLastError();
}

hipError_t launch_candidates(const CandArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(candidates_kernel, dim3((a.K + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

uint32_t breed_lds_bytes(int n) { return (uint32_t)(((2 * n + 15) & ~15) + 4 * (n / 32 + 1)); }

hipError_t launch_breed(const BreedArgs &a, int n_children, hipStream_t s)
{
    static uint32_t attr_bytes = 0;
    const uint32_t need = breed_lds_bytes(a.n);
    if (need > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)breed_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        attr_bytes = need;
    }
    hipLaunchKernelGGL(breed_kernel, dim3(n_children), dim3(256), breed_lds_bytes(a.n), s, a);
    return hipGetLastError();
}

hipError_t launch_replace(const ReplaceArgs &a, int keep, hipStream_t s)
{
    hipLaunchKernelGGL(replace_kernel, dim3(keep), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace wo
