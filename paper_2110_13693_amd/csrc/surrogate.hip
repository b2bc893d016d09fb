// Surrogate network kernels for gfx950: an MLP that predicts a plan's route
// distance from its slotting (the paper's hybrid decision making, section 1,
// Figure 1: models trained on simulated scenarios take decisions; here the
// simulator is the exact evaluator).
//
//   x   = one-hot(zone_of), 64 x 64 (row = category, column = zone) = 4096 inputs
//   h1  = GELU(x W1 + b1)      1024
//   h2  = GELU(h1 W2 + b2)     256
//   y   = h2 W3 + b3           (standardised distance)
//
// GEMMs run on MFMA (v_mfma_f32_32x32x16_bf16 or v_mfma_f32_16x16x32_bf16:
// bf16 operands, fp32 accumulation).  Weights are kept as fp32 masters in
// [out][in] layout with bf16 working copies; the one-hot operand of the
// forward products is generated in registers from the zone bytes and never
// stored.  Every GEMM here is C[M][N] = A[M][K] . B[N][K]^T with both operands
// K-contiguous.  The gradient of W1 is not a product: with a one-hot input it
// is a sum of du1 rows per (category, zone) bin (w1_grad_kernel).
#include <type_traits>

#include "wo_internal.h"
#include "wo_surrogate.h"

namespace wo {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
typedef __attribute__((__vector_size__(2 * sizeof(uint32_t)))) uint32_t u32x2;

// fp32 -> bf16, nearest with ties to even (the hardware conversion)
static __device__ __forceinline__ uint16_t f2bf(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

static __device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// tanh(a) = sign(a) (1 - 2 / (e^{2|a|} + 1)) with the hardware exp and
// reciprocal: absolute error near 1e-7, far below the bf16 rounding of the
// activations it feeds
static __device__ __forceinline__ float tanh_fast(float a)
{
    const float e = __expf(2.0f * fabsf(a));
    return copysignf(1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f), a);
}

static __device__ __forceinline__ float gelu_f(float u)
{
    const float t = tanh_fast(0.7978845608028654f * (u + 0.044715f * u * u * u));
    return 0.5f * u * (1.0f + t);
}

static __device__ __forceinline__ float gelu_grad_f(float u)
{
    const float t = tanh_fast(0.7978845608028654f * (u + 0.044715f * u * u * u));
    const float dt = (1.0f - t * t) * 0.7978845608028654f * (1.0f + 3.0f * 0.044715f * u * u);
    return 0.5f * (1.0f + t) + 0.5f * u * dt;
}

// ---------------------------------------------------------------------------
// GEMM: C[M][N] = A[M][K] . B[N][K]^T.  Block tile TM x TM (128 or 64), K
// step 64, four waves in 2 x 2, each (TM/2)^2 = (TM/32)^2 MFMA tiles of
// 16 x 16.  The next K step's operands are loaded into registers while the
// current one's MFMAs run from LDS.  M, N multiples of TM and K a multiple of
// 64 (the host pads); rows of A at or beyond M_real read as zero when
// generated from zone bytes.
// ---------------------------------------------------------------------------
constexpr int GBK = 64, GPAD = 8, GLDK = GBK + GPAD;
// zone bytes of A rows at a 68-byte stride: the 16 rows of an MFMA tile then
// read one category's bytes from 16 different LDS banks
constexpr int ZLD = 68;

template <int AMODE, int BMODE, int EPI, int TM, int MS>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g)
{
    constexpr int WT = TM / 2;                 // wave tile
    constexpr int FT = WT / MS;                // MS x MS MFMA tiles per wave and dimension
    constexpr int KM = MS == 32 ? 16 : 32;     // K depth of one MFMA
    using AccT = typename std::conditional<MS == 32, floatx16, floatx4>::type;
    constexpr int NLD = TM * GBK / 8 / 256;    // 16-byte loads per thread per operand tile
    // operand tiles in two buffers: step k reads buffer k & 1 while the next
    // step's operands are written to the other one
    __shared__ __align__(16) uint16_t As[2][(AMODE == A_BF16) ? TM * GLDK : 8];
    __shared__ __align__(16) uint16_t Bs[2][TM * GLDK];
    __shared__ __align__(16) uint8_t ZsA[(AMODE == A_ONEHOT) ? TM * ZLD : 16];
    // one-hot fragments: pattern d < 8 holds bf16 1.0 at element d, pattern 8
    // is all zeros
    __shared__ __align__(16) uint32_t OneHot[(AMODE == A_ONEHOT) ? 9 * 4 : 4];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
    // split K: this workgroup's part [kbeg, kend)
    const int kc = g.K / max(g.ksplit, 1);
    const int kbeg = (int)blockIdx.z * kc, kend = kbeg + kc;
    // v_mfma_f32_32x32x16_bf16 (MS = 32) or v_mfma_f32_16x16x32_bf16 (MS =
    // 16): lane l holds row (or column) l % MS and the 8 K elements from
    // 8 (l / MS) of a KM-deep step
    const int fr = lane & (MS - 1), fk = (lane / MS) * 8;

    AccT acc[FT][FT];
#pragma unroll
    for (int i = 0; i < FT; i++)
#pragma unroll
        for (int j = 0; j < FT; j++)
#pragma unroll
            for (int e = 0; e < (MS == 32 ? 16 : 4); e++) acc[i][j][e] = 0.f;

    if (AMODE == A_ONEHOT) {
        if (tid < 36) {
            const uint32_t d = (uint32_t)tid >> 2, e = (uint32_t)tid & 3u;
            OneHot[tid] = (d < 8u && (d >> 1) == e) ? (0x3F80u << ((d & 1u) * 16u)) : 0u;
        }
        // zone bytes of the block's rows, 0xFF past the real rows
        for (int c = tid; c < TM * 4; c += 256) {
            const int r = c >> 2, part = c & 3;
            uint4 v = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
            if (m0 + r < g.M_real) v = *(const uint4 *)(g.zoneA + (int64_t)(m0 + r) * 64 + part * 16);
            uint32_t *zw = (uint32_t *)(&ZsA[r * ZLD + part * 16]);
            zw[0] = v.x;
            zw[1] = v.y;
            zw[2] = v.z;
            zw[3] = v.w;
        }
    }

    u32x4 ra[NLD], rbv[NLD];   // native vectors, so that they stay in registers
#define WO_LOAD_TILE(k0_)                                                                                        \
    do {                                                                                                         \
        if (AMODE == A_BF16) {                                                                                   \
            _Pragma("unroll") for (int i = 0; i < NLD; i++) {                                                    \
                const int c = tid + i * 256, r = c >> 3, part = c & 7;                                           \
                ra[i] = *(const u32x4 *)(g.A + (int64_t)(m0 + r) * g.lda + (k0_) + part * 8);                    \
            }                                                                                                    \
        }                                                                                                        \
        _Pragma("unroll") for (int i = 0; i < NLD; i++) {                                                        \
            const int c = tid + i * 256, r = c >> 3, part = c & 7;                                               \
            rbv[i] = *(const u32x4 *)(g.B + (int64_t)(n0 + r) * g.ldb + (k0_) + part * 8);                       \
        }                                                                                                        \
    } while (0)
#define WO_STORE_TILE(buf)                                                                                       \
    do {                                                                                                         \
        if (AMODE == A_BF16) {                                                                                   \
            _Pragma("unroll") for (int i = 0; i < NLD; i++) {                                                    \
                const int c = tid + i * 256, r = c >> 3, part = c & 7;                                           \
                *(u32x4 *)(&As[buf][r * GLDK + part * 8]) = ra[i];                                               \
            }                                                                                                    \
        }                                                                                                        \
        _Pragma("unroll") for (int i = 0; i < NLD; i++) {                                                        \
            const int c = tid + i * 256, r = c >> 3, part = c & 7;                                               \
            *(u32x4 *)(&Bs[buf][r * GLDK + part * 8]) = rbv[i];                                                  \
        }                                                                                                        \
    } while (0)

    // one operand set per K step: the next one loads into registers while the
    // current one is multiplied from LDS, then goes to the other buffer
    WO_LOAD_TILE(kbeg);
    WO_STORE_TILE(0);
    __syncthreads();
    for (int k0 = kbeg, cur = 0; k0 < kend; k0 += GBK, cur ^= 1) {
        const bool more = k0 + GBK < kend;
        WO_LOAD_TILE(more ? k0 + GBK : k0);          // unconditional, so the operands stay in registers
        // a K step of 64 is one category: the zone of each of the wave's rows
        uint32_t zrow[FT];
        if (AMODE == A_ONEHOT) {
            const int cat = k0 >> 6;
#pragma unroll
            for (int ti = 0; ti < FT; ti++)
                zrow[ti] = cat < g.n_cat ? (uint32_t)ZsA[(wm * WT + ti * MS + fr) * ZLD + cat] : 0xFFu;
        }
#pragma unroll
        for (int ks = 0; ks < GBK; ks += KM) {
            bf16x8 af[FT], bfr[FT];
#pragma unroll
            for (int ti = 0; ti < FT; ti++) {
                const int row = wm * WT + ti * MS + fr;
                if (AMODE == A_BF16) {
                    af[ti] = *(const bf16x8 *)(&As[cur][row * GLDK + ks + fk]);
                } else {
                    af[ti] = *(const bf16x8 *)(&OneHot[4u * min(zrow[ti] - (uint32_t)(ks + fk), 8u)]);
                }
            }
#pragma unroll
            for (int tj = 0; tj < FT; tj++) {
                const int col = wn * WT + tj * MS + fr;
                bfr[tj] = *(const bf16x8 *)(&Bs[cur][col * GLDK + ks + fk]);
            }
#pragma unroll
            for (int ti = 0; ti < FT; ti++)
#pragma unroll
                for (int tj = 0; tj < FT; tj++)
                    if constexpr (MS == 32)
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[ti], bfr[tj], acc[ti][tj], 0, 0, 0);
                    else
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ti], bfr[tj], acc[ti][tj], 0, 0, 0);
        }
        if (more) WO_STORE_TILE(cur ^ 1);
        __syncthreads();
    }
#undef WO_LOAD_TILE
#undef WO_STORE_TILE

    // epilogue: of each MS x MS tile, lane l holds column l % MS and, for
    // q = 0 .. QN - 1, rows 8 q + 4 (l / MS) + r (r = 0 .. 3) in elements
    // 4 q + r (MS = 32: QN = 4; MS = 16: QN = 1)
    constexpr int QN = MS == 32 ? 4 : 1;
#pragma unroll
    for (int ti = 0; ti < FT; ti++) {
#pragma unroll
        for (int tj = 0; tj < FT; tj++) {
            const int col = n0 + wn * WT + tj * MS + fr;
            uint2 pkq[QN];                           // the transposed copy's 4-row pieces
#pragma unroll
            for (int q = 0; q < QN; q++) {
                const int rb = m0 + wm * WT + ti * MS + 8 * q + (lane / MS) * 4;
                if (EPI == EPI_STORE) {
                    float *C = g.C + (int64_t)blockIdx.z * g.c_split;
#pragma unroll
                    for (int r = 0; r < 4; r++) C[(uint32_t)((rb + r) * g.ldc + col)] = acc[ti][tj][4 * q + r];
                } else if (EPI == EPI_BIAS_GELU) {
                    const float bias = g.bias[col];
                    uint16_t hv[4];
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const float u = acc[ti][tj][4 * q + r] + bias;
                        if (g.U) g.U[(uint32_t)((rb + r) * g.ldc + col)] = u;
                        if (g.H || g.HT) hv[r] = f2bf(gelu_f(u));
                        if (g.H) g.H[(uint32_t)((rb + r) * g.ldc + col)] = hv[r];
                    }
                    if (g.HT) {
                        pkq[q] = make_uint2((uint32_t)hv[0] | ((uint32_t)hv[1] << 16),
                                            (uint32_t)hv[2] | ((uint32_t)hv[3] << 16));
                        if (MS != 32) *(uint2 *)(g.HT + (int64_t)col * g.ldt + rb) = pkq[q];
                    }
                } else {   // EPI_GELU_GRAD_T: v = acc * gelu'(U) in bf16, transposed (and row-major)
                    uint16_t hv[4];
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const float u = g.Uin[(uint32_t)((rb + r) * g.ldc + col)];
                        hv[r] = f2bf(acc[ti][tj][4 * q + r] * gelu_grad_f(u));
                    }
                    const uint2 pk = make_uint2((uint32_t)hv[0] | ((uint32_t)hv[1] << 16),
                                                (uint32_t)hv[2] | ((uint32_t)hv[3] << 16));
                    pkq[q] = pk;
                    if (MS != 32) *(uint2 *)(g.HT + (int64_t)col * g.ldt + rb) = pk;
                    if (g.H) {
                        // and in column slices, [N / DU1_SLICE][M][DU1_SLICE]: a
                        // 4 x 4 transpose within each quad of lanes (4
                        // consecutive columns), after which lane t holds row
                        // rb + t of the quad's columns
                        const int t = lane & 3;
                        const uint32_t snd = t < 2 ? pk.y : pk.x;
                        const uint32_t rcv = (uint32_t)__shfl_xor((int)snd, 2, 64);
                        const uint32_t a = t < 2 ? pk.x : rcv, b = t < 2 ? rcv : pk.y;   // rows of columns t & 1, + 2
                        const uint32_t s1 = (t & 1) ? ((a & 0xFFFFu) | (b << 16)) : ((a >> 16) | (b & 0xFFFF0000u));
                        const uint32_t r1 = (uint32_t)__shfl_xor((int)s1, 1, 64);
                        const uint2 row = (t & 1) ? make_uint2((r1 & 0xFFFFu) | (a & 0xFFFF0000u),
                                                               (r1 >> 16) | (b & 0xFFFF0000u))
                                                  : make_uint2((a & 0xFFFFu) | (r1 << 16),
                                                               (b & 0xFFFFu) | (r1 & 0xFFFF0000u));
                        *(uint2 *)(g.H + (uint32_t)((col / DU1_SLICE) * g.M * DU1_SLICE + (rb + t) * DU1_SLICE +
                                                    (col - t) % DU1_SLICE)) = row;
                    }
                }
            }
            if (MS == 32 && EPI != EPI_STORE && g.HT) {
                // the transposed copy in 16-byte pieces: lanes l and l + 32
                // hold rows 8 q .. 8 q + 3 and 8 q + 4 .. 8 q + 7 of a column;
                // they swap halves so that lane l writes rows 0 .. 15 and
                // lane l + 32 rows 16 .. 31 of the tile, 8 at a time
                const bool lo = lane < 32;
                const uint2 s0 = lo ? pkq[2 % QN] : pkq[0], s1 = lo ? pkq[3 % QN] : pkq[1 % QN];
                const uint2 r0 = make_uint2((uint32_t)__shfl_xor((int)s0.x, 32, 64), (uint32_t)__shfl_xor((int)s0.y, 32, 64));
                const uint2 r1 = make_uint2((uint32_t)__shfl_xor((int)s1.x, 32, 64), (uint32_t)__shfl_xor((int)s1.y, 32, 64));
                const uint4 w0 = lo ? make_uint4(pkq[0].x, pkq[0].y, r0.x, r0.y)
                                    : make_uint4(r0.x, r0.y, pkq[2 % QN].x, pkq[2 % QN].y);
                const uint4 w1 = lo ? make_uint4(pkq[1 % QN].x, pkq[1 % QN].y, r1.x, r1.y)
                                    : make_uint4(r1.x, r1.y, pkq[3 % QN].x, pkq[3 % QN].y);
                uint16_t *ht = g.HT + (int64_t)col * g.ldt + m0 + wm * WT + ti * MS + (lo ? 0 : 16);
                *(uint4 *)ht = w0;
                *(uint4 *)(ht + 8) = w1;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Layer 3 and the loss.  One wave per sample, L3_ROWS samples per workgroup:
// h2 = GELU(u2) in fp32, y = h2 . W3 + b3.  Training also forms
// dy = 2 (y - t) / n and du2 = dy * W3 * GELU'(u2) (bf16, row-major and
// transposed; the transposed rows of the workgroup's samples go out through
// LDS, 32 contiguous bytes per output).
// ---------------------------------------------------------------------------
constexpr int L3_ROWS = 16;
static_assert(L3_ROWS == 16 && N_H2 == 256, "a thread per output writes two 16-byte pieces");
__global__ __launch_bounds__(256) void layer3_kernel(L3Args a)
{
    __shared__ __align__(16) uint16_t t2[L3_ROWS][N_H2];   // du2 of the workgroup's samples
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int base = blockIdx.x * L3_ROWS;
#pragma unroll
    for (int r = w; r < L3_ROWS; r += 4) {
        const int b = base + r;
        if (b >= a.n) break;
        float u[4], h[4], s = 0.f;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int j = lane + 64 * q;
            u[q] = a.U2[(int64_t)b * N_H2 + j];
            h[q] = gelu_f(u[q]);
            s += h[q] * a.W3[j];
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
        const float y = s + a.b3[0];
        if (a.target == nullptr) {
            if (lane == 0) a.pred[b] = y * a.std + a.mean;
            continue;
        }
        const float t = a.target[b];
        const float dy = 2.0f * (y - t) / (float)a.n_batch;
        if (lane == 0) {
            a.dy[b] = dy;
            a.sq[b] = (y - t) * (y - t);
            if (a.pred) a.pred[b] = y;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int j = lane + 64 * q;
            a.H2[(int64_t)b * N_H2 + j] = h[q];
            const uint16_t v = f2bf(dy * a.W3[j] * gelu_grad_f(u[q]));
            a.DU2[(int64_t)b * N_H2 + j] = v;
            t2[r][j] = v;
        }
    }
    if (a.target == nullptr) return;             // the same for the whole grid
    __syncthreads();
    // du2 transposed: output j = thread, the workgroup's samples
    const int j = threadIdx.x;
    uint16_t *dst = a.DU2T + (int64_t)j * a.ld_t + base;
    if (base + L3_ROWS <= a.n) {
        uint32_t wv[L3_ROWS / 2];
#pragma unroll
        for (int r = 0; r < L3_ROWS; r += 2) wv[r / 2] = (uint32_t)t2[r][j] | ((uint32_t)t2[r + 1][j] << 16);
        ((uint4 *)dst)[0] = make_uint4(wv[0], wv[1], wv[2], wv[3]);
        ((uint4 *)dst)[1] = make_uint4(wv[4], wv[5], wv[6], wv[7]);
    } else {
        for (int r = 0; base + r < a.n; r++) dst[r] = t2[r][j];
    }
}

// Gradients that are sums over the batch, in a fixed order (deterministic):
// gW3[j] = sum_b h2[b][j] dy[b], gb3 = sum_b dy[b], gb2[j] = sum_b du2[b][j],
// gb1[i] = sum_b du1[b][i] (du from the transposed bf16 copies), the loss,
// and gW2 as the sum of its split-K parts.  Workgroups by task:
//   [0, W3_SLICES): gW3 over a slice of the batch, one thread per output
//     (rows of h2 read whole); the last of them to finish adds the slices;
//   then one wave per output of gb3, gb2, gb1 and the loss;
//   then 1,024 outputs of gW2 per workgroup (if split).
__global__ __launch_bounds__(256) void batch_sums_kernel(SumArgs a)
{
    const int tid = threadIdx.x, lane = tid & 63;
    int blk = blockIdx.x;
    if (blk < W3_SLICES) {
        __shared__ int last;
        const int per = (a.n + W3_SLICES - 1) / W3_SLICES;
        const int b0 = min(a.n, blk * per), b1 = min(a.n, b0 + per);
        float s = 0.f;
#pragma unroll 16
        for (int b = b0; b < b1; b++) s += a.H2[(int64_t)b * N_H2 + tid] * a.dy[b];
        a.w3part[blk * N_H2 + tid] = s;
        __threadfence();
        __syncthreads();
        if (tid == 0) last = atomicAdd(a.w3ctr, 1u) == (uint32_t)(W3_SLICES - 1);
        __syncthreads();
        if (last) {
            __threadfence();
            float t = 0.f;
#pragma unroll 16
            for (int k = 0; k < W3_SLICES; k++)
                t += __hip_atomic_load(&a.w3part[k * N_H2 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            a.gW3[tid] = t;
            if (tid == 0) atomicExch(a.w3ctr, 0u);   // zero for the next call
        }
        return;
    }
    blk -= W3_SLICES;
    const int n_rows = 1 + N_H2 + N_H1 + 1;
    const int row_blocks = (n_rows + 3) / 4;
    if (blk < row_blocks) {
        const int row = blk * 4 + (tid >> 6);   // one wave per output
        if (row >= n_rows) return;
        // n is a multiple of 128: 16-byte loads, 8 bf16 or 4 floats a lane
        float s = 0.f;
        if (row == 0 || row == n_rows - 1) {
            const float *x = row == 0 ? a.dy : a.sq;
            for (int b = lane * 4; b < a.n; b += 256) {
                const float4 v = *(const float4 *)(x + b);
                s += (v.x + v.y) + (v.z + v.w);
            }
        } else {
            const uint16_t *x = row < 1 + N_H2 ? a.DU2T + (int64_t)(row - 1) * a.ld_t
                                               : a.DU1T + (int64_t)(row - 1 - N_H2) * a.ld_t;
            for (int b = lane * 8; b < a.n; b += 512) {
                const uint4 v = *(const uint4 *)(x + b);
                const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 4; e++) s += bf2f((uint16_t)(w4[e] & 0xFFFFu)) + bf2f((uint16_t)(w4[e] >> 16));
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
        if (lane != 0) return;
        if (row == 0) a.gb3[0] = s;
        else if (row < 1 + N_H2) a.gb2[row - 1] = s;
        else if (row < 1 + N_H2 + N_H1) a.gb1[row - 1 - N_H2] = s;
        else a.loss[0] = s / (float)a.n;
        return;
    }
    blk -= row_blocks;
    const int64_t i = ((int64_t)blk * 256 + tid) * 4;
    if (a.w2part) {
        float4 t = *(const float4 *)(a.w2part + i);
        for (int k = 1; k < a.w2_splits; k++) {
            const float4 u = *(const float4 *)(a.w2part + k * a.w2_stride + i);
            t.x += u.x;
            t.y += u.y;
            t.z += u.z;
            t.w += u.w;
        }
        *(float4 *)(a.gW2 + i) = t;
    }
}

// ---------------------------------------------------------------------------
// dW1 without the product.  The input is one-hot per category, so
//   dW1[h][c * 64 + z] = sum of du1[s][h] over the samples s whose category c
//   lies in zone z:
// one sum of du1 rows per (category, zone) bin, 1/64 of the arithmetic of the
// dense product.  du1 comes in column slices of 128 hidden units, [8][n][128].
// Workgroup b takes category c = b / 8 and slice b % 8, two units per lane;
// consecutive workgroups go to different XCDs, so that each XCD reads one
// slice, a contiguous 256 KB per 1,024 samples that its L2 holds.
//   1. The batch's samples are sorted by their zone of category c, stably
//      (ties in sample order), into LDS: so every sum runs in a fixed order.
//      A sample's rank among the earlier samples of its group of 64 in its
//      bin comes from ballots (one per bit of the bin), its wave's running
//      count per bin from LDS.
//   2. The eight waves take equal shares of the sorted positions and add each
//      bin's rows in fp32 in list order; a bin that crosses into a wave's
//      share from an earlier one is finished there, and its parts are added
//      in wave order.
// Categories at or beyond n_cat get zeros; zone bytes of 64 or more fall in
// no bin.
// ---------------------------------------------------------------------------
constexpr int W1_SLICE = DU1_SLICE;
constexpr int W1_UNITS = W1_SLICE / 64;                      // hidden units per lane
constexpr int W1_SLICES = N_H1 / W1_SLICE;
constexpr int W1_WAVES = 16;
static_assert(W1_UNITS == 4, "four units per lane, one 8-byte load");
static_assert(8 % W1_SLICES == 0, "slices spread evenly over 8 XCDs");
constexpr int W1_GROUPS = MAX_GRAD_ROWS / (64 * W1_WAVES);   // groups of 64 samples per wave when sorting

__global__ __launch_bounds__(64 * W1_WAVES) void w1_grad_kernel(const uint16_t *du1, const uint8_t *zt, int n,
                                                                int n_cat, float *gW1)
{
    __shared__ float out[W1_SLICE][65];
    __shared__ float head[W1_WAVES][W1_SLICE];
    __shared__ int headz[W1_WAVES];
    __shared__ uint32_t cnt[W1_WAVES][64];      // per wave: samples per bin, then its first position per bin
    __shared__ __align__(16) uint32_t sidx[MAX_GRAD_ROWS];   // sorted samples, as byte offsets of their rows
    __shared__ int32_t soff[65];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform, so that the loops run on scalars
    // XCD x = b % 8 serves slice x / (8 / W1_SLICES)
    constexpr int XPS = 8 / W1_SLICES;                       // XCDs per slice
    const int x = (int)blockIdx.x & 7;
    const int c = ((int)blockIdx.x >> 3) * XPS + x % XPS, sl = x / XPS, h0 = sl * W1_SLICE;
    for (int k = tid; k < W1_SLICE * 65; k += 64 * W1_WAVES) (&out[0][0])[k] = 0.f;
    if (tid < W1_WAVES) headz[tid] = -1;
    const int per_s = (n + 64 * W1_WAVES - 1) / (64 * W1_WAVES) * 64;   // samples per wave, whole groups
    uint32_t zr[W1_GROUPS];                     // bin | rank << 8
    if (c < n_cat) {
        cnt[w][lane] = 0u;
#pragma unroll
        for (int g = 0; g < W1_GROUPS; g++) {
            const int sm = w * per_s + g * 64 + lane;
            zr[g] = g * 64 < per_s && sm < n ? min((uint32_t)zt[(int64_t)c * n + sm], 64u) : 64u;
        }
#pragma unroll
        for (int g = 0; g < W1_GROUPS; g++) {
            const uint32_t z = zr[g];
            uint64_t m = ~0ull;                 // the lanes that share this lane's bin
#pragma unroll
            for (int b = 0; b < 7; b++) {
                const uint64_t bb = __ballot((z >> b) & 1u);
                m &= ((z >> b) & 1u) ? bb : ~bb;
            }
            const uint32_t below = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            const uint32_t base = z < 64u ? cnt[w][z] : 0u;
            zr[g] = z | ((base + below) << 8);
            // the highest lane of each bin advances the bin's count
            if (z < 64u && (m >> lane) == 1ull) cnt[w][z] = base + (uint32_t)__popcll(m);
        }
    }
    __syncthreads();
    if (c < n_cat && w == 0) {
        // bins in order and, within a bin, the waves in order (sample order)
        uint32_t t[W1_WAVES], tot = 0;
#pragma unroll
        for (int k = 0; k < W1_WAVES; k++) {
            t[k] = cnt[k][lane];
            tot += t[k];
        }
        uint32_t inc = tot;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t u = __shfl_up(inc, d, 64);
            if (lane >= d) inc += u;
        }
        uint32_t run = inc - tot;
        soff[lane] = (int32_t)run;
        if (lane == 63) soff[64] = (int32_t)inc;
#pragma unroll
        for (int k = 0; k < W1_WAVES; k++) {
            cnt[k][lane] = run;
            run += t[k];
        }
    }
    __syncthreads();
    if (c < n_cat) {
#pragma unroll
        for (int g = 0; g < W1_GROUPS; g++) {
            const uint32_t z = zr[g] & 0xFFu;
            if (z < 64u) sidx[cnt[w][z] + (zr[g] >> 8)] = (uint32_t)(w * per_s + g * 64 + lane) * (2u * W1_SLICE);
        }
        // the last block of a share may read up to 15 positions past the
        // sorted ones: they name row 0 (and are not added)
        const int nv = soff[64];
        if (tid < 16 && nv + tid < MAX_GRAD_ROWS) sidx[nv + tid] = 0u;
    }
    __syncthreads();
    if (c < n_cat) {
        const int nv = __builtin_amdgcn_readfirstlane(soff[64]);
        const int per = (nv + 16 * W1_WAVES - 1) / (16 * W1_WAVES) * 16;   // positions per wave, whole blocks of 16
        const int i0 = min(nv, w * per), i1 = min(nv, i0 + per);
        if (i0 < i1) {
            int z = 0;
            while (soff[z + 1] <= i0) z++;
            z = __builtin_amdgcn_readfirstlane(z);
            int zend = __builtin_amdgcn_readfirstlane(soff[z + 1]);
            bool first = __builtin_amdgcn_readfirstlane(soff[z]) < i0;   // the bin began in an earlier share
            float a[W1_UNITS];
#pragma unroll
            for (int u = 0; u < W1_UNITS; u++) a[u] = 0.f;
            // the slice as a buffer: a position's row offset is uniform and
            // goes in a scalar register, the lane's units are the vector offset
            const __amdgpu_buffer_rsrc_t slice = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(du1 + (int64_t)sl * n * W1_SLICE), 0, n * 2 * W1_SLICE, 0x00020000);
            const int lane_off = 2 * W1_UNITS * lane;
            using Row = u32x2;
            auto ld = [&](int so) -> Row { return __builtin_amdgcn_raw_buffer_load_b64(slice, lane_off, so, 0); };
            auto add = [&](const Row &r) {
                a[0] += __uint_as_float(r[0] << 16);
                a[1] += __uint_as_float(r[0] & 0xFFFF0000u);
                a[2] += __uint_as_float(r[1] << 16);
                a[3] += __uint_as_float(r[1] & 0xFFFF0000u);
            };
            auto flush = [&](bool to_head) {
#pragma unroll
                for (int u = 0; u < W1_UNITS; u++) {
                    if (to_head) head[w][W1_UNITS * lane + u] = a[u];
                    else out[W1_UNITS * lane + u][z] = a[u];
                    a[u] = 0.f;
                }
                if (to_head && lane == 0) headz[w] = z;
            };
            // the rows of block i + 16 load while block i is added; a block's
            // positions past i1 read a row that is not added
            Row v[16], nx[16];
            auto load16 = [&](int i, Row *dst) {
#pragma unroll
                for (int k4 = 0; k4 < 4; k4++) {
                    const uint4 q = *(const uint4 *)&sidx[i + 4 * k4];
                    const uint32_t qw[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int k = 0; k < 4; k++) dst[4 * k4 + k] = ld(__builtin_amdgcn_readfirstlane((int)qw[k]));
                }
            };
            load16(i0, nx);
            for (int i = i0; i < i1; i += 16) {
#pragma unroll
                for (int k = 0; k < 16; k++) v[k] = nx[k];
                if (i + 16 < i1) load16(i + 16, nx);
                if (i + 16 <= min(zend, i1)) {
                    // the whole block lies in bin z
#pragma unroll
                    for (int k = 0; k < 16; k++) add(v[k]);
                    continue;
                }
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    if (i + k >= i1) break;
                    while (i + k == zend) {                // leave bin z
                        flush(first);
                        first = false;
                        z++;
                        zend = __builtin_amdgcn_readfirstlane(soff[z + 1]);
                    }
                    add(v[k]);
                }
            }
            flush(first);
        }
    }
    __syncthreads();
    if (tid < W1_SLICE) {
#pragma unroll
        for (int k = 1; k < W1_WAVES; k++)
            if (headz[k] >= 0) out[tid][headz[k]] += head[k][tid];
    }
    __syncthreads();
    for (int k = tid; k < W1_SLICE * 64; k += 64 * W1_WAVES) {
        const int r = k >> 6, j = k & 63;
        gW1[(int64_t)(h0 + r) * N_IN + c * 64 + j] = out[r][j];
    }
}

// Zone bytes by category: zt[c * n + b] = zb[b * 64 + c], one wave per sample.
__global__ __launch_bounds__(256) void zone_cols_kernel(const uint8_t *zb, int n, uint8_t *zt)
{
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (b < n) zt[(int64_t)lane * n + b] = zb[(int64_t)b * 64 + lane];
}

// Adam over the flat fp32 parameter vector (Kingma & Ba 2015, bias-corrected).
// Adam over the fp32 masters; the updated W1 and W2 also go straight to
// their bf16 working copies (W2 in both layouts), as refresh_bf16_kernel does.
__global__ __launch_bounds__(256) void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n,
                                                   float lr, float beta1, float beta2, float eps, float bc1,
                                                   float bc2, uint16_t *W1b, uint16_t *W2b, uint16_t *W2kn)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
        const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
        p[i] = pi;
        if (W1b && i < P_W1 + (int64_t)N_H1 * N_IN) {
            W1b[i - P_W1] = f2bf(pi);
        } else if (W1b && i >= P_W2 && i < P_W2 + (int64_t)N_H2 * N_H1) {
            const int64_t k = i - P_W2;                 // W2 [j][i2], j < 256, i2 < 1024
            const uint16_t h = f2bf(pi);
            W2b[k] = h;
            W2kn[(k % N_H1) * N_H2 + k / N_H1] = h;
        }
    }
}

// bf16 working copies: W1 [1024][4096] and W2 [256][1024] as stored, plus W2
// transposed to [1024][256] for the backward product.
__global__ __launch_bounds__(256) void refresh_bf16_kernel(const float *W1t, const float *W2t, uint16_t *W1b,
                                                           uint16_t *W2b, uint16_t *W2kn)
{
    const int64_t n1 = (int64_t)N_H1 * N_IN, n2 = (int64_t)N_H2 * N_H1;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n1 + n2; i += (int64_t)gridDim.x * 256) {
        if (i < n1) {
            W1b[i] = f2bf(W1t[i]);
        } else {
            const int64_t k = i - n1;               // W2t[j][i2], j < 256, i2 < 1024
            const int64_t j = k / N_H1, i2 = k % N_H1;
            const uint16_t v = f2bf(W2t[k]);
            W2b[k] = v;
            W2kn[i2 * N_H2 + j] = v;
        }
    }
}

// Gather a batch: zone rows and standardised targets of the given samples.
// A keyed pseudorandom permutation of [0, n): a four-round balanced Feistel
// network on 2h bits (2^2h >= n) whose round function is the SplitMix64
// finaliser of (key, round, half), with cycle walking -- values at or above
// n are encrypted again until they fall inside, which keeps a bijection of
// [0, n) (Black and Rogaway 2002).  The training shuffle is computed where the
// batch is gathered, with no table and no host work.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t feistel_perm(uint64_t x, uint64_t n, int h, uint64_t key)
{
    const uint64_t mask = (1ull << h) - 1ull;
    do {
        uint64_t l = x >> h, r = x & mask;
        for (int round = 0; round < 4; round++) {
            const uint64_t f = mix64(key + 0x9E3779B97F4A7C15ull * (uint64_t)(round + 1) + r) & mask;
            const uint64_t t = l ^ f;
            l = r;
            r = t;
        }
        x = (l << h) | r;
    } while (x >= n);
    return x;
}

__global__ __launch_bounds__(256) void gather_batch_kernel(const uint8_t *zone, const int32_t *dist, int64_t n_all,
                                                           int h, uint64_t key, int64_t first, int n, double mean,
                                                           double inv_std, uint8_t *zb, uint8_t *zt, float *tb)
{
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (b >= n) return;
    const int64_t s = (int64_t)feistel_perm((uint64_t)(first + b), (uint64_t)n_all, h, key);
    const uint8_t zv = zone[s * 64 + lane];
    zb[(int64_t)b * 64 + lane] = zv;
    zt[(int64_t)lane * n + b] = zv;
    if (lane == 0) tb[b] = (float)(((double)dist[s] - mean) * inv_std);
}

// Mean and standard deviation of int32 distances (two fixed-order passes,
// one block, double accumulation).
__global__ __launch_bounds__(1024) void moments_kernel(const int32_t *d, int64_t n, double *out)
{
    __shared__ double part[1024];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += (double)d[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int st = 512; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
        __syncthreads();
    }
    const double mean = part[0] / (double)n;
    __syncthreads();
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const double e = (double)d[i] - mean;
        q += e * e;
    }
    part[threadIdx.x] = q;
    __syncthreads();
    for (int st = 512; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = mean;
        out[1] = sqrt(part[0] / (double)n);
    }
}

// ---------------------------------------------------------------------------
// Top-k of n predictions by (value, index), one workgroup: radix selection of
// the k-th smallest value over its order-preserving bit pattern, ties taken
// in index order, then a bitonic sort of the k winners in LDS.
// ---------------------------------------------------------------------------
static __device__ __forceinline__ uint32_t order_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int TOPK_THREADS = 1024;

// MODE 0: keys are float predictions (smallest first).  MODE 1: keys are int32
// distances, largest first (the worst individuals of a population).
template <int MODE>
static __device__ __forceinline__ uint32_t topk_key(const void *src, int i)
{
    if (MODE == 0) return order_key(((const float *)src)[i]);
    const int32_t d = ((const int32_t *)src)[i];
    return (uint32_t)(0x7FFFFFFF - (d < 0 ? 0 : d));
}

template <int MODE>
__global__ __launch_bounds__(TOPK_THREADS) void topk_kernel(const void *src, int n, int k, int32_t *out)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t sel[2];               // prefix found so far, remaining rank
    __shared__ uint32_t cnt_lt[TOPK_THREADS];
    __shared__ uint32_t cnt_eq[TOPK_THREADS];
    __shared__ unsigned long long keys[TOPK_MAX];
    const int tid = threadIdx.x;
    if (tid == 0) { sel[0] = 0; sel[1] = (uint32_t)k; }
    __syncthreads();
    // k-th smallest key: 4 passes of 8 bits from the top
    for (int pass = 0; pass < 4; pass++) {
        const int shift = 24 - 8 * pass;
        if (tid < 256) hist[tid] = 0;
        __syncthreads();
        const uint32_t prefix = sel[0];
        const uint32_t hi_mask = pass == 0 ? 0u : (0xFFFFFFFFu << (shift + 8));
        for (int i = tid; i < n; i += TOPK_THREADS) {
            const uint32_t key = topk_key<MODE>(src, i);
            if ((key & hi_mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t rem = sel[1], acc = 0;
            int digit = 0;
            for (; digit < 256; digit++) {
                if (acc + hist[digit] >= rem) break;
                acc += hist[digit];
            }
            sel[0] = prefix | ((uint32_t)digit << shift);
            sel[1] = rem - acc;
        }
        __syncthreads();
    }
    const uint32_t kth = sel[0];
    const uint32_t ties_needed = sel[1];          // how many keys equal to kth to keep
    // keep keys < kth, and the first ties_needed keys == kth in index order
    const int per = (n + TOPK_THREADS - 1) / TOPK_THREADS;
    const int i0 = min(n, tid * per), i1 = min(n, i0 + per);
    uint32_t lt = 0, eq = 0;
    for (int i = i0; i < i1; i++) {
        const uint32_t key = topk_key<MODE>(src, i);
        lt += key < kth;
        eq += key == kth;
    }
    // inclusive scans of lt and eq over the threads (index order)
    cnt_lt[tid] = lt;
    cnt_eq[tid] = eq;
    __syncthreads();
    for (int d = 1; d < TOPK_THREADS; d <<= 1) {
        const uint32_t a = tid >= d ? cnt_lt[tid - d] : 0u;
        const uint32_t b = tid >= d ? cnt_eq[tid - d] : 0u;
        __syncthreads();
        cnt_lt[tid] += a;
        cnt_eq[tid] += b;
        __syncthreads();
    }
    const uint32_t total_lt = cnt_lt[TOPK_THREADS - 1];
    uint32_t pos_lt = cnt_lt[tid] - lt, pos_eq = cnt_eq[tid] - eq;
    for (int i = i0; i < i1; i++) {
        const uint32_t key = topk_key<MODE>(src, i);
        if (key < kth) {
            keys[pos_lt++] = ((unsigned long long)key << 32) | (uint32_t)i;
        } else if (key == kth) {
            if (pos_eq < ties_needed) keys[total_lt + pos_eq] = ((unsigned long long)key << 32) | (uint32_t)i;
            pos_eq++;
        }
    }
    int P2 = 1;
    while (P2 < k) P2 <<= 1;
    for (int i = k + tid; i < P2; i += TOPK_THREADS) keys[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < P2; i += TOPK_THREADS) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long a = keys[i], b = keys[j];
                    if ((a > b) == up) { keys[i] = b; keys[j] = a; }
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < k; i += TOPK_THREADS) out[i] = (int32_t)(keys[i] & 0xFFFFFFFFull);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// 128 x 128 tiles when they give at least one workgroup per CU, else 64 x 64.
// MFMA shape: 32 x 32 x 16 where there is about one workgroup per CU (the
// training products: 5 % faster); 16 x 16 x 32 for the large screening
// passes (at least 1,024 workgroups: 3 % faster)
template <int AM, int BM, int EP>
static hipError_t launch_gemm_t(const GemmArgs &g, hipStream_t s)
{
    const int ks = g.ksplit > 1 ? g.ksplit : 1;
    const int64_t t128 = (int64_t)(g.N / 128) * (g.M / 128) * ks;
    // a short K (dU1: 256) leaves the epilogue most of a workgroup's time:
    // 64 x 64 tiles, so that four workgroups per CU overlap their epilogues
    if (g.K <= 256 && t128 < 1024) {
        hipLaunchKernelGGL((gemm_kernel<AM, BM, EP, 64, 32>), dim3(g.N / 64, g.M / 64, ks), dim3(256), 0, s, g);
    } else if (t128 >= 1024) {
        hipLaunchKernelGGL((gemm_kernel<AM, BM, EP, 128, 16>), dim3(g.N / 128, g.M / 128, ks), dim3(256), 0, s, g);
    } else if (t128 >= 256) {
        hipLaunchKernelGGL((gemm_kernel<AM, BM, EP, 128, 32>), dim3(g.N / 128, g.M / 128, ks), dim3(256), 0, s, g);
    } else {
        hipLaunchKernelGGL((gemm_kernel<AM, BM, EP, 64, 32>), dim3(g.N / 64, g.M / 64, ks), dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

hipError_t launch_gemm(int amode, int bmode, int epi, const GemmArgs &g, hipStream_t s)
{
    if (g.M % 128 || g.N % 128 || g.K % GBK) return hipErrorInvalidValue;
    if (g.ksplit > 1 && (epi != EPI_STORE || g.K % (g.ksplit * GBK))) return hipErrorInvalidValue;
    if ((int64_t)g.M * g.ldc >= (int64_t)1 << 31) return hipErrorInvalidValue;   // 32-bit output offsets
    if (amode == A_ONEHOT && bmode == B_BF16 && epi == EPI_BIAS_GELU) return launch_gemm_t<A_ONEHOT, B_BF16, EPI_BIAS_GELU>(g, s);
    if (amode == A_BF16 && bmode == B_BF16 && epi == EPI_BIAS_GELU) return launch_gemm_t<A_BF16, B_BF16, EPI_BIAS_GELU>(g, s);
    if (amode == A_BF16 && bmode == B_BF16 && epi == EPI_STORE) return launch_gemm_t<A_BF16, B_BF16, EPI_STORE>(g, s);
    if (amode == A_BF16 && bmode == B_BF16 && epi == EPI_GELU_GRAD_T) return launch_gemm_t<A_BF16, B_BF16, EPI_GELU_GRAD_T>(g, s);
    return hipErrorInvalidValue;
}

hipError_t launch_layer3(const L3Args &a, hipStream_t s)
{
    if (a.target && (a.ld_t % 8 || a.n > a.ld_t)) return hipErrorInvalidValue;   // 16-byte rows of du2^T
    hipLaunchKernelGGL(layer3_kernel, dim3((a.n + L3_ROWS - 1) / L3_ROWS), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_sums(const SumArgs &a, hipStream_t s)
{
    const int n_rows = 1 + N_H2 + N_H1 + 1;
    const int blocks = W3_SLICES + (n_rows + 3) / 4 + (a.w2part ? N_H2 * N_H1 / 1024 : 0);
    hipLaunchKernelGGL(batch_sums_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, int step,
                       uint16_t *W1b, uint16_t *W2b, uint16_t *W2kn, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.0f - powf(b1, (float)step), bc2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(2048), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, 1e-8f, bc1, bc2, W1b,
                       W2b, W2kn);
    return hipGetLastError();
}

hipError_t launch_refresh_bf16(const float *W1t, const float *W2t, uint16_t *W1b, uint16_t *W2b, uint16_t *W2kn,
                               hipStream_t s)
{
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3(2048), dim3(256), 0, s, W1t, W2t, W1b, W2b, W2kn);
    return hipGetLastError();
}

hipError_t launch_zone_cols(const uint8_t *zb, int n, uint8_t *zt, hipStream_t s)
{
    hipLaunchKernelGGL(zone_cols_kernel, dim3((n + 3) / 4), dim3(256), 0, s, zb, n, zt);
    return hipGetLastError();
}

hipError_t launch_w1_grad(const uint16_t *du1, const uint8_t *zt, int n, int n_cat, float *gW1, hipStream_t s)
{
    if (n < 1 || n > MAX_GRAD_ROWS || n_cat < 1 || n_cat > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(w1_grad_kernel, dim3(64 * W1_SLICES), dim3(64 * W1_WAVES), 0, s, du1, zt, n, n_cat,
                       gW1);
    return hipGetLastError();
}

hipError_t launch_gather_batch(const uint8_t *zone, const int32_t *dist, int64_t n_all, int h, uint64_t key,
                               int64_t first, int n, double mean, double inv_std, uint8_t *zb, uint8_t *zt,
                               float *tb, hipStream_t s)
{
    hipLaunchKernelGGL(gather_batch_kernel, dim3((n + 3) / 4), dim3(256), 0, s, zone, dist, n_all, h, key, first, n,
                       mean, inv_std, zb, zt, tb);
    return hipGetLastError();
}

hipError_t launch_moments(const int32_t *d, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(moments_kernel, dim3(1), dim3(1024), 0, s, d, n, out);
    return hipGetLastError();
}

hipError_t launch_topk(const float *pred, int n, int k, int32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(topk_kernel<0>, dim3(1), dim3(TOPK_THREADS), 0, s, (const void *)pred, n, k, out);
    return hipGetLastError();
}

hipError_t launch_worst(const int32_t *dist, int n, int k, int32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(topk_kernel<1>, dim3(1), dim3(TOPK_THREADS), 0, s, (const void *)dist, n, k, out);
    return hipGetLastError();
}

}  // namespace wo
