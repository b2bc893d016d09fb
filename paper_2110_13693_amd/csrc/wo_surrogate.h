// Internal interface between the surrogate host code and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wo {

constexpr int N_IN = 4096;   // 64 categories x 64 zones, one-hot
constexpr int N_H1 = 1024;
constexpr int N_H2 = 256;
constexpr int TOPK_MAX = 4096;
constexpr int MAX_GRAD_ROWS = 4096;   // samples per training batch
constexpr int DU1_SLICE = 256;        // du1 for the dW1 bins: column slices of this many hidden units

// flat parameter vector, [out][in] weight layout
constexpr int64_t P_W1 = 0;
constexpr int64_t P_B1 = P_W1 + (int64_t)N_H1 * N_IN;
constexpr int64_t P_W2 = P_B1 + N_H1;
constexpr int64_t P_B2 = P_W2 + (int64_t)N_H2 * N_H1;
constexpr int64_t P_W3 = P_B2 + N_H2;
constexpr int64_t P_B3 = P_W3 + N_H2;
constexpr int64_t P_TOTAL = P_B3 + 1;

enum { A_BF16 = 0, A_ONEHOT = 1 };
enum { B_BF16 = 0 };
enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD_T = 2 };

struct GemmArgs {
    int M, N, K;              // padded sizes (M, N multiples of 128, K of 64)
    int M_real;               // rows of the zone operand that exist
    int n_cat;                // categories that exist: zone bytes of higher ones are ignored
    const uint16_t *A;        // A_BF16: [M][lda]
    int lda;
    const uint8_t *zoneA;     // A_ONEHOT: zone rows [M_real][64]
    const uint16_t *B;        // B_BF16: [N][ldb]
    int ldb;
    float *C;                 // EPI_STORE: [M][ldc]
    int ldc;
    const float *bias;        // EPI_BIAS_GELU
    float *U;                 // EPI_BIAS_GELU: pre-activation [M][ldc] (may be null)
    uint16_t *H;              // bf16 result (may be null): EPI_BIAS_GELU [M][ldc], EPI_GELU_GRAD_T [N / DU1_SLICE][M][DU1_SLICE]
    uint16_t *HT;             // EPI_BIAS_GELU / EPI_GELU_GRAD_T: bf16 transposed [N][ldt]
    int ldt;
    const float *Uin;         // EPI_GELU_GRAD_T: pre-activation [M][ldc]
    int ksplit;               // EPI_STORE: K cut into ksplit equal parts (0 or 1: none), part z
    int64_t c_split;          // into C + z * c_split (partial products, summed by the caller)
};

struct L3Args {
    int n;                    // rows
    int n_batch;              // divisor of the mean loss
    const float *U2;          // [n][256]
    const float *W3;          // [256]
    const float *b3;          // [1]
    const float *target;      // standardised targets; null = prediction only
    float *pred;              // prediction (de-standardised when target is null)
    float mean, std;
    float *dy, *sq, *H2;      // training outputs
    uint16_t *DU2, *DU2T;
    int ld_t;
};

// gW3 is summed over W3_SLICES slices of the batch, then over the slices by
// the last of their workgroups (w3part, w3ctr: W3_SLICES * N_H2 floats and a
// counter that is zero between calls)
constexpr int W3_SLICES = 64;
struct SumArgs {
    int n;
    const float *H2, *dy, *sq;
    const uint16_t *DU2T, *DU1T;
    int ld_t;
    float *gW3, *gb3, *gb2, *gb1, *loss;
    float *w3part;
    uint32_t *w3ctr;
    const float *w2part;      // split-K parts of gW2 (w2_splits of them, w2_stride apart), or null
    int w2_splits;
    int64_t w2_stride;
    float *gW2;
};

hipError_t launch_gemm(int amode, int bmode, int epi, const GemmArgs &g, hipStream_t s);
hipError_t launch_layer3(const L3Args &a, hipStream_t s);
// zone bytes by category: zt [64][n] from the zone rows zb [n][64]
hipError_t launch_zone_cols(const uint8_t *zb, int n, uint8_t *zt, hipStream_t s);
// gW1 [1024][4096] of a batch of n samples (at most MAX_GRAD_ROWS) from its
// zone bytes by category zt [64][n] and du1 in column slices [N_H1 / DU1_SLICE][n][DU1_SLICE] (bf16)
hipError_t launch_w1_grad(const uint16_t *du1, const uint8_t *zt, int n, int n_cat, float *gW1, hipStream_t s);
hipError_t launch_batch_sums(const SumArgs &a, hipStream_t s);
// Adam step; when W1b is non-null the updated W1 and W2 are also written to
// their bf16 copies (W2 as stored and transposed), as launch_refresh_bf16 does
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, int step,
                       uint16_t *W1b, uint16_t *W2b, uint16_t *W2kn, hipStream_t s);
hipError_t launch_refresh_bf16(const float *W1t, const float *W2t, uint16_t *W1b, uint16_t *W2b, uint16_t *W2kn,
                               hipStream_t s);
hipError_t launch_gather_batch(const uint8_t *zone, const int32_t *dist, int64_t n_all, int h, uint64_t key,
                               int64_t first, int n, double mean, double inv_std, uint8_t *zb, uint8_t *zt,
                               float *tb, hipStream_t s);
hipError_t launch_moments(const int32_t *d, int64_t n, double *out, hipStream_t s);
hipError_t launch_topk(const float *pred, int n, int k, int32_t *out, hipStream_t s);
hipError_t launch_worst(const int32_t *dist, int n, int k, int32_t *out, hipStream_t s);

}  // namespace wo
