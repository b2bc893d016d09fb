// Order categories by linear support vector machines (arXiv 2110.13693,
// section 5, subroutine 5): each order belongs to a category of orders; an
// SVM (Cortes and Vapnik 1995) learns the categories from the outputs of the
// subroutines before it, and is refreshed continuously from a window of the
// most recent orders, newer data replacing older.
//
// Readings (the paper gives no features, model or training rule):
//   - an order's features are the shares of its lines in each product
//     category (the classes of Subproblem 3): x[c] = lines in c / lines;
//   - one linear SVM per category of orders against the rest: hinge loss
//     plus lambda / 2 times the squared norm of the weights, the bias being
//     the weight of a constant feature 1; full-batch subgradient steps over
//     the window with the step sizes of Pegasos (Shalev-Shwartz et al.
//     2007), eta_t = 1 / (lambda t), t counting every step since creation;
//   - an order takes the category of the largest score (ties: the lower).
// The window is a ring of the last `window` samples on the device.  Every
// sum runs in a fixed order (features in index order, samples from the
// oldest) with one IEEE double operation at a time, so the results do not
// depend on the launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <new>

#include "wo_common.h"

// one IEEE operation at a time: no multiply-add contraction anywhere below
// (the file is also built with -ffp-contract=off)
#pragma clang fp contract(off)

struct wo_svm {
    int32_t F = 0, K = 0, W = 0;
    double lambda = 0.0;
    int64_t steps = 0;       // training steps so far
    int64_t pushed = 0;      // samples pushed so far; the window holds the last min(pushed, W)
    double *X = nullptr;     // [W][F], sample g in slot g mod W
    int32_t *L = nullptr;    // [W]
    double *Wt = nullptr;    // [K][F + 1], bias last
    int8_t *coef = nullptr;  // [W][K]: +1 / -1 inside the margin, 0 outside
    std::atomic<int> busy{0};
};

namespace {

struct SvmBusy {
    std::atomic<int> *f;
    bool ok;
    explicit SvmBusy(std::atomic<int> *flag) : f(flag)
    {
        int z = 0;
        ok = f->compare_exchange_strong(z, 1);
    }
    ~SvmBusy()
    {
        if (ok) f->store(0);
    }
};

int grid_for(int64_t n, int block) { return (int)std::min<int64_t>(std::max<int64_t>((n + block - 1) / block, 1), 65535); }

// Line counts per category, then shares, 64 orders per wave: each lane
// counts its order's lines in its own LDS row (lines clamped to
// [0, n_lines); SKUs outside [0, n_skus) and categories outside [0, F) count
// in the length only), then the wave writes the 64 rows of shares, one
// coalesced row per store (lane = feature).
constexpr int FT_LD = WO_SVM_MAX_FEATURES + 1;

__global__ __launch_bounds__(64) void features_kernel(const int32_t *off, const int32_t *skus, int32_t n_orders,
                                                     int64_t n_lines, const int32_t *sku_cat, int32_t n_skus,
                                                     int32_t F, double *x)
{
    __shared__ uint32_t cnt[64 * FT_LD];
    __shared__ double len[64];
    const int lane = threadIdx.x;
    for (int64_t o0 = (int64_t)blockIdx.x * 64; o0 < n_orders; o0 += (int64_t)gridDim.x * 64) {
        uint32_t *mine = cnt + lane * FT_LD;
        for (int32_t c = 0; c < F; c++) mine[c] = 0u;
        const int64_t o = o0 + lane;
        if (o < n_orders) {
            const int32_t a = off[o], b = off[o + 1];
            const int64_t l0 = std::max<int64_t>(a, 0), l1 = std::min<int64_t>(b, n_lines);
            for (int64_t l = l0; l < l1; l++) {
                const int32_t sk = skus[l];
                if (sk < 0 || sk >= n_skus) continue;
                const int32_t c = sku_cat[sk];
                if (c < 0 || c >= F) continue;
                mine[c] += 1u;
            }
            len[lane] = (double)(b - a);
        }
        asm volatile("" ::: "memory");   // a wave's LDS accesses take effect in program order
        const int32_t rows = (int32_t)std::min<int64_t>(64, n_orders - o0);
        for (int32_t r = 0; r < rows; r++)
            for (int32_t c = lane; c < F; c += 64) x[(o0 + r) * F + c] = (double)cnt[r * FT_LD + c] / len[r];
        asm volatile("" ::: "memory");
    }
}

__device__ __forceinline__ double score(const double *w, const double *x, int32_t F)
{
    double s = 0.0;
    for (int32_t f = 0; f < F; f++) s = s + w[f] * x[f];
    return s + w[F];
}

// One thread per (sample, class): inside the margin at the current weights?
__global__ void margin_kernel(const double *X, const int32_t *L, int32_t W, int64_t first, int64_t n, int32_t F,
                              int32_t K, const double *Wt, int8_t *coef)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n * K; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / K;
        const int32_t k = (int32_t)(q - i * K);
        const int64_t slot = (first + i) % W;
        const bool pos = L[slot] == k;
        const double s = score(Wt + (int64_t)k * (F + 1), X + slot * F, F);
        const double ys = pos ? s : -s;
        coef[i * K + k] = (int8_t)(ys < 1.0 ? (pos ? 1 : -1) : 0);
    }
}

// One thread per (class, weight): the subgradient step; the sum over the
// samples runs from the oldest, as in the step's definition.  The additions
// stay in order; the loads run a group of 32 samples ahead of them (two
// register buffers), since a weight's sum is one chain over the whole window
// and the loads' latency would otherwise set its pace.
constexpr int UP_U = 32;

__device__ __forceinline__ void update_load(const double *X, const int8_t *coef, int32_t W, int64_t i, int64_t slot,
                                            int32_t F, int32_t K, int32_t k, int32_t f, double (&v)[UP_U])
{
#pragma unroll
    for (int u = 0; u < UP_U; u++) {
        int64_t sl = slot + u;
        if (sl >= W) sl -= W;
        // every lane loads (the bias lane a feature it does not use), so
        // that no branch splits the loads of the group
        const double c = (double)coef[(i + u) * K + k];
        const double x = X[sl * F + (f < F ? f : F - 1)];
        v[u] = f < F ? c * x : c;
    }
}

__global__ __launch_bounds__(64) void update_kernel(const double *X, const int8_t *coef, int32_t W, int64_t first,
                                                   int64_t n, int32_t F, int32_t K, double *Wt, double lambda, double t)
{
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K * (F + 1)) return;
    const int32_t k = q / (F + 1), f = q - k * (F + 1);
    double g = 0.0;
    int64_t i = 0;
    int64_t slot = first;
    auto advance = [&](int64_t by) {
        slot += by;
        if (slot >= W) slot -= W;
    };
    const int64_t groups = n / UP_U;
    double a[UP_U], b[UP_U];
    if (groups > 0) update_load(X, coef, W, 0, slot, F, K, k, f, a);
    for (int64_t gi = 0; gi < groups; gi += 2) {
        // a holds group gi; load gi + 1 into b, then add a
        int64_t s1 = slot + UP_U;
        if (s1 >= W) s1 -= W;
        if (gi + 1 < groups) update_load(X, coef, W, i + UP_U, s1, F, K, k, f, b);
#pragma unroll
        for (int u = 0; u < UP_U; u++) g = g + a[u];
        i += UP_U;
        advance(UP_U);
        if (gi + 1 >= groups) break;
        // b holds group gi + 1; load gi + 2 into a, then add b
        s1 = slot + UP_U;
        if (s1 >= W) s1 -= W;
        if (gi + 2 < groups) update_load(X, coef, W, i + UP_U, s1, F, K, k, f, a);
#pragma unroll
        for (int u = 0; u < UP_U; u++) g = g + b[u];
        i += UP_U;
        advance(UP_U);
    }
    for (; i < n; i++) {
        const double c = (double)coef[i * K + k];
        g = g + (f < F ? c * X[slot * F + f] : c);
        if (++slot == W) slot = 0;
    }
    const double eta = 1.0 / (lambda * t);
    const double w = Wt[q];
    Wt[q] = w - eta * (lambda * w - g / (double)n);
}

// Prediction, one lane per order: the class of the largest score (ties: the
// lower class), a score being weights . features in feature order, then the
// bias, as in training: every wave takes 64 orders and streams their
// features through LDS in chunks of 8, read coalesced (8 lanes per 64-byte
// piece of a row; the next chunk in flight while the current one is
// multiplied), for up to 8 classes at a time; the weights sit in LDS for the
// whole grid stride.
constexpr int PK_CHUNK = 8, PK_LD = PK_CHUNK + 1, PK_KG = 8;

// A wave's LDS accesses take effect in program order, so a lane may read what
// another lane of its wave wrote before: only the compiler must keep the order.
__device__ __forceinline__ void wave_lds_order() { asm volatile("" ::: "memory"); }

__global__ __launch_bounds__(256) void predict_kernel(const double *X, int64_t n, int32_t F, int32_t K,
                                                     const double *Wt, int32_t *cls)
{
    extern __shared__ double lds[];
    const int32_t nw = K * (F + 1);
    double *wl = lds;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double *tile = lds + nw + w * 64 * PK_LD;
    for (int32_t e = tid; e < nw; e += 256) wl[e] = Wt[e];
    __syncthreads();
    for (int64_t i0 = ((int64_t)blockIdx.x * 4 + w) * 64; i0 < n; i0 += (int64_t)gridDim.x * 256) {
        const int32_t rows = (int32_t)std::min<int64_t>(64, n - i0);   // uniform in the wave
        const double *src = X + i0 * F;
        int32_t best = 0;
        double bs = 0.0;
        for (int32_t k0 = 0; k0 < K; k0 += PK_KG) {
            double acc[PK_KG];
#pragma unroll
            for (int j = 0; j < PK_KG; j++) acc[j] = 0.0;
            // a lane's 8 loads of a chunk: row idx / 8, feature idx % 8 of
            // the chunk (idx = t * 64 + lane)
            double nx[PK_CHUNK];
#pragma unroll
            for (int t = 0; t < PK_CHUNK; t++) {
                const int idx = t * 64 + lane, r = idx / PK_CHUNK, f = idx % PK_CHUNK;
                nx[t] = (r < rows && f < F) ? src[(int64_t)r * F + f] : 0.0;
            }
            for (int32_t c = 0; c < F; c += PK_CHUNK) {
                wave_lds_order();                // the previous chunk is read
#pragma unroll
                for (int t = 0; t < PK_CHUNK; t++) {
                    const int idx = t * 64 + lane, r = idx / PK_CHUNK, f = idx % PK_CHUNK;
                    tile[r * PK_LD + f] = nx[t];
                }
                wave_lds_order();
                if (c + PK_CHUNK < F) {
#pragma unroll
                    for (int t = 0; t < PK_CHUNK; t++) {
                        const int idx = t * 64 + lane, r = idx / PK_CHUNK, f = c + PK_CHUNK + idx % PK_CHUNK;
                        nx[t] = (r < rows && f < F) ? src[(int64_t)r * F + f] : 0.0;
                    }
                }
#pragma unroll
                for (int f = 0; f < PK_CHUNK; f++) {
                    if (c + f < F) {
                        const double xf = tile[lane * PK_LD + f];
#pragma unroll
                        for (int j = 0; j < PK_KG; j++)
                            if (k0 + j < K) acc[j] = acc[j] + wl[(k0 + j) * (F + 1) + c + f] * xf;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < PK_KG; j++) {
                const int32_t k = k0 + j;
                if (k < K) {
                    const double v = acc[j] + wl[k * (F + 1) + F];
                    if (k == 0 || v > bs) {
                        bs = v;
                        best = k;
                    }
                }
            }
        }
        if (lane < rows) cls[i0 + lane] = best;
    }
}

}  // namespace

extern "C" wo_status wo_order_features(const int32_t *d_order_offsets, const int32_t *d_order_skus, int32_t n_orders,
                                       int64_t n_lines, const int32_t *d_sku_category, int32_t n_skus,
                                       int32_t n_features, double *d_features, void *stream)
{
    if (!d_order_offsets || !d_order_skus || !d_sku_category || !d_features) return wo_fail(WO_E_INVAL, "NULL buffer");
    if (n_orders < 0 || n_lines < 0 || n_skus < 0) return wo_fail(WO_E_INVAL, "negative size");
    if (n_features < 1 || n_features > WO_SVM_MAX_FEATURES)
        return wo_fail(WO_E_RANGE, "n_features must be in 1 .. %d", WO_SVM_MAX_FEATURES);
    if (n_orders == 0) return WO_OK;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(features_kernel, dim3(grid_for(n_orders, 64)), dim3(64), 0, s, d_order_offsets, d_order_skus,
                       n_orders, n_lines, d_sku_category, n_skus, n_features, d_features);
    WO_HIP(hipGetLastError());
    return WO_OK;
}

extern "C" wo_status wo_svm_create(int32_t n_features, int32_t n_classes, int32_t window, double lambda,
                                   void *stream, wo_svm **out)
{
    if (!out) return wo_fail(WO_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n_features < 1 || n_features > WO_SVM_MAX_FEATURES)
        return wo_fail(WO_E_RANGE, "n_features must be in 1 .. %d", WO_SVM_MAX_FEATURES);
    if (n_classes < 2 || n_classes > WO_SVM_MAX_CLASSES)
        return wo_fail(WO_E_RANGE, "n_classes must be in 2 .. %d", WO_SVM_MAX_CLASSES);
    if (window < 1 || window > WO_SVM_MAX_WINDOW) return wo_fail(WO_E_RANGE, "window must be in 1 .. %d", WO_SVM_MAX_WINDOW);
    if (!(lambda > 0.0)) return wo_fail(WO_E_INVAL, "lambda must be > 0");
    if (wo_fault_injected()) return wo_fail(WO_E_NOMEM, "injected allocation failure");
    wo_svm *m = new (std::nothrow) wo_svm;
    if (!m) return wo_fail(WO_E_NOMEM, "host allocation failed");
    m->F = n_features;
    m->K = n_classes;
    m->W = window;
    m->lambda = lambda;
    hipStream_t s = (hipStream_t)stream;
    bool ok = hipMalloc((void **)&m->X, sizeof(double) * (size_t)window * n_features) == hipSuccess &&
              hipMalloc((void **)&m->L, sizeof(int32_t) * (size_t)window) == hipSuccess &&
              hipMalloc((void **)&m->Wt, sizeof(double) * (size_t)n_classes * (n_features + 1)) == hipSuccess &&
              hipMalloc((void **)&m->coef, (size_t)window * n_classes) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        wo_svm_free(m);
        return wo_fail(WO_E_NOMEM, "device allocation failed");
    }
    if (hipMemsetAsync(m->Wt, 0, sizeof(double) * (size_t)n_classes * (n_features + 1), s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        wo_svm_free(m);
        return wo_fail(WO_E_DEVICE, "clearing the weights failed");
    }
    *out = m;
    return WO_OK;
}

extern "C" wo_status wo_svm_free(wo_svm *m)
{
    if (!m) return WO_OK;
    if (m->X || m->L || m->Wt || m->coef) (void)hipDeviceSynchronize();
    if (m->X) (void)hipFree(m->X);
    if (m->L) (void)hipFree(m->L);
    if (m->Wt) (void)hipFree(m->Wt);
    if (m->coef) (void)hipFree(m->coef);
    delete m;
    return WO_OK;
}

extern "C" wo_status wo_svm_push(wo_svm *m, int64_t n, const double *d_features, const int32_t *d_labels, void *stream)
{
    if (!m || !d_features || !d_labels) return wo_fail(WO_E_INVAL, "NULL argument");
    if (n < 0) return wo_fail(WO_E_INVAL, "n < 0");
    SvmBusy busy(&m->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "SVM in use by another thread");
    hipStream_t s = (hipStream_t)stream;
    // only the last min(n, W) samples stay; sample g goes to slot g mod W
    const int64_t keep = std::min<int64_t>(n, m->W);
    int64_t g = m->pushed + (n - keep);
    int64_t r = n - keep;                  // row of the input
    while (r < n) {
        const int64_t slot = g % m->W;
        const int64_t run = std::min<int64_t>(n - r, m->W - slot);
        WO_HIP(hipMemcpyAsync(m->X + slot * m->F, d_features + r * m->F, sizeof(double) * (size_t)run * m->F,
                              hipMemcpyDeviceToDevice, s));
        WO_HIP(hipMemcpyAsync(m->L + slot, d_labels + r, sizeof(int32_t) * (size_t)run, hipMemcpyDeviceToDevice, s));
        r += run;
        g += run;
    }
    m->pushed += n;
    return WO_OK;
}

extern "C" wo_status wo_svm_train(wo_svm *m, int32_t iterations, void *stream)
{
    if (!m) return wo_fail(WO_E_INVAL, "NULL SVM");
    if (iterations < 0) return wo_fail(WO_E_INVAL, "iterations < 0");
    SvmBusy busy(&m->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "SVM in use by another thread");
    const int64_t n = std::min<int64_t>(m->pushed, m->W);
    if (n == 0) return wo_fail(WO_E_STATE, "the window holds no sample");
    const int64_t first = (m->pushed - n) % m->W;   // slot of the oldest sample
    hipStream_t s = (hipStream_t)stream;
    const int32_t nw = m->K * (m->F + 1);
    for (int32_t it = 0; it < iterations; it++) {
        const double t = (double)(m->steps + it + 1);
        hipLaunchKernelGGL(margin_kernel, dim3(grid_for(n * m->K, 256)), dim3(256), 0, s, m->X, m->L, m->W, first, n,
                           m->F, m->K, m->Wt, m->coef);
        hipLaunchKernelGGL(update_kernel, dim3((nw + 63) / 64), dim3(64), 0, s, m->X, m->coef, m->W, first, n, m->F,
                           m->K, m->Wt, m->lambda, t);
    }
    WO_HIP(hipGetLastError());
    m->steps += iterations;
    return WO_OK;
}

extern "C" wo_status wo_svm_predict(wo_svm *m, int64_t n, const double *d_features, int32_t *d_class, void *stream)
{
    if (!m || !d_features || !d_class) return wo_fail(WO_E_INVAL, "NULL argument");
    if (n < 0) return wo_fail(WO_E_INVAL, "n < 0");
    if (n == 0) return WO_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = sizeof(double) * ((size_t)m->K * (m->F + 1) + 4 * 64 * PK_LD);
    hipLaunchKernelGGL(predict_kernel, dim3(grid_for(n, 256)), dim3(256), lds, s, d_features, n, m->F, m->K, m->Wt,
                       d_class);
    WO_HIP(hipGetLastError());
    return WO_OK;
}

extern "C" wo_status wo_svm_get_weights(wo_svm *m, double *h_weights, int64_t *h_steps, int64_t *h_window_count,
                                        void *stream)
{
    if (!m) return wo_fail(WO_E_INVAL, "NULL SVM");
    hipStream_t s = (hipStream_t)stream;
    if (h_weights) {
        WO_HIP(hipMemcpyAsync(h_weights, m->Wt, sizeof(double) * (size_t)m->K * (m->F + 1), hipMemcpyDeviceToHost, s));
        WO_HIP(hipStreamSynchronize(s));
    }
    if (h_steps) *h_steps = m->steps;
    if (h_window_count) *h_window_count = std::min<int64_t>(m->pushed, m->W);
    return WO_OK;
}
