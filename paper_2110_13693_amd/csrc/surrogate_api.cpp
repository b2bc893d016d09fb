// Host side of the surrogate and screening entry points of include/wo.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "wo_common.h"
#include "wo_internal.h"
#include "wo_surrogate.h"

using namespace wo;

namespace {

constexpr int PRED_CHUNK = 65536;    // rows per inference pass (enough workgroups to fill the GPU)
constexpr int MAX_BATCH = MAX_GRAD_ROWS;   // training rows per step
constexpr int WORK_ROWS = PRED_CHUNK > MAX_BATCH ? PRED_CHUNK : MAX_BATCH;

uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

struct wo_sur {
    int device = 0;
    float *d_p = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr;   // P_TOTAL each
    uint16_t *d_W1b = nullptr, *d_W2b = nullptr, *d_W2kn = nullptr;
    // work buffers (WORK_ROWS rows)
    uint8_t *d_zb = nullptr;
    float *d_tb = nullptr, *d_U1 = nullptr, *d_U2 = nullptr, *d_H2 = nullptr, *d_dy = nullptr, *d_sq = nullptr;
    uint16_t *d_H1 = nullptr, *d_H1T = nullptr, *d_DU2 = nullptr, *d_DU2T = nullptr, *d_DU1T = nullptr;
    float *d_pred = nullptr;            // screening scratch [capacity]
    int64_t pred_cap = 0;
    float *d_losses = nullptr;          // training: the loss of every batch of an epoch
    int64_t losses_cap = 0;
    double *d_mom = nullptr;
    float *d_loss = nullptr;
    float *d_red = nullptr;             // gW3 slice sums, then the slices' counter (zero between calls)
    uint8_t *d_zt = nullptr;            // a training batch's zone bytes by category [64][batch]
    double mean = 0.0, std = 1.0;
    bool scaled = false;
    int step = 0;                       // Adam steps taken
    int n_cat = 64;
    std::atomic<int> busy{0};
};

namespace {

template <typename T>
wo_status alloc(T **p, size_t count)
{
    if (wo_fault_injected()) return wo_fail(WO_E_NOMEM, "injected allocation failure");
    hipError_t e = hipMalloc((void **)p, std::max<size_t>(16, count * sizeof(T)));
    if (e != hipSuccess) {
        *p = nullptr;
        return wo_fail(WO_E_NOMEM, "hipMalloc(%zu) failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    return WO_OK;
}

// forward pass of `rows` (multiple of 128 after padding) rows whose zone bytes
// are at zone; U1/H1/H1T/U2 filled.  train: keep U1 and the transposed H1.
wo_status forward(wo_sur *s, const uint8_t *zone, int rows_real, int rows, bool train, hipStream_t st)
{
    GemmArgs g{};
    g.M = rows;
    g.N = N_H1;
    g.K = N_IN;
    g.M_real = rows_real;
    g.n_cat = s->n_cat;
    g.zoneA = zone;
    g.B = s->d_W1b;
    g.ldb = N_IN;
    g.ldc = N_H1;
    g.bias = s->d_p + P_B1;
    g.U = train ? s->d_U1 : nullptr;
    g.H = s->d_H1;
    g.HT = train ? s->d_H1T : nullptr;
    g.ldt = rows;
    WO_HIP(launch_gemm(A_ONEHOT, B_BF16, EPI_BIAS_GELU, g, st));
    GemmArgs h{};
    h.M = rows;
    h.N = N_H2;
    h.K = N_H1;
    h.M_real = rows_real;
    h.A = s->d_H1;
    h.lda = N_H1;
    h.B = s->d_W2b;
    h.ldb = N_H1;
    h.ldc = N_H2;
    h.bias = s->d_p + P_B2;
    h.U = s->d_U2;
    WO_HIP(launch_gemm(A_BF16, B_BF16, EPI_BIAS_GELU, h, st));
    return WO_OK;
}

// forward + backward of one batch of `rows` (multiple of 128) whose zone rows
// are d_zb (by category in d_zt) and standardised targets d_tb; gradients into
// d_g, loss into loss_out (null: d_loss).
wo_status gradients(wo_sur *s, int rows, hipStream_t st, float *loss_out = nullptr)
{
    wo_status r = forward(s, s->d_zb, rows, rows, true, st);
    if (r) return r;
    L3Args l{};
    l.n = rows;
    l.n_batch = rows;
    l.U2 = s->d_U2;
    l.W3 = s->d_p + P_W3;
    l.b3 = s->d_p + P_B3;
    l.target = s->d_tb;
    l.dy = s->d_dy;
    l.sq = s->d_sq;
    l.H2 = s->d_H2;
    l.DU2 = s->d_DU2;
    l.DU2T = s->d_DU2T;
    l.ld_t = rows;
    WO_HIP(launch_layer3(l, st));
    // du1^T [1024][b] = (du2 [b][256] . W2 [1024][256]^T) * GELU'(u1), transposed
    GemmArgs g1{};
    g1.M = rows;
    g1.N = N_H1;
    g1.K = N_H2;
    g1.A = s->d_DU2;
    g1.lda = N_H2;
    g1.B = s->d_W2kn;
    g1.ldb = N_H2;
    g1.ldc = N_H1;
    g1.Uin = s->d_U1;
    g1.HT = s->d_DU1T;
    g1.ldt = rows;
    g1.H = s->d_H1;   // du1 in column slices as well, in h1's buffer (free after layer 2)
    WO_HIP(launch_gemm(A_BF16, B_BF16, EPI_GELU_GRAD_T, g1, st));
    // gW2^T [256][1024] = du2^T [256][b] . (h1^T [1024][b])^T: a long K over
    // few outputs, so K is split in parts (into u1's buffer, free now) that
    // the batch sums add in order
    int ks = 8;
    while (ks > 1 && rows % (ks * 64)) ks >>= 1;
    GemmArgs g2{};
    g2.M = N_H2;
    g2.N = N_H1;
    g2.K = rows;
    g2.A = s->d_DU2T;
    g2.lda = rows;
    g2.B = s->d_H1T;
    g2.ldb = rows;
    g2.C = ks > 1 ? s->d_U1 : s->d_g + P_W2;
    g2.ldc = N_H1;
    g2.ksplit = ks;
    g2.c_split = (int64_t)N_H2 * N_H1;
    WO_HIP(launch_gemm(A_BF16, B_BF16, EPI_STORE, g2, st));
    // gW1 [1024][4096] = du1^T . x with x one-hot: sums of du1 rows per
    // (category, zone) bin
    WO_HIP(launch_w1_grad(s->d_H1, s->d_zt, rows, s->n_cat, s->d_g + P_W1, st));
    SumArgs sm{};
    sm.n = rows;
    sm.H2 = s->d_H2;
    sm.dy = s->d_dy;
    sm.sq = s->d_sq;
    sm.DU2T = s->d_DU2T;
    sm.DU1T = s->d_DU1T;
    sm.ld_t = rows;
    sm.gW3 = s->d_g + P_W3;
    sm.gb3 = s->d_g + P_B3;
    sm.gb2 = s->d_g + P_B2;
    sm.gb1 = s->d_g + P_B1;
    sm.loss = loss_out ? loss_out : s->d_loss;
    sm.w3part = s->d_red;
    sm.w3ctr = (uint32_t *)(s->d_red + W3_SLICES * N_H2);
    sm.w2part = ks > 1 ? s->d_U1 : nullptr;
    sm.w2_splits = ks;
    sm.w2_stride = (int64_t)N_H2 * N_H1;
    sm.gW2 = s->d_g + P_W2;
    WO_HIP(launch_batch_sums(sm, st));
    return WO_OK;
}

wo_status predict(wo_sur *s, int64_t n, const uint8_t *d_zone, float *d_pred, hipStream_t st)
{
    for (int64_t r0 = 0; r0 < n; r0 += PRED_CHUNK) {
        const int real = (int)std::min<int64_t>(PRED_CHUNK, n - r0);
        const int rows = (real + 127) / 128 * 128;
        wo_status r = forward(s, d_zone + r0 * 64, real, rows, false, st);
        if (r) return r;
        L3Args l{};
        l.n = real;
        l.n_batch = real;
        l.U2 = s->d_U2;
        l.W3 = s->d_p + P_W3;
        l.b3 = s->d_p + P_B3;
        l.target = nullptr;
        l.pred = d_pred + r0;
        l.mean = (float)s->mean;
        l.std = (float)s->std;
        WO_HIP(launch_layer3(l, st));
    }
    return WO_OK;
}

struct SurBusy {
    std::atomic<int> *f;
    bool ok;
    explicit SurBusy(std::atomic<int> *flag) : f(flag)
    {
        int z = 0;
        ok = f->compare_exchange_strong(z, 1);
    }
    ~SurBusy()
    {
        if (ok) f->store(0);
    }
};

// canonical host layout (W1 [4096][1024], b1, W2 [1024][256], b2, W3 [256], b3)
// <-> device [out][in] layout
void host_to_device_layout(const float *h, std::vector<float> &d)
{
    d.assign(P_TOTAL, 0.f);
    const float *W1 = h, *b1 = W1 + (int64_t)N_IN * N_H1, *W2 = b1 + N_H1, *b2 = W2 + (int64_t)N_H1 * N_H2,
                *W3 = b2 + N_H2, *b3 = W3 + N_H2;
    for (int i = 0; i < N_IN; i++)
        for (int o = 0; o < N_H1; o++) d[P_W1 + (int64_t)o * N_IN + i] = W1[(int64_t)i * N_H1 + o];
    for (int o = 0; o < N_H1; o++) d[P_B1 + o] = b1[o];
    for (int i = 0; i < N_H1; i++)
        for (int o = 0; o < N_H2; o++) d[P_W2 + (int64_t)o * N_H1 + i] = W2[(int64_t)i * N_H2 + o];
    for (int o = 0; o < N_H2; o++) d[P_B2 + o] = b2[o];
    for (int i = 0; i < N_H2; i++) d[P_W3 + i] = W3[i];
    d[P_B3] = b3[0];
}

void device_to_host_layout(const std::vector<float> &d, float *h)
{
    float *W1 = h, *b1 = W1 + (int64_t)N_IN * N_H1, *W2 = b1 + N_H1, *b2 = W2 + (int64_t)N_H1 * N_H2,
          *W3 = b2 + N_H2, *b3 = W3 + N_H2;
    for (int i = 0; i < N_IN; i++)
        for (int o = 0; o < N_H1; o++) W1[(int64_t)i * N_H1 + o] = d[P_W1 + (int64_t)o * N_IN + i];
    for (int o = 0; o < N_H1; o++) b1[o] = d[P_B1 + o];
    for (int i = 0; i < N_H1; i++)
        for (int o = 0; o < N_H2; o++) W2[(int64_t)i * N_H2 + o] = d[P_W2 + (int64_t)o * N_H1 + i];
    for (int o = 0; o < N_H2; o++) b2[o] = d[P_B2 + o];
    for (int i = 0; i < N_H2; i++) W3[i] = d[P_W3 + i];
    b3[0] = d[P_B3];
}

// He-uniform initial weights from a counter generator: weight e of layer L
// gets splitmix64(seed, L, e) mapped to U(-sqrt(6/fan_in), sqrt(6/fan_in)).
void default_init(uint64_t seed, std::vector<float> &h)
{
    h.assign(P_TOTAL, 0.f);
    float *W1 = h.data(), *b1 = W1 + (int64_t)N_IN * N_H1, *W2 = b1 + N_H1, *b2 = W2 + (int64_t)N_H1 * N_H2,
          *W3 = b2 + N_H2;
    auto fill = [&](float *w, int64_t count, int fan_in, uint64_t layer) {
        const double lim = std::sqrt(6.0 / fan_in);
        for (int64_t e = 0; e < count; e++) {
            const uint64_t r = splitmix64(splitmix64(seed ^ (layer << 56)) ^ (uint64_t)e);
            const double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);   // [0, 1)
            w[e] = (float)((2.0 * u - 1.0) * lim);
        }
    };
    fill(W1, (int64_t)N_IN * N_H1, N_IN, 1);
    fill(W2, (int64_t)N_H1 * N_H2, N_H1, 2);
    fill(W3, N_H2, N_H2, 3);
    (void)b2;
}

}  // namespace

extern "C" wo_status wo_sur_create(int32_t n_categories, const float *h_init, uint64_t seed, void *stream,
                                   wo_sur **out)
{
    if (!out) return wo_fail(WO_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n_categories < 1 || n_categories > WO_MAX_CATEGORIES)
        return wo_fail(WO_E_RANGE, "n_categories must be in [1, %d]", WO_MAX_CATEGORIES);
    if (wo_fault_injected()) return wo_fail(WO_E_NOMEM, "injected allocation failure");
    wo_sur *s = new (std::nothrow) wo_sur;
    if (!s) return wo_fail(WO_E_NOMEM, "host allocation failed");
    std::unique_ptr<wo_sur, wo_status (*)(wo_sur *)> guard(s, wo_sur_free);
    s->n_cat = n_categories;
    WO_HIP(hipGetDevice(&s->device));
    wo_status r;
    if ((r = alloc(&s->d_p, P_TOTAL)) || (r = alloc(&s->d_g, P_TOTAL)) || (r = alloc(&s->d_m, P_TOTAL)) ||
        (r = alloc(&s->d_v, P_TOTAL)) || (r = alloc(&s->d_W1b, (size_t)N_H1 * N_IN)) ||
        (r = alloc(&s->d_W2b, (size_t)N_H2 * N_H1)) || (r = alloc(&s->d_W2kn, (size_t)N_H1 * N_H2)) ||
        (r = alloc(&s->d_zb, (size_t)WORK_ROWS * 64)) || (r = alloc(&s->d_tb, WORK_ROWS)) ||
        (r = alloc(&s->d_U1, (size_t)WORK_ROWS * N_H1)) || (r = alloc(&s->d_U2, (size_t)WORK_ROWS * N_H2)) ||
        (r = alloc(&s->d_H2, (size_t)WORK_ROWS * N_H2)) || (r = alloc(&s->d_dy, WORK_ROWS)) ||
        (r = alloc(&s->d_sq, WORK_ROWS)) || (r = alloc(&s->d_H1, (size_t)WORK_ROWS * N_H1)) ||
        (r = alloc(&s->d_H1T, (size_t)WORK_ROWS * N_H1)) || (r = alloc(&s->d_DU2, (size_t)WORK_ROWS * N_H2)) ||
        (r = alloc(&s->d_DU2T, (size_t)WORK_ROWS * N_H2)) || (r = alloc(&s->d_DU1T, (size_t)WORK_ROWS * N_H1)) ||
        (r = alloc(&s->d_mom, 2)) || (r = alloc(&s->d_loss, 1)) || (r = alloc(&s->d_red, W3_SLICES * N_H2 + 16)) ||
        (r = alloc(&s->d_zt, (size_t)64 * MAX_GRAD_ROWS)))
        return r;
    std::vector<float> host, dev;
    if (h_init) {
        host.assign(h_init, h_init + P_TOTAL);
    } else {
        default_init(seed, host);
    }
    for (float x : host)
        if (!std::isfinite(x)) return wo_fail(WO_E_INVAL, "initial parameters must be finite");
    host_to_device_layout(host.data(), dev);
    hipStream_t st = (hipStream_t)stream;
    WO_HIP(hipMemcpyAsync(s->d_p, dev.data(), sizeof(float) * P_TOTAL, hipMemcpyHostToDevice, st));
    WO_HIP(hipMemsetAsync(s->d_m, 0, sizeof(float) * P_TOTAL, st));
    WO_HIP(hipMemsetAsync(s->d_v, 0, sizeof(float) * P_TOTAL, st));
    WO_HIP(hipMemsetAsync(s->d_red, 0, sizeof(float) * (W3_SLICES * N_H2 + 16), st));
    WO_HIP(launch_refresh_bf16(s->d_p + P_W1, s->d_p + P_W2, s->d_W1b, s->d_W2b, s->d_W2kn, st));
    WO_HIP(hipStreamSynchronize(st));
    guard.release();
    *out = s;
    return WO_OK;
}

extern "C" wo_status wo_sur_free(wo_sur *s)
{
    if (!s) return WO_OK;
    (void)hipDeviceSynchronize();
    void *bufs[] = {s->d_p,  s->d_g,   s->d_m,  s->d_v,   s->d_W1b, s->d_W2b,  s->d_W2kn, s->d_zb,   s->d_tb,
                    s->d_U1, s->d_U2,  s->d_H2, s->d_dy,  s->d_sq,  s->d_H1,   s->d_H1T,  s->d_DU2,  s->d_DU2T,
                    s->d_DU1T, s->d_pred, s->d_losses, s->d_mom, s->d_loss, s->d_red,
                    s->d_zt};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete s;
    return WO_OK;
}

extern "C" wo_status wo_sur_set_scale(wo_sur *s, double mean, double std)
{
    if (!s) return wo_fail(WO_E_INVAL, "surrogate is NULL");
    if (!std::isfinite(mean) || !(std > 0) || !std::isfinite(std))
        return wo_fail(WO_E_INVAL, "scale needs a finite mean and a positive std");
    s->mean = mean;
    s->std = std;
    s->scaled = true;
    return WO_OK;
}

extern "C" wo_status wo_sur_get_scale(const wo_sur *s, double *mean, double *std)
{
    if (!s) return wo_fail(WO_E_INVAL, "surrogate is NULL");
    if (mean) *mean = s->mean;
    if (std) *std = s->std;
    return WO_OK;
}

extern "C" wo_status wo_sur_get_params(const wo_sur *s, float *h_out)
{
    if (!s || !h_out) return wo_fail(WO_E_INVAL, "NULL argument");
    std::vector<float> dev(P_TOTAL);
    WO_HIP(hipDeviceSynchronize());
    WO_HIP(hipMemcpy(dev.data(), s->d_p, sizeof(float) * P_TOTAL, hipMemcpyDeviceToHost));
    device_to_host_layout(dev, h_out);
    return WO_OK;
}

static_assert(P_TOTAL == WO_SUR_PARAMS, "parameter count");
static_assert(TOPK_MAX == WO_SCREEN_MAX_KEEP, "screen limit");

extern "C" wo_status wo_sur_gradients(wo_sur *s, int32_t n, const uint8_t *d_zone_of, const float *d_target,
                                      float *h_grad, float *h_loss, void *stream)
{
    if (!s) return wo_fail(WO_E_INVAL, "surrogate is NULL");
    SurBusy busy(&s->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "surrogate is in use by another thread");
    if (n < 128 || n % 128 || n > MAX_BATCH)
        return wo_fail(WO_E_RANGE, "gradient batch must be a multiple of 128 in [128, %d]", MAX_BATCH);
    if (!d_zone_of || !d_target || !h_grad) return wo_fail(WO_E_INVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    WO_HIP(hipMemcpyAsync(s->d_zb, d_zone_of, (size_t)n * 64, hipMemcpyDeviceToDevice, st));
    WO_HIP(hipMemcpyAsync(s->d_tb, d_target, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    WO_HIP(launch_zone_cols(s->d_zb, n, s->d_zt, st));
    wo_status r = gradients(s, n, st);
    if (r) return r;
    std::vector<float> dev(P_TOTAL);
    WO_HIP(hipMemcpyAsync(dev.data(), s->d_g, sizeof(float) * P_TOTAL, hipMemcpyDeviceToHost, st));
    float loss = 0.f;
    WO_HIP(hipMemcpyAsync(&loss, s->d_loss, sizeof(float), hipMemcpyDeviceToHost, st));
    WO_HIP(hipStreamSynchronize(st));
    device_to_host_layout(dev, h_grad);
    if (h_loss) *h_loss = loss;
    return WO_OK;
}

extern "C" wo_status wo_sur_train(wo_sur *s, int64_t n, const uint8_t *d_zone_of, const int32_t *d_dist,
                                  int32_t epochs, int32_t batch, float lr, uint64_t seed, float *h_last_loss,
                                  void *stream)
{
    if (!s) return wo_fail(WO_E_INVAL, "surrogate is NULL");
    SurBusy busy(&s->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "surrogate is in use by another thread");
    if (batch < 128 || batch % 128 || batch > MAX_BATCH)
        return wo_fail(WO_E_RANGE, "batch must be a multiple of 128 in [128, %d]", MAX_BATCH);
    if (n < batch) return wo_fail(WO_E_RANGE, "need at least one batch of samples");
    if (n > INT32_MAX) return wo_fail(WO_E_RANGE, "too many samples");
    if (epochs < 1 || !(lr > 0)) return wo_fail(WO_E_INVAL, "epochs >= 1 and lr > 0 required");
    if (!d_zone_of || !d_dist) return wo_fail(WO_E_INVAL, "NULL device buffer");
    hipStream_t st = (hipStream_t)stream;
    if (!s->scaled) {
        // standardise the targets with their own mean and deviation
        double mom[2];
        WO_HIP(launch_moments(d_dist, n, s->d_mom, st));
        WO_HIP(hipMemcpyAsync(mom, s->d_mom, sizeof mom, hipMemcpyDeviceToHost, st));
        WO_HIP(hipStreamSynchronize(st));
        if (!(mom[1] > 0)) return wo_fail(WO_E_INVAL, "targets have zero spread");
        s->mean = mom[0];
        s->std = mom[1];
        s->scaled = true;
    }
    const int64_t n_batches = n / batch;
    if (s->losses_cap < n_batches) {
        if (s->d_losses) (void)hipFree(s->d_losses);
        s->d_losses = nullptr;
        s->losses_cap = 0;
        wo_status r = alloc(&s->d_losses, (size_t)n_batches);
        if (r) return r;
        s->losses_cap = n_batches;
    }
    // the shuffle of an epoch: a keyed permutation of [0, n) evaluated where
    // the batch is gathered (key from the counter generator on seed and
    // epoch), over 2h bits with 2^2h >= n
    int h = 1;
    while ((1ll << (2 * h)) < n) h++;
    double loss_sum = 0.0;
    std::vector<float> losses;
    for (int ep = 0; ep < epochs; ep++) {
        const uint64_t key = splitmix64(splitmix64(seed + (uint64_t)ep * 0x100000001ull));
        const bool last = ep == epochs - 1;
        for (int64_t b = 0; b < n_batches; b++) {
            WO_HIP(launch_gather_batch(d_zone_of, d_dist, n, h, key, b * batch, batch, s->mean, 1.0 / s->std,
                                       s->d_zb, s->d_zt, s->d_tb, st));
            wo_status r = gradients(s, batch, st, last && h_last_loss ? s->d_losses + b : nullptr);
            if (r) return r;
            s->step++;
            WO_HIP(launch_adam(s->d_p, s->d_g, s->d_m, s->d_v, P_TOTAL, lr, s->step, s->d_W1b, s->d_W2b, s->d_W2kn,
                               st));
        }
    }
    if (h_last_loss) {
        losses.assign(n_batches, 0.f);
        if (n_batches)
            WO_HIP(hipMemcpyAsync(losses.data(), s->d_losses, sizeof(float) * n_batches, hipMemcpyDeviceToHost, st));
    }
    WO_HIP(hipStreamSynchronize(st));
    if (h_last_loss) {
        for (float l : losses) loss_sum += l;
        *h_last_loss = (float)(loss_sum / std::max<int64_t>(1, n_batches));
    }
    return WO_OK;
}

extern "C" wo_status wo_sur_predict(wo_sur *s, int64_t n, const uint8_t *d_zone_of, float *d_pred, void *stream)
{
    if (!s) return wo_fail(WO_E_INVAL, "surrogate is NULL");
    SurBusy busy(&s->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "surrogate is in use by another thread");
    if (n < 0) return wo_fail(WO_E_INVAL, "n < 0");
    if (n == 0) return WO_OK;
    if (!d_zone_of || !d_pred) return wo_fail(WO_E_INVAL, "NULL device buffer");
    return predict(s, n, d_zone_of, d_pred, (hipStream_t)stream);
}

extern "C" wo_status wo_screen_plans(wo_wh *wh, int32_t inst, wo_sur *s, int64_t n_plans, const uint8_t *d_zone_of,
                                     float *d_pred, int64_t keep, int32_t *d_keep_idx, void *stream)
{
    if (!wh || !s) return wo_fail(WO_E_INVAL, "NULL handle");
    int32_t n_cat = 0;
    wo_status r = wo_instance_info(wh, inst, nullptr, nullptr, &n_cat);
    if (r) return r;
    if (n_cat != s->n_cat)
        return wo_fail(WO_E_INVAL, "instance has %d categories, the surrogate %d", n_cat, s->n_cat);
    SurBusy busy(&s->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "surrogate is in use by another thread");
    if (n_plans < 1 || n_plans > (1 << 24)) return wo_fail(WO_E_RANGE, "n_plans must be in [1, 2^24]");
    if (keep < 1 || keep > n_plans || keep > TOPK_MAX)
        return wo_fail(WO_E_RANGE, "keep must be in [1, min(n_plans, %d)]", TOPK_MAX);
    if (!d_zone_of || !d_keep_idx) return wo_fail(WO_E_INVAL, "NULL device buffer");
    hipStream_t st = (hipStream_t)stream;
    float *pred = d_pred;
    if (!pred) {
        if (s->pred_cap < n_plans) {
            if (s->d_pred) (void)hipFree(s->d_pred);
            s->d_pred = nullptr;
            s->pred_cap = 0;
            if ((r = alloc(&s->d_pred, (size_t)n_plans))) return r;
            s->pred_cap = n_plans;
        }
        pred = s->d_pred;
    }
    if ((r = predict(s, n_plans, d_zone_of, pred, st))) return r;
    WO_HIP(launch_topk(pred, (int)n_plans, (int)keep, d_keep_idx, st));
    return WO_OK;
}

extern "C" wo_status wo_sur_save(const wo_sur *s, const char *path)
{
    if (!s || !path) return wo_fail(WO_E_INVAL, "NULL argument");
    std::vector<float> p(P_TOTAL), m(P_TOTAL), v(P_TOTAL);
    WO_HIP(hipDeviceSynchronize());
    WO_HIP(hipMemcpy(p.data(), s->d_p, sizeof(float) * P_TOTAL, hipMemcpyDeviceToHost));
    WO_HIP(hipMemcpy(m.data(), s->d_m, sizeof(float) * P_TOTAL, hipMemcpyDeviceToHost));
    WO_HIP(hipMemcpy(v.data(), s->d_v, sizeof(float) * P_TOTAL, hipMemcpyDeviceToHost));
    FILE *f = fopen(path, "wb");
    if (!f) return wo_fail(WO_E_INVAL, "cannot open %s for writing", path);
    const char magic[8] = {'W', 'O', 'S', 'U', 'R', '0', '0', '2'};
    const int64_t count = P_TOTAL;
    const int32_t hdr[3] = {s->step, s->scaled ? 1 : 0, s->n_cat};
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&count, 8, 1, f) == 1 && fwrite(hdr, 4, 3, f) == 3 &&
              fwrite(&s->mean, 8, 1, f) == 1 && fwrite(&s->std, 8, 1, f) == 1 &&
              fwrite(p.data(), 4, P_TOTAL, f) == (size_t)P_TOTAL && fwrite(m.data(), 4, P_TOTAL, f) == (size_t)P_TOTAL &&
              fwrite(v.data(), 4, P_TOTAL, f) == (size_t)P_TOTAL;
    ok = (fclose(f) == 0) && ok;
    return ok ? WO_OK : wo_fail(WO_E_INVAL, "write to %s failed", path);
}

extern "C" wo_status wo_sur_load(const char *path, void *stream, wo_sur **out)
{
    if (!path || !out) return wo_fail(WO_E_INVAL, "NULL argument");
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) return wo_fail(WO_E_INVAL, "cannot open %s", path);
    char magic[8];
    int64_t count = 0;
    int32_t hdr[3];
    double mean = 0, std = 1;
    std::vector<float> p(P_TOTAL), m(P_TOTAL), v(P_TOTAL);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "WOSUR002", 8) == 0 && fread(&count, 8, 1, f) == 1 &&
              count == P_TOTAL && fread(hdr, 4, 3, f) == 3 && fread(&mean, 8, 1, f) == 1 && fread(&std, 8, 1, f) == 1 &&
              fread(p.data(), 4, P_TOTAL, f) == (size_t)P_TOTAL && fread(m.data(), 4, P_TOTAL, f) == (size_t)P_TOTAL &&
              fread(v.data(), 4, P_TOTAL, f) == (size_t)P_TOTAL;
    fclose(f);
    if (!ok) return wo_fail(WO_E_INVAL, "%s is not a surrogate checkpoint", path);
    std::vector<float> host(P_TOTAL);
    device_to_host_layout(p, host.data());
    wo_sur *s = nullptr;
    wo_status r = wo_sur_create(hdr[2], host.data(), 0, stream, &s);
    if (r) return r;
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(s->d_m, m.data(), sizeof(float) * P_TOTAL, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->d_v, v.data(), sizeof(float) * P_TOTAL, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        wo_sur_free(s);
        return wo_fail(WO_E_DEVICE, "copy of the optimiser state failed");
    }
    s->step = hdr[0];
    s->scaled = hdr[1] != 0;
    s->mean = mean;
    s->std = std;
    *out = s;
    return WO_OK;
}
