// Class-based storage by K-means on pick frequency (section 5, Subproblem 3:
// products are placed by how often they are picked, with an unsupervised
// clustering such as K-means, MacQueen 1967).  The feature of a SKU is the
// number of order lines naming it; Lloyd's iteration clusters the SKUs into
// k classes, numbered by descending mean frequency, which become the
// categories the zones hold.
//
// SKUs of equal frequency always share a cluster, so after the frequencies
// and their histogram the iteration runs over the histogram's non-empty bins,
// all of it in one workgroup (km_lloyd_kernel).  The arithmetic is exact: a centroid is the
// rational S / N, and f is nearer to S_j / N_j than to S_k / N_k iff
// |f N_j - S_j| N_k < |f N_k - S_k| N_j, compared in 128 bits (ties to the
// lower index).  Start: centroid c is the distinct frequency of rank
// floor((2c + 1) D / (2k)) among the D distinct ones.  A step assigns every
// bin and moves each non-empty cluster's centroid to its members' mean; the
// iteration ends at the first assignment equal to the previous one or after
// max_iter assignments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "wo_common.h"

namespace {

constexpr int KM_MAX = 64;

struct KmState {
    long long S[KM_MAX], N[KM_MAX];       // centroids S / N
    unsigned long long S2[KM_MAX], N2[KM_MAX];   // sums of the assignment in progress
    long long cnt[KM_MAX];                // members after the last assignment
    int changed, done, n_iter, pad;
    int rank[KM_MAX];
    int k_used;
};

// a * b < c * d for a, c < 2^47 and b, d < 2^23 (products up to 2^70: 128 bits)
__device__ __forceinline__ bool less_prod(unsigned long long a, unsigned long long b, unsigned long long c,
                                          unsigned long long d)
{
    const unsigned long long h1 = __umul64hi(a, b), h2 = __umul64hi(c, d);
    return h1 < h2 || (h1 == h2 && a * b < c * d);
}

__device__ __forceinline__ unsigned long long absdiff(long long x, long long y) { return x > y ? x - y : y - x; }

// SKU ids are popularity ranks, so the low ids take most lines: their counts
// gather in the workgroup's LDS first and reach memory once per workgroup.
constexpr int KM_HOT_SKUS = 2048;
__global__ __launch_bounds__(1024) void km_freq_kernel(const int32_t *skus, int64_t n_lines, int32_t n_skus,
                                                       int32_t *freq, int32_t *err)
{
    __shared__ int32_t hot[KM_HOT_SKUS];
    for (int i = threadIdx.x; i < KM_HOT_SKUS; i += blockDim.x) hot[i] = 0;
    __syncthreads();
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < n_lines; l += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = skus[l];
        if (s < 0 || s >= n_skus) atomicOr(err, 1);
        else if (s < KM_HOT_SKUS) atomicAdd(&hot[s], 1);
        else atomicAdd(&freq[s], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < KM_HOT_SKUS && i < n_skus; i += blockDim.x)
        if (hot[i]) atomicAdd(&freq[i], hot[i]);
}

// Most SKUs share a few low frequencies (most are never picked), so the
// counts of frequencies below KM_HOT gather in the workgroup's LDS first (the
// lanes of a wave holding the first active lane's frequency add theirs with
// one atomic), and each workgroup adds them to memory once; higher
// frequencies, few SKUs each, go to memory directly.
constexpr int KM_HOT = 64;
__global__ __launch_bounds__(1024) void km_hist_kernel(const int32_t *freq, int32_t n_skus, int32_t *hist)
{
    __shared__ int32_t hot[KM_HOT];
    if (threadIdx.x < KM_HOT) hot[threadIdx.x] = 0;
    __syncthreads();
    for (int32_t s0 = blockIdx.x * blockDim.x; s0 < n_skus; s0 += gridDim.x * blockDim.x) {
        const int32_t s = s0 + threadIdx.x;
        const bool act = s < n_skus;
        const int32_t f = act ? freq[s] : -1;
        const uint64_t live = __ballot(act);
        if (!live) continue;
        const int32_t f0 = __shfl(f, __builtin_ctzll(live), 64);
        const uint64_t same = __ballot(act && f == f0);
        if (act && f == f0) {
            if ((threadIdx.x & 63) == __builtin_ctzll(same)) {
                if (f0 < KM_HOT) atomicAdd(&hot[f0], __popcll(same));
                else atomicAdd(&hist[f0], __popcll(same));
            }
        } else if (act) {
            if (f < KM_HOT) atomicAdd(&hot[f], 1);
            else atomicAdd(&hist[f], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < KM_HOT && hot[threadIdx.x]) atomicAdd(&hist[threadIdx.x], hot[threadIdx.x]);
}

__global__ void km_label_kernel(const int32_t *freq, int32_t n_skus, const int32_t *label, const KmState *st,
                                int32_t *category)
{
    for (int32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n_skus; s += gridDim.x * blockDim.x)
        category[s] = st->rank[label[freq[s]]];
}

// The whole iteration in one workgroup: the non-empty bins (the distinct
// frequencies, at most sqrt(2 n_lines) + 1 <= KM_MAX_BINS of them since the
// positive ones sum to at most n_lines) are compacted in order into LDS;
// then the start, every assignment and centroid move, and the ranking run
// with block barriers between them, and the bins' labels and the state go to
// memory once.  The same steps as the kernels above, in one launch.
constexpr int KM_MAX_BINS = 5800;
constexpr int KM_BLOCK = 1024;

__global__ __launch_bounds__(KM_BLOCK) void km_lloyd_kernel(const int32_t *hist, int32_t n_bins, int32_t k,
                                                           int32_t max_iter, int32_t *label, KmState *st)
{
    __shared__ int32_t bv[KM_MAX_BINS], bm[KM_MAX_BINS];
    __shared__ uint8_t bl[KM_MAX_BINS];
    __shared__ unsigned long long S2[KM_MAX], N2[KM_MAX];
    __shared__ long long S[KM_MAX], N[KM_MAX], cnt[KM_MAX];
    __shared__ int part[KM_BLOCK / 64];
    __shared__ int D_s, changed_s;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // ---- compaction of the non-empty bins, in order of frequency
    int base = 0;
    int m_next = tid < n_bins ? hist[tid] : 0;       // each chunk's counts are read one chunk ahead
    for (int v0 = 0; v0 < n_bins; v0 += KM_BLOCK) {
        const int v = v0 + tid;
        const int m = m_next;
        m_next = v + KM_BLOCK < n_bins ? hist[v + KM_BLOCK] : 0;
        const unsigned long long b = __ballot(m > 0);
        const int below = __popcll(b & ((1ull << lane) - 1ull));
        __syncthreads();                           // part[] of the previous chunk has been read
        if (lane == 0) part[w] = __popcll(b);
        __syncthreads();
        int off = base;
        for (int i = 0; i < w; i++) off += part[i];
        if (m > 0 && off + below < KM_MAX_BINS) {
            bv[off + below] = v;
            bm[off + below] = m;
            bl[off + below] = 0xFF;
        }
        for (int i = 0; i < KM_BLOCK / 64; i++) base += part[i];
    }
    if (tid == 0) D_s = min(base, KM_MAX_BINS);
    if (tid < KM_MAX) {
        S2[tid] = 0;
        N2[tid] = 0;
        cnt[tid] = 0;
    }
    __syncthreads();
    const int D = D_s;
    // ---- start: centroid c is the distinct frequency of rank (2c + 1) D / (2k)
    if (tid < k) {
        const long long r = (2ll * tid + 1) * D / (2ll * k);
        S[tid] = bv[r];
        N[tid] = 1;
    }
    int n_iter = 0;
    for (;;) {
        if (tid == 0) changed_s = 0;
        __syncthreads();
        // ---- assignment: the nearest centroid, exactly; ties to the lower index
        for (int i = tid; i < D; i += KM_BLOCK) {
            const long long v = bv[i];
            int best = 0;
            unsigned long long bd = absdiff(v * N[0], S[0]), bn = (unsigned long long)N[0];
            for (int c = 1; c < k; c++) {
                const unsigned long long dc = absdiff(v * N[c], S[c]);
                const unsigned long long nc = (unsigned long long)N[c];
                if (less_prod(dc, bn, bd, nc)) {
                    best = c;
                    bd = dc;
                    bn = nc;
                }
            }
            if (bl[i] != best) {
                changed_s = 1;                     // benign race: every writer stores 1
                bl[i] = (uint8_t)best;
            }
            atomicAdd(&S2[best], (unsigned long long)v * (unsigned long long)bm[i]);
            atomicAdd(&N2[best], (unsigned long long)bm[i]);
        }
        __syncthreads();
        n_iter++;
        const int changed = changed_s;
        // ---- centroids: each non-empty cluster moves to its members' mean
        if (tid < k) {
            if (changed) {
                cnt[tid] = (long long)N2[tid];
                if (N2[tid] > 0) {
                    S[tid] = (long long)S2[tid];
                    N[tid] = (long long)N2[tid];
                }
            }
            S2[tid] = 0;
            N2[tid] = 0;
        }
        __syncthreads();
        if (!changed || n_iter >= max_iter) break;
    }
    // ---- results: bin labels, state, ranks of the non-empty clusters
    for (int i = tid; i < D; i += KM_BLOCK) label[bv[i]] = bl[i];
    if (tid < KM_MAX) {
        const bool in = tid < k;
        st->S[tid] = in ? S[tid] : 0;
        st->N[tid] = in ? N[tid] : 0;
        st->cnt[tid] = in ? cnt[tid] : 0;
        int r = 0;
        const bool used = in && cnt[tid] > 0;
        for (int d = 0; d < k; d++) {
            if (cnt[d] <= 0) continue;
            const long long a = S[d] * N[tid], b = S[tid] * N[d];
            r += a > b || (a == b && d < tid);
        }
        st->rank[tid] = used ? r : -1;
        const unsigned long long u = __ballot(used);
        if (tid == 0) {
            st->k_used = __popcll(u);
            st->n_iter = n_iter;
            st->done = 1;
        }
    }
}

int grid_for(int64_t n, int block) { return (int)std::min<int64_t>(std::max<int64_t>((n + block - 1) / block, 1), 4096); }

// Scratch layout of one call: frequencies [n_skus], histogram [n_bins], bin
// labels [n_bins], the state, the error flag; each part starts on 256 bytes.
struct KmLayout {
    size_t o_hist, o_label, o_state, o_err, bytes;
};

KmLayout km_layout(int32_t n_skus, int32_t n_bins)
{
    KmLayout L;
    L.o_hist = ((size_t)n_skus * 4 + 255) & ~(size_t)255;
    L.o_label = L.o_hist + (((size_t)n_bins * 4 + 255) & ~(size_t)255);
    L.o_state = L.o_label + (((size_t)n_bins * 4 + 255) & ~(size_t)255);
    L.o_err = L.o_state + ((sizeof(KmState) + 255) & ~(size_t)255);
    L.bytes = L.o_err + 256;
    return L;
}

// Fills words [0, n) with v: clears the scratch of the allocation-free
// variant inside the stream (a kernel rather than a memset, so that the
// call can sit in a captured graph).
__global__ void km_fill_kernel(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Results of the allocation-free variant, written on the device.
__global__ void km_finish_kernel(const KmState *st, const int32_t *err, int32_t *k_used, int32_t *n_iter)
{
    if (threadIdx.x != 0) return;
    if (k_used) *k_used = *err ? -1 : st->k_used;
    if (n_iter) *n_iter = st->n_iter;
}

}  // namespace

// The allocation-free variant keeps its scratch in this array: one copy per
// device, held until the process ends.  In host code the name is only a
// stand-in: the device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and is what the launches receive.
static __device__ __align__(256) unsigned char km_scratch[WO_KMEANS_NOALLOC_SCRATCH];

namespace {

constexpr int KM_MAX_DEVICES = 64;
std::mutex km_scratch_mu;
void *km_scratch_dev[KM_MAX_DEVICES];

wo_status km_scratch_address(void **out)
{
    int dev = 0;
    WO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= KM_MAX_DEVICES) return wo_fail(WO_E_UNSUPPORTED, "device %d beyond %d", dev, KM_MAX_DEVICES);
    std::lock_guard<std::mutex> g(km_scratch_mu);
    if (!km_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(km_scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return wo_fail(WO_E_DEVICE, "hipGetSymbolAddress of the K-means scratch failed: %s", hipGetErrorString(e));
        }
        km_scratch_dev[dev] = p;
    }
    *out = km_scratch_dev[dev];
    return WO_OK;
}

}  // namespace

extern "C" wo_status wo_kmeans_categories(const int32_t *d_order_skus, int64_t n_lines, int32_t n_skus, int32_t k,
                                          int32_t max_iter, int32_t *d_category, int32_t *k_used, int32_t *n_iter,
                                          void *stream)
{
    if (!d_order_skus || !d_category) return wo_fail(WO_E_INVAL, "NULL device buffer");
    if (n_lines < 1 || n_lines > WO_MAX_LINES)
        return wo_fail(WO_E_RANGE, "n_lines must be in 1 .. %d", WO_MAX_LINES);
    if (n_skus < 1 || n_skus > WO_MAX_LOCATIONS)
        return wo_fail(WO_E_RANGE, "n_skus must be in 1 .. %d", WO_MAX_LOCATIONS);
    if (k < 1 || k > KM_MAX) return wo_fail(WO_E_RANGE, "k must be in 1 .. %d", KM_MAX);
    if (max_iter < 1) return wo_fail(WO_E_INVAL, "max_iter must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const int32_t n_bins = (int32_t)n_lines + 1;      // a frequency is at most n_lines
    // scratch: frequencies, histogram, bin labels, state, error flag
    char *buf = nullptr;
    const KmLayout Ly = km_layout(n_skus, n_bins);
    const size_t o_hist = Ly.o_hist, o_label = Ly.o_label, o_state = Ly.o_state, o_err = Ly.o_err;
    const size_t bytes = Ly.bytes;
    if (wo_fault_injected()) return wo_fail(WO_E_NOMEM, "injected allocation failure");
    if (hipMalloc((void **)&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return wo_fail(WO_E_NOMEM, "hipMalloc(%zu) failed", bytes);
    }
    int32_t *freq = (int32_t *)buf, *hist = (int32_t *)(buf + o_hist), *label = (int32_t *)(buf + o_label);
    KmState *st = (KmState *)(buf + o_state);
    int32_t *err = (int32_t *)(buf + o_err);
    wo_status ret = WO_OK;
    int32_t h_err = 0;
    KmState h{};
    auto run = [&]() -> wo_status {
        WO_HIP(hipMemsetAsync(buf, 0, o_label, s));                       // frequencies, histogram
        WO_HIP(hipMemsetAsync(label, 0xFF, o_state - o_label, s));        // no cluster yet
        WO_HIP(hipMemsetAsync(st, 0, bytes - o_state, s));                // state, error flag
        hipLaunchKernelGGL(km_freq_kernel, dim3(std::min(grid_for(n_lines, 1024), 64)), dim3(1024), 0, s, d_order_skus, n_lines,
                           n_skus, freq, err);
        hipLaunchKernelGGL(km_hist_kernel, dim3(std::min(grid_for(n_skus, 1024), 128)), dim3(1024), 0, s, freq, n_skus, hist);
        hipLaunchKernelGGL(km_lloyd_kernel, dim3(1), dim3(KM_BLOCK), 0, s, hist, n_bins, k, max_iter, label, st);
        hipLaunchKernelGGL(km_label_kernel, dim3(grid_for(n_skus, 256)), dim3(256), 0, s, freq, n_skus, label, st,
                           d_category);
        WO_HIP(hipGetLastError());
        WO_HIP(hipMemcpyAsync(&h, st, sizeof(KmState), hipMemcpyDeviceToHost, s));
        WO_HIP(hipMemcpyAsync(&h_err, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        WO_HIP(hipStreamSynchronize(s));
        if (h_err) return wo_fail(WO_E_INVAL, "an order line names a SKU outside 0 .. %d", n_skus - 1);
        return WO_OK;
    };
    ret = run();
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (ret == WO_OK) {
        if (k_used) *k_used = h.k_used;
        if (n_iter) *n_iter = h.n_iter;
    }
    return ret;
}

extern "C" wo_status wo_kmeans_categories_noalloc(const int32_t *d_order_skus, int64_t n_lines, int32_t n_skus,
                                                  int32_t k, int32_t max_iter, int32_t *d_category,
                                                  int32_t *d_k_used, int32_t *d_n_iter, void *stream)
{
    if (!d_order_skus || !d_category) return wo_fail(WO_E_INVAL, "NULL device buffer");
    if (n_lines < 1 || n_lines > WO_MAX_LINES)
        return wo_fail(WO_E_RANGE, "n_lines must be in 1 .. %d", WO_MAX_LINES);
    if (n_skus < 1 || n_skus > WO_MAX_LOCATIONS)
        return wo_fail(WO_E_RANGE, "n_skus must be in 1 .. %d", WO_MAX_LOCATIONS);
    if (k < 1 || k > KM_MAX) return wo_fail(WO_E_RANGE, "k must be in 1 .. %d", KM_MAX);
    if (max_iter < 1 || max_iter > WO_KMEANS_NOALLOC_MAX_ITER)
        return wo_fail(WO_E_RANGE, "max_iter must be in 1 .. %d", WO_KMEANS_NOALLOC_MAX_ITER);
    const int32_t n_bins = (int32_t)n_lines + 1;
    const KmLayout Ly = km_layout(n_skus, n_bins);
    if (Ly.bytes > (size_t)WO_KMEANS_NOALLOC_SCRATCH)
        return wo_fail(WO_E_RANGE, "%d SKUs and %lld lines need %zu bytes of scratch, more than the %d it has",
                       n_skus, (long long)n_lines, Ly.bytes, WO_KMEANS_NOALLOC_SCRATCH);
    void *base = nullptr;
    wo_status st0 = km_scratch_address(&base);
    if (st0) return st0;
    hipStream_t s = (hipStream_t)stream;
    char *buf = (char *)base;
    int32_t *freq = (int32_t *)buf, *hist = (int32_t *)(buf + Ly.o_hist), *label = (int32_t *)(buf + Ly.o_label);
    KmState *st = (KmState *)(buf + Ly.o_state);
    int32_t *err = (int32_t *)(buf + Ly.o_err);
    // the previous call's contents stay in the array: clear what starts at
    // zero (frequencies, histogram, state, flag) and mark no cluster yet
    const int64_t w_lab = (int64_t)(Ly.o_state - Ly.o_label) / 4, w_state = (int64_t)(Ly.bytes - Ly.o_state) / 4;
    hipLaunchKernelGGL(km_fill_kernel, dim3(grid_for((int64_t)Ly.o_label / 4, 256)), dim3(256), 0, s, freq,
                       (int64_t)Ly.o_label / 4, 0);
    hipLaunchKernelGGL(km_fill_kernel, dim3(grid_for(w_lab, 256)), dim3(256), 0, s, label, w_lab, -1);
    hipLaunchKernelGGL(km_fill_kernel, dim3(1), dim3(256), 0, s, (int32_t *)st, w_state, 0);
    hipLaunchKernelGGL(km_freq_kernel, dim3(std::min(grid_for(n_lines, 1024), 64)), dim3(1024), 0, s, d_order_skus, n_lines, n_skus,
                       freq, err);
    hipLaunchKernelGGL(km_hist_kernel, dim3(std::min(grid_for(n_skus, 1024), 128)), dim3(1024), 0, s, freq, n_skus, hist);
    hipLaunchKernelGGL(km_lloyd_kernel, dim3(1), dim3(KM_BLOCK), 0, s, hist, n_bins, k, max_iter, label, st);
    hipLaunchKernelGGL(km_label_kernel, dim3(grid_for(n_skus, 256)), dim3(256), 0, s, freq, n_skus, label, st,
                       d_category);
    hipLaunchKernelGGL(km_finish_kernel, dim3(1), dim3(64), 0, s, st, err, d_k_used, d_n_iter);
    WO_HIP(hipGetLastError());
    return WO_OK;
}
