// Measured peaks of the device: the denominators the rooflines report beside
// the ones derived from unit counts, clock and the published figures.
//   - integer VALU (the evaluator's roof): every lane runs sixteen independent
//     chains of one 32-bit add and one exclusive or per step, written in
//     assembly so that the compiler can neither fold nor pack them; the grid
//     fills every wave slot of every CU;
//   - LDS read bandwidth: every wave reads 1 KB per instruction (16 bytes a
//     lane, consecutive, so no bank conflicts) from a 16 KB table;
//   - HBM read bandwidth: a 1 GiB buffer read once with 16-byte loads;
//   - BF16 MFMA: every wave runs four independent 32 x 32 x 16 products
//     (v_mfma_f32_32x32x16_bf16: the 16 x 16 x 32 form reaches only about
//     0.6 of this rate).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wo_common.h"

namespace {

constexpr int PK_CHAINS = 16;

__global__ __launch_bounds__(256) void valu_int_kernel(uint32_t *out, int32_t steps, uint32_t seed)
{
    uint32_t a[PK_CHAINS];
#pragma unroll
    for (int k = 0; k < PK_CHAINS; k++) a[k] = seed ^ (uint32_t)(threadIdx.x * PK_CHAINS + k);
    const uint32_t c = seed | 1u, d = seed * 2654435761u;
    for (int32_t i = 0; i < steps; i++) {
#pragma unroll
        for (int k = 0; k < PK_CHAINS; k++)
            asm volatile("v_add_u32 %0, %0, %1\n\tv_xor_b32 %0, %0, %2" : "+v"(a[k]) : "v"(c), "v"(d));
    }
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < PK_CHAINS; k++) x ^= a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

__global__ __launch_bounds__(256) void lds_read_kernel(uint32_t *out, int32_t steps)
{
    __shared__ uint4 tab[1024];
    const int tid = threadIdx.x;
    for (int i = tid; i < 1024; i += 256) tab[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
    __syncthreads();
    uint4 x = make_uint4(0u, 0u, 0u, 0u);
    const int w = tid >> 6, lane = tid & 63;
    for (int32_t i = 0; i < steps; i++) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint4 v = tab[(((i * 4 + k + w) & 15) << 6) + lane];   // 1 KB contiguous per wave
            x.x ^= v.x;
            x.y += v.y;
            x.z ^= v.z;
            x.w += v.w;
        }
    }
    out[blockIdx.x * blockDim.x + tid] = x.x ^ x.y ^ x.z ^ x.w;
}

typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t pk_u32x4;

__global__ __launch_bounds__(256) void hbm_read_kernel(const pk_u32x4 *buf, int64_t n16, uint32_t *out)
{
    uint32_t x = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const pk_u32x4 v = __builtin_nontemporal_load(buf + i);
        x ^= v[0] ^ v[1] ^ v[2] ^ v[3];
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

// L2: each XCD re-reads a 2 MB slice of its own (workgroups go to the XCDs in
// turn, so workgroup b reads slice b % 8), small enough to stay in its L2,
// with 16-byte loads; passes x 8 slices are read in all
constexpr int64_t L2_SLICE16 = (int64_t)(2 << 20) / 16;   // 16-byte elements per slice (a power of 2)
__global__ __launch_bounds__(256) void l2_read_kernel(const pk_u32x4 *buf, int32_t passes, uint32_t *out)
{
    const pk_u32x4 *sl = buf + (int64_t)(blockIdx.x & 7) * L2_SLICE16;
    const int64_t stride = (int64_t)(gridDim.x >> 3) * blockDim.x, end = (int64_t)passes * L2_SLICE16;
    uint32_t x = 0;
#pragma unroll 8
    for (int64_t e = (int64_t)(blockIdx.x >> 3) * blockDim.x + threadIdx.x; e < end; e += stride) {
        const pk_u32x4 v = sl[e & (L2_SLICE16 - 1)];
        x ^= v[0] ^ v[1] ^ v[2] ^ v[3];
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 pk_bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float pk_floatx16;
constexpr int PK_MFMA_CHAINS = 4;

__global__ __launch_bounds__(256) void mfma_bf16_kernel(float *out, int32_t steps)
{
    const int lane = threadIdx.x & 63;
    pk_bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        a[e] = (__bf16)(0.001f * (float)((lane + e) & 7));
        b[e] = (__bf16)(0.002f * (float)((lane * 3 + e) & 7));
    }
    pk_floatx16 acc[PK_MFMA_CHAINS];
#pragma unroll
    for (int k = 0; k < PK_MFMA_CHAINS; k++)
#pragma unroll
        for (int e = 0; e < 16; e++) acc[k][e] = 0.f;
    for (int32_t i = 0; i < steps; i++) {
#pragma unroll
        for (int k = 0; k < PK_MFMA_CHAINS; k++) acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[k], 0, 0, 0);
    }
    float x = 0.f;
#pragma unroll
    for (int k = 0; k < PK_MFMA_CHAINS; k++)
#pragma unroll
        for (int e = 0; e < 16; e++) x += acc[k][e];
    out[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

// Best of `reps` timed launches of `launch` (after one warm-up), in ms.
template <typename F>
wo_status best_ms(hipStream_t s, int32_t reps, F launch, float *best)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    wo_status st = WO_OK;
    *best = 3.0e38f;
    auto run = [&]() -> wo_status {
        WO_HIP(hipEventCreate(&e0));
        WO_HIP(hipEventCreate(&e1));
        launch();
        WO_HIP(hipGetLastError());
        for (int r = 0; r < reps; r++) {
            WO_HIP(hipEventRecord(e0, s));
            launch();
            WO_HIP(hipEventRecord(e1, s));
            WO_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            WO_HIP(hipEventElapsedTime(&ms, e0, e1));
            *best = std::min(*best, ms);
        }
        return WO_OK;
    };
    st = run();
    (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

extern "C" wo_status wo_measure_peaks(int32_t reps, wo_peaks *out, void *stream)
{
    if (!out) return wo_fail(WO_E_INVAL, "out is NULL");
    if (reps < 1 || reps > 100) return wo_fail(WO_E_RANGE, "reps must be in 1 .. 100");
    wo_status st = wo_measure_int_peak(reps, &out->int_ops_per_s, stream);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    WO_HIP(hipGetDevice(&dev));
    WO_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t hbm_bytes = (int64_t)1 << 30;
    const int grid_small = cus * 8, grid_hbm = cus * 16;
    uint32_t *o32 = nullptr;
    float *of = nullptr;
    pk_u32x4 *buf = nullptr;
    if (wo_fault_injected()) return wo_fail(WO_E_NOMEM, "injected allocation failure");
    if (hipMalloc((void **)&o32, sizeof(uint32_t) * (size_t)grid_hbm * 256) != hipSuccess ||
        hipMalloc((void **)&of, sizeof(float) * (size_t)grid_small * 256) != hipSuccess ||
        hipMalloc((void **)&buf, (size_t)hbm_bytes) != hipSuccess) {
        (void)hipGetLastError();
        if (o32) (void)hipFree(o32);
        if (of) (void)hipFree(of);
        if (buf) (void)hipFree(buf);
        return wo_fail(WO_E_NOMEM, "hipMalloc failed");
    }
    float ms = 0.f;
    const int32_t lds_steps = 4096, mfma_steps = 2048;
    if (hipMemsetAsync(buf, 0x5A, (size_t)hbm_bytes, s) != hipSuccess) st = wo_fail(WO_E_DEVICE, "hipMemsetAsync failed");
    if (!st)
        st = best_ms(s, reps, [&] {
            hipLaunchKernelGGL(lds_read_kernel, dim3(grid_small), dim3(256), 0, s, o32, lds_steps);
        }, &ms);
    if (!st) out->lds_bytes_per_s = 4.0 * 16.0 * lds_steps * (double)grid_small * 256.0 / (ms * 1e-3);
    if (!st)
        st = best_ms(s, reps, [&] {
            hipLaunchKernelGGL(hbm_read_kernel, dim3(grid_hbm), dim3(256), 0, s, buf, hbm_bytes / 16, o32);
        }, &ms);
    if (!st) out->hbm_read_bytes_per_s = (double)hbm_bytes / (ms * 1e-3);
    const int32_t l2_passes = 64;
    if (!st)
        st = best_ms(s, reps, [&] {
            hipLaunchKernelGGL(l2_read_kernel, dim3(grid_small), dim3(256), 0, s, buf, l2_passes, o32);
        }, &ms);
    if (!st) out->l2_read_bytes_per_s = 8.0 * 16.0 * (double)L2_SLICE16 * l2_passes / (ms * 1e-3);
    if (!st)
        st = best_ms(s, reps, [&] {
            hipLaunchKernelGGL(mfma_bf16_kernel, dim3(grid_small), dim3(256), 0, s, of, mfma_steps);
        }, &ms);
    if (!st)
        out->bf16_flops_per_s =
            32.0 * 32.0 * 16.0 * 2.0 * PK_MFMA_CHAINS * mfma_steps * (double)grid_small * 4.0 / (ms * 1e-3);
    (void)hipStreamSynchronize(s);
    (void)hipFree(o32);
    (void)hipFree(of);
    (void)hipFree(buf);
    return st;
}

extern "C" wo_status wo_measure_int_peak(int32_t reps, double *ops_per_s, void *stream)
{
    if (!ops_per_s) return wo_fail(WO_E_INVAL, "ops_per_s is NULL");
    if (reps < 1 || reps > 100) return wo_fail(WO_E_RANGE, "reps must be in 1 .. 100");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0, per_cu = 0;
    WO_HIP(hipGetDevice(&dev));
    WO_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    WO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, valu_int_kernel, 256, 0));
    const int grid = cus * std::max(per_cu, 1);
    const int32_t steps = 4096;
    uint32_t *out = nullptr;
    if (wo_fault_injected()) return wo_fail(WO_E_NOMEM, "injected allocation failure");
    if (hipMalloc((void **)&out, sizeof(uint32_t) * (size_t)grid * 256) != hipSuccess) {
        (void)hipGetLastError();
        return wo_fail(WO_E_NOMEM, "hipMalloc failed");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    wo_status st = WO_OK;
    float best = 3.0e38f;
    auto run = [&]() -> wo_status {
        WO_HIP(hipEventCreate(&e0));
        WO_HIP(hipEventCreate(&e1));
        hipLaunchKernelGGL(valu_int_kernel, dim3(grid), dim3(256), 0, s, out, steps, 7u);   // warm-up
        for (int r = 0; r < reps; r++) {
            WO_HIP(hipEventRecord(e0, s));
            hipLaunchKernelGGL(valu_int_kernel, dim3(grid), dim3(256), 0, s, out, steps, (uint32_t)r);
            WO_HIP(hipEventRecord(e1, s));
            WO_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            WO_HIP(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return WO_OK;
    };
    st = run();
    (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (st) return st;
    const double ops = 2.0 * PK_CHAINS * (double)steps * (double)grid * 256.0;
    *ops_per_s = ops / (best * 1e-3);
    return WO_OK;
}
