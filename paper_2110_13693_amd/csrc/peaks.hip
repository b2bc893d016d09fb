// Measured integer VALU throughput of the device: the denominator the
// evaluator's roofline reports beside the one derived from the unit counts
// (256 CUs x 64 lanes x 2.4 GHz, one 32-bit integer operation per lane per
// clock).  Every lane runs sixteen independent chains of one 32-bit add and
// one exclusive or per step, written in assembly so that the compiler can
// neither fold nor pack them; the grid fills every wave slot of every CU.
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

}  // namespace

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
