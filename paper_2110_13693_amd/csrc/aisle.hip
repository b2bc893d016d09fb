// Aisle width design (arXiv 2110.13693, section 5, Subproblem 1, Eq. (1)):
// maximise the share of the floor the racks take, A_ind / A_max, subject to
// k * delta - a <= 0, where a is the width between racks and delta the
// picking frequency that Subproblem 2 returns for the picking plan
// (delta = f(d), Eq. (2)).  The two subproblems couple through a and delta:
// a narrower aisle shortens every route, raises delta and so the width the
// flow needs.
//
// Geometry of the single block: every aisle is a corridor of width a with a
// rack face of depth r on each side (racks of neighbouring aisles stand back
// to back), so aisles are a + 2r apart centre to centre; racks are L = S p
// long; a cross aisle of width c runs along the front and the back.  Then
//     A_ind / A_max = 2 r L / ((a + 2 r) (L + 2 c)),
// which falls with a, so the optimum is the narrowest feasible width.  delta
// falls as a grows (routes lengthen), so k delta(a) <= a holds from one width
// on: the optimum is the smallest width in [a_min, a_max] that meets it.
//
// Widths are whole decimetres, like every distance here.  The plan is
// evaluated at every width of the range in one launch of the exact
// evaluator, each copy of the plan with its own aisle spacing; the host then
// takes the first width that meets the constraint, deciding it in IEEE
// double from the integer distance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "wo_common.h"
#include "wo_internal.h"

namespace {

// rows x bytes copies of one row (bytes a multiple of 4)
__global__ void replicate_kernel(uint32_t *dst, const uint32_t *src, int64_t words_per_row, int64_t rows)
{
    const int64_t total = words_per_row * rows;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i % words_per_row];
}

}  // namespace

using namespace wo;

extern "C" wo_status wo_aisle_width(wo_wh *wh, int32_t inst, const uint8_t *d_zone_of, const uint16_t *d_order_seq,
                                    const wo_aisle_params *prm, int32_t *h_dist, void *stream, wo_aisle_result *out)
{
    if (!wh || !d_zone_of || !d_order_seq || !prm || !out) return wo_fail(WO_E_INVAL, "NULL argument");
    if (inst < 0 || inst >= instance_count(wh)) return wo_fail(WO_E_RANGE, "instance %d out of range", inst);
    const wo_aisle_params p = *prm;
    if (p.rack_depth_dm < 1 || p.cross_aisle_dm < 0 || p.min_width_dm < 1 || p.max_width_dm < p.min_width_dm ||
        !(p.k_dm >= 0.0))
        return wo_fail(WO_E_INVAL, "need rack depth >= 1, cross aisle >= 0, 1 <= min width <= max width, k >= 0");
    const int64_t G = (int64_t)p.max_width_dm - p.min_width_dm + 1;
    if (G > WO_AISLE_MAX_WIDTHS)
        return wo_fail(WO_E_RANGE, "%lld widths in the range, at most %d", (long long)G, WO_AISLE_MAX_WIDTHS);
    const InstDev &I = instance_dev(wh, inst);
    const int64_t w_max = (int64_t)p.max_width_dm + 2ll * p.rack_depth_dm;
    if (w_max >= (1ll << 24)) return wo_fail(WO_E_RANGE, "aisle spacing of %lld dm too large", (long long)w_max);
    if (I.route == WO_ROUTE_OPTIMAL &&
        4ll * w_max * (I.n_aisles + 2) + 4ll * I.L * (I.n_aisles + 1) >= (1ll << 30))
        return wo_fail(WO_E_RANGE, "the optimal route's 32-bit distances do not reach a spacing of %lld dm",
                       (long long)w_max);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = I.n_orders;
    const int64_t seq_words = (n * 2 + 3) / 4;          // a row of n uint16 ids, padded to words
    uint8_t *dz = nullptr;
    uint16_t *dq = nullptr;
    int32_t *dsp = nullptr, *dd = nullptr;
    uint32_t *dseq1 = nullptr;
    std::vector<int32_t> sp((size_t)G), dist((size_t)G);
    for (int64_t j = 0; j < G; j++) sp[(size_t)j] = p.min_width_dm + (int32_t)j + 2 * p.rack_depth_dm;
    if (wo_fault_injected()) return wo_fail(WO_E_NOMEM, "injected allocation failure");
    auto alloc = [](void **ptr, size_t bytes) -> bool {
        if (hipMalloc(ptr, bytes ? bytes : 16) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            return false;
        }
        return true;
    };
    wo_status st = WO_OK;
    if (!alloc((void **)&dz, (size_t)G * 64) || !alloc((void **)&dq, (size_t)G * n * 2) ||
        !alloc((void **)&dsp, (size_t)G * 4) || !alloc((void **)&dd, (size_t)G * 4) ||
        !alloc((void **)&dseq1, (size_t)seq_words * 4)) {
        st = wo_fail(WO_E_NOMEM, "device allocation for %lld widths failed", (long long)G);
    }
    auto run = [&]() -> wo_status {
        // the plan, once per width: zone rows, then sequence rows packed
        // back to back (a row of n ids need not fill whole words, so each
        // row is copied on its own when n is odd)
        WO_HIP(hipMemsetAsync(dseq1, 0, (size_t)seq_words * 4, s));
        WO_HIP(hipMemcpyAsync(dseq1, d_order_seq, (size_t)n * 2, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(replicate_kernel, dim3((unsigned)std::min<int64_t>((G * 16 + 255) / 256, 4096)), dim3(256),
                           0, s, (uint32_t *)dz, (const uint32_t *)d_zone_of, (int64_t)16, G);
        if ((n & 1) == 0) {
            hipLaunchKernelGGL(replicate_kernel,
                               dim3((unsigned)std::min<int64_t>((G * (n / 2) + 255) / 256, 4096)), dim3(256), 0, s,
                               (uint32_t *)dq, (const uint32_t *)dseq1, n / 2, G);
        } else {
            for (int64_t j = 0; j < G; j++)
                WO_HIP(hipMemcpyAsync(dq + j * n, d_order_seq, (size_t)n * 2, hipMemcpyDeviceToDevice, s));
        }
        WO_HIP(hipGetLastError());
        WO_HIP(hipMemcpyAsync(dsp, sp.data(), (size_t)G * 4, hipMemcpyHostToDevice, s));
        wo_status r = eval_instance(wh, inst, G, dz, dq, dd, nullptr, s, dsp);
        if (r) return r;
        WO_HIP(hipMemcpyAsync(dist.data(), dd, (size_t)G * 4, hipMemcpyDeviceToHost, s));
        WO_HIP(hipStreamSynchronize(s));
        return WO_OK;
    };
    if (!st) st = run();
    (void)hipStreamSynchronize(s);
    if (dz) (void)hipFree(dz);
    if (dq) (void)hipFree(dq);
    if (dsp) (void)hipFree(dsp);
    if (dd) (void)hipFree(dd);
    if (dseq1) (void)hipFree(dseq1);
    if (st) return st;
    if (h_dist) std::copy(dist.begin(), dist.end(), h_dist);
    // delta(a) = n_orders * window / (D / walk + t_item * items), one
    // operation per statement (no contraction), as the rate of the evaluator
    auto delta_of = [&](int32_t D) {
        const double q = (double)D / I.walk;
        const double u = I.t_item * (double)I.n_lines;
        const double T = q + u;
        const double num = (double)I.n_orders * I.window;
        return num / T;
    };
    int64_t pick = G - 1;
    bool feasible = false;
    for (int64_t j = 0; j < G; j++) {
        const double need = p.k_dm * delta_of(dist[(size_t)j]);
        if (need <= (double)(p.min_width_dm + j)) {
            pick = j;
            feasible = true;
            break;
        }
    }
    const int32_t a = p.min_width_dm + (int32_t)pick;
    const double L = (double)I.L, r = (double)p.rack_depth_dm, c = (double)p.cross_aisle_dm;
    const double num = 2.0 * r * L;
    const double den1 = (double)a + 2.0 * r;
    const double den2 = L + 2.0 * c;
    const double den = den1 * den2;
    out->width_dm = a;
    out->spacing_dm = sp[(size_t)pick];
    out->feasible = feasible ? 1 : 0;
    out->widths_evaluated = (int32_t)G;
    out->distance = dist[(size_t)pick];
    out->orders_per_window = delta_of(dist[(size_t)pick]);
    out->utilization = num / den;
    return WO_OK;
}
