// Deterministic second pass of the residual-norm reduction: one workgroup
// sums the per-workgroup FP64 partials in a fixed order and writes
// sqrt(sum / cell_snapshots) to out[*ctr], then advances the counter.  Each
// thread keeps four running sums whose loads are independent, so that the
// pass waits for memory a quarter as often as with one dependent chain.
#include "hb_device.hpp"

namespace hb {
namespace {

constexpr int kBS = 256;
constexpr int kFin = 1024;       // threads of the finalize workgroup

__global__ void __launch_bounds__(kFin) k_norm_finalize(const double *partials, int64_t n,
                                                        double inv_total, double *out, int *ctr) {
    __shared__ double red[kFin];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t k = threadIdx.x;
    for (; k + 3 * kFin < n; k += 4 * kFin) {
        a0 += partials[k];
        a1 += partials[k + kFin];
        a2 += partials[k + 2 * kFin];
        a3 += partials[k + 3 * kFin];
    }
    for (; k < n; k += kFin) a0 += partials[k];
    red[threadIdx.x] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    for (int s = kFin / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int it = *ctr;
        if (out) out[it] = sqrt(red[0] * inv_total);
        *ctr = it + 1;
    }
}

__global__ void k_reset(int *ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = 0;
}

}  // namespace

int launch_norm_finalize(hb_grid *g, const double *partials, int64_t n, double *out, int *ctr,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(kFin), 0, s, partials, n,
                       1.0 / (double)g->total_cs, out, ctr);
    return check_hip(hipGetLastError(), "norm finalize launch");
}

int launch_reset_ctr(int *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, ctr);
    return check_hip(hipGetLastError(), "counter reset launch");
}

}  // namespace hb
