// Deterministic second pass of the residual-norm reduction: one workgroup
// sums the per-workgroup FP64 partials in a fixed order and writes
// sqrt(sum / cell_snapshots) to out[*ctr], then advances the counter.
#include "hb_device.hpp"

namespace hb {
namespace {

constexpr int kBS = 256;

__global__ void k_norm_finalize(const double *partials, int64_t n, double inv_total,
                                double *out, int *ctr) {
    __shared__ double red[kBS];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += kBS) acc += partials[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
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
    hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(kBS), 0, s, partials, n,
                       1.0 / (double)g->total_cs, out, ctr);
    return check_hip(hipGetLastError(), "norm finalize launch");
}

int launch_reset_ctr(int *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, ctr);
    return check_hip(hipGetLastError(), "counter reset launch");
}

}  // namespace hb
