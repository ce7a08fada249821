// XCD-aware workgroup order for kernels with one thread per item and
// 256-thread workgroups.  The hardware deals workgroups round-robin to the
// 8 XCDs (one L2 each).  A kernel launched with xcd_grid(n) workgroups for
// n items takes logical workgroup (w mod 8) ceil(W/8) + w / 8 of the
// W = ceil(n / 256) it needs, so that each XCD walks a contiguous range of
// items and the stencil rows that neighbouring rows share stay in its L2.
// xcd_group returns -1 for the padding workgroups (at most 7).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hb {

constexpr int kXcdBS = 256;

inline unsigned xcd_grid(int64_t n) {
    const int64_t wg = (n + kXcdBS - 1) / kXcdBS;
    return (unsigned)(8 * ((wg + 7) / 8));
}

__device__ __forceinline__ int64_t xcd_group(int64_t n) {
    const int64_t wg = (n + kXcdBS - 1) / kXcdBS, per = (wg + 7) / 8;
    const int64_t L = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    return L < wg ? L : -1;
}

}  // namespace hb
