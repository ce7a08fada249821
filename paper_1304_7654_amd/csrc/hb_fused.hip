// Fused batched line-tile kernel (placeholder until written).
#include "hb_device.hpp"

namespace hb {
int fused_build_tiles(hb_grid *g) { g->n_tiles = 1; return HB_OK; }
int fused_residual(hb_grid *, const double *, double *, hipStream_t) {
    return fail(HB_ERR_UNSUPPORTED, "fused path not built");
}
int fused_rk_iterate(hb_grid *, double *, int, double *, hipStream_t) {
    return fail(HB_ERR_UNSUPPORTED, "fused path not built");
}
}  // namespace hb
