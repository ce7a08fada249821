// Reverse-mode residual and force kernels (placeholder until written).
#include "hb_device.hpp"

namespace hb {
int launch_residual_adjoint(hb_grid *, const double *, const double *, double *, double *,
                            double *, hipStream_t) {
    return fail(HB_ERR_UNSUPPORTED, "adjoint not built");
}
int launch_forces_adjoint(hb_grid *, const double *, const double *, double *, double *,
                          double *, hipStream_t) {
    return fail(HB_ERR_UNSUPPORTED, "forces adjoint not built");
}
}  // namespace hb
