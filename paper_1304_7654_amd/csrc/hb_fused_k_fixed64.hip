// Instantiation of the fused stage kernel (hb_fused_kernel.hpp), FP32 bulk
// and FP64: fixed grid, 64-bit halo offsets (states of 4 GiB or more).
#include "hb_fused_kernel.hpp"

namespace hb {
namespace fk {
template int launch_stage<float, false, true>(hb_grid *, const FusedArgs<float> &, bool, int, hipStream_t);
template int launch_stage<double, false, true>(hb_grid *, const FusedArgs<double> &, bool, int, hipStream_t);
}  // namespace fk
}  // namespace hb
