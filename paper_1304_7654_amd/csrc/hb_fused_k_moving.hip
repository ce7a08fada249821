// Instantiation of the fused stage kernel (hb_fused_kernel.hpp), FP32 bulk
// and FP64: rigidly moving grid, 32-bit halo offsets.
#include "hb_fused_kernel.hpp"

namespace hb {
namespace fk {
template int launch_stage<float, true, false>(hb_grid *, const FusedArgs<float> &, bool, int, hipStream_t);
template int launch_stage<double, true, false>(hb_grid *, const FusedArgs<double> &, bool, int, hipStream_t);
}  // namespace fk
}  // namespace hb
