// kernels_tri_fused_f32.hip -- the multi-step tridiagonal kernel in FP32.
#include "tri_fused_impl.hpp"

namespace ent {
template hipError_t launch_tri_fused<float>(const TriFusedArgs &, int32_t, hipStream_t);
}  // namespace ent
