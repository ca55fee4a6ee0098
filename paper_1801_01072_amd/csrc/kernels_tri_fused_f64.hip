// kernels_tri_fused_f64.hip -- the multi-step tridiagonal kernel in FP64.
#include "tri_fused_impl.hpp"

namespace ent {
template hipError_t launch_tri_fused<double>(const TriFusedArgs &, int32_t, hipStream_t);
}  // namespace ent
