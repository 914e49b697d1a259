// Instantiation of the operator-apply kernels in FP32 (inner CG of the mixed path).
#include "kernels.hpp"
#include "launch.hpp"

namespace fillk {
template hipError_t launch_r2c<float>(int, const RowArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_c2r<float>(int, const RowArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_col<float>(int, const ColArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_proj<float>(bool, const RowArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
template int row_block_rows<float>(int);
template hipError_t launch_xr<float>(bool, const RowArgs<float>&, int, hipStream_t);
}  // namespace fillk
