// Instantiation of the operator-apply kernels in FP64.
#include "kernels.hpp"
#include "launch.hpp"

namespace fillk {
template hipError_t launch_r2c<double>(int, const RowArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_c2r<double>(int, const RowArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_col<double>(int, const ColArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_proj<double>(bool, const RowArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template int row_block_rows<double>(int);
template hipError_t launch_xr<double>(bool, const RowArgs<double>&, int, hipStream_t);
}  // namespace fillk
