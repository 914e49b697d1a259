// Host-callable launchers of the device kernels (declarations).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fillk {

struct CGScalars;
template <typename T> struct RowArgs;
template <typename T> struct ColArgs;

// e0/e1 (may be null): events timestamped at the start and end of the dispatch.
template <typename T>
hipError_t launch_r2c(int mode, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_c2r(int mode, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_col(int ny, const ColArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_proj(const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T> int row_block_rows(int nx);

// Reset the device CG scalars at the start of an inner solve.
hipError_t launch_cg_init(CGScalars* sc, double tol2, int max_iter, hipStream_t s);
hipError_t launch_sum(double* out, const double* part, int n, hipStream_t s);

// Elementwise helpers.
hipError_t launch_to_f32_scaled(float* out, const double* in, double scale, int n, hipStream_t s);
hipError_t launch_scale_f64(double* out, const double* in, double scale, int n, hipStream_t s);
hipError_t launch_axpy_f64(double* y, const double* x, double a, int n, hipStream_t s);
hipError_t launch_axpy_f64_f32(double* y, const float* x, double a, int n, hipStream_t s);
hipError_t launch_scatter_add(double* full, const double* c, const int* pos, int n, hipStream_t s);
hipError_t launch_scatter(double* full, const double* c, const int* pos, int n, hipStream_t s);
hipError_t launch_scatter_f32(double* full, const float* c, const int* pos, int n, hipStream_t s);
hipError_t launch_gather(double* c, const double* full, const int* pos, int n, hipStream_t s);
hipError_t launch_mean_prep(double* x_out, double* t, const double* d, const uint8_t* mask, size_t npix,
                            hipStream_t s);
hipError_t launch_philox_words(uint64_t* out, uint64_t seed, uint64_t stream, int64_t nblocks,
                               hipStream_t s);

}  // namespace fillk
