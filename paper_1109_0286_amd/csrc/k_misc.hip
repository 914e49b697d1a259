// CG scalar recurrences (Hestenes-Stiefel, Sec. 2.4) and elementwise helpers.
#include "kernels.hpp"
#include "launch.hpp"

namespace fillk {

namespace {
constexpr int RT = 256;  // threads of the single-workgroup reductions

// Deterministic sum: thread t adds part[t], part[t+RT], ... in order, then a
// fixed tree over the workgroup.
__device__ double fixed_sum(const double* part, int n) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += RT) v += part[i];
  double w = 0.0;
  block_sum2<RT>(v, w);
  return v;  // valid in thread 0
}
}  // namespace

// Start of an inner solve: rho[0] = 1 so that the first iteration's
// p = z + beta p (p = 0) is p = z for any finite beta.
__global__ void k_cg_init(CGScalars* sc, double tol2, int max_iter) {
  if (threadIdx.x == 0) {
    sc->rho[0] = 1.0;
    sc->rho[1] = 1.0;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->rr = 0.0;
    sc->tol2 = tol2;
    sc->done = 0;
    sc->iter = 0;
    sc->max_iter = max_iter;
    sc->status = 0;
    sc->cap = 0;
  }
}

__global__ __launch_bounds__(RT) void k_sum(double* out, const double* part, int n) {
  const double s = fixed_sum(part, n);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ void k_to_f32_scaled(float* out, const double* in, double scale, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = (float)(in[i] * scale);
}
__global__ void k_scale_f64(double* out, const double* in, double scale, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = in[i] * scale;
}
__global__ void k_axpy_f64(double* y, const double* x, double a, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] += a * x[i];
}
__global__ void k_axpy_f64_f32(double* y, const float* x, double a, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    y[i] += a * (double)x[i];
}
__global__ void k_scatter_add(double* full, const double* c, const int* pos, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) full[pos[i]] += c[i];
}
__global__ void k_scatter(double* full, const double* c, const int* pos, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) full[pos[i]] = c[i];
}
__global__ void k_scatter_f32(double* full, const float* c, const int* pos, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    full[pos[i]] = (double)c[i];
}
__global__ void k_gather(double* c, const double* full, const int* pos, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c[i] = full[pos[i]];
}
__global__ void k_mean_prep(double* x_out, double* t, const double* d, const uint8_t* mask, size_t npix) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npix; i += (size_t)gridDim.x * blockDim.x) {
    const bool m = mask[i] != 0;
    const double v = d[i];
    x_out[i] = m ? 0.0 : v;
    t[i] = m ? 0.0 : v;
  }
}
__global__ void k_philox_words(uint64_t* out, uint64_t seed, uint64_t stream, int64_t nblocks) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nblocks;
       j += (int64_t)gridDim.x * blockDim.x) {
    const u64x4 w = philox4x64_10((uint64_t)j, 0, 0, 0, seed, stream);
    out[4 * j + 0] = w.w0;
    out[4 * j + 1] = w.w1;
    out[4 * j + 2] = w.w2;
    out[4 * j + 3] = w.w3;
  }
}

namespace {
inline dim3 grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g == 0) g = 1;
  return dim3((unsigned)g);
}
}  // namespace

hipError_t launch_cg_init(CGScalars* sc, double tol2, int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(64), 0, s, sc, tol2, max_iter);
  return hipGetLastError();
}
hipError_t launch_sum(double* out, const double* part, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(RT), 0, s, out, part, n);
  return hipGetLastError();
}
hipError_t launch_to_f32_scaled(float* out, const double* in, double scale, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32_scaled, grid_for(n), dim3(256), 0, s, out, in, scale, n);
  return hipGetLastError();
}
hipError_t launch_scale_f64(double* out, const double* in, double scale, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_f64, grid_for(n), dim3(256), 0, s, out, in, scale, n);
  return hipGetLastError();
}
hipError_t launch_axpy_f64(double* y, const double* x, double a, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_f64, grid_for(n), dim3(256), 0, s, y, x, a, n);
  return hipGetLastError();
}
hipError_t launch_axpy_f64_f32(double* y, const float* x, double a, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_f64_f32, grid_for(n), dim3(256), 0, s, y, x, a, n);
  return hipGetLastError();
}
hipError_t launch_scatter_add(double* full, const double* c, const int* pos, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_add, grid_for(n), dim3(256), 0, s, full, c, pos, n);
  return hipGetLastError();
}
hipError_t launch_scatter(double* full, const double* c, const int* pos, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, grid_for(n), dim3(256), 0, s, full, c, pos, n);
  return hipGetLastError();
}
hipError_t launch_scatter_f32(double* full, const float* c, const int* pos, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_f32, grid_for(n), dim3(256), 0, s, full, c, pos, n);
  return hipGetLastError();
}
hipError_t launch_gather(double* c, const double* full, const int* pos, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, grid_for(n), dim3(256), 0, s, c, full, pos, n);
  return hipGetLastError();
}
hipError_t launch_mean_prep(double* x_out, double* t, const double* d, const uint8_t* mask, size_t npix,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_mean_prep, grid_for(npix), dim3(256), 0, s, x_out, t, d, mask, npix);
  return hipGetLastError();
}
hipError_t launch_philox_words(uint64_t* out, uint64_t seed, uint64_t stream, int64_t nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_words, grid_for((size_t)nblocks), dim3(256), 0, s, out, seed, stream, nblocks);
  return hipGetLastError();
}

}  // namespace fillk
