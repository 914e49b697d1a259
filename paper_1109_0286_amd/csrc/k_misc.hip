// CG set-up, per-problem sums and elementwise helpers of the refinement loop
// (Sec. 2.4 solve; FP64 true residual and correction of the mixed path).
// Batched launches use blockIdx.y = problem; compact vectors of problem b
// occupy [comp_off[b], comp_off[b+1]).
#include "kernels.hpp"
#include "launch.hpp"

namespace fillk {

namespace {
constexpr int RT = 256;  // threads of the per-problem reductions

inline dim3 grid_for(size_t n, int ny = 1) {
  size_t g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  if (g == 0) g = 1;
  return dim3((unsigned)g, (unsigned)ny);
}
}  // namespace

// Start of an inner solve: rho[0] = 1 so that the first iteration's
// p = z + beta p (p = 0) is p = z for any finite beta.  Inactive problems
// (converged or failed in the refinement loop) are marked done at once.
__global__ void k_cg_init(CGScalars* sc, const double* tol2, const int* cap, const int* active, int nprob) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nprob) return;
  CGScalars& s = sc[b];
  s.rho[0] = 1.0;
  s.rho[1] = 1.0;
  s.alpha = 0.0;
  s.beta = 0.0;
  s.alph[0] = __builtin_huge_val();  // single-reduction CG: the first alpha is rho / mu
  s.alph[1] = __builtin_huge_val();
  s.rr = 0.0;
  s.tol2 = tol2[b];
  s.done = active[b] ? 0 : 1;
  s.iter = 0;
  s.max_iter = cap[b];
  s.status = 0;
  s.cap = 0;
}

// out[b] = sum of part[b*stride + i], i < n: fixed order (thread t adds
// i = t, t+RT, ...; then a fixed tree), hence deterministic.
__global__ __launch_bounds__(RT) void k_sum(double* out, const double* part, size_t stride, int n) {
  const double* p = part + (size_t)blockIdx.x * stride;
  double v = 0.0, w = 0.0;
  for (int i = threadIdx.x; i < n; i += RT) v += p[i];
  block_sum2<RT>(v, w);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

template <typename TO, typename TI>
__global__ void k_scale(TO* out, const TI* in, const double* scale, const int* comp_off) {
  const int b = blockIdx.y;
  const int c0 = comp_off[b], c1 = comp_off[b + 1];
  const double s = scale[b];
  for (int c = c0 + blockIdx.x * blockDim.x + threadIdx.x; c < c1; c += gridDim.x * blockDim.x)
    out[c] = (TO)((double)in[c] * s);
}

// out = s in, with z0 and z1 (and zu when given) cleared over the same range
// (the start of an inner solve: r = scaled residual, x = p = 0; on the first
// refinement step also the FP64 solution u = 0).
template <typename TO>
__global__ void k_scale_init(TO* out, const double* in, const double* scale, const int* comp_off, TO* z0, TO* z1,
                             double* zu) {
  const int b = blockIdx.y;
  const int c0 = comp_off[b], c1 = comp_off[b + 1];
  const double s = scale[b];
  for (int c = c0 + blockIdx.x * blockDim.x + threadIdx.x; c < c1; c += gridDim.x * blockDim.x) {
    out[c] = (TO)(in[c] * s);
    z0[c] = TO(0);
    z1[c] = TO(0);
    if (zu) zu[c] = 0.0;
  }
}

template <typename TX>
__global__ void k_axpy(double* y, const TX* x, const double* a, const int* comp_off) {
  const int b = blockIdx.y;
  const int c0 = comp_off[b], c1 = comp_off[b + 1];
  const double s = a[b];
  if (s == 0.0) return;
  for (int c = c0 + blockIdx.x * blockDim.x + threadIdx.x; c < c1; c += gridDim.x * blockDim.x)
    y[c] += s * (double)x[c];
}

__global__ void k_scatter_add(double* const* full, const double* c, const int* pos, const int* comp_off) {
  const int b = blockIdx.y;
  const int c0 = comp_off[b], c1 = comp_off[b + 1];
  double* f = full[b];
  for (int i = c0 + blockIdx.x * blockDim.x + threadIdx.x; i < c1; i += gridDim.x * blockDim.x) f[pos[i]] += c[i];
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

// Conditional-mean set-up: x_out = mask ? 0 : d, t = mask ? 0 : d (problem blockIdx.y).
__global__ void k_mean_prep(double* const* x_out, double* t, const double* const* d, const uint8_t* mask,
                            size_t npix) {
  const size_t b = blockIdx.y;
  double* xo = x_out[b];
  const double* dd = d[b];
  double* tt = t + b * npix;
  const uint8_t* m = mask + b * npix;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npix; i += (size_t)gridDim.x * blockDim.x) {
    const bool mk = m[i] != 0;
    const double v = dd[i];
    xo[i] = mk ? 0.0 : v;
    tt[i] = mk ? 0.0 : v;
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

hipError_t launch_cg_init(CGScalars* sc, const double* tol2, const int* cap, const int* active, int nprob,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3((nprob + 63) / 64), dim3(64), 0, s, sc, tol2, cap, active, nprob);
  return hipGetLastError();
}
hipError_t launch_sum(double* out, const double* part, size_t stride, int n, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(nprob), dim3(RT), 0, s, out, part, stride, n);
  return hipGetLastError();
}
hipError_t launch_scale_to_f32(float* out, const double* in, const double* scale, const int* comp_off, int nmax,
                               int nprob, hipStream_t s) {
  hipLaunchKernelGGL((k_scale<float, double>), grid_for(nmax, nprob), dim3(256), 0, s, out, in, scale, comp_off);
  return hipGetLastError();
}
hipError_t launch_scale_f64(double* out, const double* in, const double* scale, const int* comp_off, int nmax,
                            int nprob, hipStream_t s) {
  hipLaunchKernelGGL((k_scale<double, double>), grid_for(nmax, nprob), dim3(256), 0, s, out, in, scale, comp_off);
  return hipGetLastError();
}
hipError_t launch_scale_init_f32(float* out, const double* in, const double* scale, const int* comp_off, float* z0,
                                 float* z1, double* zu, int nmax, int nprob, hipStream_t s) {
  hipLaunchKernelGGL((k_scale_init<float>), grid_for(nmax, nprob), dim3(256), 0, s, out, in, scale, comp_off, z0, z1,
                     zu);
  return hipGetLastError();
}
hipError_t launch_scale_init_f64(double* out, const double* in, const double* scale, const int* comp_off, double* z0,
                                 double* z1, double* zu, int nmax, int nprob, hipStream_t s) {
  hipLaunchKernelGGL((k_scale_init<double>), grid_for(nmax, nprob), dim3(256), 0, s, out, in, scale, comp_off, z0, z1,
                     zu);
  return hipGetLastError();
}
hipError_t launch_axpy_f64(double* y, const double* x, const double* a, const int* comp_off, int nmax, int nprob,
                           hipStream_t s) {
  hipLaunchKernelGGL((k_axpy<double>), grid_for(nmax, nprob), dim3(256), 0, s, y, x, a, comp_off);
  return hipGetLastError();
}
hipError_t launch_axpy_f32(double* y, const float* x, const double* a, const int* comp_off, int nmax, int nprob,
                           hipStream_t s) {
  hipLaunchKernelGGL((k_axpy<float>), grid_for(nmax, nprob), dim3(256), 0, s, y, x, a, comp_off);
  return hipGetLastError();
}
hipError_t launch_scatter_add(double* const* full, const double* c, const int* pos, const int* comp_off, int nmax,
                              int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_add, grid_for(nmax, nprob), dim3(256), 0, s, full, c, pos, comp_off);
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
hipError_t launch_mean_prep(double* const* x_out, double* t, const double* const* d, const uint8_t* mask,
                            size_t npix, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_mean_prep, grid_for(npix, nprob), dim3(256), 0, s, x_out, t, d, mask, npix);
  return hipGetLastError();
}
hipError_t launch_philox_words(uint64_t* out, uint64_t seed, uint64_t stream, int64_t nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_words, grid_for((size_t)nblocks), dim3(256), 0, s, out, seed, stream, nblocks);
  return hipGetLastError();
}

}  // namespace fillk
