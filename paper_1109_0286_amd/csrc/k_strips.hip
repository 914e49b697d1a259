// Strip subdivision of the masked region (Sec. 6.2): the top-hat convolution
// of the observed indicator with a periodic disk, as exact integer counts from
// per-row prefix sums, and the threshold test that puts a masked pixel into
// the strip of width w.  Also the per-pixel kernel classes and the
// class-wise update of the kernel-based Laplace relaxation (Sec. 6.3).
#include "launch.hpp"

namespace fillk {

namespace {
constexpr int ST = 256;
}

// pre[y][0] = 0, pre[y][x + 1] = pre[y][x] + (mask[y][x] == 0): one thread per row.
__global__ void k_row_prefix(const uint8_t* mask, int* pre, int nx, int ny) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= ny) return;
  const uint8_t* m = mask + (size_t)y * nx;
  int* p = pre + (size_t)y * (nx + 1);
  int acc = 0;
  p[0] = 0;
  for (int x = 0; x < nx; ++x) {
    acc += m[x] == 0 ? 1 : 0;
    p[x + 1] = acc;
  }
}

// out[i] = 1 for a masked pixel whose disk (row dy in [-r, r] spans columns
// x - hw[dy + r] .. x + hw[dy + r], periodic, 2 hw + 1 <= nx) holds more than
// thr_count observed pixels; 0 elsewhere.
__global__ __launch_bounds__(ST) void k_disk_strip(const uint8_t* mask, const int* pre, const int* hw, int r, int nx,
                                                   int ny, double thr_count, uint8_t* out) {
  const size_t npix = (size_t)nx * ny;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npix; i += (size_t)gridDim.x * blockDim.x) {
    if (mask[i] == 0) {
      out[i] = 0;
      continue;
    }
    const int y = (int)(i / nx), x = (int)(i % nx);
    long long cnt = 0;
    for (int dy = -r; dy <= r; ++dy) {
      int yy = (y + dy) % ny;
      if (yy < 0) yy += ny;
      const int h = hw[dy + r];
      const int* p = pre + (size_t)yy * (nx + 1);
      const int a = x - h, b = x + h;  // inclusive span
      if (a >= 0 && b < nx) cnt += p[b + 1] - p[a];
      else if (a < 0) cnt += (p[b + 1] - p[0]) + (p[nx] - p[nx + a]);
      else cnt += (p[nx] - p[a]) + (p[b - nx + 1] - p[0]);
    }
    out[i] = (double)cnt > thr_count ? 1 : 0;
  }
}

// x[i] = mask[i] ? 0 : d[i]
__global__ __launch_bounds__(ST) void k_select_observed(double* x, const double* d, const uint8_t* mask, size_t npix) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npix; i += (size_t)gridDim.x * blockDim.x)
    x[i] = mask[i] != 0 ? 0.0 : d[i];
}

// cls[i] = j for masked pixels whose disk touches no observed pixel (flag 0).
__global__ __launch_bounds__(ST) void k_class_raise(uint8_t* cls, const uint8_t* touch, const uint8_t* mask, int j,
                                                    size_t npix) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npix; i += (size_t)gridDim.x * blockDim.x)
    if (mask[i] != 0 && touch[i] == 0) cls[i] = (uint8_t)j;
}

// cls[i] = mask ? 0 : 255
__global__ __launch_bounds__(ST) void k_class_init(uint8_t* cls, const uint8_t* mask, size_t npix) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npix; i += (size_t)gridDim.x * blockDim.x)
    cls[i] = mask[i] != 0 ? 0 : 255;
}

// x[i] = avg[i] on the pixels of class j
__global__ __launch_bounds__(ST) void k_take_class(double* x, const double* avg, const uint8_t* cls, int j,
                                                   size_t npix) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npix; i += (size_t)gridDim.x * blockDim.x)
    if (cls[i] == (uint8_t)j) x[i] = avg[i];
}

// tab[i] = X[i].x * scale (real part of a real even kernel's spectrum)
__global__ __launch_bounds__(ST) void k_real_scale(double* tab, const double2* X, double scale, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    tab[i] = X[i].x * scale;
}

namespace {
dim3 sgrid(size_t n) {
  size_t g = (n + ST - 1) / ST;
  if (g > 4096) g = 4096;
  if (g == 0) g = 1;
  return dim3((unsigned)g);
}
}  // namespace

hipError_t launch_class_init(uint8_t* cls, const uint8_t* mask, size_t npix, hipStream_t s) {
  hipLaunchKernelGGL(k_class_init, sgrid(npix), dim3(ST), 0, s, cls, mask, npix);
  return hipGetLastError();
}
hipError_t launch_class_raise(uint8_t* cls, const uint8_t* touch, const uint8_t* mask, int j, size_t npix,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_class_raise, sgrid(npix), dim3(ST), 0, s, cls, touch, mask, j, npix);
  return hipGetLastError();
}
hipError_t launch_take_class(double* x, const double* avg, const uint8_t* cls, int j, size_t npix, hipStream_t s) {
  hipLaunchKernelGGL(k_take_class, sgrid(npix), dim3(ST), 0, s, x, avg, cls, j, npix);
  return hipGetLastError();
}
hipError_t launch_real_scale(double* tab, const double2* X, double scale, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_real_scale, sgrid(n), dim3(ST), 0, s, tab, X, scale, n);
  return hipGetLastError();
}

hipError_t launch_strip_flags(const uint8_t* mask, int* pre, const int* hw, int r, int nx, int ny, double thr_count,
                              uint8_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_row_prefix, dim3((ny + 63) / 64), dim3(64), 0, s, mask, pre, nx, ny);
  const size_t npix = (size_t)nx * ny;
  size_t g = (npix + ST - 1) / ST;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_disk_strip, dim3((unsigned)g), dim3(ST), 0, s, mask, pre, hw, r, nx, ny, thr_count, out);
  return hipGetLastError();
}

hipError_t launch_select_observed(double* x, const double* d, const uint8_t* mask, size_t npix, hipStream_t s) {
  size_t g = (npix + ST - 1) / ST;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_select_observed, dim3((unsigned)g), dim3(ST), 0, s, x, d, mask, npix);
  return hipGetLastError();
}

}  // namespace fillk
