// Adjoint of the fill (gradient of a loss on the filled map with respect to
// the observed pixels and the band powers of P(k)).  The method is the
// constrained realization of Sec. 2.1 / 2.3; its derivative follows from the
// same linear algebra:
//   lambda = A^-1 g_x  (A = Px C^-1 Px, one extra CG solve with the operators
//   of Sec. 2.4), dL/dy = g_y - (C^-1 lambda)_y,
//   dL/dlnP_k = (1/N) [ sqrt(P_k)/2 Re(conj h_k w_k) + Re(conj lambda_k v_k)/P_k ]
// with h = Px g + Py C^-1 lambda, v = Py (y - s) + Px u, w the white noise.
// These kernels are FP64: the forward-only column FFT (with the packed
// DC/Nyquist column separated), the elementwise maps, the per-mode gradient
// and the per-band reduction.
#include "kernels.hpp"
#include "launch.hpp"

namespace fillk {

namespace {
constexpr int AT = 256;

inline dim3 grid_for(size_t n) {
  size_t g = (n + AT - 1) / AT;
  if (g > 4096) g = 4096;
  if (g == 0) g = 1;
  return dim3((unsigned)g);
}
}  // namespace

// Forward FFT along y of the nx/2 packed spectral columns; column 0 carries
// the real DC (real part) and Nyquist (imaginary part) sequences and is
// separated into columns 0 and nx/2 of the output (ncol = nx/2 + 1 columns).
template <int N>
__global__ __launch_bounds__((ColCfg<double, N>::THREADS)) void col_fwd_kernel(const double2* Xt, double2* Xs,
                                                                                int ldx, int nhalf,
                                                                                const double2* tw) {
  using C = double2;
  using CF = ColCfg<double, N>;
  using PL = typename CF::PL;
  constexpr int E = CF::E, TPL = CF::TPL, W = CF::W;
  constexpr int LE = lds_line_elems<PL>();
  __shared__ C lds[W * LE];
  __shared__ C twq[tw_elems<PL>() > 0 ? tw_elems<PL>() : 1];
  const int l = threadIdx.x / TPL, tid = threadIdx.x % TPL;
  const int kx = blockIdx.x * W + l;
  const bool valid = kx < nhalf;
  const C* g = Xt + (size_t)(valid ? kx : 0) * ldx;
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = valid ? g[tid + e * TPL] : C{0.0, 0.0};
  tw_stage<PL>(twq, tw, threadIdx.x, CF::THREADS);
  C* line = lds + l * LE;
  fft_line<C, PL, -1>(v, tid, line, twq);
  if (blockIdx.x == 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) line[lpad<PL>(tid + e * TPL)] = v[e];
    __syncthreads();
  }
  if (!valid) return;
  C* o = Xs + (size_t)kx * ldx;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int ky = tid + e * TPL;
    if (blockIdx.x == 0 && l == 0) {
      const C zk = v[e], zm = line[lpad<PL>(ky == 0 ? 0 : N - ky)];
      o[ky] = C{0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y)};                           // DC column
      Xs[(size_t)nhalf * ldx + ky] = C{0.5 * (zk.y + zm.y), 0.5 * (zm.x - zk.x)};    // Nyquist column
    } else {
      o[ky] = v[e];
    }
  }
}

// Elementwise maps of the adjoint, one problem:
//   grad_y = m ? 0 : g - cl;  h = m ? g : cl;  v = m ? x - s : d - s
__global__ void k_adj_maps(const uint8_t* mask, const double* g, const double* cl, const double* x,
                           const double* s, const double* d, double* grad_y, double* h, double* v, size_t npix) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npix; i += (size_t)gridDim.x * blockDim.x) {
    const bool m = mask[i] != 0;
    const double gi = g[i], ci = cl[i], si = s[i];
    grad_y[i] = m ? 0.0 : gi - ci;
    h[i] = m ? gi : ci;
    v[i] = m ? x[i] - si : d[i] - si;
  }
}

// b = g on masked pixels (compact), problem blockIdx.y
__global__ void k_adj_gather(double* b, double* const* g_tab, const int* pos, const int* comp_off) {
  const int p = blockIdx.y;
  const int c0 = comp_off[p], c1 = comp_off[p + 1];
  const double* g = g_tab[p];
  for (int c = c0 + blockIdx.x * blockDim.x + threadIdx.x; c < c1; c += gridDim.x * blockDim.x) b[c] = g[pos[c]];
}

// Per-mode gradient dL/dlnP on the half spectrum (transposed layout kx-major),
// with the multiplicity of each half-spectrum entry in the full grid.
__global__ void k_spec_grad(const double2* Xh, const double2* Xw, const double2* Xl, const double2* Xv,
                            const double* Dhalf, const double* Dinv, int nx, int ny, double* G,
                            double* G_api) {
  const size_t nt = (size_t)(nx / 2 + 1) * ny;
  const double Ntot = (double)nx * (double)ny;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt; i += (size_t)gridDim.x * blockDim.x) {
    const int kx = (int)(i / ny), ky = (int)(i % ny);
    const double wgt = (kx == 0 || kx == nx / 2) ? 1.0 : 2.0;
    const double sqrtP = Dhalf[i] * Ntot, invP = Dinv[i] * Ntot;
    const double2 h = Xh[i], w = Xw[i], l = Xl[i], v = Xv[i];
    const double val = wgt * (0.5 * sqrtP * (h.x * w.x + h.y * w.y) + (l.x * v.x + l.y * v.y) * invP) / Ntot;
    G[i] = val;
    if (G_api) G_api[(size_t)ky * (nx / 2 + 1) + kx] = val;
  }
}

// Hat weight of band b at ln|k| (nodes lnk[0..nb), increasing); k = 0 belongs to band 0.
__device__ __forceinline__ double band_weight(double lk, bool k0, const double* lnk, int nb, int b) {
  if (k0 || lk <= lnk[0]) return b == 0 ? 1.0 : 0.0;
  if (lk >= lnk[nb - 1]) return b == nb - 1 ? 1.0 : 0.0;
  if (b > 0 && lk >= lnk[b - 1] && lk < lnk[b]) return (lk - lnk[b - 1]) / (lnk[b] - lnk[b - 1]);
  if (b < nb - 1 && lk >= lnk[b] && lk < lnk[b + 1]) return 1.0 - (lk - lnk[b]) / (lnk[b + 1] - lnk[b]);
  return 0.0;
}

// out[b] += sum_k phi_b(k) G_k, one workgroup per band, fixed order.
__global__ __launch_bounds__(AT) void k_band_reduce(const double* G, int nx, int ny, const double* lnk, int nb,
                                                    double* out) {
  const int b = blockIdx.x;
  const size_t nt = (size_t)(nx / 2 + 1) * ny;
  double acc = 0.0, unused = 0.0;
  for (size_t i = threadIdx.x; i < nt; i += AT) {
    const int kx = (int)(i / ny), ky0 = (int)(i % ny);
    const int ky = ky0 <= ny / 2 ? ky0 : ky0 - ny;
    const double k2 = (double)kx * kx + (double)ky * ky;
    const double lk = k2 > 0.0 ? 0.5 * log(k2) : 0.0;
    const double wb = band_weight(lk, k2 == 0.0, lnk, nb, b);
    if (wb != 0.0) acc += wb * G[i];
  }
  block_sum2<AT>(acc, unused);
  if (threadIdx.x == 0) out[b] += acc;
}

// out[p] = sum of v[c]^2 over problem p's compact range, fixed order.
__global__ __launch_bounds__(AT) void k_cnorm2(double* out, const double* v, const int* comp_off) {
  const int p = blockIdx.x;
  double acc = 0.0, unused = 0.0;
  for (int c = comp_off[p] + threadIdx.x; c < comp_off[p + 1]; c += AT) acc += v[c] * v[c];
  block_sum2<AT>(acc, unused);
  if (threadIdx.x == 0) out[p] = acc;
}

hipError_t launch_cnorm2(double* out, const double* v, const int* comp_off, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(k_cnorm2, dim3(nprob), dim3(AT), 0, st, out, v, comp_off);
  return hipGetLastError();
}

template <int N>
hipError_t launch_col_fwd_n(const double2* Xt, double2* Xs, int ldx, int nhalf, const double2* tw, hipStream_t s) {
  using CF = ColCfg<double, N>;
  hipLaunchKernelGGL((col_fwd_kernel<N>), dim3((nhalf + CF::W - 1) / CF::W), dim3(CF::THREADS), 0, s, Xt, Xs, ldx,
                     nhalf, tw);
  return hipGetLastError();
}

hipError_t launch_col_fwd(int ny, const double2* Xt, double2* Xs, int ldx, int nhalf, const double2* tw,
                          hipStream_t s) {
  switch (ny) {
#define FILL_CASE(n) case n: return launch_col_fwd_n<n>(Xt, Xs, ldx, nhalf, tw, s);
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adj_maps(const uint8_t* mask, const double* g, const double* cl, const double* x, const double* s,
                           const double* d, double* grad_y, double* h, double* v, size_t npix, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_maps, grid_for(npix), dim3(AT), 0, st, mask, g, cl, x, s, d, grad_y, h, v, npix);
  return hipGetLastError();
}

hipError_t launch_adj_gather(double* b, double* const* g_tab, const int* pos, const int* comp_off, int nmax, int nprob,
                             hipStream_t st) {
  dim3 gr = grid_for(nmax);
  gr.y = nprob;
  hipLaunchKernelGGL(k_adj_gather, gr, dim3(AT), 0, st, b, g_tab, pos, comp_off);
  return hipGetLastError();
}

hipError_t launch_spec_grad(const double2* Xh, const double2* Xw, const double2* Xl, const double2* Xv,
                            const double* Dhalf, const double* Dinv, int nx, int ny, double* G, double* G_api,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_spec_grad, grid_for((size_t)(nx / 2 + 1) * ny), dim3(AT), 0, st, Xh, Xw, Xl, Xv, Dhalf, Dinv,
                     nx, ny, G, G_api);
  return hipGetLastError();
}

hipError_t launch_band_reduce(const double* G, int nx, int ny, const double* lnk, int nb, double* out,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_band_reduce, dim3(nb), dim3(AT), 0, st, G, nx, ny, lnk, nb, out);
  return hipGetLastError();
}

}  // namespace fillk
