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

// Sum of p[0..n) by a workgroup of RT threads in a fixed order (thread t adds
// i = t, t+RT, ...; then a fixed tree), hence deterministic; the result is
// valid in thread 0.
__device__ __forceinline__ double fixed_sum(const double* p, int n) {
  double v = 0.0, w = 0.0;
  for (int i = threadIdx.x; i < n; i += RT) v += p[i];
  block_sum2<RT>(v, w);
  return v;
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

__global__ void k_scatter_add(double* const* full, const double* c, const int* pos, const int* comp_off,
                              const SolveState* gate, int nprob) {
  if (gate)
    for (int i = 0; i < nprob; ++i)
      if (!gate[i].done) return;
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

// ---------------------------------------------------------------------------
// Refinement control: the decisions of the FP64 refinement loop around the
// inner CG solves, taken on the device (one workgroup, one thread per problem)
// so that a solve needs no host round trip between its steps.
// ---------------------------------------------------------------------------
// The next step of problem b from its state (thread 0 of its workgroup):
// stop (converged, failed, out of budget, stalled) or the parameters of the
// next inner solve, whose CG scalars are reset here as well.
__device__ void ctl_decide_one(const RefineArgs& a, int b) {
  SolveState& s = a.st[b];
  const SolveCfg& c = *a.cfg;
  int act = 0;
  double scale = 0.0, unscale = 0.0, tol2 = 0.0;
  int cap = 1;
  if (!s.done) {
    const double rel = s.bnorm2 == 0.0 ? 0.0 : sqrt(s.rnorm2 / s.bnorm2);
    s.rel = rel;
    if (s.bnorm2 == 0.0) {  // v = 0: u = 0 is exact
      s.done = 1;
    } else if (!(rel == rel)) {
      s.done = 1;
      s.status = -6;
    } else if (rel <= c.rtol) {
      s.done = 1;
    } else if (s.total >= c.max_iter || s.outer >= c.max_outer || (s.outer >= 3 && !s.cut && rel > 0.5 * s.prev)) {
      // out of iterations or steps, or stalled: three steps in and the last
      // one (an inner solve that reached its tolerance) did not halve the residual
      s.done = 1;
      s.status = -4;
    } else {
      s.prev = rel;
      const double rn = sqrt(s.rnorm2);
      const double target = c.rtol / rel;  // inner relative reduction that reaches rtol
      const double tol = c.fp64 ? 0.5 * target : fmax(0.5 * target, c.inner_tol);
      act = 1;
      scale = 1.0 / rn;
      unscale = rn;
      tol2 = tol * tol;
      cap = c.max_iter - s.total;
    }
  }
  a.active[b] = act;
  a.scale[b] = scale;
  a.unscale[b] = unscale;
  a.tol2[b] = tol2;
  a.cap[b] = cap;
  // CG scalars of the next inner solve: rho[0] = 1 so that the first
  // iteration's p = z + beta p (p = 0) is p = z for any finite beta; a
  // problem without a step is done at once
  CGScalars& g = a.sc[b];
  g.rho[0] = 1.0;
  g.rho[1] = 1.0;
  g.alpha = 0.0;
  g.beta = 0.0;
  g.alph[0] = __builtin_huge_val();  // single-reduction CG: the first alpha is rho / mu
  g.alph[1] = __builtin_huge_val();
  g.rr = 0.0;
  g.tol2 = tol2;
  g.done = act ? 0 : 1;
  g.iter = 0;
  g.max_iter = cap;
  g.status = 0;
  g.cap = 0;
}

__global__ __launch_bounds__(RT) void k_ctl(RefineArgs a, const double* part, size_t stride, int n, int begin) {
  const int b = blockIdx.x;
  const double sum = fixed_sum(part + (size_t)b * stride, n);
  if (threadIdx.x != 0) return;
  SolveState& s = a.st[b];
  if (begin) {
    s.bnorm2 = sum;
    s.rnorm2 = sum;
    s.prev = 1.0;
    s.rel = 1.0;
    s.total = 0;
    s.outer = 0;
    s.done = 0;
    s.status = 0;
    s.first_iters = 0;
    s.cut = 0;
    for (int j = 0; j < kStateIts; ++j) s.its[j] = 0;
  } else {
    s.rnorm2 = sum;
  }
  ctl_decide_one(a, b);
}

// r.r of the last CG iteration of problem b meets its tolerance (the
// iteration after it would stop there).
__device__ __forceinline__ bool rr_met(const CGScalars& c, const double* rr_part, int nb, size_t stride, int b) {
  const double rr = fixed_sum(rr_part + (size_t)b * stride, nb);
  return rr <= c.tol2;  // valid in thread 0
}

// The accounting of problem b's inner solve (a workgroup of RT threads).
__device__ __forceinline__ void ctl_after_one(const RefineArgs& a, const double* rr_part, int nb, size_t stride,
                                              int first, int b) {
  if (!a.active[b]) return;  // no inner solve ran for this problem
  const CGScalars& c = a.sc[b];
  const bool check = !c.done && rr_part;
  const bool met = check ? rr_met(c, rr_part, nb, stride, b) : false;
  if (threadIdx.x != 0) return;
  SolveState& s = a.st[b];
  const int it = c.iter;
  int stat = c.status;
  bool conv = c.done != 0;
  if (met) {
    conv = true;
    stat = 0;
  }
  s.cut = conv ? 0 : 1;
  if (first) s.first_iters = it;
  if (s.outer < kStateIts) s.its[s.outer] = it;
  s.total += it;
  s.outer += 1;
  if (stat == -6) {
    s.done = 1;
    s.status = -6;
  }
}

// u += unscale x (the inner solution into the FP64 solution) with the inner
// solve's accounting in the same launch: the last workgroup of each grid row
// takes problem blockIdx.y's accounting, the others the update (the two
// touch different data: u and the refinement state).
template <typename TX>
__global__ __launch_bounds__(RT) void k_axpy_after(double* y, const TX* x, const int* comp_off, RefineArgs a,
                                                   const double* rr_part, int nb, size_t stride, int first) {
  const int b = blockIdx.y;
  const int nw = gridDim.x - 1;
  if ((int)blockIdx.x == nw) {
    ctl_after_one(a, rr_part, nb, stride, first, b);
    return;
  }
  const int c0 = comp_off[b], c1 = comp_off[b + 1];
  const double s = a.unscale[b];
  if (s == 0.0) return;
  for (int c = c0 + blockIdx.x * RT + threadIdx.x; c < c1; c += nw * RT) y[c] += s * (double)x[c];
}

__global__ __launch_bounds__(RT) void k_rr_check(CGScalars* sc, const double* rr_part, int nb, size_t stride) {
  const int b = blockIdx.x;
  CGScalars& c = sc[b];
  if (c.done) return;
  const bool met = rr_met(c, rr_part, nb, stride, b);
  if (threadIdx.x == 0 && met) c.done = 1;
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
hipError_t launch_scatter_add(double* const* full, const double* c, const int* pos, const int* comp_off, int nmax,
                              int nprob, hipStream_t s, const SolveState* gate) {
  hipLaunchKernelGGL(k_scatter_add, grid_for(nmax, nprob), dim3(256), 0, s, full, c, pos, comp_off, gate, nprob);
  return hipGetLastError();
}
hipError_t launch_ctl(const RefineArgs& a, const double* part, size_t stride, int n, bool begin, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl, dim3(a.nprob), dim3(RT), 0, s, a, part, stride, n, begin ? 1 : 0);
  return hipGetLastError();
}
template <typename TX>
hipError_t launch_axpy_after_t(double* u, const TX* x, const int* comp_off, const RefineArgs& a,
                               const double* rr_part, int nb, size_t stride, bool first, int nmax, hipStream_t s) {
  const dim3 g = grid_for(nmax, a.nprob);
  hipLaunchKernelGGL((k_axpy_after<TX>), dim3(g.x + 1, g.y), dim3(RT), 0, s, u, x, comp_off, a, rr_part, nb, stride,
                     first ? 1 : 0);
  return hipGetLastError();
}
hipError_t launch_axpy_after_f32(double* u, const float* x, const int* comp_off, const RefineArgs& a,
                                 const double* rr_part, int nb, size_t stride, bool first, int nmax, hipStream_t s) {
  return launch_axpy_after_t<float>(u, x, comp_off, a, rr_part, nb, stride, first, nmax, s);
}
hipError_t launch_axpy_after_f64(double* u, const double* x, const int* comp_off, const RefineArgs& a,
                                 const double* rr_part, int nb, size_t stride, bool first, int nmax, hipStream_t s) {
  return launch_axpy_after_t<double>(u, x, comp_off, a, rr_part, nb, stride, first, nmax, s);
}
hipError_t launch_rr_check(CGScalars* sc, const double* rr_part, int nb, size_t stride, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_rr_check, dim3(nprob), dim3(RT), 0, s, sc, rr_part, nb, stride);
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
