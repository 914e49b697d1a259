// C ABI of the constrained-realization fill-in: plan, solve driver, entry
// points (declarations and contracts in include/fill.h).
//
// A solve (Sec. 2.3 / 2.4):
//   1. s = C^{1/2} w from counter-based white noise (one apply, noise generated
//      inside the first row pass); the same pass writes x_out = d on observed
//      pixels and s on masked ones, and t = Py (d - s);
//   2. v = -Px C^-1 t (one apply), ||v|| on the host;
//   3. refinement loop in FP64: r = v - A u (FP64 apply), then an inner
//      preconditioned CG on A d = r / ||r|| in the plan's precision (FP64, or
//      FP32 operators with FP64 dot products and scalars), u += ||r|| d;
//   4. x_out += u on masked pixels.
// Inner CG (Hestenes-Stiefel) with M^-1 = E E, E = Px C^{1/2} Px: the paper's
// split form E A E u' = E v, u = E u', has the same iterates u.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fill.h"
#include "kernels.hpp"
#include "launch.hpp"

using namespace fillk;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(FILL_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

#define FILL_TRY(expr)         \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ < 0) return rc_;   \
  } while (0)

constexpr uint64_t kRealizationStream = 0x52;
constexpr int kChunk = 16;  // CG iterations between host polls of the convergence flag

template <typename T> struct Vecs {
  T* x = nullptr;
  T* r = nullptr;
  T* z = nullptr;
  T* p = nullptr;
  T* q = nullptr;
  T* t = nullptr;
};

}  // namespace

struct fill_plan_s {
  int nx = 0, ny = 0, ncol = 0, prec = 0;
  size_t npix = 0;
  hipStream_t stream = nullptr;
  int n_m = 0;
  int max_iter = 20000;
  double inner_tol32 = 1e-4;
  int nblk64 = 0, nblk32 = 0;

  uint8_t* mask = nullptr;
  int* pos = nullptr;
  int* row_off = nullptr;
  double* Dinv64 = nullptr;
  double* Dhalf64 = nullptr;
  float* Dinv32 = nullptr;
  float* Dhalf32 = nullptr;
  double2* twx64 = nullptr;
  double2* twy64 = nullptr;
  float2* twx32 = nullptr;
  float2* twy32 = nullptr;
  void* Xt = nullptr;
  double* tfull = nullptr;
  double* b = nullptr;
  double* u = nullptr;
  double* res = nullptr;
  Vecs<double> v64;
  Vecs<float> v32;
  double* part0 = nullptr;
  double* part1 = nullptr;
  double* part2 = nullptr;
  double* dsum = nullptr;
  CGScalars* sc = nullptr;
  CGScalars* h_sc = nullptr;
  double* h_sum = nullptr;
  fill_stats stats{};
  std::vector<void*> allocs;
  // optional HIP-event timing of every launch of one kernel during solves
  int timed_kernel = -1;
  int timed_prec = 0;
  std::vector<hipEvent_t> events;  // start/stop pairs
  size_t events_used = 0;
  double timed_ms = 0.0;
  long long timed_count = 0;
};

namespace {

template <typename P> int dalloc(fill_plan p, P** out, size_t count) {
  void* ptr = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(P), 256);
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) return fail(FILL_ENOMEM, std::string("hipMalloc ") + std::to_string(bytes) + " bytes: " +
                                                    hipGetErrorString(e));
  p->allocs.push_back(ptr);
  *out = static_cast<P*>(ptr);
  return FILL_OK;
}

template <typename T> struct TypeSel;
template <> struct TypeSel<double> {
  static const cplx<double>* twx(fill_plan p) { return p->twx64; }
  static const cplx<double>* twy(fill_plan p) { return p->twy64; }
  static const double* Dinv(fill_plan p) { return p->Dinv64; }
  static const double* Dhalf(fill_plan p) { return p->Dhalf64; }
  static int nblk(fill_plan p) { return p->nblk64; }
  static Vecs<double>& vecs(fill_plan p) { return p->v64; }
};
template <> struct TypeSel<float> {
  static const cplx<float>* twx(fill_plan p) { return p->twx32; }
  static const cplx<float>* twy(fill_plan p) { return p->twy32; }
  static const float* Dinv(fill_plan p) { return p->Dinv32; }
  static const float* Dhalf(fill_plan p) { return p->Dhalf32; }
  static int nblk(fill_plan p) { return p->nblk32; }
  static Vecs<float>& vecs(fill_plan p) { return p->v32; }
};

template <typename T> RowArgs<T> row_base(fill_plan p) {
  RowArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.nx = p->nx;
  a.ny = p->ny;
  a.ldx = p->ny;
  a.row_off = p->row_off;
  a.pos = p->pos;
  a.Xt = static_cast<cplx<T>*>(p->Xt);
  a.tw = TypeSel<T>::twx(p);
  a.scale = T(1);
  a.mask = p->mask;
  return a;
}

// Sum the elapsed times of the recorded event pairs (stream synchronised) and recycle them.
int drain_timing(fill_plan p) {
  if (p->events_used == 0) return FILL_OK;
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (size_t i = 0; i + 1 < p->events_used; i += 2) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p->events[i], p->events[i + 1]));
    p->timed_ms += ms;
    p->timed_count += 1;
  }
  p->events_used = 0;
  return FILL_OK;
}

// Launch wrapper: when this kernel is the timed one, hand the launch a pair
// of events that the dispatch itself timestamps at its start and end.
template <typename T, typename F>
int timed_launch(fill_plan p, int kernel, F&& launch) {
  const bool on = p->timed_kernel == kernel && p->timed_prec == (sizeof(T) == 4 ? FILL_PREC_FP32_OP : FILL_PREC_FP64);
  if (!on) {
    HIP_TRY(launch(nullptr, nullptr));
    return FILL_OK;
  }
  if (p->events_used + 2 > p->events.size()) {
    FILL_TRY(drain_timing(p));
    while (p->events.size() < 2048) {
      // timing-only events: no system-scope fence (no cache write-back on record)
      hipEvent_t e;
      HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      p->events.push_back(e);
    }
  }
  HIP_TRY(launch(p->events[p->events_used], p->events[p->events_used + 1]));
  p->events_used += 2;
  return FILL_OK;
}

// One operator apply: r2c (mode rm, args ai) -> column pass with table D -> c2r (mode cm, args ao).
template <typename T>
int apply3(fill_plan p, int rm, const RowArgs<T>& ai, const T* D, int cm, const RowArgs<T>& ao,
           const CGScalars* sc) {
  FILL_TRY(timed_launch<T>(p, FILL_K_R2C, [&](hipEvent_t a, hipEvent_t b) { return launch_r2c<T>(rm, ai, p->stream, a, b); }));
  ColArgs<T> ca;
  ca.Xt = static_cast<cplx<T>*>(p->Xt);
  ca.ldx = p->ny;
  ca.ncol = p->nx / 2;  // the Nyquist column travels in column 0
  ca.D = D;
  ca.tw = TypeSel<T>::twy(p);
  ca.sc = sc;
  FILL_TRY(timed_launch<T>(p, FILL_K_COL, [&](hipEvent_t a, hipEvent_t b) { return launch_col<T>(p->ny, ca, p->stream, a, b); }));
  FILL_TRY(timed_launch<T>(p, FILL_K_C2R, [&](hipEvent_t a, hipEvent_t b) { return launch_c2r<T>(cm, ao, p->stream, a, b); }));
  return FILL_OK;
}

// Two applies of E in a row, E (E u): r2c (mode rm) -> column pass (sqrt P)
// -> projection row pass -> column pass (sqrt P) -> c2r (C2R_DOT2).
template <typename T>
int apply_EE(fill_plan p, int rm, const RowArgs<T>& ai, const RowArgs<T>& amid, const RowArgs<T>& ao,
             const CGScalars* sc) {
  FILL_TRY(timed_launch<T>(p, FILL_K_R2C, [&](hipEvent_t a, hipEvent_t b) { return launch_r2c<T>(rm, ai, p->stream, a, b); }));
  ColArgs<T> ca;
  ca.Xt = static_cast<cplx<T>*>(p->Xt);
  ca.ldx = p->ny;
  ca.ncol = p->nx / 2;
  ca.D = TypeSel<T>::Dhalf(p);
  ca.tw = TypeSel<T>::twy(p);
  ca.sc = sc;
  FILL_TRY(timed_launch<T>(p, FILL_K_COL, [&](hipEvent_t a, hipEvent_t b) { return launch_col<T>(p->ny, ca, p->stream, a, b); }));
  FILL_TRY(timed_launch<T>(p, FILL_K_PROJ, [&](hipEvent_t a, hipEvent_t b) { return launch_proj<T>(amid, p->stream, a, b); }));
  FILL_TRY(timed_launch<T>(p, FILL_K_COL, [&](hipEvent_t a, hipEvent_t b) { return launch_col<T>(p->ny, ca, p->stream, a, b); }));
  FILL_TRY(timed_launch<T>(p, FILL_K_C2R, [&](hipEvent_t a, hipEvent_t b) { return launch_c2r<T>(C2R_DOT2, ao, p->stream, a, b); }));
  return FILL_OK;
}

int read_sum(fill_plan p, const double* part, int n, double* out) {
  HIP_TRY(launch_sum(p->dsum, part, n, p->stream));
  HIP_TRY(hipMemcpyAsync(p->h_sum, p->dsum, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  *out = *p->h_sum;
  return FILL_OK;
}

// Inner preconditioned CG on A d = r (r already in v.r, ||r|| = 1), d in v.x.
template <typename T>
int inner_pcg(fill_plan p, double tol, int cap, int* iters, int* status) {
  Vecs<T>& v = TypeSel<T>::vecs(p);
  const int nb = TypeSel<T>::nblk(p);
  const T* Dinv = TypeSel<T>::Dinv(p);
  const T* Dhalf = TypeSel<T>::Dhalf(p);
  const size_t vb = (size_t)p->n_m * sizeof(T);
  HIP_TRY(hipMemsetAsync(v.x, 0, vb, p->stream));
  HIP_TRY(hipMemsetAsync(v.p, 0, vb, p->stream));

  // z = E (E r); its partial sums (r.z, r.r) feed the first iteration
  RowArgs<T> a_in = row_base<T>(p), a_mid = row_base<T>(p), a_out = row_base<T>(p);
  a_in.v0 = v.r;
  a_out.v0 = v.z;
  a_out.v1 = v.r;
  a_out.part0 = p->part0;
  a_out.part1 = p->part1;
  FILL_TRY(apply_EE<T>(p, R2C_COMPACT, a_in, a_mid, a_out, nullptr));
  HIP_TRY(launch_cg_init(p->sc, tol * tol, cap, p->stream));

  // Iteration k (parity k % 2), all scalars on the device:
  //   q = A p, with beta = (r.z)/rho and p = z + beta p fused in front
  //       (partials of r.z, r.r from the previous E E r pass), p.q behind;
  //   z = E E r, with alpha = rho/(p.q), x += alpha p, r -= alpha q fused in
  //       front, r.z and r.r behind.
  RowArgs<T> pa_in[2], pa_out = row_base<T>(p), e_in[2], e_mid = row_base<T>(p), e_out = row_base<T>(p);
  for (int par = 0; par < 2; ++par) {
    pa_in[par] = row_base<T>(p);
    pa_in[par].v0 = v.z;
    pa_in[par].v1 = v.p;
    pa_in[par].sc = p->sc;
    pa_in[par].red0 = p->part0;
    pa_in[par].red1 = p->part1;
    pa_in[par].nred = nb;
    pa_in[par].parity = par;
    e_in[par] = row_base<T>(p);
    e_in[par].v0 = v.x;
    e_in[par].v1 = v.r;
    e_in[par].v2 = v.p;
    e_in[par].v3 = v.q;
    e_in[par].sc = p->sc;
    e_in[par].red0 = p->part2;
    e_in[par].nred = nb;
    e_in[par].parity = par;
  }
  pa_out.v0 = v.q;
  pa_out.v1 = v.p;
  pa_out.part0 = p->part2;
  pa_out.sc = p->sc;
  e_mid.sc = p->sc;
  e_out.v0 = v.z;
  e_out.v1 = v.r;
  e_out.part0 = p->part0;
  e_out.part1 = p->part1;
  e_out.sc = p->sc;

  for (;;) {
    for (int k = 0; k < kChunk; ++k) {
      const int par = k & 1;
      FILL_TRY(apply3<T>(p, R2C_PUPDATE, pa_in[par], Dinv, C2R_COMPACT, pa_out, p->sc));
      FILL_TRY(apply_EE<T>(p, R2C_XRUPDATE, e_in[par], e_mid, e_out, p->sc));
    }
    HIP_TRY(hipMemcpyAsync(p->h_sc, p->sc, sizeof(CGScalars), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (p->h_sc->done) break;
  }
  *iters = p->h_sc->iter;
  *status = p->h_sc->status;
  return FILL_OK;
}

// Solve A u = b (b, u compact FP64) to true relative residual rtol.
int solve(fill_plan p, double bnorm2, double rtol) {
  const int n = p->n_m;
  HIP_TRY(hipMemsetAsync(p->u, 0, (size_t)n * sizeof(double), p->stream));
  p->stats.iters_inner = 0;
  p->stats.iters_outer = 0;
  p->stats.rel_resid = 0.0;
  if (bnorm2 == 0.0) return FILL_OK;
  HIP_TRY(hipMemcpyAsync(p->res, p->b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  double rnorm2 = bnorm2;
  int total = 0, outer = 0, status = FILL_OK;
  double prev_rel = 1.0;
  for (;;) {
    const double rel = std::sqrt(rnorm2 / bnorm2);
    p->stats.rel_resid = rel;
    if (!(rel == rel)) return fail(FILL_ENOTSPD, "residual is not finite");
    if (rel <= rtol) {
      status = FILL_OK;
      break;
    }
    if (total >= p->max_iter || outer >= 60 || (outer > 0 && rel > 0.5 * prev_rel && outer >= 3)) {
      status = fail(FILL_ENOCONV, "no convergence: true relative residual " + std::to_string(rel) +
                                      " after " + std::to_string(total) + " CG iterations");
      break;
    }
    prev_rel = rel;
    const double rn = std::sqrt(rnorm2);
    const double target = rtol / rel;  // inner relative reduction that reaches rtol
    int it = 0, st = 0;
    if (p->prec == FILL_PREC_FP64) {
      HIP_TRY(launch_scale_f64(p->v64.r, p->res, 1.0 / rn, n, p->stream));
      FILL_TRY(inner_pcg<double>(p, 0.5 * target, p->max_iter - total, &it, &st));
      HIP_TRY(launch_axpy_f64(p->u, p->v64.x, rn, n, p->stream));
    } else {
      HIP_TRY(launch_to_f32_scaled(p->v32.r, p->res, 1.0 / rn, n, p->stream));
      const double tol = std::max(0.5 * target, p->inner_tol32);
      FILL_TRY(inner_pcg<float>(p, tol, p->max_iter - total, &it, &st));
      HIP_TRY(launch_axpy_f64_f32(p->u, p->v32.x, rn, n, p->stream));
    }
    total += it;
    outer += 1;
    p->stats.iters_inner = total;
    p->stats.iters_outer = outer;
    if (st == -6) return fail(FILL_ENOTSPD, "CG breakdown: p.Ap <= 0 or r.Mr <= 0");
    // true FP64 residual res = b - A u
    RowArgs<double> ai = row_base<double>(p), ao = row_base<double>(p);
    ai.v0 = p->u;
    ao.v0 = p->res;
    ao.v1 = p->b;
    ao.part0 = p->part0;
    FILL_TRY(apply3<double>(p, R2C_COMPACT, ai, p->Dinv64, C2R_RESID, ao, nullptr));
    FILL_TRY(read_sum(p, p->part0, p->nblk64, &rnorm2));
  }
  p->stats.rel_resid = std::sqrt(rnorm2 / bnorm2);
  return status;
}

bool size_ok(int n) {
  switch (n) {
    case 16: case 32: case 64: case 128: case 256: case 512: case 768: case 1024: case 2048: case 4096:
      return true;
  }
  return false;
}

// Twiddle table of the length-N transform in the per-pass LO/HI layout the
// kernels read (see fft_device.hpp), each entry exp(-2 pi i t/N) evaluated in
// long double and rounded to double (and to float for the FP32 kernels).
template <int N> void make_twiddles(std::vector<double2>& w64, std::vector<float2>& w32) {
  const int total = std::max(tw_elems<N>(), 1);
  w64.assign(total, double2{1.0, 0.0});
  w32.assign(total, float2{1.0f, 0.0f});
  const long double pi = 3.141592653589793238462643383279502884L;
  auto put = [&](int idx, long long t) {
    t %= N;
    const long double a = 2.0L * pi * (long double)t / (long double)N;
    const double c = (double)cosl(a), sn = (double)-sinl(a);
    w64[idx] = double2{c, sn};
    w32[idx] = float2{(float)c, (float)sn};
  };
  for (int p = 0; p < FFTPlan<N>::NP; ++p) {
    const int ns = pass_ns<N>(p);
    if (ns == 1) continue;
    const int R = FFTPlan<N>::radix(p), S = N / (ns * R), off = tw_pass_off<N>(p);
    for (int i = 0; i < R; ++i)
      for (int klo = 0; klo < 16; ++klo) put(off + 16 * i + klo, (long long)i * klo * S);
    if (ns > 16)
      for (int i = 0; i < R; ++i)
        for (int khi = 0; khi < ns / 16; ++khi) put(off + 16 * R + i * (ns / 16) + khi, 16LL * i * khi * S);
  }
}

int twiddles(int n, std::vector<double2>& w64, std::vector<float2>& w32) {
  switch (n) {
#define FILL_CASE(nn) \
  case nn:            \
    make_twiddles<nn>(w64, w32); \
    return FILL_OK;
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return fail(FILL_EUNSUPPORTED_SIZE, "no FFT plan for length " + std::to_string(n));
}

int upload_pk(fill_plan p, const double* Pk) {
  const int nx = p->nx, ny = p->ny, nc = p->ncol;
  const size_t nt = (size_t)nc * ny;
  std::vector<double> inv(nt), half(nt);
  std::vector<float> inv32(nt), half32(nt);
  const double scale = 1.0 / ((double)nx * (double)ny);
  for (int iy = 0; iy < ny; ++iy) {
    for (int ix = 0; ix < nc; ++ix) {
      const double P = Pk[(size_t)iy * nc + ix];
      if (!(P > 0.0) || !std::isfinite(P))
        return fail(FILL_ENOTSPD, "Pk[" + std::to_string(iy) + "," + std::to_string(ix) + "] = " +
                                      std::to_string(P) + " is not positive and finite");
      const size_t o = (size_t)ix * ny + iy;  // transposed: spectral column kx contiguous in ky
      inv[o] = scale / P;
      half[o] = scale * std::sqrt(P);
      inv32[o] = (float)inv[o];
      half32[o] = (float)half[o];
    }
  }
  HIP_TRY(hipMemcpy(p->Dinv64, inv.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->Dhalf64, half.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->Dinv32, inv32.data(), nt * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->Dhalf32, half32.data(), nt * sizeof(float), hipMemcpyHostToDevice));
  return FILL_OK;
}

int plan_build(fill_plan p, const uint8_t* mask, const double* Pk) {
  const int nx = p->nx, ny = p->ny;
  const size_t npix = p->npix, nt = (size_t)p->ncol * ny;
  // mask -> compact index (row-major) and per-row offsets
  std::vector<int> pos;
  std::vector<int> row_off(ny + 1, 0);
  std::vector<uint8_t> m01(npix);
  for (int y = 0; y < ny; ++y) {
    row_off[y] = (int)pos.size();
    for (int x = 0; x < nx; ++x) {
      const size_t i = (size_t)y * nx + x;
      m01[i] = mask[i] ? 1 : 0;
      if (m01[i]) pos.push_back((int)i);
    }
  }
  row_off[ny] = (int)pos.size();
  p->n_m = (int)pos.size();
  p->stats.n_masked = p->n_m;
  const int nm = std::max(p->n_m, 1);
  FILL_TRY(dalloc(p, &p->mask, npix));
  FILL_TRY(dalloc(p, &p->pos, nm));
  FILL_TRY(dalloc(p, &p->row_off, ny + 1));
  FILL_TRY(dalloc(p, &p->Dinv64, nt));
  FILL_TRY(dalloc(p, &p->Dhalf64, nt));
  FILL_TRY(dalloc(p, &p->Dinv32, nt));
  FILL_TRY(dalloc(p, &p->Dhalf32, nt));
  std::vector<double2> twx64, twy64;
  std::vector<float2> twx32, twy32;
  FILL_TRY(twiddles(nx, twx64, twx32));
  FILL_TRY(twiddles(ny, twy64, twy32));
  FILL_TRY(dalloc(p, &p->twx64, twx64.size()));
  FILL_TRY(dalloc(p, &p->twy64, twy64.size()));
  FILL_TRY(dalloc(p, &p->twx32, twx32.size()));
  FILL_TRY(dalloc(p, &p->twy32, twy32.size()));
  double2* xt = nullptr;
  FILL_TRY(dalloc(p, &xt, nt));
  p->Xt = xt;
  FILL_TRY(dalloc(p, &p->tfull, npix));
  FILL_TRY(dalloc(p, &p->b, nm));
  FILL_TRY(dalloc(p, &p->u, nm));
  FILL_TRY(dalloc(p, &p->res, nm));
  for (double** q : {&p->v64.x, &p->v64.r, &p->v64.z, &p->v64.p, &p->v64.q, &p->v64.t}) FILL_TRY(dalloc(p, q, nm));
  for (float** q : {&p->v32.x, &p->v32.r, &p->v32.z, &p->v32.p, &p->v32.q, &p->v32.t}) FILL_TRY(dalloc(p, q, nm));
  FILL_TRY(dalloc(p, &p->part0, ny));
  FILL_TRY(dalloc(p, &p->part1, ny));
  FILL_TRY(dalloc(p, &p->part2, ny));
  FILL_TRY(dalloc(p, &p->dsum, 4));
  FILL_TRY(dalloc(p, &p->sc, 1));
  HIP_TRY(hipHostMalloc((void**)&p->h_sc, sizeof(CGScalars), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void**)&p->h_sum, 4 * sizeof(double), hipHostMallocDefault));

  HIP_TRY(hipMemcpy(p->mask, m01.data(), npix, hipMemcpyHostToDevice));
  if (!pos.empty()) HIP_TRY(hipMemcpy(p->pos, pos.data(), pos.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->row_off, row_off.data(), (ny + 1) * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->twx64, twx64.data(), twx64.size() * sizeof(double2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->twx32, twx32.data(), twx32.size() * sizeof(float2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->twy64, twy64.data(), twy64.size() * sizeof(double2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->twy32, twy32.data(), twy32.size() * sizeof(float2), hipMemcpyHostToDevice));
  return upload_pk(p, Pk);
}

// Steps 2-4 of a solve, after x_out and t = Py(d - s) (or Py d) are in place.
int rhs_solve_assemble(fill_plan p, double* x_out, double rtol) {
  RowArgs<double> ai = row_base<double>(p), ao = row_base<double>(p);
  ai.full_in = p->tfull;
  ao.v0 = p->b;
  ao.scale = -1.0;
  ao.part0 = p->part0;
  FILL_TRY(apply3<double>(p, R2C_FULL, ai, p->Dinv64, C2R_COMPACT, ao, nullptr));
  double bnorm2 = 0.0;
  FILL_TRY(read_sum(p, p->part0, p->nblk64, &bnorm2));
  const int st = solve(p, bnorm2, rtol);
  if (st != FILL_OK && st != FILL_ENOCONV) return st;
  HIP_TRY(launch_scatter_add(x_out, p->u, p->pos, p->n_m, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return st;
}

using clk = std::chrono::steady_clock;

}  // namespace

namespace {
template <typename T>
int time_kernel(fill_plan p, int kernel, int reps, double* avg_ms) {
  Vecs<T>& v = TypeSel<T>::vecs(p);
  const size_t vb = (size_t)std::max(p->n_m, 1) * sizeof(T);
  HIP_TRY(hipMemsetAsync(v.p, 0, vb, p->stream));
  RowArgs<T> ai = row_base<T>(p), ao = row_base<T>(p);
  ai.v0 = v.p;
  ao.v0 = v.q;
  ao.v1 = v.p;
  ao.part0 = p->part0;
  ColArgs<T> ca;
  ca.Xt = static_cast<cplx<T>*>(p->Xt);
  ca.ldx = p->ny;
  ca.ncol = p->nx / 2;
  ca.D = TypeSel<T>::Dinv(p);
  ca.tw = TypeSel<T>::twy(p);
  ca.sc = nullptr;
  auto launch = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    if (kernel == FILL_K_R2C || kernel == FILL_K_APPLY) e = launch_r2c<T>(R2C_COMPACT, ai, p->stream);
    if (e == hipSuccess && (kernel == FILL_K_COL || kernel == FILL_K_APPLY)) e = launch_col<T>(p->ny, ca, p->stream);
    if (e == hipSuccess && (kernel == FILL_K_C2R || kernel == FILL_K_APPLY))
      e = launch_c2r<T>(C2R_COMPACT, ao, p->stream);
    return e;
  };
  HIP_TRY(launch());  // warm-up
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, p->stream));
  for (int i = 0; i < reps; ++i) HIP_TRY(launch());
  HIP_TRY(hipEventRecord(e1, p->stream));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = (double)ms / reps;
  return FILL_OK;
}
}  // namespace

extern "C" {

int fill_supported_size(int n) { return size_ok(n) ? 1 : 0; }

int fill_plan_create(int nx, int ny, const uint8_t* mask, const double* Pk, int prec, void* stream,
                     fill_plan* out) {
  g_last_error.clear();
  if (!out) return fail(FILL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mask || !Pk) return fail(FILL_EINVAL, "mask or Pk is NULL");
  if (prec != FILL_PREC_FP64 && prec != FILL_PREC_FP32_OP) return fail(FILL_EINVAL, "unknown precision");
  if (!size_ok(nx) || !size_ok(ny))
    return fail(FILL_EUNSUPPORTED_SIZE, "grid " + std::to_string(nx) + "x" + std::to_string(ny) +
                                            " is not a supported FFT size");
  fill_plan p = new (std::nothrow) fill_plan_s();
  if (!p) return fail(FILL_ENOMEM, "host allocation");
  p->nx = nx;
  p->ny = ny;
  p->ncol = nx / 2 + 1;
  p->prec = prec;
  p->npix = (size_t)nx * ny;
  p->stream = static_cast<hipStream_t>(stream);
  const int r64 = row_block_rows<double>(nx), r32 = row_block_rows<float>(nx);
  if (r64 <= 0 || r32 <= 0 || ny % r64 || ny % r32) {
    delete p;
    return fail(FILL_EUNSUPPORTED_SIZE, "ny not a multiple of the row block");
  }
  p->nblk64 = ny / r64;
  p->nblk32 = ny / r32;
  const int rc = plan_build(p, mask, Pk);
  if (rc != FILL_OK) {
    fill_plan_destroy(p);
    return rc;
  }
  *out = p;
  return FILL_OK;
}

int fill_plan_set_pk(fill_plan p, const double* Pk) {
  g_last_error.clear();
  if (!p || !Pk) return fail(FILL_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(p->stream));
  return upload_pk(p, Pk);
}

int fill_plan_set_max_iter(fill_plan p, int max_iter) {
  if (!p || max_iter < 1) return fail(FILL_EINVAL, "bad argument");
  p->max_iter = max_iter;
  return FILL_OK;
}

int fill_plan_set_inner_tol(fill_plan p, double tol) {
  if (!p || !(tol > 0.0) || !(tol < 1.0)) return fail(FILL_EINVAL, "inner tolerance must be in (0, 1)");
  p->inner_tol32 = tol;
  return FILL_OK;
}

void fill_plan_destroy(fill_plan p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  for (void* a : p->allocs) (void)hipFree(a);
  if (p->h_sc) (void)hipHostFree(p->h_sc);
  if (p->h_sum) (void)hipHostFree(p->h_sum);
  delete p;
}

int fill_realize(fill_plan p, const double* d_obs, uint64_t seed, double* x_out, double rtol) {
  g_last_error.clear();
  if (!p || !d_obs || !x_out) return fail(FILL_EINVAL, "NULL argument");
  if (!(rtol > 0.0)) return fail(FILL_EINVAL, "rtol must be > 0");
  if ((const void*)d_obs == (const void*)x_out) return fail(FILL_EINVAL, "x_out aliases d_obs");
  const auto t0 = clk::now();
  p->stats = fill_stats{0, 0, p->n_m, 0, 0.0, 0.0};
  if (p->n_m == 0) {
    HIP_TRY(hipMemcpyAsync(x_out, d_obs, p->npix * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return FILL_OK;
  }
  // s = C^{1/2} w; x_out = mask ? s : d; t = mask ? 0 : d - s
  RowArgs<double> ai = row_base<double>(p), ao = row_base<double>(p);
  ai.seed = seed;
  ai.stream = kRealizationStream;
  ao.full_in = d_obs;
  ao.full_out = x_out;
  ao.full_out2 = p->tfull;
  FILL_TRY(apply3<double>(p, R2C_NOISE, ai, p->Dhalf64, C2R_REALIZE, ao, nullptr));
  const int st = rhs_solve_assemble(p, x_out, rtol);
  p->stats.status = st;
  p->stats.solve_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  return st;
}

int fill_mean(fill_plan p, const double* d_obs, double* x_out, double rtol) {
  g_last_error.clear();
  if (!p || !d_obs || !x_out) return fail(FILL_EINVAL, "NULL argument");
  if (!(rtol > 0.0)) return fail(FILL_EINVAL, "rtol must be > 0");
  if ((const void*)d_obs == (const void*)x_out) return fail(FILL_EINVAL, "x_out aliases d_obs");
  const auto t0 = clk::now();
  p->stats = fill_stats{0, 0, p->n_m, 0, 0.0, 0.0};
  if (p->n_m == 0) {
    HIP_TRY(hipMemcpyAsync(x_out, d_obs, p->npix * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return FILL_OK;
  }
  HIP_TRY(launch_mean_prep(x_out, p->tfull, d_obs, p->mask, p->npix, p->stream));
  const int st = rhs_solve_assemble(p, x_out, rtol);
  p->stats.status = st;
  p->stats.solve_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  return st;
}

int fill_get_stats(fill_plan p, fill_stats* out) {
  if (!p || !out) return fail(FILL_EINVAL, "NULL argument");
  *out = p->stats;
  return FILL_OK;
}

int fill_apply(fill_plan p, int op, int prec, const double* in, double* out) {
  g_last_error.clear();
  if (!p || !in || !out) return fail(FILL_EINVAL, "NULL argument");
  if (in == out) return fail(FILL_EINVAL, "out aliases in");
  if (op < FILL_OP_CINV || op > FILL_OP_E) return fail(FILL_EINVAL, "unknown operator");
  if (prec != FILL_PREC_FP64 && prec != FILL_PREC_FP32_OP) return fail(FILL_EINVAL, "unknown precision");
  const bool inv = (op == FILL_OP_CINV || op == FILL_OP_A);
  const int n = p->n_m;
  if (op == FILL_OP_CINV || op == FILL_OP_CHALF) {
    if (prec == FILL_PREC_FP64) {
      RowArgs<double> ai = row_base<double>(p), ao = row_base<double>(p);
      ai.full_in = in;
      ao.full_out = out;
      FILL_TRY(apply3<double>(p, R2C_FULL, ai, inv ? p->Dinv64 : p->Dhalf64, C2R_FULL, ao, nullptr));
    } else {
      RowArgs<float> ai = row_base<float>(p), ao = row_base<float>(p);
      ai.full_in = in;
      ao.full_out = out;
      FILL_TRY(apply3<float>(p, R2C_FULL, ai, inv ? p->Dinv32 : p->Dhalf32, C2R_FULL, ao, nullptr));
    }
  } else {
    HIP_TRY(hipMemsetAsync(out, 0, p->npix * sizeof(double), p->stream));
    if (n > 0) {
      HIP_TRY(launch_gather(p->res, in, p->pos, n, p->stream));
      if (prec == FILL_PREC_FP64) {
        RowArgs<double> ai = row_base<double>(p), ao = row_base<double>(p);
        ai.v0 = p->res;
        ao.v0 = p->v64.q;
        FILL_TRY(apply3<double>(p, R2C_COMPACT, ai, inv ? p->Dinv64 : p->Dhalf64, C2R_COMPACT, ao, nullptr));
        HIP_TRY(launch_scatter(out, p->v64.q, p->pos, n, p->stream));
      } else {
        HIP_TRY(launch_to_f32_scaled(p->v32.t, p->res, 1.0, n, p->stream));
        RowArgs<float> ai = row_base<float>(p), ao = row_base<float>(p);
        ai.v0 = p->v32.t;
        ao.v0 = p->v32.q;
        FILL_TRY(apply3<float>(p, R2C_COMPACT, ai, inv ? p->Dinv32 : p->Dhalf32, C2R_COMPACT, ao, nullptr));
        HIP_TRY(launch_scatter_f32(out, p->v32.q, p->pos, n, p->stream));
      }
    }
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  return FILL_OK;
}

int fill_realize_unconstrained(fill_plan p, uint64_t seed, double* out) {
  g_last_error.clear();
  if (!p || !out) return fail(FILL_EINVAL, "NULL argument");
  RowArgs<double> ai = row_base<double>(p), ao = row_base<double>(p);
  ai.seed = seed;
  ai.stream = kRealizationStream;
  ao.full_out = out;
  FILL_TRY(apply3<double>(p, R2C_NOISE, ai, p->Dhalf64, C2R_REALIZE, ao, nullptr));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return FILL_OK;
}

int fill_philox_words(uint64_t seed, uint64_t stream, int64_t n_blocks, uint64_t* out) {
  g_last_error.clear();
  if (!out || n_blocks < 0) return fail(FILL_EINVAL, "bad argument");
  HIP_TRY(launch_philox_words(out, seed, stream, n_blocks, nullptr));
  HIP_TRY(hipStreamSynchronize(nullptr));
  return FILL_OK;
}

int fill_time_kernel(fill_plan p, int kernel, int prec, int reps, double* avg_ms) {
  g_last_error.clear();
  if (!p || !avg_ms || reps < 1) return fail(FILL_EINVAL, "bad argument");
  if (kernel < FILL_K_R2C || kernel > FILL_K_APPLY) return fail(FILL_EINVAL, "unknown kernel");
  if (prec == FILL_PREC_FP64) return time_kernel<double>(p, kernel, reps, avg_ms);
  if (prec == FILL_PREC_FP32_OP) return time_kernel<float>(p, kernel, reps, avg_ms);
  return fail(FILL_EINVAL, "unknown precision");
}

int fill_kernel_timing(fill_plan p, int kernel, int prec) {
  g_last_error.clear();
  if (!p) return fail(FILL_EINVAL, "NULL plan");
  if (kernel < -1 || kernel > FILL_K_PROJ || kernel == FILL_K_APPLY) return fail(FILL_EINVAL, "unknown kernel");
  if (prec != FILL_PREC_FP64 && prec != FILL_PREC_FP32_OP) return fail(FILL_EINVAL, "unknown precision");
  FILL_TRY(drain_timing(p));
  p->timed_kernel = kernel;
  p->timed_prec = prec;
  p->timed_ms = 0.0;
  p->timed_count = 0;
  return FILL_OK;
}

int fill_kernel_timing_read(fill_plan p, double* total_ms, int64_t* count) {
  g_last_error.clear();
  if (!p || !total_ms || !count) return fail(FILL_EINVAL, "NULL argument");
  FILL_TRY(drain_timing(p));
  *total_ms = p->timed_ms;
  *count = p->timed_count;
  p->timed_ms = 0.0;
  p->timed_count = 0;
  return FILL_OK;
}

const char* fill_strerror(int code) {
  switch (code) {
    case FILL_OK: return "ok";
    case FILL_EINVAL: return "invalid argument";
    case FILL_ENOMEM: return "out of memory";
    case FILL_EHIP: return "HIP runtime error";
    case FILL_ENOCONV: return "conjugate gradient did not converge";
    case FILL_EUNSUPPORTED_SIZE: return "unsupported grid size";
    case FILL_ENOTSPD: return "spectrum or operator not positive definite";
  }
  return "unknown error";
}

const char* fill_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
