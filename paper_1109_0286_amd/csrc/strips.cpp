// Noise-boosted strip refinement on the torus (Sec. 6.2 subdivision, Sec. 6.4
// refinement), built on the public plan API: one plan per strip, with the
// strip as its mask and P_signal + beta N as its spectrum, solved for a fixed
// number of CG iterations.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/fill.h"
#include "launch.hpp"

struct fill_strips_s {
  int nx = 0, ny = 0, nstrips = 0;
  hipStream_t stream = nullptr;
  std::vector<fill_plan> plans;               // null for an empty strip
  std::vector<std::vector<uint8_t>> masks;    // host copies of the strips
  uint8_t* dmask = nullptr;                   // the full mask (device)
  double* tmp = nullptr;                      // one map (device)
};

namespace {

thread_local std::string g_strip_error;

int sfail(int code, const std::string& msg) {
  g_strip_error = msg;
  return code;
}

#define S_HIP(expr)                                                                           \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return sfail(FILL_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Half-widths of the disk of radius w per row offset dy in [-r, r], r = floor(w):
// the largest h with h^2 + dy^2 <= w^2.
std::vector<int> disk_half_widths(double w, int r, long long* area) {
  std::vector<int> hw(2 * r + 1);
  *area = 0;
  for (int dy = -r; dy <= r; ++dy) {
    int h = (int)std::floor(std::sqrt(std::max(0.0, w * w - (double)dy * dy)));
    while ((double)(h + 1) * (h + 1) + (double)dy * dy <= w * w) ++h;
    while (h > 0 && (double)h * h + (double)dy * dy > w * w) --h;
    hw[dy + r] = h;
    *area += 2 * h + 1;
  }
  return hw;
}

void destroy(fill_strips s) {
  if (!s) return;
  for (fill_plan p : s->plans)
    if (p) fill_plan_destroy(p);
  if (s->dmask) (void)hipFree(s->dmask);
  if (s->tmp) (void)hipFree(s->tmp);
  delete s;
}

int build(fill_strips s, const uint8_t* mask, const double* Ps, double noise, const double* betas,
          const double* widths, double threshold, int iters, int prec) {
  const int nx = s->nx, ny = s->ny;
  const size_t npix = (size_t)nx * ny, nt = (size_t)ny * (nx / 2 + 1);
  S_HIP(hipMalloc(&s->dmask, npix));
  S_HIP(hipMalloc(&s->tmp, npix * sizeof(double)));
  S_HIP(hipMemcpy(s->dmask, mask, npix, hipMemcpyHostToDevice));
  int* pre = nullptr;
  int* dhw = nullptr;
  uint8_t* flags = nullptr;
  int rc = FILL_OK;
  std::vector<double> P(nt);
  auto cleanup = [&]() {
    if (pre) (void)hipFree(pre);
    if (dhw) (void)hipFree(dhw);
    if (flags) (void)hipFree(flags);
  };
  if (hipMalloc(&pre, (size_t)ny * (nx + 1) * sizeof(int)) != hipSuccess || hipMalloc(&flags, npix) != hipSuccess ||
      hipMalloc(&dhw, (size_t)std::min(nx, ny) * sizeof(int)) != hipSuccess) {
    cleanup();
    return sfail(FILL_ENOMEM, "device workspace of the subdivision");
  }
  for (int i = 0; i < s->nstrips && rc == FILL_OK; ++i) {
    const int r = (int)std::floor(widths[i]);
    long long area = 0;
    const std::vector<int> hw = disk_half_widths(widths[i], r, &area);
    hipError_t e = hipMemcpy(dhw, hw.data(), hw.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = fillk::launch_strip_flags(s->dmask, pre, dhw, r, nx, ny, threshold * (double)area, flags, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    s->masks[i].resize(npix);
    if (e == hipSuccess) e = hipMemcpy(s->masks[i].data(), flags, npix, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      rc = sfail(FILL_EHIP, std::string("strip subdivision: ") + hipGetErrorString(e));
      break;
    }
    bool any = false;
    for (size_t k = 0; k < npix && !any; ++k) any = s->masks[i][k] != 0;
    if (!any) continue;
    for (size_t k = 0; k < nt; ++k) P[k] = Ps[k] + betas[i] * noise;
    rc = fill_plan_create(nx, ny, s->masks[i].data(), P.data(), prec, s->stream, &s->plans[i]);
    if (rc == FILL_OK) rc = fill_plan_set_max_iter(s->plans[i], iters);
    if (rc != FILL_OK) g_strip_error = std::string("strip ") + std::to_string(i) + ": " + fill_last_error();
  }
  cleanup();
  return rc;
}

}  // namespace

extern "C" {

int fill_strips_create(int nx, int ny, const uint8_t* mask, const double* P_signal, double noise, int nstrips,
                       const double* betas, const double* widths, double threshold, int iters, int prec,
                       void* stream, fill_strips* out) {
  g_strip_error.clear();
  if (!out) return sfail(FILL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mask || !P_signal || !betas || !widths) return sfail(FILL_EINVAL, "NULL argument");
  if (!fill_supported_size(nx) || !fill_supported_size(ny)) return sfail(FILL_EUNSUPPORTED_SIZE, "grid size");
  if (nstrips < 1 || nstrips > 64) return sfail(FILL_EINVAL, "nstrips must be in [1, 64]");
  if (!(noise >= 0.0) || !std::isfinite(noise)) return sfail(FILL_EINVAL, "noise must be finite and >= 0");
  if (!(threshold >= 0.0 && threshold < 1.0)) return sfail(FILL_EINVAL, "threshold must be in [0, 1)");
  if (iters < 1) return sfail(FILL_EINVAL, "iters must be >= 1");
  if (prec != FILL_PREC_FP64 && prec != FILL_PREC_FP32_OP) return sfail(FILL_EINVAL, "unknown precision");
  for (int i = 0; i < nstrips; ++i) {
    if (!(widths[i] >= 1.0) || 2 * (int)std::floor(widths[i]) + 1 > std::min(nx, ny))
      return sfail(FILL_EINVAL, "strip " + std::to_string(i) + ": width must be >= 1 and its disk must fit the grid");
    if (!(betas[i] > 0.0) || !std::isfinite(betas[i])) return sfail(FILL_EINVAL, "noise boosts must be > 0");
  }
  fill_strips s = new (std::nothrow) fill_strips_s();
  if (!s) return sfail(FILL_ENOMEM, "host allocation");
  s->nx = nx;
  s->ny = ny;
  s->nstrips = nstrips;
  s->stream = static_cast<hipStream_t>(stream);
  s->plans.assign(nstrips, nullptr);
  s->masks.resize(nstrips);
  const int rc = build(s, mask, P_signal, noise, betas, widths, threshold, iters, prec);
  if (rc != FILL_OK) {
    destroy(s);
    return rc;
  }
  *out = s;
  return FILL_OK;
}

int fill_strips_refine(fill_strips s, double* x) {
  g_strip_error.clear();
  if (!s || !x) return sfail(FILL_EINVAL, "NULL argument");
  const size_t npix = (size_t)s->nx * s->ny;
  for (int i = 0; i < s->nstrips; ++i) {
    if (!s->plans[i]) continue;
    // every pixel outside strip i is data; rtol 1e-300 makes the solve run its
    // iteration cap, which it reports as FILL_ENOCONV
    const int rc = fill_mean(s->plans[i], x, s->tmp, 1e-300);
    if (rc != FILL_OK && rc != FILL_ENOCONV)
      return sfail(rc, std::string("strip ") + std::to_string(i) + ": " + fill_last_error());
    S_HIP(hipMemcpyAsync(x, s->tmp, npix * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
  }
  return FILL_OK;
}

int fill_strips_mean(fill_strips s, const double* d_obs, double* x_out) {
  g_strip_error.clear();
  if (!s || !d_obs || !x_out) return sfail(FILL_EINVAL, "NULL argument");
  if (d_obs == x_out) return sfail(FILL_EINVAL, "x_out may not alias d_obs");
  S_HIP(fillk::launch_select_observed(x_out, d_obs, s->dmask, (size_t)s->nx * s->ny, s->stream));
  return fill_strips_refine(s, x_out);
}

int fill_strips_mask(fill_strips s, int i, uint8_t* out) {
  g_strip_error.clear();
  if (!s || !out || i < 0 || i >= s->nstrips) return sfail(FILL_EINVAL, "bad argument");
  const std::vector<uint8_t>& m = s->masks[i];
  for (size_t k = 0; k < m.size(); ++k) out[k] = m[k];
  return FILL_OK;
}

int fill_strips_plan(fill_strips s, int i, fill_plan* out) {
  g_strip_error.clear();
  if (!s || !out || i < 0 || i >= s->nstrips) return sfail(FILL_EINVAL, "bad argument");
  *out = s->plans[i];
  return FILL_OK;
}

const char* fill_strips_last_error(void) { return g_strip_error.c_str(); }

void fill_strips_destroy(fill_strips s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  destroy(s);
}

}  // extern "C"
