// Host-callable launchers of the device kernels (declarations).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fillk {

struct CGScalars;
struct RefineArgs;
template <typename T> struct RowArgs;
template <typename T> struct ColArgs;
template <typename T> struct BandArgs;
template <typename T> struct BlockArgs;
template <typename T> struct CombArgs;

// e0/e1 (may be null): events timestamped at the start and end of the dispatch.
template <typename T>
hipError_t launch_r2c(int mode, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_c2r(int mode, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_col(int ny, const ColArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
// dot: also write the projected values in compact order with DOT2 partials
template <typename T>
hipError_t launch_proj(bool dot, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T> int row_block_rows(int nx);
// CG vector update without a preconditioner (init: only the r.r partials),
// nblk row blocks per problem.
template <typename T> hipError_t launch_xr(bool init, const RowArgs<T>& a, int nblk, hipStream_t s);

// Block preconditioner: banded per-frequency solves of nruns band runs (the
// largest padded to max_hp rows), dense block products, combination with the
// r.z / r.r partials over nblk row blocks.
template <typename T>
hipError_t launch_band_solve(const BandArgs<T>& a, int nruns, int max_hp, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_block_mv(const BlockArgs<T>& a, int nblocks, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
// Both of the above in one launch (band solves of nruns runs, nitems block
// product work items); needs nx/2 a multiple of 4.
template <typename T>
hipError_t launch_band_block(const BandArgs<T>& ba, const BlockArgs<T>& bk, int nruns, int max_hp, int nitems,
                             hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_combine(const CombArgs<T>& a, int nblk, int nprob, hipStream_t s, hipEvent_t e0, hipEvent_t e1);

// Set-up of the dense block inverses, one size class m at a time (blist:
// count blocks with at most m pixels; boff, px: the blocks' pixel lists):
// A holds count column-major m x m matrices stride apart, C^-1 on each
// block's pixels from the kernel map kmap (FP64) padded with the identity;
// the inverses from their lower triangles into dst at moff[b] (column
// stride 4 ceil(n / 4)) in the plan's precision.
hipError_t launch_block_assemble(double* A, size_t stride, const int* blist, int count, const int* boff,
                                 const int* px, int m, const double* kmap, int nx, int ny, hipStream_t s);
template <typename T>
hipError_t launch_block_store(T* dst, const size_t* moff, const int* blist, int count, const int* boff,
                              const double* A, size_t stride, int m, hipStream_t s);

// Per-problem elementwise helpers over compact vectors (problem b: comp_off[b]..comp_off[b+1]).
hipError_t launch_scale_to_f32(float* out, const double* in, const double* scale, const int* comp_off, int nmax,
                               int nprob, hipStream_t s);
hipError_t launch_scale_f64(double* out, const double* in, const double* scale, const int* comp_off, int nmax,
                            int nprob, hipStream_t s);
// out = scale * in, z0 = z1 = 0 (and zu = 0 when not null) over every problem's range
hipError_t launch_scale_init_f32(float* out, const double* in, const double* scale, const int* comp_off, float* z0,
                                 float* z1, double* zu, int nmax, int nprob, hipStream_t s);
hipError_t launch_scale_init_f64(double* out, const double* in, const double* scale, const int* comp_off, double* z0,
                                 double* z1, double* zu, int nmax, int nprob, hipStream_t s);
struct SolveState;
// gate (may be null): skip unless every one of the nprob states is done
hipError_t launch_scatter_add(double* const* full, const double* c, const int* pos, const int* comp_off, int nmax,
                              int nprob, hipStream_t s, const SolveState* gate = nullptr);
// Refinement control, one workgroup per problem.  The per-problem sum of
// part[b*stride .. b*stride+n) (fixed order) is ||v||^2 (begin: the state is
// reset) or ||v - A u||^2; then the next step is decided (active, scale,
// unscale, tol2, cap and the CG scalars of the next inner solve; done and
// status for problems that stop).
hipError_t launch_ctl(const RefineArgs& a, const double* part, size_t stride, int n, bool begin, hipStream_t s);
// After an inner solve, in one launch: u += unscale x over every problem's
// range, and the solve's accounting (iterations and status from the CG
// scalars; a problem not yet stopped whose last r.r partials, rr_part with nb
// per problem or null, meet its tolerance counts as converged).
hipError_t launch_axpy_after_f32(double* u, const float* x, const int* comp_off, const RefineArgs& a,
                                 const double* rr_part, int nb, size_t stride, bool first, int nmax, hipStream_t s);
hipError_t launch_axpy_after_f64(double* u, const double* x, const int* comp_off, const RefineArgs& a,
                                 const double* rr_part, int nb, size_t stride, bool first, int nmax, hipStream_t s);
// Between inner-CG chunks: stop every problem whose last r.r partials meet
// its tolerance (the same test, in the same summation order, as above).
hipError_t launch_rr_check(CGScalars* sc, const double* rr_part, int nb, size_t stride, int nprob, hipStream_t s);
hipError_t launch_mean_prep(double* const* x_out, double* t, const double* const* d, const uint8_t* mask,
                            size_t npix, int nprob, hipStream_t s);

// Single-problem helpers (operator applies on full maps).
hipError_t launch_scatter(double* full, const double* c, const int* pos, int n, hipStream_t s);
hipError_t launch_scatter_f32(double* full, const float* c, const int* pos, int n, hipStream_t s);
hipError_t launch_gather(double* c, const double* full, const int* pos, int n, hipStream_t s);
hipError_t launch_philox_words(uint64_t* out, uint64_t seed, uint64_t stream, int64_t nblocks, hipStream_t s);

// Adjoint (FP64).
hipError_t launch_col_fwd(int ny, const double2* Xt, double2* Xs, int ldx, int nhalf, const double2* tw,
                          hipStream_t s);
hipError_t launch_adj_maps(const uint8_t* mask, const double* g, const double* cl, const double* x, const double* s,
                           const double* d, double* grad_y, double* h, double* v, size_t npix, hipStream_t st);
hipError_t launch_adj_gather(double* b, double* const* g_tab, const int* pos, const int* comp_off, int nmax, int nprob,
                             hipStream_t st);
hipError_t launch_spec_grad(const double2* Xh, const double2* Xw, const double2* Xl, const double2* Xv,
                            const double* Dhalf, const double* Dinv, int nx, int ny, double* G, double* G_api,
                            hipStream_t st);
hipError_t launch_band_reduce(const double* G, int nx, int ny, const double* lnk, int nb, double* out,
                              hipStream_t st);
hipError_t launch_cnorm2(double* out, const double* v, const int* comp_off, int nprob, hipStream_t st);

// Strip subdivision (exact periodic-disk counts of observed pixels) and map selection.
hipError_t launch_strip_flags(const uint8_t* mask, int* pre, const int* hw, int r, int nx, int ny, double thr_count,
                              uint8_t* out, hipStream_t s);
hipError_t launch_select_observed(double* x, const double* d, const uint8_t* mask, size_t npix, hipStream_t s);
// Laplace relaxation helpers: kernel classes, class-wise update, kernel spectra.
hipError_t launch_class_init(uint8_t* cls, const uint8_t* mask, size_t npix, hipStream_t s);
hipError_t launch_class_raise(uint8_t* cls, const uint8_t* touch, const uint8_t* mask, int j, size_t npix,
                              hipStream_t s);
hipError_t launch_take_class(double* x, const double* avg, const uint8_t* cls, int j, size_t npix, hipStream_t s);
hipError_t launch_real_scale(double* tab, const double2* X, double scale, size_t n, hipStream_t s);

}  // namespace fillk
