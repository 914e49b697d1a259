/*
 * fill.h -- C ABI of the MI355X (gfx950) constrained-Gaussian-realization
 * fill-in of masked maps on the periodic flat sky.
 *
 * Method: Bucher & Louis, "Filling in CMB map missing data using constrained
 * Gaussian realizations", arXiv:1109.0286.
 *
 * Problem statement (Sec. 2.1): a map z = (x, y) on an nx-by-ny periodic grid
 * is Gaussian with covariance C = P + N; x are the masked (unobserved)
 * pixels, y the observed ones.  On the torus (Sec. 3) C is circulant and
 * diagonal in Fourier space, with eigenvalue P(k) at integer frequency k.
 * fill_realize returns a draw of x from P(x | y) by the Hoffman-Ribak
 * construction (Sec. 2.3): an unconstrained draw s ~ N(0, C), then
 * x = s_x + M (y - s_y) with M = -(Px C^-1 Px)^-1 (Px C^-1 Py) (Sec. 2.1),
 * where the masked-pixel system (Px C^-1 Px) u = v (eq. ModEq) is solved by
 * conjugate gradients preconditioned with E = Px C^{1/2} Px (Sec. 2.4).
 *
 * Layouts and ownership (all calls):
 *   - maps are double, ny rows of nx pixels, row-major, pixel (y, x) at
 *     index y*nx + x;
 *   - mask is uint8, same layout, nonzero = masked (unobserved);
 *   - the spectrum table Pk is double, ny rows of nx/2+1 entries: entry
 *     [iy*(nx/2+1) + ix] is P at frequency (ky, kx) with kx = ix and
 *     ky = iy for iy <= ny/2, iy - ny otherwise; P(k) is the eigenvalue of C
 *     under the unnormalised 2D DFT (pixel variance = mean of P over the
 *     full frequency grid);
 *   - "host" pointers are read during the call and copied; the library keeps
 *     no reference to them;
 *   - "device" pointers are HIP device memory owned by the caller (e.g. torch
 *     tensors), valid for the duration of the call; the library never frees
 *     them;
 *   - every GPU step runs on the stream given at plan creation; calls that
 *     return a result synchronise that stream before returning.
 *
 * Errors: negative return codes (enum fill_status), never exceptions; the
 * text of a code is fill_strerror(code); fill_last_error() gives details of
 * the last failure on the calling thread.
 */
#ifndef FILL_H
#define FILL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fill_plan_s* fill_plan;

enum fill_status {
  FILL_OK = 0,
  FILL_EINVAL = -1,             /* bad argument (null pointer, size, rtol <= 0, ...) */
  FILL_ENOMEM = -2,             /* device or host allocation failed */
  FILL_EHIP = -3,               /* a HIP runtime call failed */
  FILL_ENOCONV = -4,            /* max iterations reached; outputs hold the best iterate */
  FILL_EUNSUPPORTED_SIZE = -5,  /* nx or ny not a supported FFT length */
  FILL_ENOTSPD = -6             /* P(k) <= 0 or not finite, or p.Ap <= 0 in CG */
};

enum fill_precision {
  FILL_PREC_FP64 = 0,    /* every operator apply, vector and scalar in FP64 */
  FILL_PREC_FP32_OP = 1  /* FP32 FFT/operator/CG vectors inside CG; FP64 dot products,
                            scalars, true residual and refinement correction */
};

/* Preconditioners of the inner CG (fill_plan_set_precond). */
enum fill_precond {
  FILL_PRECOND_NONE = 0,   /* plain CG on A */
  FILL_PRECOND_SPLIT = 1,  /* M^-1 = E E, the split form of Sec. 2.4 (default) */
  FILL_PRECOND_CXX = 2,    /* M^-1 = Px C Px */
  FILL_PRECOND_BLOCK = 3   /* M^-1 = block (additive Schwarz) inverse of A: see fill_plan_set_precond */
};

/* Size of a plan's block preconditioner (fill_get_block_info). */
typedef struct {
  int runs;               /* band runs, all problems */
  int blocks;             /* dense blocks, all problems */
  int64_t band_rows;      /* sum over runs of the rows padded to a multiple of 32 */
  int64_t block_pixels;   /* sum over blocks of their pixels n */
  int64_t block_entries;  /* sum over blocks of their inverse entries n * 4 ceil(n / 4) */
  int64_t bytes;          /* device memory it holds (problems with equal factors share them) */
  int elem_bytes;         /* 4 (FP32-operator plan) or 8 (FP64 plan) */
  int64_t band_stream_values; /* sum over runs of the values of their banded factors as stored
                                 (repeating chunks of the factor rows stored once) */
  int halo_min, halo_max;     /* the halos of the problems' blocks (fill_plan_set_block_halo) */
} fill_block_info;

/* Recurrences of the inner CG (fill_plan_set_cg). */
enum fill_cg_variant {
  FILL_CG_STANDARD = 0,         /* Hestenes-Stiefel: two reduction points per iteration (default) */
  FILL_CG_SINGLE_REDUCTION = 1  /* Chronopoulos-Gear: one reduction point per iteration */
};

/* Operators on full maps for fill_apply (Sec. 2.4 notation). */
enum fill_op {
  FILL_OP_CINV = 0,   /* out = C^-1 in */
  FILL_OP_CHALF = 1,  /* out = C^{1/2} in */
  FILL_OP_A = 2,      /* out = Px C^-1 Px in   (zero on observed pixels) */
  FILL_OP_E = 3,      /* out = Px C^{1/2} Px in (zero on observed pixels) */
  FILL_OP_MINV = 4    /* out = M^-1 in, the block preconditioner (zero on observed pixels) */
};

typedef struct fill_stats {
  int iters_inner;       /* CG iterations summed over refinement steps, last solve */
  int iters_outer;       /* refinement (true-residual) steps, last solve */
  int n_masked;          /* masked pixel count of the plan */
  int status;            /* fill_status of the last solve */
  double rel_resid;      /* true FP64 ||v - A u|| / ||v|| at return, last solve */
  double solve_ms;       /* wall time of the last solve, host clock */
  int whole_graph;       /* 1: the last solve ran as one graph replay (see fill_plan_set_graph) */
} fill_stats;

/*
 * Supported grid sizes: nx and ny each one of 16, 32, 64, 96, 128, 192, 256,
 * 384, 512, 768, 1024, 1536, 2048, 3072, 4096 (powers of two from 16 to 4096
 * and three times the powers of two from 32 to 1024: the FFT lengths built
 * into the library, radix 16/8/4/2 and one radix-3 pass); else
 * FILL_EUNSUPPORTED_SIZE.  Other {2,3}-smooth lengths are not built.
 */
int fill_supported_size(int n);

/*
 * Create a plan for an nx-by-ny grid (Sec. 2.1 problem statement; Sec. 3
 * periodic flat domain).
 *   mask      host, ny*nx uint8, nonzero = masked.
 *   Pk        host, ny*(nx/2+1) doubles, every entry > 0 and finite
 *             (else FILL_ENOTSPD).  Must satisfy P(-k) = P(k) on the
 *             kx = 0 and kx = nx/2 columns (any function of |k| does).
 *   prec      enum fill_precision.
 *   stream    hipStream_t to run on (NULL = the null stream).
 *   out       receives the plan; *out is NULL on error.
 * The plan holds the device copies of the mask, the spectral tables 1/P,
 * sqrt(P) and P in FP64 and FP32, and all workspaces; it is used from one
 * host thread at a time (separate plans on separate streams may run
 * concurrently).
 */
int fill_plan_create(int nx, int ny, const uint8_t* mask, const double* Pk, int prec,
                     void* stream, fill_plan* out);

/*
 * Batched plan: nprob problems on the same nx-by-ny grid, solved together
 * (Monte-Carlo draws, many masks; each problem has its own mask, data, seed
 * and CG state, and stops on its own residual).  Every GPU step of a solve
 * covers all problems in one launch.
 *   masks     host, nprob*ny*nx uint8 (problem b at offset b*ny*nx).
 *   Pk        host, n_pk*ny*(nx/2+1) doubles: n_pk = 1 (one spectrum shared by
 *             all problems) or n_pk = nprob (one per problem).
 * Other arguments and errors as fill_plan_create.  A plan from
 * fill_plan_create is a batched plan with nprob = 1.
 */
int fill_plan_create_batch(int nx, int ny, int nprob, const uint8_t* masks, const double* Pk, int n_pk,
                           int prec, void* stream, fill_plan* out);

/* Number of problems of a plan (0 for NULL). */
int fill_plan_nprob(fill_plan plan);

/* Replace the spectrum of an existing plan (host Pk, same layout/rules; n_pk
 * tables as at creation).  A spectrum equal bit for bit to the plan's current
 * one is a no-op (no upload, no preconditioner rebuild). */
int fill_plan_set_pk(fill_plan plan, const double* Pk);

/* Iteration cap of the CG solves (default 20000 summed over refinement steps). */
int fill_plan_set_max_iter(fill_plan plan, int max_iter);

/*
 * Relative tolerance of each FP32-operator inner CG solve between FP64
 * residual recomputations (FILL_PREC_FP32_OP only; default 1e-4, must lie in
 * (0, 1)).  Smaller values mean fewer refinement steps, each longer.
 */
int fill_plan_set_inner_tol(fill_plan plan, double tol);

/*
 * Preconditioner of the inner CG (enum fill_precond, default
 * FILL_PRECOND_SPLIT, the paper's), for later solves; every choice reaches
 * the same solution to rtol.  The fastest is FILL_PRECOND_BLOCK (9 CG
 * iterations at 2048^2 with a 10% band and 200 holes, against 312 - 378 with
 * the split form): it is not the default because it is not the paper's and
 * its set-up costs time and memory (see below); select it for throughput.
 *   FILL_PRECOND_SPLIT  M^-1 = E E, E = Px C^{1/2} Px: equivalent to the split
 *                       system E A E u' = E v of Sec. 2.4 (two applies of E
 *                       per iteration, fused into five passes).
 *   FILL_PRECOND_CXX    M^-1 = Px C Px, the covariance block of the masked
 *                       pixels: the same idea (the powers of C cancel) with
 *                       one apply (three passes) per iteration.
 *   FILL_PRECOND_NONE   CG on A itself, as Sec. 3 does for point-source masks
 *                       (one vector pass per iteration; many more iterations
 *                       on wide cuts).
 *   FILL_PRECOND_BLOCK  not from the paper: an additive-Schwarz inverse of A
 *                       built on the short range of C^-1.  Runs of fully
 *                       masked rows (bands, at most ny - 64 rows) are solved
 *                       exactly per x-frequency kx (their part of A is one
 *                       symmetric Toeplitz matrix per kx, kept to bandwidth 32,
 *                       shifted by a bound of the discarded part where the
 *                       truncation is not safely positive definite, and
 *                       factored by banded Cholesky); every other
 *                       connected piece of the mask (4-neighbours, periodic;
 *                       pieces over 1024 pixels are cut into 16 x 16 cells),
 *                       grown by 8 pixels into the mask, is solved exactly by a
 *                       dense inverse (at most 2048 pixels).  Selecting it
 *                       builds these from the kernel of C^-1 (one GPU
 *                       apply), in the plan's precision: the layout and the
 *                       banded factors on the host (chunks of a factor that
 *                       repeat, where its rows reach their Toeplitz limit,
 *                       are stored once), the dense inverses on the device
 *                       (rocSOLVER, FP64); the time and memory grow with the
 *                       band height times nx and with the sum of squared
 *                       piece sizes.  It is rebuilt by fill_plan_set_pk /
 *                       fill_plan_set_bands.  Batched plans build one per
 *                       problem, once for problems with identical masks and
 *                       spectra (which then share it).  Spectra must satisfy
 *                       P(kx, ky) = P(kx, -ky), else FILL_EINVAL
 *                       (FILL_ENOTSPD if a factor is not positive definite).
 *                       Used with the standard CG recurrence.
 */
int fill_plan_set_precond(fill_plan plan, int mode);

/*
 * Recurrence of the inner CG (enum fill_cg_variant), for later solves.  Both
 * compute the conjugate-gradient iterates of Sec. 2.4 (the same alpha_j and
 * beta_j in exact arithmetic) and reach the same solution to rtol.
 *   FILL_CG_STANDARD          alpha = r.z / p.Ap, then beta = r'.z' / r.z: two
 *                             reduction points, so the operator apply and the
 *                             preconditioner apply are separate pass chains.
 *   FILL_CG_SINGLE_REDUCTION  z = M^-1 r and w = A z are formed back to back
 *                             and r.z, r.r, w.z are summed together; alpha and
 *                             beta follow from them (p.Ap = w.z - beta r.z /
 *                             alpha_prev), with s = A p carried by recurrence.
 *                             The preconditioner's last row pass and the
 *                             operator's first are fused: one launch fewer per
 *                             iteration with every preconditioner.
 * The non-Hermitian study (fill_plan_set_skew) is defined on the standard
 * recurrence.  Returns FILL_EINVAL for an unknown variant.
 */
int fill_plan_set_cg(fill_plan plan, int variant);

/*
 * Halo of the block preconditioner's pieces: each piece of the mask outside
 * the band runs (or each TILE x TILE cell of a large piece) is grown by
 * `halo` pixels (Chebyshev, periodic) within the mask before its dense block
 * is inverted, so that neighbouring pieces and the band overlap (additive
 * Schwarz).  A wider halo couples them over more rows (fewer CG iterations)
 * for more dense entries per apply.
 *   halo in [0, 14]         that halo for every problem;
 *   FILL_BLOCK_HALO_AUTO    (default) per problem from 8 up by 2 (to 14) while
 *                           the blocks hold at most nx*ny/2 more inverse
 *                           entries than with halo 8.
 * A built block preconditioner is rebuilt.  FILL_EINVAL for other values.
 * Callers: tuning of the block preconditioner (Sec. 2.4 leaves the
 * preconditioner open; this one is this library's).
 */
#define FILL_BLOCK_HALO_AUTO (-1)
int fill_plan_set_block_halo(fill_plan plan, int halo);

/*
 * Size of the plan's block preconditioner (its runs, blocks and memory), for
 * the traffic of its kernels: per apply the band solves read
 * 2 * (nx/2 + 1) * 32 * band_rows factor values and read and write the runs'
 * spectra, nx/2 * band_rows complex values; the block products read
 * block_entries inverse entries.  FILL_EINVAL if it is not built.
 */
int fill_get_block_info(fill_plan plan, fill_block_info* out);

/*
 * Lanczos data of the solves (Sec. 6.4): record the CG step lengths alpha_j
 * and direction coefficients beta_j of the first inner CG of each later solve
 * (x0 = 0, the Krylov space of the right-hand side), at most cap steps per
 * problem; cap = 0 stops recording.  Allocates 16*cap*nprob bytes of device
 * memory on growth (cap <= 2^20).  Recording costs one store per coefficient.
 */
int fill_plan_set_lanczos(fill_plan plan, int cap);

/*
 * The recorded coefficients of problem `problem` of the last solve.
 *   alpha, beta  host arrays of cap entries; alpha[0..k) and beta[0..k-1)
 *                are written, k = min(n, cap).
 *   n            out: number of CG steps recorded (0 if the problem needed
 *                none).
 * For the mixed path they are those of the FP32-operator inner CG.
 * FILL_EINVAL without a record (fill_plan_set_lanczos) or for a bad index.
 */
int fill_get_lanczos(fill_plan plan, int problem, double* alpha, double* beta, int cap, int* n);

/*
 * Extreme eigenvalues of the Lanczos matrix of the recorded steps (diagonal
 * 1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j),
 * found by Sturm-sequence bisection on the host: estimates of the smallest
 * and largest eigenvalue of E A E (of A without the preconditioner); their
 * ratio estimates the condition number that sets the iteration count
 * (Sec. 2.4, Sec. 6.4).  The estimates lie inside the operator's spectrum and
 * approach its ends as steps accumulate.  n: steps used.  FILL_EINVAL when
 * nothing was recorded.
 */
int fill_lanczos_extremes(fill_plan plan, int problem, double* lam_min, double* lam_max, int* n);

/*
 * Non-Hermitian study (Sec. 3 reports that CG stalls on operators that are
 * not exactly Hermitian, the more so the larger the condition number): with
 * eps != 0 the A applies inside the inner CG, and fill_apply(FILL_OP_A), use
 *   A_eps = Px C^-1 (I + eps K) Px,
 * K the real antisymmetric circulant with eigenvalues i sin(2 pi kx / nx)
 * (the central difference along x), i.e. each spectral mode of C^-1 is
 * multiplied by 1 + i eps sin(2 pi kx / nx).  The FP64 true residual of the
 * refinement loop keeps the exact A.  eps = 0 (default) restores A; |eps| < 1,
 * else FILL_EINVAL.  For experiments only.
 */
int fill_plan_set_skew(fill_plan plan, double eps);

/*
 * Graph replay (default 1).  The decisions of the refinement loop (when to
 * stop, the next inner tolerance and scaling) are taken on the device, after
 * every step.  A solve runs in one of two ways:
 *   - step by step: the host reads the device state after each refinement
 *     step; the inner CG runs in chunks of 16 iterations (8 with the block
 *     preconditioner) between host checks, each chunk captured once per plan
 *     (per precision, preconditioner and coefficient record) as a HIP graph
 *     and replayed (with 0: launched one by one, bitwise the same);
 *   - as one graph: when the previous solve on the plan was of the same kind
 *     (realize or mean, preconditioner, recurrence; not the single-reduction
 *     recurrence without the block preconditioner) and took at most 8
 *     refinement steps and 128 inner iterations, the whole solve (start
 *     passes, that many steps of that many iterations, assembly) is captured
 *     once and replayed, and the host waits only at its end.  A problem that
 *     converges early stops on the device; one that needs more iterations
 *     than the previous solve had its inner solve cut there and the
 *     refinement continues, step by step after the graph if needed.  With
 *     the same iteration counts the result is bitwise that of the step-by-step
 *     solve; otherwise it differs within the tolerance.
 * fill_stats.whole_graph tells which way the last solve ran.  Kernels are
 * launched directly while fill_kernel_timing is on.
 */
int fill_plan_set_graph(fill_plan plan, int on);

/*
 * Kernel-based Laplace relaxation of the masked pixels (Sec. 6.1, 6.3): in the
 * far interior of a wide cut the fill nearly solves the Laplace equation, and
 * a harmonic function equals its average over an annulus around any point.
 * Kernel j (0 <= j < nkernels) is the annulus r_{j-1}^2 < dx^2 + dy^2 <= r_j^2
 * (r_{-1} = 0), r_j = r0 ratio^j, normalised to sum 1; a masked pixel uses the
 * largest j >= 1 whose disk of radius r_j holds no observed pixel, else 0 (the
 * boundary layer, whose small kernel reaches the data).  x_out (device ny*nx,
 * may not alias d_obs) = d_obs on observed pixels; masked pixels start at 0
 * and take `iters` Jacobi sweeps (each: one FFT convolution per kernel in use,
 * FP64, problem 0's mask; one-problem plans only).  1 <= nkernels <= 16,
 * r0 >= 1, ratio > 1, 2 floor(r_max) + 1 <= min(nx, ny), else FILL_EINVAL.
 * The kernel spectra and classes are kept in the plan while the parameters
 * repeat.  An approximation: it is the start of fill_strips_refine.
 */
int fill_laplace(fill_plan plan, const double* d_obs, double* x_out, int nkernels, double r0, double ratio, int iters);

/*
 * Warm start of the solves of a one-problem plan (Sec. 6.1, 6.3: the paper
 * fills the far interior of a wide cut with its kernel Laplace solver before
 * refining): with iters > 0 every later fill_realize / fill_mean starts the CG
 * refinement from u0 = the fill_laplace relaxation (nkernels, r0, ratio,
 * iters sweeps) of y - s_y (y for the mean) instead of u0 = 0, i.e. its first
 * step solves A d = v - A u0.  The solution (to rtol) is the same; the
 * relaxation's FFT convolutions are extra work, and the solves run step by
 * step (no whole-solve graph).  iters = 0 (default) turns it off.  Arguments
 * as fill_laplace; FILL_EINVAL for a batched plan or a kernel that does not
 * fit the grid.
 */
int fill_plan_set_warm_start(fill_plan plan, int iters, int nkernels, double r0, double ratio);

/*
 * Noise-boosted strip refinement (Sec. 6.2 subdivision, Sec. 6.4 refinement):
 * an approximate maximum-likelihood fill by a few CG iterations on nested
 * strips along the boundary of the masked region.
 *
 * fill_strips_create: subdivision and one plan per strip.
 *   mask       host uint8 ny*nx, 1 = masked (copied).
 *   P_signal   host FP64 ny*(nx/2+1), the signal part of the spectrum (layout
 *              as fill_plan_create); noise: the white-noise level N >= 0.
 *   nstrips    strips 1..64 with noise boosts betas[i] > 0 and widths
 *              widths[i] >= 1 (host arrays; widths decreasing for nested
 *              strips); 2 floor(w) + 1 must not exceed min(nx, ny).
 *   threshold  in [0, 1): strip i holds the masked pixels whose periodic disk
 *              {dx^2 + dy^2 <= w_i^2} contains more than threshold * (pixels
 *              in the disk) observed pixels (the paper uses 0.03).
 *   iters      CG iterations per strip (>= 1; the paper uses 20).
 *   prec       enum fill_precision of the strip solves (with FILL_PREC_FP32_OP
 *              the iterations are counted over the FP32 inner solves and
 *              their FP64 refinement restarts together).
 * Strip i is solved with spectrum P_signal + betas[i] * noise (FILL_ENOTSPD
 * if not positive).  Empty strips are skipped.  Owned by the library.
 */
typedef struct fill_strips_s* fill_strips;
int fill_strips_create(int nx, int ny, const uint8_t* mask, const double* P_signal, double noise, int nstrips,
                       const double* betas, const double* widths, double threshold, int iters, int prec,
                       void* hip_stream, fill_strips* out);

/*
 * The refined fill: x_out (device ny*nx, may not alias d_obs) = d_obs on
 * observed pixels; masked pixels start at 0 and each strip in order replaces
 * its pixels by `iters` CG iterations of the maximum-likelihood fill given
 * every other pixel of the current map.  Masked values of d_obs are ignored.
 */
int fill_strips_mean(fill_strips strips, const double* d_obs, double* x_out);

/*
 * The strip sequence on an already filled map, in place: x (device ny*nx)
 * holds the data on observed pixels and a start on masked ones (for example
 * the output of fill_laplace, as the paper starts from its Laplace fill).
 */
int fill_strips_refine(fill_strips strips, double* x);

/* Strip i as a host uint8 ny*nx mask (out must hold ny*nx bytes). */
int fill_strips_mask(fill_strips strips, int i, uint8_t* out);

/* The plan of strip i (owned by the strips object; NULL for an empty strip),
 * e.g. to record its CG coefficients with fill_plan_set_lanczos. */
int fill_strips_plan(fill_strips strips, int i, fill_plan* out);

/* Message of the last failed fill_strips_* call on this thread. */
const char* fill_strips_last_error(void);

/* Release the strips object and its plans (NULL is accepted). */
void fill_strips_destroy(fill_strips strips);

/* Release every resource of the plan (NULL is accepted). */
void fill_plan_destroy(fill_plan plan);

/*
 * Constrained Gaussian realization (Sec. 2.3, Hoffman-Ribak construction).
 *   d_obs   device, ny*nx doubles; values on masked pixels are ignored (may be
 *           0 or NaN, Sec. 3 sets them to zero).
 *   seed    key of the white noise: Philox4x64-10, key (seed, 0x52), counter
 *           (j, 0, 0, 0) for pixels 4j .. 4j+3 of row-major index i
 *           (j = i/4), four normals per block by Box-Muller, two from each
 *           word pair (words 0,1 -> pixels 4j, 4j+1; words 2,3 -> 4j+2,
 *           4j+3; radius sqrt(-2 ln u_a), angle 2 pi u_b, cosine then sine;
 *           u = ((w >> 11) + 0.5) 2^-53).
 *   x_out   device, ny*nx doubles (may not alias d_obs): observed pixels are
 *           bitwise copies of d_obs; masked pixels are s + u with s = C^{1/2} w
 *           and u = M (y - s_y).
 *   rtol    > 0: stop when the true FP64 residual ||v - A u||_2 <= rtol ||v||_2
 *           over masked pixels, v = -Px C^-1 Py (y - s).
 * Returns FILL_OK, FILL_ENOCONV (x_out holds the best iterate) or an error.
 */
int fill_realize(fill_plan plan, const double* d_obs, uint64_t seed, double* x_out, double rtol);

/* Conditional mean / Wiener fill x_ML = M y (Sec. 2.1): as fill_realize with s = 0. */
int fill_mean(fill_plan plan, const double* d_obs, double* x_out, double rtol);

/*
 * fill_realize / fill_mean for every problem of a batched plan.
 *   d_obs, x_out  host arrays of nprob device pointers (ny*nx doubles each;
 *                 x_out[b] may not alias d_obs[b]).
 *   seeds         host array of nprob seeds (key (seeds[b], 0x52)).
 * Each problem stops when its own true residual is <= rtol.  Returns
 * FILL_OK, FILL_ENOCONV if any problem did not converge (its x_out holds the
 * best iterate), or an error.  fill_realize/fill_mean require nprob = 1.
 */
int fill_realize_batch(fill_plan plan, const double* const* d_obs, const uint64_t* seeds,
                       double* const* x_out, double rtol);
int fill_mean_batch(fill_plan plan, const double* const* d_obs, double* const* x_out, double rtol);

/*
 * Several batched plans at once (for example one per grid size of a
 * Monte-Carlo study with uneven sizes): plan i runs fill_realize_batch with
 * d_obs[i], seeds[i], x_out[i] on its own host thread, so plans created on
 * different streams overlap on the GPU.  Returns the worst status;
 * fill_last_error names the plan.
 */
int fill_realize_multi(int nplans, const fill_plan* plans, const double* const* const* d_obs,
                       const uint64_t* const* seeds, double* const* const* x_out, double rtol);

/*
 * A group of batched plans solved together (a Monte-Carlo step over maps of
 * uneven sizes, Sec. 1: one batched plan per grid size, each with its own
 * masks, spectra, data and seeds).  The group refers to the plans (which must
 * outlive it and appear once each) and launches on `stream`.
 *
 * fill_group_realize runs fill_realize_batch on every plan (d_obs[i],
 * seeds[i], x_out[i] as there).  The first call, and any call after which a
 * plan's step counts change, runs the plans step by step, each on its own
 * stream and host thread; once every plan's previous solve gives its step
 * counts (see fill_plan_set_graph: same kind of solve, at most 8 steps and
 * 128 inner iterations, graphs on), the plans' solves are captured as one
 * HIP graph -- one branch per plan, each branch the plan's whole solve with
 * its per-problem descriptors (map pointers, seeds, refinement state) read
 * from device tables and every convergence decision taken on the device --
 * and every later call is that graph launched once on the group's stream,
 * with one host wait at the end.  A plan whose problems need more steps than
 * predicted continues step by step after the graph.  Results as
 * fill_realize_batch per plan; returns the worst status (fill_last_error
 * names the plan).  fill_group_last_graph: 1 if the last call ran as one
 * graph launch.  fill_group_destroy releases the group (not the plans; NULL
 * is accepted).
 */
typedef struct fill_group_s* fill_group;
int fill_group_create(int nplans, const fill_plan* plans, void* stream, fill_group* out);
int fill_group_realize(fill_group group, const double* const* const* d_obs, const uint64_t* const* seeds,
                       double* const* const* x_out, double rtol);
int fill_group_last_graph(fill_group group);
void fill_group_destroy(fill_group group);

/* Statistics of the last solve on this plan (fill_realize, fill_mean or the
 * adjoint solve of fill_adjoint; for a batch: iteration counts and residual
 * are the maxima over problems, n_masked the total). */
int fill_get_stats(fill_plan plan, fill_stats* out);

/* Per-problem statistics of the last solve: out has nprob entries. */
int fill_get_stats_batch(fill_plan plan, fill_stats* out);

/*
 * Apply one operator of enum fill_op (with problem 0's mask and spectrum) to
 * a full map (device in/out, ny*nx doubles, may not alias) in precision prec (enum fill_precision; FP32
 * rounds the input to float and returns the float result widened).  The
 * operators are the ones every CG iteration applies (Sec. 2.4).
 * FILL_OP_MINV applies the block preconditioner; it needs FILL_PRECOND_BLOCK
 * selected and prec equal to the plan's precision, else FILL_EINVAL.
 */
int fill_apply(fill_plan plan, int op, int prec, const double* in, double* out);

/* The unconstrained draw s = C^{1/2} w for a seed (problem 0's spectrum; device out, ny*nx). */
int fill_realize_unconstrained(fill_plan plan, uint64_t seed, double* out);

/*
 * fill_realize_unconstrained without allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same draw, bit for bit, as
 * fill_realize_unconstrained: the transposed half spectrum of the three
 * passes lives in a file-scope device array of the library (64 MiB per GPU,
 * held until the process ends) instead of the plan's workspace.
 *   plan  created beforehand (plan creation allocates); its device must be
 *         the current device, else FILL_EINVAL.
 *   out   device, ny*nx doubles (caller-owned).
 * Limit: (nx/2) * ny * 16 bytes <= 64 MiB, i.e. nx * ny <= 8388608 (up to
 * 2048 x 4096), else FILL_EINVAL.  Calls hipMalloc/hipFree never.  The
 * kernels are enqueued on the plan's stream and the call returns without
 * synchronising: out is ready when the stream reaches that point.  Every call
 * on one GPU shares that GPU's array (each call overwrites all it reads), so
 * calls that overlap on one GPU (on different streams or host threads) race.
 */
int fill_realize_unconstrained_noalloc(fill_plan plan, uint64_t seed, double* out);

/*
 * Raw Philox4x64-10 words (Salmon et al. 2011) for counters (j, 0, 0, 0),
 * j = 0..n_blocks-1, key (seed, stream): out is device, 4*n_blocks uint64,
 * block j at out[4j..4j+3].  Runs on the null stream and synchronises.
 */
int fill_philox_words(uint64_t seed, uint64_t stream, int64_t n_blocks, uint64_t* out);

/*
 * Band-power spectrum: theta[b] = ln P at ln k = lnk_nodes[b] (nbands nodes,
 * strictly increasing), ln P(k) piecewise linear in ln k between nodes and
 * constant outside [lnk_nodes[0], lnk_nodes[nbands-1]] (k = 0 takes
 * theta[0]).  Computes the tables of every problem of the plan from theta
 * (host arrays; replaces any previous spectrum; tables equal bit for bit to
 * the current ones are not uploaded again and do not rebuild the block
 * preconditioner).  The model stands in for the paper's P = w C + N (Sec. 3)
 * when the spectrum is to be differentiated.
 */
int fill_plan_set_bands(fill_plan plan, int nbands, const double* lnk_nodes, const double* theta);

/*
 * Gradient of a loss L on the filled map (the output of fill_realize with the
 * same d_obs, seed and plan), given g = dL/dx_out (the derivative of the
 * fill of Sec. 2.1 / 2.3; the paper does not give it).  One extra CG solve
 * A lambda = g_x with the operators of Sec. 2.4, in the plan's precision
 * with FP64 refinement to true relative residual rtol; then
 *   grad_dobs = dL/dd_obs = g - C^-1 lambda on observed pixels, 0 on masked;
 *   grad_logP[k] = dL/d ln P_k on the half spectrum (layout of Pk);
 *   grad_theta[b] = sum_k phi_b(k) grad_logP[k] for the band model of
 *   fill_plan_set_bands (required if grad_theta is not NULL).
 *   d_obs, x_out, g   device, ny*nx doubles (x_out as returned by fill_realize).
 *   grad_dobs         device, ny*nx doubles.
 *   grad_theta        host, nbands doubles, or NULL.
 *   grad_logP         host, ny*(nx/2+1) doubles, or NULL.
 * Returns FILL_OK, FILL_ENOCONV (gradients from the best iterate) or an error.
 */
int fill_adjoint(fill_plan plan, const double* d_obs, uint64_t seed, const double* x_out, const double* g,
                 double* grad_dobs, double* grad_theta, double* grad_logP, double rtol);

/*
 * fill_adjoint for every problem of a batched plan (host arrays of nprob
 * device pointers); one batched adjoint solve.  grad_theta is the sum over
 * problems (the band powers are shared); grad_logP (if not NULL) holds
 * nprob per-problem blocks of ny*(nx/2+1).
 */
int fill_adjoint_batch(fill_plan plan, const double* const* d_obs, const uint64_t* seeds,
                       const double* const* x_out, const double* const* g, double* const* grad_dobs,
                       double* grad_theta, double* grad_logP, double rtol);

/* Kernels that fill_time_kernel can time (one operator apply, Sec. 2.4). */
enum fill_kernel {
  FILL_K_R2C = 0,    /* row pass: compact masked vector -> transposed half spectrum */
  FILL_K_COL = 1,    /* column pass: FFT along y, times 1/P, inverse FFT along y */
  FILL_K_C2R = 2,    /* row pass: half spectrum -> masked pixels (compact) */
  FILL_K_APPLY = 3,  /* the three in sequence: one apply of A = Px C^-1 Px */
  FILL_K_PROJ = 4,   /* row pass between the two C^{1/2} applies of E E r */
  FILL_K_BAND = 5,   /* block preconditioner: banded per-frequency solves of the band runs */
  FILL_K_BLOCKMV = 6, /* block preconditioner: dense products with the block inverses */
  FILL_K_COMBINE = 7 /* block preconditioner: combination and the r.z / r.r partials */
};

/*
 * Measurement helper: launch one kernel of the A apply, or of the block
 * preconditioner (FILL_K_BAND, FILL_K_BLOCKMV, FILL_K_COMBINE: it must be
 * built, and prec must be the plan's precision), `reps` times on the plan's
 * stream with the arguments a CG iteration uses, bracketed by HIP events on
 * that stream; *avg_ms = elapsed / reps.  prec selects the FP64 or FP32
 * kernels.  Overwrites the plan's workspaces (not d_obs/x_out).
 */
int fill_time_kernel(fill_plan plan, int kernel, int prec, int reps, double* avg_ms);

/*
 * Measurement helper: from now on, bracket every launch of one kernel
 * (FILL_K_R2C, FILL_K_COL, FILL_K_C2R, FILL_K_PROJ, FILL_K_BAND, FILL_K_BLOCKMV or
 * FILL_K_COMBINE; -1 = off) in precision
 * prec during solves on this plan with a pair of HIP events on the plan's
 * stream.  Resets the accumulated totals.
 */
int fill_kernel_timing(fill_plan plan, int kernel, int prec);

/*
 * Sum of the event-measured durations (ms) and the number of timed launches
 * since the last read or fill_kernel_timing call; synchronises the stream and
 * resets the totals.
 */
int fill_kernel_timing_read(fill_plan plan, double* total_ms, int64_t* count);

/* Text for a status code. */
const char* fill_strerror(int code);

/* Detail of the last error raised on this host thread ("" if none). */
const char* fill_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FILL_H */
