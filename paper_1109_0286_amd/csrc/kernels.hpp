// The three passes of an operator apply on the nx-by-ny torus (Sec. 2.4):
//
//   r2c  : ROWS image rows per workgroup -> real FFT along x of each row (two
//          rows packed as the real and imaginary parts of one complex line) ->
//          half spectrum written TRANSPOSED, Xt[kx][y], so that
//   col  : each spectral column kx is a contiguous line of ny complex values:
//          forward FFT along y, multiply by the diagonal D(k) in {1/P, sqrt(P)}
//          (scaled by 1/(nx ny)), inverse FFT along y, in place;
//   c2r  : transposed half spectrum -> inverse real FFT along x -> the pixels
//          the caller wants (the masked pixels in compact order, or full rows).
//
// The projections Px / Py are the input/output selections of the row passes:
// compact vectors hold only the masked pixels (row-major order), pos[c] is the
// pixel index of compact element c and row_off[y] the first compact element of
// row y.  The CG vector updates and the FP64 partial dot products of each
// iteration are fused into the row passes (prologue of r2c, epilogue of c2r).
#pragma once

#include <hip/hip_ext.h>

#include "fft_device.hpp"

namespace fillk {

// Scalars of one conjugate-gradient solve, resident on the device.  rho is
// double-buffered by iteration parity: the kernel that forms rho_new reads
// rho[parity] while its workgroup 0 stores rho[parity ^ 1].
struct CGScalars {
  double rho[2];  // r.z
  double alpha;   // rho / (p.q)
  double beta;    // rho_new / rho_old
  double alph[2]; // single-reduction CG: alpha by iteration parity, as rho
  double rr;      // r.r of the recursive residual
  double tol2;    // stop when rr <= tol2
  int done;       // set when converged, failed or capped: every kernel then returns at once
  int iter;       // completed iterations
  int max_iter;
  int status;     // 0 ok, -4 iteration cap, -6 p.q <= 0 or r.z <= 0
  int cap;        // iteration cap reached; the next iteration stops
  int pad;
};

// Refinement-loop state of one problem (the Sec. 2.4 solve with FP64 true
// residuals), resident on the device: the control kernels between the inner
// CG solves decide each next step from it, so a whole solve can run without
// the host; the host reads it back when the solve ends.
struct SolveState {
  double bnorm2;    // ||v||^2
  double rnorm2;    // ||v - A u||^2 of the last true residual
  double prev;      // relative residual before the last inner solve
  double rel;       // relative residual now
  int total;        // inner iterations so far
  int outer;        // refinement steps so far
  int done;         // converged or failed: no further step
  int status;       // 0, -4 (no convergence), -6 (breakdown or non-finite residual)
  int first_iters;  // iterations of the first inner solve
  int cut;          // the last inner solve stopped at its iteration budget above its tolerance
  int its[8];       // iterations of inner solves 0..7
};
constexpr int kStateIts = 8;

// Per-call settings of the refinement loop (device copy).
struct SolveCfg {
  double rtol;       // true relative residual to reach
  double inner_tol;  // floor of the FP32-operator inner tolerance
  int max_iter;      // inner iterations summed over refinement steps
  int max_outer;     // refinement steps
  int fp64;          // FP64 inner solves: tolerance 0.5 rtol / rel without the floor
  int pad;
};

// Arguments of the control kernels: the state, the per-call settings, and the
// parameters and CG scalars of the next inner solve that they write.
struct RefineArgs {
  SolveState* st;
  const SolveCfg* cfg;
  CGScalars* sc;        // reset for the next inner solve when it is decided
  double* scale;        // r = scale * res
  double* unscale;      // u += unscale * x
  double* tol2;
  int* cap;
  int* active;
  int nprob;
};

enum R2CMode {
  R2C_COMPACT = 0,   // input v0[c]
  R2C_PUPDATE = 1,   // p = z + beta p   (v0 = z, v1 = p), input p
  R2C_XRUPDATE = 2,  // x += alpha p, r -= alpha q (v0 = x, v1 = r, v2 = p, v3 = q), input r
  R2C_FULL = 3,      // input full map full_in (double)
  R2C_NOISE = 4,     // input white noise of (seed, stream)
  // single-reduction CG step: p = z + beta p, s = w + beta s, x += alpha p,
  // r -= alpha s (v0 = x, v1 = r, v2 = p, v3 = s, v4 = z or null for z = r,
  // v5 = w), input r; with part0, the r.r partials of the new r
  R2C_CG1UPDATE = 5
};

enum C2RMode {
  C2R_COMPACT = 0,   // v0[c] = scale*val; if part0: part0 += v0[c] * (v1 ? v1[c] : v0[c])
  C2R_DOT2 = 1,      // v0[c] = val; part0 += v1[c]*val, part1 += v1[c]^2
  C2R_RESID = 2,     // v0[c] = v1[c] - val; part0 += v0[c]^2
  C2R_REALIZE = 3,   // s = val; full_out = mask ? s : d, full_out2 = mask ? 0 : d - s (d = full_in)
  C2R_FULL = 4       // full_out = scale*val
};

// A band run of the block preconditioner as the row passes see it: its rows
// are a grid of hp rows of its own (row offsets at row_off, pixel positions
// relative to cb0, spectrum at bt_off complex values), solved with the CG
// state of problem prob.
struct RunRow {
  size_t row_off;
  size_t bt_off;
  int hp;
  int cb0;
  int prob;
  int pad;
};

// Arguments of the row passes.  A launch covers nprob problems of the same
// grid (blockIdx.y = problem): pointers are problem 0's and bind_problem()
// moves them to problem blockIdx.y (compact vectors by comp_off, the rest by
// the strides).  With runs set, blockIdx.y is a band run instead (ny: the
// largest run's rows; workgroups past a run's rows return).
template <typename T> struct RowArgs {
  int nx, ny, ldx;
  int nprob;
  const int* comp_off;           // nprob+1 compact offsets (null: one problem)
  size_t xt_stride;              // complex values between problems' spectra
  size_t part_stride;            // partial-sum slots per problem
  size_t pix_stride;             // pixels between problems' internal maps and masks
  const double* const* fin_tab;  // caller input maps per problem (null: full_in + b*pix_stride)
  double* const* fout_tab;       // caller output maps per problem (null: full_out + b*pix_stride)
  const uint64_t* seeds;         // per-problem seeds (null: seed)
  const int* row_off;
  const int* pos;
  cplx<T>* Xt;
  const cplx<T>* tw;
  T* v0;
  T* v1;
  T* v2;
  T* v3;
  T* v4;
  T* v5;
  T scale;
  CGScalars* sc;
  double* part0;
  double* part1;
  const double* red0;  // partial sums of the previous row pass (CG scalar inputs)
  const double* red1;
  const double* red2;
  int nred;
  int parity;          // iteration parity (selects the rho buffer)
  double* hist;        // CG coefficient record (alpha_j at 2j, beta_j at 2j+1), or null
  int hist_cap;        // coefficients recorded per problem
  const double* full_in;
  double* full_out;
  double* full_out2;
  const uint8_t* mask;
  uint64_t seed, stream;
  const RunRow* runs;
};

template <typename T> struct ColArgs {
  cplx<T>* Xt;
  int ldx, ncol;
  const T* D;
  const cplx<T>* tw;
  const CGScalars* sc;
  int nprob;
  size_t xt_stride;  // complex values between problems' spectra
  size_t d_stride;   // table entries between problems' tables (0: one shared table)
  double skew;       // 0, or eps of the non-Hermitian study: D(k) (1 + i eps sin(2 pi kx / nx))
};

// Block preconditioner (k_block.hip): the banded per-frequency solves of the
// band runs, the dense block products and their combination.
constexpr int kBlockMax = 2048;  // largest block (dense inverse)
template <typename T> struct BandArgs {
  cplx<T>* Bt;            // the runs' transposed row spectra, run r at run_bt[r]: [nx/2][hp]
  const T* fwd;           // factor streams: (run, kx) at kx_off[run_k0[run] + kx]: [32][hp - 32 d]
  const int* run_hp;      // padded rows of each run (multiple of 32)
  const size_t* run_bt;
  const int* run_k0;      // per run: index of its (kx = 0) entry in kx_off / kx_dup
  const size_t* kx_off;
  const int* kx_dup;      // per (run, kx): s0, d (chunks s0 .. s0 + d stored once, as chunk s0)
  int nruns;
  int max_hp;             // the largest run's padded rows
  int ncol;               // nx/2
  const int* run_prob;    // problem of each run (its CG scalars: sc + problem)
  const CGScalars* sc;
};
template <typename T> struct BlockArgs {
  const T* r;             // compact input
  T* seg;                 // outputs of the work items
  const int* items;       // work items: block, first row, first column, output offset
  const int* boff;        // nblocks+1 offsets into bidx
  const int* bidx;        // compact indices of the blocks' pixels
  const size_t* moff;     // offsets of the n x n inverses
  const T* binv;
  const int* block_prob;  // problem of each block
  const CGScalars* sc;
};
template <typename T> struct CombArgs {
  T* z;                   // in: band part on band pixels; out: M^-1 r
  const T* r;
  const T* seg;
  const int* cst;         // n_m+1: block entries covering each element (CSR)
  const int* cix;
  const uint8_t* inb;     // element lies in a band run
  const int* row_off;     // ny+1 per problem, relative to the problem's compact offset
  const int* comp_off;    // nprob+1 compact offsets
  int ny;
  size_t part_stride;     // partial slots per problem
  int rows;               // rows per workgroup (partials per row block)
  double* part0;          // r.z partials (or null)
  double* part1;          // r.r partials (or null)
  const CGScalars* sc;
};

template <typename T> __device__ __forceinline__ RowArgs<T> bind_problem(RowArgs<T> a) {
  const int b = blockIdx.y;
  if (a.runs != nullptr) {
    const RunRow rr = a.runs[b];
    a.row_off += rr.row_off;
    a.pos -= rr.cb0;
    a.Xt += rr.bt_off;
    a.ny = a.ldx = rr.hp;
    if (a.sc) a.sc += rr.prob;
    return a;
  }
  if (b == 0) return a;
  const int coff = a.comp_off ? a.comp_off[b] : 0;
  a.row_off += (size_t)b * (a.ny + 1);
  a.pos += coff;
  if (a.v0) a.v0 += coff;
  if (a.v1) a.v1 += coff;
  if (a.v2) a.v2 += coff;
  if (a.v3) a.v3 += coff;
  if (a.v4) a.v4 += coff;
  if (a.v5) a.v5 += coff;
  a.Xt += (size_t)b * a.xt_stride;
  if (a.sc) a.sc += b;
  if (a.part0) a.part0 += (size_t)b * a.part_stride;
  if (a.part1) a.part1 += (size_t)b * a.part_stride;
  if (a.red0) a.red0 += (size_t)b * a.part_stride;
  if (a.red1) a.red1 += (size_t)b * a.part_stride;
  if (a.red2) a.red2 += (size_t)b * a.part_stride;
  if (a.hist) a.hist += (size_t)b * 2 * a.hist_cap;
  if (a.mask) a.mask += (size_t)b * a.pix_stride;
  if (a.full_in) a.full_in += (size_t)b * a.pix_stride;
  if (a.full_out) a.full_out += (size_t)b * a.pix_stride;
  if (a.full_out2) a.full_out2 += (size_t)b * a.pix_stride;
  return a;
}
// Per-problem caller maps and seeds (valid for every problem index, 0 included).
template <typename T> __device__ __forceinline__ void bind_caller(RowArgs<T>& a) {
  const int b = blockIdx.y;
  if (a.fin_tab) a.full_in = a.fin_tab[b];
  if (a.fout_tab) a.full_out = a.fout_tab[b];
  if (a.seeds) a.seed = a.seeds[b];
}

// A kernel's first batch of loads (the CG state, the previous pass's
// partials, the row offsets) is issued before it branches on any of them, so
// that the batch costs one memory round trip instead of one per dependent
// read.  issue_fence() keeps the loads above it in program order (no pass
// may sink them below the branch that follows).
__device__ __forceinline__ void issue_fence() { asm volatile("" ::: "memory"); }

// The fields of a problem's CG state that the kernels read, in registers
// (null state: idle, not done).  Indexing by parity goes through selects so
// that nothing of it lives in memory.
struct CGView {
  double rho0, rho1, alph0, alph1, tol2;
  int done, iter, max_iter, cap;
  __device__ __forceinline__ double rho(int p) const { return p ? rho1 : rho0; }
  __device__ __forceinline__ double alph(int p) const { return p ? alph1 : alph0; }
};
// A per-lane zero that the compiler cannot see through.  A uniform address
// plus it is read by the vector memory path, whose loads return in order with
// the kernel's other vector loads; a scalar-cache load would not do: those
// return out of order, so the first use of any scalar load (a kernel
// argument, say) waits for every one in flight, the state's included.
__device__ __forceinline__ int lane_zero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}

// The state a null pointer stands for: idle, not done (all zero).
static __device__ CGScalars g_idle_state;

// The done flag of a problem's CG state (null: 0), a vector load.
__device__ __forceinline__ int load_done(const CGScalars* sc) {
  return ((sc != nullptr ? sc : &g_idle_state) + lane_zero())->done;
}

// Unconditional vector loads (no branch whose join would wait for them).
__device__ __forceinline__ CGView load_scalars(const CGScalars* sc_in) {
  const CGScalars* sc = (sc_in != nullptr ? sc_in : &g_idle_state) + lane_zero();
  CGView v;
  v.rho0 = sc->rho[0];
  v.rho1 = sc->rho[1];
  v.alph0 = sc->alph[0];
  v.alph1 = sc->alph[1];
  v.tol2 = sc->tol2;
  v.done = sc->done;
  v.iter = sc->iter;
  v.max_iter = sc->max_iter;
  v.cap = sc->cap;
  return v;
}

// Per-thread sums of the previous pass's partials (red0, red1 and, for the
// single-reduction step, red2), four loads in flight per thread before the
// additions; the order of the additions is fixed.
template <int NR, int NT, typename T>
__device__ __forceinline__ void cg_partials(const RowArgs<T>& a, double& s0, double& s1, double& s2) {
  s0 = s1 = s2 = 0.0;
  const double* r[3] = {a.red0, a.red1, a.red2};
  int i = threadIdx.x;
  for (; i + 3 * NT < a.nred; i += 4 * NT) {
    double v[NR][4];
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) v[q][u] = r[q][i + u * NT];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s0 += v[0][u];
      if constexpr (NR > 1) s1 += v[1][u];
      if constexpr (NR > 2) s2 += v[2][u];
    }
  }
  for (; i < a.nred; i += NT) {
    s0 += r[0][i];
    if constexpr (NR > 1) s1 += r[1][i];
    if constexpr (NR > 2) s2 += r[2][i];
  }
}

// One CG scalar step, taken redundantly by every workgroup of the row pass
// that needs it: the previous pass's per-workgroup partial sums (s0, s1: this
// thread's share, cg_partials) are added in a fixed order, so every
// workgroup obtains the same bits; workgroup 0 alone persists the new state.
// cs is the state as the kernel found it (load_scalars).  Returns the
// coefficient (beta or alpha), or sets *stop when the solve ends here.
//   PUPDATE (start of an iteration): rz = r.z, rr = r.r from the previous
//     E E r pass; stop if rr <= tol2, if the cap was reached or rz <= 0;
//     beta = rz / rho[parity]; rho[parity^1] = rz.
//   XRUPDATE: pq = p.q from the A apply; stop if pq <= 0;
//     alpha = rho[parity^1] / pq; iter += 1.
// With a coefficient record (a.hist), workgroup 0 also stores alpha_j and
// beta_j of iteration j: the data of the Lanczos matrix of the solve.
template <int MODE, int NT, typename T>
__device__ __forceinline__ double cg_scalar_step(const RowArgs<T>& a, const CGView& cs, double s0, double s1,
                                                 bool* stop) {
  __shared__ double s_coef;
  __shared__ int s_stop;
  block_sum2<NT>(s0, s1);
  if (threadIdx.x == 0) {
    CGScalars* sc = a.sc;
    const bool w = (blockIdx.x == 0);
    int st = 0, stat = 0;
    double coef = 0.0;
    if constexpr (MODE == 1) {  // PUPDATE
      const double rz = s0, rr = s1;
      if (rr <= cs.tol2) st = 1;
      else if (cs.cap) { st = 1; stat = -4; }
      else if (!(rz > 0.0)) { st = 1; stat = -6; }
      coef = rz / cs.rho(a.parity);
      if (w) {
        sc->rr = rr;
        if (st) {
          sc->status = stat;
          sc->done = 1;
        } else {
          sc->rho[a.parity ^ 1] = rz;
          sc->beta = coef;
          const int j = cs.iter - 1;  // beta_j forms p_{j+1}
          if (a.hist && j >= 0 && j < a.hist_cap) a.hist[2 * j + 1] = coef;
        }
      }
    } else {  // XRUPDATE
      const double pq = s0;
      if (!(pq > 0.0)) { st = 1; stat = -6; }
      coef = cs.rho(a.parity ^ 1) / pq;
      if (w) {
        if (st) {
          sc->status = stat;
          sc->done = 1;
        } else {
          sc->alpha = coef;
          if (a.hist && cs.iter < a.hist_cap) a.hist[2 * cs.iter] = coef;
          sc->iter = cs.iter + 1;
          if (cs.iter + 1 >= cs.max_iter) sc->cap = 1;
        }
      }
    }
    s_coef = coef;
    s_stop = st;
  }
  __syncthreads();
  *stop = s_stop != 0;
  return s_coef;
}

// The scalar step of single-reduction CG (Chronopoulos and Gear): one pass of
// partial sums per iteration gives rho = r.z (red0), r.r (red1) and
// mu = w.z (red2), w = A z.  With p = z + beta p_{j-1}, A p_{j-1} =
// (r_{j-1} - r_j) / alpha_{j-1} and z.r_{j-1} = 0, p.Ap = mu - beta rho / alpha_{j-1}:
//   beta = rho / rho_{j-1},  alpha = rho / (mu - beta rho / alpha_{j-1}),
// the coefficients of the standard recurrence in exact arithmetic.  The first
// step sees rho_{-1} = 1, alpha_{-1} = inf (so alpha = rho / mu) and p = s = 0.
// Stops as the standard step does (rr <= tol2, the cap, rho or p.Ap not > 0);
// workgroup 0 persists rho and alpha by parity, the record and the count.
template <int NT, typename T>
__device__ __forceinline__ void cg1_scalar_step(const RowArgs<T>& a, const CGView& cs, double s0, double s1,
                                                double s2, bool* stop, double* beta, double* alpha) {
  __shared__ double s_ab[2];
  __shared__ int s_stop;
  double unused = 0.0;
  block_sum2<NT>(s0, s1);
  __syncthreads();
  block_sum2<NT>(s2, unused);
  if (threadIdx.x == 0) {
    CGScalars* sc = a.sc;
    const double rz = s0, rr = s1, mu = s2;
    int st = 0, stat = 0;
    const double b = rz / cs.rho(a.parity);
    const double pap = mu - b * rz / cs.alph(a.parity);
    if (rr <= cs.tol2) st = 1;
    else if (cs.cap) { st = 1; stat = -4; }
    else if (!(rz > 0.0) || !(pap > 0.0)) { st = 1; stat = -6; }
    const double al = rz / pap;
    if (blockIdx.x == 0) {
      sc->rr = rr;
      if (st) {
        sc->status = stat;
        sc->done = 1;
      } else {
        const int j = cs.iter;
        sc->rho[a.parity ^ 1] = rz;
        sc->alph[a.parity ^ 1] = al;
        sc->beta = b;
        sc->alpha = al;
        if (a.hist && j < a.hist_cap) a.hist[2 * j] = al;
        if (a.hist && j >= 1 && j - 1 < a.hist_cap) a.hist[2 * (j - 1) + 1] = b;  // beta_{j-1} forms p_j
        sc->iter = j + 1;
        if (j + 1 >= cs.max_iter) sc->cap = 1;
      }
    }
    s_ab[0] = b;
    s_ab[1] = al;
    s_stop = st;
  }
  __syncthreads();
  *stop = s_stop != 0;
  *beta = s_ab[0];
  *alpha = s_ab[1];
}

// Twiddle table of plan PL held in registers between its loads and its LDS
// stores, so that the loads share a round trip with the data loads issued
// after them (the counter of outstanding loads is in order).
template <typename PL, typename C, int NT> struct TwPrefetch {
  static constexpr int TW = tw_elems<PL>();
  static constexpr int TWP = (TW + NT - 1) / NT;
  C wv[TWP > 0 ? TWP : 1];
  __device__ __forceinline__ void load(const C* tw, int t) {
#pragma unroll
    for (int u = 0; u < TWP; ++u) {
      const int i = t + u * NT;
      if (i < TW) wv[u] = tw[i];
    }
  }
  __device__ __forceinline__ void store(C* twq, int t) const {
#pragma unroll
    for (int u = 0; u < TWP; ++u) {
      const int i = t + u * NT;
      if (i < TW) twq[i] = wv[u];
    }
  }
};

// The ROWS x NH block of the transposed spectrum that one row block owns
// (rows y0.., columns 0..NH-1: column kx at Xt[kx*ldx + y0 .. + ROWS-1]) into
// LDS rows of stride HS.  Every thread holds exactly ROWS*NH/NT loads in
// flight before any LDS store, instead of one round trip per element.
// The twiddle table of plan PL is staged into twq in the same batch of loads.
// Largest divisor of n that is at most m (m >= 1).
constexpr int divisor_at_most(int n, int m) {
  for (int c = m < n ? m : n; c > 1; --c)
    if (n % c == 0) return c;
  return 1;
}

// At most MAXB bytes of loads in flight per thread (a budget on the staging
// registers; more would spill in the register-heavy FP64 kernels).
template <typename C, typename PL, int ROWS, int NH, int NT, int HS, int MAXB = 128>
__device__ __forceinline__ void transposed_read(C* lds, const C* Xt, size_t ldx, int y0, int t, C* twq,
                                                const C* tw) {
  static_assert((ROWS * NH) % NT == 0, "transposed tiling");
  constexpr int PER = ROWS * NH / NT;
  constexpr int CH = divisor_at_most(PER, MAXB / (int)sizeof(C) > 0 ? MAXB / (int)sizeof(C) : 1);
  // FP32: the twiddle loads join the first batch; FP64: staged before it
  // (no registers to spare)
  constexpr bool PRE = sizeof(C) == 8;
  TwPrefetch<PL, C, NT> twp;
  if constexpr (PRE) twp.load(tw, t);
  else tw_stage<PL>(twq, tw, t, NT);
#pragma unroll
  for (int ch = 0; ch < PER; ch += CH) {
    C tv[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int o = t + (ch + u) * NT;
      tv[u] = Xt[(size_t)(o / ROWS) * ldx + y0 + (o % ROWS)];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int o = t + (ch + u) * NT;
      lds[(o % ROWS) * HS + o / ROWS] = tv[u];
    }
  }
  if constexpr (PRE) twp.store(twq, t);
}

template <int MODE> constexpr bool r2c_is_compact() { return MODE <= R2C_XRUPDATE || MODE == R2C_CG1UPDATE; }
template <int MODE> constexpr bool c2r_is_compact() { return MODE <= C2R_RESID; }

// ---------------------------------------------------------------------------
// r2c
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ __launch_bounds__((RowCfg<T, N>::THREADS)) void r2c_kernel(RowArgs<T> a_in) {
  using C = cplx<T>;
  RowArgs<T> a = bind_problem(a_in);
  bind_caller(a);
  using CF = RowCfg<T, N>;
  using PL = typename CF::PL;
  constexpr int E = CF::E, TPL = CF::TPL, ROWS = CF::ROWS, NT = CF::THREADS, H = CF::H;
  constexpr int LE = lds_line_elems<PL>();
  constexpr int LDS_C = (CF::LINES * LE > (ROWS * N) / 2) ? CF::LINES * LE : (ROWS * N) / 2;
  __shared__ C lds[LDS_C];
  __shared__ C twq[tw_elems<PL>() > 0 ? tw_elems<PL>() : 1];
  T* ldr = reinterpret_cast<T*>(lds);

  const int blk = xcd_remap<CF::XG>(blockIdx.x, gridDim.x);
  const int y0 = blk * ROWS;
  if (y0 >= a.ny) return;  // past a band run's rows
  const int t = threadIdx.x;
  const int l = t / TPL, tid = t % TPL;
  const size_t ldx = (size_t)a.ldx;
  C v[E];

  constexpr bool CG1 = MODE == R2C_CG1UPDATE;
  // Band runs (a.runs): rows past a run's end (its padding to a multiple of
  // 32) get an exact zero spectrum.  The two-rows-per-line transform leaves
  // there the rounding residue of the partner row's separation, which the
  // banded solve would carry into M^-1 r.
  __shared__ unsigned char s_empty[ROWS];
  if constexpr (r2c_is_compact<MODE>()) {
    if (a.runs != nullptr && t < ROWS) s_empty[t] = a.row_off[y0 + t + 1] == a.row_off[y0 + t];
  }
  // first batch of loads: the row offsets, the state, the partials
  int c0 = 0, c1 = 0;
  if constexpr (r2c_is_compact<MODE>()) {
    c0 = a.row_off[y0];
    c1 = a.row_off[y0 + ROWS];
  }
  const CGView cs = load_scalars(a.sc);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if constexpr (MODE == R2C_PUPDATE) cg_partials<2, NT>(a, s0, s1, s2);
  else if constexpr (MODE == R2C_XRUPDATE) cg_partials<1, NT>(a, s0, s1, s2);
  else if constexpr (CG1) cg_partials<3, NT>(a, s0, s1, s2);
  issue_fence();
  if (__builtin_amdgcn_readfirstlane(cs.done)) return;

  double acc = 0.0;  // CG1: r.r of the new r
  if constexpr (r2c_is_compact<MODE>()) {
    T coef = T(0), coef2 = T(0);  // beta (PUPDATE, CG1) or alpha (XRUPDATE); CG1: alpha
    if constexpr (MODE == R2C_PUPDATE || MODE == R2C_XRUPDATE) {
      bool stop = false;
      coef = (T)cg_scalar_step<MODE, NT>(a, cs, s0, s1, &stop);
      if (stop) return;
    } else if constexpr (CG1) {
      bool stop = false;
      double b = 0.0, al = 0.0;
      cg1_scalar_step<NT>(a, cs, s0, s1, s2, &stop, &b, &al);
      if (stop) return;
      coef = (T)b;
      coef2 = (T)al;
    }
    if (c0 == c1) {  // no masked pixel in these rows: the spectrum is zero
      for (int o = t; o < ROWS * (N / 2); o += NT) a.Xt[(size_t)(o / ROWS) * ldx + y0 + (o % ROWS)] = C{T(0), T(0)};
      if (CG1 && t == 0 && a.part0) a.part0[blk] = 0.0;
      return;
    }
    // FP32: twiddle loads share the data loads' round trip; FP64 has no
    // registers to spare for them
    TwPrefetch<PL, C, NT> twp;
    if constexpr (sizeof(T) == 4) twp.load(a.tw, t);
    else tw_stage<PL>(twq, a.tw, t, NT);
    const int base = y0 * a.nx;
    if (c1 - c0 == ROWS * N) {
      // Every pixel of these rows is masked (a band): compact element c0 + i
      // is pixel i of the block, so no index loads and no zero fill.
      constexpr int PER = ROWS * N / NT;
      constexpr int FB = CG1 ? (sizeof(T) == 4 ? 8 : 4) : (sizeof(T) == 4 ? 16 : 8);
      static_assert(PER % FB == 0, "chunking");
#pragma unroll 1
      for (int ch = 0; ch < PER; ch += FB) {
        T val[FB], xv[FB], pv[FB], sv[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) {
          const int c = c0 + t + (ch + u) * NT;
          if constexpr (MODE == R2C_COMPACT) {
            val[u] = a.v0[c];
          } else if constexpr (MODE == R2C_PUPDATE) {
            val[u] = a.v0[c] + coef * a.v1[c];
          } else if constexpr (CG1) {
            const T r = a.v1[c];
            pv[u] = (a.v4 ? a.v4[c] : r) + coef * a.v2[c];
            sv[u] = a.v5[c] + coef * a.v3[c];
            xv[u] = a.v0[c] + coef2 * pv[u];
            val[u] = r - coef2 * sv[u];
          } else {
            val[u] = a.v1[c] - coef * a.v3[c];
            xv[u] = a.v0[c] + coef * a.v2[c];
          }
        }
#pragma unroll
        for (int u = 0; u < FB; ++u) {
          const int i = t + (ch + u) * NT, c = c0 + i;
          if constexpr (MODE == R2C_PUPDATE) a.v1[c] = val[u];
          if constexpr (MODE == R2C_XRUPDATE || CG1) {
            a.v1[c] = val[u];
            a.v0[c] = xv[u];
          }
          if constexpr (CG1) {
            a.v2[c] = pv[u];
            a.v3[c] = sv[u];
            acc += (double)val[u] * (double)val[u];
          }
          ldr[i] = val[u];
        }
      }
      __syncthreads();
    } else {
    for (int i = t; i < ROWS * N; i += NT) ldr[i] = T(0);
    __syncthreads();
    constexpr int KB = CG1 ? 4 : kBatch;
    for (int cb = c0 + t; cb < c1; cb += NT * KB) {
      int pp[KB];
      T val[KB], xv[KB], pv[KB], sv[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int c = cb + u * NT;
        if (c < c1) {
          pp[u] = a.pos[c];
          if constexpr (MODE == R2C_COMPACT) {
            val[u] = a.v0[c];
          } else if constexpr (MODE == R2C_PUPDATE) {
            val[u] = a.v0[c] + coef * a.v1[c];
          } else if constexpr (CG1) {
            const T r = a.v1[c];
            pv[u] = (a.v4 ? a.v4[c] : r) + coef * a.v2[c];
            sv[u] = a.v5[c] + coef * a.v3[c];
            xv[u] = a.v0[c] + coef2 * pv[u];
            val[u] = r - coef2 * sv[u];
          } else {
            val[u] = a.v1[c] - coef * a.v3[c];
            xv[u] = a.v0[c] + coef * a.v2[c];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int c = cb + u * NT;
        if (c < c1) {
          if constexpr (MODE == R2C_PUPDATE) a.v1[c] = val[u];
          if constexpr (MODE == R2C_XRUPDATE || CG1) {
            a.v1[c] = val[u];
            a.v0[c] = xv[u];
          }
          if constexpr (CG1) {
            a.v2[c] = pv[u];
            a.v3[c] = sv[u];
            acc += (double)val[u] * (double)val[u];
          }
          ldr[pp[u] - base] = val[u];
        }
      }
    }
    __syncthreads();
    }
    if constexpr (sizeof(T) == 4) twp.store(twq, t);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = tid + e * TPL;
      v[e] = C{ldr[(2 * l) * N + x], ldr[(2 * l + 1) * N + x]};
    }
    __syncthreads();
  } else if constexpr (MODE == R2C_FULL) {
    const size_t ra = (size_t)(y0 + 2 * l) * a.nx, rb = ra + a.nx;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = tid + e * TPL;
      v[e] = C{(T)a.full_in[ra + x], (T)a.full_in[rb + x]};
    }
    tw_stage<PL>(twq, a.tw, t, NT);  // after the row loads: one round trip for both
  } else {
    // white noise: pixels 4j .. 4j+3 share one Philox block (two Box-Muller
    // pairs), so each thread draws whole blocks of the row block into LDS,
    // then takes its elements
    static_assert((ROWS * N) % 4 == 0, "noise blocks of four pixels");
    const uint64_t blk0 = ((uint64_t)y0 * a.nx) >> 2;  // rows of 4k pixels start a block
    for (int j = t; j < ROWS * N / 4; j += NT) {
      const u64x4 w = philox4x64_10(blk0 + j, 0, 0, 0, a.seed, a.stream);
      double n0, n1, n2, n3;
      box_muller2(w.w0, w.w1, &n0, &n1);
      box_muller2(w.w2, w.w3, &n2, &n3);
      ldr[4 * j] = (T)n0;
      ldr[4 * j + 1] = (T)n1;
      ldr[4 * j + 2] = (T)n2;
      ldr[4 * j + 3] = (T)n3;
    }
    tw_stage<PL>(twq, a.tw, t, NT);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = tid + e * TPL;
      v[e] = C{ldr[(2 * l) * N + x], ldr[(2 * l + 1) * N + x]};
    }
    __syncthreads();  // the FFT reuses the LDS
  }

  C* line = lds + l * LE;
  fft_line<C, PL, -1>(v, tid, line, twq);
#pragma unroll
  for (int e = 0; e < E; ++e) line[lpad<PL>(tid + e * TPL)] = v[e];
  __syncthreads();
  // Separate the two packed rows: A_k = (Z_k + conj Z_-k)/2, B_k = (Z_k - conj Z_-k)/(2i).
  // The real DC and Nyquist bins of a row share column 0: (A_0, A_{N/2}).
  static_assert((ROWS * (N / 2)) % NT == 0, "transposed tiling");
  constexpr int WU = sizeof(T) == 4 ? ROWS * (N / 2) / NT : 1;  // FP64: registers are short
#pragma unroll WU
  for (int u = 0; u < ROWS * (N / 2) / NT; ++u) {
    const int o = t + u * NT;
    const int kx = o / ROWS, r = o % ROWS;
    const C* ln = lds + (r >> 1) * LE;
    C out;
    if (kx == 0) {
      const C z0 = ln[lpad<PL>(0)], zh = ln[lpad<PL>(N / 2)];
      out = (r & 1) ? C{z0.y, zh.y} : C{z0.x, zh.x};
    } else {
      const C zk = ln[lpad<PL>(kx)];
      const C zm = ln[lpad<PL>(N - kx)];
      if (r & 1) out = C{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
      else out = C{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
    }
    if constexpr (r2c_is_compact<MODE>()) {
      if (a.runs != nullptr && s_empty[r]) out = C{T(0), T(0)};
    }
    a.Xt[(size_t)kx * ldx + y0 + r] = out;
  }
  if constexpr (CG1) {
    if (a.part0) {
      double unused = 0.0;
      block_sum2<NT>(acc, unused);
      if (t == 0) a.part0[blk] = acc;
    }
  }
}

// The compact output of a c2r-type pass (modes C2R_COMPACT, C2R_DOT2,
// C2R_RESID): the ROWS x N block of real rows is in LDS (ldr); compact
// elements c0..c1-1 (pixels pos[c]) are written to v0 with the mode's FP64
// partial sums into part0/part1 at slot blk.
template <int MODE, int N, int ROWS, int NT, typename T>
__device__ __forceinline__ void compact_out(const RowArgs<T>& a, const T* ldr, int y0, int c0, int c1, int t,
                                            int blk) {
  const int base = y0 * a.nx;
  double acc0 = 0.0, acc1 = 0.0;
  const bool dot_self = (a.v1 == nullptr);
  if (c1 - c0 == ROWS * N) {
    // fully masked rows: compact element c0 + i is pixel i of the block
    constexpr int PER = ROWS * N / NT, FB = sizeof(T) == 4 ? 16 : 8;
#pragma unroll 1
    for (int ch = 0; ch < PER; ch += FB) {
      T w[FB];
#pragma unroll
      for (int u = 0; u < FB; ++u) w[u] = dot_self ? T(0) : a.v1[c0 + t + (ch + u) * NT];
#pragma unroll
      for (int u = 0; u < FB; ++u) {
        const int i = t + (ch + u) * NT, c = c0 + i;
        const T val = ldr[i];
        if constexpr (MODE == C2R_COMPACT) {
          const T o = a.scale * val;
          a.v0[c] = o;
          acc0 += (double)o * (double)(dot_self ? o : w[u]);
        } else if constexpr (MODE == C2R_DOT2) {
          a.v0[c] = val;
          const double r = (double)w[u];
          acc0 += r * (double)val;
          acc1 += r * r;
        } else {
          const T r = w[u] - val;
          a.v0[c] = r;
          acc0 += (double)r * (double)r;
        }
      }
    }
  } else
  for (int cb = c0 + t; cb < c1; cb += NT * kBatch) {
    int pp[kBatch];
    T w[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int c = cb + u * NT;
      if (c < c1) {
        pp[u] = a.pos[c];
        w[u] = dot_self ? T(0) : a.v1[c];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int c = cb + u * NT;
      if (c < c1) {
        const T val = ldr[pp[u] - base];
        if constexpr (MODE == C2R_COMPACT) {
          const T o = a.scale * val;
          a.v0[c] = o;
          acc0 += (double)o * (double)(dot_self ? o : w[u]);
        } else if constexpr (MODE == C2R_DOT2) {
          a.v0[c] = val;
          const double r = (double)w[u];
          acc0 += r * (double)val;
          acc1 += r * r;
        } else {
          const T r = w[u] - val;
          a.v0[c] = r;
          acc0 += (double)r * (double)r;
        }
      }
    }
  }
  if (a.part0) {
    block_sum2<NT>(acc0, acc1);
    if (t == 0) {
      a.part0[blk] = acc0;
      if (a.part1) a.part1[blk] = acc1;
    }
  }
}

// ---------------------------------------------------------------------------
// c2r
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ __launch_bounds__((RowCfg<T, N>::THREADS)) void c2r_kernel(RowArgs<T> a_in) {
  using C = cplx<T>;
  RowArgs<T> a = bind_problem(a_in);
  bind_caller(a);
  using CF = RowCfg<T, N>;
  using PL = typename CF::PL;
  constexpr int E = CF::E, TPL = CF::TPL, ROWS = CF::ROWS, NT = CF::THREADS, H = CF::H;
  constexpr int LE = lds_line_elems<PL>();
  constexpr int HS = CF::HS;
  constexpr int LDS_C = (CF::LINES * LE > ROWS * HS) ? CF::LINES * LE : ROWS * HS;
  __shared__ C lds[LDS_C];
  __shared__ C twq[tw_elems<PL>() > 0 ? tw_elems<PL>() : 1];
  T* ldr = reinterpret_cast<T*>(lds);

  const int blk = xcd_remap<CF::XG>(blockIdx.x, gridDim.x);
  const int y0 = blk * ROWS;
  if (y0 >= a.ny) return;  // past a band run's rows
  const int t = threadIdx.x;
  const int l = t / TPL, tid = t % TPL;
  const size_t ldx = (size_t)a.ldx;
  int c0 = 0, c1 = 0;
  if constexpr (c2r_is_compact<MODE>()) {
    c0 = a.row_off[y0];
    c1 = a.row_off[y0 + ROWS];
  }
  const int done = load_done(a.sc);
  issue_fence();  // the state and the row offsets in one round trip
  if (__builtin_amdgcn_readfirstlane(done)) return;
  if constexpr (c2r_is_compact<MODE>()) {
    if (c0 == c1) {  // nothing to write; partial sums are zero
      if (t == 0) {
        if (a.part0) a.part0[blk] = 0.0;
        if (a.part1) a.part1[blk] = 0.0;
      }
      return;
    }
  }
  transposed_read<C, PL, ROWS, N / 2, NT, HS>(lds, a.Xt, ldx, y0, t, twq, a.tw);
  __syncthreads();
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = tid + e * TPL;
    C A, B;
    if (k == 0 || k == N / 2) {  // real DC / Nyquist bins, packed in column 0
      const C p0 = lds[(2 * l) * HS], q0 = lds[(2 * l + 1) * HS];
      A = C{k == 0 ? p0.x : p0.y, T(0)};
      B = C{k == 0 ? q0.x : q0.y, T(0)};
    } else if (k < N / 2) {
      A = lds[(2 * l) * HS + k];
      B = lds[(2 * l + 1) * HS + k];
    } else {
      const C a0 = lds[(2 * l) * HS + (N - k)], b0 = lds[(2 * l + 1) * HS + (N - k)];
      A = C{a0.x, -a0.y};
      B = C{b0.x, -b0.y};
    }
    v[e] = C{A.x - B.y, A.y + B.x};  // Z = A + iB
  }
  __syncthreads();
  C* line = lds + l * LE;
  fft_line<C, PL, +1>(v, tid, line, twq);

  if constexpr (c2r_is_compact<MODE>()) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = tid + e * TPL;
      ldr[(2 * l) * N + x] = v[e].x;
      ldr[(2 * l + 1) * N + x] = v[e].y;
    }
    __syncthreads();
    compact_out<MODE, N, ROWS, NT>(a, ldr, y0, c0, c1, t, blk);
  } else {
    const size_t ra = (size_t)(y0 + 2 * l) * a.nx, rb = ra + a.nx;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = tid + e * TPL;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const size_t pix = (h ? rb : ra) + x;
        const double s = (double)(h ? v[e].y : v[e].x);
        if constexpr (MODE == C2R_REALIZE) {
          if (a.full_in) {
            const bool m = a.mask[pix] != 0;
            const double d = a.full_in[pix];
            a.full_out[pix] = m ? s : d;
            a.full_out2[pix] = m ? 0.0 : d - s;
          } else {
            a.full_out[pix] = s;
          }
        } else {
          a.full_out[pix] = (double)a.scale * s;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// proj: the row pass between two column passes: inverse real FFT along x,
// projection Px (masked pixels kept, observed ones zeroed), forward real FFT
// along x, transposed half spectrum written back.  The projected map never
// leaves the chip.  Between the two applies of C^{1/2} in E E r (Sec. 2.4)
// it is the whole row pass; with DOT it also writes the masked values to v0
// in compact order with the partials of v1.v0 and v1.v1 (C2R_DOT2): in
// single-reduction CG it ends z = M^-1 r and starts w = A z in one pass.
// ---------------------------------------------------------------------------
template <typename T, int N, bool DOT>
__global__ __launch_bounds__((RowCfg<T, N>::THREADS)) void proj_kernel(RowArgs<T> a_in) {
  using C = cplx<T>;
  RowArgs<T> a = bind_problem(a_in);
  bind_caller(a);
  using CF = RowCfg<T, N>;
  using PL = typename CF::PL;
  constexpr int E = CF::E, TPL = CF::TPL, ROWS = CF::ROWS, NT = CF::THREADS;
  constexpr int LE = lds_line_elems<PL>();
  constexpr int HS = CF::HS;
  constexpr int LDS_C = (CF::LINES * LE > ROWS * HS) ? CF::LINES * LE : ROWS * HS;
  __shared__ C lds[LDS_C];
  __shared__ C twq[tw_elems<PL>() > 0 ? tw_elems<PL>() : 1];
  T* ldr = reinterpret_cast<T*>(lds);

  const int blk = xcd_remap<CF::XG>(blockIdx.x, gridDim.x);
  const int y0 = blk * ROWS;
  const int t = threadIdx.x;
  const int l = t / TPL, tid = t % TPL;
  const size_t ldx = (size_t)a.ldx;
  const int c0 = a.row_off[y0], c1 = a.row_off[y0 + ROWS];
  const int done = load_done(a.sc);
  issue_fence();  // the state and the row offsets in one round trip
  if (__builtin_amdgcn_readfirstlane(done)) return;
  if (c0 == c1) {  // no masked pixel: the projection is zero
    for (int o = t; o < ROWS * (N / 2); o += NT) a.Xt[(size_t)(o / ROWS) * ldx + y0 + (o % ROWS)] = C{T(0), T(0)};
    if (DOT && t == 0) {
      if (a.part0) a.part0[blk] = 0.0;
      if (a.part1) a.part1[blk] = 0.0;
    }
    return;
  }
  const size_t ra = (size_t)(y0 + 2 * l) * a.nx, rb = ra + a.nx;
  uint8_t ma[E], mb[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    ma[e] = a.mask[ra + tid + e * TPL];
    mb[e] = a.mask[rb + tid + e * TPL];
  }
  transposed_read<C, PL, ROWS, N / 2, NT, HS, (sizeof(T) == 8 ? 32 : 128)>(lds, a.Xt, ldx, y0, t, twq, a.tw);
  __syncthreads();
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = tid + e * TPL;
    C A, B;
    if (k == 0 || k == N / 2) {
      const C p0 = lds[(2 * l) * HS], q0 = lds[(2 * l + 1) * HS];
      A = C{k == 0 ? p0.x : p0.y, T(0)};
      B = C{k == 0 ? q0.x : q0.y, T(0)};
    } else if (k < N / 2) {
      A = lds[(2 * l) * HS + k];
      B = lds[(2 * l + 1) * HS + k];
    } else {
      const C a0 = lds[(2 * l) * HS + (N - k)], b0 = lds[(2 * l + 1) * HS + (N - k)];
      A = C{a0.x, -a0.y};
      B = C{b0.x, -b0.y};
    }
    v[e] = C{A.x - B.y, A.y + B.x};
  }
  __syncthreads();
  C* line = lds + l * LE;
  fft_line<C, PL, +1>(v, tid, line, twq);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = C{ma[e] ? v[e].x : T(0), mb[e] ? v[e].y : T(0)};
  if constexpr (DOT) {
    __syncthreads();  // every line's FFT is done with LDS
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = tid + e * TPL;
      ldr[(2 * l) * N + x] = v[e].x;
      ldr[(2 * l + 1) * N + x] = v[e].y;
    }
    __syncthreads();
    compact_out<C2R_DOT2, N, ROWS, NT>(a, ldr, y0, c0, c1, t, blk);
    __syncthreads();  // the gather is done with LDS before the forward FFT
  }
  fft_line<C, PL, -1>(v, tid, line, twq);
#pragma unroll
  for (int e = 0; e < E; ++e) line[lpad<PL>(tid + e * TPL)] = v[e];
  __syncthreads();
  static_assert((ROWS * (N / 2)) % NT == 0, "transposed tiling");
  constexpr int WU = sizeof(T) == 4 ? ROWS * (N / 2) / NT : 1;  // FP64: registers are short
#pragma unroll WU
  for (int u = 0; u < ROWS * (N / 2) / NT; ++u) {
    const int o = t + u * NT;
    const int kx = o / ROWS, r = o % ROWS;
    const C* ln = lds + (r >> 1) * LE;
    C out;
    if (kx == 0) {
      const C z0 = ln[lpad<PL>(0)], zh = ln[lpad<PL>(N / 2)];
      out = (r & 1) ? C{z0.y, zh.y} : C{z0.x, zh.x};
    } else {
      const C zk = ln[lpad<PL>(kx)];
      const C zm = ln[lpad<PL>(N - kx)];
      if (r & 1) out = C{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
      else out = C{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
    }
    a.Xt[(size_t)kx * ldx + y0 + r] = out;
  }
}

// ---------------------------------------------------------------------------
// column pass: forward FFT along y, multiply by D, inverse FFT along y
// ---------------------------------------------------------------------------
// SKEW: the non-Hermitian study's variant (a.skew != 0); the solver's
// kernel is instantiated without it.
template <typename T, int N, bool SKEW>
__global__ __launch_bounds__((ColCfg<T, N>::THREADS)) void col_kernel(ColArgs<T> a_in) {
  using C = cplx<T>;
  using CF = ColCfg<T, N>;
  using PL = typename CF::PL;
  constexpr int E = CF::E, TPL = CF::TPL, W = CF::W;
  constexpr int LE = lds_line_elems<PL>();
  __shared__ C lds[W * LE];
  __shared__ C twq[tw_elems<PL>() > 0 ? tw_elems<PL>() : 1];
  ColArgs<T> a = a_in;
  a.Xt += (size_t)blockIdx.y * a.xt_stride;
  a.D += (size_t)blockIdx.y * a.d_stride;
  if (a.sc) a.sc += blockIdx.y;
  const int done = load_done(a.sc);
  const int l = threadIdx.x / TPL, tid = threadIdx.x % TPL;
  const int kx = blockIdx.x * W + l;
  const bool valid = kx < a.ncol;
  C* g = a.Xt + (size_t)(valid ? kx : 0) * a.ldx;
  const T* d = a.D + (size_t)(valid ? kx : 0) * a.ldx;
  C v[E];
  T dv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = valid ? g[tid + e * TPL] : C{T(0), T(0)};
    dv[e] = valid ? d[tid + e * TPL] : T(0);
  }
  tw_stage<PL>(twq, a.tw, threadIdx.x, CF::THREADS);
  issue_fence();  // the state and the column in one round trip
  if (__builtin_amdgcn_readfirstlane(done)) return;
  C* line = lds + l * LE;
  fft_line<C, PL, -1>(v, tid, line, twq);
  if (blockIdx.x == 0) {
    // Column 0 carries two real sequences, DC (real part) and Nyquist
    // (imaginary part) of every row: Z = U + iV.  Separate them in frequency,
    // U_k = (Z_k + conj Z_-k)/2, V_k = (Z_k - conj Z_-k)/(2i), apply each its
    // own table column, and recombine Z' = U' + i V'.
    T dn[E];
    const T* dnyq = a.D + (size_t)a.ncol * a.ldx;
#pragma unroll
    for (int e = 0; e < E; ++e) dn[e] = (l == 0) ? dnyq[tid + e * TPL] : T(0);
#pragma unroll
    for (int e = 0; e < E; ++e) line[lpad<PL>(tid + e * TPL)] = v[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int ky = tid + e * TPL;
      if (l == 0) {
        const C zk = v[e], zm = line[lpad<PL>(ky == 0 ? 0 : N - ky)];
        const C u{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
        const C w{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
        const C u2{u.x * dv[e], u.y * dv[e]}, w2{w.x * dn[e], w.y * dn[e]};
        v[e] = C{u2.x - w2.y, u2.y + w2.x};
      } else {
        v[e].x *= dv[e];
        v[e].y *= dv[e];
      }
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e].x *= dv[e];
      v[e].y *= dv[e];
    }
  }
  if (SKEW && kx > 0) {
    // column kx > 0: multiply by 1 + i f, f = eps sin(pi kx / ncol) (f = 0 on
    // the packed DC/Nyquist column), an antisymmetric real-space perturbation
    const T f = (T)(a.skew * sin(3.14159265358979323846 * (double)kx / (double)a.ncol));
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = C{v[e].x - f * v[e].y, v[e].y + f * v[e].x};
  }
  fft_line<C, PL, +1>(v, tid, line, twq);
  if (valid) {
#pragma unroll
    for (int e = 0; e < E; ++e) g[tid + e * TPL] = v[e];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers (instantiated per precision)
// ---------------------------------------------------------------------------

// Launch with optional start/stop events timestamped by the dispatch itself
// (hipExtLaunchKernelGGL), so a timed launch adds no packets to the stream.
#define FILL_LAUNCH(kern, grid, block, s, ev0, ev1, ...)                                   \
  do {                                                                                     \
    if (ev0) hipExtLaunchKernelGGL(kern, grid, block, 0, s, ev0, ev1, 0, __VA_ARGS__);     \
    else hipLaunchKernelGGL(kern, grid, block, 0, s, __VA_ARGS__);                         \
  } while (0)

// ---------------------------------------------------------------------------
// Vector update of CG without a preconditioner (z = r)
// ---------------------------------------------------------------------------
// alpha = rho / (p.q) (partials in red0), x += alpha p, r -= alpha q, then the
// per-block partial sums of r.r into part0 and part1 (r.z = r.r), which the
// next p = r + beta p pass reads.  INIT only sums the current r.  Block b of
// grid.x covers the b-th of grid.x equal slices of the problem's compact
// range; there are as many as row blocks of the row passes, so both passes
// see the same number of partials.
constexpr int kXrThreads = 256;

template <typename T, bool INIT>
__global__ __launch_bounds__(kXrThreads) void xr_kernel(RowArgs<T> a_in, int rows) {
  RowArgs<T> a = bind_problem(a_in);
  // equal slices of the problem's compact range (row blocks would leave the
  // few workgroups on a band with nearly all the work)
  const int blk = blockIdx.x, nblk = gridDim.x;
  const long long nm = a.row_off[(size_t)nblk * rows];
  const CGView cs = load_scalars(a.sc);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if constexpr (!INIT) cg_partials<1, kXrThreads>(a, s0, s1, s2);
  issue_fence();  // the state, the range and the partials in one round trip
  if (__builtin_amdgcn_readfirstlane(cs.done)) return;
  T coef = T(0);
  if constexpr (!INIT) {
    bool stop = false;
    coef = (T)cg_scalar_step<R2C_XRUPDATE, kXrThreads>(a, cs, s0, s1, &stop);
    if (stop) return;
  }
  const int c0 = (int)(nm * blk / nblk), c1 = (int)(nm * (blk + 1) / nblk);
  double acc = 0.0, unused = 0.0;
  for (int c = c0 + (int)threadIdx.x; c < c1; c += kXrThreads) {
    T r;
    if constexpr (INIT) {
      r = a.v1[c];
    } else {
      r = a.v1[c] - coef * a.v3[c];
      a.v0[c] = a.v0[c] + coef * a.v2[c];
      a.v1[c] = r;
    }
    acc += (double)r * (double)r;
  }
  if (a.part0) {
    block_sum2<kXrThreads>(acc, unused);
    if (threadIdx.x == 0) {
      a.part0[blk] = acc;
      a.part1[blk] = acc;
    }
  }
}

template <typename T>
hipError_t launch_xr(bool init, const RowArgs<T>& a, int nblk, hipStream_t s) {
  if (nblk <= 0 || a.ny % nblk != 0) return hipErrorInvalidValue;
  const dim3 grid(nblk, a.nprob), block(kXrThreads);
  if (init) hipLaunchKernelGGL((xr_kernel<T, true>), grid, block, 0, s, a, a.ny / nblk);
  else hipLaunchKernelGGL((xr_kernel<T, false>), grid, block, 0, s, a, a.ny / nblk);
  return hipGetLastError();
}

template <typename T, int N, int MODE>
hipError_t launch_r2c_nm(const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  using CF = RowCfg<T, N>;
  FILL_LAUNCH((r2c_kernel<T, N, MODE>), dim3(a.ny / CF::ROWS, a.nprob), dim3(CF::THREADS), s, e0, e1, a);
  return hipGetLastError();
}
template <typename T, int N, int MODE>
hipError_t launch_c2r_nm(const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  using CF = RowCfg<T, N>;
  FILL_LAUNCH((c2r_kernel<T, N, MODE>), dim3(a.ny / CF::ROWS, a.nprob), dim3(CF::THREADS), s, e0, e1, a);
  return hipGetLastError();
}
template <typename T, int N>
hipError_t launch_proj_n(bool dot, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  using CF = RowCfg<T, N>;
  if (dot) FILL_LAUNCH((proj_kernel<T, N, true>), dim3(a.ny / CF::ROWS, a.nprob), dim3(CF::THREADS), s, e0, e1, a);
  else FILL_LAUNCH((proj_kernel<T, N, false>), dim3(a.ny / CF::ROWS, a.nprob), dim3(CF::THREADS), s, e0, e1, a);
  return hipGetLastError();
}
template <typename T, int N>
hipError_t launch_col_n(const ColArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  using CF = ColCfg<T, N>;
  if (a.skew != 0.0)
    FILL_LAUNCH((col_kernel<T, N, true>), dim3((a.ncol + CF::W - 1) / CF::W, a.nprob), dim3(CF::THREADS), s, e0, e1,
                a);
  else
    FILL_LAUNCH((col_kernel<T, N, false>), dim3((a.ncol + CF::W - 1) / CF::W, a.nprob), dim3(CF::THREADS), s, e0,
                e1, a);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_r2c_n(int mode, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (mode) {
    case R2C_COMPACT: return launch_r2c_nm<T, N, R2C_COMPACT>(a, s, e0, e1);
    case R2C_PUPDATE: return launch_r2c_nm<T, N, R2C_PUPDATE>(a, s, e0, e1);
    case R2C_XRUPDATE: return launch_r2c_nm<T, N, R2C_XRUPDATE>(a, s, e0, e1);
    case R2C_FULL: return launch_r2c_nm<T, N, R2C_FULL>(a, s, e0, e1);
    case R2C_NOISE: return launch_r2c_nm<T, N, R2C_NOISE>(a, s, e0, e1);
    case R2C_CG1UPDATE: return launch_r2c_nm<T, N, R2C_CG1UPDATE>(a, s, e0, e1);
  }
  return hipErrorInvalidValue;
}
template <typename T, int N>
hipError_t launch_c2r_n(int mode, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (mode) {
    case C2R_COMPACT: return launch_c2r_nm<T, N, C2R_COMPACT>(a, s, e0, e1);
    case C2R_DOT2: return launch_c2r_nm<T, N, C2R_DOT2>(a, s, e0, e1);
    case C2R_RESID: return launch_c2r_nm<T, N, C2R_RESID>(a, s, e0, e1);
    case C2R_REALIZE: return launch_c2r_nm<T, N, C2R_REALIZE>(a, s, e0, e1);
    case C2R_FULL: return launch_c2r_nm<T, N, C2R_FULL>(a, s, e0, e1);
  }
  return hipErrorInvalidValue;
}

#define FILL_FOR_EACH_N(X) \
  X(16) X(32) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096)

template <typename T>
hipError_t launch_r2c(int mode, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  switch (a.nx) {
#define FILL_CASE(n) case n: return launch_r2c_n<T, n>(mode, a, s, e0, e1);
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t launch_c2r(int mode, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  switch (a.nx) {
#define FILL_CASE(n) case n: return launch_c2r_n<T, n>(mode, a, s, e0, e1);
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t launch_proj(bool dot, const RowArgs<T>& a, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr) {
  switch (a.nx) {
#define FILL_CASE(n) case n: return launch_proj_n<T, n>(dot, a, s, e0, e1);
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t launch_col(int ny, const ColArgs<T>& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  switch (ny) {
#define FILL_CASE(n) case n: return launch_col_n<T, n>(a, s, e0, e1);
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return hipErrorInvalidValue;
}
template <typename T> int row_block_rows(int nx) {
  switch (nx) {
#define FILL_CASE(n) case n: return RowCfg<T, n>::ROWS;
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return 0;
}

}  // namespace fillk
