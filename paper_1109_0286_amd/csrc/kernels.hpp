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

#include "fft_device.hpp"

namespace fillk {

// Scalars of one conjugate-gradient solve, resident on the device.
struct CGScalars {
  double rho;    // r.z
  double alpha;  // rho / (p.q)
  double beta;   // rho_new / rho_old
  double pq;
  double rr;     // r.r of the recursive residual
  double tol2;   // stop when rr <= tol2
  double spare0, spare1;
  int done;      // set when converged, failed or capped: every kernel then returns at once
  int iter;
  int max_iter;
  int status;    // 0 ok, -4 iteration cap, -6 p.q <= 0 or r.z <= 0
};

enum R2CMode {
  R2C_COMPACT = 0,   // input v0[c]
  R2C_PUPDATE = 1,   // p = z + beta p   (v0 = z, v1 = p), input p
  R2C_XRUPDATE = 2,  // x += alpha p, r -= alpha q (v0 = x, v1 = r, v2 = p, v3 = q), input r
  R2C_FULL = 3,      // input full map full_in (double)
  R2C_NOISE = 4      // input white noise of (seed, stream)
};

enum C2RMode {
  C2R_COMPACT = 0,   // v0[c] = scale*val; part0 += v0[c] * (v1 ? v1[c] : v0[c])
  C2R_DOT2 = 1,      // v0[c] = val; part0 += v1[c]*val, part1 += v1[c]^2
  C2R_RESID = 2,     // v0[c] = v1[c] - val; part0 += v0[c]^2
  C2R_REALIZE = 3,   // s = val; full_out = mask ? s : d, full_out2 = mask ? 0 : d - s (d = full_in)
  C2R_FULL = 4       // full_out = scale*val
};

template <typename T> struct RowArgs {
  int nx, ny, ldx;
  const int* row_off;
  const int* pos;
  cplx<T>* Xt;
  const cplx<T>* tw;
  T* v0;
  T* v1;
  T* v2;
  T* v3;
  T scale;
  const CGScalars* sc;
  double* part0;
  double* part1;
  const double* full_in;
  double* full_out;
  double* full_out2;
  const uint8_t* mask;
  uint64_t seed, stream;
};

template <typename T> struct ColArgs {
  cplx<T>* Xt;
  int ldx, ncol;
  const T* D;
  const cplx<T>* tw;
  const CGScalars* sc;
};

template <int MODE> constexpr bool r2c_is_compact() { return MODE <= R2C_XRUPDATE; }
template <int MODE> constexpr bool c2r_is_compact() { return MODE <= C2R_RESID; }

// ---------------------------------------------------------------------------
// r2c
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ __launch_bounds__((RowCfg<T, N>::THREADS)) void r2c_kernel(RowArgs<T> a) {
  using C = cplx<T>;
  using CF = RowCfg<T, N>;
  constexpr int E = CF::E, TPL = CF::TPL, ROWS = CF::ROWS, NT = CF::THREADS, H = CF::H;
  constexpr int LE = lds_line_elems<N>();
  constexpr int LDS_C = (CF::LINES * LE > (ROWS * N) / 2) ? CF::LINES * LE : (ROWS * N) / 2;
  __shared__ C lds[LDS_C];
  T* ldr = reinterpret_cast<T*>(lds);
  if (a.sc != nullptr && a.sc->done) return;

  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int y0 = blk * ROWS;
  const int t = threadIdx.x;
  const int l = t / TPL, tid = t % TPL;
  const size_t ldx = (size_t)a.ldx;
  C v[E];

  if constexpr (r2c_is_compact<MODE>()) {
    const int c0 = a.row_off[y0], c1 = a.row_off[y0 + ROWS];
    if (c0 == c1) {  // no masked pixel in these rows: the spectrum is zero
      for (int o = t; o < ROWS * H; o += NT) a.Xt[(size_t)(o / ROWS) * ldx + y0 + (o % ROWS)] = C{T(0), T(0)};
      return;
    }
    for (int i = t; i < ROWS * N; i += NT) ldr[i] = T(0);
    __syncthreads();
    T coef = T(0);
    if constexpr (MODE == R2C_PUPDATE) coef = (T)a.sc->beta;
    if constexpr (MODE == R2C_XRUPDATE) coef = (T)a.sc->alpha;
    const int base = y0 * a.nx;
    for (int c = c0 + t; c < c1; c += NT) {
      T val;
      if constexpr (MODE == R2C_COMPACT) {
        val = a.v0[c];
      } else if constexpr (MODE == R2C_PUPDATE) {
        val = a.v0[c] + coef * a.v1[c];
        a.v1[c] = val;
      } else {
        a.v0[c] = a.v0[c] + coef * a.v2[c];
        val = a.v1[c] - coef * a.v3[c];
        a.v1[c] = val;
      }
      ldr[a.pos[c] - base] = val;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = tid + e * TPL;
      v[e] = C{ldr[(2 * l) * N + x], ldr[(2 * l + 1) * N + x]};
    }
    __syncthreads();
  } else {
    const size_t ra = (size_t)(y0 + 2 * l) * a.nx, rb = ra + a.nx;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = tid + e * TPL;
      if constexpr (MODE == R2C_FULL) {
        v[e] = C{(T)a.full_in[ra + x], (T)a.full_in[rb + x]};
      } else {
        v[e] = C{(T)white_noise_at(ra + x, a.seed, a.stream), (T)white_noise_at(rb + x, a.seed, a.stream)};
      }
    }
  }

  C* line = lds + l * LE;
  fft_line<C, N, -1>(v, tid, line, a.tw);
#pragma unroll
  for (int e = 0; e < E; ++e) line[lpad(tid + e * TPL)] = v[e];
  __syncthreads();
  // Separate the two packed rows: A_k = (Z_k + conj Z_-k)/2, B_k = (Z_k - conj Z_-k)/(2i)
  for (int o = t; o < ROWS * H; o += NT) {
    const int kx = o / ROWS, r = o % ROWS;
    const C* ln = lds + (r >> 1) * LE;
    const C zk = ln[lpad(kx)];
    const C zm = ln[lpad(kx == 0 ? 0 : N - kx)];
    C out;
    if (r & 1) out = C{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
    else out = C{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
    a.Xt[(size_t)kx * ldx + y0 + r] = out;
  }
}

// ---------------------------------------------------------------------------
// c2r
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ __launch_bounds__((RowCfg<T, N>::THREADS)) void c2r_kernel(RowArgs<T> a) {
  using C = cplx<T>;
  using CF = RowCfg<T, N>;
  constexpr int E = CF::E, TPL = CF::TPL, ROWS = CF::ROWS, NT = CF::THREADS, H = CF::H;
  constexpr int LE = lds_line_elems<N>();
  constexpr int LDS_C = (CF::LINES * LE > ROWS * H) ? CF::LINES * LE : ROWS * H;
  __shared__ C lds[LDS_C];
  T* ldr = reinterpret_cast<T*>(lds);
  if (a.sc != nullptr && a.sc->done) return;

  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int y0 = blk * ROWS;
  const int t = threadIdx.x;
  const int l = t / TPL, tid = t % TPL;
  const size_t ldx = (size_t)a.ldx;
  int c0 = 0, c1 = 0;
  if constexpr (c2r_is_compact<MODE>()) {
    c0 = a.row_off[y0];
    c1 = a.row_off[y0 + ROWS];
    if (c0 == c1) {  // nothing to write; partial sums are zero
      if (t == 0) {
        if (a.part0) a.part0[blk] = 0.0;
        if (a.part1) a.part1[blk] = 0.0;
      }
      return;
    }
  }
  for (int o = t; o < ROWS * H; o += NT) {
    const int kx = o / ROWS, r = o % ROWS;
    lds[r * H + kx] = a.Xt[(size_t)kx * ldx + y0 + r];
  }
  __syncthreads();
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = tid + e * TPL;
    C A, B;
    if (k <= N / 2) {
      A = lds[(2 * l) * H + k];
      B = lds[(2 * l + 1) * H + k];
      if (k == 0 || k == N / 2) {  // real bins of a real row
        A.y = T(0);
        B.y = T(0);
      }
    } else {
      const C a0 = lds[(2 * l) * H + (N - k)], b0 = lds[(2 * l + 1) * H + (N - k)];
      A = C{a0.x, -a0.y};
      B = C{b0.x, -b0.y};
    }
    v[e] = C{A.x - B.y, A.y + B.x};  // Z = A + iB
  }
  __syncthreads();
  C* line = lds + l * LE;
  fft_line<C, N, +1>(v, tid, line, a.tw);

  if constexpr (c2r_is_compact<MODE>()) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = tid + e * TPL;
      ldr[(2 * l) * N + x] = v[e].x;
      ldr[(2 * l + 1) * N + x] = v[e].y;
    }
    __syncthreads();
    const int base = y0 * a.nx;
    double acc0 = 0.0, acc1 = 0.0;
    for (int c = c0 + t; c < c1; c += NT) {
      const T val = ldr[a.pos[c] - base];
      if constexpr (MODE == C2R_COMPACT) {
        const T o = a.scale * val;
        a.v0[c] = o;
        if (a.part0) acc0 += (double)o * (double)(a.v1 ? a.v1[c] : o);
      } else if constexpr (MODE == C2R_DOT2) {
        a.v0[c] = val;
        const double r = (double)a.v1[c];
        acc0 += r * (double)val;
        acc1 += r * r;
      } else {
        const T r = a.v1[c] - val;
        a.v0[c] = r;
        acc0 += (double)r * (double)r;
      }
    }
    if (a.part0) {
      block_sum2<NT>(acc0, acc1);
      if (t == 0) {
        a.part0[blk] = acc0;
        if (a.part1) a.part1[blk] = acc1;
      }
    }
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
// column pass: forward FFT along y, multiply by D, inverse FFT along y
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__((ColCfg<T, N>::THREADS)) void col_kernel(ColArgs<T> a) {
  using C = cplx<T>;
  using CF = ColCfg<T, N>;
  constexpr int E = CF::E, TPL = CF::TPL, W = CF::W;
  constexpr int LE = lds_line_elems<N>();
  __shared__ C lds[W * LE];
  if (a.sc != nullptr && a.sc->done) return;
  const int l = threadIdx.x / TPL, tid = threadIdx.x % TPL;
  const int kx = blockIdx.x * W + l;
  const bool valid = kx < a.ncol;
  C* g = a.Xt + (size_t)(valid ? kx : 0) * a.ldx;
  const T* d = a.D + (size_t)(valid ? kx : 0) * a.ldx;
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = valid ? g[tid + e * TPL] : C{T(0), T(0)};
  C* line = lds + l * LE;
  fft_line<C, N, -1>(v, tid, line, a.tw);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const T dv = valid ? d[tid + e * TPL] : T(0);
    v[e].x *= dv;
    v[e].y *= dv;
  }
  fft_line<C, N, +1>(v, tid, line, a.tw);
  if (valid) {
#pragma unroll
    for (int e = 0; e < E; ++e) g[tid + e * TPL] = v[e];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers (instantiated per precision)
// ---------------------------------------------------------------------------

template <typename T, int N, int MODE>
hipError_t launch_r2c_nm(const RowArgs<T>& a, hipStream_t s) {
  using CF = RowCfg<T, N>;
  hipLaunchKernelGGL((r2c_kernel<T, N, MODE>), dim3(a.ny / CF::ROWS), dim3(CF::THREADS), 0, s, a);
  return hipGetLastError();
}
template <typename T, int N, int MODE>
hipError_t launch_c2r_nm(const RowArgs<T>& a, hipStream_t s) {
  using CF = RowCfg<T, N>;
  hipLaunchKernelGGL((c2r_kernel<T, N, MODE>), dim3(a.ny / CF::ROWS), dim3(CF::THREADS), 0, s, a);
  return hipGetLastError();
}
template <typename T, int N>
hipError_t launch_col_n(const ColArgs<T>& a, hipStream_t s) {
  using CF = ColCfg<T, N>;
  hipLaunchKernelGGL((col_kernel<T, N>), dim3((a.ncol + CF::W - 1) / CF::W), dim3(CF::THREADS), 0, s, a);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_r2c_n(int mode, const RowArgs<T>& a, hipStream_t s) {
  switch (mode) {
    case R2C_COMPACT: return launch_r2c_nm<T, N, R2C_COMPACT>(a, s);
    case R2C_PUPDATE: return launch_r2c_nm<T, N, R2C_PUPDATE>(a, s);
    case R2C_XRUPDATE: return launch_r2c_nm<T, N, R2C_XRUPDATE>(a, s);
    case R2C_FULL: return launch_r2c_nm<T, N, R2C_FULL>(a, s);
    case R2C_NOISE: return launch_r2c_nm<T, N, R2C_NOISE>(a, s);
  }
  return hipErrorInvalidValue;
}
template <typename T, int N>
hipError_t launch_c2r_n(int mode, const RowArgs<T>& a, hipStream_t s) {
  switch (mode) {
    case C2R_COMPACT: return launch_c2r_nm<T, N, C2R_COMPACT>(a, s);
    case C2R_DOT2: return launch_c2r_nm<T, N, C2R_DOT2>(a, s);
    case C2R_RESID: return launch_c2r_nm<T, N, C2R_RESID>(a, s);
    case C2R_REALIZE: return launch_c2r_nm<T, N, C2R_REALIZE>(a, s);
    case C2R_FULL: return launch_c2r_nm<T, N, C2R_FULL>(a, s);
  }
  return hipErrorInvalidValue;
}

#define FILL_FOR_EACH_N(X) X(16) X(32) X(64) X(128) X(256) X(512) X(768) X(1024) X(2048) X(4096)

template <typename T> hipError_t launch_r2c(int mode, const RowArgs<T>& a, hipStream_t s) {
  switch (a.nx) {
#define FILL_CASE(n) case n: return launch_r2c_n<T, n>(mode, a, s);
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return hipErrorInvalidValue;
}
template <typename T> hipError_t launch_c2r(int mode, const RowArgs<T>& a, hipStream_t s) {
  switch (a.nx) {
#define FILL_CASE(n) case n: return launch_c2r_n<T, n>(mode, a, s);
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return hipErrorInvalidValue;
}
template <typename T> hipError_t launch_col(int ny, const ColArgs<T>& a, hipStream_t s) {
  switch (ny) {
#define FILL_CASE(n) case n: return launch_col_n<T, n>(a, s);
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
