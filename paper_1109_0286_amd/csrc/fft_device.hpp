// Device-side building blocks of the 2D real FFT used by every operator apply
// of the fill-in (Sec. 2.4: each apply of C^-1, C^{1/2} on the torus is a
// forward FFT, a diagonal multiply and an inverse FFT; the torus DFT is exactly
// unitary, Sec. 4).
//
// One "line" is a complex sequence of length N held across TPL = N/E threads,
// E elements per thread, thread tid holding elements tid + e*TPL (e < E).  A
// transform is a sequence of Stockham autosort passes of radix R (R | E): each
// thread runs E/R radix-R butterflies in registers on its own elements, and
// between passes the line is exchanged through LDS into the next pass's order.
// The first pass consumes, and the last pass produces, the natural strided
// order, so global loads/stores before and after a transform are coalesced and
// need no LDS round trip.  Forward transforms use exp(-2 pi i jk/N), inverse
// ones exp(+2 pi i jk/N), both unnormalised.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fillk {

template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using cplx = typename cvec<T>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }

// a * (DIR * i): DIR = -1 forward, +1 inverse
template <int DIR, typename C> __device__ __forceinline__ C mul_di(C a) {
  if constexpr (DIR < 0) return C{a.y, -a.x};
  else return C{-a.y, a.x};
}

// a * w (forward) or a * conj(w) (inverse), w from the table exp(-2 pi i t/N)
template <int DIR, typename C> __device__ __forceinline__ C twmul(C a, C w) {
  if constexpr (DIR < 0) return C{a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
  else return C{a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}

// ---------------------------------------------------------------------------
// small DFT kernels on registers, sign DIR
// ---------------------------------------------------------------------------

template <int DIR, typename C> __device__ __forceinline__ void dft2(C& a0, C& a1) {
  C t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

template <int DIR, typename C> __device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
  C t0 = cadd(a0, a2), t1 = csub(a0, a2);
  C t2 = cadd(a1, a3), t3 = mul_di<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int DIR, typename C> __device__ __forceinline__ void dft3(C& a0, C& a1, C& a2) {
  using T = decltype(a0.x);
  const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
  C t1 = cadd(a1, a2);
  C t2 = mul_di<DIR>(csub(a1, a2));
  t2.x *= h;
  t2.y *= h;
  C m = C{a0.x - T(0.5) * t1.x, a0.y - T(0.5) * t1.y};
  a0 = cadd(a0, t1);
  a1 = cadd(m, t2);
  a2 = csub(m, t2);
}

template <int DIR, typename C> __device__ __forceinline__ void dft8(C (&a)[8]) {
  using T = decltype(a[0].x);
  const T r = T(0.70710678118654752440084436210485);  // 1/sqrt(2)
  // even and odd halves as radix-4 transforms
  dft4<DIR>(a[0], a[2], a[4], a[6]);
  dft4<DIR>(a[1], a[3], a[5], a[7]);
  // odd half times w8^k, w8 = exp(DIR 2 pi i / 8)
  C o1 = a[3], o2 = a[5], o3 = a[7];
  // w8^1 = (r, DIR r)
  o1 = C{r * (o1.x - T(DIR) * o1.y), r * (o1.y + T(DIR) * o1.x)};
  // w8^2 = DIR i
  o2 = mul_di<DIR>(o2);
  // w8^3 = (-r, DIR r)
  o3 = C{-r * (o3.x + T(DIR) * o3.y), r * (T(DIR) * o3.x - o3.y)};
  C e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  C o0 = a[1];
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1);
  a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2);
  a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3);
  a[7] = csub(e3, o3);
}

// a * (cr + i*DIR*ci), a constant twiddle of sign DIR
template <int DIR, typename C, typename T>
__device__ __forceinline__ C cmulc(C a, T cr, T ci) {
  return C{a.x * cr - T(DIR) * ci * a.y, a.y * cr + T(DIR) * ci * a.x};
}

// 16-point DFT as 4 x 4: inner DFT4 over n1 (n = 4 n1 + n2), twiddle
// w16^(n2 k1), outer DFT4 over n2; output index k = k1 + 4 k2.
template <int DIR, typename C> __device__ __forceinline__ void dft16(C (&a)[16]) {
  using T = decltype(a[0].x);
  const T c1 = T(0.92387953251128675612818318939679);  // cos(pi/8)
  const T s1 = T(0.38268343236508977172845998403040);  // sin(pi/8)
  const T r = T(0.70710678118654752440084436210485);   // cos(pi/4)
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<DIR>(a[n2], a[4 + n2], a[8 + n2], a[12 + n2]);
  // a[4*k1 + n2] now holds Y[n2][k1]; apply w16^(n2 k1) = exp(DIR 2 pi i n2 k1 / 16)
  a[5] = cmulc<DIR>(a[5], c1, s1);     // n2=1,k1=1: w^1
  a[9] = cmulc<DIR>(a[9], r, r);       // n2=1,k1=2: w^2
  a[13] = cmulc<DIR>(a[13], s1, c1);   // n2=1,k1=3: w^3
  a[6] = cmulc<DIR>(a[6], r, r);       // n2=2,k1=1: w^2
  a[10] = mul_di<DIR>(a[10]);          // n2=2,k1=2: w^4
  a[14] = cmulc<DIR>(a[14], -r, r);    // n2=2,k1=3: w^6
  a[7] = cmulc<DIR>(a[7], s1, c1);     // n2=3,k1=1: w^3
  a[11] = cmulc<DIR>(a[11], -r, r);    // n2=3,k1=2: w^6
  a[15] = cmulc<DIR>(a[15], -c1, -s1); // n2=3,k1=3: w^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<DIR>(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3]);
  // a[4*k1 + k2] holds X[k1 + 4 k2]: transpose the 4x4 index
  C t[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) t[i] = a[i];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[4 * k1 + k2];
}

template <int R, int DIR, typename C> __device__ __forceinline__ void dft(C (&a)[R]) {
  if constexpr (R == 2) dft2<DIR>(a[0], a[1]);
  else if constexpr (R == 3) dft3<DIR>(a[0], a[1], a[2]);
  else if constexpr (R == 4) dft4<DIR>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<DIR>(a);
  else if constexpr (R == 16) dft16<DIR>(a);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// radix plans: E elements per thread, radices dividing E, product = N
// ---------------------------------------------------------------------------

// Radix plans.  A plan fixes the length N, the elements per thread E and the
// radix of each Stockham pass (every radix divides E).  Two variants per
// length: 0 holds E = 16 elements per thread where N allows (radix-16 passes,
// fewest LDS exchanges, fewest threads), 1 holds E = 8 (radix <= 8: twice the
// threads per line, so more waves per CU to hide memory latency, one more
// exchange).  Which variant each kernel uses is chosen per precision, length
// and pass kind by measurement (fft_tuned.hpp).
template <int N_, int E_, int... Rs> struct RadixPlan {
  static constexpr int N = N_;
  static constexpr int E = E_;
  static constexpr int NP = sizeof...(Rs);
  static constexpr int radix(int p) {
    constexpr int r[] = {Rs...};
    return r[p];
  }
};
template <int N, int V> struct FFTPlanV;
template <> struct FFTPlanV<16, 0> : RadixPlan<16, 16, 16> {};
template <> struct FFTPlanV<32, 0> : RadixPlan<32, 8, 8, 4> {};
template <> struct FFTPlanV<64, 0> : RadixPlan<64, 8, 8, 8> {};
template <> struct FFTPlanV<128, 0> : RadixPlan<128, 16, 16, 8> {};
template <> struct FFTPlanV<256, 0> : RadixPlan<256, 16, 16, 16> {};
template <> struct FFTPlanV<512, 0> : RadixPlan<512, 16, 16, 16, 2> {};
template <> struct FFTPlanV<768, 0> : RadixPlan<768, 24, 8, 8, 4, 3> {};
template <> struct FFTPlanV<96, 0> : RadixPlan<96, 24, 8, 4, 3> {};
template <> struct FFTPlanV<192, 0> : RadixPlan<192, 24, 8, 8, 3> {};
template <> struct FFTPlanV<384, 0> : RadixPlan<384, 24, 8, 4, 4, 3> {};
template <> struct FFTPlanV<1536, 0> : RadixPlan<1536, 24, 8, 8, 8, 3> {};
template <> struct FFTPlanV<3072, 0> : RadixPlan<3072, 24, 8, 8, 4, 4, 3> {};
template <> struct FFTPlanV<1024, 0> : RadixPlan<1024, 16, 16, 16, 4> {};
template <> struct FFTPlanV<2048, 0> : RadixPlan<2048, 16, 16, 16, 8> {};
template <> struct FFTPlanV<4096, 0> : RadixPlan<4096, 16, 16, 16, 16> {};
template <> struct FFTPlanV<128, 1> : RadixPlan<128, 8, 8, 4, 4> {};
template <> struct FFTPlanV<256, 1> : RadixPlan<256, 8, 8, 8, 4> {};
template <> struct FFTPlanV<512, 1> : RadixPlan<512, 8, 8, 8, 8> {};
template <> struct FFTPlanV<1024, 1> : RadixPlan<1024, 8, 8, 8, 4, 4> {};
template <> struct FFTPlanV<2048, 1> : RadixPlan<2048, 8, 8, 8, 8, 4> {};
template <> struct FFTPlanV<4096, 1> : RadixPlan<4096, 8, 8, 8, 8, 8> {};
// Lengths with a single plan answer variant 1 with variant 0.
template <> struct FFTPlanV<16, 1> : FFTPlanV<16, 0> {};
template <> struct FFTPlanV<32, 1> : FFTPlanV<32, 0> {};
template <> struct FFTPlanV<64, 1> : FFTPlanV<64, 0> {};
template <> struct FFTPlanV<768, 1> : FFTPlanV<768, 0> {};
template <> struct FFTPlanV<96, 1> : FFTPlanV<96, 0> {};
template <> struct FFTPlanV<192, 1> : FFTPlanV<192, 0> {};
template <> struct FFTPlanV<384, 1> : FFTPlanV<384, 0> {};
template <> struct FFTPlanV<1536, 1> : FFTPlanV<1536, 0> {};
template <> struct FFTPlanV<3072, 1> : FFTPlanV<3072, 0> {};

enum FFTPass { kRowPass = 0, kColPass = 1 };

}  // namespace fillk
#include "fft_tuned.hpp"
namespace fillk {

// The plan of the row passes (length nx) or the column pass (length ny) in
// precision T.  Building with FILL_FFT_FORCE_VARIANT=v gives every kernel
// variant v (the autotuner's candidate builds).
#ifdef FILL_FFT_FORCE_VARIANT
constexpr int fft_variant(bool, int, int) { return FILL_FFT_FORCE_VARIANT; }
#else
constexpr int fft_variant(bool f32, int n, int pass) { return tuned_fft_variant(f32, n, pass); }
#endif
// Rows per row-pass workgroup relative to the 64 KiB default (1 or 2); the
// autotuner's candidate builds force it with FILL_FFT_FORCE_ROWS=s.
#ifdef FILL_FFT_FORCE_ROWS
constexpr int row_scale(bool, int) { return FILL_FFT_FORCE_ROWS; }
#else
constexpr int row_scale(bool f32, int n) { return tuned_row_scale(f32, n); }
#endif
template <typename T, int N, int PASS>
using FFTPlanFor = FFTPlanV<N, fft_variant(sizeof(T) == 4, N, PASS)>;

template <typename PL, int P = 0> constexpr int plan_product() {
  if constexpr (P == PL::NP) return 1;
  else return PL::radix(P) * plan_product<PL, P + 1>();
}
template <typename PL, int P = 0> constexpr bool plan_divides_E() {
  if constexpr (P == PL::NP) return true;
  else return (PL::E % PL::radix(P) == 0) && plan_divides_E<PL, P + 1>();
}

// LDS index padding: one spare element every R0 elements (R0 = the first
// radix) turns the first pass's stride-R0 scatter into distinct banks.
template <typename PL> constexpr int lds_pad_shift() { return PL::radix(0) >= 16 ? 4 : 3; }
template <typename PL> __device__ __forceinline__ int lpad(int i) { return i + (i >> lds_pad_shift<PL>()); }
template <typename PL> constexpr int lds_line_elems() { return PL::N + (PL::N >> lds_pad_shift<PL>()); }

// Twiddles.  Pass p (radix R, NS = product of the earlier radices, S =
// N/(NS R)) needs w(i, k) = exp(-2 pi i * i k S / N) for k = j mod NS.  With
// k = klo + 16 khi the table stores LO[i][klo] = w(i, klo) and, when NS > 16,
// HI[i][khi] = w(i, 16 khi), so w(i, k) = LO[i][klo] * HI[i][khi]: lanes with
// consecutive j read consecutive LO entries and share HI entries, which keeps
// the LDS reads free of bank conflicts.  Passes with NS = 1 need no table.
template <typename PL> constexpr int pass_ns(int p) {
  int s = 1;
  for (int q = 0; q < p; ++q) s *= PL::radix(q);
  return s;
}
template <typename PL> constexpr int tw_pass_size(int p) {
  const int R = PL::radix(p), ns = pass_ns<PL>(p);
  if (ns == 1) return 0;
  return R * 16 + (ns > 16 ? R * (ns / 16) : 0);
}
template <typename PL> constexpr int tw_pass_off(int p) {
  int o = 0;
  for (int q = 0; q < p; ++q) o += tw_pass_size<PL>(q);
  return o;
}
template <typename PL> constexpr int tw_elems() { return tw_pass_off<PL>(PL::NP); }

// Copy the whole twiddle table from global memory into LDS; callers place a
// barrier between this and the first use.
template <typename PL, typename C>
__device__ __forceinline__ void tw_stage(C* q, const C* __restrict__ tw, int t, int nt) {
  for (int i = t; i < tw_elems<PL>(); i += nt) q[i] = tw[i];
}

template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// One Stockham pass in registers (butterflies j = tid + b*TPL, b < E/R).
template <typename C, typename PL, int P, int R, int NS, int DIR>
__device__ __forceinline__ void stockham_pass(C (&v)[PL::E], int tid, const C* tw) {
  constexpr int E = PL::E;
  constexpr int TPL = PL::N / E;
  constexpr int B = E / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    C a[R];
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = v[b + i * B];
    if constexpr (NS > 1) {
      const int j = tid + b * TPL;
      const int k = j % NS;
      const C* lo = tw + tw_pass_off<PL>(P) + (k & 15);
#pragma unroll
      for (int i = 1; i < R; ++i) {
        C w = lo[16 * i];
        if constexpr (NS > 16) w = cmul(w, tw[tw_pass_off<PL>(P) + 16 * R + i * (NS / 16) + (k >> 4)]);
        a[i] = twmul<DIR>(a[i], w);
      }
    }
    dft<R, DIR>(a);
#pragma unroll
    for (int i = 0; i < R; ++i) v[b + i * B] = a[i];
  }
}

// Scatter the pass outputs y[(j/NS)*NS*R + j%NS + i*NS] to LDS, gather the
// next pass's inputs x[tid + e*TPL].
template <typename C, typename PL, int R, int NS>
__device__ __forceinline__ void stockham_exchange(C (&v)[PL::E], int tid, C* lds) {
  constexpr int E = PL::E;
  constexpr int TPL = PL::N / E;
  constexpr int B = E / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = tid + b * TPL;
    const int k = j % NS;
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int i = 0; i < R; ++i) lds[lpad<PL>(base + i * NS)] = v[b + i * B];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = lds[lpad<PL>(tid + e * TPL)];
  __syncthreads();
}

// Full length-N transform of one line; v holds x[tid + e*TPL] on entry and
// X[tid + e*TPL] on exit; tw is the LDS twiddle table.  Every thread of
// the workgroup must call it (it contains workgroup barriers).
template <typename C, typename PL, int DIR, int P = 0, int NS = 1>
__device__ __forceinline__ void fft_line(C (&v)[PL::E], int tid, C* lds, const C* tw) {
  static_assert(plan_product<PL>() == PL::N, "radix plan does not multiply to N");
  static_assert(plan_divides_E<PL>(), "every radix must divide E");
  constexpr int R = PL::radix(P);
  stockham_pass<C, PL, P, R, NS, DIR>(v, tid, tw);
  if constexpr (P + 1 < PL::NP) {
    stockham_exchange<C, PL, R, NS>(v, tid, lds);
    fft_line<C, PL, DIR, P + 1, NS * R>(v, tid, lds, tw);
  }
}

// ---------------------------------------------------------------------------
// launch geometry per (precision, length)
// ---------------------------------------------------------------------------

// Row kernels: ROWS image rows per workgroup (two rows per complex line), the
// workgroup's LDS held near 64 KiB (or twice that, by tuning: longer
// contiguous pieces of the transposed spectrum, fewer workgroups).
template <typename T, int N> struct RowCfg {
  using PL = FFTPlanFor<T, N, kRowPass>;
  static constexpr int E = PL::E;
  static constexpr int TPL = N / E;
  static constexpr int RAW = row_scale(sizeof(T) == 4, N) * (64 * 1024) / (N * 8);
  static constexpr int ROWS = RAW >= 16 ? 16 : RAW >= 8 ? 8 : RAW >= 4 ? 4 : 2;  // power of two
  // consecutive row blocks that share a 128-byte line of the transposed spectrum
  static constexpr int XG0 = 128 / (ROWS * 2 * (int)sizeof(T));
  static constexpr int XG = XG0 < 1 ? 1 : XG0;
  static constexpr int LINES = ROWS / 2;
  static constexpr int THREADS = LINES * TPL;
  static constexpr int H = N / 2 + 1;
  // Row stride of the transposed-spectrum staging buffer in LDS.  Lanes of
  // one LDS cycle (256 bytes: G complex values) read ROWS rows at G/ROWS
  // consecutive kx; a stride congruent to G/ROWS modulo G puts them in
  // distinct banks.
  static constexpr int G = 256 / (2 * (int)sizeof(T));
  static constexpr int GR = G / ROWS > 0 ? G / ROWS : 1;
  static constexpr int HS = H + ((GR - H % G) % G + G) % G;
};

// Column kernel: W spectral columns (lines of length N = ny) per workgroup.
template <typename T, int N> struct ColCfg {
  using PL = FFTPlanFor<T, N, kColPass>;
  static constexpr int E = PL::E;
  static constexpr int TPL = N / E;
  static constexpr int RAW = (64 * 1024) / (N * 16);
  static constexpr int W0 = RAW > 16 ? 16 : (RAW < 1 ? 1 : RAW);
  static constexpr int W = (W0 * TPL > 1024) ? (1024 / TPL) : W0;
  static constexpr int THREADS = W * TPL;
};

// Workgroups are dispatched round-robin over the 8 XCDs.  Row blocks are
// handed out in groups of G neighbours (G blocks fill whole 128-byte lines of
// the transposed spectrum, so a group meets in one XCD's L2) and the groups go
// round-robin over the XCDs, which spreads a band of heavy rows over all of
// them.  Grids that are not a multiple of 8 G blocks keep the identity map.
template <int G>
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  if (nblk % (8 * G)) return bid;
  const int x = bid & 7, s = bid >> 3;
  return G * ((s / G) * 8 + x) + (s % G);
}

// Loads batched ahead of their uses: U elements per thread in flight.
constexpr int kBatch = 8;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals
// ---------------------------------------------------------------------------

struct u64x4 { uint64_t w0, w1, w2, w3; };

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return u64x4{c0, c1, c2, c3};
}

__device__ __forceinline__ double unit_open(uint64_t w) {
  return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

// Box-Muller: two independent standard normals from two 64-bit words, the
// radius from the first and the angle from the second (*c: the cosine one,
// *s: the sine one).  Pixels 4j .. 4j+3 come from Philox block j: words 0, 1
// give 4j (cosine) and 4j+1 (sine), words 2, 3 give 4j+2 and 4j+3.
__device__ __forceinline__ void box_muller2(uint64_t a, uint64_t b, double* c, double* s) {
  const double r = sqrt(-2.0 * log(unit_open(a)));
  double sn, cs;
  sincos(2.0 * 3.14159265358979323846 * unit_open(b), &sn, &cs);
  *c = r * cs;
  *s = r * sn;
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic workgroup sum of two values; result valid in thread 0.
// Workgroups narrower than a wave go through LDS only (a 64-lane shuffle
// would read inactive lanes).
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  if constexpr (NT % 64 == 0) {
    constexpr int NW = NT / 64;
    __shared__ double red[2][NW];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
      red[0][w] = a;
      red[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double sa = 0.0, sb = 0.0;
      for (int i = 0; i < NW; ++i) {
        sa += red[0][i];
        sb += red[1][i];
      }
      a = sa;
      b = sb;
    }
  } else {
    __shared__ double red[2][NT];
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sa = 0.0, sb = 0.0;
      for (int i = 0; i < NT; ++i) {
        sa += red[0][i];
        sb += red[1][i];
      }
      a = sa;
      b = sb;
    }
  }
}

}  // namespace fillk
