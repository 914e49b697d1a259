// Kernels of the block preconditioner M^-1 r (additive Schwarz; the host side
// is block.cpp):
//   band_solve_kernel  per (run, kx): solve (nx T_kx) u = rhat by the banded
//                      factor L L^T, forward then backward substitution, in
//                      place on the run's transposed row spectrum;
//   block_mv_kernel    per work item (block, 256 rows, 128 columns): partial
//                      products of A_b^-1 r_b (dense inverse, FP32/FP64);
//   combine_kernel     per slice of the compact range: z = band part (already in z on band
//                      pixels) + the block entries covering each element, and
//                      the FP64 partials of r.z and r.r.
// The row transforms of the band runs are the r2c / c2r kernels of the
// operator, launched on each run's rows as a grid of its own.
#include <type_traits>

#include "kernels.hpp"
#include "launch.hpp"

namespace fillk {

namespace {

// Lane U of the caller's half of the wave (lanes 0..31 get lane U, lanes
// 32..63 get lane 32 + U).  FP32: two lane reads and a select; FP64:
// ds_swizzle in bit mode (and_mask 0, or_mask U: every lane reads lane U of
// its group of 32) on both words, which measured faster there than four
// lane reads.
template <int U>
__device__ __forceinline__ float half_lane(float v, bool hi) {
  const float lo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), U));
  const float up = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32 + U));
  return hi ? up : lo;
}
template <int U>
__device__ __forceinline__ double half_lane(double v, bool) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffLL), U << 5);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), U << 5);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Lane U of the caller's half in FP32 as mr lo + mi hi, with the lane's
// constants (mr, mi) = (1, 0) in lanes 0..31 and (0, 1) in lanes 32..63: the
// same value as the select (one factor is exactly 0, the other exactly 1),
// but the two lane reads feed a multiply and an FMA that each take one of
// them as a scalar operand, where a select (its mask on the scalar bus too)
// needs both copied to vector registers first.
template <int U>
__device__ __forceinline__ float half_mix(float v, float mr, float mi) {
  const float lo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), U));
  const float up = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32 + U));
  return __builtin_fmaf(mi, up, mr * lo);
}
template <int U>
__device__ __forceinline__ double half_mix(double v, double, double) {
  return half_lane<U>(v, false);
}

// Calls fn(std::integral_constant<int, U>) for U = B .. E-1 in order.
template <int B, int E, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>{});
    static_for<B + 1, E>(fn);
  }
}

// 32 consecutive values of one lane's stream (aligned to 32 elements).
__device__ __forceinline__ void load32(float (&f)[32], const float* p) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const float4 v = q[u];
    f[4 * u] = v.x;
    f[4 * u + 1] = v.y;
    f[4 * u + 2] = v.z;
    f[4 * u + 3] = v.w;
  }
}
__device__ __forceinline__ void load32(double (&f)[32], const double* p) {
  const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const double2 v = q[u];
    f[2 * u] = v.x;
    f[2 * u + 1] = v.y;
  }
}

// The stored chunk of chunk c (32 positions of every lane's stream) of a
// (run, kx) whose chunks s0 .. s0 + d share chunk s0's storage.
__device__ __forceinline__ int stored_chunk(int c, int s0, int d) {
  return c < s0 ? c : (c <= s0 + d ? s0 : c - d);
}

// One wave per (column kx of the run's spectrum, run).  Column 0 carries the
// DC values in its real parts and the Nyquist values in its imaginary parts,
// which use the factors of kx = 0 and kx = nx/2.  The factor is stored
// unit-diagonal, L = Lu D: the forward pass solves Lu z = rhat and keeps
// z D^-2 = D^-1 y, the right-hand side of the backward pass Lu^T x = D^-1 y.
// Window: lane k (mod 32) of each half (real parts in lanes 0..31, imaginary
// parts in 32..63, one factor stream read serving both) holds the element
// i + ((k - i) mod 32) (forward) or i - ((i - k) mod 32) (backward) of the
// running right-hand side; the head lane of step i (k = i mod 32) holds the
// finished element i, which every lane of its half takes with a lane read,
// the others subtracting their coupling times it.  The steps are
// branch-free: each lane keeps its finished element of the chunk in a
// register and the chunk's results are stored together; the factor entries
// of the next chunk are loaded during the current one (two register sets
// taking turns).  Where the rows have reached their Toeplitz limit the
// chunks repeat and are stored once: a register set that already holds the
// repeated chunk is not loaded again.
// Column col of band run `run`, one wave (lanes threadIdx.x mod 64); smem:
// the wave's 2 hp values of LDS.  The workgroup's waves (all of one run)
// meet at its barriers.
template <typename T>
__device__ __forceinline__ void band_solve_column(const BandArgs<T>& a, int run, int col, unsigned char* smem) {
  // the problem's state is read beside the run's spectrum column
  const int prob = a.sc != nullptr ? a.run_prob[run] : 0;
  const int hp = a.run_hp[run];
  cplx<T>* X = a.Bt + a.run_bt[run] + (size_t)col * hp;
  T* sre = reinterpret_cast<T*>(smem);
  T* sim = sre + hp;
  const int lane = threadIdx.x & 63, k = lane & 31, half = lane >> 5;
  const int done = load_done(a.sc != nullptr ? a.sc + prob : nullptr);
  const int kx = (col == 0 && half) ? a.ncol : col;
  const int ki = a.run_k0[run] + kx;
  const T* F0 = a.fwd + a.kx_off[ki];  // this frequency's 32 lane streams
  const int s0 = a.kx_dup[2 * ki], dd = a.kx_dup[2 * ki + 1];
  for (int i = lane; i < hp; i += 64) {
    const cplx<T> c = X[i];
    sre[i] = c.x;
    sim[i] = c.y;
  }
  issue_fence();
  if (__builtin_amdgcn_readfirstlane(done)) return;
  __syncthreads();
  T* s = half ? sim : sre;
  const int L = hp - 32 * dd;  // stream length
  const T* F = F0 + (size_t)k * L;
  T w_;
  T fa[32], fb[32];

  // forward: Lu z = rhat, stored as z D^-2 (lane k's stream holds D^-2 of
  // element i at the steps i where k is the head).  The element that enters
  // lane k's slot during a chunk (c0 + 32 + k) is read from LDS at the
  // chunk's start.  The set loaded for chunk c held chunk c - 2.
  // FP32 steps read the next head from the FMA result (up): the head lane of
  // step u + 1 is not the head of step u, so its up is its new w_, and the
  // lane read does not wait for the select.
  const T mr = half ? T(0) : T(1), mi = half ? T(1) : T(0);
  auto fwd_chunk = [&](const T (&f)[32], T (&fn)[32], int c0) {
    if (c0 + 32 < hp) {
      const int c = (c0 >> 5) + 1;
      if (!(c - 2 >= s0 && c <= s0 + dd)) load32(fn, F + 32 * stored_chunk(c, s0, dd));
    }
    const T nxt = (c0 + 32 < hp) ? s[c0 + 32 + k] : T(0);
    // D^-2 of this lane's element c0 + k: its own stream's entry k of the chunk
    const T dg = F[32 * stored_chunk(c0 >> 5, s0, dd) + k];
    T zo = w_;  // this lane's finished element of the chunk (c0 + k)
    T src = w_;
    static_for<0, 32>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      T z;
      if constexpr (sizeof(T) == 4) z = half_mix<u>(src, mr, mi);
      else z = half_lane<u>(w_, half);
      const bool head = k == u;
      const T up = w_ - f[u] * z;
      zo = head ? w_ : zo;
      w_ = head ? nxt : up;
      src = up;
    });
    s[c0 + k] = zo * dg;
  };
  w_ = s[k];
  load32(fa, F + 32 * stored_chunk(0, s0, dd));
  for (int c0 = 0; c0 < hp; c0 += 64) {
    fwd_chunk(fa, fb, c0);
    if (c0 + 32 < hp) fwd_chunk(fb, fa, c0 + 32);
  }
  __syncthreads();

  // backward: Lu^T x = D^-1 y (the element entering lane k's slot during a
  // chunk is hp - 64 - c0 + k).  Step i = hp - 1 - (c0 + u) of the chunk
  // whose rows are forward chunk C = (hp - 32 - c0) / 32 needs row i of Lu:
  // Lu(i, i - d) for the lane holding element i - d, d = (i - k) mod 32,
  // which is entry i - d of the forward stream of lane hl = i mod 32 = 31 - u:
  // offset k of chunk C if k + u <= 31, else of chunk C - 1.  With the two
  // chunks stored one after the other that is po[u] below from the start of
  // C's storage; when both share one stored chunk, po[u] + 32 (k + u > 31).
  // Lanes past the first row read the zero guard or the previous stream and
  // hold nothing that is used.
  int po[32];
#pragma unroll
  for (int u = 0; u < 32; ++u) po[u] = (31 - u) * L + k - ((k + u > 31) ? 32 : 0);
  auto back_load = [&](T (&gr)[32], int c0) {
    const int C = (hp - 32 - c0) >> 5;
    const int mC = stored_chunk(C, s0, dd);
    const T* Fb = F0 + 32 * mC;
    if (stored_chunk(C - 1, s0, dd) == mC - 1) {
#pragma unroll
      for (int u = 0; u < 32; ++u) gr[u] = Fb[po[u]];
    } else {
#pragma unroll
      for (int u = 0; u < 32; ++u) gr[u] = Fb[po[u] + ((k + u) & 32)];
    }
  };
  // the chunks C and C - 1 both shared (the set loaded for the step of
  // chunk C held the one of chunk C + 2)
  auto shared2 = [&](int C) { return C > s0 && C <= s0 + dd; };
  auto bwd_chunk = [&](const T (&f)[32], T (&fn)[32], int c0) {
    if (c0 + 32 < hp) {
      const int C = ((hp - 32 - c0) >> 5) - 1;
      if (!(shared2(C) && shared2(C + 2))) back_load(fn, c0 + 32);
    }
    const T nxt = (c0 + 64 <= hp) ? s[hp - 64 - c0 + k] : T(0);
    T xo = w_;  // this lane's finished element of the chunk (hp - 32 - c0 + k)
    T src = w_;
    static_for<0, 32>([&](auto uc) {
      constexpr int u = decltype(uc)::value, hl = 31 - u;  // head lane of step i = hp - 1 - (c0 + u)
      T x;
      if constexpr (sizeof(T) == 4) x = half_mix<hl>(src, mr, mi);
      else x = half_lane<hl>(w_, half);
      const bool head = k == hl;
      const T up = w_ - f[u] * x;
      xo = head ? w_ : xo;
      w_ = head ? nxt : up;
      src = up;
    });
    s[hp - 32 - c0 + k] = xo;
  };
  w_ = s[hp - 32 + k];
  back_load(fa, 0);
  for (int c0 = 0; c0 < hp; c0 += 64) {
    bwd_chunk(fa, fb, c0);
    if (c0 + 32 < hp) bwd_chunk(fb, fa, c0 + 32);
  }
  __syncthreads();
  for (int i = lane; i < hp; i += 64) X[i] = cplx<T>{sre[i], sim[i]};
}

// Group u of ncol / CPG * nruns groups of CPG consecutive columns of one run.
// Workgroups run on XCD (index mod 8): when the groups of a run are a
// multiple of 8, u = 8 (nruns g + run) + (q mod 8) with group q = 8 g +
// (u mod 8) sends the runs' copies of one group of columns (one factor, when
// identical problems share it) to one XCD, one after another.
template <int CPG>
__device__ __forceinline__ void band_group(int u, int ncol, int nruns, int* run, int* q) {
  const int nq = ncol / CPG;
  if (nq % 8 == 0) {
    const int s = u >> 3, g = s / nruns;
    *run = s - g * nruns;
    *q = 8 * g + (u & 7);
  } else {
    *run = u / nq;
    *q = u - *run * nq;
  }
}

// One wave per (column, run).
template <typename T>
__global__ __launch_bounds__(64) void band_solve_kernel(BandArgs<T> a) {
  extern __shared__ unsigned char band_smem[];
  int run, col;
  band_group<1>(blockIdx.x, a.ncol, a.nruns, &run, &col);
  band_solve_column(a, run, col, band_smem);
}

constexpr int kBlkThreads = 256;           // 4 waves
constexpr int kBlkWaves = kBlkThreads / 64;
constexpr int kBlkRows = 256;              // rows of a work item: 4 per lane
constexpr int kBlkCols = 128;              // columns of a work item
constexpr int kBlkUnroll = 8;              // columns in flight per wave

// 4 consecutive entries of a column (16-byte aligned in FP32).
__device__ __forceinline__ void load4(float (&v)[4], const float* p) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
__device__ __forceinline__ void load4(double (&v)[4], const double* p) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}

// One workgroup per work item (block b, rows r0 .. r0+255, columns
// c0 .. c0+127): seg[so + i] = sum_{j in the columns} Ainv[j][i] r[bidx[o + j]]
// (the inverse is symmetric; column j is contiguous with stride
// ld = 4 ceil(n / 4)).  Lane l takes four consecutive rows, wave w the
// columns j = c0 + w (mod 4), kBlkUnroll of them in flight; the waves' sums
// are added in a fixed order, and the column chunks' outputs by the
// combination (deterministic).
template <typename T>
__device__ __forceinline__ void block_mv_item(const BlockArgs<T>& a, int it) {
  __shared__ T rv[kBlkCols];
  __shared__ T red[kBlkWaves][kBlkRows];
  const int t = threadIdx.x;
  const int* item = a.items + 4 * (size_t)it;
  const int b = item[0], r0 = item[1], c0 = item[2], so = item[3];
  // the problem's state is read beside the block's extent, then the gather
  const int prob = a.sc != nullptr ? a.block_prob[b] : 0;
  const int o = a.boff[b], n = a.boff[b + 1] - o;
  const int c1 = min(n, c0 + kBlkCols);
  const int done = load_done(a.sc != nullptr ? a.sc + prob : nullptr);
  if (t < c1 - c0) rv[t] = a.r[a.bidx[o + c0 + t]];
  issue_fence();
  if (__builtin_amdgcn_readfirstlane(done)) return;
  __syncthreads();
  const int ld = (n + 3) / 4 * 4;
  const int w = t >> 6, lane = t & 63;
  const int row = r0 + 4 * lane;
  T acc[4] = {T(0), T(0), T(0), T(0)};
  if (row < n) {
    const T* M = a.binv + a.moff[b] + row;
    int j = c0 + w;
    for (; j + (kBlkUnroll - 1) * kBlkWaves < c1; j += kBlkUnroll * kBlkWaves) {
      T v[kBlkUnroll][4];
#pragma unroll
      for (int u = 0; u < kBlkUnroll; ++u) load4(v[u], M + (size_t)(j + u * kBlkWaves) * ld);
#pragma unroll
      for (int u = 0; u < kBlkUnroll; ++u) {
        const T rj = rv[j + u * kBlkWaves - c0];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] += v[u][e] * rj;
      }
    }
    for (; j < c1; j += kBlkWaves) {
      T v[4];
      load4(v, M + (size_t)j * ld);
      const T rj = rv[j - c0];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] += v[e] * rj;
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) red[w][4 * lane + e] = acc[e];
  __syncthreads();
  if (r0 + t < n) {
    T s = red[0][t];
#pragma unroll
    for (int q = 1; q < kBlkWaves; ++q) s += red[q][t];
    a.seg[so + r0 + t] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlkThreads) void block_mv_kernel(BlockArgs<T> a) {
  block_mv_item(a, blockIdx.x);
}

// The band solves and the block products in one launch: workgroups
// 0 .. nband-1 take kBlkWaves columns of one run each (a wave per column),
// the rest one work item of the products each.  The two are independent:
// the products fill the issue slots the latency-bound substitutions leave.
template <typename T>
__global__ __launch_bounds__(kBlkThreads) void band_block_kernel(BandArgs<T> ba, BlockArgs<T> bk, int nband) {
  extern __shared__ unsigned char band_smem[];
  if ((int)blockIdx.x < nband) {
    const int wv = threadIdx.x >> 6;
    int run, q;
    band_group<kBlkWaves>(blockIdx.x, ba.ncol, ba.nruns, &run, &q);
    band_solve_column(ba, run, kBlkWaves * q + wv, band_smem + (size_t)wv * 2 * ba.max_hp * sizeof(T));
  } else {
    block_mv_item(bk, (int)blockIdx.x - nband);
  }
}

constexpr int kCombThreads = 1024;

// z[c] += the covering block entries of element c, taken four at a time (the
// four index loads, then the four value loads, then the additions in order).
template <typename T>
__device__ __forceinline__ T add_entries(const CombArgs<T>& a, T zc, int e, int e1) {
  for (; e + 4 <= e1; e += 4) {
    const int i0 = a.cix[e], i1 = a.cix[e + 1], i2 = a.cix[e + 2], i3 = a.cix[e + 3];
    const T s0 = a.seg[i0], s1 = a.seg[i1], s2 = a.seg[i2], s3 = a.seg[i3];
    zc += s0;
    zc += s1;
    zc += s2;
    zc += s3;
  }
  for (; e < e1; ++e) zc += a.seg[a.cix[e]];
  return zc;
}

// 4 consecutive values at p (16-byte aligned in FP32, 32 in FP64).
__device__ __forceinline__ void ld4(float (&v)[4], const float* p) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
__device__ __forceinline__ void ld4(double (&v)[4], const double* p) {
  const double2 q0 = *reinterpret_cast<const double2*>(p);
  const double2 q1 = *reinterpret_cast<const double2*>(p + 2);
  v[0] = q0.x;
  v[1] = q0.y;
  v[2] = q1.x;
  v[3] = q1.y;
}
__device__ __forceinline__ void st4(float* p, const float (&v)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(double* p, const double (&v)[4]) {
  *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
}

// One workgroup per equal slice of a problem's compact range.  In a slice of
// at least 4 elements per thread, elements up to the first multiple of 4 and
// after the last one go one per thread and the rest four consecutive ones per
// thread, with vector loads of the band flags, z, r and the CSR starts (most
// elements are band pixels with no block entry); smaller slices go one
// element per thread.
template <typename T>
__global__ __launch_bounds__(kCombThreads) void combine_kernel(CombArgs<T> a) {
  const int blk = blockIdx.x, pb = blockIdx.y;
  const int done = load_done(a.sc != nullptr ? a.sc + pb : nullptr);
  // equal slices of the problem's compact range (as many as row blocks)
  const long long nm = a.row_off[(size_t)pb * (a.ny + 1) + a.ny];
  const int nblk = gridDim.x;
  const int base = a.comp_off ? a.comp_off[pb] : 0;
  issue_fence();  // the state and the range in one round trip
  if (__builtin_amdgcn_readfirstlane(done)) return;
  const int c0 = base + (int)(nm * blk / nblk), c1 = base + (int)(nm * (blk + 1) / nblk);
  const int t = threadIdx.x;
  double acc0 = 0.0, acc1 = 0.0;
  auto one = [&](int c) {
    T zc = a.inb[c] ? a.z[c] : T(0);
    zc = add_entries(a, zc, a.cst[c], a.cst[c + 1]);
    a.z[c] = zc;
    const double rc = (double)a.r[c];
    acc0 += rc * (double)zc;
    acc1 += rc * rc;
  };
  // groups of 4 only where every thread gets at least one (small slices keep
  // one element per thread: more elements in flight)
  const bool quads = c1 - c0 >= 4 * kCombThreads;
  const int ca = quads ? min(c1, (c0 + 3) & ~3) : c1;  // first multiple of 4
  const int cb = ca + ((c1 - ca) & ~3);                // end of the groups of 4
  for (int c = c0 + t; c < ca; c += kCombThreads) one(c);
  for (int c = ca + 4 * t; c < cb; c += 4 * kCombThreads) {
    const uchar4 fl = *reinterpret_cast<const uchar4*>(a.inb + c);
    const int4 st = *reinterpret_cast<const int4*>(a.cst + c);
    const int se = a.cst[c + 4];
    T zv[4], rv[4];
    ld4(zv, a.z + c);
    ld4(rv, a.r + c);
    zv[0] = fl.x ? zv[0] : T(0);
    zv[1] = fl.y ? zv[1] : T(0);
    zv[2] = fl.z ? zv[2] : T(0);
    zv[3] = fl.w ? zv[3] : T(0);
    if (se != st.x) {
      zv[0] = add_entries(a, zv[0], st.x, st.y);
      zv[1] = add_entries(a, zv[1], st.y, st.z);
      zv[2] = add_entries(a, zv[2], st.z, st.w);
      zv[3] = add_entries(a, zv[3], st.w, se);
    }
    st4(a.z + c, zv);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double rc = (double)rv[k];
      acc0 += rc * (double)zv[k];
      acc1 += rc * rc;
    }
  }
  for (int c = cb + t; c < c1; c += kCombThreads) one(c);
  if (a.part0) {
    block_sum2<kCombThreads>(acc0, acc1);
    if (threadIdx.x == 0) {
      a.part0[(size_t)pb * a.part_stride + blk] = acc0;
      if (a.part1) a.part1[(size_t)pb * a.part_stride + blk] = acc1;
    }
  }
}

// Blocks of one size class m (blist: the class's blocks), each C^-1
// restricted to its n <= m pixels and padded with the identity to m x m,
// column-major, the class's matrices stride apart:
// A(i, j) = k(y_i - y_j, x_i - x_j) for i, j < n, k the periodic kernel of C^-1.
__global__ __launch_bounds__(256) void block_assemble_kernel(double* A, size_t stride, const int* blist,
                                                             const int* boff, const int* px, int m,
                                                             const double* kmap, int nx, int ny) {
  const int q = blockIdx.z, j = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const int b = blist[q], o = boff[b], n = boff[b + 1] - o;
  double v = (i == j) ? 1.0 : 0.0;
  if (i < n && j < n) {
    const int pi = px[o + i], pj = px[o + j];
    const int dy = ((pi / nx - pj / nx) % ny + ny) % ny, dx = ((pi % nx - pj % nx) % nx + nx) % nx;
    v = kmap[(size_t)dy * nx + dx];
  }
  A[(size_t)q * stride + (size_t)j * m + i] = v;
}

// The inverses held in the lower triangles of a class's matrices into dst:
// block b's column j at dst + moff[b] + j ld, ld = 4 ceil(n / 4) (rows 0..n-1),
// in the plan's precision.
template <typename T>
__global__ __launch_bounds__(256) void block_store_kernel(T* dst, const size_t* moff, const int* blist,
                                                          const int* boff, const double* A, size_t stride, int m) {
  const int q = blockIdx.z, j = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int b = blist[q], n = boff[b + 1] - boff[b];
  if (i >= n || j >= n) return;
  const double* Aq = A + (size_t)q * stride;
  dst[moff[b] + (size_t)j * ((n + 3) / 4 * 4) + i] = (T)(i >= j ? Aq[(size_t)j * m + i] : Aq[(size_t)i * m + j]);
}

}  // namespace

hipError_t launch_block_assemble(double* A, size_t stride, const int* blist, int count, const int* boff,
                                 const int* px, int m, const double* kmap, int nx, int ny, hipStream_t s) {
  if (count <= 0 || m <= 0) return hipSuccess;
  if (count > 65535 || stride < (size_t)m * m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(block_assemble_kernel, dim3((m + 255) / 256, m, count), dim3(256), 0, s, A, stride, blist,
                     boff, px, m, kmap, nx, ny);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_block_store(T* dst, const size_t* moff, const int* blist, int count, const int* boff,
                              const double* A, size_t stride, int m, hipStream_t s) {
  if (count <= 0 || m <= 0) return hipSuccess;
  if (count > 65535 || stride < (size_t)m * m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(block_store_kernel<T>, dim3((m + 255) / 256, m, count), dim3(256), 0, s, dst, moff, blist, boff,
                     A, stride, m);
  return hipGetLastError();
}
template hipError_t launch_block_store<float>(float*, const size_t*, const int*, int, const int*, const double*,
                                              size_t, int, hipStream_t);
template hipError_t launch_block_store<double>(double*, const size_t*, const int*, int, const int*, const double*,
                                               size_t, int, hipStream_t);

template <typename T>
hipError_t launch_band_solve(const BandArgs<T>& a, int nruns, int max_hp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (nruns <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * max_hp * sizeof(T);
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&band_solve_kernel<T>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (a.nruns != nruns) return hipErrorInvalidValue;
  const dim3 grid((unsigned)a.ncol * (unsigned)nruns);
  if (e0) hipExtLaunchKernelGGL(band_solve_kernel<T>, grid, dim3(64), lds, s, e0, e1, 0, a);
  else hipLaunchKernelGGL(band_solve_kernel<T>, grid, dim3(64), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_band_block(const BandArgs<T>& ba, const BlockArgs<T>& bk, int nruns, int max_hp, int nitems,
                             hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (nruns <= 0 || ba.nruns != nruns || ba.max_hp != max_hp || ba.ncol % kBlkWaves != 0)
    return hipErrorInvalidValue;
  const size_t lds = (size_t)kBlkWaves * 2 * max_hp * sizeof(T);
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&band_block_kernel<T>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int nband = ba.ncol / kBlkWaves * nruns;
  const dim3 grid((unsigned)(nband + nitems));
  if (e0) hipExtLaunchKernelGGL(band_block_kernel<T>, grid, dim3(kBlkThreads), lds, s, e0, e1, 0, ba, bk, nband);
  else hipLaunchKernelGGL(band_block_kernel<T>, grid, dim3(kBlkThreads), lds, s, ba, bk, nband);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_block_mv(const BlockArgs<T>& a, int nblocks, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid(nblocks);  // nblocks: work items
  if (e0) hipExtLaunchKernelGGL(block_mv_kernel<T>, grid, dim3(kBlkThreads), 0, s, e0, e1, 0, a);
  else hipLaunchKernelGGL(block_mv_kernel<T>, grid, dim3(kBlkThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_combine(const CombArgs<T>& a, int nblk, int nprob, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (nblk <= 0 || nprob <= 0) return hipErrorInvalidValue;
  if (e0) hipExtLaunchKernelGGL(combine_kernel<T>, dim3(nblk, nprob), dim3(kCombThreads), 0, s, e0, e1, 0, a);
  else hipLaunchKernelGGL(combine_kernel<T>, dim3(nblk, nprob), dim3(kCombThreads), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_band_solve<float>(const BandArgs<float>&, int, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_band_solve<double>(const BandArgs<double>&, int, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_band_block<float>(const BandArgs<float>&, const BlockArgs<float>&, int, int, int,
                                             hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_band_block<double>(const BandArgs<double>&, const BlockArgs<double>&, int, int, int,
                                              hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_block_mv<float>(const BlockArgs<float>&, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_block_mv<double>(const BlockArgs<double>&, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_combine<float>(const CombArgs<float>&, int, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_combine<double>(const CombArgs<double>&, int, int, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace fillk
