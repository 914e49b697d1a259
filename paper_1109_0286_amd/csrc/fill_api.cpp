// C ABI of the constrained-realization fill-in: plans, the batched solve
// driver and the entry points (contracts in include/fill.h).
//
// A plan holds nprob problems on the same nx x ny grid (own mask, seed, data
// and CG state; one shared spectrum or one per problem).  Every GPU step
// covers all problems of the plan in one launch.  A solve (Sec. 2.3 / 2.4):
//   1. s = C^{1/2} w from counter-based white noise (one apply, noise generated
//      inside the first row pass); the same pass writes x_out = d on observed
//      pixels and s on masked ones, and t = Py (d - s);
//   2. v = -Px C^-1 t (one apply), ||v|| per problem on the host;
//   3. refinement loop in FP64: r = v - A u (FP64 apply), then an inner
//      preconditioned CG on A d = r / ||r|| in the plan's precision (FP64, or
//      FP32 operators with FP64 dot products and scalars), u += ||r|| d;
//      each problem stops on its own true residual;
//   4. x_out += u on masked pixels.
// Inner CG (Hestenes-Stiefel) with M^-1 = E E, E = Px C^{1/2} Px: the paper's
// split form E A E u' = E v, u = E u', has the same iterates u.
#include <hip/hip_runtime.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/fill.h"
#include "block.hpp"
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
constexpr int kChunk = 16;  // CG iterations between host polls (even: keeps the rho parity)
constexpr int kChunkBlock = 8;  // the same with the block preconditioner (few iterations per solve)
constexpr int kMaxOuter = 60;

template <typename T> struct Vecs {
  T* x = nullptr;
  T* r = nullptr;
  T* z = nullptr;
  T* p = nullptr;
  T* q = nullptr;  // A p (s of single-reduction CG)
  T* t = nullptr;
  T* w = nullptr;  // A z (single-reduction CG)
};

// Per-call parameters, mirrored host (pinned) -> device in one copy.
struct Params {
  double* scale;      // r_in = res * scale
  double* unscale;    // u += unscale * x
  double* tol2;
  int* cap;
  int* active;
  const double** in_tab;
  double** out_tab;
  uint64_t* seeds;
  SolveCfg* cfg;      // refinement settings of the call
};

// Device side of the block preconditioner (FILL_PRECOND_BLOCK), built for the
// plan's precision from its mask and spectrum.
struct BlockDev {
  bool built = false;
  std::vector<void*> allocs;
  std::vector<fillb::Run> runs;
  std::vector<size_t> run_brow;  // offset of each run's virtual row offsets in brow_off
  std::vector<int> run_prob;     // problem of each run
  int* run_prob_d = nullptr;
  int* block_prob = nullptr;     // problem of each block
  int* items = nullptr;          // block product work items
  int nitems = 0;
  fill_block_info info{};
  int max_hp = 0, nblocks = 0;
  int* brow_off = nullptr;
  int* bpos = nullptr;           // 0, 1, 2, ...: a run's pixel index relative to its first pixel
  void* Bt = nullptr;
  void* fwd = nullptr;
  int* run_hp = nullptr;
  size_t* run_bt = nullptr;
  RunRow* run_rows = nullptr;  // the runs for the row passes
  int* run_k0 = nullptr;
  size_t* kx_off = nullptr;
  int* kx_dup = nullptr;
  int* boff = nullptr;
  int* bidx = nullptr;
  size_t* moff = nullptr;
  void* binv = nullptr;
  void* seg = nullptr;
  int* cst = nullptr;
  int* cix = nullptr;
  uint8_t* inb = nullptr;
};

}  // namespace

struct fill_plan_s {
  rocblas_handle rocblas = nullptr;  // block inverses at set-up (created on first use)
  int block_halo = fillb::HALO_AUTO;  // halo of the block preconditioner's pieces (or the automatic choice)
  struct {
    const double* part;  // the last iteration's r.r partials (or null)
    int nb;              // partial slots per problem
    bool first;          // the solve's first inner solve
  } after{nullptr, 0, false};  // an inner solve's accounting, launched with the update of u
  int nx = 0, ny = 0, ncol = 0, prec = 0, nprob = 1, npk = 1;
  int device = 0;  // the HIP device current at creation
  size_t npix = 0, nt = 0;
  hipStream_t stream = nullptr;
  std::vector<int> n_m, coff;
  int n_m_total = 0, n_m_max = 0;
  int max_iter = 20000;
  double inner_tol32 = 1e-4;
  int precond = FILL_PRECOND_SPLIT;
  int cg_variant = FILL_CG_STANDARD;
  BlockDev blk;
  std::vector<uint8_t> hmask;  // host copies: masks (0/1) and spectrum tables
  std::vector<double> hpk;
  double skew = 0.0;  // non-Hermitian study: eps of the perturbed A inside the inner CG
  // CG coefficient record of the first inner solve of the last solve (Lanczos data)
  int hist_cap = 0;
  double* hist = nullptr;
  std::vector<int> hist_n;
  // inner-CG chunks (an even number of iterations, 2..16) as HIP graphs,
  // captured on first use per [FP32?][preconditioner + 4 * CG variant]
  // [coefficient record][length / 2] and replayed by every solve
  int use_graph = 1;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph[2][8][2][9] = {};
  hipGraphExec_t graph_exec[2][8][2][9] = {};
  // iterations of the last inner solve per [FP32?][refinement step]: the
  // length of the first chunk of the next one
  int pred_iters[2][4] = {};
  int cur_outer = 0;
  // refinement state on the device (control kernels) and its host copy
  SolveState* st = nullptr;
  SolveState* h_st = nullptr;
  // the last solve's refinement steps and inner iterations per step (maximum
  // over problems) for a key (operation, preconditioner, recurrence): with
  // them a solve runs as one captured graph, no host round trip inside
  int pred_key = -1, pred_R = 0;
  int last_whole_graph = 0;  // the last solve ran as one graph replay
  unsigned gen = 0;          // bumped whenever captured graphs are dropped (groups re-capture)
  int pred_L[kStateIts] = {};
  std::map<std::vector<int>, std::pair<hipGraph_t, hipGraphExec_t>> solve_graphs;
  int nblk64 = 0, nblk32 = 0;

  uint8_t* mask = nullptr;
  int* pos = nullptr;
  int* row_off = nullptr;
  int* comp_off = nullptr;
  double* Dinv64 = nullptr;
  double* Dhalf64 = nullptr;
  double* Dfull64 = nullptr;  // P/N: the Px C Px preconditioner
  float* Dinv32 = nullptr;
  float* Dhalf32 = nullptr;
  float* Dfull32 = nullptr;
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
  double* part3 = nullptr;
  double* dsum = nullptr;
  CGScalars* sc = nullptr;
  void* par_dev = nullptr;
  void* par_host = nullptr;
  size_t par_bytes = 0;
  Params dp{}, hp{};
  CGScalars* h_sc = nullptr;
  double* h_sum = nullptr;
  std::vector<fill_stats> pstats;
  fill_stats stats{};
  std::vector<void*> allocs;
  // band-power spectrum model and adjoint workspaces (allocated on first use)
  int nbands = 0;
  double* lnk = nullptr;
  double* adj_s = nullptr;
  double* adj_cl = nullptr;
  double* adj_h = nullptr;
  double* adj_v = nullptr;
  double2* adj_X[4] = {nullptr, nullptr, nullptr, nullptr};
  double* adj_G = nullptr;
  double* adj_Gapi = nullptr;
  double* adj_gth = nullptr;
  // kernel-based Laplace relaxation (Sec. 6.3): kernel spectra and classes
  int lap_k = 0;
  double lap_r0 = 0.0, lap_ratio = 0.0;
  // Laplace warm start of the solves (fill_plan_set_warm_start): sweeps (0 = off) and kernels
  int ws_iters = 0, ws_k = 8;
  double ws_r0 = 1.5, ws_ratio = 2.0;
  std::vector<double*> lap_tab;
  std::vector<int> lap_used;
  uint8_t* lap_cls = nullptr;
  double* lap_x[3] = {nullptr, nullptr, nullptr};
  int* lap_pre = nullptr;
  int* lap_hw = nullptr;
  uint8_t* lap_touch = nullptr;
  // optional HIP-event timing of every launch of one kernel during solves
  int timed_kernel = -1;
  int timed_prec = 0;
  std::vector<hipEvent_t> events;  // start/stop pairs
  size_t events_used = 0;
  double timed_ms = 0.0;
  long long timed_count = 0;
};

// A group of batched plans solved together (fill_group_*): the graph that
// holds every plan's predicted solve as one branch, and what it was captured
// for (each plan's step counts and graph generation).
struct fill_group_s {
  std::vector<fill_plan> plans;
  hipStream_t stream = nullptr;   // where the group's graph is launched
  hipStream_t cap = nullptr;      // capture origin
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  std::vector<int> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int last_graph = 0;             // the last call ran as one graph launch
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
  static const double* Dfull(fill_plan p) { return p->Dfull64; }
  static int nblk(fill_plan p) { return p->nblk64; }
  static Vecs<double>& vecs(fill_plan p) { return p->v64; }
};
template <> struct TypeSel<float> {
  static const cplx<float>* twx(fill_plan p) { return p->twx32; }
  static const cplx<float>* twy(fill_plan p) { return p->twy32; }
  static const float* Dinv(fill_plan p) { return p->Dinv32; }
  static const float* Dhalf(fill_plan p) { return p->Dhalf32; }
  static const float* Dfull(fill_plan p) { return p->Dfull32; }
  static int nblk(fill_plan p) { return p->nblk32; }
  static Vecs<float>& vecs(fill_plan p) { return p->v32; }
};

// Row-pass arguments covering problems 0..nprob-1 of the plan.
template <typename T> RowArgs<T> row_base(fill_plan p, int nprob) {
  RowArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.nx = p->nx;
  a.ny = p->ny;
  a.ldx = p->ny;
  a.nprob = nprob;
  a.comp_off = p->comp_off;
  a.xt_stride = p->nt;
  a.part_stride = (size_t)p->ny;
  a.pix_stride = p->npix;
  a.row_off = p->row_off;
  a.pos = p->pos;
  a.Xt = static_cast<cplx<T>*>(p->Xt);
  a.tw = TypeSel<T>::twx(p);
  a.scale = T(1);
  a.mask = p->mask;
  return a;
}
template <typename T> ColArgs<T> col_base(fill_plan p, int nprob, const T* D, const CGScalars* sc) {
  ColArgs<T> ca;
  ca.Xt = static_cast<cplx<T>*>(p->Xt);
  ca.ldx = p->ny;
  ca.ncol = p->nx / 2;  // the Nyquist column travels in column 0
  ca.D = D;
  ca.tw = TypeSel<T>::twy(p);
  ca.sc = sc;
  ca.nprob = nprob;
  ca.xt_stride = p->nt;
  ca.d_stride = p->npk > 1 ? p->nt : 0;
  ca.skew = 0.0;
  return ca;
}

// Arguments for problem b alone (one-problem launches).
template <typename T> RowArgs<T> row_for(fill_plan p, int b) {
  RowArgs<T> a = row_base<T>(p, 1);
  a.row_off += (size_t)b * (p->ny + 1);
  a.pos += p->coff[b];
  a.mask += (size_t)b * p->npix;
  a.Xt += (size_t)b * p->nt;
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
           const CGScalars* sc, double skew = 0.0) {
  FILL_TRY(timed_launch<T>(p, FILL_K_R2C, [&](hipEvent_t a, hipEvent_t b) { return launch_r2c<T>(rm, ai, p->stream, a, b); }));
  ColArgs<T> ca = col_base<T>(p, ai.nprob, D, sc);
  ca.skew = skew;
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
  const ColArgs<T> ca = col_base<T>(p, ai.nprob, TypeSel<T>::Dhalf(p), sc);
  FILL_TRY(timed_launch<T>(p, FILL_K_COL, [&](hipEvent_t a, hipEvent_t b) { return launch_col<T>(p->ny, ca, p->stream, a, b); }));
  FILL_TRY(timed_launch<T>(p, FILL_K_PROJ, [&](hipEvent_t a, hipEvent_t b) { return launch_proj<T>(false, amid, p->stream, a, b); }));
  FILL_TRY(timed_launch<T>(p, FILL_K_COL, [&](hipEvent_t a, hipEvent_t b) { return launch_col<T>(p->ny, ca, p->stream, a, b); }));
  FILL_TRY(timed_launch<T>(p, FILL_K_C2R, [&](hipEvent_t a, hipEvent_t b) { return launch_c2r<T>(C2R_DOT2, ao, p->stream, a, b); }));
  return FILL_OK;
}

int upload_params(fill_plan p) {
  HIP_TRY(hipMemcpyAsync(p->par_dev, p->par_host, p->par_bytes, hipMemcpyHostToDevice, p->stream));
  return FILL_OK;
}

// The graph of one inner-CG chunk for (precision, preconditioner, record),
// captured on a private stream on first use (launch helpers follow
// p->stream, which is switched to that stream for the capture).
template <typename F>
int chunk_graph(fill_plan p, int f32, int mode, int rec, int len, F&& chunk, hipGraphExec_t* out) {
  hipGraphExec_t& ex = p->graph_exec[f32][mode][rec][len / 2];
  if (!ex) {
    if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    const hipStream_t saved = p->stream;
    p->stream = p->cap_stream;
    const hipError_t e0 = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    const int rc = e0 == hipSuccess ? chunk() : FILL_OK;
    hipGraph_t g = nullptr;
    const hipError_t e1 = e0 == hipSuccess ? hipStreamEndCapture(p->cap_stream, &g) : hipSuccess;
    p->stream = saved;
    if (e0 != hipSuccess) return fail(FILL_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e0));
    if (rc < 0 || e1 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      if (rc < 0) return rc;
      return fail(FILL_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e1));
    }
    const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
      ex = nullptr;
      (void)hipGraphDestroy(g);
      return fail(FILL_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    }
    p->graph[f32][mode][rec][len / 2] = g;
  }
  *out = ex;
  return FILL_OK;
}

// Drop captured chunk graphs (all, or only those that record coefficients),
// and every captured whole-solve graph.
void drop_graphs(fill_plan p, bool record_only) {
  ++p->gen;
  for (auto& kv : p->solve_graphs) {
    if (kv.second.second) (void)hipGraphExecDestroy(kv.second.second);
    if (kv.second.first) (void)hipGraphDestroy(kv.second.first);
  }
  p->solve_graphs.clear();
  for (int a = 0; a < 2; ++a)
    for (int m = 0; m < 8; ++m)
      for (int r = record_only ? 1 : 0; r < 2; ++r)
        for (int l = 0; l < 9; ++l) {
          if (p->graph_exec[a][m][r][l]) (void)hipGraphExecDestroy(p->graph_exec[a][m][r][l]);
          if (p->graph[a][m][r][l]) (void)hipGraphDestroy(p->graph[a][m][r][l]);
          p->graph_exec[a][m][r][l] = nullptr;
          p->graph[a][m][r][l] = nullptr;
        }
}

// ---------------------------------------------------------------------------
// Block preconditioner (FILL_PRECOND_BLOCK): host set-up and apply
// ---------------------------------------------------------------------------
template <typename P> int balloc(fill_plan p, P** out, size_t count) {
  void* ptr = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(P), 256);
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) return fail(FILL_ENOMEM, std::string("hipMalloc ") + std::to_string(bytes) + " bytes: " +
                                                    hipGetErrorString(e));
  p->blk.allocs.push_back(ptr);
  *out = static_cast<P*>(ptr);
  return FILL_OK;
}
template <typename P> int bupload(fill_plan p, P** out, const std::vector<P>& v) {
  FILL_TRY(balloc(p, out, v.size()));
  if (!v.empty()) HIP_TRY(hipMemcpy(*out, v.data(), v.size() * sizeof(P), hipMemcpyHostToDevice));
  return FILL_OK;
}
template <typename T> int bupload_as(fill_plan p, void** out, const std::vector<double>& v) {
  std::vector<T> c(v.begin(), v.end());
  T* d = nullptr;
  FILL_TRY(bupload(p, &d, c));
  *out = d;
  return FILL_OK;
}

void block_free(fill_plan p) {
  for (void* a : p->blk.allocs) (void)hipFree(a);
  p->blk = BlockDev();
}

// Dense inverses of a layout's blocks on the device: C^-1 on each block's
// pixels assembled from the kernel map dk (device, FP64), factored and
// inverted in FP64 by rocSOLVER (potrf, potri), stored in the plan's
// precision with the layout's column strides.  The blocks go by size class
// (n rounded up to a multiple of 32, padded with the identity, whose inverse
// leaves the block's own unchanged), one strided batch per class.  *out
// (allocated here, null if there are no blocks) holds L.inv_total values.
constexpr size_t kInvBatchBytes = size_t(256) << 20;
int block_inverses(fill_plan p, const fillb::Layout& L, const double* dk, void** out) {
  *out = nullptr;
  const int nb = (int)L.moff.size();
  if (nb == 0) return FILL_OK;
  const bool f32 = p->prec == FILL_PREC_FP32_OP;
  const size_t ts = f32 ? sizeof(float) : sizeof(double);
  std::map<int, std::vector<int>> cls;  // class size m -> its blocks
  for (int b = 0; b < nb; ++b) {
    const int n = L.boff[b + 1] - L.boff[b];
    cls[(n + 31) / 32 * 32].push_back(b);
  }
  std::vector<int> list;
  for (const auto& c : cls) list.insert(list.end(), c.second.begin(), c.second.end());
  void* inv = nullptr;
  int *dpx = nullptr, *dboff = nullptr, *dlist = nullptr, *dinfo = nullptr;
  size_t* dmoff = nullptr;
  double* dA = nullptr;
  size_t a_cap = 0;
  auto cleanup = [&](bool keep) {
    for (void* q : {(void*)dpx, (void*)dboff, (void*)dlist, (void*)dinfo, (void*)dmoff, (void*)dA})
      if (q) (void)hipFree(q);
    if (!keep && inv) (void)hipFree(inv);
  };
  auto hip_fail = [&](hipError_t e) {
    cleanup(false);
    return fail(FILL_EHIP, std::string("block set-up: ") + hipGetErrorString(e));
  };
  if (hipMalloc(&inv, L.inv_total * ts) != hipSuccess || hipMalloc(&dpx, L.bpix.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&dboff, L.boff.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&dlist, list.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&dmoff, L.moff.size() * sizeof(size_t)) != hipSuccess ||
      hipMalloc(&dinfo, 2 * (size_t)nb * sizeof(int)) != hipSuccess) {
    cleanup(false);
    return fail(FILL_ENOMEM, "block set-up: inverse workspace");
  }
  hipError_t e = hipMemsetAsync(inv, 0, L.inv_total * ts, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(dinfo, 0, 2 * (size_t)nb * sizeof(int), p->stream);
  if (e == hipSuccess) e = hipMemcpy(dpx, L.bpix.data(), L.bpix.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dboff, L.boff.data(), L.boff.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dlist, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dmoff, L.moff.data(), L.moff.size() * sizeof(size_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e);
  if ((p->rocblas == nullptr && rocblas_create_handle(&p->rocblas) != rocblas_status_success) ||
      rocblas_set_stream(p->rocblas, p->stream) != rocblas_status_success) {
    cleanup(false);
    return fail(FILL_EHIP, "block set-up: rocBLAS handle");
  }
  rocblas_handle h = p->rocblas;
  size_t off = 0;  // position of the current chunk in list
  for (const auto& c : cls) {
    const int m = c.first;
    const size_t mm = (size_t)m * m;
    const int per = (int)std::max<size_t>(1, std::min<size_t>(65535, kInvBatchBytes / (mm * sizeof(double))));
    for (size_t c0 = 0; c0 < c.second.size(); c0 += per) {
      const int cnt = (int)std::min<size_t>(per, c.second.size() - c0);
      if ((size_t)cnt * mm > a_cap) {  // grow the batch of matrices (after the work that uses it)
        if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e);
        if (dA) (void)hipFree(dA);
        dA = nullptr;
        a_cap = (size_t)cnt * mm;
        if (hipMalloc(&dA, a_cap * sizeof(double)) != hipSuccess) {
          cleanup(false);
          return fail(FILL_ENOMEM, "block set-up: inverse workspace");
        }
      }
      int* info_f = dinfo + off;
      int* info_i = dinfo + nb + off;
      e = launch_block_assemble(dA, mm, dlist + off, cnt, dboff, dpx, m, dk, p->nx, p->ny, p->stream);
      if (e != hipSuccess) return hip_fail(e);
      if (rocsolver_dpotrf_strided_batched(h, rocblas_fill_lower, m, dA, m, (rocblas_stride)mm, info_f, cnt) !=
              rocblas_status_success ||
          rocsolver_dpotri_strided_batched(h, rocblas_fill_lower, m, dA, m, (rocblas_stride)mm, info_i, cnt) !=
              rocblas_status_success) {
        cleanup(false);
        return fail(FILL_EHIP, "block set-up: rocSOLVER");
      }
      e = f32 ? launch_block_store<float>(static_cast<float*>(inv), dmoff, dlist + off, cnt, dboff, dA, mm, m,
                                          p->stream)
              : launch_block_store<double>(static_cast<double*>(inv), dmoff, dlist + off, cnt, dboff, dA, mm, m,
                                           p->stream);
      if (e != hipSuccess) return hip_fail(e);
      off += cnt;
    }
  }
  std::vector<int> info(2 * (size_t)nb, 0);
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e);
  if ((e = hipMemcpy(info.data(), dinfo, info.size() * sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e);
  for (int v : info)
    if (v != 0) {
      cleanup(false);
      return fail(FILL_ENOTSPD, "block preconditioner: a block of C^-1 is not positive definite");
    }
  cleanup(true);
  *out = inv;
  return FILL_OK;
}

// Layout of problem b: kernel of C^-1 from a unit impulse (one FP64 apply with
// problem b's table), its row transform for the band symbols, the host
// construction, then the dense inverses on the device (*inv, see
// block_inverses).
int block_layout_for(fill_plan p, int b, fillb::Layout* L, void** inv) {
  const int nx = p->nx, ny = p->ny, nc = p->ncol;
  const size_t npix = p->npix;
  const int tab = p->npk > 1 ? b : 0;
  if (p->hpk.size() != (size_t)p->npk * p->nt)
    return fail(FILL_EINVAL, "block preconditioner: the plan has no valid spectrum (a previous upload failed)");
  const double* P = p->hpk.data() + (size_t)tab * p->nt;
  for (int iy = 1; iy < ny; ++iy)
    for (int ix = 0; ix < nc; ++ix) {
      const double u = P[(size_t)iy * nc + ix], v = P[(size_t)((ny - iy) % ny) * nc + ix];
      if (std::fabs(u - v) > 1e-12 * std::max(u, v))
        return fail(FILL_EINVAL, "block preconditioner: the spectrum must satisfy P(kx, ky) = P(kx, -ky)");
    }
  std::vector<double> impulse(npix, 0.0), tsym;
  double* din = nullptr;
  double* dout = nullptr;
  std::vector<void*> tmp;
  auto release = [&]() {
    for (void* a : tmp) (void)hipFree(a);
  };
  if (hipMalloc(&din, npix * sizeof(double)) != hipSuccess) return fail(FILL_ENOMEM, "block set-up workspace");
  tmp.push_back(din);
  if (hipMalloc(&dout, npix * sizeof(double)) != hipSuccess) {
    release();
    return fail(FILL_ENOMEM, "block set-up workspace");
  }
  tmp.push_back(dout);
  impulse[0] = 1.0;
  int rc = FILL_OK;
  hipError_t e = hipMemcpy(din, impulse.data(), npix * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    RowArgs<double> ai = row_base<double>(p, 1), ao = row_base<double>(p, 1);
    ai.full_in = din;
    ao.full_out = dout;
    rc = apply3<double>(p, R2C_FULL, ai, p->Dinv64 + (size_t)tab * p->nt, C2R_FULL, ao, nullptr);
  }
  if (rc == FILL_OK && e == hipSuccess) e = hipStreamSynchronize(p->stream);
  // band symbols t_kx(d): the row transform of the kernel (real: k is even in x)
  const int ncx = nx / 2;
  std::vector<double2> xt((size_t)ncx * ny);
  if (rc == FILL_OK && e == hipSuccess) {
    RowArgs<double> at = row_base<double>(p, 1);
    at.full_in = dout;
    e = launch_r2c<double>(R2C_FULL, at, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess) e = hipMemcpy(xt.data(), p->Xt, xt.size() * sizeof(double2), hipMemcpyDeviceToHost);
  }
  if (rc != FILL_OK || e != hipSuccess) {
    release();
    return rc != FILL_OK ? rc : fail(FILL_EHIP, std::string("block set-up: ") + hipGetErrorString(e));
  }
  tsym.assign((size_t)ny * nc, 0.0);
  for (int d = 0; d < ny; ++d) {
    tsym[(size_t)d * nc] = xt[d].x;        // DC: column 0, real part
    tsym[(size_t)d * nc + ncx] = xt[d].y;  // Nyquist: column 0, imaginary part
    for (int kx = 1; kx < ncx; ++kx) tsym[(size_t)d * nc + kx] = xt[(size_t)kx * ny + d].x;
  }
  std::string err;
  const double pivot_min = p->prec == FILL_PREC_FP32_OP ? fillb::PIVOT_MIN_F32 : fillb::PIVOT_MIN;
  if (fillb::build_layout(nx, ny, p->hmask.data() + (size_t)b * npix, tsym.data(), pivot_min,
                          p->prec == FILL_PREC_FP32_OP, p->block_halo, L, &err) != 0) {
    release();
    return fail(FILL_ENOTSPD, "problem " + std::to_string(b) + ": " + err);
  }
  rc = block_inverses(p, *L, dout, inv);  // dout: the kernel map
  release();
  return rc;
}

// Build the block preconditioner for every problem of the plan (its mask,
// spectrum and precision): the problems' layouts are laid end to end, with
// compact indices offset by the problems' compact offsets.
int block_setup(fill_plan p) {
  static_assert(fillb::NBMAX == kBlockMax, "block size limit");
  HIP_TRY(hipStreamSynchronize(p->stream));
  drop_graphs(p, false);  // captured chunks hold the old tables
  block_free(p);
  const int np = p->nprob;
  fillb::Layout L;  // merged
  std::vector<int> run_prob, block_prob;
  L.boff.push_back(0);
  // Problems with identical masks and spectra (a Monte-Carlo batch) share
  // one built copy of the factors and inverses: the first such problem's.
  std::vector<fillb::Layout> kept;  // per built problem, without its factor values
  kept.reserve(np);
  struct Built {
    int prob;
    size_t fbase, mbase;
  };
  std::vector<Built> built;
  struct InvPart {
    void* dev;
    size_t n, off;
  };
  std::vector<InvPart> inv_parts;
  auto free_parts = [&]() {
    for (InvPart& q : inv_parts) (void)hipFree(q.dev);
    inv_parts.clear();
  };
  struct PartsGuard {  // frees what an early return leaves
    std::vector<InvPart>* v;
    ~PartsGuard() {
      for (InvPart& q : *v) (void)hipFree(q.dev);
    }
  } parts_guard{&inv_parts};
  size_t inv_total = 0, binv_logical = 0;
  struct ItemRange {
    size_t first, n, key;  // the problem's work items and the offset of the inverses they read
  };
  std::vector<ItemRange> item_range;
  auto same_problem = [&](int a, int b) {
    if (std::memcmp(p->hmask.data() + (size_t)a * p->npix, p->hmask.data() + (size_t)b * p->npix, p->npix) != 0)
      return false;
    if (p->npk <= 1) return true;
    return std::memcmp(p->hpk.data() + (size_t)a * p->nt, p->hpk.data() + (size_t)b * p->nt,
                       p->nt * sizeof(double)) == 0;
  };
  for (int b = 0; b < np; ++b) {
    int same = -1;
    for (size_t q = 0; q < built.size() && same < 0; ++q)
      if (same_problem(built[q].prob, b)) same = (int)q;
    if (same < 0) {
      fillb::Layout Lb;
      void* inv = nullptr;
      const int rc = block_layout_for(p, b, &Lb, &inv);
      if (rc != FILL_OK) {
        free_parts();
        return rc;
      }
      if (inv != nullptr) inv_parts.push_back({inv, Lb.inv_total, inv_total});
      built.push_back({b, L.fwd.size(), inv_total});
      inv_total += Lb.inv_total;
      L.fwd.insert(L.fwd.end(), Lb.fwd.begin(), Lb.fwd.end());
      std::vector<double>().swap(Lb.fwd);
      kept.push_back(std::move(Lb));
      same = (int)built.size() - 1;
    }
    const fillb::Layout& Lb = kept[same];
    const size_t fbase = built[same].fbase, mbase = built[same].mbase;
    const int co = p->coff[b];
    const int kbase = (int)L.kx_off.size();
    for (size_t o : Lb.kx_off) L.kx_off.push_back(o + fbase);
    L.kx_dup.insert(L.kx_dup.end(), Lb.kx_dup.begin(), Lb.kx_dup.end());
    L.stream_values += Lb.stream_values;
    size_t ro = 0;
    for (fillb::Run r : Lb.runs) {
      r.cb0 += co;
      r.bt_off += L.bt_total;
      r.k0 += kbase;
      L.runs.push_back(r);
      run_prob.push_back(b);
      for (int j = 0; j <= r.hp; ++j) L.brow_off.push_back(Lb.brow_off[ro + j] + co);
      ro += (size_t)r.hp + 1;
    }
    L.bt_total += Lb.bt_total;
    L.max_run_pixels = std::max(L.max_run_pixels, Lb.max_run_pixels);
    const int nbase = (int)L.bidx.size();
    const int bbase = (int)L.boff.size() - 1;
    const size_t sbase = L.seg_total;
    for (size_t q = 1; q < Lb.boff.size(); ++q) {
      L.boff.push_back(Lb.boff[q] + nbase);
      L.moff.push_back(Lb.moff[q - 1] + mbase);
      block_prob.push_back(b);
    }
    item_range.push_back({L.items.size() / 4, Lb.items.size() / 4, mbase});
    for (size_t q = 0; q < Lb.items.size(); q += 4) {
      L.items.push_back(Lb.items[q] + bbase);
      L.items.push_back(Lb.items[q + 1]);
      L.items.push_back(Lb.items[q + 2]);
      L.items.push_back((int)(Lb.items[q + 3] + sbase));
    }
    L.seg_total += Lb.seg_total;
    if (L.seg_total > (size_t)INT32_MAX) {
      free_parts();
      return fail(FILL_EINVAL, "block preconditioner: too many block outputs");
    }
    for (int c : Lb.bidx) L.bidx.push_back(c + co);
    binv_logical += Lb.inv_total;
    const int ebase = L.cst.empty() ? 0 : L.cst.back();
    if (L.cst.empty()) L.cst.push_back(0);
    for (int c = 1; c <= Lb.n_m; ++c) L.cst.push_back(Lb.cst[c] + ebase);
    for (int e : Lb.cix) L.cix.push_back((int)(e + sbase));
    L.inb.insert(L.inb.end(), Lb.inb.begin(), Lb.inb.end());
    L.n_m += Lb.n_m;
  }
  if (L.cst.empty()) L.cst.push_back(0);
  // Problems that share their inverses take turns in groups of 8 work items:
  // work item w runs on XCD w mod 8, so the copies of one item go to one XCD
  // back to back and read the inverse through its L2.  Others keep their order.
  {
    std::vector<int> order;  // work items in launch order
    std::vector<bool> placed(item_range.size(), false);
    for (size_t i = 0; i < item_range.size(); ++i) {
      if (placed[i]) continue;
      std::vector<size_t> grp;
      for (size_t j = i; j < item_range.size(); ++j)
        if (!placed[j] && item_range[j].key == item_range[i].key && item_range[j].n == item_range[i].n) {
          grp.push_back(j);
          placed[j] = true;
        }
      const size_t n = item_range[i].n;
      for (size_t i0 = 0; i0 < n; i0 += 8)
        for (size_t j : grp)
          for (size_t t = i0; t < std::min(n, i0 + 8); ++t) order.push_back((int)(item_range[j].first + t));
    }
    std::vector<int> items(L.items.size());
    for (size_t w = 0; w < order.size(); ++w)
      std::copy(L.items.begin() + 4 * (size_t)order[w], L.items.begin() + 4 * (size_t)order[w] + 4, items.begin() + 4 * w);
    L.items.swap(items);
  }
  BlockDev& B = p->blk;
  const bool f32 = p->prec == FILL_PREC_FP32_OP;
  const size_t ts = f32 ? sizeof(float) : sizeof(double);
  B.runs = L.runs;
  B.run_prob = run_prob;
  size_t ro = 0;
  std::vector<int> hp, k0, bpos(std::max(L.max_run_pixels, 1));
  std::vector<size_t> bt;
  for (const fillb::Run& r : L.runs) {
    B.run_brow.push_back(ro);
    ro += (size_t)r.hp + 1;
    B.max_hp = std::max(B.max_hp, r.hp);
    hp.push_back(r.hp);
    bt.push_back(r.bt_off);
    k0.push_back(r.k0);
  }
  for (size_t i = 0; i < bpos.size(); ++i) bpos[i] = (int)i;
  B.nblocks = (int)L.boff.size() - 1;
  FILL_TRY(bupload(p, &B.brow_off, L.brow_off));
  FILL_TRY(bupload(p, &B.bpos, bpos));
  FILL_TRY(bupload(p, &B.run_hp, hp));
  FILL_TRY(bupload(p, &B.run_bt, bt));
  FILL_TRY(bupload(p, &B.run_k0, k0));
  {
    std::vector<RunRow> rr;
    for (size_t q = 0; q < L.runs.size(); ++q)
      rr.push_back(RunRow{B.run_brow[q], L.runs[q].bt_off, L.runs[q].hp, L.runs[q].cb0, run_prob[q], 0});
    FILL_TRY(bupload(p, &B.run_rows, rr));
  }
  FILL_TRY(bupload(p, &B.kx_off, L.kx_off));
  FILL_TRY(bupload(p, &B.kx_dup, L.kx_dup));
  FILL_TRY(bupload(p, &B.run_prob_d, run_prob));
  FILL_TRY(bupload(p, &B.block_prob, block_prob));
  FILL_TRY(bupload(p, &B.boff, L.boff));
  FILL_TRY(bupload(p, &B.items, L.items));
  B.nitems = (int)(L.items.size() / 4);
  FILL_TRY(bupload(p, &B.bidx, L.bidx));
  FILL_TRY(bupload(p, &B.moff, L.moff));
  FILL_TRY(bupload(p, &B.cst, L.cst));
  FILL_TRY(bupload(p, &B.cix, L.cix));
  FILL_TRY(bupload(p, &B.inb, L.inb));
  {
    uint8_t* bt_raw = nullptr;
    FILL_TRY(balloc(p, &bt_raw, std::max<size_t>(L.bt_total, 1) * 2 * ts));
    B.Bt = bt_raw;
    uint8_t* seg_raw = nullptr;
    FILL_TRY(balloc(p, &seg_raw, std::max<size_t>(L.seg_total, 1) * ts));
    B.seg = seg_raw;
  }
  if (f32) FILL_TRY(bupload_as<float>(p, &B.fwd, L.fwd));
  else FILL_TRY(bupload_as<double>(p, &B.fwd, L.fwd));
  {
    // the built problems' inverses, end to end
    uint8_t* binv_raw = nullptr;
    const int rc = balloc(p, &binv_raw, std::max<size_t>(inv_total, 1) * ts);
    if (rc != FILL_OK) {
      free_parts();
      return rc;
    }
    B.binv = binv_raw;
    hipError_t e = hipSuccess;
    for (const InvPart& q : inv_parts)
      if (e == hipSuccess)
        e = hipMemcpyAsync(binv_raw + q.off * ts, q.dev, q.n * ts, hipMemcpyDeviceToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    free_parts();
    if (e != hipSuccess) return fail(FILL_EHIP, std::string("block set-up: ") + hipGetErrorString(e));
  }
  B.info.runs = (int)L.runs.size();
  B.info.blocks = B.nblocks;
  for (const fillb::Run& r : L.runs) B.info.band_rows += r.hp;
  B.info.block_pixels = (int64_t)L.bidx.size();
  B.info.block_entries = (int64_t)binv_logical;
  B.info.band_stream_values = (int64_t)L.stream_values;
  B.info.halo_min = B.info.halo_max = kept.empty() ? fillb::HALO : kept[0].halo;
  for (const fillb::Layout& k : kept) {
    B.info.halo_min = std::min(B.info.halo_min, k.halo);
    B.info.halo_max = std::max(B.info.halo_max, k.halo);
  }
  B.info.elem_bytes = (int)ts;
  B.info.bytes = (int64_t)((L.fwd.size() + inv_total + L.bidx.size() + 2 * L.bt_total) * ts +
                           (L.brow_off.size() + bpos.size() + L.boff.size() + L.bidx.size() + L.cst.size() +
                            L.cix.size() + L.kx_dup.size()) * sizeof(int) +
                           L.kx_off.size() * sizeof(size_t) + L.inb.size());
  B.built = true;
  return FILL_OK;
}

// After a change of spectrum: rebuild a built block preconditioner (if that
// fails, the plan falls back to M^-1 = Px C Px and the error is returned).
int block_follow_pk(fill_plan p) {
  if (!p->blk.built) return FILL_OK;
  const int rc = block_setup(p);
  if (rc != FILL_OK && p->precond == FILL_PRECOND_BLOCK) p->precond = FILL_PRECOND_CXX;
  return rc;
}

// z = M^-1 r (compact vectors of the plan's precision), with the partials of
// r.z and r.r over the row blocks (part0/part1 may be null).  Launches: the
// forward row transforms of the band runs' rows, the banded solves of every
// (run, kx) together with the dense block products, the inverse row
// transforms into z and the combination.  only >= 0 launches that kernel
// alone (FILL_K_BAND: the band solves only, FILL_K_BLOCKMV or
// FILL_K_COMBINE: timing).
constexpr size_t kFusedBandLds = 48 * 1024;
template <typename T>
int block_apply(fill_plan p, const T* r, T* z, double* part0, double* part1, CGScalars* sc, int only = -1) {
  BlockDev& B = p->blk;
  if (!B.built || (sizeof(T) == 4) != (p->prec == FILL_PREC_FP32_OP))
    return fail(FILL_EINVAL, "block preconditioner not built for this precision");
  const int nruns = (int)B.runs.size();
  // the row passes of every band run in one launch (blockIdx.y = run)
  auto run_args = [&]() {
    RowArgs<T> a = row_base<T>(p, nruns);
    a.ny = B.max_hp;
    a.ldx = B.max_hp;
    a.comp_off = nullptr;
    a.row_off = B.brow_off;
    a.pos = B.bpos;  // pos[c] = c - cb0: the pixel index within the run's rows
    a.Xt = static_cast<cplx<T>*>(B.Bt);
    a.sc = sc;
    a.runs = B.run_rows;
    return a;
  };
  BlockArgs<T> bk;
  bk.r = r;
  bk.seg = static_cast<T*>(B.seg);
  bk.items = B.items;
  bk.boff = B.boff;
  bk.bidx = B.bidx;
  bk.moff = B.moff;
  bk.binv = static_cast<const T*>(B.binv);
  bk.block_prob = B.block_prob;
  bk.sc = sc;
  BandArgs<T> ba;
  ba.Bt = static_cast<cplx<T>*>(B.Bt);
  ba.fwd = static_cast<const T*>(B.fwd);
  ba.run_hp = B.run_hp;
  ba.run_bt = B.run_bt;
  ba.run_k0 = B.run_k0;
  ba.kx_off = B.kx_off;
  ba.kx_dup = B.kx_dup;
  ba.nruns = nruns;
  ba.max_hp = B.max_hp;
  ba.ncol = p->nx / 2;
  ba.run_prob = B.run_prob_d;
  ba.sc = sc;
  // The band solves and the block products share one launch (timed as the
  // band kernel) where the band's LDS leaves room for the products'
  // workgroups beside it.
  const bool fused = only < 0 && nruns > 0 && B.nitems > 0 && ba.ncol % 4 == 0 &&
                     (size_t)4 * 2 * B.max_hp * sizeof(T) <= kFusedBandLds;
  if (!fused && (only < 0 || only == FILL_K_BLOCKMV))
    FILL_TRY(timed_launch<T>(p, FILL_K_BLOCKMV, [&](hipEvent_t e0, hipEvent_t e1) {
      return launch_block_mv<T>(bk, B.nitems, p->stream, e0, e1);
    }));
  if (nruns > 0 && only < 0) {
    RowArgs<T> a = run_args();
    a.v0 = const_cast<T*>(r);
    HIP_TRY(launch_r2c<T>(R2C_COMPACT, a, p->stream));
  }
  if (fused)
    FILL_TRY(timed_launch<T>(p, FILL_K_BAND, [&](hipEvent_t e0, hipEvent_t e1) {
      return launch_band_block<T>(ba, bk, nruns, B.max_hp, B.nitems, p->stream, e0, e1);
    }));
  else if (nruns > 0 && (only < 0 || only == FILL_K_BAND))
    FILL_TRY(timed_launch<T>(p, FILL_K_BAND, [&](hipEvent_t e0, hipEvent_t e1) {
      return launch_band_solve<T>(ba, nruns, B.max_hp, p->stream, e0, e1);
    }));
  if (nruns > 0 && only < 0) {
    RowArgs<T> a = run_args();
    a.v0 = z;
    HIP_TRY(launch_c2r<T>(C2R_COMPACT, a, p->stream));
  }
  if (only >= 0 && only != FILL_K_COMBINE) return FILL_OK;
  const int nb = TypeSel<T>::nblk(p);
  CombArgs<T> cb;
  cb.z = z;
  cb.r = r;
  cb.seg = static_cast<const T*>(B.seg);
  cb.cst = B.cst;
  cb.cix = B.cix;
  cb.inb = B.inb;
  cb.row_off = p->row_off;
  cb.comp_off = p->comp_off;
  cb.ny = p->ny;
  cb.part_stride = (size_t)p->ny;
  cb.rows = p->ny / nb;
  cb.part0 = part0;
  cb.part1 = part1;
  cb.sc = sc;
  FILL_TRY(timed_launch<T>(p, FILL_K_COMBINE, [&](hipEvent_t e0, hipEvent_t e1) {
    return launch_combine<T>(cb, nb, p->nprob, p->stream, e0, e1);
  }));
  return FILL_OK;
}

// Arguments of the refinement control kernels.
RefineArgs refine_args(fill_plan p) {
  RefineArgs a;
  a.st = p->st;
  a.cfg = p->dp.cfg;
  a.sc = p->sc;
  a.scale = p->dp.scale;
  a.unscale = p->dp.unscale;
  a.tol2 = p->dp.tol2;
  a.cap = p->dp.cap;
  a.active = p->dp.active;
  a.nprob = p->nprob;
  return a;
}

// Run inner-CG chunks (graph replays, or direct launches) until every problem
// is done: a first chunk of len0 iterations, then chunks of len1; chunk(len)
// launches one directly, exec(len) returns its graph or null.  After each
// chunk a device check (rr_part: the r.r partials of the last iteration, nb
// per problem) also stops a problem whose r.r meets its tolerance, which the
// kernels would only see at the next chunk's first step; then the host reads
// the CG scalars.  Per-problem iteration counts and statuses.
template <typename C, typename E>
int run_chunks(fill_plan p, int len0, int len1, C&& chunk, E&& exec, const double* rr_part, int nb,
               std::vector<int>& iters, std::vector<int>& status) {
  const int np = p->nprob;
  int len = len0;
  for (;;) {
    hipGraphExec_t ex = nullptr;
    FILL_TRY(exec(len, &ex));
    if (ex) HIP_TRY(hipGraphLaunch(ex, p->stream));
    else FILL_TRY(chunk(len));
    if (rr_part) HIP_TRY(launch_rr_check(p->sc, rr_part, nb, (size_t)p->ny, np, p->stream));
    HIP_TRY(hipMemcpyAsync(p->h_sc, p->sc, np * sizeof(CGScalars), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    bool all = true;
    for (int b = 0; b < np; ++b) all = all && p->h_sc[b].done;
    if (all) break;
    len = len1;
  }
  iters.resize(np);
  status.resize(np);
  for (int b = 0; b < np; ++b) {
    iters[b] = p->h_sc[b].iter;
    status[b] = p->h_sc[b].status;
  }
  return FILL_OK;
}

// Inner CG in single-reduction form (Chronopoulos and Gear), same contract as
// inner_pcg.  Iteration j: one r2c pass takes the scalar step from the
// partials of r.z, r.r and w.z, applies p = z + beta p, s = w + beta s,
// x += alpha p, r -= alpha s and transforms the new r; z = M^-1 r and w = A z
// follow with no scalar in between, so the preconditioner's closing row pass
// and the operator's opening one are a single projection pass:
//   Px C Px: r2c -> col(P) -> proj(z; r.z, r.r) -> col(1/P) -> c2r(w; w.z)
//   E E:     r2c -> col(sqrt P) -> proj -> col(sqrt P) -> proj(z; r.z, r.r) -> col(1/P) -> c2r(w; w.z)
//   none:    r2c (with r.r of the new r) -> col(1/P) -> c2r(w; w.r)
// (one launch fewer per iteration than the standard form).
template <typename T>
int inner_pcg_cg1(fill_plan p, bool record, int fixed) {
  Vecs<T>& v = TypeSel<T>::vecs(p);
  const int nb = TypeSel<T>::nblk(p), np = p->nprob;
  const int mode = p->precond;
  const bool pre = mode != FILL_PRECOND_NONE;
  double* hist = record && p->hist_cap > 0 ? p->hist : nullptr;
  const size_t vb = (size_t)std::max(p->n_m_total, 1) * sizeof(T);
  // r holds the scaled residual and x = p = 0 (the caller's scale pass)
  HIP_TRY(hipMemsetAsync(v.q, 0, vb, p->stream));
  // without a preconditioner the r.r partials of the r2c pass alternate
  // between two buffers by iteration parity
  double* const rrb[2] = {p->part0, p->part3};

  // z = M^-1 r and w = A z from the transformed r (every kernel returns at
  // once for a finished problem when sc is set)
  auto tail = [&](CGScalars* sc) -> int {
    const ColArgs<T> cm = col_base<T>(p, np, mode == FILL_PRECOND_SPLIT ? TypeSel<T>::Dhalf(p) : TypeSel<T>::Dfull(p), sc);
    ColArgs<T> ca = col_base<T>(p, np, TypeSel<T>::Dinv(p), sc);
    ca.skew = p->skew;
    if (pre) {
      FILL_TRY(timed_launch<T>(p, FILL_K_COL, [&](hipEvent_t a, hipEvent_t b) { return launch_col<T>(p->ny, cm, p->stream, a, b); }));
      if (mode == FILL_PRECOND_SPLIT) {
        RowArgs<T> mid = row_base<T>(p, np);
        mid.sc = sc;
        FILL_TRY(timed_launch<T>(p, FILL_K_PROJ, [&](hipEvent_t a, hipEvent_t b) { return launch_proj<T>(false, mid, p->stream, a, b); }));
        FILL_TRY(timed_launch<T>(p, FILL_K_COL, [&](hipEvent_t a, hipEvent_t b) { return launch_col<T>(p->ny, cm, p->stream, a, b); }));
      }
      RowArgs<T> zp = row_base<T>(p, np);
      zp.sc = sc;
      zp.v0 = v.z;
      zp.v1 = v.r;
      zp.part0 = p->part0;
      zp.part1 = p->part1;
      FILL_TRY(timed_launch<T>(p, FILL_K_PROJ, [&](hipEvent_t a, hipEvent_t b) { return launch_proj<T>(true, zp, p->stream, a, b); }));
    }
    FILL_TRY(timed_launch<T>(p, FILL_K_COL, [&](hipEvent_t a, hipEvent_t b) { return launch_col<T>(p->ny, ca, p->stream, a, b); }));
    RowArgs<T> wo = row_base<T>(p, np);
    wo.sc = sc;
    wo.v0 = v.w;
    wo.v1 = pre ? v.z : v.r;
    wo.part0 = p->part2;
    FILL_TRY(timed_launch<T>(p, FILL_K_C2R, [&](hipEvent_t a, hipEvent_t b) { return launch_c2r<T>(C2R_DOT2, wo, p->stream, a, b); }));
    return FILL_OK;
  };

  // z_0, w_0 and the partials of the first scalar step
  if (!pre) {
    RowArgs<T> a0 = row_base<T>(p, np);
    a0.v1 = v.r;
    a0.part0 = rrb[0];
    a0.part1 = p->part1;
    HIP_TRY(launch_xr<T>(true, a0, nb, p->stream));
  }
  {
    RowArgs<T> ai = row_base<T>(p, np);
    ai.v0 = v.r;
    FILL_TRY(timed_launch<T>(p, FILL_K_R2C, [&](hipEvent_t a, hipEvent_t b) { return launch_r2c<T>(R2C_COMPACT, ai, p->stream, a, b); }));
    FILL_TRY(tail(nullptr));
  }

  RowArgs<T> up[2];
  for (int par = 0; par < 2; ++par) {
    RowArgs<T>& u = up[par];
    u = row_base<T>(p, np);
    u.v0 = v.x;
    u.v1 = v.r;
    u.v2 = v.p;
    u.v3 = v.q;
    u.v4 = pre ? v.z : nullptr;
    u.v5 = v.w;
    u.sc = p->sc;
    u.nred = nb;
    u.parity = par;
    u.red0 = pre ? p->part0 : rrb[par];
    u.red1 = pre ? p->part1 : rrb[par];
    u.red2 = p->part2;
    u.part0 = pre ? nullptr : rrb[par ^ 1];
    u.hist = hist;
    u.hist_cap = p->hist_cap;
  }
  auto chunk = [&](int len) -> int {
    for (int k = 0; k < len; ++k) {
      const RowArgs<T>& u = up[k & 1];
      FILL_TRY(timed_launch<T>(p, FILL_K_R2C, [&](hipEvent_t a, hipEvent_t b) { return launch_r2c<T>(R2C_CG1UPDATE, u, p->stream, a, b); }));
      FILL_TRY(tail(p->sc));
    }
    return FILL_OK;
  };
  auto exec = [&](int len, hipGraphExec_t* out) -> int {
    *out = nullptr;
    if (p->use_graph && p->timed_kernel < 0)
      FILL_TRY(chunk_graph(p, sizeof(T) == 4, mode + 4, hist != nullptr, len, [&]() { return chunk(len); }, out));
    return FILL_OK;
  };
  if (fixed > 0) FILL_TRY(chunk(fixed));
  else {
    std::vector<int> iters, status;
    FILL_TRY(run_chunks(p, kChunk, kChunk, chunk, exec, nullptr, nb, iters, status));
  }
  p->after = {nullptr, nb, record};  // accounted for with the caller's update of u
  return FILL_OK;
}

// Inner preconditioned CG for every active problem on A d = r (r in v.r with
// ||r|| = 1, d in v.x; x and p are zero on entry); tolerances, caps and the
// active set are in the device parameters.  fixed > 0: exactly `fixed`
// iterations are enqueued (problems that converge earlier stop on the
// device), with no host interaction; else chunks run until the host sees
// every problem done.  Either way the control kernel then accounts for the
// solve in the device refinement state.
template <typename T>
int inner_pcg(fill_plan p, bool record, int fixed) {
  if (p->cg_variant == FILL_CG_SINGLE_REDUCTION && p->precond != FILL_PRECOND_BLOCK)
    return inner_pcg_cg1<T>(p, record, fixed);
  Vecs<T>& v = TypeSel<T>::vecs(p);
  const int nb = TypeSel<T>::nblk(p), np = p->nprob;
  const T* Dinv = TypeSel<T>::Dinv(p);
  const int mode = p->precond;
  double* hist = record && p->hist_cap > 0 ? p->hist : nullptr;
  // r holds the scaled residual and x = p = 0 (the caller's scale pass)

  // z = M^-1 r: E (E r), Px C Px r, or r without a preconditioner; the
  // partial sums (r.z, r.r) feed the first iteration
  if (mode != FILL_PRECOND_NONE) {
    RowArgs<T> a_in = row_base<T>(p, np), a_mid = row_base<T>(p, np), a_out = row_base<T>(p, np);
    a_in.v0 = v.r;
    a_out.v0 = v.z;
    a_out.v1 = v.r;
    a_out.part0 = p->part0;
    a_out.part1 = p->part1;
    if (mode == FILL_PRECOND_SPLIT) FILL_TRY(apply_EE<T>(p, R2C_COMPACT, a_in, a_mid, a_out, nullptr));
    else if (mode == FILL_PRECOND_BLOCK) FILL_TRY(block_apply<T>(p, v.r, v.z, p->part0, p->part1, nullptr));
    else FILL_TRY(apply3<T>(p, R2C_COMPACT, a_in, TypeSel<T>::Dfull(p), C2R_DOT2, a_out, nullptr));
  } else {
    RowArgs<T> a0 = row_base<T>(p, np);
    a0.v1 = v.r;
    a0.part0 = p->part0;
    a0.part1 = p->part1;
    HIP_TRY(launch_xr<T>(true, a0, nb, p->stream));
  }

  // Iteration k (parity k % 2), all scalars on the device:
  //   q = A p, with beta = (r.z)/rho and p = z + beta p fused in front
  //       (partials of r.z, r.r from the previous E E r pass), p.q behind;
  //   z = E E r, with alpha = rho/(p.q), x += alpha p, r -= alpha q fused in
  //       front, r.z and r.r behind.
  //   With M^-1 = Px C Px the second half is one apply (table P);
  //   without a preconditioner it is one vector-update pass (z = r: r.z = r.r).
  RowArgs<T> pa_in[2], e_in[2], xr[2];
  RowArgs<T> pa_out = row_base<T>(p, np), e_mid = row_base<T>(p, np), e_out = row_base<T>(p, np);
  for (int par = 0; par < 2; ++par) {
    pa_in[par] = row_base<T>(p, np);
    pa_in[par].v0 = mode != FILL_PRECOND_NONE ? v.z : v.r;
    pa_in[par].v1 = v.p;
    pa_in[par].sc = p->sc;
    pa_in[par].red0 = p->part0;
    pa_in[par].red1 = p->part1;
    pa_in[par].nred = nb;
    pa_in[par].parity = par;
    e_in[par] = row_base<T>(p, np);
    e_in[par].v0 = v.x;
    e_in[par].v1 = v.r;
    e_in[par].v2 = v.p;
    e_in[par].v3 = v.q;
    e_in[par].sc = p->sc;
    e_in[par].red0 = p->part2;
    e_in[par].nred = nb;
    e_in[par].parity = par;
    pa_in[par].hist = e_in[par].hist = hist;
    pa_in[par].hist_cap = e_in[par].hist_cap = p->hist_cap;
    xr[par] = e_in[par];
    xr[par].part0 = p->part0;
    xr[par].part1 = p->part1;
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

  auto chunk = [&](int len) -> int {
    for (int k = 0; k < len; ++k) {
      const int par = k & 1;
      FILL_TRY(apply3<T>(p, R2C_PUPDATE, pa_in[par], Dinv, C2R_COMPACT, pa_out, p->sc, p->skew));
      if (mode == FILL_PRECOND_SPLIT) FILL_TRY(apply_EE<T>(p, R2C_XRUPDATE, e_in[par], e_mid, e_out, p->sc));
      else if (mode == FILL_PRECOND_CXX)
        FILL_TRY(apply3<T>(p, R2C_XRUPDATE, e_in[par], TypeSel<T>::Dfull(p), C2R_DOT2, e_out, p->sc));
      else if (mode == FILL_PRECOND_BLOCK) {
        RowArgs<T> u = e_in[par];  // x += alpha p, r -= alpha q; the r.z, r.r partials come after M^-1
        HIP_TRY(launch_xr<T>(false, u, nb, p->stream));
        FILL_TRY(block_apply<T>(p, v.r, v.z, p->part0, p->part1, p->sc));
      } else HIP_TRY(launch_xr<T>(false, xr[par], nb, p->stream));
    }
    return FILL_OK;
  };
  // Every argument of the chunk is a plan-owned pointer or a constant, so the
  // chunk is captured once and replayed (not while a kernel is being timed:
  // timed launches carry their own events).
  auto exec = [&](int len, hipGraphExec_t* out) -> int {
    *out = nullptr;
    if (p->use_graph && p->timed_kernel < 0)
      FILL_TRY(chunk_graph(p, sizeof(T) == 4, mode, hist != nullptr, len, [&]() { return chunk(len); }, out));
    return FILL_OK;
  };
  // chunk lengths: even (the rho parity), the first one the length of the
  // same refinement step's last inner solve
  if (fixed > 0) {
    FILL_TRY(chunk(fixed));
  } else {
    const int len1 = mode == FILL_PRECOND_BLOCK ? kChunkBlock : kChunk;
    const int pred = p->pred_iters[sizeof(T) == 4][std::min(p->cur_outer, 3)];
    const int len0 = pred > 0 ? std::min(16, std::max(2, (pred + 1) / 2 * 2)) : len1;
    std::vector<int> iters, status;
    FILL_TRY(run_chunks(p, len0, len1, chunk, exec, p->part1, nb, iters, status));
    int mx = 0;
    for (int b = 0; b < np; ++b) mx = std::max(mx, iters[b]);
    p->pred_iters[sizeof(T) == 4][std::min(p->cur_outer, 3)] = mx;
  }
  p->after = {p->part1, nb, record};  // accounted for with the caller's update of u
  return FILL_OK;
}

// One refinement step for every active problem (Sec. 2.4 solve with FP64
// true residuals): r = res / ||res|| (v itself at the first step, which also
// clears u), the inner CG (host-checked chunks, or exactly `fixed`
// iterations), u += ||res|| d, the FP64 true residual res = v - A u, its
// per-problem norms and the device's decision of the next step.  Every
// scalar is read from and written to the device state: nothing here waits
// for the host.
int refine_step(fill_plan p, bool first, int fixed, bool warm = false) {
  const int np = p->nprob;
  // from v with u = 0, unless a warm start has put u and res = v - A u in place
  const bool from_v = first && !warm;
  if (p->prec == FILL_PREC_FP64) {
    HIP_TRY(launch_scale_init_f64(p->v64.r, from_v ? p->b : p->res, p->dp.scale, p->comp_off, p->v64.x, p->v64.p,
                                  from_v ? p->u : nullptr, p->n_m_max, np, p->stream));
    FILL_TRY(inner_pcg<double>(p, first, fixed));
    HIP_TRY(launch_axpy_after_f64(p->u, p->v64.x, p->comp_off, refine_args(p), p->after.part, p->after.nb,
                                  (size_t)p->ny, p->after.first, p->n_m_max, p->stream));
  } else {
    HIP_TRY(launch_scale_init_f32(p->v32.r, from_v ? p->b : p->res, p->dp.scale, p->comp_off, p->v32.x, p->v32.p,
                                  from_v ? p->u : nullptr, p->n_m_max, np, p->stream));
    FILL_TRY(inner_pcg<float>(p, first, fixed));
    HIP_TRY(launch_axpy_after_f32(p->u, p->v32.x, p->comp_off, refine_args(p), p->after.part, p->after.nb,
                                  (size_t)p->ny, p->after.first, p->n_m_max, p->stream));
  }
  RowArgs<double> ai = row_base<double>(p, np), ao = row_base<double>(p, np);
  ai.v0 = p->u;
  ao.v0 = p->res;
  ao.v1 = p->b;
  ao.part0 = p->part0;
  FILL_TRY(apply3<double>(p, R2C_COMPACT, ai, p->Dinv64, C2R_RESID, ao, nullptr));
  HIP_TRY(launch_ctl(refine_args(p), p->part0, (size_t)p->ny, p->nblk64, false, p->stream));
  return FILL_OK;
}

// The refinement state on the host (synchronises the stream).
int read_state(fill_plan p) {
  HIP_TRY(hipMemcpyAsync(p->h_st, p->st, p->nprob * sizeof(SolveState), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return FILL_OK;
}

// Every problem done, by the host copy of the state.
bool all_done(fill_plan p) {
  for (int b = 0; b < p->nprob; ++b)
    if (!p->h_st[b].done) return false;
  return true;
}

// Host-driven refinement: with the state on the host, run steps (each read
// back) until every problem is done.  first: no step has run yet in this
// solve (the first one clears u and records the CG coefficients).
int refine_host(fill_plan p, bool first, bool warm = false) {
  if (first && !warm && all_done(p))  // nothing to solve: u = 0
    HIP_TRY(hipMemsetAsync(p->u, 0, (size_t)std::max(p->n_m_total, 1) * sizeof(double), p->stream));
  for (int pass = 0; !all_done(p); ++pass) {
    p->cur_outer = pass;
    FILL_TRY(refine_step(p, first, 0, warm));
    first = false;
    FILL_TRY(read_state(p));
  }
  return FILL_OK;
}

// Per-call settings of the control kernels (uploaded with the parameters).
void set_cfg(fill_plan p, double rtol) {
  SolveCfg& c = *p->hp.cfg;
  c.rtol = rtol;
  c.inner_tol = p->inner_tol32;
  c.max_iter = p->max_iter;
  c.max_outer = kMaxOuter;
  c.fp64 = p->prec == FILL_PREC_FP64 ? 1 : 0;
  c.pad = 0;
}

// Statistics and status from the host copy of the final state; the step
// counts become the prediction for the next solve of the same key.
int finish_solve(fill_plan p, int key) {
  const int np = p->nprob;
  int worst = FILL_OK, R = 0;
  int L[kStateIts] = {};
  for (int b = 0; b < np; ++b) {
    const SolveState& s = p->h_st[b];
    fill_stats& ps = p->pstats[b];
    ps.iters_inner = s.total;
    ps.iters_outer = s.outer;
    ps.rel_resid = s.bnorm2 > 0.0 ? std::sqrt(s.rnorm2 / s.bnorm2) : 0.0;
    ps.status = s.status == -6 ? FILL_ENOTSPD : s.status == -4 ? FILL_ENOCONV : FILL_OK;
    ps.whole_graph = p->last_whole_graph;
    if (b < (int)p->hist_n.size()) p->hist_n[b] = s.outer > 0 ? std::min(s.first_iters, p->hist_cap) : 0;
    if (ps.status == FILL_ENOTSPD) worst = FILL_ENOTSPD;
    else if (ps.status == FILL_ENOCONV && worst == FILL_OK) worst = FILL_ENOCONV;
    R = std::max(R, s.outer);
    for (int j = 0; j < std::min(s.outer, kStateIts); ++j) L[j] = std::max(L[j], s.its[j]);
  }
  p->pred_key = key;
  p->pred_R = R;
  std::memcpy(p->pred_L, L, sizeof(L));
  if (worst == FILL_ENOTSPD) return fail(FILL_ENOTSPD, "CG breakdown (p.Ap <= 0 or r.Mr <= 0) or non-finite residual");
  if (worst == FILL_ENOCONV) return fail(FILL_ENOCONV, "no convergence to the requested true residual");
  return FILL_OK;
}

bool size_ok(int n) {
  switch (n) {
    case 16: case 32: case 64: case 96: case 128: case 192: case 256: case 384: case 512: case 768: case 1024:
    case 1536: case 2048: case 3072: case 4096:
      return true;
  }
  return false;
}

// Twiddle table of the radix plan PL in the per-pass LO/HI layout the kernels
// read (see fft_device.hpp), each entry exp(-2 pi i t/N) evaluated in long
// double and rounded to the table's precision.
template <typename PL, typename C> void make_twiddles(std::vector<C>& w) {
  constexpr int N = PL::N;
  w.assign(std::max(tw_elems<PL>(), 1), C{1, 0});
  const long double pi = 3.141592653589793238462643383279502884L;
  auto put = [&](int idx, long long t) {
    t %= N;
    const long double a = 2.0L * pi * (long double)t / (long double)N;
    const double c = (double)cosl(a), sn = (double)-sinl(a);
    w[idx] = C{(decltype(C{}.x))c, (decltype(C{}.x))sn};
  };
  for (int p = 0; p < PL::NP; ++p) {
    const int ns = pass_ns<PL>(p);
    if (ns == 1) continue;
    const int R = PL::radix(p), S = N / (ns * R), off = tw_pass_off<PL>(p);
    for (int i = 0; i < R; ++i)
      for (int klo = 0; klo < 16; ++klo) put(off + 16 * i + klo, (long long)i * klo * S);
    if (ns > 16)
      for (int i = 0; i < R; ++i)
        for (int khi = 0; khi < ns / 16; ++khi) put(off + 16 * R + i * (ns / 16) + khi, 16LL * i * khi * S);
  }
}

// Twiddle tables of the plans that the pass kind `pass` uses at length n in
// FP64 and in FP32 (the two precisions may use different plans).
int twiddles(int n, int pass, std::vector<double2>& w64, std::vector<float2>& w32) {
  switch (n) {
#define FILL_CASE(nn)                                                  \
  case nn:                                                             \
    if (pass == kRowPass) {                                            \
      make_twiddles<FFTPlanFor<double, nn, kRowPass>>(w64);            \
      make_twiddles<FFTPlanFor<float, nn, kRowPass>>(w32);             \
    } else {                                                           \
      make_twiddles<FFTPlanFor<double, nn, kColPass>>(w64);            \
      make_twiddles<FFTPlanFor<float, nn, kColPass>>(w32);             \
    }                                                                  \
    return FILL_OK;
    FILL_FOR_EACH_N(FILL_CASE)
#undef FILL_CASE
  }
  return fail(FILL_EUNSUPPORTED_SIZE, "no FFT plan for length " + std::to_string(n));
}

// Tables 1/(P N) and sqrt(P)/N, transposed (spectral column kx contiguous in ky).
// Every table is checked before anything is uploaded, and the host copy hpk
// changes only after the upload succeeded: a rejected spectrum leaves the
// plan's spectrum as it was.
int upload_pk(fill_plan p, const double* Pk, int npk) {
  const int nx = p->nx, ny = p->ny, nc = p->ncol;
  const size_t nt = p->nt;
  for (int k = 0; k < npk; ++k) {
    const double* P0 = Pk + (size_t)k * ny * nc;
    for (int iy = 0; iy < ny; ++iy)
      for (int ix = 0; ix < nc; ++ix) {
        const double P = P0[(size_t)iy * nc + ix];
        if (!(P > 0.0) || !std::isfinite(P))
          return fail(FILL_ENOTSPD, "Pk[" + std::to_string(k) + "][" + std::to_string(iy) + "," +
                                        std::to_string(ix) + "] = " + std::to_string(P) +
                                        " is not positive and finite");
      }
  }
  std::vector<double> inv(nt), half(nt), full(nt);
  std::vector<float> inv32(nt), half32(nt), full32(nt);
  const double scale = 1.0 / ((double)nx * (double)ny);
  p->hpk.clear();  // until every table is on the device, no host copy is current
  for (int k = 0; k < npk; ++k) {
    const double* P0 = Pk + (size_t)k * ny * nc;
    for (int iy = 0; iy < ny; ++iy) {
      for (int ix = 0; ix < nc; ++ix) {
        const double P = P0[(size_t)iy * nc + ix];
        const size_t o = (size_t)ix * ny + iy;
        inv[o] = scale / P;
        half[o] = scale * std::sqrt(P);
        full[o] = scale * P;
        inv32[o] = (float)inv[o];
        half32[o] = (float)half[o];
        full32[o] = (float)full[o];
      }
    }
    HIP_TRY(hipMemcpy(p->Dinv64 + k * nt, inv.data(), nt * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->Dhalf64 + k * nt, half.data(), nt * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->Dinv32 + k * nt, inv32.data(), nt * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->Dhalf32 + k * nt, half32.data(), nt * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->Dfull64 + k * nt, full.data(), nt * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->Dfull32 + k * nt, full32.data(), nt * sizeof(float), hipMemcpyHostToDevice));
  }
  p->hpk.assign(Pk, Pk + (size_t)npk * nt);
  return FILL_OK;
}

int plan_build(fill_plan p, const uint8_t* mask, const double* Pk) {
  const int nx = p->nx, ny = p->ny, np = p->nprob;
  const size_t npix = p->npix, nt = p->nt;
  // masks -> compact index (row-major per problem) and per-row offsets
  std::vector<int> pos, row_off((size_t)np * (ny + 1), 0);
  std::vector<uint8_t> m01(npix * np);
  p->n_m.assign(np, 0);
  p->coff.assign(np + 1, 0);
  // compact vectors are indexed with 32-bit ints in the kernels
  size_t total = 0;
  for (size_t i = 0; i < npix * np; ++i) total += mask[i] != 0;
  if (total > (size_t)INT32_MAX - 1) return fail(FILL_EINVAL, "more than 2^31 masked pixels in one plan");
  pos.reserve(total);
  for (int b = 0; b < np; ++b) {
    p->coff[b] = (int)pos.size();
    for (int y = 0; y < ny; ++y) {
      row_off[(size_t)b * (ny + 1) + y] = (int)pos.size() - p->coff[b];
      for (int x = 0; x < nx; ++x) {
        const size_t i = (size_t)y * nx + x;
        const bool m = mask[(size_t)b * npix + i] != 0;
        m01[(size_t)b * npix + i] = m ? 1 : 0;
        if (m) pos.push_back((int)i);
      }
    }
    p->n_m[b] = (int)pos.size() - p->coff[b];
    row_off[(size_t)b * (ny + 1) + ny] = p->n_m[b];
  }
  p->coff[np] = (int)pos.size();
  p->n_m_total = (int)pos.size();
  p->n_m_max = *std::max_element(p->n_m.begin(), p->n_m.end());
  const int nm = std::max(p->n_m_total, 1);
  FILL_TRY(dalloc(p, &p->mask, npix * np));
  FILL_TRY(dalloc(p, &p->pos, nm));
  FILL_TRY(dalloc(p, &p->row_off, (size_t)np * (ny + 1)));
  FILL_TRY(dalloc(p, &p->comp_off, np + 1));
  FILL_TRY(dalloc(p, &p->Dinv64, nt * p->npk));
  FILL_TRY(dalloc(p, &p->Dhalf64, nt * p->npk));
  FILL_TRY(dalloc(p, &p->Dinv32, nt * p->npk));
  FILL_TRY(dalloc(p, &p->Dhalf32, nt * p->npk));
  FILL_TRY(dalloc(p, &p->Dfull64, nt * p->npk));
  FILL_TRY(dalloc(p, &p->Dfull32, nt * p->npk));
  std::vector<double2> twx64, twy64;
  std::vector<float2> twx32, twy32;
  FILL_TRY(twiddles(nx, kRowPass, twx64, twx32));
  FILL_TRY(twiddles(ny, kColPass, twy64, twy32));
  FILL_TRY(dalloc(p, &p->twx64, twx64.size()));
  FILL_TRY(dalloc(p, &p->twy64, twy64.size()));
  FILL_TRY(dalloc(p, &p->twx32, twx32.size()));
  FILL_TRY(dalloc(p, &p->twy32, twy32.size()));
  double2* xt = nullptr;
  FILL_TRY(dalloc(p, &xt, nt * np));
  p->Xt = xt;
  FILL_TRY(dalloc(p, &p->tfull, npix * np));
  FILL_TRY(dalloc(p, &p->b, nm));
  FILL_TRY(dalloc(p, &p->u, nm));
  FILL_TRY(dalloc(p, &p->res, nm));
  for (double** q : {&p->v64.x, &p->v64.r, &p->v64.z, &p->v64.p, &p->v64.q, &p->v64.t, &p->v64.w})
    FILL_TRY(dalloc(p, q, nm));
  for (float** q : {&p->v32.x, &p->v32.r, &p->v32.z, &p->v32.p, &p->v32.q, &p->v32.t, &p->v32.w})
    FILL_TRY(dalloc(p, q, nm));
  FILL_TRY(dalloc(p, &p->part0, (size_t)ny * np));
  FILL_TRY(dalloc(p, &p->part1, (size_t)ny * np));
  FILL_TRY(dalloc(p, &p->part2, (size_t)ny * np));
  FILL_TRY(dalloc(p, &p->part3, (size_t)ny * np));
  FILL_TRY(dalloc(p, &p->dsum, np));
  FILL_TRY(dalloc(p, &p->sc, np));
  // per-call parameter block: same layout on host (pinned) and device
  const size_t n8 = (size_t)np * 8;
  p->par_bytes = 8 * n8 + sizeof(SolveCfg);
  char* dpar = nullptr;
  FILL_TRY(dalloc(p, &dpar, p->par_bytes));
  p->par_dev = dpar;
  HIP_TRY(hipHostMalloc(&p->par_host, p->par_bytes, hipHostMallocDefault));
  std::memset(p->par_host, 0, p->par_bytes);
  auto carve = [&](char* base, Params& q) {
    q.scale = reinterpret_cast<double*>(base + 0 * n8);
    q.unscale = reinterpret_cast<double*>(base + 1 * n8);
    q.tol2 = reinterpret_cast<double*>(base + 2 * n8);
    q.cap = reinterpret_cast<int*>(base + 3 * n8);
    q.active = reinterpret_cast<int*>(base + 4 * n8);
    q.in_tab = reinterpret_cast<const double**>(base + 5 * n8);
    q.out_tab = reinterpret_cast<double**>(base + 6 * n8);
    q.seeds = reinterpret_cast<uint64_t*>(base + 7 * n8);
    q.cfg = reinterpret_cast<SolveCfg*>(base + 8 * n8);
  };
  carve(dpar, p->dp);
  carve(static_cast<char*>(p->par_host), p->hp);
  FILL_TRY(dalloc(p, &p->st, np));
  HIP_TRY(hipHostMalloc((void**)&p->h_st, np * sizeof(SolveState), hipHostMallocDefault));
  std::memset(p->h_st, 0, np * sizeof(SolveState));
  HIP_TRY(hipHostMalloc((void**)&p->h_sc, np * sizeof(CGScalars), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void**)&p->h_sum, np * sizeof(double), hipHostMallocDefault));
  p->pstats.assign(np, fill_stats{});
  for (int b = 0; b < np; ++b) p->pstats[b].n_masked = p->n_m[b];

  HIP_TRY(hipMemcpy(p->mask, m01.data(), npix * np, hipMemcpyHostToDevice));
  p->hmask = m01;
  if (!pos.empty()) HIP_TRY(hipMemcpy(p->pos, pos.data(), pos.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->row_off, row_off.data(), row_off.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->comp_off, p->coff.data(), (np + 1) * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->twx64, twx64.data(), twx64.size() * sizeof(double2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->twx32, twx32.data(), twx32.size() * sizeof(float2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->twy64, twy64.data(), twy64.size() * sizeof(double2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->twy32, twy32.data(), twy32.size() * sizeof(float2), hipMemcpyHostToDevice));
  return upload_pk(p, Pk, p->npk);
}

int check_maps(fill_plan p, const double* const* d, double* const* x) {
  if (!d || !x) return fail(FILL_EINVAL, "NULL map array");
  for (int b = 0; b < p->nprob; ++b) {
    if (!d[b] || !x[b]) return fail(FILL_EINVAL, "NULL map for problem " + std::to_string(b));
    if ((const void*)d[b] == (const void*)x[b]) return fail(FILL_EINVAL, "x_out aliases d_obs");
  }
  return FILL_OK;
}

// The first passes of a solve: x_out and t = Py (d - s) (or Py d for the
// mean), then the right-hand side v = -Px C^-1 t with its norms, and the
// device's decision of the first refinement step.  Per-call maps and seeds
// come from the parameter tables, so the passes can be captured.
int enqueue_start(fill_plan p, bool mean) {
  const int np = p->nprob;
  if (mean) {
    HIP_TRY(launch_mean_prep(p->dp.out_tab, p->tfull, p->dp.in_tab, p->mask, p->npix, np, p->stream));
  } else {
    // s = C^{1/2} w; x_out = mask ? s : d; t = mask ? 0 : d - s
    RowArgs<double> ai = row_base<double>(p, np), ao = row_base<double>(p, np);
    ai.seeds = p->dp.seeds;
    ai.stream = kRealizationStream;
    ao.fin_tab = p->dp.in_tab;
    ao.fout_tab = p->dp.out_tab;
    ao.full_in = p->tfull;  // non-null: the observed-data branch (the maps come from the tables)
    ao.full_out2 = p->tfull;
    FILL_TRY(apply3<double>(p, R2C_NOISE, ai, p->Dhalf64, C2R_REALIZE, ao, nullptr));
  }
  RowArgs<double> ai = row_base<double>(p, np), ao = row_base<double>(p, np);
  ai.full_in = p->tfull;
  ao.v0 = p->b;
  ao.scale = -1.0;
  ao.part0 = p->part0;
  FILL_TRY(apply3<double>(p, R2C_FULL, ai, p->Dinv64, C2R_COMPACT, ao, nullptr));
  HIP_TRY(launch_ctl(refine_args(p), p->part0, (size_t)p->ny, p->nblk64, true, p->stream));
  return FILL_OK;
}

// Key of the predictions: operation, preconditioner, recurrence.
int solve_key(fill_plan p, bool mean) { return (mean ? 1 : 0) + 2 * p->precond + 16 * p->cg_variant; }

// Whether this solve can run as one captured graph: the same kind of solve
// ran last on this plan, with at most kStateIts refinement steps and few
// iterations (with hundreds of iterations per solve the host's checks cost
// nothing that matters), graphs are on and no kernel is being timed.  The
// single-reduction recurrence clears a vector with a memset at its start,
// which is kept out of graphs.
bool whole_graph_ok(fill_plan p, bool mean) {
  if (!p->use_graph || p->timed_kernel >= 0 || p->n_m_total == 0 || p->ws_iters > 0) return false;
  if (p->cg_variant == FILL_CG_SINGLE_REDUCTION && p->precond != FILL_PRECOND_BLOCK) return false;
  if (p->pred_key != solve_key(p, mean) || p->pred_R < 1 || p->pred_R > kStateIts) return false;
  int sum = 0;
  for (int j = 0; j < p->pred_R; ++j) {
    if (p->pred_L[j] < 1) return false;
    sum += p->pred_L[j];
  }
  return sum <= 128;
}

// The predicted solve on p->stream: start passes, pred_R refinement steps of
// pred_L[j] inner iterations each, and the assembly x_out += u, which runs
// only if every problem is done by then (otherwise the host continues).
int enqueue_whole_solve(fill_plan p, bool mean) {
  FILL_TRY(enqueue_start(p, mean));
  for (int j = 0; j < p->pred_R; ++j) {
    p->cur_outer = j;
    FILL_TRY(refine_step(p, j == 0, p->pred_L[j]));
  }
  HIP_TRY(launch_scatter_add(p->dp.out_tab, p->u, p->pos, p->comp_off, p->n_m_max, p->nprob, p->stream, p->st));
  return FILL_OK;
}

// The whole solve as one graph (captured on first use per key and step
// lengths): start passes, pred_R refinement steps of pred_L[j] inner
// iterations each, and the assembly x_out += u, which runs only if every
// problem is done by then (otherwise the host continues the refinement).
int whole_graph(fill_plan p, bool mean, hipGraphExec_t* out) {
  std::vector<int> key = {mean ? 1 : 0, p->prec, p->precond, p->cg_variant, p->hist_cap > 0 ? 1 : 0, p->pred_R};
  for (int j = 0; j < p->pred_R; ++j) key.push_back(p->pred_L[j]);
  auto it = p->solve_graphs.find(key);
  if (it != p->solve_graphs.end()) {
    *out = it->second.second;
    return FILL_OK;
  }
  if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  const hipStream_t saved = p->stream;
  p->stream = p->cap_stream;
  const hipError_t e0 = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
  const int rc = e0 == hipSuccess ? enqueue_whole_solve(p, mean) : FILL_OK;
  hipGraph_t g = nullptr;
  const hipError_t e1 = e0 == hipSuccess ? hipStreamEndCapture(p->cap_stream, &g) : hipSuccess;
  p->stream = saved;
  if (e0 != hipSuccess) return fail(FILL_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e0));
  if (rc < 0 || e1 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (rc < 0) return rc;
    return fail(FILL_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e1));
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(FILL_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
  }
  p->solve_graphs[key] = {g, ex};
  *out = ex;
  return FILL_OK;
}

int laplace_run(fill_plan p, const double* in, int nkernels, double r0, double ratio, int iters, const double** out);

// Warm start of the solve (Sec. 6.1, 6.3: the far interior of a wide cut is
// nearly harmonic): the kernel Laplace relaxation of t = Py (d - s) (or Py d)
// gives u on the masked pixels, then res = v - A u (FP64) and the device's
// decision of the first step from it.  One-problem plans.
int warm_start(fill_plan p) {
  const double* lap = nullptr;
  FILL_TRY(laplace_run(p, p->tfull, p->ws_k, p->ws_r0, p->ws_ratio, p->ws_iters, &lap));
  HIP_TRY(launch_gather(p->u, lap, p->pos, p->n_m[0], p->stream));
  RowArgs<double> ai = row_base<double>(p, 1), ao = row_base<double>(p, 1);
  ai.v0 = p->u;
  ao.v0 = p->res;
  ao.v1 = p->b;
  ao.part0 = p->part0;
  FILL_TRY(apply3<double>(p, R2C_COMPACT, ai, p->Dinv64, C2R_RESID, ao, nullptr));
  HIP_TRY(launch_ctl(refine_args(p), p->part0, (size_t)p->ny, p->nblk64, false, p->stream));
  return FILL_OK;
}

// After the parameters are uploaded: the solve (one graph replay when the
// previous solve's step counts are known, else step by step with the host
// reading the state after each), then the assembly x_out += u.
int run_solve(fill_plan p, bool mean) {
  const bool graph = whole_graph_ok(p, mean);
  p->last_whole_graph = 0;
  if (graph) {
    hipGraphExec_t ex = nullptr;
    FILL_TRY(whole_graph(p, mean, &ex));
    HIP_TRY(hipGraphLaunch(ex, p->stream));
  } else {
    FILL_TRY(enqueue_start(p, mean));
  }
  const bool warm = !graph && p->ws_iters > 0;
  if (warm) FILL_TRY(warm_start(p));
  FILL_TRY(read_state(p));
  const bool done = all_done(p);
  p->last_whole_graph = graph && done ? 1 : 0;
  if (!graph || !done) {
    // not every problem finished inside the graph (or no graph): continue
    // step by step, then assemble
    FILL_TRY(refine_host(p, !graph, warm));
    HIP_TRY(launch_scatter_add(p->dp.out_tab, p->u, p->pos, p->comp_off, p->n_m_max, p->nprob, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  return finish_solve(p, solve_key(p, mean));
}

void finish_stats(fill_plan p, int st, double ms) {
  fill_stats agg{0, 0, p->n_m_total, st, 0.0, ms, p->last_whole_graph};
  for (int b = 0; b < p->nprob; ++b) {
    p->pstats[b].solve_ms = ms;
    p->pstats[b].whole_graph = p->last_whole_graph;
    agg.iters_inner = std::max(agg.iters_inner, p->pstats[b].iters_inner);
    agg.iters_outer = std::max(agg.iters_outer, p->pstats[b].iters_outer);
    agg.rel_resid = std::max(agg.rel_resid, p->pstats[b].rel_resid);
  }
  p->stats = agg;
}

using clk = std::chrono::steady_clock;

// Checks of a call and its parameters into the plan's pinned staging block
// (after the previous call's upload has completed).
int prepare_call(fill_plan p, const double* const* d, const uint64_t* seeds, double* const* x, double rtol,
                 bool mean) {
  if (!p) return fail(FILL_EINVAL, "NULL plan");
  if (!(rtol > 0.0)) return fail(FILL_EINVAL, "rtol must be > 0");
  FILL_TRY(check_maps(p, d, x));
  if (!mean && !seeds) return fail(FILL_EINVAL, "NULL seeds");
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (int b = 0; b < p->nprob; ++b) {
    p->pstats[b] = fill_stats{0, 0, p->n_m[b], 0, 0.0, 0.0};
    p->hp.in_tab[b] = d[b];
    p->hp.out_tab[b] = x[b];
    p->hp.seeds[b] = mean ? 0 : seeds[b];
  }
  set_cfg(p, rtol);
  return FILL_OK;
}

int realize_impl(fill_plan p, const double* const* d, const uint64_t* seeds, double* const* x, double rtol,
                 bool mean) {
  g_last_error.clear();
  const auto t0 = clk::now();
  FILL_TRY(prepare_call(p, d, seeds, x, rtol, mean));
  const int np = p->nprob;
  if (p->n_m_total == 0) {
    p->last_whole_graph = 0;
    for (int b = 0; b < np; ++b)
      HIP_TRY(hipMemcpyAsync(x[b], d[b], p->npix * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    finish_stats(p, FILL_OK, std::chrono::duration<double, std::milli>(clk::now() - t0).count());
    return FILL_OK;
  }
  FILL_TRY(upload_params(p));
  const int st = run_solve(p, mean);
  finish_stats(p, st, std::chrono::duration<double, std::milli>(clk::now() - t0).count());
  return st;
}

template <typename T>
int time_kernel(fill_plan p, int kernel, int reps, double* avg_ms) {
  Vecs<T>& v = TypeSel<T>::vecs(p);
  const size_t vb = (size_t)std::max(p->n_m_total, 1) * sizeof(T);
  HIP_TRY(hipMemsetAsync(v.p, 0, vb, p->stream));
  RowArgs<T> ai = row_base<T>(p, 1), ao = row_base<T>(p, 1);
  ai.v0 = v.p;
  ao.v0 = v.q;
  ao.v1 = v.p;
  ao.part0 = p->part0;
  const ColArgs<T> ca = col_base<T>(p, 1, TypeSel<T>::Dinv(p), nullptr);
  RowArgs<T> am = row_base<T>(p, 1);
  auto launch = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    if (kernel == FILL_K_R2C || kernel == FILL_K_APPLY) e = launch_r2c<T>(R2C_COMPACT, ai, p->stream);
    if (e == hipSuccess && (kernel == FILL_K_COL || kernel == FILL_K_APPLY)) e = launch_col<T>(p->ny, ca, p->stream);
    if (e == hipSuccess && (kernel == FILL_K_C2R || kernel == FILL_K_APPLY))
      e = launch_c2r<T>(C2R_COMPACT, ao, p->stream);
    if (e == hipSuccess && kernel == FILL_K_PROJ) e = launch_proj<T>(false, am, p->stream);
    return e;
  };
  if (kernel >= FILL_K_BAND) {  // block preconditioner kernels, on the CG vectors
    if (!p->blk.built) return fail(FILL_EINVAL, "the block preconditioner is not built");
    FILL_TRY(block_apply<T>(p, v.r, v.z, p->part0, p->part1, nullptr, kernel));  // warm-up
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, p->stream));
    for (int i = 0; i < reps; ++i) FILL_TRY(block_apply<T>(p, v.r, v.z, p->part0, p->part1, nullptr, kernel));
    HIP_TRY(hipEventRecord(e1, p->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
    return FILL_OK;
  }
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

int plan_create_impl(int nx, int ny, int nprob, const uint8_t* masks, const double* Pk, int npk, int prec,
                     void* stream, fill_plan* out);

// ln P(k) piecewise linear in ln k between the band nodes, constant outside;
// k = 0 takes the first band.
double band_lnP(double k, const double* lnk, const double* theta, int nb) {
  if (k <= 0.0) return theta[0];
  const double lk = std::log(k);
  if (lk <= lnk[0]) return theta[0];
  if (lk >= lnk[nb - 1]) return theta[nb - 1];
  int j = int(std::upper_bound(lnk, lnk + nb, lk) - lnk) - 1;
  const double t = (lk - lnk[j]) / (lnk[j + 1] - lnk[j]);
  return (1.0 - t) * theta[j] + t * theta[j + 1];
}

int adjoint_workspace(fill_plan p) {
  if (p->adj_s) return FILL_OK;
  FILL_TRY(dalloc(p, &p->adj_s, p->npix));
  FILL_TRY(dalloc(p, &p->adj_cl, p->npix));
  FILL_TRY(dalloc(p, &p->adj_h, p->npix));
  FILL_TRY(dalloc(p, &p->adj_v, p->npix));
  for (int i = 0; i < 4; ++i) FILL_TRY(dalloc(p, &p->adj_X[i], p->nt));
  FILL_TRY(dalloc(p, &p->adj_G, p->nt));
  FILL_TRY(dalloc(p, &p->adj_Gapi, p->nt));
  return FILL_OK;
}

// Forward 2D FFT of problem b's map, into adjoint spectrum slot `slot`:
// r2c of (mode, args) then the forward-only column pass.
int forward_spectrum(fill_plan p, int b, int mode, const RowArgs<double>& a, int slot) {
  HIP_TRY(launch_r2c<double>(mode, a, p->stream));
  HIP_TRY(launch_col_fwd(p->ny, static_cast<const double2*>(a.Xt), p->adj_X[slot], p->ny, p->nx / 2, p->twy64,
                         p->stream));
  (void)b;
  return FILL_OK;
}

int adjoint_impl(fill_plan p, const double* const* d, const uint64_t* seeds, const double* const* x,
                 const double* const* g, double* const* gy, double* grad_theta, double* grad_logP, double rtol) {
  g_last_error.clear();
  if (!p || !d || !seeds || !x || !g || !gy) return fail(FILL_EINVAL, "NULL argument");
  if (!(rtol > 0.0)) return fail(FILL_EINVAL, "rtol must be > 0");
  if (p->nbands < 1 && grad_theta) return fail(FILL_EINVAL, "grad_theta needs fill_plan_set_bands first");
  const int np = p->nprob;
  for (int b = 0; b < np; ++b)
    if (!d[b] || !x[b] || !g[b] || !gy[b]) return fail(FILL_EINVAL, "NULL map for problem " + std::to_string(b));
  FILL_TRY(adjoint_workspace(p));
  HIP_TRY(hipStreamSynchronize(p->stream));
  const auto t_adj = clk::now();
  for (int b = 0; b < np; ++b) p->hp.in_tab[b] = g[b];
  set_cfg(p, rtol);
  FILL_TRY(upload_params(p));
  // lambda = A^-1 g_x for every problem (the plan's precision, FP64 refinement)
  HIP_TRY(launch_adj_gather(p->b, const_cast<double* const*>(p->dp.in_tab), p->pos, p->comp_off, p->n_m_max, np,
                            p->stream));
  HIP_TRY(launch_cnorm2(p->dsum, p->b, p->comp_off, np, p->stream));
  HIP_TRY(launch_ctl(refine_args(p), p->dsum, 1, 1, true, p->stream));
  FILL_TRY(read_state(p));
  FILL_TRY(refine_host(p, true));
  // (no prediction key: the adjoint solve always runs step by step)
  p->last_whole_graph = 0;
  const int st = finish_solve(p, -2);
  finish_stats(p, st, std::chrono::duration<double, std::milli>(clk::now() - t_adj).count());
  if (st != FILL_OK && st != FILL_ENOCONV) return st;
  if (p->nbands > 0) HIP_TRY(hipMemsetAsync(p->adj_gth, 0, p->nbands * sizeof(double), p->stream));
  for (int b = 0; b < np; ++b) {
    const size_t doff = p->npk > 1 ? (size_t)b * p->nt : 0;
    const double* Dinv = p->Dinv64 + doff;
    const double* Dhalf = p->Dhalf64 + doff;
    double* lam = p->u + p->coff[b];
    // s = C^{1/2} w (problem b's seed)
    RowArgs<double> ai = row_for<double>(p, b), ao = row_for<double>(p, b);
    ai.seed = seeds[b];
    ai.stream = kRealizationStream;
    ao.full_out = p->adj_s;
    ColArgs<double> ca = col_base<double>(p, 1, Dhalf, nullptr);
    ca.Xt = ai.Xt;
    HIP_TRY(launch_r2c<double>(R2C_NOISE, ai, p->stream));
    HIP_TRY(launch_col<double>(p->ny, ca, p->stream));
    HIP_TRY(launch_c2r<double>(C2R_REALIZE, ao, p->stream));
    // cl = C^-1 lambda~ (full map)
    ai = row_for<double>(p, b);
    ai.v0 = lam;
    ao = row_for<double>(p, b);
    ao.full_out = p->adj_cl;
    ca.D = Dinv;
    HIP_TRY(launch_r2c<double>(R2C_COMPACT, ai, p->stream));
    HIP_TRY(launch_col<double>(p->ny, ca, p->stream));
    HIP_TRY(launch_c2r<double>(C2R_FULL, ao, p->stream));
    // dL/dy, h, v
    HIP_TRY(launch_adj_maps(p->mask + (size_t)b * p->npix, g[b], p->adj_cl, x[b], p->adj_s, d[b], gy[b], p->adj_h,
                            p->adj_v, p->npix, p->stream));
    if (!grad_theta && !grad_logP) continue;
    // spectra of h, w, lambda~, v
    RowArgs<double> a = row_for<double>(p, b);
    a.full_in = p->adj_h;
    FILL_TRY(forward_spectrum(p, b, R2C_FULL, a, 0));
    a = row_for<double>(p, b);
    a.seed = seeds[b];
    a.stream = kRealizationStream;
    FILL_TRY(forward_spectrum(p, b, R2C_NOISE, a, 1));
    a = row_for<double>(p, b);
    a.v0 = lam;
    FILL_TRY(forward_spectrum(p, b, R2C_COMPACT, a, 2));
    a = row_for<double>(p, b);
    a.full_in = p->adj_v;
    FILL_TRY(forward_spectrum(p, b, R2C_FULL, a, 3));
    HIP_TRY(launch_spec_grad(p->adj_X[0], p->adj_X[1], p->adj_X[2], p->adj_X[3], Dhalf, Dinv, p->nx, p->ny,
                             p->adj_G, grad_logP ? p->adj_Gapi : nullptr, p->stream));
    if (grad_theta)
      HIP_TRY(launch_band_reduce(p->adj_G, p->nx, p->ny, p->lnk, p->nbands, p->adj_gth, p->stream));
    if (grad_logP)
      HIP_TRY(hipMemcpyAsync(grad_logP + (size_t)b * p->nt, p->adj_Gapi, p->nt * sizeof(double),
                             hipMemcpyDeviceToHost, p->stream));
  }
  if (grad_theta)
    HIP_TRY(hipMemcpyAsync(grad_theta, p->adj_gth, p->nbands * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return st;
}

}  // namespace

namespace {

// Kernel j of the Laplace relaxation: offsets with r_in^2 < dy^2 + dx^2 <= r_out^2.
std::vector<std::pair<int, int>> annulus(double r_in, double r_out) {
  std::vector<std::pair<int, int>> off;
  const int r = (int)std::floor(r_out);
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx) {
      const double d2 = (double)dy * dy + (double)dx * dx;
      if (d2 > r_in * r_in && d2 <= r_out * r_out) off.emplace_back(dy, dx);
    }
  return off;
}

// Kernel spectra (as D tables: real spectrum / N) and per-pixel kernel
// classes for (nkernels, r0, ratio); kept while the parameters repeat.
int laplace_setup(fill_plan p, int nk, double r0, double ratio) {
  if (p->lap_k == nk && p->lap_r0 == r0 && p->lap_ratio == ratio) return FILL_OK;
  const int nx = p->nx, ny = p->ny;
  const size_t npix = p->npix, nt = p->nt;
  FILL_TRY(adjoint_workspace(p));
  if (!p->lap_cls) {
    FILL_TRY(dalloc(p, &p->lap_cls, npix));
    for (int i = 0; i < 3; ++i) FILL_TRY(dalloc(p, &p->lap_x[i], npix));
    FILL_TRY(dalloc(p, &p->lap_pre, (size_t)ny * (nx + 1)));
    FILL_TRY(dalloc(p, &p->lap_hw, (size_t)std::min(nx, ny)));
    FILL_TRY(dalloc(p, &p->lap_touch, npix));
  }
  while ((int)p->lap_tab.size() < nk) {
    double* t = nullptr;
    FILL_TRY(dalloc(p, &t, nt));
    p->lap_tab.push_back(t);
  }
  p->lap_k = 0;  // invalid until complete
  std::vector<double> radii(nk);
  for (int j = 0; j < nk; ++j) radii[j] = r0 * std::pow(ratio, (double)j);
  // spectra: forward FFT of the normalised kernel image
  std::vector<double> img(npix);
  for (int j = 0; j < nk; ++j) {
    const auto off = annulus(j == 0 ? 0.0 : radii[j - 1], radii[j]);
    if (off.empty()) return fail(FILL_EINVAL, "empty Laplace kernel " + std::to_string(j));
    std::fill(img.begin(), img.end(), 0.0);
    const double w = 1.0 / (double)off.size();
    for (const auto& o : off) img[(size_t)((o.first % ny + ny) % ny) * nx + (size_t)((o.second % nx + nx) % nx)] = w;
    HIP_TRY(hipMemcpyAsync(p->adj_h, img.data(), npix * sizeof(double), hipMemcpyHostToDevice, p->stream));
    RowArgs<double> a = row_for<double>(p, 0);
    a.full_in = p->adj_h;
    FILL_TRY(forward_spectrum(p, 0, R2C_FULL, a, 0));
    HIP_TRY(launch_real_scale(p->lap_tab[j], p->adj_X[0], 1.0 / (double)npix, nt, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));  // img is reused
  }
  // classes: the largest j >= 1 whose disk of radius r_j touches no observed pixel, else 0
  int* pre = p->lap_pre;
  int* dhw = p->lap_hw;
  uint8_t* touch = p->lap_touch;
  HIP_TRY(launch_class_init(p->lap_cls, p->mask, npix, p->stream));
  for (int j = 1; j < nk; ++j) {
    const int r = (int)std::floor(radii[j]);
    std::vector<int> hw(2 * r + 1);
    for (int dy = -r; dy <= r; ++dy) {
      int h = (int)std::floor(std::sqrt(std::max(0.0, radii[j] * radii[j] - (double)dy * dy)));
      while ((double)(h + 1) * (h + 1) + (double)dy * dy <= radii[j] * radii[j]) ++h;
      while (h > 0 && (double)h * h + (double)dy * dy > radii[j] * radii[j]) --h;
      hw[dy + r] = h;
    }
    HIP_TRY(hipMemcpyAsync(dhw, hw.data(), hw.size() * sizeof(int), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(launch_strip_flags(p->mask, pre, dhw, r, nx, ny, 0.0, touch, p->stream));
    HIP_TRY(launch_class_raise(p->lap_cls, touch, p->mask, j, npix, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));  // hw is reused
  }
  std::vector<uint8_t> cls(npix);
  HIP_TRY(hipMemcpy(cls.data(), p->lap_cls, npix, hipMemcpyDeviceToHost));
  std::vector<char> seen(nk, 0);
  for (uint8_t c : cls)
    if (c < nk) seen[c] = 1;
  p->lap_used.clear();
  for (int j = 0; j < nk; ++j)
    if (seen[j]) p->lap_used.push_back(j);
  p->lap_k = nk;
  p->lap_r0 = r0;
  p->lap_ratio = ratio;
  return FILL_OK;
}

// Arguments of the Laplace relaxation (one-problem plans; the largest kernel
// must fit the grid).
int laplace_check(fill_plan p, int nkernels, double r0, double ratio, int iters) {
  if (p->nprob != 1) return fail(FILL_EINVAL, "the Laplace relaxation needs a one-problem plan");
  if (nkernels < 1 || nkernels > 16 || !(r0 >= 1.0) || !(ratio > 1.0) || iters < 1)
    return fail(FILL_EINVAL, "need 1 <= nkernels <= 16, r0 >= 1, ratio > 1, iters >= 1");
  const double rmax = r0 * std::pow(ratio, (double)(nkernels - 1));
  if (!(2.0 * std::floor(rmax) + 1.0 <= (double)std::min(p->nx, p->ny)))
    return fail(FILL_EINVAL, "the largest Laplace kernel does not fit the grid");
  return FILL_OK;
}

// `iters` Jacobi sweeps of the kernel relaxation from in (observed pixels
// kept, masked ones from 0); *out points to the plan's buffer holding the
// result (valid until the next relaxation).
int laplace_run(fill_plan p, const double* in, int nkernels, double r0, double ratio, int iters, const double** out) {
  FILL_TRY(laplace_setup(p, nkernels, r0, ratio));
  const size_t npix = p->npix;
  double* a = p->lap_x[0];
  double* b = p->lap_x[1];
  double* avg = p->lap_x[2];
  HIP_TRY(launch_select_observed(a, in, p->mask, npix, p->stream));
  HIP_TRY(hipMemcpyAsync(b, a, npix * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  // Jacobi sweeps: every used kernel's average of the current map, written to its class
  for (int it = 0; it < iters; ++it) {
    for (int j : p->lap_used) {
      RowArgs<double> ai = row_base<double>(p, 1), ao = row_base<double>(p, 1);
      ai.full_in = a;
      ao.full_out = avg;
      FILL_TRY(apply3<double>(p, R2C_FULL, ai, p->lap_tab[j], C2R_FULL, ao, nullptr));
      HIP_TRY(launch_take_class(b, avg, p->lap_cls, j, npix, p->stream));
    }
    std::swap(a, b);
  }
  *out = a;
  return FILL_OK;
}

// Lanczos matrix of k CG steps (Sec. 6.4; CG-Lanczos relation): diagonal
// 1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j.
void lanczos_matrix(const double* al, const double* be, int k, std::vector<double>& d, std::vector<double>& e) {
  d.assign(k, 0.0);
  e.assign(k > 0 ? k - 1 : 0, 0.0);
  for (int j = 0; j < k; ++j) {
    d[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < k) e[j] = std::sqrt(be[j]) / al[j];
  }
}

// Eigenvalues of the symmetric tridiagonal (d, e) below x: the number of
// negative pivots of the LDL^T factorisation of T - x I (Sturm count); a
// pivot smaller than pivmin in magnitude is taken as -pivmin.
int sturm_below(const std::vector<double>& d, const std::vector<double>& e, double x, double pivmin) {
  int c = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    q = d[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

// The i-th smallest eigenvalue (0-based) by bisection inside the Gershgorin interval.
double tridiag_eig(const std::vector<double>& d, const std::vector<double>& e, int i) {
  const int n = (int)d.size();
  double lo = d[0], hi = d[0], emax2 = 0.0;
  for (int j = 0; j < n; ++j) {
    const double r = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < n ? std::fabs(e[j]) : 0.0);
    lo = std::min(lo, d[j] - r);
    hi = std::max(hi, d[j] + r);
    if (j + 1 < n) emax2 = std::max(emax2, e[j] * e[j]);
  }
  const double pivmin = 2.2250738585072014e-308 * std::max(1.0, emax2);
  for (int it = 0; it < 400 && hi - lo > 4.0 * 2.220446049250313e-16 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(d, e, mid, pivmin) > i) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

int read_lanczos(fill_plan p, int problem, std::vector<double>& al, std::vector<double>& be) {
  if (!p) return fail(FILL_EINVAL, "plan is NULL");
  if (problem < 0 || problem >= p->nprob) return fail(FILL_EINVAL, "problem index out of range");
  if (p->hist_cap <= 0 || !p->hist) return fail(FILL_EINVAL, "no coefficient record: call fill_plan_set_lanczos first");
  const int n = (int)p->hist_n.size() > problem ? p->hist_n[problem] : 0;
  std::vector<double> h((size_t)2 * std::max(n, 1));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (n > 0)
    HIP_TRY(hipMemcpy(h.data(), p->hist + (size_t)problem * 2 * p->hist_cap, (size_t)2 * n * sizeof(double),
                      hipMemcpyDeviceToHost));
  al.resize(n);
  be.resize(n > 0 ? n - 1 : 0);
  for (int j = 0; j < n; ++j) al[j] = h[2 * j];
  for (int j = 0; j + 1 < n; ++j) be[j] = h[2 * j + 1];
  return FILL_OK;
}

}  // namespace

namespace {

void group_drop_graph(fill_group g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
  g->key.clear();
}

// The group's graph for the plans' current predictions: one branch per plan
// (forked from and joined into the capture origin), each the plan's whole
// predicted solve on its own capture stream.
int group_graph(fill_group g) {
  std::vector<int> key;
  for (fill_plan p : g->plans) {
    key.push_back((int)p->gen);
    key.push_back(p->hist_cap > 0 ? 1 : 0);
    key.push_back(p->pred_R);
    for (int j = 0; j < p->pred_R; ++j) key.push_back(p->pred_L[j]);
  }
  if (g->exec && key == g->key) return FILL_OK;
  group_drop_graph(g);
  if (!g->cap) HIP_TRY(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
  for (fill_plan p : g->plans)
    if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  const hipError_t e0 = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
  if (e0 != hipSuccess) return fail(FILL_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e0));
  int rc = FILL_OK;
  hipError_t e = hipEventRecord(g->fork, g->cap);
  for (size_t i = 0; i < g->plans.size() && rc == FILL_OK && e == hipSuccess; ++i) {
    fill_plan p = g->plans[i];
    e = hipStreamWaitEvent(p->cap_stream, g->fork, 0);
    if (e != hipSuccess) break;
    const hipStream_t saved = p->stream;
    p->stream = p->cap_stream;
    rc = enqueue_whole_solve(p, false);
    p->stream = saved;
    if (rc != FILL_OK) break;
    e = hipEventRecord(g->join[i], p->cap_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(g->cap, g->join[i], 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t e1 = hipStreamEndCapture(g->cap, &graph);
  if (rc != FILL_OK || e != hipSuccess || e1 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != FILL_OK) return rc;
    return fail(FILL_EHIP, std::string("group capture: ") + hipGetErrorString(e != hipSuccess ? e : e1));
  }
  const hipError_t e2 = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    g->exec = nullptr;
    (void)hipGraphDestroy(graph);
    return fail(FILL_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
  }
  g->graph = graph;
  g->key = key;
  return FILL_OK;
}

// Plans i of the group in threads of their own: each runs fn(i) (a solve on
// its own stream).  Returns the worst status; g_last_error names the plan.
template <typename Fn> int per_plan_threads(int n, Fn&& fn) {
  std::vector<int> rc(n, FILL_OK);
  std::vector<std::string> err(n);
  std::vector<std::thread> th;
  for (int i = 0; i < n; ++i)
    th.emplace_back([&, i] {
      g_last_error.clear();
      rc[i] = fn(i);
      err[i] = g_last_error;
    });
  for (auto& t : th) t.join();
  int worst = FILL_OK;
  for (int i = 0; i < n; ++i)
    if (rc[i] != FILL_OK && (worst == FILL_OK || worst == FILL_ENOCONV)) {
      worst = rc[i];
      g_last_error = "plan " + std::to_string(i) + ": " + err[i];
    }
  return worst;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of fill_realize_unconstrained_noalloc: the transposed half spectrum
// of the draw lives in this file-scope device array instead of the plan's
// workspace, so the call allocates nothing.  Each GPU holds its own copy, at
// its own address, for the life of the process.  In host code the name
// `scratch` is only a host-side stand-in: kernels are given the device address
// obtained once per device with hipGetSymbolAddress (scratch_address()).
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device
// (resolved on the first call for that device, then kept).
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(FILL_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FILL_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[device] = ptr;
  }
  *out = g_scratch_dev[device];
  return FILL_OK;
}
}  // namespace

extern "C" {

int fill_supported_size(int n) { return size_ok(n) ? 1 : 0; }

int fill_plan_create(int nx, int ny, const uint8_t* mask, const double* Pk, int prec, void* stream,
                     fill_plan* out) {
  return plan_create_impl(nx, ny, 1, mask, Pk, 1, prec, stream, out);
}

int fill_plan_create_batch(int nx, int ny, int nprob, const uint8_t* masks, const double* Pk, int n_pk, int prec,
                           void* stream, fill_plan* out) {
  return plan_create_impl(nx, ny, nprob, masks, Pk, n_pk, prec, stream, out);
}

int fill_plan_nprob(fill_plan p) { return p ? p->nprob : 0; }

// True if Pk (npk tables) equals the spectrum the plan holds, bit for bit:
// then there is nothing to upload and no preconditioner to rebuild.
static bool same_pk(fill_plan p, const double* Pk) {
  const size_t n = (size_t)p->npk * p->nt;
  return p->hpk.size() == n && std::memcmp(p->hpk.data(), Pk, n * sizeof(double)) == 0;
}

int fill_plan_set_pk(fill_plan p, const double* Pk) {
  g_last_error.clear();
  if (!p || !Pk) return fail(FILL_EINVAL, "NULL argument");
  if (same_pk(p, Pk)) return FILL_OK;
  HIP_TRY(hipStreamSynchronize(p->stream));
  FILL_TRY(upload_pk(p, Pk, p->npk));
  return block_follow_pk(p);
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

int fill_plan_set_precond(fill_plan p, int mode) {
  g_last_error.clear();
  if (!p || mode < FILL_PRECOND_NONE || mode > FILL_PRECOND_BLOCK) return fail(FILL_EINVAL, "unknown preconditioner");
  if (mode == FILL_PRECOND_BLOCK && !p->blk.built) FILL_TRY(block_setup(p));
  p->precond = mode;
  return FILL_OK;
}

int fill_plan_set_block_halo(fill_plan p, int halo) {
  g_last_error.clear();
  if (!p) return fail(FILL_EINVAL, "NULL plan");
  if (halo != FILL_BLOCK_HALO_AUTO && (halo < 0 || halo > fillb::HALO_MAX))
    return fail(FILL_EINVAL, "halo must be FILL_BLOCK_HALO_AUTO or in [0, 14]");
  static_assert(FILL_BLOCK_HALO_AUTO == fillb::HALO_AUTO && fillb::HALO_MAX == 14, "halo range of the header");
  if (halo == p->block_halo) return FILL_OK;
  p->block_halo = halo;
  return block_follow_pk(p);  // rebuilds a built block preconditioner
}

int fill_get_block_info(fill_plan p, fill_block_info* out) {
  g_last_error.clear();
  if (!p || !out) return fail(FILL_EINVAL, "NULL argument");
  if (!p->blk.built) return fail(FILL_EINVAL, "the block preconditioner is not built");
  *out = p->blk.info;
  return FILL_OK;
}

int fill_plan_set_cg(fill_plan p, int variant) {
  g_last_error.clear();
  if (!p || (variant != FILL_CG_STANDARD && variant != FILL_CG_SINGLE_REDUCTION))
    return fail(FILL_EINVAL, "unknown CG variant");
  p->cg_variant = variant;
  return FILL_OK;
}

int fill_plan_set_lanczos(fill_plan p, int cap) {
  g_last_error.clear();
  if (!p || cap < 0 || cap > (1 << 20)) return fail(FILL_EINVAL, "cap must be in [0, 2^20]");
  HIP_TRY(hipStreamSynchronize(p->stream));
  drop_graphs(p, true);  // recording graphs hold the record's address and size
  if (cap > p->hist_cap) {
    double* h = nullptr;
    FILL_TRY(dalloc(p, &h, (size_t)p->nprob * 2 * cap));
    p->hist = h;
  }
  p->hist_cap = cap;
  p->hist_n.assign(p->nprob, 0);
  return FILL_OK;
}

int fill_get_lanczos(fill_plan p, int problem, double* alpha, double* beta, int cap, int* n) {
  g_last_error.clear();
  if (!alpha || !beta || !n || cap < 0) return fail(FILL_EINVAL, "bad argument");
  std::vector<double> al, be;
  FILL_TRY(read_lanczos(p, problem, al, be));
  const int k = std::min((int)al.size(), cap);
  for (int j = 0; j < k; ++j) alpha[j] = al[j];
  for (int j = 0; j + 1 < k; ++j) beta[j] = be[j];
  *n = (int)al.size();
  return FILL_OK;
}

int fill_lanczos_extremes(fill_plan p, int problem, double* lam_min, double* lam_max, int* n) {
  g_last_error.clear();
  if (!lam_min || !lam_max || !n) return fail(FILL_EINVAL, "NULL argument");
  std::vector<double> al, be, d, e;
  FILL_TRY(read_lanczos(p, problem, al, be));
  *n = (int)al.size();
  if (al.empty()) return fail(FILL_EINVAL, "no CG step recorded for this problem");
  lanczos_matrix(al.data(), be.data(), (int)al.size(), d, e);
  *lam_min = tridiag_eig(d, e, 0);
  *lam_max = tridiag_eig(d, e, (int)d.size() - 1);
  return FILL_OK;
}

int fill_plan_set_skew(fill_plan p, double eps) {
  g_last_error.clear();
  if (!p || !(std::fabs(eps) < 1.0)) return fail(FILL_EINVAL, "eps must lie in (-1, 1)");
  HIP_TRY(hipStreamSynchronize(p->stream));
  drop_graphs(p, false);  // captured chunks hold the old value
  p->skew = eps;
  return FILL_OK;
}

int fill_plan_set_graph(fill_plan p, int on) {
  if (!p || (on != 0 && on != 1)) return fail(FILL_EINVAL, "bad argument");
  p->use_graph = on;
  return FILL_OK;
}

void fill_plan_destroy(fill_plan p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  drop_graphs(p, false);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  for (void* a : p->allocs) (void)hipFree(a);
  for (void* a : p->blk.allocs) (void)hipFree(a);
  if (p->h_sc) (void)hipHostFree(p->h_sc);
  if (p->h_sum) (void)hipHostFree(p->h_sum);
  if (p->h_st) (void)hipHostFree(p->h_st);
  if (p->par_host) (void)hipHostFree(p->par_host);
  if (p->rocblas) (void)rocblas_destroy_handle(p->rocblas);
  delete p;
}

int fill_realize(fill_plan p, const double* d_obs, uint64_t seed, double* x_out, double rtol) {
  if (p && p->nprob != 1) return fail(FILL_EINVAL, "plan holds several problems: use fill_realize_batch");
  return realize_impl(p, &d_obs, &seed, &x_out, rtol, false);
}

int fill_mean(fill_plan p, const double* d_obs, double* x_out, double rtol) {
  if (p && p->nprob != 1) return fail(FILL_EINVAL, "plan holds several problems: use fill_mean_batch");
  return realize_impl(p, &d_obs, nullptr, &x_out, rtol, true);
}

int fill_realize_batch(fill_plan p, const double* const* d_obs, const uint64_t* seeds, double* const* x_out,
                       double rtol) {
  return realize_impl(p, d_obs, seeds, x_out, rtol, false);
}

int fill_mean_batch(fill_plan p, const double* const* d_obs, double* const* x_out, double rtol) {
  return realize_impl(p, d_obs, nullptr, x_out, rtol, true);
}

int fill_realize_multi(int nplans, const fill_plan* plans, const double* const* const* d_obs,
                       const uint64_t* const* seeds, double* const* const* x_out, double rtol) {
  g_last_error.clear();
  if (nplans < 1 || !plans || !d_obs || !seeds || !x_out) return fail(FILL_EINVAL, "bad argument");
  return per_plan_threads(nplans, [&](int i) { return realize_impl(plans[i], d_obs[i], seeds[i], x_out[i], rtol, false); });
}

int fill_group_create(int nplans, const fill_plan* plans, void* stream, fill_group* out) {
  g_last_error.clear();
  if (!out) return fail(FILL_EINVAL, "out is NULL");
  *out = nullptr;
  if (nplans < 1 || !plans) return fail(FILL_EINVAL, "need at least one plan");
  for (int i = 0; i < nplans; ++i) {
    if (!plans[i]) return fail(FILL_EINVAL, "NULL plan " + std::to_string(i));
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(FILL_EINVAL, "plan " + std::to_string(i) + " appears twice");
  }
  fill_group g = new (std::nothrow) fill_group_s();
  if (!g) return fail(FILL_ENOMEM, "host allocation");
  g->plans.assign(plans, plans + nplans);
  g->stream = static_cast<hipStream_t>(stream);
  g->join.assign(nplans, nullptr);
  hipError_t e = hipEventCreateWithFlags(&g->fork, hipEventDisableTiming);
  for (int i = 0; i < nplans && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&g->join[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    fill_group_destroy(g);
    return fail(FILL_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
  }
  *out = g;
  return FILL_OK;
}

int fill_group_realize(fill_group g, const double* const* const* d_obs, const uint64_t* const* seeds,
                       double* const* const* x_out, double rtol) {
  g_last_error.clear();
  if (!g || !d_obs || !seeds || !x_out) return fail(FILL_EINVAL, "bad argument");
  const int n = (int)g->plans.size();
  const auto t0 = clk::now();
  bool graph = true;
  for (int i = 0; i < n; ++i) {
    fill_plan p = g->plans[i];
    if (!d_obs[i] || !seeds[i] || !x_out[i]) return fail(FILL_EINVAL, "NULL arrays for plan " + std::to_string(i));
    FILL_TRY(prepare_call(p, d_obs[i], seeds[i], x_out[i], rtol, false));
    graph = graph && whole_graph_ok(p, false);
  }
  g->last_graph = 0;
  if (!graph) {
    // step by step, each plan on its own stream and host thread; the solves
    // give the step counts the next call's graph is captured for
    return per_plan_threads(n, [&](int i) {
      fill_plan p = g->plans[i];
      const auto t1 = clk::now();
      int rc = upload_params(p);
      if (rc == FILL_OK) rc = run_solve(p, false);
      finish_stats(p, rc, std::chrono::duration<double, std::milli>(clk::now() - t1).count());
      return rc;
    });
  }
  FILL_TRY(group_graph(g));
  for (fill_plan p : g->plans)
    HIP_TRY(hipMemcpyAsync(p->par_dev, p->par_host, p->par_bytes, hipMemcpyHostToDevice, g->stream));
  HIP_TRY(hipGraphLaunch(g->exec, g->stream));
  for (fill_plan p : g->plans)
    HIP_TRY(hipMemcpyAsync(p->h_st, p->st, p->nprob * sizeof(SolveState), hipMemcpyDeviceToHost, g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  bool all = true;
  for (fill_plan p : g->plans) all = all && all_done(p);
  g->last_graph = all ? 1 : 0;
  const double ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  return per_plan_threads(n, [&](int i) {
    fill_plan p = g->plans[i];
    p->last_whole_graph = g->last_graph;
    int rc = FILL_OK;
    if (!all_done(p)) {  // this plan's steps did not suffice: continue on its own stream
      rc = refine_host(p, false);
      if (rc == FILL_OK) {
        const hipError_t e = launch_scatter_add(p->dp.out_tab, p->u, p->pos, p->comp_off, p->n_m_max, p->nprob,
                                                p->stream);
        if (e == hipSuccess) (void)hipStreamSynchronize(p->stream);
        else rc = fail(FILL_EHIP, std::string("launch_scatter_add: ") + hipGetErrorString(e));
      }
    }
    if (rc == FILL_OK) rc = finish_solve(p, solve_key(p, false));
    finish_stats(p, rc, ms);
    return rc;
  });
}

int fill_group_last_graph(fill_group g) { return g ? g->last_graph : 0; }

void fill_group_destroy(fill_group g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  group_drop_graph(g);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  if (g->fork) (void)hipEventDestroy(g->fork);
  for (hipEvent_t e : g->join)
    if (e) (void)hipEventDestroy(e);
  delete g;
}

int fill_laplace(fill_plan p, const double* d_obs, double* x_out, int nkernels, double r0, double ratio, int iters) {
  g_last_error.clear();
  if (!p || !d_obs || !x_out) return fail(FILL_EINVAL, "NULL argument");
  if (d_obs == x_out) return fail(FILL_EINVAL, "x_out may not alias d_obs");
  FILL_TRY(laplace_check(p, nkernels, r0, ratio, iters));
  const double* res = nullptr;
  FILL_TRY(laplace_run(p, d_obs, nkernels, r0, ratio, iters, &res));
  HIP_TRY(hipMemcpyAsync(x_out, res, p->npix * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  return FILL_OK;
}

int fill_plan_set_warm_start(fill_plan p, int iters, int nkernels, double r0, double ratio) {
  g_last_error.clear();
  if (!p) return fail(FILL_EINVAL, "NULL plan");
  if (iters < 0) return fail(FILL_EINVAL, "iters must be >= 0");
  if (iters > 0) FILL_TRY(laplace_check(p, nkernels, r0, ratio, iters));
  p->ws_iters = iters;
  p->ws_k = nkernels;
  p->ws_r0 = r0;
  p->ws_ratio = ratio;
  return FILL_OK;
}

int fill_plan_set_bands(fill_plan p, int nbands, const double* lnk_nodes, const double* theta) {
  g_last_error.clear();
  if (!p || !lnk_nodes || !theta || nbands < 1) return fail(FILL_EINVAL, "bad argument");
  for (int b = 1; b < nbands; ++b)
    if (!(lnk_nodes[b] > lnk_nodes[b - 1])) return fail(FILL_EINVAL, "band nodes must increase");
  for (int b = 0; b < nbands; ++b)
    if (!std::isfinite(theta[b]) || !std::isfinite(lnk_nodes[b])) return fail(FILL_ENOTSPD, "non-finite band power");
  HIP_TRY(hipStreamSynchronize(p->stream));
  const int nx = p->nx, ny = p->ny, nc = p->ncol;
  std::vector<double> Pk((size_t)p->npk * ny * nc);
  for (int iy = 0; iy < ny; ++iy) {
    const int ky = iy <= ny / 2 ? iy : iy - ny;
    for (int ix = 0; ix < nc; ++ix) {
      const double k = std::sqrt((double)ix * ix + (double)ky * ky);
      const double P = std::exp(band_lnP(k, lnk_nodes, theta, nbands));
      for (int t = 0; t < p->npk; ++t) Pk[((size_t)t * ny + iy) * nc + ix] = P;
    }
  }
  (void)nx;
  // the spectrum first: if it is rejected, the plan keeps its nodes and tables
  const bool same = same_pk(p, Pk.data());
  if (!same) FILL_TRY(upload_pk(p, Pk.data(), p->npk));
  if (p->nbands != nbands) {
    FILL_TRY(dalloc(p, &p->lnk, nbands));
    FILL_TRY(dalloc(p, &p->adj_gth, nbands));
    p->nbands = nbands;
  }
  HIP_TRY(hipMemcpy(p->lnk, lnk_nodes, nbands * sizeof(double), hipMemcpyHostToDevice));
  return same ? FILL_OK : block_follow_pk(p);
}

int fill_adjoint(fill_plan p, const double* d_obs, uint64_t seed, const double* x_out, const double* g,
                 double* grad_dobs, double* grad_theta, double* grad_logP, double rtol) {
  if (p && p->nprob != 1) return fail(FILL_EINVAL, "plan holds several problems: use fill_adjoint_batch");
  return adjoint_impl(p, &d_obs, &seed, &x_out, &g, &grad_dobs, grad_theta, grad_logP, rtol);
}

int fill_adjoint_batch(fill_plan p, const double* const* d_obs, const uint64_t* seeds, const double* const* x_out,
                       const double* const* g, double* const* grad_dobs, double* grad_theta, double* grad_logP,
                       double rtol) {
  return adjoint_impl(p, d_obs, seeds, x_out, g, grad_dobs, grad_theta, grad_logP, rtol);
}

int fill_get_stats(fill_plan p, fill_stats* out) {
  if (!p || !out) return fail(FILL_EINVAL, "NULL argument");
  *out = p->stats;
  return FILL_OK;
}

int fill_get_stats_batch(fill_plan p, fill_stats* out) {
  if (!p || !out) return fail(FILL_EINVAL, "NULL argument");
  for (int b = 0; b < p->nprob; ++b) out[b] = p->pstats[b];
  return FILL_OK;
}

int fill_apply(fill_plan p, int op, int prec, const double* in, double* out) {
  g_last_error.clear();
  if (!p || !in || !out) return fail(FILL_EINVAL, "NULL argument");
  if (in == out) return fail(FILL_EINVAL, "out aliases in");
  if (op < FILL_OP_CINV || op > FILL_OP_MINV) return fail(FILL_EINVAL, "unknown operator");
  if (prec != FILL_PREC_FP64 && prec != FILL_PREC_FP32_OP) return fail(FILL_EINVAL, "unknown precision");
  if (op == FILL_OP_MINV) {
    if (p->precond != FILL_PRECOND_BLOCK || !p->blk.built)
      return fail(FILL_EINVAL, "FILL_OP_MINV applies the block preconditioner: select FILL_PRECOND_BLOCK first");
    if (prec != p->prec) return fail(FILL_EINVAL, "FILL_OP_MINV runs in the plan's precision");
    const int nm = p->n_m[0];
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipMemsetAsync(out, 0, p->npix * sizeof(double), p->stream));
    if (nm > 0) {
      HIP_TRY(launch_gather(p->res, in, p->pos, nm, p->stream));
      if (prec == FILL_PREC_FP64) {
        FILL_TRY(block_apply<double>(p, p->res, p->v64.q, nullptr, nullptr, nullptr));
        HIP_TRY(launch_scatter(out, p->v64.q, p->pos, nm, p->stream));
      } else {
        p->hp.scale[0] = 1.0;
        FILL_TRY(upload_params(p));
        HIP_TRY(launch_scale_to_f32(p->v32.t, p->res, p->dp.scale, p->comp_off, nm, 1, p->stream));
        FILL_TRY(block_apply<float>(p, p->v32.t, p->v32.q, nullptr, nullptr, nullptr));
        HIP_TRY(launch_scatter_f32(out, p->v32.q, p->pos, nm, p->stream));
      }
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    return FILL_OK;
  }
  const bool inv = (op == FILL_OP_CINV || op == FILL_OP_A);
  const int n = p->n_m[0];
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (op == FILL_OP_CINV || op == FILL_OP_CHALF) {
    if (prec == FILL_PREC_FP64) {
      RowArgs<double> ai = row_base<double>(p, 1), ao = row_base<double>(p, 1);
      ai.full_in = in;
      ao.full_out = out;
      FILL_TRY(apply3<double>(p, R2C_FULL, ai, inv ? p->Dinv64 : p->Dhalf64, C2R_FULL, ao, nullptr));
    } else {
      RowArgs<float> ai = row_base<float>(p, 1), ao = row_base<float>(p, 1);
      ai.full_in = in;
      ao.full_out = out;
      FILL_TRY(apply3<float>(p, R2C_FULL, ai, inv ? p->Dinv32 : p->Dhalf32, C2R_FULL, ao, nullptr));
    }
  } else {
    HIP_TRY(hipMemsetAsync(out, 0, p->npix * sizeof(double), p->stream));
    if (n > 0) {
      HIP_TRY(launch_gather(p->res, in, p->pos, n, p->stream));
      if (prec == FILL_PREC_FP64) {
        RowArgs<double> ai = row_base<double>(p, 1), ao = row_base<double>(p, 1);
        ai.v0 = p->res;
        ao.v0 = p->v64.q;
        FILL_TRY(apply3<double>(p, R2C_COMPACT, ai, inv ? p->Dinv64 : p->Dhalf64, C2R_COMPACT, ao, nullptr,
                                inv ? p->skew : 0.0));
        HIP_TRY(launch_scatter(out, p->v64.q, p->pos, n, p->stream));
      } else {
        p->hp.scale[0] = 1.0;
        FILL_TRY(upload_params(p));
        HIP_TRY(launch_scale_to_f32(p->v32.t, p->res, p->dp.scale, p->comp_off, n, 1, p->stream));
        RowArgs<float> ai = row_base<float>(p, 1), ao = row_base<float>(p, 1);
        ai.v0 = p->v32.t;
        ao.v0 = p->v32.q;
        FILL_TRY(apply3<float>(p, R2C_COMPACT, ai, inv ? p->Dinv32 : p->Dhalf32, C2R_COMPACT, ao, nullptr,
                               inv ? p->skew : 0.0));
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
  RowArgs<double> ai = row_base<double>(p, 1), ao = row_base<double>(p, 1);
  ai.seed = seed;
  ai.stream = kRealizationStream;
  ao.full_out = out;
  FILL_TRY(apply3<double>(p, R2C_NOISE, ai, p->Dhalf64, C2R_REALIZE, ao, nullptr));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return FILL_OK;
}

int fill_realize_unconstrained_noalloc(fill_plan p, uint64_t seed, double* out) {
  g_last_error.clear();
  if (!p || !out) return fail(FILL_EINVAL, "NULL argument");
  const size_t need = (size_t)(p->nx / 2) * p->ny * sizeof(double2);
  if (need > kNoAllocScratchBytes)
    return fail(FILL_EINVAL, "grid " + std::to_string(p->nx) + "x" + std::to_string(p->ny) + " needs " +
                                 std::to_string(need) + " bytes of spectrum scratch; the limit is " +
                                 std::to_string(kNoAllocScratchBytes) + " (nx * ny <= 8388608)");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != p->device) return fail(FILL_EINVAL, "the plan's device must be the current device");
  void* sp = nullptr;
  FILL_TRY(scratch_address(cur, &sp));
  // the same three passes as fill_realize_unconstrained, on the scratch
  // spectrum; every pass overwrites what the next one reads, so nothing needs
  // clearing between calls
  RowArgs<double> ai = row_base<double>(p, 1), ao = row_base<double>(p, 1);
  ai.Xt = ao.Xt = static_cast<cplx<double>*>(sp);
  ai.seed = seed;
  ai.stream = kRealizationStream;
  ao.full_out = out;
  ColArgs<double> ca = col_base<double>(p, 1, p->Dhalf64, nullptr);
  ca.Xt = static_cast<cplx<double>*>(sp);
  HIP_TRY(launch_r2c<double>(R2C_NOISE, ai, p->stream, nullptr, nullptr));
  HIP_TRY(launch_col<double>(p->ny, ca, p->stream, nullptr, nullptr));
  HIP_TRY(launch_c2r<double>(C2R_REALIZE, ao, p->stream, nullptr, nullptr));
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
  if (kernel < FILL_K_R2C || kernel > FILL_K_COMBINE) return fail(FILL_EINVAL, "unknown kernel");
  if (prec == FILL_PREC_FP64) return time_kernel<double>(p, kernel, reps, avg_ms);
  if (prec == FILL_PREC_FP32_OP) return time_kernel<float>(p, kernel, reps, avg_ms);
  return fail(FILL_EINVAL, "unknown precision");
}

int fill_kernel_timing(fill_plan p, int kernel, int prec) {
  g_last_error.clear();
  if (!p) return fail(FILL_EINVAL, "NULL plan");
  if (kernel < -1 || kernel > FILL_K_COMBINE || kernel == FILL_K_APPLY) return fail(FILL_EINVAL, "unknown kernel");
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

namespace {

int plan_create_impl(int nx, int ny, int nprob, const uint8_t* masks, const double* Pk, int npk, int prec,
                     void* stream, fill_plan* out) {
  g_last_error.clear();
  if (!out) return fail(FILL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!masks || !Pk) return fail(FILL_EINVAL, "mask or Pk is NULL");
  if (nprob < 1) return fail(FILL_EINVAL, "nprob must be >= 1");
  if (npk != 1 && npk != nprob) return fail(FILL_EINVAL, "n_pk must be 1 or nprob");
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
  p->nprob = nprob;
  p->npk = npk;
  p->npix = (size_t)nx * ny;
  p->nt = (size_t)p->ncol * ny;
  p->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(FILL_EHIP, "hipGetDevice failed");
  }
  const int r64 = row_block_rows<double>(nx), r32 = row_block_rows<float>(nx);
  if (r64 <= 0 || r32 <= 0 || ny % r64 || ny % r32) {
    delete p;
    return fail(FILL_EUNSUPPORTED_SIZE, "ny not a multiple of the row block");
  }
  p->nblk64 = ny / r64;
  p->nblk32 = ny / r32;
  const int rc = plan_build(p, masks, Pk);
  if (rc != FILL_OK) {
    fill_plan_destroy(p);
    return rc;
  }
  *out = p;
  return FILL_OK;
}

}  // namespace
