// Host construction of the block preconditioner M^-1 ~ (Px C^-1 Px)^-1:
// per-frequency banded factors for the runs of fully masked rows and dense
// inverses of the grown pieces of the rest of the mask (additive Schwarz).
//
//   band runs   maximal runs y0..y0+h-1 of fully masked rows, h <= ny - 2 BW;
//               per kx = 0..nx/2 the matrix nx T_kx, T_kx[i][j] = t_kx(i - j)
//               for |i - j| < BW plus sigma_kx on the diagonal, where
//               t_kx(d) = sum_dx k(d, dx) cos(2 pi kx dx/nx) (k the kernel of
//               C^-1); sigma_kx = 0 if every Cholesky pivot of the truncation
//               exceeds pivot_min times its diagonal (PIVOT_MIN for FP64
//               factors, PIVOT_MIN_F32 for FP32 ones), else
//               sigma_kx = 2 sum_{BW <= d < h} |t_kx(d)|, which bounds the
//               discarded part (keeps T_kx positive definite); factored as
//               L L^T (banded Cholesky);
//   cells       connected pieces (4-neighbours, periodic) of the masked pixels
//               outside the runs; a piece of more than CMAX pixels, or whose
//               grown block would exceed NBMAX, is cut by the TILE x TILE grid;
//   blocks      each cell grown by a halo h (Chebyshev, periodic) within the
//               mask, with the dense inverse of C^-1 restricted to its pixels
//               (the layout is built here, the inverses on the device); h is
//               given, or chosen: from h = HALO up by 2 (to HALO_MAX) while
//               the blocks hold at most npix / 2 more inverse entries than
//               those of h = HALO.  A wider halo couples the pieces to
//               the band and to each other over more rows (fewer CG
//               iterations); the cap keeps the extra product work per
//               iteration at about half an entry per pixel.
//
// The applies of the band factors run as two sequential substitutions, one
// wave per (run, kx): lanes 0..31 carry the real parts, 32..63 the imaginary
// parts, lane k holding the window element j = k (mod 32).  The factor is
// stored unit-diagonal (L = Lu D, D^-2 in the diagonal slots) as one stream
// per (kx, lane) in the order the forward substitution uses it (see
// block.cpp), so each lane reads its own contiguous stream; 32 zeros precede
// the first run's streams.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fillb {

constexpr int BW = 32;       // band bandwidth (one window lane per coupled row)
constexpr int HALO = 8;      // Chebyshev growth of each cell into the mask (the reference choice)
constexpr int HALO_MAX = 14; // widest halo: a grown TILE x TILE cell always fits a block
constexpr int HALO_AUTO = -1;
constexpr int TILE = 16;     // cell grid for large pieces
constexpr int CMAX = 1024;   // largest piece kept whole
constexpr int NBMAX = 2048;  // largest block (dense inverse)
static_assert((TILE + 2 * HALO_MAX) * (TILE + 2 * HALO_MAX) <= NBMAX, "a grown cell must fit a block");
// band truncation kept unshifted if every Cholesky pivot exceeds this times
// its diagonal: FP64 factors, and FP32 factors (whose rounding, relative 2^-24,
// is amplified by up to the truncation's condition number, which the pivot
// ratio bounds from below)
constexpr double PIVOT_MIN = 1e-9;
constexpr double PIVOT_MIN_F32 = 1e-4;
constexpr int BROWS = 256;   // rows of a block product work item
constexpr int BCOLS = 128;   // columns of a block product work item

// Column stride of a block inverse of n pixels (16-byte aligned columns in FP32).
inline int block_ld(int n) { return (n + 3) / 4 * 4; }

struct Run {
  int y0 = 0, h = 0, hp = 0;  // first row, rows, rows padded to a multiple of 32
  int cb0 = 0;                // compact index of the run's first pixel
  size_t bt_off = 0;          // complex offset of the run's spectrum [nx/2][hp]
  int k0 = 0;                 // index of the run's (kx = 0) entry in kx_off / kx_dup
};

struct Layout {
  int nx = 0, ny = 0, n_m = 0;
  std::vector<Run> runs;
  std::vector<int> brow_off;   // per run: hp+1 compact offsets of the virtual rows
  size_t bt_total = 0;         // complex values of all runs' spectra
  // Factor streams (see block.cpp), per (run, kx): 32 lane streams of
  // hp - 32 d values at fwd[kx_off], where chunks (32 positions) s0 .. s0 + d
  // of the full-length streams are equal and stored once, as chunk s0
  // (kx_dup = {s0, d}; d = 0: nothing shared).  fwd starts with 32 zeros.
  std::vector<double> fwd;
  std::vector<size_t> kx_off;
  std::vector<int> kx_dup;     // 2 per (run, kx)
  size_t stream_values = 0;    // sum over runs of their streams' values
  // blocks
  std::vector<int> boff;       // nblocks+1 offsets into bidx
  std::vector<int> bidx;       // compact indices of each block's pixels
  // block product work items, 4 ints each: block, first row, first column,
  // offset of the item's output rows in seg (the item's column chunk of the
  // block has its own n outputs: seg holds sum_b n_b ceil(n_b / BCOLS) values)
  std::vector<int> items;
  size_t seg_total = 0;
  std::vector<size_t> moff;    // offsets of each block's inverse: n columns of stride block_ld(n)
  size_t inv_total = 0;        // values of all blocks' inverses
  std::vector<int> bpix;       // pixel (flat index) of each block entry, as bidx
  // combine: contributions of block entries to compact elements (CSR), band flags
  std::vector<int> cst;        // n_m+1
  std::vector<int> cix;        // entries: positions in seg (one per column chunk of each covering block)
  std::vector<uint8_t> inb;    // 1 if the element lies in a band run
  int max_run_pixels = 0;
  int halo = HALO;             // the blocks' halo
};

// mask: ny*nx (1 = masked); tsym: ny*(nx/2+1), tsym[d*(nx/2+1) + kx] =
// t_kx(d); pivot_min: the threshold of the unshifted band truncation
// (PIVOT_MIN or PIVOT_MIN_F32); f32: the factor is used in FP32 (chunks of
// the streams are shared when their values rounded to FP32 are equal; FP64:
// when they are equal).  Returns 0, or -1 with *err set (a band factor is
// not positive definite, or a block is too large).  halo: 0 .. HALO_MAX, or
// HALO_AUTO (the rule above).
int build_layout(int nx, int ny, const uint8_t* mask, const double* tsym, double pivot_min, bool f32, int halo,
                 Layout* out, std::string* err);

// The stored chunk of chunk c of a (run, kx) whose chunks s0 .. s0 + d share
// chunk s0's storage.
inline int stored_chunk(int c, int s0, int d) { return c < s0 ? c : (c <= s0 + d ? s0 : c - d); }

}  // namespace fillb
