// Host construction of the block preconditioner (see block.hpp).
#include "block.hpp"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdint>
#include <thread>

namespace fillb {
namespace {

// Work items 0..n-1 over the host's cores.
template <typename F> void parallel_for(int n, F&& f) {
  const int nt = std::max(1, std::min<int>(n, (int)std::thread::hardware_concurrency()));
  std::atomic<int> next{0};
  auto worker = [&]() {
    for (int i = next++; i < n; i = next++) f(i);
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

}  // namespace

int build_layout(int nx, int ny, const uint8_t* mask, const double* tsym, double pivot_min, bool f32, int halo,
                 Layout* L, std::string* err) {
  if (halo != HALO_AUTO && (halo < 0 || halo > HALO_MAX)) {
    *err = "block preconditioner: halo out of range";
    return -1;
  }
  L->nx = nx;
  L->ny = ny;
  const size_t npix = (size_t)nx * ny;
  std::vector<int> comp_of(npix, -1);  // compact index of each masked pixel
  int n_m = 0;
  for (size_t q = 0; q < npix; ++q)
    if (mask[q]) comp_of[q] = n_m++;
  L->n_m = n_m;

  // ---- band runs
  std::vector<uint8_t> in_run(ny, 0);
  for (int y = 0; y < ny;) {
    bool full = true;
    for (int x = 0; x < nx && full; ++x) full = mask[(size_t)y * nx + x] != 0;
    if (!full) {
      ++y;
      continue;
    }
    const int y0 = y;
    while (y < ny) {
      bool f = true;
      for (int x = 0; x < nx && f; ++x) f = mask[(size_t)y * nx + x] != 0;
      if (!f) break;
      ++y;
    }
    const int h = y - y0;
    if (h <= ny - 2 * BW) {
      Run r;
      r.y0 = y0;
      r.h = h;
      r.hp = (h + 31) / 32 * 32;
      r.cb0 = comp_of[(size_t)y0 * nx];
      L->runs.push_back(r);
      for (int j = y0; j < y; ++j) in_run[j] = 1;
    }
  }
  const int ncol = nx / 2, nk = nx / 2 + 1;
  // 32 zeros before the first stream: the backward substitution's loads for
  // the lanes past the first row reach up to 31 values before a stream
  L->fwd.clear();
  if (!L->runs.empty()) L->fwd.assign(32, 0.0);
  for (Run& r : L->runs) {
    r.bt_off = L->bt_total;
    L->bt_total += (size_t)ncol * r.hp;
    for (int j = 0; j <= r.hp; ++j) L->brow_off.push_back(r.cb0 + std::min(j, r.h) * nx);
    L->max_run_pixels = std::max(L->max_run_pixels, r.h * nx);
  }
  if (!L->runs.empty()) {
    const double* t = tsym;
    std::atomic<int> bad{-1};
    for (Run& r : L->runs) {
      const int h = r.h, hp = r.hp, nch = hp / 32;
      r.k0 = (int)L->kx_off.size();
      std::vector<std::vector<double>> packed(nk);  // per kx: the stored streams
      std::vector<int> dup(2 * (size_t)nk, 0);
      parallel_for(nk, [&](int kx) {
        // banded Cholesky of nx T_kx: Lb[i*BW + d] = L(i, i-d); false if a
        // pivot is not above pivot_min (its square root is not taken then)
        std::vector<double> Lb((size_t)h * BW, 0.0);
        auto l = [&](int i, int j) -> double& { return Lb[(size_t)i * BW + (i - j)]; };
        auto factor = [&](double sigma, double pivot_min) {
          for (int i = 0; i < h; ++i) {
            for (int j = std::max(0, i - BW + 1); j <= i; ++j) {
              double s = (double)nx * (t[(size_t)(i - j) * nk + kx] + (i == j ? sigma : 0.0));
              for (int m = std::max(0, i - BW + 1); m < j; ++m) s -= l(i, m) * l(j, m);
              if (i == j) {
                if (!(s > pivot_min)) return false;
                l(i, i) = std::sqrt(s);
              } else {
                l(i, j) = s / l(j, j);
              }
            }
          }
          return true;
        };
        // the plain truncation where it is safely positive definite (every
        // pivot above pivot_min times the diagonal nx t_kx(0)), else the
        // shift by the Gershgorin bound of the part beyond the bandwidth
        if (!factor(0.0, pivot_min * (double)nx * t[kx])) {
          double sigma = 0.0;
          for (int d = BW; d < h; ++d) sigma += 2.0 * std::fabs(t[(size_t)d * nk + kx]);
          if (!factor(sigma, 0.0)) {
            bad = kx;
            return;
          }
        }
        // The factor is stored unit-diagonal, L = Lu D (Lu(i, j) = L(i, j) /
        // L(j, j)).  Stream of lane k, position i (forward substitution, i
        // ascending): the head lane of step i is i mod 32 and reads
        // 1/L(i,i)^2 (the scaling between the two substitutions); lane
        // k != head holds window element i + d, d = (k - i) mod 32, and reads
        // its coupling Lu(i+d, i).  Padded rows are the identity.  (The
        // backward substitution reads the same streams across the lanes:
        // entries i-31 .. i-1 of lane i mod 32 hold row i of Lu.)
        std::vector<double> full((size_t)32 * hp);
        for (int k = 0; k < 32; ++k) {
          double* f = full.data() + (size_t)k * hp;
          for (int i = 0; i < hp; ++i) {
            const int d = ((k - i) % 32 + 32) % 32;
            if (d == 0) f[i] = i < h ? 1.0 / (l(i, i) * l(i, i)) : 1.0;
            else f[i] = (i + d < h && d < BW) ? l(i + d, i) / l(i, i) : 0.0;
          }
        }
        // Far from the run's ends the rows of the factor reach their
        // Toeplitz limit, and whole chunks of 32 positions repeat in every
        // lane's stream: the longest run of equal consecutive chunks (equal
        // in the precision the factor is used in) is stored once.
        auto same = [&](double u, double v) { return f32 ? (float)u == (float)v : u == v; };
        auto chunk_eq = [&](int c1, int c2) {
          for (int k = 0; k < 32; ++k) {
            const double* f = full.data() + (size_t)k * hp;
            for (int j = 0; j < 32; ++j)
              if (!same(f[32 * c1 + j], f[32 * c2 + j])) return false;
          }
          return true;
        };
        int s0 = 0, d = 0;
        for (int c = 1, a = 0; c < nch; ++c) {
          if (!chunk_eq(c, c - 1)) a = c;
          else if (c - a > d) {
            s0 = a;
            d = c - a;
          }
        }
        const int len = hp - 32 * d;
        std::vector<double>& out = packed[kx];
        out.resize((size_t)32 * len);
        for (int k = 0; k < 32; ++k)
          for (int c = 0; c < nch; ++c) {
            if (c > s0 && c <= s0 + d) continue;
            const int sc = stored_chunk(c, s0, d);
            std::copy(full.data() + (size_t)k * hp + 32 * c, full.data() + (size_t)k * hp + 32 * c + 32,
                      out.data() + (size_t)k * len + 32 * sc);
          }
        dup[2 * (size_t)kx] = s0;
        dup[2 * (size_t)kx + 1] = d;
      });
      if (bad >= 0) {
        *err = "block preconditioner: the band factor of kx = " + std::to_string(bad.load()) +
               " is not positive definite";
        return -1;
      }
      for (int kx = 0; kx < nk; ++kx) {
        L->kx_off.push_back(L->fwd.size());
        L->kx_dup.push_back(dup[2 * (size_t)kx]);
        L->kx_dup.push_back(dup[2 * (size_t)kx + 1]);
        L->fwd.insert(L->fwd.end(), packed[kx].begin(), packed[kx].end());
        L->stream_values += packed[kx].size();
      }
    }
  }

  // ---- cells: pieces of the masked pixels outside the runs, grown by h
  auto other = [&](size_t q) { return mask[q] && !in_run[q / nx]; };
  std::vector<int> stamp(npix, -1), incell(npix, -1);
  int stamp_id = 0;
  auto make_blocks = [&](int h, std::vector<std::vector<int>>* blocks) -> bool {
    blocks->clear();
    std::vector<int> piece(npix, -1);
    // The cell and every masked pixel within distance h of it.  A pixel
    // within h of the cell is within h of one of the cell's edge pixels
    // (those with a neighbour, diagonals included, outside the cell) or in
    // the cell itself: a shortest king's path from the cell pixel leaves the
    // cell through an edge pixel, which is closer.  So only the edge pixels'
    // squares are visited.
    auto grow = [&](const std::vector<int>& cell, std::vector<int>* out) {
      const int id = stamp_id++;
      out->clear();
      for (int q : cell) incell[q] = id;
      for (int q : cell) {
        stamp[q] = id;
        out->push_back(q);
      }
      for (int q : cell) {
        const int y = q / nx, x = q % nx;
        bool edge = false;
        for (int dy = -1; dy <= 1 && !edge; ++dy)
          for (int dx = -1; dx <= 1 && !edge; ++dx)
            edge = incell[(size_t)((y + dy + ny) % ny) * nx + (x + dx + nx) % nx] != id;
        if (!edge) continue;
        for (int dy = -h; dy <= h; ++dy)
          for (int dx = -h; dx <= h; ++dx) {
            const int yy = ((y + dy) % ny + ny) % ny, xx = ((x + dx) % nx + nx) % nx;
            const int qq = yy * nx + xx;
            if (mask[qq] && stamp[qq] != id) {
              stamp[qq] = id;
              out->push_back(qq);
            }
          }
      }
      std::sort(out->begin(), out->end());
    };
    std::vector<int> grown;
    int npieces = 0;
    for (size_t q0 = 0; q0 < npix; ++q0) {
      if (!other(q0) || piece[q0] >= 0) continue;
      std::vector<int> comp, stack{(int)q0};
      piece[q0] = npieces;
      while (!stack.empty()) {
        const int q = stack.back();
        stack.pop_back();
        comp.push_back(q);
        const int y = q / nx, x = q % nx;
        const int nb[4] = {((y + 1) % ny) * nx + x, ((y + ny - 1) % ny) * nx + x, y * nx + (x + 1) % nx,
                           y * nx + (x + nx - 1) % nx};
        for (int qq : nb)
          if (other(qq) && piece[qq] < 0) {
            piece[qq] = npieces;
            stack.push_back(qq);
          }
      }
      ++npieces;
      bool whole = (int)comp.size() <= CMAX;
      if (whole) {
        grow(comp, &grown);
        whole = (int)grown.size() <= NBMAX;
      }
      if (whole) {
        blocks->push_back(grown);
        continue;
      }
      // cut along the absolute TILE grid
      std::sort(comp.begin(), comp.end(), [&](int a, int b) {
        const long ka = (long)(a / nx / TILE) * (nx / TILE + 1) + (a % nx) / TILE;
        const long kb = (long)(b / nx / TILE) * (nx / TILE + 1) + (b % nx) / TILE;
        return ka != kb ? ka < kb : a < b;
      });
      size_t s = 0;
      while (s < comp.size()) {
        const long key = (long)(comp[s] / nx / TILE) * (nx / TILE + 1) + (comp[s] % nx) / TILE;
        size_t e = s;
        std::vector<int> cell;
        while (e < comp.size() &&
               (long)(comp[e] / nx / TILE) * (nx / TILE + 1) + (comp[e] % nx) / TILE == key)
          cell.push_back(comp[e++]);
        grow(cell, &grown);
        if ((int)grown.size() > NBMAX) {
          *err = "block preconditioner: a grown cell exceeds the block size limit";
          return false;
        }
        blocks->push_back(grown);
        s = e;
      }
    }
    return true;
  };
  auto entries = [](const std::vector<std::vector<int>>& b) {
    size_t e = 0;
    for (const auto& v : b) e += v.size() * (size_t)block_ld((int)v.size());
    return e;
  };
  std::vector<std::vector<int>> blocks;
  if (halo == HALO_AUTO) {
    // widen from HALO by 2 while the inverse entries stay within npix / 2
    // of those at HALO
    if (!make_blocks(HALO, &blocks)) return -1;
    const size_t e0 = entries(blocks);
    L->halo = HALO;
    std::vector<std::vector<int>> cand;
    for (int h = HALO + 2; h <= HALO_MAX; h += 2) {
      if (!make_blocks(h, &cand)) return -1;
      if (entries(cand) > e0 + npix / 2) break;
      blocks.swap(cand);
      L->halo = h;
    }
  } else {
    if (!make_blocks(halo, &blocks)) return -1;
    L->halo = halo;
  }

  // ---- block layout (the dense inverses are computed on the device)
  const int nb = (int)blocks.size();
  L->boff.assign(nb + 1, 0);
  L->moff.assign(nb, 0);
  size_t mt = 0;
  for (int b = 0; b < nb; ++b) {
    L->boff[b + 1] = L->boff[b] + (int)blocks[b].size();
    L->moff[b] = mt;
    mt += blocks[b].size() * (size_t)block_ld((int)blocks[b].size());
  }
  L->inv_total = mt;
  L->bidx.resize(L->boff[nb]);
  L->bpix.resize(L->boff[nb]);
  for (int b = 0; b < nb; ++b)
    for (size_t i = 0; i < blocks[b].size(); ++i) {
      L->bpix[L->boff[b] + i] = blocks[b][i];
      L->bidx[L->boff[b] + i] = comp_of[blocks[b][i]];
    }

  // ---- block product work items and their output segments
  std::vector<size_t> segb(nb);  // seg offset of block b's first column chunk
  for (int b = 0; b < nb; ++b) {
    const int n = L->boff[b + 1] - L->boff[b], ncc = (n + BCOLS - 1) / BCOLS;
    segb[b] = L->seg_total;
    for (int cc = 0; cc < ncc; ++cc)
      for (int r0 = 0; r0 < n; r0 += BROWS) {
        L->items.push_back(b);
        L->items.push_back(r0);
        L->items.push_back(cc * BCOLS);
        L->items.push_back((int)(L->seg_total + (size_t)cc * n));
      }
    L->seg_total += (size_t)n * ncc;
  }
  if (L->seg_total > (size_t)INT32_MAX) {
    *err = "block preconditioner: too many block outputs";
    return -1;
  }

  // ---- combine tables: every column chunk of every block covering an element
  L->cst.assign(n_m + 1, 0);
  for (int b = 0; b < nb; ++b) {
    const int n = L->boff[b + 1] - L->boff[b], ncc = (n + BCOLS - 1) / BCOLS;
    for (int i = L->boff[b]; i < L->boff[b + 1]; ++i) L->cst[L->bidx[i] + 1] += ncc;
  }
  for (int c = 0; c < n_m; ++c) L->cst[c + 1] += L->cst[c];
  L->cix.assign(L->cst[n_m], 0);
  std::vector<int> fill(L->cst.begin(), L->cst.end() - 1);
  for (int b = 0; b < nb; ++b) {
    const int n = L->boff[b + 1] - L->boff[b], ncc = (n + BCOLS - 1) / BCOLS;
    for (int i = 0; i < n; ++i)
      for (int cc = 0; cc < ncc; ++cc) L->cix[fill[L->bidx[L->boff[b] + i]]++] = (int)(segb[b] + (size_t)cc * n + i);
  }
  L->inb.assign(n_m, 0);
  for (const Run& r : L->runs)
    for (int c = r.cb0; c < r.cb0 + r.h * nx; ++c) L->inb[c] = 1;
  return 0;
}

}  // namespace fillb
