"""FP64 oracle of the library's block preconditioner for the masked system.

TEST INFRASTRUCTURE ONLY (see fill_oracle).

Not a construction of the paper: the paper preconditions its CG with powers
of C (Sec. 2.4) and treats wide cuts with noise-boosted strips (Sec. 6).  This
is an additive-Schwarz preconditioner M^-1 ~ A^-1 for A = Px C^-1 Px built on
two facts of the torus problem: C^-1 is a short-range convolution (its kernel
k = F^-1 (1/P) decays within tens of pixels for the workloads' spectra), so A
nearly decouples into the connected pieces of the mask; and on a run of fully
masked rows (a band) A is translation-invariant along x, so it splits into one
symmetric Toeplitz system per frequency kx.  The solution it leads to is the
same (it only changes the CG path); the definition below fixes the operator so
that the GPU's application of it can be checked element by element.

This module specifies the library's own operator, parameter for parameter;
it is not an oracle of the paper.  Every end-to-end check of a fill that uses
it goes through fill_oracle's solution (or a direct pin), which this
preconditioner cannot change: it only sets the CG path.

Definition (parameters BW = 32, HALO = 8, TILE = 16, CMAX = 1024, NBMAX = 2048,
pivot_min = PIVOT_MIN = 1e-9 for FP64 factors and PIVOT_MIN_F32 = 1e-4 for
FP32 factors, whose rounding the truncation's conditioning amplifies):

1. Band runs: maximal runs of consecutive rows y0..y0+h-1 (not wrapping)
   whose every pixel is masked, with h <= ny - 2 BW.
2. Band part, per run and per kx = 0..nx/2:
   t_kx(d) = sum_dx k(d mod ny, dx) cos(2 pi kx dx / nx)   (real: k is even
   in dx and, for spectra symmetric under ky -> -ky, in dy), T_kx[i, j] =
   t_kx(i - j) for |i - j| < BW and 0 beyond, plus sigma_kx on the diagonal.
   sigma_kx = 0 if the truncated matrix is safely positive definite: every
   pivot of its Cholesky factorization exceeds pivot_min times its diagonal
   entry t_kx(0); otherwise sigma_kx = 2 sum_{d = BW}^{h-1} |t_kx(d)|, a bound
   (Gershgorin) on the norm of the discarded part, so that T_kx stays positive
   definite however slowly t_kx decays (the shift costs iterations where it
   is not needed).  The band rows' part of M^-1 r is
   IDFT_x(T_kx^-1 DFT_x(r on the run)).
3. The other masked pixels (outside band runs) split into connected components
   (4-neighbours, periodic); a component of more than CMAX pixels, or whose
   grown block (step 4) would hold more than NBMAX pixels, is cut into cells by
   the absolute TILE x TILE grid, otherwise it is one cell.
4. Each cell grows into a block: every masked pixel (band rows included)
   within Chebyshev distance h (periodic) of the cell, h the halo (HALO = 8
   unless given).  The block's part of M^-1 r is A_b^-1 r_b, A_b = A
   restricted to the block's pixels.
5. M^-1 r = sum of the band parts and the block parts (overlaps add).
6. The library's default halo (auto_halo): h = 8, then 10, 12, 14 in turn
   for as long as the blocks (steps 3-4 with that h) hold at most
   floor(ny nx / 2) more inverse entries than those of h = 8, counting
   n * 4 ceil(n / 4) entries for a block of n pixels.

Each part is symmetric positive definite on its pixels and every masked pixel
is covered, so M^-1 is SPD.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.ndimage as ndi

__all__ = ["BW", "HALO", "TILE", "CMAX", "NBMAX", "PIVOT_MIN", "PIVOT_MIN_F32", "safely_pd", "kernel_cinv", "band_runs", "band_symbols", "cells", "blocks",
           "block_entries", "auto_halo", "BlockPrecond", "pcg_block"]

BW, HALO, TILE, CMAX, NBMAX = 32, 8, 16, 1024, 2048
PIVOT_MIN = 1e-9
PIVOT_MIN_F32 = 1e-4


def kernel_cinv(P: np.ndarray) -> np.ndarray:
    """k with C^-1 v = k (*) v (periodic convolution): k = irfft2(1/P)."""
    ny = P.shape[0]
    nx = 2 * (P.shape[1] - 1)
    return sfft.irfft2(1.0 / P, s=(ny, nx))


def band_runs(mask: np.ndarray, bw: int = BW) -> list:
    """[(y0, h)] of the maximal runs of fully masked rows with h <= ny - 2 bw."""
    ny = mask.shape[0]
    full = np.all(mask != 0, axis=1)
    runs, y = [], 0
    while y < ny:
        if full[y]:
            y0 = y
            while y < ny and full[y]:
                y += 1
            if y - y0 <= ny - 2 * bw:
                runs.append((y0, y - y0))
        else:
            y += 1
    return runs


def band_symbols(k: np.ndarray, nd: int = BW) -> np.ndarray:
    """t[d, kx] = sum_dx k(d, dx) cos(2 pi kx dx / nx) for d = 0..nd-1."""
    nx = k.shape[1]
    dx = np.arange(nx)
    kx = np.arange(nx // 2 + 1)
    cos = np.cos(2.0 * np.pi * np.outer(dx, kx) / nx)
    return k[:nd] @ cos


def _components(sel: np.ndarray) -> list:
    """Connected components of sel (4-neighbours, periodic): lists of (y, x)."""
    ny, nx = sel.shape
    lab, n = ndi.label(sel)
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in ((lab[:, 0], lab[:, nx - 1]), (lab[0, :], lab[ny - 1, :])):
        for u, v in zip(a, b):
            if u and v:
                ru, rv = find(u), find(v)
                if ru != rv:
                    parent[max(ru, rv)] = min(ru, rv)
    root = np.array([find(i) for i in range(n + 1)])
    lab = root[lab]
    comps = {}
    ys, xs = np.nonzero(lab)
    for y, x in zip(ys, xs):
        comps.setdefault(lab[y, x], []).append((y, x))
    return [np.array(c) for _, c in sorted(comps.items())]


def cells(mask: np.ndarray, runs: list, halo: int = HALO) -> list:
    """Cells (arrays of (y, x)) of the masked pixels outside the band runs."""
    sel = mask != 0
    for y0, h in runs:
        sel[y0:y0 + h] = False
    out = []
    for c in _components(sel):
        if len(c) <= CMAX and len(blocks(mask, [c], halo)[0]) <= NBMAX:
            out.append(c)
            continue
        key = (c[:, 0] // TILE) * (mask.shape[1] // TILE + 1) + c[:, 1] // TILE
        for kv in np.unique(key):
            out.append(c[key == kv])
    return out


def blocks(mask: np.ndarray, cell_list: list, halo: int = HALO) -> list:
    """Each cell grown by the halo (Chebyshev, periodic) within the mask:
    sorted flat pixel indices."""
    ny, nx = mask.shape
    m = mask != 0
    out = []
    for c in cell_list:
        grown = np.zeros_like(m)
        for dy in range(-halo, halo + 1):
            for dx in range(-halo, halo + 1):
                grown[(c[:, 0] + dy) % ny, (c[:, 1] + dx) % nx] = True
        ys, xs = np.nonzero(grown & m)
        out.append(np.sort(ys * nx + xs))
    return out


def block_entries(block_list: list) -> int:
    """Inverse entries of the blocks: n * 4 ceil(n / 4) for n pixels."""
    return sum(len(b) * (-(-len(b) // 4) * 4) for b in block_list)


def auto_halo(mask: np.ndarray) -> int:
    """The default halo of step 6."""
    runs = band_runs(mask)
    base = block_entries(blocks(mask, cells(mask, runs, HALO), HALO))
    best = HALO
    for h in (10, 12, 14):
        if block_entries(blocks(mask, cells(mask, runs, h), h)) > base + mask.size // 2:
            break
        best = h
    return best


def safely_pd(T: np.ndarray, pivot_min: float = PIVOT_MIN) -> bool:
    """True if the Cholesky factorization of the symmetric matrix T has every
    pivot L_ii^2 above pivot_min T_ii (False if it breaks down)."""
    try:
        L = np.linalg.cholesky(T)
    except np.linalg.LinAlgError:
        return False
    return bool(np.all(np.diag(L) ** 2 > pivot_min * np.diag(T)))


class BlockPrecond:
    """M^-1 of the definition above for one mask and spectrum (FP64
    arithmetic; pivot_min selects the threshold of the FP64 or FP32 plans;
    halo: the blocks' h, or "auto" for step 6's choice)."""

    def __init__(self, mask: np.ndarray, P: np.ndarray, bw: int = BW, pivot_min: float = PIVOT_MIN,
                 halo=HALO):
        self.mask = mask
        self.halo = auto_halo(mask) if halo == "auto" else int(halo)
        ny, nx = mask.shape
        self.shape = (ny, nx)
        k = kernel_cinv(P)
        self.runs = band_runs(mask, bw)
        t = band_symbols(k, max([h for _, h in self.runs], default=1))
        self.band_T = []
        for y0, h in self.runs:
            d = np.abs(np.arange(h)[:, None] - np.arange(h)[None, :])
            Ts = np.zeros((nx // 2 + 1, h, h))
            for kx in range(nx // 2 + 1):
                Ts[kx] = np.where(d < bw, t[d, kx], 0.0)
                if not safely_pd(Ts[kx], pivot_min):
                    Ts[kx] += 2.0 * np.abs(t[bw:h, kx]).sum() * np.eye(h)
            self.band_T.append(Ts)
        self.cells = cells(mask, self.runs, self.halo)
        self.blocks = blocks(mask, self.cells, self.halo)
        self.block_A = []
        for b in self.blocks:
            y, x = b // nx, b % nx
            self.block_A.append(k[(y[:, None] - y[None, :]) % ny, (x[:, None] - x[None, :]) % nx])

    def apply(self, r: np.ndarray) -> np.ndarray:
        """M^-1 r for a map r (values at observed pixels are ignored)."""
        ny, nx = self.shape
        r = np.where(self.mask != 0, r, 0.0)
        z = np.zeros_like(r)
        for (y0, h), Ts in zip(self.runs, self.band_T):
            R = np.fft.rfft(r[y0:y0 + h], axis=1)                  # (h, nx/2+1)
            Z = np.stack([np.linalg.solve(Ts[kx], R[:, kx]) for kx in range(nx // 2 + 1)], axis=1)
            z[y0:y0 + h] += np.fft.irfft(Z, n=nx, axis=1)
        flat = z.reshape(-1)
        rf = r.reshape(-1)
        for b, Ab in zip(self.blocks, self.block_A):
            flat[b] += np.linalg.solve(Ab, rf[b])
        return z


def pcg_block(v: np.ndarray, mask: np.ndarray, P: np.ndarray, rtol: float, max_iter: int = 20000,
              M: BlockPrecond | None = None):
    """Solve A u = v (Sec. 2.4's system) by Hestenes-Stiefel PCG from u = 0
    with M^-1 the block preconditioner; stop when the recursive residual
    reaches rtol ||v||, then recompute it and restart if it is too large.
    Returns (u, PCGInfo) with the first run's alpha_j and beta_j."""
    from .fill_oracle import PCGInfo, apply_A
    M = M or BlockPrecond(mask, P)
    vnorm = float(np.linalg.norm(v))
    u = np.zeros_like(v)
    alphas, betas = [], []
    total = 0
    if vnorm == 0.0:
        return u, PCGInfo(0, 0.0, True, [])
    r = v.copy()
    rel = 1.0
    for restart in range(20):
        z = M.apply(r)
        p = z.copy()
        rz = float(np.vdot(r, z))
        done = False
        while total < max_iter:
            q = apply_A(p, mask, P)
            alpha = rz / float(np.vdot(p, q))
            if restart == 0:
                alphas.append(alpha)
            u += alpha * p
            r -= alpha * q
            total += 1
            rel = float(np.linalg.norm(r)) / vnorm
            if rel <= rtol:
                done = True
                break
            z = M.apply(r)
            rz_new = float(np.vdot(r, z))
            if restart == 0:
                betas.append(rz_new / rz)
            p = z + (rz_new / rz) * p
            rz = rz_new
        r = v - apply_A(u, mask, P)
        rel = float(np.linalg.norm(r)) / vnorm
        if rel <= rtol or not done:
            break
    return u, PCGInfo(total, rel, rel <= rtol, [], alphas, betas)
