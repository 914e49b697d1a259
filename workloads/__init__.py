"""Seeded synthetic inputs for the flat-sky constrained-realization fill-in.

This module builds the *inputs* of the method and nothing else: the power
spectrum table P(k) on the half-spectrum grid, the mask (a band of rows, the
flat stand-in for a Galactic cut, plus circular point-source holes) and an
observed map drawn from P(k).  It holds none of the method's arithmetic (no
operator, no solve, no realization of the constrained field); both the GPU
path and the CPU oracle take its arrays as they are.

Conventions (shared by every consumer):

* maps are float64 arrays of shape (ny, nx), row-major, pixel (y, x);
* the mask is uint8 of shape (ny, nx), 1 = masked (unobserved, the paper's
  x block), 0 = observed (the y block), Sec. 2.1;
* the spectrum table has shape (ny, nx//2 + 1): entry [iy, ix] is P at the
  integer frequency (ky, kx) with kx = ix and ky = iy for iy <= ny/2, else
  iy - ny; k = sqrt(kx^2 + ky^2).  P(k) is the eigenvalue of the circulant
  pixel covariance C = F^-1 diag(P) F with F the unnormalised 2D DFT, so the
  pixel variance is the mean of P over the full frequency grid.  The spectra
  follow the paper's model of a beam-damped CMB spectrum plus a white-noise
  floor (Sec. 3, P = w C + N);
* masked pixels of the observed map are set to zero, as the paper does for
  its point-source mask (Sec. 3).

The observed map is a Gaussian field with spectrum P, drawn with numpy's
PCG64 normal generator and shaped with numpy.fft; it is input data (the
paper's simulated sky maps), not part of the fill.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "kgrid",
    "damped_power_law",
    "laplacian_spectrum",
    "band_rows",
    "band_holes_mask",
    "observed_map",
    "Problem",
    "make_problem",
    "CONFIGS",
    "make_mixed_batch",
]


def kgrid(nx: int, ny: int) -> np.ndarray:
    """|k| on the half-spectrum grid, shape (ny, nx//2+1), integer frequencies."""
    kx = np.arange(nx // 2 + 1, dtype=np.float64)
    ky = np.fft.fftfreq(ny, d=1.0 / ny)  # 0..ny/2-1, -ny/2..-1 (Nyquist as -ny/2)
    return np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)


def damped_power_law(nx: int, ny: int, k0sq: float, damping: float, floor: float) -> np.ndarray:
    """P(k) = (k^2 + k0sq)^-1 * exp(-(k/damping)^2) + floor on the half grid.

    Signal ~ k^-2 (the scale-invariant case of Sec. 2.2) regularised at low k,
    a Gaussian beam damping, and a white-noise floor N (Sec. 3, P = w C + N).
    """
    k = kgrid(nx, ny)
    return 1.0 / (k * k + k0sq) * np.exp(-((k / damping) ** 2)) + floor


def laplacian_spectrum(nx: int, ny: int, mu2: float) -> np.ndarray:
    """Spectrum whose inverse is the screened 5-point Laplacian.

    1/P = 4 - 2 cos(2 pi kx/nx) - 2 cos(2 pi ky/ny) + mu2, so C^-1 is exactly
    the discrete -Laplacian + mu2 on the torus: the lattice analogue of the
    paper's scale-invariant toy model where C^-1 is the Laplacian (Sec. 2.2,
    Sec. 6.1).  Used only to pin the oracle against closed forms.
    """
    kx = np.arange(nx // 2 + 1, dtype=np.float64)
    ky = np.fft.fftfreq(ny, d=1.0 / ny)
    inv = (4.0 - 2.0 * np.cos(2 * np.pi * kx[None, :] / nx)
           - 2.0 * np.cos(2 * np.pi * ky[:, None] / ny) + mu2)
    return 1.0 / inv


def band_rows(ny: int, frac: float) -> tuple[int, int]:
    """A centred band of round(frac*ny) rows: returns (first_row, n_rows)."""
    h = int(round(frac * ny))
    return (ny - h) // 2, h


def band_holes_mask(nx: int, ny: int, band: tuple[int, int] | None, n_holes: int,
                    rmin: float, rmax: float, mask_seed: int) -> np.ndarray:
    """Band of rows plus circular holes (periodic minimum-image disks).

    band = (first_row, n_rows) or None.  Hole centres are integer-uniform on
    the grid, radii continuous-uniform in [rmin, rmax]; overlaps are allowed.
    A pixel is in a hole when dx^2 + dy^2 <= r^2 with dx, dy the periodic
    minimum-image offsets.
    """
    m = np.zeros((ny, nx), dtype=np.uint8)
    if band is not None:
        r0, h = band
        m[r0:r0 + h, :] = 1
    rng = np.random.default_rng(mask_seed)
    if n_holes > 0:
        cx = rng.integers(0, nx, size=n_holes)
        cy = rng.integers(0, ny, size=n_holes)
        rad = rng.uniform(rmin, rmax, size=n_holes)
        for x0, y0, r in zip(cx, cy, rad):
            ri = int(math.ceil(r))
            dy = np.arange(-ri, ri + 1)
            dx = np.arange(-ri, ri + 1)
            inside = dx[None, :] ** 2 + dy[:, None] ** 2 <= r * r
            yy = (y0 + dy) % ny
            xx = (x0 + dx) % nx
            sub = m[np.ix_(yy, xx)]
            m[np.ix_(yy, xx)] = np.maximum(sub, inside.astype(np.uint8))
    return m


def observed_map(P: np.ndarray, nx: int, ny: int, seed: int, mask: np.ndarray | None = None) -> np.ndarray:
    """A Gaussian map with spectrum P (input data), masked pixels set to 0."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, nx))
    d = np.fft.irfft2(np.sqrt(P) * np.fft.rfft2(w), s=(ny, nx))
    d = np.ascontiguousarray(d, dtype=np.float64)
    if mask is not None:
        d[mask != 0] = 0.0
    return d


@dataclass
class Problem:
    """One fill-in problem: grid, spectrum, mask, observed map, seed, tolerance."""
    name: str
    nx: int
    ny: int
    P: np.ndarray
    mask: np.ndarray
    d_obs: np.ndarray
    seed: int
    rtol: float
    meta: dict = field(default_factory=dict)

    @property
    def n_masked(self) -> int:
        return int(self.mask.sum())


# The workloads, with the sizes and structure of the paper's experiments
# (ACT-like point-source holes, Galactic-band cuts, Sec. 3).
CONFIGS = {
    # 64^2 plain FP64: band rows 28-35 + 5 holes of radius 3.
    "grid64": dict(n=64, k0sq=1.0, damping=8.0, floor=1e-6, band=(28, 8), n_holes=5,
                   rmin=3.0, rmax=3.0, mask_seed=1, dobs_seed=0, seed=1, rtol=1e-10),
    # 2048^2: 10% band + 200 holes r~U(2,12).
    "grid2048": dict(n=2048, k0sq=4.0, damping=256.0, floor=1e-7, band_frac=0.10, n_holes=200,
                     rmin=2.0, rmax=12.0, mask_seed=2, dobs_seed=0, seed=1, rtol=1e-8),
    # 2048^2 point sources only: the 200 holes of the 2048^2 workload, no band.
    "holes2048": dict(n=2048, k0sq=4.0, damping=256.0, floor=1e-7, band_frac=0.0, n_holes=200,
                      rmin=2.0, rmax=12.0, mask_seed=2, dobs_seed=0, seed=1, rtol=1e-8),
    # 4096^2 wide cut: 30% band + 500 holes r~U(2,16).
    "grid4096": dict(n=4096, k0sq=4.0, damping=512.0, floor=1e-7, band_frac=0.30, n_holes=500,
                     rmin=2.0, rmax=16.0, mask_seed=4, dobs_seed=0, seed=1, rtol=1e-8),
}


def make_problem(name: str = "grid2048", n: int | None = None, **over) -> Problem:
    """Build a named workload; n rescales the grid keeping the band fraction,
    the damping scale (as a fraction of n) and the hole count per area."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    n0 = cfg["n"]
    n = n or n0
    scale = n / n0
    damping = cfg["damping"] * scale
    P = damped_power_law(n, n, cfg["k0sq"], damping, cfg["floor"])
    if "band_frac" in cfg:
        band = band_rows(n, cfg["band_frac"])
    else:
        r0, h = cfg["band"]
        band = (int(round(r0 * scale)), max(1, int(round(h * scale))))
    n_holes = int(round(cfg["n_holes"] * scale * scale)) if n != n0 else cfg["n_holes"]
    mask = band_holes_mask(n, n, band, n_holes, cfg["rmin"], cfg["rmax"], cfg["mask_seed"])
    d = observed_map(P, n, n, cfg["dobs_seed"], mask)
    return Problem(name=f"{name}@{n}", nx=n, ny=n, P=P, mask=mask, d_obs=d, seed=cfg["seed"],
                   rtol=cfg["rtol"], meta=dict(band=band, n_holes=n_holes, damping=damping, **{
                       k: cfg[k] for k in ("k0sq", "floor", "rmin", "rmax", "mask_seed", "dobs_seed")}))


def make_mixed_batch(nprob: int = 64, sizes=(256, 512, 768, 1024), seed: int = 2024) -> list[Problem]:
    """Monte-Carlo batch of uneven grids: problem i has n ~ U{sizes}, a band of
    U(5, 20)% of the rows plus U{20..100} holes of radius U(2, 10) px (mask
    seed 1000 + i), P of the 2048^2 form with damping n/8, observed map seed
    2 i and fill seed 2 i + 1; tolerance 1e-6."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nprob):
        n = int(rng.choice(sizes))
        frac = float(rng.uniform(0.05, 0.20))
        nh = int(rng.integers(20, 101))
        P = damped_power_law(n, n, 4.0, n / 8.0, 1e-7)
        mask = band_holes_mask(n, n, band_rows(n, frac), nh, 2.0, 10.0, 1000 + i)
        d = observed_map(P, n, n, 2 * i, mask)
        out.append(Problem(name=f"batch{i}@{n}", nx=n, ny=n, P=P, mask=mask, d_obs=d, seed=2 * i + 1,
                           rtol=1e-6, meta=dict(band_frac=frac, n_holes=nh, damping=n / 8.0)))
    return out
