"""FP64 oracle of the noise-boosted strip refinement (Sec. 6.2 and 6.4) on the torus.

TEST INFRASTRUCTURE ONLY (see fill_oracle).

Subdivision (Sec. 6.2): the observed region R0 gets indicator 1, the masked
region 0; the indicator is convolved with a top-hat disk and the masked
pixels where the disk average exceeds a small threshold (0.03) lie near the
boundary.  Here the disk of radius w holds the offsets with dx^2 + dy^2 <= w^2
(periodic), the convolution is the integer count of observed pixels in it,
and a masked pixel belongs to the strip of width w when
count > threshold * (pixels in the disk).

Refinement (Sec. 6.4): strips D_1 > ... > D_n of widths w_1 > ... > w_n with
noise boosts beta_1 > ... > beta_n = 1.  Starting from a map (masked pixels
0 here), each step solves the maximum-likelihood fill of the pixels of D_i,
taking every other pixel of the current map as data, with spectrum
P_signal + beta_i N, by a fixed number of CG iterations (split form, Sec. 2.4),
and writes the result into D_i.
"""

from __future__ import annotations

import numpy as np

from . import fill_oracle as F

__all__ = ["disk_offsets", "observed_counts", "strip_mask", "strip_fill"]


def disk_offsets(w: float) -> np.ndarray:
    """Integer offsets (dy, dx) with dy^2 + dx^2 <= w^2."""
    r = int(np.floor(w))
    dy, dx = np.mgrid[-r:r + 1, -r:r + 1]
    keep = dy * dy + dx * dx <= w * w
    return np.stack([dy[keep], dx[keep]], axis=1)


def observed_counts(mask: np.ndarray, w: float) -> np.ndarray:
    """Number of observed pixels in the periodic disk of radius w around each
    pixel: the top-hat convolution of the observed indicator, by FFT, rounded
    to the integer it is.  The disk must fit the torus: 2 floor(w) + 1 <= min(nx, ny)."""
    ny, nx = mask.shape
    if 2 * int(np.floor(w)) + 1 > min(nx, ny):
        raise ValueError(f"disk of radius {w} does not fit a {nx}x{ny} torus")
    obs = (mask == 0).astype(np.float64)
    ker = np.zeros((ny, nx))
    off = disk_offsets(w)
    ker[off[:, 0] % ny, off[:, 1] % nx] = 1.0
    conv = np.fft.irfft2(np.fft.rfft2(obs) * np.fft.rfft2(ker), s=(ny, nx))
    return np.rint(conv).astype(np.int64)


def strip_mask(mask: np.ndarray, w: float, threshold: float = 0.03) -> np.ndarray:
    """Masked pixels within (about) w of the observed region: uint8 0/1."""
    area = len(disk_offsets(w))
    return ((mask != 0) & (observed_counts(mask, w) > threshold * area)).astype(np.uint8)


def strip_fill(d_obs, mask, P_signal, noise, betas, widths, iters, threshold=0.03,
               start=None) -> tuple[np.ndarray, list]:
    """The strip sequence of Sec. 6.4: returns (filled map, strip masks)."""
    x = np.where(mask != 0, 0.0, d_obs) if start is None else np.where(mask != 0, start, d_obs)
    strips = []
    for beta, w in zip(betas, widths):
        D = strip_mask(mask, w, threshold)
        strips.append(D)
        if not D.any():
            continue
        P = P_signal + beta * noise
        v = F.rhs(np.where(D != 0, 0.0, x), D, P)
        u, _ = F.pcg_split(v, D, P, rtol=0.0, max_iter=iters)
        x = np.where(D != 0, u, x)
    return x, strips
