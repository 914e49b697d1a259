"""FP64 oracle of the kernel-based Laplace solver (Sec. 6.1, 6.3) on the torus.

TEST INFRASTRUCTURE ONLY (see fill_oracle).

In the far interior of a wide masked region the maximum-likelihood fill
nearly solves the Laplace equation (Sec. 6.1).  A harmonic function equals
its average over any annulus centred on a point, so relaxation replaces each
masked value by such an average; to converge in a number of sweeps that grows
only like a power of log(width), every pixel uses the largest kernel of a
geometric series that stays inside the masked region, and the pixels of the
thin boundary layer use the smallest, solid kernel, which reaches the data
(Sec. 6.3).

Here kernel j (j = 0..K-1) is the annulus of offsets with
r_{j-1}^2 < dx^2 + dy^2 <= r_j^2 (r_{-1} = 0, so kernel 0 is the disk of radius
r_0 without its centre), r_j = r_0 ratio^j, normalised to sum 1; a masked
pixel takes the largest j >= 1 whose whole disk of radius r_j is masked, else
j = 0.  Each sweep (Jacobi) computes every needed kernel average of the
current map by FFT convolution and writes it to the pixels of that class;
observed pixels keep the data, masked pixels start at 0 (or at `start`).
"""

from __future__ import annotations

import numpy as np

from .strips import observed_counts

__all__ = ["laplace_radii", "annulus_offsets", "kernel_classes", "laplace_fill"]


def laplace_radii(nkernels: int, r0: float = 1.5, ratio: float = 2.0) -> list:
    return [r0 * ratio ** j for j in range(nkernels)]


def annulus_offsets(r_in: float, r_out: float) -> np.ndarray:
    """Integer offsets (dy, dx) with r_in^2 < dy^2 + dx^2 <= r_out^2."""
    r = int(np.floor(r_out))
    dy, dx = np.mgrid[-r:r + 1, -r:r + 1]
    d2 = dy * dy + dx * dx
    keep = (d2 > r_in * r_in) & (d2 <= r_out * r_out)
    return np.stack([dy[keep], dx[keep]], axis=1)


def kernel_classes(mask: np.ndarray, radii) -> np.ndarray:
    """Kernel index per masked pixel (-1 on observed pixels)."""
    cls = np.where(mask != 0, 0, -1)
    for j in range(1, len(radii)):
        inside = (mask != 0) & (observed_counts(mask, radii[j]) == 0)
        cls[inside] = j
    return cls


def _kernel_spectrum(j: int, radii, shape) -> np.ndarray:
    ny, nx = shape
    off = annulus_offsets(0.0 if j == 0 else radii[j - 1], radii[j])
    ker = np.zeros(shape)
    ker[off[:, 0] % ny, off[:, 1] % nx] = 1.0 / len(off)
    return np.fft.rfft2(ker)


def laplace_fill(d_obs: np.ndarray, mask: np.ndarray, radii, iters: int, start=None):
    """(filled map, masked-pixel update norm per sweep)."""
    m = mask != 0
    cls = kernel_classes(mask, radii)
    used = [j for j in range(len(radii)) if np.any(cls == j)]
    spectra = {j: _kernel_spectrum(j, radii, mask.shape) for j in used}
    x = np.where(m, 0.0 if start is None else start, d_obs)
    hist = []
    for _ in range(iters):
        X = np.fft.rfft2(x)
        xn = x.copy()
        for j in used:
            avg = np.fft.irfft2(X * spectra[j], s=mask.shape)
            sel = cls == j
            xn[sel] = avg[sel]
        hist.append(float(np.linalg.norm((xn - x)[m])))
        x = xn
    return x, hist
