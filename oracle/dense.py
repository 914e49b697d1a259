"""Dense FP64 forms of the conditional Gaussian (small grids only).

TEST INFRASTRUCTURE ONLY (see fill_oracle).  O(N^3) in the pixel count.

On a small torus the pixel covariance is formed as an explicit N x N matrix
and the constrained draw is written out as the textbook conditional Gaussian
(Sec. 2.1, Sec. 2.3, eq. starH):

    M = C_xy C_yy^-1,   x_out[x] = s_x + M (y - s_y),
    conditional covariance  C_xx - C_xy C_yy^-1 C_yx,

with C_yy factored by Cholesky, as in the paper's brute-force discussion
(Sec. 2.3) and its validation by direct elimination (Sec. 6.5).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = ["covariance_function", "dense_covariance", "conditional_mean_dense",
           "conditional_covariance_dense"]


def covariance_function(P: np.ndarray) -> np.ndarray:
    """xi(r) = (1/N) sum_k P(k) exp(2 pi i k.r / N): C_ij = xi(r_i - r_j)."""
    ny = P.shape[0]
    nx = 2 * (P.shape[1] - 1)
    return np.fft.irfft2(P, s=(ny, nx))


def dense_covariance(P: np.ndarray) -> np.ndarray:
    """The N x N circulant pixel covariance, pixels in row-major order."""
    ny = P.shape[0]
    nx = 2 * (P.shape[1] - 1)
    xi = covariance_function(P)
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    dy = (iy[:, None] - iy[None, :]) % ny
    dx = (ix[:, None] - ix[None, :]) % nx
    return xi[dy, dx]


def conditional_mean_dense(t: np.ndarray, mask: np.ndarray, P: np.ndarray) -> np.ndarray:
    """u = C_xy C_yy^-1 t_y on masked pixels (zero elsewhere)."""
    C = dense_covariance(P)
    m = mask.ravel() != 0
    Cyy = C[np.ix_(~m, ~m)]
    Cxy = C[np.ix_(m, ~m)]
    cf = sla.cho_factor(Cyy, lower=True)
    u = np.zeros(mask.size)
    u[m] = Cxy @ sla.cho_solve(cf, t.ravel()[~m])
    return u.reshape(mask.shape)


def conditional_covariance_dense(mask: np.ndarray, P: np.ndarray) -> np.ndarray:
    """C_xx - C_xy C_yy^-1 C_yx (eq. starH), masked pixels in row-major order."""
    C = dense_covariance(P)
    m = mask.ravel() != 0
    Cyy = C[np.ix_(~m, ~m)]
    Cxy = C[np.ix_(m, ~m)]
    Cxx = C[np.ix_(m, m)]
    cf = sla.cho_factor(Cyy, lower=True)
    return Cxx - Cxy @ sla.cho_solve(cf, Cxy.T)
