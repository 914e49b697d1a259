"""FP64 oracle of the gradient of a loss on the filled map (adjoint of the fill).

TEST INFRASTRUCTURE ONLY (see fill_oracle).

Spectrum parameterisation: band powers theta_b = ln P(k_b) at nodes k_b
(log-spaced), ln P(k) piecewise linear in ln k between nodes and constant
outside [k_1, k_B]; k = 0 takes theta_1.  So P(k) = exp(sum_b phi_b(k)
theta_b) with hat weights phi_b.

Loss: L = sum over all pixels of wts * x_out^2, x_out the constrained
realization of Sec. 2.3 (x_out = y on observed pixels, s_x + M (y - s_y) on
masked ones) for a fixed seed.

Adjoint (derived from the construction of Sec. 2.1 and 2.3; the paper does
not differentiate the fill).  With g = dL/dx_out = 2 wts x_out:
* lambda = A^-1 g_x, A = Px C^-1 Px (one extra CG solve with the same operator);
* dL/dy = g_y - (C^-1 lambda~)_y on observed pixels, 0 on masked ones;
* with h = Px g + Py C^-1 lambda~ (dL/ds) and v = Py (y - s) + Px u,
  dL/d ln P_k = (1/N) [ 1/2 sqrt(P_k) Re(conj(h_k) w_k) + Re(conj(lambda_k) v_k) / P_k ]
  per mode k of the full frequency grid (w the white noise, ^ the unnormalised
  DFT); on the half spectrum the interior columns carry weight 2;
* dL/d theta_b = sum_k phi_b(k) dL/d ln P_k.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import fill_oracle as F
from .fill_oracle import _Px, _Py

__all__ = ["band_nodes", "band_weights", "pk_from_bands", "fill_loss", "adjoint_gradient",
           "dense_torch_loss_and_grad", "half_spectrum_weights"]


def band_nodes(n: int, nbands: int = 50) -> np.ndarray:
    """ln k of nbands nodes log-spaced in [1, sqrt(2) n/2]."""
    return np.linspace(0.0, np.log(np.sqrt(2.0) * n / 2.0), nbands)


def band_weights(nx: int, ny: int, lnk: np.ndarray) -> np.ndarray:
    """phi[b, iy, ix]: hat weights of ln|k| on the nodes lnk (half-spectrum grid)."""
    kx = np.arange(nx // 2 + 1, dtype=np.float64)
    ky = np.fft.fftfreq(ny, d=1.0 / ny)
    k = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    lk = np.log(np.maximum(k, 1e-300))
    lk = np.where(k == 0.0, lnk[0], lk)
    nb = len(lnk)
    phi = np.zeros((nb,) + k.shape)
    lo = lk <= lnk[0]
    hi = lk >= lnk[-1]
    phi[0][lo] = 1.0
    phi[-1][hi] = 1.0
    mid = ~(lo | hi)
    j = np.searchsorted(lnk, lk[mid], side="right") - 1
    t = (lk[mid] - lnk[j]) / (lnk[j + 1] - lnk[j])
    idx = np.nonzero(mid)
    for b in range(nb - 1):
        sel = j == b
        phi[b][idx[0][sel], idx[1][sel]] += 1.0 - t[sel]
        phi[b + 1][idx[0][sel], idx[1][sel]] += t[sel]
    return phi


def pk_from_bands(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """P(k) = exp(sum_b phi_b(k) theta_b)."""
    return np.exp(np.tensordot(theta, phi, axes=(0, 0)))


def half_spectrum_weights(nx: int, ny: int) -> np.ndarray:
    """Multiplicity of each half-spectrum entry in the full DFT grid (1 or 2)."""
    w = np.full((ny, nx // 2 + 1), 2.0)
    w[:, 0] = 1.0
    w[:, nx // 2] = 1.0
    return w


def fill_loss(d_obs, mask, theta, phi, seed, wts, rtol=1e-13) -> float:
    P = pk_from_bands(theta, phi)
    x = F.fill_realize(d_obs, mask, P, seed, rtol).x_out
    return float(np.sum(wts * x * x))


def adjoint_gradient(d_obs, mask, theta, phi, seed, wts, rtol=1e-13, solver="split"):
    """(L, dL/dy, dL/d ln P half-spectrum, dL/dtheta) by the adjoint recipe
    above.  solver: the oracle CG of both solves (fill_oracle's "split" or
    "cxx"; both stop on the same true residual)."""
    ny, nx = d_obs.shape
    N = nx * ny
    P = pk_from_bands(theta, phi)
    r = F.fill_realize(d_obs, mask, P, seed, rtol, solver=solver)
    x, s, u = r.x_out, r.s, r.u
    L = float(np.sum(wts * x * x))
    g = 2.0 * wts * x
    lam, _ = F._solve(_Px(g, mask), mask, P, rtol, 20000, solver)
    cl = F.circulant_apply(lam, P, -1.0)
    grad_y = _Py(g - cl, mask)
    h = _Px(g, mask) + _Py(cl, mask)
    v = _Py(d_obs - s, mask) + _Px(u, mask)
    w = F.white_noise(nx, ny, seed)
    hk, wk, lk, vk = (sfft.rfft2(a) for a in (h, w, lam, v))
    gP = (0.5 * np.sqrt(P) * np.real(np.conj(hk) * wk) + np.real(np.conj(lk) * vk) / P) / N
    gP = gP * half_spectrum_weights(nx, ny)
    gtheta = np.tensordot(phi, gP, axes=([1, 2], [0, 1]))
    return L, grad_y, gP, gtheta


def dense_torch_loss_and_grad(d_obs, mask, theta, phi, seed, wts):
    """The same loss through the dense conditional Gaussian (Cholesky of C_yy),
    differentiated by torch autograd on the CPU in FP64: an independent check
    of the adjoint recipe on small grids."""
    import torch
    ny, nx = d_obs.shape
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    y = torch.tensor(np.where(mask != 0, 0.0, d_obs), dtype=torch.float64, requires_grad=True)
    ph = torch.tensor(phi, dtype=torch.float64)
    P = torch.exp(torch.tensordot(th, ph, dims=([0], [0])))
    w = torch.tensor(F.white_noise(nx, ny, seed), dtype=torch.float64)
    s = torch.fft.irfft2(torch.sqrt(P) * torch.fft.rfft2(w), s=(ny, nx))
    xi = torch.fft.irfft2(P, s=(ny, nx))
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    m = mask.ravel() != 0
    ox, oy = np.nonzero(m)[0], np.nonzero(~m)[0]
    def cov(a, b):
        dy = (iy[a][:, None] - iy[b][None, :]) % ny
        dx = (ix[a][:, None] - ix[b][None, :]) % nx
        return xi[torch.tensor(dy), torch.tensor(dx)]
    Cyy = cov(oy, oy)
    Cxy = cov(ox, oy)
    t = (y.reshape(-1) - s.reshape(-1))[torch.tensor(oy)]
    Lc = torch.linalg.cholesky(Cyy)
    u = Cxy @ torch.cholesky_solve(t[:, None], Lc)[:, 0]
    xo = y.reshape(-1).clone()
    xo = xo.index_put((torch.tensor(ox),), s.reshape(-1)[torch.tensor(ox)] + u)
    L = torch.sum(torch.tensor(wts.ravel(), dtype=torch.float64) * xo * xo)
    L.backward()
    gy = y.grad.numpy().copy()
    gy[mask != 0] = 0.0
    return float(L.detach()), gy, th.grad.numpy().copy()
