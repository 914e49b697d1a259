"""Pins: forms of the fill-in solution computed without the oracle's code.

Shared by the oracle pin tests and the GPU parity tests.  Nothing here
imports the oracle or the GPU package.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W

# --------------------------------------------------------------------------
# helpers (pins): brute-force forms built without the oracle's FFT code path
# --------------------------------------------------------------------------

def _p_of_k(k, k0sq, damping, floor):
    return 1.0 / (k * k + k0sq) * np.exp(-((k / damping) ** 2)) + floor


def _dft_matrix(nx, ny):
    """Explicit 2D DFT matrix F[k, r] = exp(-2 pi i (kx x / nx + ky y / ny))."""
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    ky, kx = iy, ix  # full frequency grid in the same row-major order
    ph = np.outer(kx, ix) / nx + np.outer(ky, iy) / ny
    return np.exp(-2j * np.pi * ph), kx, ky


def _full_spectrum(nx, ny, fn):
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    kxs = np.where(ix <= nx // 2, ix, ix - nx)
    kys = np.where(iy <= ny // 2, iy, iy - ny)
    return fn(np.sqrt(kxs ** 2.0 + kys ** 2.0))


def brute_circulant(nx, ny, fn, power):
    Fm, _, _ = _dft_matrix(nx, ny)
    Pf = _full_spectrum(nx, ny, fn)
    return (Fm.conj().T @ np.diag(Pf ** power) @ Fm / (nx * ny)).real


def brute_circulant_case(nx=8, ny=6, power=-1.0, seed=3, table=None):
    """(P table, input v, expected C^power v) on a tiny grid by explicit DFT matrices."""
    fn = lambda k: _p_of_k(k, 1.0, 2.5, 1e-3)  # noqa: E731
    P = W.damped_power_law(nx, ny, 1.0, 2.5, 1e-3) if table is None else table
    v = np.random.default_rng(seed).standard_normal((ny, nx))
    ref = (brute_circulant(nx, ny, fn, power) @ v.ravel()).reshape(ny, nx)
    return P, v, ref


def band_direct(t, r0, h, fn):
    """x_ML for a band mask (rows r0..r0+h-1), one dense solve per x-frequency.

    A band mask is invariant under x-translations, so after a 1D DFT along x
    the system decouples: for each kx the operator along y is the circulant
    Q(j, j') = (1/ny) sum_ky exp(2 pi i ky (j - j')/ny) / P(kx, ky), and
    x_ML = -Q_xx^-1 Q_xy y on the band rows (Sec. 2.1).
    """
    ny, nx = t.shape
    that = np.fft.fft(t, axis=1)
    j = np.arange(ny)
    xb = np.zeros(ny, bool)
    xb[r0:r0 + h] = True
    kys = np.fft.fftfreq(ny, d=1.0 / ny)
    uh = np.zeros((ny, nx), complex)
    jb = j[xb]
    lag = (jb[:, None] - j[None, :]) % ny  # rows of Q on the band only
    for kx in range(nx // 2 + 1):
        q = np.fft.ifft(1.0 / fn(np.sqrt(kx ** 2 + kys ** 2)))
        Qx = q[lag]
        uh[xb, kx] = -np.linalg.solve(Qx[:, xb], Qx[:, ~xb] @ that[~xb, kx])
        if 0 < kx < nx - kx:  # the real field's spectrum is Hermitian in kx
            uh[xb, nx - kx] = np.conj(uh[xb, kx])
    return np.fft.ifft(uh, axis=1).real


def band_direct_modes(t, r0, h, fn, kxs):
    """The x-frequency modes kxs of x_ML on the band rows r0..r0+h-1, each by
    its own dense solve (band_direct for a sample of frequencies, for grids
    where solving every kx would take too long): out[:, i] is the 1D DFT
    along x (numpy's forward convention) of x_ML on the band rows at
    kx = kxs[i]."""
    ny, nx = t.shape
    j = np.arange(ny)
    xb = np.zeros(ny, bool)
    xb[r0:r0 + h] = True
    kys = np.fft.fftfreq(ny, d=1.0 / ny)
    jb = j[xb]
    lag = (jb[:, None] - j[None, :]) % ny
    that = np.fft.fft(t, axis=1)
    out = np.zeros((h, len(kxs)), complex)
    for i, kx in enumerate(kxs):
        q = np.fft.ifft(1.0 / fn(np.sqrt(kx ** 2 + kys ** 2)))
        Qx = q[lag]
        out[:, i] = -np.linalg.solve(Qx[:, xb], Qx[:, ~xb] @ that[~xb, kx])
    return out


def laplace_band_closed_form(y, r0, h, mu2):
    """Lattice analogue of the periodic-strip Laplace solution (Sec. 6.1).

    With C^-1 the screened 5-point Laplacian, the ML field in a band of rows
    r0..r1 obeys (4 + mu2) z - (sum of 4 neighbours) = 0; per x-frequency
    z_k(j) = [sinh(th (j1 - j)) z_k(j0) + sinh(th (j - j0)) z_k(j1)] / sinh(th L)
    with j0 = r0 - 1, j1 = r1 + 1, L = j1 - j0 and
    cosh th = 1 + mu2/2 + 2 sin^2(pi kx / nx).
    """
    ny, nx = y.shape
    j0, j1 = r0 - 1, r0 + h
    L = j1 - j0
    kx = np.arange(nx)
    th = np.arccosh(1.0 + mu2 / 2.0 + 2.0 * np.sin(np.pi * kx / nx) ** 2)
    a, b = np.fft.fft(y[j0]), np.fft.fft(y[j1])
    out = np.zeros((ny, nx))
    for j in range(r0, r0 + h):
        zk = (np.sinh(th * (j1 - j)) * a + np.sinh(th * (j - j0)) * b) / np.sinh(th * L)
        out[j] = np.fft.ifft(zk).real
    return out


def laplace_sparse_direct(y, mask, mu2):
    """ML field for the 5-point Laplacian precision by sparse direct elimination."""
    ny, nx = mask.shape
    m = mask.ravel() != 0
    idx = -np.ones(nx * ny, int)
    idx[m] = np.arange(m.sum())
    rows, cols, vals = [], [], []
    rhs = np.zeros(m.sum())
    yf = y.ravel()
    for p in np.nonzero(m)[0]:
        i = idx[p]
        rows.append(i); cols.append(i); vals.append(4.0 + mu2)  # noqa: E702
        py, px = divmod(p, nx)
        for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            q = ((py + dy) % ny) * nx + (px + dx) % nx
            if m[q]:
                rows.append(i); cols.append(idx[q]); vals.append(-1.0)  # noqa: E702
            else:
                rhs[i] += yf[q]
    A = sp.csc_matrix((vals, (rows, cols)), shape=(m.sum(), m.sum()))
    out = np.zeros(nx * ny)
    out[m] = spla.spsolve(A, rhs)
    return out.reshape(ny, nx)


def rel(a, b, m=None):
    if m is not None:
        a, b = a[m], b[m]
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))




def masked_circulant_block(P, mask, power):
    """Dense block of C^power on the masked pixels, C the circulant with
    eigenvalues P (rows/columns in row-major masked-pixel order).  Built from
    the covariance function by numpy's inverse FFT and index arithmetic."""
    ny, nx = mask.shape
    xi = np.fft.irfft2(P ** power, s=(ny, nx))
    iy, ix = np.divmod(np.flatnonzero(mask.ravel() != 0), nx)
    return xi[(iy[:, None] - iy[None, :]) % ny, (ix[:, None] - ix[None, :]) % nx]


def explicit_lanczos(M, q0, k):
    """k steps of Lanczos with full reorthogonalisation on the dense symmetric
    matrix M from q0: returns (diagonal, off-diagonal) of the tridiagonal."""
    n = M.shape[0]
    Q = np.zeros((n, k + 1))
    Q[:, 0] = q0 / np.linalg.norm(q0)
    a = np.zeros(k)
    b = np.zeros(k)
    for j in range(k):
        w = M @ Q[:, j]
        a[j] = Q[:, j] @ w
        w -= Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        w -= Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        b[j] = np.linalg.norm(w)
        Q[:, j + 1] = w / b[j]
    return a, b[:k - 1]
