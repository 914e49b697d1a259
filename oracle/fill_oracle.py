"""FP64 CPU oracle for the flat-sky constrained Gaussian realization fill-in.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU path and imports nothing from it.

Reference: Bucher & Louis, "Filling in CMB map missing data using constrained
Gaussian realizations" (arXiv:1109.0286).

What is computed (plain definitions, FP64):

* Pixel model (Sec. 2.1): z = (x, y), x the masked pixels, y the observed
  ones, z ~ N(0, C) with C = P + N.  On the periodic flat domain (Sec. 3) C is
  circulant: C v = F^-1 [P(k) * F v] with F the unnormalised 2D DFT, so
  C^a v = irfft2(P^a * rfft2(v)) for any power a.
* Conditional mean, Sec. 2.1:  x_ML = -((C^-1)_xx)^-1 (C^-1)_xy y
  = -(Px C^-1 Px)^-1 (Px C^-1 Py) y = M y.
* Hoffman-Ribak construction, Sec. 2.3: draw an unconstrained s ~ N(0, C);
  the constrained draw is x = s_x + M (y - s_y), y unchanged.
* Solve of (Px C^-1 Px) u = v (eq. ModEq) by conjugate gradients on the
  paper's split-preconditioned system (Sec. 2.4):
  (E A E) u' = E v,  u = E u',  with A = Px C^-1 Px and E = Px C^{1/2} Px.

Readings of the paper used here (ambiguous or garbled passages):

* the sign of x_ML follows the Sec. 2.1 derivation (with the minus sign); the
  introduction's version drops it;
* the residual that decides convergence is the unpreconditioned one,
  r = v - A u (Sec. 3 defines r = y - A x), 2-norm over masked pixels,
  relative to ||v||, recomputed from scratch at the end;
* initial guess u = 0;
* the white noise is drawn with Philox4x64-10 (Salmon et al., SC'11),
  key = (seed, stream), counter = (j, 0, 0, 0) for the pixels 4j .. 4j+3
  (j = i // 4 of row-major pixel index i); each block of four words gives
  four normals by Box-Muller, both outputs of each word pair: words (0, 1)
  give pixels 4j, 4j+1 and words (2, 3) pixels 4j+2, 4j+3 as r cos t and
  r sin t, u = ((w >> 11) + 0.5) * 2^-53, r = sqrt(-2 ln u_a), t = 2 pi u_b.
"""

from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

__all__ = [
    "PHILOX_M0", "PHILOX_M1", "PHILOX_W0", "PHILOX_W1", "REALIZATION_STREAM",
    "philox4x64_10", "white_noise", "circulant_apply", "unconstrained_realization",
    "rhs", "apply_A", "apply_A_skew", "apply_E", "cg_residual_history", "pcg_split", "pcg_cxx",
    "fill_realize", "fill_mean", "FillResult",
]

# FFT threads: ORACLE_WORKERS if set, else every core this process may run on.
_WORKERS = int(os.environ.get("ORACLE_WORKERS", "0")) or len(os.sched_getaffinity(0)) or 1

# Philox4x64 round multipliers and Weyl key increments (Salmon et al. 2011).
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
REALIZATION_STREAM = 0x52

_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a: np.ndarray, b: np.uint64) -> tuple[np.ndarray, np.ndarray]:
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b  # wraps modulo 2^64
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Philox4x64 with 10 rounds: counter (c0..c3), key (k0, k1) -> 4 words.

    One round maps (c0, c1, c2, c3) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)),
    and the key is advanced by the Weyl constants between rounds.
    """
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64).copy() for v in (c0, c1, c2, c3))
        k0 = np.asarray(k0, dtype=np.uint64).copy()
        k1 = np.asarray(k1, dtype=np.uint64).copy()
        for rnd in range(10):
            hi0, lo0 = _mulhilo64(c0, PHILOX_M0)
            hi1, lo1 = _mulhilo64(c2, PHILOX_M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            if rnd < 9:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
    return c0, c1, c2, c3


def _unit_open(w: np.ndarray) -> np.ndarray:
    """Top 53 bits of a 64-bit word, mapped to the open interval (0, 1)."""
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def white_noise(nx: int, ny: int, seed: int, stream: int = REALIZATION_STREAM) -> np.ndarray:
    """w ~ N(0, I) on the (ny, nx) grid, from the counter-based generator
    above: block j (counter (j, 0, 0, 0)) gives pixels 4j .. 4j+3, two by
    Box-Muller from each pair of its words (radius from the first, angle from
    the second: the cosine and the sine)."""
    n = nx * ny
    assert n % 4 == 0
    j = np.arange(n // 4, dtype=np.uint64)
    z = np.zeros_like(j)
    w0, w1, w2, w3 = philox4x64_10(j, z, z, z, np.uint64(seed), np.uint64(stream))
    out = np.empty(n, dtype=np.float64)
    for k, (wa, wb) in enumerate(((w0, w1), (w2, w3))):
        r = np.sqrt(-2.0 * np.log(_unit_open(wa)))
        th = 2.0 * np.pi * _unit_open(wb)
        out[2 * k::4] = r * np.cos(th)
        out[2 * k + 1::4] = r * np.sin(th)
    return out.reshape(ny, nx)


def _workers(n: int) -> int:
    return _WORKERS if n >= 1 << 16 else 1


def circulant_apply(v: np.ndarray, P: np.ndarray, power: float) -> np.ndarray:
    """C^power v on the torus: C is diagonal, with eigenvalues P(k), in Fourier space."""
    ny, nx = v.shape
    wk = _workers(v.size)
    vk = sfft.rfft2(v, workers=wk)
    return sfft.irfft2(vk * P ** power, s=(ny, nx), workers=wk)


def unconstrained_realization(P: np.ndarray, seed: int, stream: int = REALIZATION_STREAM) -> np.ndarray:
    """s = C^{1/2} w, an isotropic draw with covariance C (Sec. 2.3)."""
    ny = P.shape[0]
    nx = 2 * (P.shape[1] - 1)
    return circulant_apply(white_noise(nx, ny, seed, stream), P, 0.5)


def _Px(v: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Projection onto the masked (unobserved) pixels."""
    return np.where(mask != 0, v, 0.0)


def _Py(v: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Projection onto the observed pixels."""
    return np.where(mask != 0, 0.0, v)


def apply_A(v: np.ndarray, mask: np.ndarray, P: np.ndarray) -> np.ndarray:
    """A v = Px C^-1 Px v, the operator of eq. ModEq."""
    return _Px(circulant_apply(_Px(v, mask), P, -1.0), mask)


def apply_A_skew(v: np.ndarray, mask: np.ndarray, P: np.ndarray, eps: float) -> np.ndarray:
    """A deliberately non-Hermitian variant of A for the Hermiticity study of Sec. 3.

    Each spectral mode of C^-1 Px v is multiplied by 1 + i eps sin(2 pi kx / nx):
    A_eps = Px C^-1 (I + eps K) Px with K the circulant of eigenvalues
    i sin(2 pi kx / nx), a real antisymmetric operator (the central
    difference along x).  eps = 0 gives A.
    """
    ny, nx = v.shape
    kx = np.arange(nx // 2 + 1)
    f = 1.0 + 1j * eps * np.sin(2.0 * np.pi * kx / nx)
    w = sfft.irfft2(sfft.rfft2(_Px(v, mask), workers=_workers(v.size)) / P * f[None, :], s=v.shape,
                    workers=_workers(v.size))
    return _Px(w, mask)


def cg_residual_history(op, b: np.ndarray, iters: int) -> np.ndarray:
    """Plain Hestenes-Stiefel CG (x0 = 0) on op x = b for a fixed number of
    steps: the recursive residual norms ||r_0||, ..., ||r_iters|| (the
    quantity whose per-step ratio Sec. 3 tracks on non-Hermitian operators)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.vdot(r, r))
    hist = [np.sqrt(rr)]
    for _ in range(iters):
        q = op(p)
        pq = float(np.vdot(p, q))
        if pq == 0.0 or rr == 0.0:
            break
        alpha = rr / pq
        x += alpha * p
        r -= alpha * q
        rr_new = float(np.vdot(r, r))
        hist.append(np.sqrt(rr_new))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return np.asarray(hist)


def apply_E(v: np.ndarray, mask: np.ndarray, P: np.ndarray) -> np.ndarray:
    """E v = Px C^{1/2} Px v, the split preconditioner of Sec. 2.4."""
    return _Px(circulant_apply(_Px(v, mask), P, 0.5), mask)


def rhs(y_minus_sy: np.ndarray, mask: np.ndarray, P: np.ndarray) -> np.ndarray:
    """v = -Px C^-1 Py t: the right-hand side whose solution is M t (Sec. 2.1)."""
    return -_Px(circulant_apply(_Py(y_minus_sy, mask), P, -1.0), mask)


@dataclass
class PCGInfo:
    iterations: int
    rel_residual: float
    converged: bool
    history: list
    # CG step lengths alpha_j and direction coefficients beta_j of the first
    # CG run (x0 = 0, before any restart): the Lanczos data of Sec. 6.4.
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)


def pcg_split(v: np.ndarray, mask: np.ndarray, P: np.ndarray, rtol: float,
              max_iter: int = 20000, history: bool = False,
              precond: bool = True) -> tuple[np.ndarray, PCGInfo]:
    """Solve A u = v with CG on the split system (E A E) u' = E v, u = E u' (Sec. 2.4).

    Plain Hestenes-Stiefel CG on the symmetric positive definite operator
    E A E restricted to the masked pixels.  Alongside u' the routine carries
    u = E u' and the unpreconditioned residual v - A u (both are linear in the
    CG updates), stops when that residual is below rtol * ||v||, and then
    recomputes it from scratch; if the recomputed residual is still too large
    it restarts CG from the current u.

    precond=False replaces E by the plain projection Px: CG on A itself, as
    Sec. 3 does for point-source masks.  The step lengths and direction
    coefficients of the first CG run are kept in the returned info.
    """
    E = apply_E if precond else (lambda a, m, _P: _Px(a, m))
    vnorm = float(np.linalg.norm(v))
    u = np.zeros_like(v)
    hist = []
    alphas, betas = [], []
    total = 0
    if vnorm == 0.0:
        return u, PCGInfo(0, 0.0, True, hist)
    res = v.copy()
    for restart in range(20):
        # CG on E A E d' = E res, accumulating d = E d' into u.
        r = E(res, mask, P)
        p = r.copy()
        rr = float(np.vdot(r, r))
        done = False
        while total < max_iter:
            Ep = E(p, mask, P)
            AEp = apply_A(Ep, mask, P)
            q = E(AEp, mask, P)
            alpha = rr / float(np.vdot(p, q))
            if restart == 0:
                alphas.append(alpha)
            u += alpha * Ep
            res -= alpha * AEp
            r -= alpha * q
            total += 1
            rel = float(np.linalg.norm(res)) / vnorm
            if history:
                hist.append(rel)
            if rel <= rtol:
                done = True
                break
            rr_new = float(np.vdot(r, r))
            if rr_new == 0.0:  # the split system is solved exactly: check the true residual
                done = True
                break
            if restart == 0:
                betas.append(rr_new / rr)
            p = r + (rr_new / rr) * p
            rr = rr_new
        res = v - apply_A(u, mask, P)
        rel = float(np.linalg.norm(res)) / vnorm
        if rel <= rtol or not done:
            return u, PCGInfo(total, rel, rel <= rtol, hist, alphas, betas)
    return u, PCGInfo(total, rel, rel <= rtol, hist, alphas, betas)


def pcg_cxx(v: np.ndarray, mask: np.ndarray, P: np.ndarray, rtol: float,
            max_iter: int = 20000) -> tuple[np.ndarray, PCGInfo]:
    """Solve A u = v by preconditioned CG with M^-1 = Px C Px.

    The preconditioner is the covariance restricted to the masked pixels,
    C_xx, an approximate inverse of A = (C^-1)_xx in the spirit of Sec. 2.4
    (the powers of C cancel) with one operator apply instead of the two of
    the split form.  Hestenes-Stiefel PCG from u = 0 on the unpreconditioned
    residual; stop when ||v - A u|| <= rtol ||v|| (recursive residual, then
    recomputed, restarting if the recomputed one is too large).  The step
    lengths and direction coefficients of the first CG run are kept.
    """
    def Minv(a):
        return _Px(circulant_apply(_Px(a, mask), P, 1.0), mask)

    vnorm = float(np.linalg.norm(v))
    u = np.zeros_like(v)
    hist, alphas, betas = [], [], []
    total = 0
    if vnorm == 0.0:
        return u, PCGInfo(0, 0.0, True, hist)
    r = v.copy()
    rel = 1.0
    for restart in range(20):
        z = Minv(r)
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
            z = Minv(r)
            rz_new = float(np.vdot(r, z))
            if rz_new == 0.0:
                done = True
                break
            if restart == 0:
                betas.append(rz_new / rz)
            p = z + (rz_new / rz) * p
            rz = rz_new
        r = v - apply_A(u, mask, P)
        rel = float(np.linalg.norm(r)) / vnorm
        if rel <= rtol or not done:
            return u, PCGInfo(total, rel, rel <= rtol, hist, alphas, betas)
    return u, PCGInfo(total, rel, rel <= rtol, hist, alphas, betas)


@dataclass
class FillResult:
    x_out: np.ndarray   # filled map: observed pixels = d_obs, masked = s + u
    s: np.ndarray       # unconstrained realization
    u: np.ndarray       # M (y - s_y), zero outside the mask
    info: PCGInfo


def _solve(v: np.ndarray, mask: np.ndarray, P: np.ndarray, rtol: float, max_iter: int, solver: str):
    """A u = v to true relative residual rtol.  solver "split" is the paper's
    split-preconditioned CG (Sec. 2.4); "cxx" is PCG with M^-1 = Px C Px (one
    apply fewer per iteration); "block" is PCG with the block
    preconditioner of oracle.block_precond, which converges in far fewer
    iterations on wide cuts.  Both stop on the same true residual
    ||v - A u|| <= rtol ||v|| of this module's A, so the solution they return
    does not depend on the preconditioner (it only sets the CG path)."""
    if solver == "split":
        return pcg_split(v, mask, P, rtol, max_iter)
    if solver == "cxx":
        return pcg_cxx(v, mask, P, rtol, max_iter)
    if solver == "block":
        from .block_precond import pcg_block
        return pcg_block(v, mask, P, rtol, max_iter)
    raise ValueError(f"unknown solver {solver!r}")


def fill_realize(d_obs: np.ndarray, mask: np.ndarray, P: np.ndarray, seed: int,
                 rtol: float, max_iter: int = 20000, solver: str = "split") -> FillResult:
    """Constrained realization by the Hoffman-Ribak construction (Sec. 2.3).

    s = C^{1/2} w; t = Py (d_obs - s); v = -Px C^-1 t; solve A u = v;
    x_out = d_obs on observed pixels and s + u on masked pixels.
    """
    s = unconstrained_realization(P, seed)
    t = _Py(d_obs - s, mask)
    v = rhs(t, mask, P)
    u, info = _solve(v, mask, P, rtol, max_iter, solver)
    x = np.where(mask != 0, s + u, d_obs)
    return FillResult(x, s, u, info)


def fill_mean(d_obs: np.ndarray, mask: np.ndarray, P: np.ndarray, rtol: float,
              max_iter: int = 20000, solver: str = "split") -> FillResult:
    """The conditional mean (Wiener fill) x_ML = M y on masked pixels (Sec. 2.1)."""
    t = _Py(d_obs, mask)
    v = rhs(t, mask, P)
    u, info = _solve(v, mask, P, rtol, max_iter, solver)
    x = np.where(mask != 0, u, d_obs)
    return FillResult(x, np.zeros_like(d_obs), u, info)
