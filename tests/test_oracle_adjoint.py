"""Pins of the oracle's adjoint gradient (CPU only).

The adjoint recipe is checked against the dense conditional Gaussian
differentiated by torch autograd (an independent formula: Cholesky of C_yy,
no CG, no adjoint algebra) and against central finite differences of the
oracle's own forward fill.  Mutations of the recipe must fail the dense pin.
"""

from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as AD
import oracle.fill_oracle as F

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def setup(n=48, nb=50, seed_mask=7):
    lnk = AD.band_nodes(n, nb)
    phi = AD.band_weights(n, n, lnk)
    kb = np.exp(lnk)
    theta = np.log(1.0 / (kb ** 2 + 4) * np.exp(-(kb / (n / 8)) ** 2) + 1e-7)
    mask = W.band_holes_mask(n, n, W.band_rows(n, 0.1), 4, 2, 5, seed_mask)
    P = AD.pk_from_bands(theta, phi)
    d = W.observed_map(P, n, n, 3, mask)
    wts = np.random.default_rng(5).uniform(0, 1, (n, n))
    return d, mask, theta, phi, wts


def test_band_weights_partition_of_unity_and_linear_interpolation():
    n = 64
    lnk = AD.band_nodes(n, 20)
    phi = AD.band_weights(n, n, lnk)
    assert np.allclose(phi.sum(0), 1.0, atol=1e-14)
    assert phi.min() >= 0.0
    # theta linear in ln k is reproduced exactly inside [k_1, k_B]
    theta = 0.3 - 1.7 * lnk
    lnP = np.log(AD.pk_from_bands(theta, phi))
    k = W.kgrid(n, n)
    inside = (k >= 1.0) & (np.log(np.maximum(k, 1e-300)) <= lnk[-1])
    assert np.allclose(lnP[inside], (0.3 - 1.7 * np.log(k))[inside], atol=1e-12)
    # clamped outside: k = 0 takes theta_1
    assert np.isclose(lnP[0, 0], theta[0])


def test_adjoint_matches_dense_autograd():
    d, mask, theta, phi, wts = setup()
    L, gy, gP, gth = AD.adjoint_gradient(d, mask, theta, phi, 9, wts)
    L2, gy2, gth2 = AD.dense_torch_loss_and_grad(d, mask, theta, phi, 9, wts)
    assert abs(L - L2) < 1e-10 * abs(L2)
    assert np.linalg.norm(gy - gy2) < 1e-8 * np.linalg.norm(gy2)
    assert np.linalg.norm(gth - gth2) < 1e-8 * np.linalg.norm(gth2)


def test_adjoint_matches_central_differences():
    d, mask, theta, phi, wts = setup()
    _, gy, _, gth = AD.adjoint_gradient(d, mask, theta, phi, 9, wts)
    h = 1e-4
    scale = np.abs(gth).max()
    for b in (0, 17, 33, 49):
        e = np.zeros_like(theta)
        e[b] = h
        fd = (AD.fill_loss(d, mask, theta + e, phi, 9, wts) - AD.fill_loss(d, mask, theta - e, phi, 9, wts)) / (2 * h)
        assert abs(fd - gth[b]) < 1e-6 * scale, b
    rng = np.random.default_rng(1)
    for _ in range(3):
        dirn = np.where(mask != 0, 0.0, rng.standard_normal(d.shape))
        P = AD.pk_from_bands(theta, phi)
        def Lof(dd):
            x = F.fill_realize(dd, mask, P, 9, 1e-13).x_out
            return float(np.sum(wts * x * x))
        fd = (Lof(d + h * dirn) - Lof(d - h * dirn)) / (2 * h)
        an = float(np.sum(gy * dirn))
        assert abs(fd - an) < 1e-6 * abs(an)


def test_adjoint_solve_is_symmetric():
    d, mask, theta, phi, _ = setup()
    P = AD.pk_from_bands(theta, phi)
    rng = np.random.default_rng(2)
    a, b = (np.where(mask != 0, rng.standard_normal(d.shape), 0.0) for _ in range(2))
    xa, _ = F.pcg_split(a, mask, P, 1e-13)
    xb, _ = F.pcg_split(b, mask, P, 1e-13)
    assert abs(np.vdot(xa, b) - np.vdot(a, xb)) < 1e-9 * abs(np.vdot(xa, b))


def test_mutation_dropped_half_factor_is_caught(monkeypatch):
    d, mask, theta, phi, wts = setup()
    orig = AD.half_spectrum_weights
    monkeypatch.setattr(AD, "half_spectrum_weights", lambda nx, ny: np.ones_like(orig(nx, ny)))
    _, _, _, gth = AD.adjoint_gradient(d, mask, theta, phi, 9, wts)
    _, _, gth2 = AD.dense_torch_loss_and_grad(d, mask, theta, phi, 9, wts)
    assert np.linalg.norm(gth - gth2) > 1e-3 * np.linalg.norm(gth2)
