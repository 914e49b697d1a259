"""Pins of the oracle's kernel-based Laplace solver (Sec. 6.1, 6.3), CPU only."""

from __future__ import annotations

import numpy as np
import pytest

import oracle.laplace as L
import workloads as W


def _hole_case(n=128, h=40):
    mask = np.zeros((n, n), np.uint8)
    a = (n - h) // 2
    mask[a:a + h, a + 5:a + h - 3] = 1
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    y -= n / 2
    x -= n / 2
    f = 0.7 + 0.01 * x - 0.02 * y + 1e-3 * (x * x - y * y) + 2e-3 * x * y  # harmonic
    return mask, f


def test_harmonic_data_is_the_fixed_point():
    # symmetric annulus averages reproduce harmonic polynomials exactly, so
    # the relaxation converges to the harmonic extension of the data
    mask, f = _hole_case()
    radii = L.laplace_radii(5)
    x, hist = L.laplace_fill(np.where(mask != 0, 0.0, f), mask, radii, 600)
    m = mask != 0
    assert np.abs(x[m] - f[m]).max() <= 1e-8 * np.abs(f[m]).max()
    assert hist[-1] < 1e-6 * hist[0]


def test_kernel_classes_brute_force():
    mask = W.band_holes_mask(64, 48, (14, 18), 5, 2.0, 5.0, 7)
    radii = L.laplace_radii(4, 1.5, 2.0)
    cls = L.kernel_classes(mask, radii)
    ny, nx = mask.shape
    obs = np.argwhere(mask == 0)
    for (y, x) in np.argwhere(mask != 0)[::7]:
        dy = np.abs(obs[:, 0] - y)
        dx = np.abs(obs[:, 1] - x)
        d2 = (np.minimum(dy, ny - dy) ** 2 + np.minimum(dx, nx - dx) ** 2).min()
        j = max([0] + [k for k in range(1, len(radii)) if d2 > radii[k] ** 2])
        assert cls[y, x] == j
    assert np.all(cls[mask == 0] == -1)


def test_one_sweep_brute_force():
    mask = W.band_holes_mask(48, 40, (10, 14), 4, 2.0, 4.0, 3)
    d = np.random.default_rng(4).standard_normal(mask.shape)
    start = np.random.default_rng(5).standard_normal(mask.shape)
    radii = L.laplace_radii(3, 1.5, 2.0)
    x, _ = L.laplace_fill(d, mask, radii, 1, start=start)
    cur = np.where(mask != 0, start, d)
    cls = L.kernel_classes(mask, radii)
    ref = cur.copy()
    for j in range(len(radii)):
        off = L.annulus_offsets(0.0 if j == 0 else radii[j - 1], radii[j])
        acc = np.zeros_like(cur)
        for dy, dx in off:
            acc += np.roll(np.roll(cur, -dy, axis=0), -dx, axis=1)
        sel = cls == j
        ref[sel] = acc[sel] / len(off)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


def test_mutation_unnormalised_kernel_is_caught(monkeypatch):
    mask, f = _hole_case()
    orig = L._kernel_spectrum

    def wrong(j, radii, shape):
        return orig(j, radii, shape) * (1.0 + 1e-3)   # averages no longer sum to one

    monkeypatch.setattr(L, "_kernel_spectrum", wrong)
    x, _ = L.laplace_fill(np.where(mask != 0, 0.0, f), mask, L.laplace_radii(5), 600)
    m = mask != 0
    assert np.abs(x[m] - f[m]).max() > 1e-4 * np.abs(f[m]).max()
