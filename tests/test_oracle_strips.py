"""Pins of the oracle's strip subdivision and noise-boosted strip refinement
(Sec. 6.2, 6.4), CPU only."""

from __future__ import annotations

import numpy as np
import pytest

import oracle.dense as D
import oracle.fill_oracle as F
import oracle.strips as S
import workloads as W


def _brute_counts(mask, w):
    obs = (mask == 0).astype(np.int64)
    out = np.zeros_like(obs)
    r = int(np.floor(w))
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dy * dy + dx * dx <= w * w:
                out += np.roll(np.roll(obs, -dy, axis=0), -dx, axis=1)
    return out


@pytest.mark.parametrize("w", [1.0, 2.5, 4.0, 6.3])
def test_observed_counts_brute_force(w):
    mask = W.band_holes_mask(40, 24, (8, 6), 4, 1.0, 4.0, 5)
    assert np.array_equal(S.observed_counts(mask, w), _brute_counts(mask, w))


def test_disk_must_fit_the_torus():
    with pytest.raises(ValueError):
        S.observed_counts(np.zeros((16, 32), np.uint8), 8.0)
    S.observed_counts(np.zeros((16, 32), np.uint8), 7.9)


def test_strip_nesting_and_adjacency():
    mask = W.band_holes_mask(64, 64, (20, 24), 6, 2.0, 6.0, 8)
    prev = None
    for w in (20, 10, 5, 2, 1):
        Dw = S.strip_mask(mask, w)
        assert np.all(Dw <= mask)
        if prev is not None:
            assert np.all(Dw <= prev)  # D_1 > D_2 > ...
        prev = Dw
    # every masked pixel with an observed 4-neighbour is in the width-1 strip
    obs = mask == 0
    near = (np.roll(obs, 1, 0) | np.roll(obs, -1, 0) | np.roll(obs, 1, 1) | np.roll(obs, -1, 1)) & (mask != 0)
    assert np.all(S.strip_mask(mask, 1.0)[near] == 1)


def test_band_strip_rows_closed_form():
    # a straight band: the pixel d rows inside the edge sees the disk offsets
    # with dy >= d (band higher than the disk), so the strip holds the rows
    # with #{dy >= d} > 0.03 * area, counted directly from the offsets
    n, r0, h, w = 64, 16, 32, 9.0
    mask = np.zeros((n, n), np.uint8)
    mask[r0:r0 + h] = 1
    off = S.disk_offsets(w)
    area = len(off)
    dmax = max(d for d in range(1, int(w) + 1) if np.count_nonzero(off[:, 0] >= d) > 0.03 * area)
    Dw = S.strip_mask(mask, w)
    rows = np.nonzero(Dw.any(axis=1))[0]
    expect = sorted(set(range(r0, r0 + dmax)) | set(range(r0 + h - dmax, r0 + h)))
    assert list(rows) == expect
    assert np.all(Dw[rows] == 1)


def test_one_strip_step_is_the_conditional_mean():
    # one step with enough iterations: the ML fill of D with spectrum P_s + beta N
    # given every other pixel of the current map (dense Cholesky at 32^2)
    n = 32
    P = W.damped_power_law(n, n, 1.0, 4.0, 1e-3)
    floor = 1e-3
    mask = W.band_holes_mask(n, n, (12, 8), 2, 2.0, 3.0, 4)
    d = W.observed_map(P, n, n, 3, mask)
    start = np.random.default_rng(2).standard_normal((n, n))
    beta, w = 40.0, 2.5
    x, strips = S.strip_fill(d, mask, P - floor, floor, [beta], [w], iters=400, start=start)
    Dm = strips[0]
    cur = np.where(mask != 0, start, d)
    ref = D.conditional_mean_dense(np.where(Dm != 0, 0.0, cur), Dm, P - floor + beta * floor)
    m = Dm != 0
    assert np.linalg.norm(x[m] - ref[m]) <= 1e-8 * np.linalg.norm(ref[m])
    # pixels outside the strip keep the current map
    assert np.array_equal(x[~m], cur[~m])


def test_whole_mask_strip_with_beta_one_is_the_exact_fill():
    p = W.make_problem("grid64")
    floor = 1e-6
    x, strips = S.strip_fill(p.d_obs, p.mask, p.P - floor, floor, [1.0], [31.0], iters=600)
    assert np.array_equal(strips[0], p.mask)
    ref = F.fill_mean(p.d_obs, p.mask, p.P, 1e-12)
    m = p.mask != 0
    assert np.linalg.norm(x[m] - ref.x_out[m]) <= 1e-7 * np.linalg.norm(ref.x_out[m])
