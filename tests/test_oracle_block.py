"""Pins of the oracle's block preconditioner (oracle.block_precond).

* With a band shorter than the bandwidth the definition is an exact sum of
  inverses: M^-1 equals sum_parts R^T (A restricted to the part)^-1 R, built
  here from a dense covariance block (numpy irfft2 + index arithmetic) and
  parts found by brute-force flood fill and dilation;
* on a band taller than the bandwidth, each x-frequency goes through the
  truncated Toeplitz matrix formed from the dense covariance, shifted by the
  Gershgorin bound of the discarded part unless the truncation is safely
  positive definite (decided here from eigenvalues); with a slowly decaying
  kernel some frequencies' plain truncation is indefinite and gets the shift,
  the others keep the plain truncation;
* exactness: band-only and single-hole masks give M^-1 A = I;
* M^-1 is symmetric positive definite;
* structure: periodic components, tiling above CMAX, band-run rules;
* PCG with it reaches the dense solution, in far fewer iterations than
  M^-1 = Px C Px.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle.block_precond as B
import oracle.fill_oracle as OF
import workloads as W
from pins import masked_circulant_block, rel


def spectrum(nx, ny, damping=6.0):
    return W.damped_power_law(nx, ny, 2.0, damping, 1e-6)


def disk(mask, cy, cx, r):
    ny, nx = mask.shape
    y, x = np.mgrid[:ny, :nx]
    dy = (y - cy + ny // 2) % ny - ny // 2
    dx = (x - cx + nx // 2) % nx - nx // 2
    mask[dy * dy + dx * dx <= r * r] = 1


def dense_A(P, sel):
    """A = C^-1 restricted to the flat pixel set sel (sorted), dense."""
    ny = P.shape[0]
    nx = 2 * (P.shape[1] - 1)
    m = np.zeros(ny * nx, np.uint8)
    m[sel] = 1
    return masked_circulant_block(P, m.reshape(ny, nx), -1.0)


def flood_parts(mask, band_rows):
    """Components of masked pixels outside band_rows (4-neighbours, periodic),
    by breadth-first search, as sorted flat index arrays."""
    ny, nx = mask.shape
    free = (mask != 0).copy()
    free[list(band_rows)] = False
    seen = np.zeros_like(free)
    parts = []
    for y in range(ny):
        for x in range(nx):
            if free[y, x] and not seen[y, x]:
                stack, comp = [(y, x)], []
                seen[y, x] = True
                while stack:
                    a, b = stack.pop()
                    comp.append(a * nx + b)
                    for c, d in ((a + 1, b), (a - 1, b), (a, b + 1), (a, b - 1)):
                        c, d = c % ny, d % nx
                        if free[c, d] and not seen[c, d]:
                            seen[c, d] = True
                            stack.append((c, d))
                parts.append(np.sort(np.array(comp)))
    return parts


def grow(mask, part, halo):
    ny, nx = mask.shape
    out = set()
    for p in part:
        y, x = divmod(int(p), nx)
        for dy in range(-halo, halo + 1):
            for dx in range(-halo, halo + 1):
                q = ((y + dy) % ny) * nx + (x + dx) % nx
                if mask.reshape(-1)[q]:
                    out.add(q)
    return np.array(sorted(out))


def dense_M_oracle(M, mask):
    idx = np.flatnonzero(mask.reshape(-1) != 0)
    cols = []
    for j in idx:
        e = np.zeros(mask.size)
        e[j] = 1.0
        cols.append(M.apply(e.reshape(mask.shape)).reshape(-1)[idx])
    return np.array(cols).T, idx


def test_short_band_and_holes_equal_sum_of_inverses():
    ny, nx = 96, 32
    P = spectrum(nx, ny)
    mask = np.zeros((ny, nx), np.uint8)
    mask[40:52] = 1                    # a 12-row band (< BW: no truncation)
    disk(mask, 55, 10, 3)              # touches the band: its halo reaches in
    disk(mask, 10, 0, 2)               # straddles the x edge
    disk(mask, 80, 20, 2)
    M = B.BlockPrecond(mask, P)
    assert M.runs == [(40, 12)]
    Md, idx = dense_M_oracle(M, mask)
    pos = {int(p): i for i, p in enumerate(idx)}
    ref = np.zeros_like(Md)
    band = np.arange(40 * nx, 52 * nx)
    parts = [band]
    for part in flood_parts(mask, range(40, 52)):
        parts.append(grow(mask, part, B.HALO))
    assert len(parts) == 4
    for part in parts:
        Ai = np.linalg.inv(dense_A(P, part))
        ii = np.array([pos[int(p)] for p in part])
        ref[np.ix_(ii, ii)] += Ai
    assert np.abs(Md - ref).max() <= 1e-9 * np.abs(ref).max()


def expected_shift(T, t):
    """The diagonal shift the definition adds to the truncated matrix T of the
    symbols t, decided from eigenvalues: Cholesky pivots are at least the
    smallest eigenvalue, so lambda_min > PIVOT_MIN t(0) means no shift and
    lambda_min < 0 means the Gershgorin bound of the discarded part; a case
    in between is not decidable this way and fails."""
    lam = np.linalg.eigvalsh(T).min()
    if lam > B.PIVOT_MIN * t[0]:
        return 0.0
    assert lam < 0.0, "borderline case"
    return 2.0 * np.abs(t[B.BW:]).sum()


def test_tall_band_uses_truncated_toeplitz_per_frequency():
    ny, nx, h, y0 = 160, 32, 40, 60    # 40 rows > BW = 32
    P = spectrum(nx, ny)
    mask = np.zeros((ny, nx), np.uint8)
    mask[y0:y0 + h] = 1
    M = B.BlockPrecond(mask, P)
    assert M.runs == [(y0, h)] and M.blocks == []
    Ab = dense_A(P, np.arange(y0 * nx, (y0 + h) * nx))   # rows (i, x) row-major
    rng = np.random.default_rng(1)
    for kx in (0, 3, nx // 2):
        # t(d) from the dense block: sum over x of A[(0, 0), (d, x)] cos(2 pi kx x / nx)
        t = np.array([sum(Ab[0, d * nx + x] * np.cos(2 * np.pi * kx * x / nx) for x in range(nx))
                      for d in range(h)])
        d = np.abs(np.arange(h)[:, None] - np.arange(h)[None, :])
        T = np.where(d < B.BW, t[d], 0.0)
        T += expected_shift(T, t) * np.eye(h)
        a = rng.standard_normal(h)
        u = np.zeros((ny, nx))
        u[y0:y0 + h] = a[:, None] * np.cos(2 * np.pi * kx * np.arange(nx) / nx)[None, :]
        z = M.apply(u)
        b = np.linalg.solve(T, a)
        expect = b[:, None] * np.cos(2 * np.pi * kx * np.arange(nx) / nx)[None, :]
        assert rel(z[y0:y0 + h], expect) < 1e-10


def test_slow_decay_truncation_needs_the_shift():
    ny, nx, h, y0 = 256, 128, 51, 90   # sharp spectral knee: t_kx(d) decays slowly in d
    P = W.damped_power_law(nx, ny, 2.0, 12.0, 1e-6)
    mask = np.zeros((ny, nx), np.uint8)
    mask[y0:y0 + h] = 1
    t = B.band_symbols(B.kernel_cinv(P), h)
    d = np.abs(np.arange(h)[:, None] - np.arange(h)[None, :])
    plain_min = min(np.linalg.eigvalsh(np.where(d < B.BW, t[d, kx], 0.0)).min() for kx in range(nx // 2 + 1))
    assert plain_min < 0.0
    M = B.BlockPrecond(mask, P)
    assert min(np.linalg.eigvalsh(T).min() for T in M.band_T[0]) > 0.0
    # frequencies whose truncation is safely positive definite keep it unshifted
    kept = 0
    for kx in range(nx // 2 + 1):
        T0 = np.where(d < B.BW, t[d, kx], 0.0)
        sh = expected_shift(T0, t[:, kx])
        assert np.abs(M.band_T[0][kx] - (T0 + sh * np.eye(h))).max() <= 1e-12 * abs(t[0, kx])
        kept += sh == 0.0
    assert 0 < kept < nx // 2 + 1
    # the shifted factor still approximates the band well: M^-1 A close to I
    rng = np.random.default_rng(4)
    v = np.where(mask != 0, rng.standard_normal((ny, nx)), 0.0)
    assert rel(M.apply(OF.apply_A(v, mask, P)), v, mask != 0) < 0.5


def test_band_only_and_single_hole_are_exact():
    ny, nx = 128, 64
    P = spectrum(nx, ny, 10.0)
    rng = np.random.default_rng(2)
    for kind in ("band", "hole"):
        mask = np.zeros((ny, nx), np.uint8)
        if kind == "band":
            mask[50:60] = 1
        else:
            disk(mask, 70, 30, 6)
        M = B.BlockPrecond(mask, P)
        v = np.where(mask != 0, rng.standard_normal((ny, nx)), 0.0)
        back = M.apply(OF.apply_A(v, mask, P))
        assert rel(back, v, mask != 0) < 1e-8, kind


def test_symmetric_positive_definite():
    p = W.make_problem("grid64")
    M = B.BlockPrecond(p.mask, p.P)
    Md, _ = dense_M_oracle(M, p.mask)
    assert np.abs(Md - Md.T).max() <= 1e-10 * np.abs(Md).max()
    assert np.linalg.eigvalsh(0.5 * (Md + Md.T)).min() > 0.0


def test_structure_rules():
    ny, nx = 64, 64
    # a hole across the corner is one periodic component
    mask = np.zeros((ny, nx), np.uint8)
    disk(mask, 0, 0, 3)
    cells = B.cells(mask, [])
    assert len(cells) == 1 and len(cells[0]) == int(mask.sum())
    # a component above CMAX is cut along the absolute TILE grid
    mask = np.zeros((ny, nx), np.uint8)
    mask[8:48, 4:44] = 1               # 1600 pixels
    cells = B.cells(mask, [])
    assert sum(len(c) for c in cells) == 1600 and len(cells) == 9
    for c in cells:
        assert len({(y // B.TILE, x // B.TILE) for y, x in c}) == 1
    # runs: fully masked rows only; a run taller than ny - 2 BW is not a band
    mask = np.zeros((160, 32), np.uint8)
    mask[10:20] = 1
    mask[30:130] = 1
    mask[140, :31] = 1
    assert B.band_runs(mask) == [(10, 10)]
    # halo: a cell grows into the band by HALO rows
    mask = np.zeros((160, 32), np.uint8)
    mask[50:60] = 1
    mask[60:63, 5:8] = 1               # a 3x3 square under the band
    runs = B.band_runs(mask)
    cells = B.cells(mask, runs)
    blk = B.blocks(mask, cells)[0]
    ys = blk // 32
    assert ys.min() == 60 - B.HALO and ys.max() == 62


def test_halo_rule_counts_by_hand():
    """Step 6 of the definition on masks whose block sizes follow by hand."""
    # isolated holes: their pieces do not grow (the halo only takes masked
    # pixels), so every halo costs the same and the widest is chosen
    mask = np.zeros((64, 64), np.uint8)
    mask[10:13, 10:13] = 1
    mask[40:42, 30:35] = 1
    assert B.block_entries(B.blocks(mask, B.cells(mask, []), 14)) == 9 * 12 + 10 * 12
    assert B.auto_halo(mask) == 14
    # a 3 x 3 hole right under a 20-row band: its block takes the band
    # pixels within Chebyshev distance h, (3 + 2h) columns by h rows
    mask = np.zeros((128, 64), np.uint8)
    mask[40:60] = 1
    mask[60:63, 20:23] = 1
    runs = B.band_runs(mask)
    assert runs == [(40, 20)]
    for h in (8, 10, 12, 14):
        (blk,) = B.blocks(mask, B.cells(mask, runs, h), h)
        n = 9 + (3 + 2 * h) * h
        assert len(blk) == n
    entries = {h: n * (-(-n // 4) * 4) for h, n in ((h, 9 + (3 + 2 * h) * h) for h in (8, 10, 12, 14))}
    # 128 * 64 / 2 = 4096 entries of slack: h = 10 adds 239*240 - 161*164 = 30956
    assert all(entries[h] - entries[8] > 4096 for h in (10, 12, 14))
    assert B.auto_halo(mask) == 8
    # with a wider grid the same growth fits the slack: 1024 x 256 / 2 = 131072
    big = np.zeros((1024, 256), np.uint8)
    big[40:60] = 1
    big[60:63, 20:23] = 1
    assert entries[12] - entries[8] <= 131072 < entries[14] - entries[8]
    assert B.auto_halo(big) == 12


def test_pcg_block_reaches_dense_solution():
    p = W.make_problem("grid64")
    s = OF.unconstrained_realization(p.P, p.seed)
    v = OF.rhs(np.where(p.mask != 0, 0.0, p.d_obs - s), p.mask, p.P)
    u, info = B.pcg_block(v, p.mask, p.P, 1e-12)
    A = masked_circulant_block(p.P, p.mask, -1.0)
    idx = np.flatnonzero(p.mask.reshape(-1) != 0)
    ud = np.linalg.solve(A, v.reshape(-1)[idx])
    assert info.converged
    assert np.linalg.norm(u.reshape(-1)[idx] - ud) <= 1e-9 * np.linalg.norm(ud)


def test_far_fewer_iterations_than_cxx_on_band_and_holes():
    p = W.make_problem("grid2048", n=256)
    s = OF.unconstrained_realization(p.P, p.seed)
    v = OF.rhs(np.where(p.mask != 0, 0.0, p.d_obs - s), p.mask, p.P)
    _, ib = B.pcg_block(v, p.mask, p.P, 1e-8)
    _, ic = OF.pcg_cxx(v, p.mask, p.P, 1e-8)
    assert ib.converged and ic.converged
    assert ib.iterations * 4 <= ic.iterations, (ib.iterations, ic.iterations)
