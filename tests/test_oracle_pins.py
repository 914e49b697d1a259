"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each pin checks the oracle against something it does not itself compute:
an independent implementation of the random generator, brute-force DFT
matrices, the textbook conditional Gaussian through an explicit matrix
inverse, per-frequency direct solves, the lattice-Laplacian closed form,
sparse direct elimination and sampling statistics.  The mutation tests at the
end plant plausible mistakes in the oracle and check that a pin catches each.
"""

from __future__ import annotations

import numpy as np
import pytest
import scipy.stats as st

import oracle as O
import oracle.fill_oracle as F
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


from pins import (_p_of_k, brute_circulant, brute_circulant_case, band_direct,  # noqa: E402
                  laplace_band_closed_form, laplace_sparse_direct, rel)


def err_circulant(nx=8, ny=6, power=-1.0, seed=3, table=None):
    P, v, ref = brute_circulant_case(nx, ny, power, seed, table)
    got = F.circulant_apply(v, P, power)
    return np.abs(got - ref).max() / np.abs(ref).max()


# --------------------------------------------------------------------------
# random generator
# --------------------------------------------------------------------------

def test_philox_matches_numpy_bitwise():
    # numpy's Philox is an independent Philox4x64-10; it advances its counter
    # before producing each block, so block c of ours is its first block at c-1.
    for seed, stream in ((0, 0x52), (12345, 0x4F), (2 ** 63 + 7, 1)):
        for c in (1, 2, 17, 2 ** 40 + 3):
            bg = np.random.Philox(key=np.array([seed, stream], dtype=np.uint64),
                                  counter=np.array([c - 1, 0, 0, 0], dtype=np.uint64))
            ref = bg.random_raw(4)
            got = O.philox4x64_10(np.uint64(c), 0, 0, 0, np.uint64(seed), np.uint64(stream))
            assert [int(g) for g in got] == [int(r) for r in ref]


def test_philox_full_counter_words():
    # all four counter words enter the rounds
    bg = np.random.Philox(key=np.array([9, 8], dtype=np.uint64),
                          counter=np.array([4, 5, 6, 7], dtype=np.uint64))
    ref = bg.random_raw(4)
    got = O.philox4x64_10(np.uint64(5), np.uint64(5), np.uint64(6), np.uint64(7),
                          np.uint64(9), np.uint64(8))
    assert [int(g) for g in got] == [int(r) for r in ref]


def test_white_noise_is_standard_normal():
    w = O.white_noise(256, 128, seed=7)
    assert abs(w.mean()) < 5 / np.sqrt(w.size)
    assert abs(w.var() - 1) < 5 * np.sqrt(2 / w.size)
    assert st.kstest(w.ravel(), "norm").pvalue > 1e-4
    # the two pixels of a Box-Muller pair (cosine and sine of one angle) and
    # the two pairs of a block are uncorrelated
    c = np.corrcoef(w.ravel()[0::2], w.ravel()[1::2])[0, 1]
    assert abs(c) < 5 / np.sqrt(w.size / 2)
    c4 = np.corrcoef(w.ravel()[0::4], w.ravel()[2::4])[0, 1]
    assert abs(c4) < 5 / np.sqrt(w.size / 4)
    # squares of a pair: r^2 (cos^2 + sin^2) = -2 ln u is exponential with mean 2
    q = w.ravel()[0::2] ** 2 + w.ravel()[1::2] ** 2
    assert st.kstest(q / 2.0, "expon").pvalue > 1e-4
    # different seeds are uncorrelated
    c2 = np.corrcoef(w.ravel(), O.white_noise(256, 128, seed=8).ravel())[0, 1]
    assert abs(c2) < 5 / np.sqrt(w.size)


def _white_noise_pin_error(noise=None):
    """Largest deviation of white_noise from pixels 4j .. 4j+3 recomputed one
    by one from numpy's independent Philox words (counter one behind, see
    above) with the math module's log, cos and sin, relative to
    max(1, |value|)."""
    import math
    nx, ny, seed = 64, 32, 2 ** 61 + 11
    w = (noise or O.white_noise)(nx, ny, seed).ravel()
    worst = 0.0
    # (block 0 is out of reach: numpy's counter -1 carries into its second word)
    for j in (1, 2, 257, nx * ny // 4 - 1):
        bg = np.random.Philox(key=np.array([seed, O.REALIZATION_STREAM], dtype=np.uint64),
                              counter=np.array([j - 1, 0, 0, 0], dtype=np.uint64))
        words = [int(v) for v in bg.random_raw(4)]
        u = [((x >> 11) + 0.5) * 2.0 ** -53 for x in words]
        want = []
        for a, b in ((0, 1), (2, 3)):
            r, th = math.sqrt(-2.0 * math.log(u[a])), 2.0 * math.pi * u[b]
            want += [r * math.cos(th), r * math.sin(th)]
        for k in range(4):
            worst = max(worst, abs(w[4 * j + k] - want[k]) / max(1.0, abs(want[k])))
    return worst


def test_white_noise_pixels_from_independent_words():
    # exact pin of the Box-Muller mapping (to libm rounding)
    assert _white_noise_pin_error() <= 4e-16


# --------------------------------------------------------------------------
# circulant covariance and the FFT convention
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny", [(8, 6), (6, 9), (4, 4), (12, 5)])
@pytest.mark.parametrize("power", [-1.0, 0.5, 1.0])
def test_circulant_apply_matches_explicit_dft_matrices(nx, ny, power):
    assert err_circulant(nx, ny, power) < 1e-12


def test_dense_covariance_matches_explicit_dft_matrices():
    nx, ny = 6, 4
    fn = lambda k: _p_of_k(k, 1.0, 2.5, 1e-3)  # noqa: E731
    P = W.damped_power_law(nx, ny, 1.0, 2.5, 1e-3)
    assert np.allclose(O.dense.dense_covariance(P), brute_circulant(nx, ny, fn, 1.0), atol=1e-14)


def test_circulant_power_composition_and_unitarity():
    # C^{1/2} C^{1/2} = C, C^-1 C = I: the torus DFT is exactly unitary (Sec. 4)
    P = W.damped_power_law(32, 24, 4.0, 6.0, 1e-5)
    v = np.random.default_rng(1).standard_normal((24, 32))
    h = O.circulant_apply(O.circulant_apply(v, P, 0.5), P, 0.5)
    assert rel(h, O.circulant_apply(v, P, 1.0)) < 1e-13
    assert rel(O.circulant_apply(O.circulant_apply(v, P, 1.0), P, -1.0), v) < 1e-10


# --------------------------------------------------------------------------
# conditional mean: dense, Schur, PCG
# --------------------------------------------------------------------------

def test_dense_conditional_mean_equals_precision_block_form():
    # C_xy C_yy^-1 y = -((C^-1)_xx)^-1 (C^-1)_xy y (Sec. 2.1 / Sec. 2.3)
    nx, ny = 8, 6
    P = W.damped_power_law(nx, ny, 1.0, 3.0, 1e-3)
    mask = np.zeros((ny, nx), np.uint8)
    mask[2:4, 1:5] = 1
    mask[5, 7] = 1
    t = np.random.default_rng(2).standard_normal((ny, nx))
    Cinv = np.linalg.inv(O.dense.dense_covariance(P))
    m = mask.ravel() != 0
    ref = -np.linalg.solve(Cinv[np.ix_(m, m)], Cinv[np.ix_(m, ~m)] @ t.ravel()[~m])
    got = O.dense.conditional_mean_dense(t, mask, P).ravel()[m]
    assert rel(got, ref) < 1e-10


def _pcg_vs_dense_grid64(rtol=1e-12):
    p = W.make_problem("grid64")
    r = O.fill_realize(p.d_obs, p.mask, p.P, p.seed, rtol)
    t = np.where(p.mask != 0, 0.0, p.d_obs - r.s)
    ud = O.dense.conditional_mean_dense(t, p.mask, p.P)
    return rel(r.u, ud, p.mask != 0), r


def test_pcg_matches_dense_cholesky_grid64():
    e, r = _pcg_vs_dense_grid64()
    assert r.info.converged
    assert e < 1e-9


def test_fill_realize_keeps_observed_pixels_bitwise():
    p = W.make_problem("grid64")
    d = p.d_obs.copy()
    d[p.mask != 0] = np.nan  # masked inputs are ignored
    r = O.fill_realize(d, p.mask, p.P, p.seed, 1e-10)
    obs = p.mask == 0
    assert np.array_equal(r.x_out[obs].view(np.uint64), p.d_obs[obs].view(np.uint64))
    assert np.all(np.isfinite(r.x_out))


def test_pcg_matches_band_direct_solve():
    n = 256
    p = W.make_problem("grid2048", n=n, n_holes=0)
    r0, h = p.meta["band"]
    fn = lambda k: _p_of_k(k, 4.0, p.meta["damping"], 1e-7)  # noqa: E731
    t = np.where(p.mask != 0, 0.0, p.d_obs)
    ref = band_direct(t, r0, h, fn)
    got = O.fill_mean(p.d_obs, p.mask, p.P, 1e-12).u
    assert rel(got, ref, p.mask != 0) < 1e-9


def test_pcg_matches_laplacian_strip_closed_form():
    n, mu2 = 128, 1e-3
    P = W.laplacian_spectrum(n, n, mu2)
    r0, h = 50, 28
    mask = W.band_holes_mask(n, n, (r0, h), 0, 0, 0, 0)
    y = W.observed_map(P, n, n, seed=5, mask=mask)
    ref = laplace_band_closed_form(y, r0, h, mu2)
    got = O.fill_mean(y, mask, P, 1e-13).u
    assert rel(got, ref, mask != 0) < 1e-10


def test_pcg_matches_laplacian_sparse_direct_with_holes():
    n, mu2 = 96, 1e-2
    P = W.laplacian_spectrum(n, n, mu2)
    mask = W.band_holes_mask(n, n, (40, 9), 12, 2.0, 6.0, mask_seed=3)
    y = W.observed_map(P, n, n, seed=6, mask=mask)
    ref = laplace_sparse_direct(y, mask, mu2)
    got = O.fill_mean(y, mask, P, 1e-13).u
    assert rel(got, ref, mask != 0) < 1e-10


def test_ml_condition_and_scale_invariance():
    # Px C^-1 x_out_ML = 0 on the masked pixels (the ML condition of Sec. 5),
    # and M is unchanged under P -> c P.
    p = W.make_problem("grid64")
    a = O.fill_mean(p.d_obs, p.mask, p.P, 1e-12)
    g = O.circulant_apply(a.x_out, p.P, -1.0)
    m = p.mask != 0
    assert np.linalg.norm(g[m]) < 1e-8 * np.linalg.norm(O.circulant_apply(np.where(m, 0, p.d_obs), p.P, -1.0)[m])
    b = O.fill_mean(p.d_obs, p.mask, 37.0 * p.P, 1e-12)
    assert rel(b.u, a.u, m) < 1e-9


def test_linearity_and_translation_equivariance():
    p = W.make_problem("grid64")
    m = p.mask != 0
    y2 = W.observed_map(p.P, 64, 64, seed=11, mask=p.mask)
    u1 = O.fill_mean(p.d_obs, p.mask, p.P, 1e-12).u
    u2 = O.fill_mean(y2, p.mask, p.P, 1e-12).u
    u12 = O.fill_mean(2.0 * p.d_obs - 3.0 * y2, p.mask, p.P, 1e-12).u
    assert rel(u12, 2.0 * u1 - 3.0 * u2, m) < 1e-9
    sh = (5, 13)
    us = O.fill_mean(np.roll(p.d_obs, sh, (0, 1)), np.roll(p.mask, sh, (0, 1)), p.P, 1e-12).u
    assert rel(us, np.roll(u1, sh, (0, 1)), np.roll(m, sh, (0, 1))) < 1e-9


def test_operators_are_symmetric():
    # <u, A v> = <A u, v> and the same for E (Hermiticity, Sec. 3)
    p = W.make_problem("grid64")
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal((2, 64, 64))
    for op in (O.apply_A, O.apply_E):
        a = np.vdot(u, op(v, p.mask, p.P))
        b = np.vdot(op(u, p.mask, p.P), v)
        assert abs(a - b) <= 1e-12 * abs(a)


# --------------------------------------------------------------------------
# statistics of the realization and of the constrained draw
# --------------------------------------------------------------------------

def test_realization_spectrum_matches_P():
    # E |s_k|^2 / N = P(k) for every mode; check per |k| annulus over seeds
    n, S = 32, 300
    P = W.damped_power_law(n, n, 1.0, 6.0, 1e-4)
    kk = W.kgrid(n, n)
    ratio = np.zeros((S,) + P.shape)
    for s in range(S):
        sk = np.fft.rfft2(O.unconstrained_realization(P, seed=s))
        ratio[s] = np.abs(sk) ** 2 / (n * n) / P
    # real modes (kx = 0 or n/2 with ky = 0 or n/2) have variance 2, others 1
    var = np.ones(P.shape)
    for iy in (0, n // 2):
        for ix in (0, n // 2):
            var[iy, ix] = 2.0
    # modes with kx = 0 or n/2 appear twice (ky and -ky) in the half grid, so
    # bin only kx in 1..n/2-1 plus ky >= 0 of the two real columns
    sel = np.zeros(P.shape, bool)
    sel[:, 1:n // 2] = True
    sel[: n // 2 + 1, 0] = True
    sel[: n // 2 + 1, n // 2] = True
    bins = np.floor(kk).astype(int)
    for b in np.unique(bins[sel]):
        cell = sel & (bins == b)
        mean = ratio[:, cell].mean()
        se = np.sqrt(var[cell].sum() / (S * cell.sum() ** 2))
        assert abs(mean - 1.0) < 5 * se, (b, mean, se)


def _tiny_problem():
    nx, ny = 8, 8
    P = W.damped_power_law(nx, ny, 1.0, 3.0, 1e-3)
    mask = np.zeros((ny, nx), np.uint8)
    mask[3:5, 2:6] = 1
    mask[6, 1] = 1
    return nx, ny, P, mask


def test_constrained_draw_has_schur_covariance():
    # x_out - x_ML has covariance C_xx - C_xy C_yy^-1 C_yx (eq. starH, Sec. 2.3)
    nx, ny, P, mask = _tiny_problem()
    m = mask.ravel() != 0
    d = W.observed_map(P, nx, ny, seed=1, mask=mask)
    xml = O.fill_mean(d, mask, P, 1e-13).x_out.ravel()[m]
    S = 3000
    e = np.array([O.fill_realize(d, mask, P, s, 1e-13).x_out.ravel()[m] - xml for s in range(S)])
    Sig = O.dense.conditional_covariance_dense(mask, P)
    emp = e.T @ e / S
    se = np.sqrt((np.outer(np.diag(Sig), np.diag(Sig)) + Sig ** 2) / S)
    assert np.all(np.abs(emp - Sig) < 5 * se)
    assert np.all(np.abs(e.mean(0)) < 5 * np.sqrt(np.diag(Sig) / S))


def test_constrained_draw_with_fresh_data_is_unconditionally_C():
    # with y drawn from P for every trial, the filled map is N(0, C) exactly
    nx, ny, P, mask = _tiny_problem()
    S = 3000
    X = np.array([O.fill_realize(W.observed_map(P, nx, ny, seed=10_000 + s, mask=mask),
                                 mask, P, s, 1e-13).x_out.ravel() for s in range(S)])
    C = O.dense.dense_covariance(P)
    emp = X.T @ X / S
    se = np.sqrt((np.outer(np.diag(C), np.diag(C)) + C ** 2) / S)
    assert np.all(np.abs(emp - C) < 5.5 * se)


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------

def test_no_masked_pixels_returns_data():
    P = W.damped_power_law(16, 16, 1.0, 3.0, 1e-4)
    d = W.observed_map(P, 16, 16, seed=1)
    r = O.fill_realize(d, np.zeros((16, 16), np.uint8), P, 3, 1e-10)
    assert np.array_equal(r.x_out, d)
    assert r.info.iterations == 0


def test_all_masked_returns_unconstrained_realization():
    P = W.damped_power_law(16, 16, 1.0, 3.0, 1e-4)
    d = np.zeros((16, 16))
    r = O.fill_realize(d, np.ones((16, 16), np.uint8), P, 3, 1e-10)
    assert np.array_equal(r.x_out, O.unconstrained_realization(P, 3))


# --------------------------------------------------------------------------
# mutation tests: plausible mistakes planted in the oracle must fail a pin
# --------------------------------------------------------------------------

def test_mutation_rhs_sign_is_caught(monkeypatch):
    orig = F.rhs
    monkeypatch.setattr(F, "rhs", lambda t, m, P: -orig(t, m, P))
    e, _ = _pcg_vs_dense_grid64(1e-10)
    assert e > 1.0


def test_mutation_operator_power_is_caught(monkeypatch):
    def bad_A(v, mask, P):
        return F._Px(F.circulant_apply(F._Px(v, mask), P, 1.0), mask)
    monkeypatch.setattr(F, "apply_A", bad_A)
    e, _ = _pcg_vs_dense_grid64(1e-10)
    assert e > 1e-3


def test_mutation_transposed_spectrum_table_is_caught():
    nx, ny = 8, 6
    P = W.damped_power_law(nx, ny, 1.0, 2.5, 1e-3)
    # a (kx, ky)-swapped table of the right shape
    bad = W.damped_power_law(2 * (ny // 2 + 1 - 1), 2 * (nx // 2), 1.0, 2.5, 1e-3)
    bad = np.resize(bad.T, P.shape)
    assert err_circulant(nx, ny, 1.0, table=bad) > 1e-3


def test_mutation_missing_normalisation_is_caught(monkeypatch):
    orig = F.circulant_apply
    monkeypatch.setattr(F, "circulant_apply", lambda v, P, a: orig(v, P, a) * v.size)
    assert err_circulant(8, 6, 0.5) > 1.0


def test_mutation_white_noise_mapping_is_caught():
    # cosine and sine exchanged, the word pairs of a block swapped, or radius
    # and angle words exchanged: each fails the exact pin
    def noise(nx, ny, seed, swap=False, trig=False, ra=False):
        j = np.arange(nx * ny // 4, dtype=np.uint64)
        z = np.zeros_like(j)
        w = list(O.philox4x64_10(j, z, z, z, np.uint64(seed), np.uint64(O.REALIZATION_STREAM)))
        if swap:
            w = [w[2], w[3], w[0], w[1]]
        if ra:
            w = [w[1], w[0], w[3], w[2]]
        un = [((x >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53 for x in w]
        f0, f1 = (np.sin, np.cos) if trig else (np.cos, np.sin)
        out = np.empty(nx * ny)
        for k in range(2):
            r, th = np.sqrt(-2.0 * np.log(un[2 * k])), 2.0 * np.pi * un[2 * k + 1]
            out[2 * k::4] = r * f0(th)
            out[2 * k + 1::4] = r * f1(th)
        return out.reshape(ny, nx)

    assert _white_noise_pin_error(noise) <= 4e-16  # the helper's own control
    assert _white_noise_pin_error(lambda a, b, c: noise(a, b, c, trig=True)) > 1e-3
    assert _white_noise_pin_error(lambda a, b, c: noise(a, b, c, ra=True)) > 1e-3
    assert _white_noise_pin_error(lambda a, b, c: noise(a, b, c, swap=True)) > 1e-3
