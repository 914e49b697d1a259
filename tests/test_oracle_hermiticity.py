"""Pins of the oracle's deliberately non-Hermitian operator and plain-CG
residual history (the Hermiticity study of Sec. 3), CPU only."""

from __future__ import annotations

import numpy as np
import pytest

import oracle.fill_oracle as F
import workloads as W
from pins import _p_of_k, brute_circulant


def _case(nx=8, ny=6, seed=5):
    fn = lambda k: _p_of_k(k, 1.0, 2.5, 1e-3)  # noqa: E731
    P = W.damped_power_law(nx, ny, 1.0, 2.5, 1e-3)
    rng = np.random.default_rng(seed)
    mask = (rng.uniform(size=(ny, nx)) < 0.5).astype(np.uint8)
    Cinv = brute_circulant(nx, ny, fn, -1.0)
    return P, mask, Cinv, rng


def _K(v):
    # central difference along x on the torus: the real antisymmetric circulant
    return 0.5 * (np.roll(v, -1, axis=1) - np.roll(v, 1, axis=1))


@pytest.mark.parametrize("eps", [0.0, 1e-3, 0.3])
def test_skew_operator_matches_real_space_form(eps):
    P, mask, Cinv, rng = _case()
    m = mask != 0
    v = rng.standard_normal(mask.shape)
    pv = np.where(m, v, 0.0)
    ref = (Cinv @ (pv + eps * _K(pv)).ravel()).reshape(v.shape)
    ref = np.where(m, ref, 0.0)
    got = F.apply_A_skew(v, mask, P, eps)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_skew_zero_is_A_and_antisymmetric_part_closed_form():
    P, mask, Cinv, rng = _case(16, 12, 9)
    u, v = rng.standard_normal((2,) + mask.shape)
    assert np.allclose(F.apply_A_skew(v, mask, P, 0.0), F.apply_A(v, mask, P), rtol=0, atol=1e-13)
    eps = 0.05
    asym = np.vdot(u, F.apply_A_skew(v, mask, P, eps)) - np.vdot(F.apply_A_skew(u, mask, P, eps), v)
    m = mask != 0
    # <u, A v> - <A u, v> = 2 eps <u, Px C^-1 K Px v> since C^-1 K is antisymmetric
    pv = np.where(m, v, 0.0)
    ck = np.where(m, F.circulant_apply(_K(pv), P, -1.0), 0.0)
    assert asym == pytest.approx(2 * eps * np.vdot(u, ck), rel=1e-10)
    # and the symmetric part is untouched
    sym = np.vdot(u, F.apply_A_skew(v, mask, P, eps)) + np.vdot(F.apply_A_skew(u, mask, P, eps), v)
    assert sym == pytest.approx(2 * np.vdot(u, F.apply_A(v, mask, P)), rel=1e-10)


def test_cg_history_finite_termination():
    # SPD with n distinct eigenvalues: CG's residual vanishes at step n (exact arithmetic)
    d = np.array([1.0, 2.0, 3.5, 7.0, 11.0, 20.0])
    b = np.ones_like(d)
    h = F.cg_residual_history(lambda x: d * x, b, 6)
    assert h[0] == pytest.approx(np.sqrt(6.0))
    assert h[-1] <= 1e-10 * h[0]
    assert np.all(h[1:5] > 1e-6)


def test_cg_history_symmetric_vs_skewed_grid64():
    # on the fill operator: the skewed system stalls where the symmetric one converges
    p = W.make_problem("grid64")
    v = F.rhs(np.where(p.mask != 0, 0.0, p.d_obs), p.mask, p.P)
    h0 = F.cg_residual_history(lambda x: F.apply_A(x, p.mask, p.P), v, 800)
    h1 = F.cg_residual_history(lambda x: F.apply_A_skew(x, p.mask, p.P, 0.1), v, 800)
    assert h0[-1] / h0[0] < 1e-8
    assert h1[-1] / h1[0] > 1e3 * h0[-1] / h0[0]
