"""Pins of the oracle's Lanczos condition estimate (Sec. 6.4), CPU only.

The CG coefficients recorded by the oracle's solver give a tridiagonal
matrix; it is checked against (a) an explicit Lanczos run with full
reorthogonalisation on the dense operator and (b) the dense operator's
eigenvalues (Ritz values lie inside the spectrum and the extreme ones
converge to its ends).  A planted index slip in the tridiagonal must fail.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle.fill_oracle as F
import oracle.lanczos as L
import workloads as W
from pins import explicit_lanczos, masked_circulant_block


@pytest.fixture(scope="module")
def case64():
    p = W.make_problem("grid64")
    m = p.mask
    s = F.unconstrained_realization(p.P, p.seed)
    v = F.rhs(np.where(m != 0, 0.0, p.d_obs - s), m, p.P)
    Ci = masked_circulant_block(p.P, m, -1.0)
    Ch = masked_circulant_block(p.P, m, 0.5)
    vc = v.ravel()[m.ravel() != 0]
    out = {}
    for pre in (True, False):
        _, info = F.pcg_split(v, m, p.P, 1e-12, precond=pre)
        M = Ch @ Ci @ Ch if pre else Ci
        r0 = Ch @ vc if pre else vc
        out[pre] = (info, M, r0, np.linalg.eigvalsh(M))
    return out


def _tri_eigs(d, o):
    return np.linalg.eigvalsh(np.diag(d) + np.diag(o, 1) + np.diag(o, -1))


@pytest.mark.parametrize("pre,k", [(True, 10), (False, 40)])
def test_cg_tridiagonal_equals_explicit_lanczos(case64, pre, k):
    info, M, r0, _ = case64[pre]
    a, b = explicit_lanczos(M, r0, k)
    d, o = L.lanczos_tridiagonal(info.alphas[:k], info.betas[:k - 1])
    assert np.abs(d - a).max() <= 1e-9 * np.abs(a).max()
    assert np.abs(o - b).max() <= 1e-9 * np.abs(b).max()


@pytest.mark.parametrize("pre,tol_min", [(True, 0.05), (False, 1e-4)])
def test_ritz_values_bracketed_and_converged(case64, pre, tol_min):
    info, _, _, ev = case64[pre]
    rv = L.ritz_values(info.alphas, info.betas)
    assert len(rv) == info.iterations
    slack = 1e-9 * ev[-1]
    assert rv[0] >= ev[0] - slack and rv[-1] <= ev[-1] + slack
    assert abs(rv[-1] - ev[-1]) <= 1e-4 * ev[-1]
    assert abs(rv[0] - ev[0]) <= tol_min * ev[0]
    lo, hi, kappa = L.condition_estimate(info.alphas, info.betas)
    assert kappa == pytest.approx(ev[-1] / ev[0], rel=tol_min)


def test_preconditioner_lowers_condition_number(case64):
    # Sec. 2.4: E A E is better conditioned than A (here by more than 3x), and CG needs fewer steps.
    assert case64[True][3][-1] / case64[True][3][0] < case64[False][3][-1] / case64[False][3][0] / 3
    assert case64[True][0].iterations < case64[False][0].iterations


def test_unpreconditioned_solution_matches_preconditioned():
    p = W.make_problem("grid64")
    v = F.rhs(np.where(p.mask != 0, 0.0, p.d_obs), p.mask, p.P)
    u1, i1 = F.pcg_split(v, p.mask, p.P, 1e-11)
    u0, i0 = F.pcg_split(v, p.mask, p.P, 1e-11, precond=False)
    assert i0.converged and i1.converged
    assert np.linalg.norm(u1 - u0) <= 1e-6 * np.linalg.norm(u1)


def test_mutation_shifted_beta_index_fails(case64):
    info, M, r0, _ = case64[True]
    k = 10
    a, b = explicit_lanczos(M, r0, k)

    def wrong(alphas, betas):  # beta_j / alpha_j on the diagonal instead of beta_{j-1} / alpha_{j-1}
        al = np.asarray(alphas[:k])
        be = np.asarray(betas[:k])
        d = 1.0 / al
        d[1:] += be[1:k] / al[1:]
        return d, np.sqrt(be[:k - 1]) / al[:-1]

    d, o = wrong(info.alphas, info.betas)
    assert np.abs(d - a).max() > 1e-3 * np.abs(a).max()


# --------------------------------------------------------------------------
# PCG with M^-1 = Px C Px (covariance restricted to the masked pixels)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def case_cxx():
    p = W.make_problem("grid64")
    m = p.mask
    s = F.unconstrained_realization(p.P, p.seed)
    v = F.rhs(np.where(m != 0, 0.0, p.d_obs - s), m, p.P)
    Ci = masked_circulant_block(p.P, m, -1.0)
    Cxx = masked_circulant_block(p.P, m, 1.0)
    Lc = np.linalg.cholesky(Cxx)
    u, info = F.pcg_cxx(v, m, p.P, 1e-12)
    return p, v, u, info, Ci, Cxx, Lc


def test_pcg_cxx_solves_the_dense_system(case_cxx):
    # u* = A^-1 v with A the dense (C^-1)_xx block: direct solve
    p, v, u, info, Ci, _, _ = case_cxx
    m = p.mask.ravel() != 0
    ref = np.linalg.solve(Ci, v.ravel()[m])
    assert info.converged
    assert np.linalg.norm(u.ravel()[m] - ref) <= 1e-8 * np.linalg.norm(ref)
    assert np.all(u.ravel()[~m] == 0.0)


def test_pcg_cxx_tridiagonal_equals_explicit_lanczos(case_cxx):
    # PCG with M^-1 = L L^T on A is CG on L^T A L from L^T r0
    p, v, _, info, Ci, _, Lc = case_cxx
    k = 10
    vc = v.ravel()[p.mask.ravel() != 0]
    a, b = explicit_lanczos(Lc.T @ Ci @ Lc, Lc.T @ vc, k)
    d, o = L.lanczos_tridiagonal(info.alphas[:k], info.betas[:k - 1])
    assert np.abs(d - a).max() <= 1e-9 * np.abs(a).max()
    assert np.abs(o - b).max() <= 1e-9 * np.abs(b).max()


def test_pcg_cxx_ritz_values_inside_spectrum(case_cxx):
    _, _, _, info, Ci, _, Lc = case_cxx
    ev = np.linalg.eigvalsh(Lc.T @ Ci @ Lc)
    rv = L.ritz_values(info.alphas, info.betas)
    assert rv[0] >= ev[0] * (1 - 1e-9) and rv[-1] <= ev[-1] * (1 + 1e-9)
    assert abs(rv[-1] - ev[-1]) <= 1e-4 * ev[-1]
    assert abs(rv[0] - ev[0]) <= 0.05 * ev[0]


def test_pcg_cxx_matches_split_solution():
    p = W.make_problem("grid2048", n=128)
    v = F.rhs(np.where(p.mask != 0, 0.0, p.d_obs), p.mask, p.P)
    u1, i1 = F.pcg_split(v, p.mask, p.P, 1e-11)
    u2, i2 = F.pcg_cxx(v, p.mask, p.P, 1e-11)
    assert i1.converged and i2.converged
    assert np.linalg.norm(u2 - u1) <= 1e-6 * np.linalg.norm(u1)
