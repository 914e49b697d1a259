"""GPU: the Lanczos record of the CG solves, CG without the preconditioner
and CG with the Px C Px preconditioner.

* CG coefficients (alpha_j, beta_j) of the first inner solve against the
  oracle's (same Krylov space: agreement to 1e-8 over the first steps, before
  the loss of orthogonality of finite-precision CG lets the two drift);
* extreme Ritz values from the library's bisection: inside the dense
  spectrum of E A E (or A) at 64^2 and converged to its ends, equal to
  LAPACK's eigenvalues of the same tridiagonal to 1e-10;
* the solve without the preconditioner reaches the oracle's solution to the
  usual bars (1e-9 FP64, 1e-5 mixed);
* a batched plan records each problem's coefficients as a one-problem plan does.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle.fill_oracle as OF
import oracle.lanczos as OL
import workloads as W
from pins import masked_circulant_block, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_0286_amd as F
    return F


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def grid64():
    p = W.make_problem("grid64")
    s = OF.unconstrained_realization(p.P, p.seed)
    v = OF.rhs(np.where(p.mask != 0, 0.0, p.d_obs - s), p.mask, p.P)
    Ci = masked_circulant_block(p.P, p.mask, -1.0)
    Ch = masked_circulant_block(p.P, p.mask, 0.5)
    dense = {True: np.linalg.eigvalsh(Ch @ Ci @ Ch), False: np.linalg.eigvalsh(Ci)}
    return p, v, dense


@pytest.mark.parametrize("pre,k", [(True, 10), (False, 40)])
def test_coefficients_match_oracle(F, grid64, pre, k):
    p, v, _ = grid64
    _, info = OF.pcg_split(v, p.mask, p.P, 1e-12, precond=pre)
    plan = F.Plan(p.nx, p.ny, p.mask, p.P)
    plan.set_precond(pre)
    plan.set_lanczos(4096)
    plan.realize(dev(p.d_obs), p.seed, 1e-12)
    al, be = plan.lanczos()
    assert len(al) >= k
    assert np.abs(al[:k] - info.alphas[:k]).max() <= 1e-8 * np.abs(info.alphas[:k]).max()
    assert np.abs(be[:k - 1] - info.betas[:k - 1]).max() <= 1e-8 * np.abs(info.betas[:k - 1]).max()


@pytest.mark.parametrize("pre,tol_min", [(True, 0.05), (False, 1e-4)])
def test_ritz_extremes_inside_and_converged(F, grid64, pre, tol_min):
    p, _, dense = grid64
    ev = dense[pre]
    plan = F.Plan(p.nx, p.ny, p.mask, p.P)
    plan.set_precond(pre)
    plan.set_lanczos(4096)
    plan.realize(dev(p.d_obs), p.seed, 1e-12)
    lo, hi, n = plan.lanczos_extremes()
    al, be = plan.lanczos()
    assert n == len(al) == plan.stats()["iters_inner"]
    lap = OL.ritz_values(al, be)
    assert lo == pytest.approx(lap[0], rel=1e-10) and hi == pytest.approx(lap[-1], rel=1e-10)
    slack = 1e-9 * ev[-1]
    assert lo >= ev[0] - slack and hi <= ev[-1] + slack
    assert abs(hi - ev[-1]) <= 1e-4 * ev[-1]
    assert abs(lo - ev[0]) <= tol_min * ev[0]


@pytest.mark.parametrize("prec,tol,rtol", [(0, 1e-9, 1e-12), (1, 1e-5, 1e-11)])
def test_unpreconditioned_fill_matches_oracle(F, grid64, prec, tol, rtol):
    p, _, _ = grid64
    ref = OF.fill_realize(p.d_obs, p.mask, p.P, p.seed, 1e-13)
    plan = F.Plan(p.nx, p.ny, p.mask, p.P, prec=prec)
    plan.set_precond(False)
    x = host(plan.realize(dev(p.d_obs), p.seed, rtol))
    m = p.mask != 0
    assert rel(x, ref.x_out, m) < tol
    assert np.array_equal(x[~m].view(np.uint64), p.d_obs[~m].view(np.uint64))


def test_unpreconditioned_holes_only_mixed(F):
    # point-source mask without a band (the setting of Sec. 3), 256^2, mixed path
    n = 256
    P = W.damped_power_law(n, n, 4.0, n / 8, 1e-7)
    mask = W.band_holes_mask(n, n, None, 40, 2.0, 8.0, 11)
    d = W.observed_map(P, n, n, 5, mask)
    ref = OF.fill_realize(d, mask, P, 3, 1e-12)
    plan = F.Plan(n, n, mask, P, prec=1)
    plan.set_precond(False)
    x = host(plan.realize(dev(d), 3, 1e-10))
    assert rel(x, ref.x_out, mask != 0) < 1e-5


def test_batch_records_per_problem(F):
    n = 128
    probs = []
    for i in range(3):
        P = W.damped_power_law(n, n, 4.0, n / 8, 1e-7)
        mask = W.band_holes_mask(n, n, W.band_rows(n, 0.05 + 0.05 * i), 10 + 5 * i, 2.0, 6.0, 50 + i)
        probs.append((P, mask, W.observed_map(P, n, n, 60 + i, mask)))
    for pre in (True, False):
        bp = F.BatchPlan(n, n, np.stack([m for _, m, _ in probs]), probs[0][0])
        bp.set_precond(pre)
        bp.set_lanczos(2048)
        bp.realize(dev(np.stack([d for _, _, d in probs])), [7, 8, 9], 1e-10)
        for i, (P, mask, d) in enumerate(probs):
            plan = F.Plan(n, n, mask, P)
            plan.set_precond(pre)
            plan.set_lanczos(2048)
            plan.realize(dev(d), 7 + i, 1e-10)
            a1, b1 = plan.lanczos()
            ab, bb = bp.lanczos(i)
            assert len(a1) == len(ab) > 0
            assert np.allclose(ab, a1, rtol=1e-12, atol=0) and np.allclose(bb, b1, rtol=1e-12, atol=0)


def test_condition_estimate_256_matches_oracle(F):
    # the 2048^2 workload's structure at 256^2: FP64 path, preconditioned and plain
    p = W.make_problem("grid2048", n=256)
    s = OF.unconstrained_realization(p.P, p.seed)
    v = OF.rhs(np.where(p.mask != 0, 0.0, p.d_obs - s), p.mask, p.P)
    for pre in (True, False):
        _, info = OF.pcg_split(v, p.mask, p.P, 1e-8, precond=pre)
        lo_o, hi_o, _ = OL.condition_estimate(info.alphas, info.betas)
        plan = F.Plan(p.nx, p.ny, p.mask, p.P)
        plan.set_precond(pre)
        plan.set_lanczos(20000)
        plan.realize(dev(p.d_obs), p.seed, 1e-8)
        lo, hi, n = plan.lanczos_extremes()
        print(f"precond={pre}: GPU {n} steps lambda [{lo:.6g}, {hi:.6g}] kappa {hi / lo:.6g}; "
              f"oracle {len(info.alphas)} steps [{lo_o:.6g}, {hi_o:.6g}] kappa {hi_o / lo_o:.6g}")
        assert hi == pytest.approx(hi_o, rel=1e-6)
        assert lo == pytest.approx(lo_o, rel=1e-2)


def test_lanczos_errors(F, grid64):
    p, _, _ = grid64
    plan = F.Plan(p.nx, p.ny, p.mask, p.P)
    with pytest.raises(F.FillError):
        plan.lanczos_extremes()  # nothing recorded
    with pytest.raises(F.FillError):
        F.fill_plan_set_lanczos(plan.handle, -1)
    assert F.fill._lib.fill_plan_set_precond(plan.handle, 4) == F.FILL_EINVAL
    assert F.fill._lib.fill_plan_set_precond(plan.handle, -1) == F.FILL_EINVAL
    plan.set_lanczos(16)
    plan.realize(dev(p.d_obs), p.seed, 1e-10)
    al, be = plan.lanczos()
    assert len(al) == 16 and len(be) == 15  # capped record
    with pytest.raises(F.FillError):
        plan.lanczos_extremes(problem=1)


# ---------------------------------------------------------------------------
# M^-1 = Px C Px
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cxx64(grid64):
    p, v, _ = grid64
    _, info = OF.pcg_cxx(v, p.mask, p.P, 1e-12)
    Ci = masked_circulant_block(p.P, p.mask, -1.0)
    Lc = np.linalg.cholesky(masked_circulant_block(p.P, p.mask, 1.0))
    return p, info, np.linalg.eigvalsh(Lc.T @ Ci @ Lc)


def test_cxx_coefficients_and_ritz_values(F, cxx64):
    p, info, ev = cxx64
    plan = F.Plan(p.nx, p.ny, p.mask, p.P)
    plan.set_precond(F.FILL_PRECOND_CXX)
    plan.set_lanczos(4096)
    plan.realize(dev(p.d_obs), p.seed, 1e-12)
    al, be = plan.lanczos()
    k = 10
    assert np.abs(al[:k] - info.alphas[:k]).max() <= 1e-8 * np.abs(info.alphas[:k]).max()
    assert np.abs(be[:k - 1] - info.betas[:k - 1]).max() <= 1e-8 * np.abs(info.betas[:k - 1]).max()
    lo, hi, _ = plan.lanczos_extremes()
    assert lo >= ev[0] * (1 - 1e-9) and hi <= ev[-1] * (1 + 1e-9)
    assert abs(hi - ev[-1]) <= 1e-4 * ev[-1] and abs(lo - ev[0]) <= 0.05 * ev[0]


@pytest.mark.parametrize("prec,tol,rtol", [(0, 1e-9, 1e-12), (1, 1e-5, 1e-11)])
def test_cxx_fill_matches_oracle(F, grid64, prec, tol, rtol):
    p, _, _ = grid64
    ref = OF.fill_realize(p.d_obs, p.mask, p.P, p.seed, 1e-13)
    plan = F.Plan(p.nx, p.ny, p.mask, p.P, prec=prec)
    plan.set_precond(F.FILL_PRECOND_CXX)
    x = host(plan.realize(dev(p.d_obs), p.seed, rtol))
    m = p.mask != 0
    assert rel(x, ref.x_out, m) < tol
    assert np.array_equal(x[~m].view(np.uint64), p.d_obs[~m].view(np.uint64))


def test_cxx_mixed_512_matches_oracle(F):
    p = W.make_problem("grid2048", n=512)
    ref = OF.fill_realize(p.d_obs, p.mask, p.P, p.seed, 1e-11)
    plan = F.Plan(p.nx, p.ny, p.mask, p.P, prec=1)
    plan.set_precond(F.FILL_PRECOND_CXX)
    x = host(plan.realize(dev(p.d_obs), p.seed, 1e-10))
    assert rel(x, ref.x_out, p.mask != 0) < 1e-5
    assert plan.stats()["rel_resid"] <= 1e-10


def test_cxx_batch_matches_single(F):
    n = 256
    probs = []
    for i in range(2):
        P = W.damped_power_law(n, n, 4.0, n / 8, 1e-7)
        mask = W.band_holes_mask(n, n, W.band_rows(n, 0.1 + 0.05 * i), 20, 2.0, 8.0, 70 + i)
        probs.append((P, mask, W.observed_map(P, n, n, 80 + i, mask)))
    bp = F.BatchPlan(n, n, np.stack([m for _, m, _ in probs]), probs[0][0], prec=1)
    bp.set_precond(F.FILL_PRECOND_CXX)
    xb = host(bp.realize(dev(np.stack([d for _, _, d in probs])), [3, 4], 1e-9))
    for i, (P, mask, d) in enumerate(probs):
        ref = OF.fill_realize(d, mask, P, 3 + i, 1e-12)
        assert rel(xb[i], ref.x_out, mask != 0) < 1e-5
