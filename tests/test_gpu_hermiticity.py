"""GPU: the deliberately non-Hermitian operator of the Hermiticity study.

* the perturbed apply A_eps against the oracle's (FP64 1e-12, FP32 1e-4);
* plain CG on A_eps: the residual ratios sqrt(beta_j) from the device record
  against the oracle's CG residual history (1e-7 over the first 30 steps);
* the FP64 refinement loop (exact A in the true residual) still reaches the
  oracle's solution with a slightly skewed inner operator.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle.fill_oracle as OF
import workloads as W
from pins import rel

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


@pytest.mark.parametrize("nx,ny", [(64, 64), (256, 128)])
@pytest.mark.parametrize("eps", [1e-3, 0.2])
def test_skewed_apply_matches_oracle(F, nx, ny, eps):
    P = W.damped_power_law(nx, ny, 4.0, max(nx, ny) / 8, 1e-5)
    mask = W.band_holes_mask(nx, ny, W.band_rows(ny, 0.1), 6, 2.0, 6.0, 3)
    v = np.random.default_rng(1).standard_normal((ny, nx))
    ref = OF.apply_A_skew(v, mask, P, eps)
    plan = F.Plan(nx, ny, mask, P)
    plan.set_skew(eps)
    got64 = host(plan.apply(F.FILL_OP_A, dev(v), prec=F.FILL_PREC_FP64))
    got32 = host(plan.apply(F.FILL_OP_A, dev(v), prec=F.FILL_PREC_FP32_OP))
    assert rel(got64, ref) < 1e-12
    assert rel(got32, ref) < 1e-4
    plan.set_skew(0.0)
    assert rel(host(plan.apply(F.FILL_OP_A, dev(v), prec=F.FILL_PREC_FP64)), OF.apply_A(v, mask, P)) < 1e-12


def test_plain_cg_history_on_skewed_operator(F):
    p = W.make_problem("grid64")
    s = OF.unconstrained_realization(p.P, p.seed)
    v = OF.rhs(np.where(p.mask != 0, 0.0, p.d_obs - s), p.mask, p.P)
    eps, k = 0.1, 30
    h = OF.cg_residual_history(lambda x: OF.apply_A_skew(x, p.mask, p.P, eps), v, k)
    plan = F.Plan(p.nx, p.ny, p.mask, p.P)
    plan.set_precond(F.FILL_PRECOND_NONE)
    plan.set_skew(eps)
    plan.set_lanczos(64)
    plan.set_max_iter(64)
    plan.realize(dev(p.d_obs), p.seed, 1e-12, allow_noconv=True)
    _, be = plan.lanczos()
    ratio_gpu = np.sqrt(be[:k - 1])
    ratio_ref = h[1:k] / h[:k - 1]
    assert np.abs(ratio_gpu - ratio_ref).max() <= 1e-7 * ratio_ref.max()


def test_refinement_reaches_exact_solution_with_skewed_inner_operator(F):
    p = W.make_problem("grid64")
    ref = OF.fill_realize(p.d_obs, p.mask, p.P, p.seed, 1e-13)
    plan = F.Plan(p.nx, p.ny, p.mask, p.P)
    plan.set_skew(1e-3)
    x = host(plan.realize(dev(p.d_obs), p.seed, 1e-11))
    assert plan.stats()["rel_resid"] <= 1e-11
    assert rel(x, ref.x_out, p.mask != 0) < 1e-8
