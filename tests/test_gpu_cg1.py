"""GPU: the single-reduction (Chronopoulos-Gear) form of the inner CG.

The recurrence forms z = M^-1 r and w = A z back to back and takes alpha and
beta from r.z, r.r and w.z; in exact arithmetic its iterates are those of the
standard recurrence (Sec. 2.4's PCG).  Checked here, against the oracle's
standard-recurrence PCG:

* the fill with each preconditioner (E E, Px C Px, none), FP64 and mixed, on
  grids of several tiles with ragged masks, reaches the oracle's solution to
  the usual bars (1e-9 FP64 at rtol 1e-12, 1e-5 mixed);
* the recorded CG coefficients equal the oracle's over the first steps (to
  1e-8, before the loss of orthogonality lets the two drift);
* iteration counts stay within 10% of the standard recurrence (the FP32
  recurrence for s = A p drifts a little faster than a fresh A p);
* graph replays are bitwise equal to direct launches; a batched plan matches
  one-problem plans; the 2048^2 workload meets its FP64 residual by the oracle.
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


def case(nx, ny, seed, band=0.1, holes=12):
    P = W.damped_power_law(nx, ny, 4.0, min(nx, ny) / 8, 1e-7)
    mask = W.band_holes_mask(nx, ny, W.band_rows(ny, band) if band else None, holes, 2.0, 7.0, seed)
    return P, mask, W.observed_map(P, nx, ny, seed + 1, mask)


def plan_for(F, nx, ny, mask, P, prec, pc, cg=1):
    plan = F.Plan(nx, ny, mask, P, prec=prec)
    plan.set_precond(pc)
    plan.set_cg(cg)
    return plan


@pytest.mark.parametrize("nx,ny,seed", [(256, 256, 31), (768, 512, 32), (1024, 128, 33)])
@pytest.mark.parametrize("pc", [0, 1, 2])
@pytest.mark.parametrize("prec,tol,rtol", [(0, 1e-9, 1e-12), (1, 1e-5, 1e-10)])
def test_fill_matches_oracle(F, nx, ny, seed, pc, prec, tol, rtol):
    # the band makes plain CG slow: no band for pc = 0
    P, mask, d = case(nx, ny, seed, band=0.0 if pc == 0 else 0.1, holes=12 if pc else 40)
    ref = OF.fill_realize(d, mask, P, 7, 1e-13)
    plan = plan_for(F, nx, ny, mask, P, prec, pc)
    x = host(plan.realize(dev(d), 7, rtol))
    m = mask != 0
    assert plan.stats()["status"] == 0
    assert rel(x, ref.x_out, m) < tol
    assert np.array_equal(x[~m].view(np.uint64), d[~m].view(np.uint64))


@pytest.mark.parametrize("pc,k", [(1, 10), (2, 10), (0, 40)])
def test_coefficients_match_oracle(F, pc, k):
    p = W.make_problem("grid64")
    s = OF.unconstrained_realization(p.P, p.seed)
    v = OF.rhs(np.where(p.mask != 0, 0.0, p.d_obs - s), p.mask, p.P)
    if pc == 2:
        _, info = OF.pcg_cxx(v, p.mask, p.P, 1e-12)
    else:
        _, info = OF.pcg_split(v, p.mask, p.P, 1e-12, precond=(pc == 1))
    plan = plan_for(F, p.nx, p.ny, p.mask, p.P, 0, pc)
    plan.set_lanczos(4096)
    plan.realize(dev(p.d_obs), p.seed, 1e-12)
    al, be = plan.lanczos()
    assert len(al) >= k
    assert np.abs(al[:k] - info.alphas[:k]).max() <= 1e-8 * np.abs(info.alphas[:k]).max()
    assert np.abs(be[:k - 1] - info.betas[:k - 1]).max() <= 1e-8 * np.abs(info.betas[:k - 1]).max()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("pc", [1, 2])
def test_iterations_close_to_standard(F, prec, pc):
    p = W.make_problem("grid2048", n=512)
    dd = dev(p.d_obs)
    it = {}
    for cg in (0, 1):
        plan = plan_for(F, p.nx, p.ny, p.mask, p.P, prec, pc, cg)
        plan.realize(dd, p.seed, 1e-8)
        st = plan.stats()
        assert st["status"] == 0 and st["rel_resid"] <= 1e-8
        it[cg] = st["iters_inner"]
    # Same iterates in exact arithmetic; in floating point the single-reduction
    # recurrence carries A p by its own recurrence (s = w + beta s), whose
    # rounding drifts from the explicit product at a different rate.  In FP64
    # the counts agree within 5%.  With FP32 operators the drift is 2^-24 per
    # step instead of 2^-53, and each refinement restart cuts it at a
    # different point, so the counts may part by up to 10% (measured: 495 and
    # 535 at this size).  The paper gives no counts: parity unpinned.
    bound = 0.05 if prec == 0 else 0.10
    assert abs(it[1] - it[0]) <= bound * it[0] + 2, it


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("pc", [0, 1, 2])
def test_graph_replay_bitwise(F, prec, pc):
    P, mask, d = case(256, 256, 41, band=0.1 if pc else 0.0, holes=25)
    dd = dev(d)
    ref_plan = plan_for(F, 256, 256, mask, P, prec, pc)
    ref_plan.set_graph(False)
    g_plan = plan_for(F, 256, 256, mask, P, prec, pc)
    junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for seed in (5, 6, 5):
        ref = host(ref_plan.realize(dd, seed, 1e-9))
        for rep in range(2):
            junk = junk * 1.0001 + 1.0  # eager work between replays
            got = host(g_plan.realize(dd, seed, 1e-9))
            st = g_plan.stats()
            assert st["status"] == 0 and st["rel_resid"] <= 1e-9
            if rep == 1:  # the iteration counts of the solve before: bitwise the step-by-step solve
                assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
                assert st["iters_inner"] == ref_plan.stats()["iters_inner"]


def test_batch_matches_single_and_oracle(F):
    n = 256
    probs = [case(n, n, 50 + i, band=0.1 + 0.05 * i, holes=10 + 5 * i) for i in range(3)]
    bp = F.BatchPlan(n, n, np.stack([m for _, m, _ in probs]), probs[0][0], prec=1)
    bp.set_precond(2)
    bp.set_cg(1)
    xb = host(bp.realize(dev(np.stack([d for _, _, d in probs])), [3, 4, 5], 1e-9))
    for i, (P, mask, d) in enumerate(probs):
        P0 = probs[0][0]
        ref = OF.fill_realize(d, mask, P0, 3 + i, 1e-12)
        assert rel(xb[i], ref.x_out, mask != 0) < 1e-5
        one = plan_for(F, n, n, mask, P0, 1, 2)
        x1 = host(one.realize(dev(d), 3 + i, 1e-9))
        assert rel(xb[i], x1, mask != 0) < 1e-6


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_2048_workload_residual(F, prec):
    # the 2048^2 workload as the benchmark runs it (Px C Px): the oracle's
    # FP64 residual of the GPU solution meets rtol; observed pixels untouched
    p = W.make_problem("grid2048")
    plan = plan_for(F, p.nx, p.ny, p.mask, p.P, prec, 2)
    x = host(plan.realize(dev(p.d_obs), p.seed, p.rtol))
    st = plan.stats()
    m = p.mask != 0
    s = OF.unconstrained_realization(p.P, p.seed)
    v = OF.rhs(np.where(m, 0.0, p.d_obs - s), p.mask, p.P)
    u = np.where(m, x - s, 0.0)
    res = np.linalg.norm(v - OF.apply_A(u, p.mask, p.P)) / np.linalg.norm(v)
    assert st["status"] == 0 and res < 1.5 * p.rtol
    assert np.array_equal(x[~m].view(np.uint64), p.d_obs[~m].view(np.uint64))


def test_cap_and_errors(F):
    P, mask, d = case(128, 128, 60)
    plan = plan_for(F, 128, 128, mask, P, 0, 2)
    plan.set_max_iter(3)
    plan.realize(dev(d), 1, 1e-12, allow_noconv=True)
    st = plan.stats()
    assert st["iters_inner"] <= 3 * max(1, st["iters_outer"])
    with pytest.raises(Exception):
        plan.set_cg(2)
