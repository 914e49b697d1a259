"""GPU: batched plans (several problems per launch) and concurrent plans.

A batched solve must give each problem the result of its own single-problem
solve, and match the FP64 oracle to the same bars as single solves.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W
from pins import rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_0286_amd as F
    return F


def problems(n, nprob, seed0, per_problem_pk=False):
    masks, ds, Ps = [], [], []
    for i in range(nprob):
        damping = n / 8 * (1.0 + 0.25 * i) if per_problem_pk else n / 8
        P = W.damped_power_law(n, n, 4.0, damping, 1e-7)
        band = W.band_rows(n, 0.05 + 0.05 * (i % 3))
        m = W.band_holes_mask(n, n, band, 5 + 7 * i, 2.0, 8.0, mask_seed=seed0 + i)
        masks.append(m)
        Ps.append(P)
        ds.append(W.observed_map(P, n, n, seed=seed0 + 50 + i, mask=m))
    return np.stack(masks), np.stack(ds), (np.stack(Ps) if per_problem_pk else Ps[0]), Ps


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_single_solves(F, prec):
    n, nprob = 256, 3
    masks, ds, P, _ = problems(n, nprob, 10)
    seeds = [7, 8, 9]
    bp = F.BatchPlan(n, n, masks, P, prec)
    xb = bp.realize(torch.from_numpy(ds).cuda(), seeds, 1e-9).cpu().numpy()
    stb = bp.stats()
    for i in range(nprob):
        sp = F.Plan(n, n, masks[i], P, prec)
        xs = sp.realize(torch.from_numpy(ds[i]).cuda(), seeds[i], 1e-9).cpu().numpy()
        st = sp.stats()
        assert st["iters_inner"] == stb[i]["iters_inner"]
        assert np.array_equal(xb[i], xs), i


@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 1e-5)])
def test_batch_per_problem_spectra_match_oracle(F, prec, tol):
    n, nprob = 256, 4
    masks, ds, Pb, Ps = problems(n, nprob, 20, per_problem_pk=True)
    seeds = [11, 12, 13, 14]
    rtol = 1e-12 if prec == 0 else 1e-8
    bp = F.BatchPlan(n, n, masks, Pb, prec)
    xb = bp.realize(torch.from_numpy(ds).cuda(), seeds, rtol, allow_noconv=(prec == 0)).cpu().numpy()
    for i in range(nprob):
        ref = O.fill_realize(ds[i], masks[i], Ps[i], seeds[i], 1e-12)
        m = masks[i] != 0
        assert rel(xb[i], ref.x_out, m) < tol, i
        assert np.array_equal(xb[i][~m].view(np.uint64), ds[i][~m].view(np.uint64))


def test_batch_mean_matches_oracle(F):
    n, nprob = 128, 3
    masks, ds, P, _ = problems(n, nprob, 30)
    bp = F.BatchPlan(n, n, masks, P, 0)
    xb = bp.mean(torch.from_numpy(ds).cuda(), 1e-12, allow_noconv=True).cpu().numpy()
    for i in range(nprob):
        ref = O.fill_mean(ds[i], masks[i], P, 1e-12)
        assert rel(xb[i], ref.x_out, masks[i] != 0) < 1e-9


def test_batch_with_degenerate_problems(F):
    # an unmasked problem and an all-masked one next to an ordinary one
    n = 64
    masks, ds, P, _ = problems(n, 3, 40)
    masks[1] = 0
    masks[2] = 1
    ds[2] = 0.0
    bp = F.BatchPlan(n, n, masks, P, 1)
    xb = bp.realize(torch.from_numpy(ds).cuda(), [1, 2, 3], 1e-8).cpu().numpy()
    assert np.array_equal(xb[1], ds[1])
    sp = F.Plan(n, n, masks[2], P, 1)
    assert np.array_equal(xb[2], sp.realize_unconstrained(3).cpu().numpy())
    ref = O.fill_realize(ds[0], masks[0], P, 1, 1e-12)
    assert rel(xb[0], ref.x_out, masks[0] != 0) < 1e-5
    st = bp.stats()
    assert st[1]["iters_inner"] == 0 and st[2]["iters_inner"] == 0


def test_multi_plans_of_different_sizes(F):
    plans, dl, sl, singles = [], [], [], []
    for n, nprob, s0 in ((256, 2, 50), (768, 2, 60)):
        masks, ds, P, _ = problems(n, nprob, s0)
        stream = torch.cuda.Stream()
        plans.append(F.BatchPlan(n, n, masks, P, 1, stream=stream))
        dl.append(torch.from_numpy(ds).cuda())
        sl.append([s0 + 1, s0 + 2])
        singles.append((n, masks, ds, P))
    torch.cuda.synchronize()
    outs = F.realize_multi(plans, dl, sl, 1e-8)
    torch.cuda.synchronize()
    for (n, masks, ds, P), o, seeds in zip(singles, outs, sl):
        o = o.cpu().numpy()
        for i in range(len(seeds)):
            sp = F.Plan(n, n, masks[i], P, 1)
            xs = sp.realize(torch.from_numpy(ds[i]).cuda(), seeds[i], 1e-8).cpu().numpy()
            assert np.array_equal(o[i], xs)
