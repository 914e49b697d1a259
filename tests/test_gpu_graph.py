"""GPU: graph replay of the inner CG chunks against direct launches.

The chunk graph is captured once per plan and replayed by every solve, so
each test runs several solves in a row (with the program's own eager work
and synchronisations between them) and requires every result to be bitwise
equal to the one from one-by-one launches: the kernels are deterministic,
so any difference would be a replay fault.
"""

from __future__ import annotations

import numpy as np
import pytest

import workloads as W

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


def case(n=256, seed=21, band=0.1, holes=25):
    P = W.damped_power_law(n, n, 4.0, n / 8, 1e-7)
    mask = W.band_holes_mask(n, n, W.band_rows(n, band) if band else None, holes, 2.0, 8.0, seed)
    return P, mask, W.observed_map(P, n, n, seed + 1, mask)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("pc", [0, 1, 2])
def test_graph_replay_bitwise(F, prec, pc):
    P, mask, d = case()
    dd = dev(d)
    ref_plan = F.Plan(256, 256, mask, P, prec=prec)
    ref_plan.set_graph(False)
    ref_plan.set_precond(pc)
    g_plan = F.Plan(256, 256, mask, P, prec=prec)
    g_plan.set_precond(pc)
    junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for seed in (5, 6, 5):
        ref = host(ref_plan.realize(dd, seed, 1e-9))
        junk = junk * 1.0001 + 1.0  # eager work between replays
        got = host(g_plan.realize(dd, seed, 1e-9))
        torch.cuda.synchronize()
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
        assert g_plan.stats()["iters_inner"] == ref_plan.stats()["iters_inner"]


def test_graph_batch_and_record(F):
    cases = [case(128, 30 + i, 0.05 * (i + 1), 10) for i in range(3)]
    masks = np.stack([c[1] for c in cases])
    d = dev(np.stack([c[2] for c in cases]))
    plans = []
    for on in (False, True):
        bp = F.BatchPlan(128, 128, masks, cases[0][0], prec=1)
        bp.set_graph(on)
        bp.set_precond(F.FILL_PRECOND_CXX)
        plans.append(bp)
    for rep in range(3):
        if rep == 1:
            for bp in plans:
                bp.set_lanczos(64)
        if rep == 2:
            for bp in plans:
                bp.set_lanczos(4096)  # grows the record: recording graphs are captured again
        xs = [host(bp.realize(d, [1, 2, 3], 1e-9)) for bp in plans]
        assert np.array_equal(xs[0].view(np.uint64), xs[1].view(np.uint64))
        if rep >= 1:
            for i in range(3):
                a0, b0 = plans[0].lanczos(i)
                a1, b1 = plans[1].lanczos(i)
                assert np.array_equal(a0, a1) and np.array_equal(b0, b1) and len(a0) > 0


def test_graph_concurrent_capture_multi(F):
    # realize_multi runs each plan on its own host thread: captures happen concurrently
    sizes = (128, 256)
    plans, ds, seeds, outs, refs = [], [], [], [], []
    for i, n in enumerate(sizes):
        cs = [case(n, 40 + 3 * i + j, 0.1, 15) for j in range(2)]
        bp = F.BatchPlan(n, n, np.stack([c[1] for c in cs]), cs[0][0], prec=1, stream=torch.cuda.Stream())
        plans.append(bp)
        ds.append(dev(np.stack([c[2] for c in cs])))
        seeds.append([7, 8])
        ref = F.BatchPlan(n, n, np.stack([c[1] for c in cs]), cs[0][0], prec=1)
        ref.set_graph(False)
        refs.append(host(ref.realize(ds[-1], [7, 8], 1e-9)))
    torch.cuda.synchronize()
    for _ in range(2):
        outs = [torch.empty_like(x) for x in ds]
        F.realize_multi(plans, ds, seeds, 1e-9, outs=outs)
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert np.array_equal(host(o).view(np.uint64), r.view(np.uint64))
