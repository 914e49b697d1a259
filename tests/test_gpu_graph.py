"""GPU: graph replays against direct launches.

Chunk graphs are captured once per plan and replayed by every solve, and a
solve whose kind ran last on the plan replays one whole-solve graph sized by
that solve's iteration counts.  Each test runs several solves in a row (with
the program's own eager work and synchronisations between them).  A solve
whose iteration counts equal those of the solve before it (the same seed
again) must be bitwise equal to the step-by-step solve with one-by-one
launches: the kernels are deterministic, so any difference would be a replay
fault.  A solve after one with other counts must meet its tolerance and stay
within kappa * rtol of it.
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
        assert ref_plan.stats()["whole_graph"] == 0
        for rep in range(2):
            junk = junk * 1.0001 + 1.0  # eager work between replays
            got = host(g_plan.realize(dd, seed, 1e-9))
            torch.cuda.synchronize()
            st = g_plan.stats()
            assert st["status"] == 0 and st["rel_resid"] <= 1e-9
            if rep == 1:  # the counts of the solve before: bitwise the step-by-step solve
                assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
                assert st["iters_inner"] == ref_plan.stats()["iters_inner"]
            else:
                m = mask != 0
                assert np.linalg.norm(got[m] - ref[m]) <= 1e-5 * np.linalg.norm(ref[m])


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


@pytest.mark.parametrize("prec", [0, 1])
def test_whole_solve_graph_is_used_and_exact(F, prec):
    # block preconditioner (few iterations): after one step-by-step solve the
    # same solve replays as one graph; bitwise equal to the step-by-step one,
    # with the Lanczos record of its first inner solve
    P, mask, d = case(256, 51, 0.1, 25)
    dd = dev(d)
    ref = F.Plan(256, 256, mask, P, prec=prec)
    ref.set_precond(F.FILL_PRECOND_BLOCK)
    ref.set_graph(False)
    ref.set_lanczos(64)
    g = F.Plan(256, 256, mask, P, prec=prec)
    g.set_precond(F.FILL_PRECOND_BLOCK)
    g.set_lanczos(64)
    want = host(ref.realize(dd, 9, 1e-9))
    first = host(g.realize(dd, 9, 1e-9))
    assert g.stats()["whole_graph"] == 0
    assert np.array_equal(first.view(np.uint64), want.view(np.uint64))
    for _ in range(3):
        got = host(g.realize(dd, 9, 1e-9))
        st = g.stats()
        assert st["whole_graph"] == 1 and st["status"] == 0
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
        assert st["iters_inner"] == ref.stats()["iters_inner"]
        assert st["iters_outer"] == ref.stats()["iters_outer"]
        a0, b0 = ref.lanczos()
        a1, b1 = g.lanczos()
        assert np.array_equal(a0, a1) and np.array_equal(b0, b1) and len(a0) > 0
    # the mean uses its own counts: step by step first, then a graph
    mref = host(ref.mean(dd, 1e-9))
    m1 = host(g.mean(dd, 1e-9))
    assert g.stats()["whole_graph"] == 0
    m2 = host(g.mean(dd, 1e-9))
    assert g.stats()["whole_graph"] == 1
    assert np.array_equal(m1.view(np.uint64), mref.view(np.uint64))
    assert np.array_equal(m2.view(np.uint64), mref.view(np.uint64))


def test_whole_solve_graph_with_too_few_iterations_continues(F):
    # a tighter tolerance than the solve before: the graph's steps stop short,
    # the refinement continues step by step and reaches the tolerance
    P, mask, d = case(256, 52, 0.1, 25)
    dd = dev(d)
    g = F.Plan(256, 256, mask, P, prec=1)
    g.set_precond(F.FILL_PRECOND_BLOCK)
    ref = F.Plan(256, 256, mask, P, prec=0)
    ref.set_precond(F.FILL_PRECOND_BLOCK)
    want = host(ref.realize(dd, 3, 1e-12))
    g.realize(dd, 3, 1e-6)
    got = host(g.realize(dd, 3, 1e-10))
    st = g.stats()
    assert st["status"] == 0 and st["rel_resid"] <= 1e-10 and st["whole_graph"] == 0
    m = mask != 0
    assert np.linalg.norm(got[m] - want[m]) <= 1e-5 * np.linalg.norm(want[m])
