"""GPU: a group of batched plans of uneven grid sizes (256^2, 512^2, 768^2,
1024^2) solved as one graph launch (fill_group_realize), against the oracle.

The first call runs step by step (it gives the step counts); every later call
is one graph launch with one branch per plan.  Each problem's fill must match
the oracle's constrained realization solved to 1e-12 (block-preconditioned
oracle CG, stopped on the true residual of the oracle's own operator) on the
masked pixels to 1e-5 (FP32 operators, FP64 refinement, rtol 1e-8: the bar of
the mixed path); observed pixels are bitwise the data; the graph call is
bitwise the step-by-step call (same seeds, same counts).  A tighter tolerance
than the counts were taken at makes the plans continue step by step after
the graph and still meet it.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SIZES = (256, 512, 768, 1024)
PER = 2  # problems per size


@pytest.fixture(scope="module")
def problems():
    probs = {}
    for i, n in enumerate(SIZES):
        P = W.damped_power_law(n, n, 4.0, n / 8, 1e-7)
        lst = []
        for j in range(PER):
            k = PER * i + j
            rng = np.random.default_rng(900 + k)
            frac = float(rng.uniform(0.05, 0.2))
            nh = int(rng.integers(20, 101))
            mask = W.band_holes_mask(n, n, W.band_rows(n, frac), nh, 2.0, 10.0, 1000 + k)
            d = W.observed_map(P, n, n, 2 * k, mask)
            lst.append((mask, d, 2 * k + 1))
        probs[n] = (P, lst)
    return probs


@pytest.fixture(scope="module")
def oracle_fills(problems):
    out = {}
    for n, (P, lst) in problems.items():
        for j, (mask, d, seed) in enumerate(lst):
            print(f"oracle {n}^2 problem {j} seed {seed}", flush=True)
            r = O.fill_realize(d, mask, P, seed, 1e-12, solver="block")
            assert r.info.converged
            out[(n, j)] = r.x_out
    return out


def make_group(F, problems):
    plans, ds, seeds = [], [], []
    for n, (P, lst) in problems.items():
        bp = F.BatchPlan(n, n, np.stack([m for m, _, _ in lst]), P, F.FILL_PREC_FP32_OP)
        bp.set_precond(F.FILL_PRECOND_BLOCK)
        plans.append(bp)
        ds.append(dev(np.stack([d for _, d, _ in lst])))
        seeds.append([s for _, _, s in lst])
    return F.Group(plans), plans, ds, seeds


def check(problems, oracle_fills, outs, tol):
    for (n, (P, lst)), o in zip(problems.items(), outs):
        x = o.cpu().numpy()
        for j, (mask, d, _) in enumerate(lst):
            m = mask != 0
            e = rel(x[j], oracle_fills[(n, j)], m)
            print(f"{n}^2 problem {j}: masked rel L2 {e:.2e}")
            assert e < tol, (n, j, e)
            assert np.array_equal(x[j][~m].view(np.uint64), d[~m].view(np.uint64))


def test_group_of_uneven_sizes_matches_oracle(F, problems, oracle_fills):
    g, plans, ds, seeds = make_group(F, problems)
    print("group call 1 (step by step)", flush=True)
    out1 = g.realize(ds, seeds, 1e-8)
    torch.cuda.synchronize()
    assert not g.last_graph()
    check(problems, oracle_fills, out1, 1e-5)
    for rep in range(2):
        print(f"group call {rep + 2} (one graph launch)", flush=True)
        out2 = g.realize(ds, seeds, 1e-8)
        torch.cuda.synchronize()
        assert g.last_graph()
        for pl in plans:
            for st in pl.stats():
                assert st["status"] == 0 and st["rel_resid"] <= 1e-8 and st["whole_graph"] == 1
        for a, b in zip(out1, out2):
            assert np.array_equal(a.cpu().numpy().view(np.uint64), b.cpu().numpy().view(np.uint64))
    g.close()


def test_group_continues_past_the_graph(F, problems, oracle_fills):
    g, plans, ds, seeds = make_group(F, problems)
    g.realize(ds, seeds, 1e-6)
    print("group call at a tighter tolerance than the counts", flush=True)
    out = g.realize(ds, seeds, 1e-10)
    torch.cuda.synchronize()
    for pl in plans:
        for st in pl.stats():
            assert st["status"] == 0 and st["rel_resid"] <= 1e-10
    check(problems, oracle_fills, out, 1e-5)
    g.close()


def test_group_errors(F, problems):
    n = 256
    P, lst = problems[n]
    bp = F.BatchPlan(n, n, np.stack([m for m, _, _ in lst]), P, F.FILL_PREC_FP32_OP)
    with pytest.raises(F.FillError) as e:
        F.fill_group_create([bp.handle, bp.handle], None)
    assert e.value.code == F.FILL_EINVAL
    with pytest.raises(F.FillError) as e:
        F.fill_group_create([], None)
    assert e.value.code == F.FILL_EINVAL
