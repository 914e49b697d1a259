"""GPU: adjoint of the fill (gradients with respect to observed pixels and
band powers) against the oracle's adjoint and against central differences.

Bars: 1e-8 relative for the FP64 path; 1e-6 for FP32 operators with FP64
refinement (both solves refined to a tight true residual so that the solve
error stays below the bar).
"""

from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as AD
from pins import rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_0286_amd as F
    return F


def setup(n, nb=50, mseed=7, dseed=3, nholes=4):
    lnk = AD.band_nodes(n, nb)
    phi = AD.band_weights(n, n, lnk)
    kb = np.exp(lnk)
    theta = np.log(1.0 / (kb ** 2 + 4) * np.exp(-(kb / (n / 8)) ** 2) + 1e-7)
    mask = W.band_holes_mask(n, n, W.band_rows(n, 0.1), nholes, 2, 5, mseed)
    d = W.observed_map(AD.pk_from_bands(theta, phi), n, n, dseed, mask)
    wts = np.random.default_rng(mseed + 100).uniform(0, 1, (n, n))
    return lnk, phi, theta, mask, d, wts


def gpu_grad(F, n, lnk, theta, mask, d, wts, seed, prec, rtol):
    plan = F.Plan(n, n, mask, np.ones((n, n // 2 + 1)), prec)
    plan.set_bands(lnk, theta)
    dd = torch.from_numpy(d).cuda()
    x = plan.realize(dd, seed, rtol, allow_noconv=True)
    w = torch.from_numpy(wts).cuda()
    L = float(torch.sum(w * x * x))
    g = (2.0 * w * x).contiguous()
    gd, gth, glp = plan.adjoint(dd, seed, x, g, rtol, want_logP=True, allow_noconv=True)
    return L, gd.cpu().numpy(), gth, glp


@pytest.mark.parametrize("prec,rtol,tol", [(0, 1e-12, 1e-8), (1, 1e-11, 1e-6)])
def test_adjoint_matches_oracle(F, prec, rtol, tol):
    n = 64
    lnk, phi, theta, mask, d, wts = setup(n)
    L, gd, gth, glp = gpu_grad(F, n, lnk, theta, mask, d, wts, 9, prec, rtol)
    L0, gy0, gP0, gth0 = AD.adjoint_gradient(d, mask, theta, phi, 9, wts, 1e-13)
    assert abs(L - L0) < tol * abs(L0)
    assert rel(gth, gth0) < tol
    assert rel(gd, gy0) < tol
    assert rel(glp, gP0) < tol
    assert np.all(gd[mask != 0] == 0.0)


def test_adjoint_matches_gpu_central_differences(F):
    n = 128
    lnk, phi, theta, mask, d, wts = setup(n, nholes=12)
    # gradient under test: the mixed path; the finite differences come from
    # FP64 solves at 1e-12, whose error divided by 2h stays below the bar
    L, gd, gth, _ = gpu_grad(F, n, lnk, theta, mask, d, wts, 5, 1, 1e-11)
    plan = F.Plan(n, n, mask, np.ones((n, n // 2 + 1)), 0)
    w = torch.from_numpy(wts).cuda()

    def loss(th, dd):
        plan.set_bands(lnk, th)
        x = plan.realize(torch.from_numpy(dd).cuda(), 5, 1e-12, allow_noconv=True)
        return float(torch.sum(w * x * x))

    h = 1e-4
    scale = np.abs(gth).max()
    for b in range(len(theta)):  # every band power
        e = np.zeros_like(theta)
        e[b] = h
        fd = (loss(theta + e, d) - loss(theta - e, d)) / (2 * h)
        assert abs(fd - gth[b]) < 1e-6 * scale, (b, fd, gth[b])
    rng = np.random.default_rng(3)
    for _ in range(2):
        dirn = np.where(mask != 0, 0.0, rng.standard_normal(d.shape))
        fd = (loss(theta, d + h * dirn) - loss(theta, d - h * dirn)) / (2 * h)
        an = float(np.sum(gd * dirn))
        assert abs(fd - an) < 1e-6 * abs(an)


def test_batch_adjoint_and_autograd_function(F):
    n, nprob = 64, 3
    lnk = AD.band_nodes(n, 50)
    phi = AD.band_weights(n, n, lnk)
    kb = np.exp(lnk)
    theta = np.log(1.0 / (kb ** 2 + 4) * np.exp(-(kb / (n / 8)) ** 2) + 1e-7)
    masks, ds, wl = [], [], []
    for i in range(nprob):
        m = W.band_holes_mask(n, n, W.band_rows(n, 0.1), 3 + i, 2, 5, 20 + i)
        masks.append(m)
        ds.append(W.observed_map(AD.pk_from_bands(theta, phi), n, n, 30 + i, m))
        wl.append(np.random.default_rng(40 + i).uniform(0, 1, (n, n)))
    seeds = [5, 6, 7]
    bp = F.BatchPlan(n, n, np.stack(masks), np.ones((n, n // 2 + 1)), 0)
    FillFn = F.autograd_fill()
    dd = torch.from_numpy(np.stack(ds)).cuda().requires_grad_(True)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    x = FillFn.apply(dd, th, bp, seeds, lnk, 1e-11, 1e-11)
    L = torch.sum(torch.from_numpy(np.stack(wl)).cuda() * x * x)
    L.backward()
    gth_ref = np.zeros_like(theta)
    for i in range(nprob):
        L0, gy0, _, gth0 = AD.adjoint_gradient(ds[i], masks[i], theta, phi, seeds[i], wl[i], 1e-13)
        gth_ref += gth0
        assert rel(dd.grad[i].cpu().numpy(), gy0) < 1e-8, i
    assert rel(th.grad.numpy(), gth_ref) < 1e-8


@pytest.mark.parametrize("pc,prec,tol", [(2, 0, 1e-8), (2, 1, 1e-6), (0, 1, 1e-6)])
def test_adjoint_with_other_preconditioners(F, pc, prec, tol):
    # the adjoint solve uses the plan's preconditioner (Px C Px or none):
    # same gradient as the oracle's
    n = 64
    lnk, phi, theta, mask, d, wts = setup(n)
    plan = F.Plan(n, n, mask, np.ones((n, n // 2 + 1)), prec)
    plan.set_precond(pc)
    plan.set_bands(lnk, theta)
    dd = torch.from_numpy(d).cuda()
    rtol = 1e-12 if prec == 0 else 1e-11
    x = plan.realize(dd, 9, rtol, allow_noconv=True)
    g = (2.0 * torch.from_numpy(wts).cuda() * x).contiguous()
    gd, gth, _ = plan.adjoint(dd, 9, x, g, rtol, allow_noconv=True)
    _, gy0, _, gth0 = AD.adjoint_gradient(d, mask, theta, phi, 9, wts, 1e-13)
    assert rel(gth, gth0) < tol
    assert rel(gd.cpu().numpy(), gy0) < tol


def test_autograd_backward_uses_its_forwards_band_powers(F):
    # two forwards on one shared plan at different band powers, then backward
    # through the first: the gradient is the oracle's at the first theta
    n, nprob = 64, 1
    lnk, phi, theta, mask, d, wts = setup(n)
    theta2 = theta + 0.3
    bp = F.BatchPlan(n, n, mask[None], np.ones((n, n // 2 + 1)), 0)
    FillFn = F.autograd_fill()
    w = torch.from_numpy(wts[None]).cuda()
    dd = torch.from_numpy(d[None].copy()).cuda().requires_grad_(True)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    x = FillFn.apply(dd, th, bp, [9], lnk, 1e-11, 1e-11)
    L = torch.sum(w * x * x)
    th2 = torch.tensor(theta2, dtype=torch.float64, requires_grad=True)
    x2 = FillFn.apply(dd.detach(), th2, bp, [9], lnk, 1e-11, 1e-11)
    assert not torch.equal(x, x2)
    L.backward()
    _, gy0, _, gth0 = AD.adjoint_gradient(d, mask, theta, phi, 9, wts, 1e-13)
    assert rel(th.grad.numpy(), gth0) < 1e-8
    assert rel(dd.grad[0].cpu().numpy(), gy0) < 1e-8


def test_autograd_backward_raises_on_nonconvergence(F):
    n = 64
    lnk, phi, theta, mask, d, wts = setup(n)
    bp = F.BatchPlan(n, n, mask[None], np.ones((n, n // 2 + 1)), 0)
    FillFn = F.autograd_fill()
    dd = torch.from_numpy(d[None].copy()).cuda()
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    x = FillFn.apply(dd, th, bp, [9], lnk, 1e-10, 1e-10)
    bp.set_max_iter(2)  # the adjoint solve cannot reach 1e-10 in two iterations
    with pytest.raises(F.FillError) as e:
        torch.sum(x * x).backward()
    assert e.value.code == F.FILL_ENOCONV


@pytest.fixture(scope="module")
def grad1024():
    # the differentiation workload's grid: 1024^2, 10% band + 100 holes
    # r~U(2,10), 50 band powers; the oracle's adjoint with Px C Px PCG to 1e-12
    # for both of its solves
    n = 1024
    lnk = AD.band_nodes(n, 50)
    phi = AD.band_weights(n, n, lnk)
    kb = np.exp(lnk)
    theta = np.log(1.0 / (kb ** 2 + 4) * np.exp(-(kb / (n / 8)) ** 2) + 1e-7)
    mask = W.band_holes_mask(n, n, W.band_rows(n, 0.1), 100, 2.0, 10.0, 500)
    d = W.observed_map(AD.pk_from_bands(theta, phi), n, n, 600, mask)
    wts = np.random.default_rng(7).uniform(0, 1, (n, n))
    print("oracle adjoint at 1024^2", flush=True)
    ref = AD.adjoint_gradient(d, mask, theta, phi, 1, wts, 1e-12, solver="cxx")
    return n, lnk, theta, mask, d, wts, ref


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,rtol,tol", [(0, 1e-12, 1e-8), (1, 1e-10, 1e-6)])
def test_adjoint_at_1024_matches_oracle(F, grad1024, prec, rtol, tol):
    n, lnk, theta, mask, d, wts, (L0, gy0, gP0, gth0) = grad1024
    plan = F.Plan(n, n, mask, np.ones((n, n // 2 + 1)), prec)
    plan.set_precond(F.FILL_PRECOND_CXX)
    plan.set_bands(lnk, theta)
    dd = torch.from_numpy(d).cuda()
    x = plan.realize(dd, 1, rtol, allow_noconv=True)
    st = plan.stats()
    L = float(torch.sum(torch.from_numpy(wts).cuda() * x * x))
    g = (2.0 * torch.from_numpy(wts).cuda() * x).contiguous()
    gd, gth, glp = plan.adjoint(dd, 1, x, g, rtol, want_logP=True, allow_noconv=True)
    sa = plan.stats()
    print(f"prec {prec}: forward {st['iters_inner']} / {st['iters_outer']} rel resid {st['rel_resid']:.2e}; "
          f"adjoint status {sa['status']} rel resid {sa['rel_resid']:.2e}")
    print(f"  L rel {abs(L - L0) / abs(L0):.2e}, theta {rel(gth, gth0):.2e}, "
          f"y {rel(gd.cpu().numpy(), gy0):.2e}, lnP {rel(glp, gP0):.2e}")
    assert abs(L - L0) < tol * abs(L0)
    assert rel(gth, gth0) < tol
    assert rel(gd.cpu().numpy(), gy0) < tol
    assert rel(glp, gP0) < tol
