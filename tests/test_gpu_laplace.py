"""GPU: the kernel-based Laplace relaxation (Sec. 6.1, 6.3) and the strips
started from it (Sec. 6.4), against the oracle.

* fill_laplace equals the oracle's sweeps to 1e-10 relative L2 on masked
  pixels (the same Jacobi sweeps; averaging does not amplify rounding);
* harmonic polynomial data around an interior hole is reproduced (1e-8);
* strips refined from the Laplace fill equal the oracle's to 1e-9.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle.laplace as OL
import oracle.strips as OS
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


@pytest.mark.parametrize("nx,ny,band,nk,iters", [(128, 128, (40, 40), 5, 40), (256, 128, (40, 44), 6, 25),
                                                 (128, 256, None, 4, 30)])
def test_laplace_matches_oracle(F, nx, ny, band, nk, iters):
    P = W.damped_power_law(nx, ny, 4.0, max(nx, ny) / 8, 1e-7)
    mask = W.band_holes_mask(nx, ny, band, 10, 2.0, 9.0, 23)
    d = W.observed_map(P, nx, ny, 6, mask)
    radii = OL.laplace_radii(nk, 1.5, 2.0)
    ref, _ = OL.laplace_fill(d, mask, radii, iters)
    plan = F.Plan(nx, ny, mask, P)
    x = host(plan.laplace(dev(d), nkernels=nk, r0=1.5, ratio=2.0, iters=iters))
    m = mask != 0
    assert rel(x, ref, m) < 1e-10
    assert np.array_equal(x[~m].view(np.uint64), d[~m].view(np.uint64))
    # repeated call with the same parameters reuses the kernel spectra and classes
    x2 = host(plan.laplace(dev(d), nkernels=nk, r0=1.5, ratio=2.0, iters=iters))
    assert np.array_equal(x2.view(np.uint64), x.view(np.uint64))


def test_laplace_harmonic_fixed_point(F):
    n, h = 128, 40
    mask = np.zeros((n, n), np.uint8)
    a = (n - h) // 2
    mask[a:a + h, a + 5:a + h - 3] = 1
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    y -= n / 2
    x -= n / 2
    f = 0.7 + 0.01 * x - 0.02 * y + 1e-3 * (x * x - y * y) + 2e-3 * x * y
    plan = F.Plan(n, n, mask, W.damped_power_law(n, n, 4.0, 16.0, 1e-7))
    got = host(plan.laplace(dev(np.where(mask != 0, 0.0, f)), nkernels=5, iters=600))
    m = mask != 0
    assert np.abs(got[m] - f[m]).max() <= 1e-8 * np.abs(f[m]).max()


def test_strips_from_laplace_match_oracle(F):
    n = 256
    P = W.damped_power_law(n, n, 4.0, n / 8, 1e-7)
    floor = 1e-7
    mask = W.band_holes_mask(n, n, W.band_rows(n, 0.2), 13, 2.0, 12.0, 2)
    d = W.observed_map(P, n, n, 0, mask)
    radii = OL.laplace_radii(6, 1.5, 2.0)
    start, _ = OL.laplace_fill(d, mask, radii, 30)
    betas, widths = [2000.0, 400.0, 40.0, 1.0], [25.0, 9.0, 4.0, 2.0]
    ref, _ = OS.strip_fill(d, mask, P - floor, floor, betas, widths, 20, start=start)
    plan = F.Plan(n, n, mask, P)
    s = F.Strips(n, n, mask, P - floor, floor, betas, widths, iters=20)
    x = plan.laplace(dev(d), nkernels=6, iters=30)
    x = host(s.refine(x))
    assert rel(x, ref, mask != 0) < 1e-9


def test_laplace_errors(F):
    n = 64
    mask = W.band_holes_mask(n, n, (28, 8), 2, 2.0, 3.0, 1)
    plan = F.Plan(n, n, mask, np.ones((n, n // 2 + 1)))
    d = dev(np.zeros((n, n)))
    for kw in (dict(nkernels=0), dict(nkernels=7), dict(r0=0.5), dict(ratio=1.0), dict(iters=0)):
        with pytest.raises(F.FillError):
            plan.laplace(d, **{**dict(nkernels=4, r0=1.5, ratio=2.0, iters=3), **kw})
