"""GPU: the noise-boosted strip refinement (Sec. 6.2, 6.4) against the oracle.

* strip masks from the GPU subdivision equal the oracle's bit for bit
  (both count observed pixels in the periodic disk exactly);
* the refined fill (a fixed number of CG iterations per strip, FP64) equals
  the oracle's to 1e-9 relative L2 on masked pixels: the same iterates up to
  rounding; observed pixels are bitwise copies of d_obs.
"""

from __future__ import annotations

import numpy as np
import pytest

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


@pytest.mark.parametrize("nx,ny,band,widths", [(64, 64, (28, 8), (20.0, 8.0, 4.0, 2.0)),
                                               (256, 128, (50, 30), (40.5, 12.0, 5.0, 1.5)),
                                               (128, 256, None, (30.0, 6.3, 2.0))])
def test_strip_masks_and_fill_match_oracle(F, nx, ny, band, widths):
    P = W.damped_power_law(nx, ny, 4.0, max(nx, ny) / 8, 1e-5)
    floor = 1e-5
    mask = W.band_holes_mask(nx, ny, band, 12, 2.0, 9.0, 17)  # holes may cross the periodic edges
    d = W.observed_map(P, nx, ny, 4, mask)
    betas = [2000.0, 400.0, 40.0, 1.0][:len(widths)]
    s = F.Strips(nx, ny, mask, P - floor, floor, betas, widths, iters=20)
    ref, ref_strips = OS.strip_fill(d, mask, P - floor, floor, betas, list(widths), 20)
    for i, rs in enumerate(ref_strips):
        assert np.array_equal(s.mask(i), rs), i
    x = host(s.mean(dev(d)))
    m = mask != 0
    assert rel(x, ref, m) < 1e-9
    assert np.array_equal(x[~m].view(np.uint64), d[~m].view(np.uint64))


def test_strip_condition_numbers(F):
    # the Lanczos record of each strip's CG: boosted strips are well conditioned
    n = 256
    P = W.damped_power_law(n, n, 4.0, n / 8, 1e-7)
    floor = 1e-7
    mask = W.band_holes_mask(n, n, W.band_rows(n, 0.1), 13, 2.0, 12.0, 2)
    d = W.observed_map(P, n, n, 0, mask)
    s = F.Strips(n, n, mask, P - floor, floor, [2000.0, 400.0, 40.0, 1.0], [25.0, 9.0, 4.0, 2.0], iters=20)
    plans = [s.plan(i) for i in range(4)]
    for h in plans:
        F.fill_plan_set_lanczos(h, 64)
    s.mean(dev(d))
    torch.cuda.synchronize()
    kappa = []
    for h in plans:
        lo, hi, k = F.fill_lanczos_extremes(h, 0)
        assert k == 20 and 0 < lo <= hi
        kappa.append(hi / lo)
    assert kappa[0] < kappa[-1]
