"""GPU: fill_realize_unconstrained_noalloc, the entry point that allocates
nothing (its spectrum scratch is a file-scope device array of the library),
called through the C ABI against fill_realize_unconstrained, which runs the
same kernels on the plan's own workspace: the draws must be equal bit for bit
(same kernels, same arithmetic, same order).  Two calls in a row, the second
on a smaller grid, then the size limit.
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


def test_noalloc_draw_equals_allocating_entry_point(F):
    for n, seed in ((1024, 11), (256, 12)):
        P = W.damped_power_law(n, n, 4.0, n / 8, 1e-7)
        mask = W.band_holes_mask(n, n, W.band_rows(n, 0.1), 20, 2.0, 8.0, 5)
        plan = F.Plan(n, n, mask, P)
        ref = plan.realize_unconstrained(seed)
        torch.cuda.synchronize()
        got = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        print(f"noalloc draw {n}x{n} seed {seed}", flush=True)
        F.fill_realize_unconstrained_noalloc(plan.handle, seed, got.data_ptr())
        torch.cuda.synchronize()
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), n
        plan.close()


def test_noalloc_rejects_grids_beyond_its_scratch(F):
    n = 4096  # (n/2) n 16 bytes = 128 MiB > 64 MiB
    plan = F.Plan(n, n, np.zeros((n, n), np.uint8), np.ones((n, n // 2 + 1)))
    out = torch.empty((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(F.FillError) as e:
        F.fill_realize_unconstrained_noalloc(plan.handle, 1, out.data_ptr())
    assert e.value.code == F.FILL_EINVAL
    assert "64 MiB" in str(e.value) or "67108864" in str(e.value)
    plan.close()
