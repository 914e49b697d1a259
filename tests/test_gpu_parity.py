"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle and pins.

Tolerances:
* integer work (Philox words) is bit-exact; observed pixels are bitwise
  copies of d_obs;
* FP64 operator applies: relative L2 <= 1e-12 (FFT rounding is ~1e-16 per
  pass times log2 N; the oracle's FFT rounds differently);
* FP32 operator applies: relative L2 <= 2e-5 for C^{1/2} / E and <= 1e-4 for
  C^-1 / A, whose 1/P weights amplify the FP32 rounding of the high-k modes
  by up to the dynamic range of P within the input's support;
* fill results on masked pixels: relative L2 <= 1e-9 for FP64 and <= 1e-5 for
  FP32 operators with FP64 refinement, both solved with tolerances tight
  enough that the iterative error is below these bars.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W
from pins import _p_of_k, band_direct, rel

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


def problem(nx, ny, band_frac=0.1, n_holes=10, rmin=2.0, rmax=6.0, mask_seed=3, damping=None, floor=1e-7):
    P = W.damped_power_law(nx, ny, 4.0, damping or max(nx, ny) / 8, floor)
    band = W.band_rows(ny, band_frac) if band_frac else None
    mask = W.band_holes_mask(nx, ny, band, n_holes, rmin, rmax, mask_seed)
    d = W.observed_map(P, nx, ny, seed=mask_seed + 100, mask=mask)
    return P, mask, d


# ---------------------------------------------------------------------------
# random generator and realization
# ---------------------------------------------------------------------------

def test_philox_words_bit_exact(F):
    for seed, stream, n in ((0, 0x52, 1000), (2 ** 64 - 1, 0x4F, 4097), (123456789, 7, 65536)):
        got = host(F.philox_words(seed, stream, n)).view(np.uint64).reshape(n, 4)
        j = np.arange(n, dtype=np.uint64)
        z = np.zeros_like(j)
        ref = np.stack(O.philox4x64_10(j, z, z, z, np.uint64(seed), np.uint64(stream)), axis=1)
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("nx,ny", [(64, 64), (256, 128), (16, 768), (768, 32), (2048, 16)])
def test_unconstrained_realization_matches_oracle(F, nx, ny):
    P, mask, _ = problem(nx, ny)
    plan = F.Plan(nx, ny, mask, P)
    for seed in (0, 1, 2 ** 40 + 5):
        s = host(plan.realize_unconstrained(seed))
        ref = O.unconstrained_realization(P, seed)
        assert rel(s, ref) < 1e-12


def test_realization_spectrum(F):
    n, S = 64, 200
    P = W.damped_power_law(n, n, 1.0, 10.0, 1e-4)
    plan = F.Plan(n, n, np.zeros((n, n), np.uint8), P)
    ratio = np.zeros(P.shape)
    for s in range(S):
        sk = np.fft.rfft2(host(plan.realize_unconstrained(s)))
        ratio += np.abs(sk) ** 2 / (n * n) / P
    ratio /= S
    sel = np.zeros(P.shape, bool)
    sel[:, 1:n // 2] = True
    kk = np.floor(W.kgrid(n, n)).astype(int)
    for b in np.unique(kk[sel]):
        c = sel & (kk == b)
        assert abs(ratio[c].mean() - 1) < 5 / np.sqrt(S * c.sum()), b


# ---------------------------------------------------------------------------
# operator applies
# ---------------------------------------------------------------------------

OPS = {0: ("cinv", -1.0, False), 1: ("chalf", 0.5, False), 2: ("A", -1.0, True), 3: ("E", 0.5, True)}


def oracle_op(op, v, mask, P):
    _, power, proj = OPS[op]
    if not proj:
        return O.circulant_apply(v, P, power)
    return O.apply_A(v, mask, P) if op == 2 else O.apply_E(v, mask, P)


@pytest.mark.parametrize("nx,ny", [(16, 16), (64, 32), (128, 512), (768, 768), (1024, 64), (4096, 16),
                                   (32, 4096), (2048, 2048), (96, 192), (384, 1536), (3072, 96), (192, 3072)])
@pytest.mark.parametrize("prec", [0, 1])
def test_operator_apply_matches_oracle(F, nx, ny, prec):
    P, mask, _ = problem(nx, ny, n_holes=max(1, nx * ny // 20000))
    plan = F.Plan(nx, ny, mask, P, prec)
    v = np.random.default_rng(nx * 7 + ny).standard_normal((ny, nx))
    x = dev(v)
    for op in OPS:
        got = host(plan.apply(op, x))
        ref = oracle_op(op, v, mask, P)
        tol = 1e-12 if prec == 0 else (1e-4 if OPS[op][1] < 0 else 2e-5)
        e = rel(got, ref)
        assert e < tol, (OPS[op][0], e)
        if OPS[op][2]:
            assert np.all(got[mask == 0] == 0.0)


def test_operator_symmetry_on_gpu(F):
    n = 256
    P, mask, _ = problem(n, n, n_holes=30)
    plan = F.Plan(n, n, mask, P)
    rng = np.random.default_rng(1)
    u, w = rng.standard_normal((2, n, n))
    for op in (2, 3):
        a = np.vdot(u, host(plan.apply(op, dev(w))))
        b = np.vdot(host(plan.apply(op, dev(u))), w)
        assert abs(a - b) <= 1e-12 * abs(a)


# ---------------------------------------------------------------------------
# the fill
# ---------------------------------------------------------------------------

def run_fill(F, P, mask, d, prec, seed, rtol, mean=False, allow_noconv=False):
    ny, nx = mask.shape
    plan = F.Plan(nx, ny, mask, P, prec)
    dd = dev(d)
    x = plan.mean(dd, rtol, allow_noconv=allow_noconv) if mean else plan.realize(dd, seed, rtol, allow_noconv=allow_noconv)
    return host(x), plan.stats(), plan


def test_fill_grid64_matches_dense_cholesky(F):
    p = W.make_problem("grid64")
    x, st, plan = run_fill(F, p.P, p.mask, p.d_obs, 0, p.seed, 1e-12, allow_noconv=True)
    m = p.mask != 0
    s = host(plan.realize_unconstrained(p.seed))
    t = np.where(m, 0.0, p.d_obs - s)
    ud = O.dense.conditional_mean_dense(t, p.mask, p.P)
    assert st["rel_resid"] < 1e-11
    assert rel(x - s, ud, m) < 1e-9
    assert np.array_equal(x[~m].view(np.uint64), p.d_obs[~m].view(np.uint64))


def test_fill_grid64_at_its_tolerance(F):
    p = W.make_problem("grid64")
    x, st, _ = run_fill(F, p.P, p.mask, p.d_obs, 0, p.seed, p.rtol)
    assert st["status"] == 0 and st["rel_resid"] <= p.rtol
    ref = O.fill_realize(p.d_obs, p.mask, p.P, p.seed, 1e-12)
    assert rel(x, ref.x_out, p.mask != 0) < 1e-7


@pytest.mark.parametrize("nx,ny,seed", [(256, 256, 1), (512, 256, 9), (768, 768, 4), (384, 192, 12), (96, 384, 13)])
def test_fill_fp64_matches_oracle(F, nx, ny, seed):
    P, mask, d = problem(nx, ny, n_holes=nx * ny // 6000)
    x, st, _ = run_fill(F, P, mask, d, 0, seed, 1e-12, allow_noconv=True)
    ref = O.fill_realize(d, mask, P, seed, 1e-12)
    m = mask != 0
    assert st["rel_resid"] < 2e-11
    assert rel(x, ref.x_out, m) < 1e-9
    assert np.array_equal(x[~m].view(np.uint64), d[~m].view(np.uint64))


@pytest.mark.parametrize("nx,ny,seed", [(256, 256, 1), (1024, 512, 3), (768, 768, 4), (1536, 384, 14)])
def test_fill_mixed_matches_oracle(F, nx, ny, seed):
    P, mask, d = problem(nx, ny, n_holes=nx * ny // 6000)
    x, st, _ = run_fill(F, P, mask, d, 1, seed, 1e-8)
    ref = O.fill_realize(d, mask, P, seed, 1e-12)
    m = mask != 0
    assert st["status"] == 0 and st["rel_resid"] <= 1e-8
    assert st["iters_outer"] >= 1
    assert rel(x, ref.x_out, m) < 1e-5
    assert np.array_equal(x[~m].view(np.uint64), d[~m].view(np.uint64))


def test_fill_mean_matches_oracle(F):
    P, mask, d = problem(512, 512, n_holes=40)
    x, st, _ = run_fill(F, P, mask, d, 0, 0, 1e-12, mean=True, allow_noconv=True)
    ref = O.fill_mean(d, mask, P, 1e-12)
    assert rel(x, ref.x_out, mask != 0) < 1e-9


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_band_mask_matches_direct_solve(F, prec):
    # 2048^2 with the damped spectrum of the 2048^2 workload, band mask only:
    # exact conditional mean by per-frequency direct solves.
    n = 2048
    P = W.damped_power_law(n, n, 4.0, 256.0, 1e-7)
    r0, h = W.band_rows(n, 0.10)
    mask = W.band_holes_mask(n, n, (r0, h), 0, 0, 0, 0)
    d = W.observed_map(P, n, n, seed=0, mask=mask)
    rtol = 1e-12 if prec == 0 else 1e-9
    x, st, _ = run_fill(F, P, mask, d, prec, 0, rtol, mean=True, allow_noconv=True)
    ref = band_direct(np.where(mask != 0, 0.0, d), r0, h, lambda k: _p_of_k(k, 4.0, 256.0, 1e-7))
    assert rel(x, ref, mask != 0) < (1e-9 if prec == 0 else 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_2048_workload_properties(F, prec):
    # The 2048^2 workload at its tolerance: the unconstrained draw equals the
    # oracle's, the oracle's FP64 residual of the GPU solution meets rtol, and
    # observed pixels are untouched.
    p = W.make_problem("grid2048")
    x, st, plan = run_fill(F, p.P, p.mask, p.d_obs, prec, p.seed, p.rtol)
    m = p.mask != 0
    s = host(plan.realize_unconstrained(p.seed))
    assert rel(s, O.unconstrained_realization(p.P, p.seed)) < 1e-12
    v = O.rhs(np.where(m, 0.0, p.d_obs - s), p.mask, p.P)
    u = np.where(m, x - s, 0.0)
    res = np.linalg.norm(v - O.apply_A(u, p.mask, p.P)) / np.linalg.norm(v)
    assert st["status"] == 0 and res < 1.5 * p.rtol
    assert np.array_equal(x[~m].view(np.uint64), p.d_obs[~m].view(np.uint64))


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_4096_wide_cut_properties(F, prec):
    # 4096^2, 30% band + 500 holes: the oracle's FP64 residual of the GPU
    # solution meets rtol; observed pixels untouched; finite everywhere.
    p = W.make_problem("grid4096")
    x, st, plan = run_fill(F, p.P, p.mask, p.d_obs, prec, p.seed, p.rtol)
    m = p.mask != 0
    s = host(plan.realize_unconstrained(p.seed))
    v = O.rhs(np.where(m, 0.0, p.d_obs - s), p.mask, p.P)
    u = np.where(m, x - s, 0.0)
    res = np.linalg.norm(v - O.apply_A(u, p.mask, p.P)) / np.linalg.norm(v)
    assert st["status"] == 0 and res < 1.5 * p.rtol
    assert np.array_equal(x[~m].view(np.uint64), p.d_obs[~m].view(np.uint64))
    assert np.all(np.isfinite(x))


# ---------------------------------------------------------------------------
# edge cases and errors
# ---------------------------------------------------------------------------

def test_no_masked_pixel_returns_data(F):
    P, _, d = problem(64, 64)
    x, st, _ = run_fill(F, P, np.zeros((64, 64), np.uint8), d, 0, 3, 1e-10)
    assert np.array_equal(x, d) and st["iters_inner"] == 0


def test_all_masked_returns_unconstrained_draw(F):
    P, _, _ = problem(64, 64)
    mask = np.ones((64, 64), np.uint8)
    x, st, plan = run_fill(F, P, mask, np.zeros((64, 64)), 1, 3, 1e-10)
    assert np.array_equal(x, host(plan.realize_unconstrained(3)))


def test_masked_inputs_are_ignored_and_runs_are_deterministic(F):
    P, mask, d = problem(256, 128, n_holes=20)
    dn = d.copy()
    dn[mask != 0] = np.nan
    a, _, _ = run_fill(F, P, mask, d, 1, 5, 1e-8)
    b, _, _ = run_fill(F, P, mask, dn, 1, 5, 1e-8)
    assert np.array_equal(a, b)


def test_rejected_spectrum_leaves_the_plan_unchanged(F):
    # an invalid spectrum is rejected every time it is offered, and the plan
    # keeps solving with the spectrum it had
    P, mask, d = problem(64, 64)
    plan = F.Plan(64, 64, mask, P)
    dd = dev(d)
    x0 = host(plan.realize(dd, 2, 1e-12))
    bad = P * 2.0
    bad[5, 7] = -1.0
    for _ in range(2):
        with pytest.raises(F.FillError) as e:
            plan.set_pk(bad)
        assert e.value.code == F.FILL_ENOTSPD
    x1 = host(plan.realize(dd, 2, 1e-12))
    assert np.array_equal(x0.view(np.uint64), x1.view(np.uint64))
    plan.set_pk(P * 2.0)  # a valid change still takes effect
    x2 = host(plan.realize(dd, 2, 1e-12))
    assert rel(x2, O.fill_realize(d, mask, P * 2.0, 2, 1e-13).x_out, mask != 0) < 1e-9


def test_error_paths(F):
    P, mask, d = problem(64, 64)
    bad = P.copy()
    bad[3, 4] = 0.0
    with pytest.raises(F.FillError) as e:
        F.Plan(64, 64, mask, bad)
    assert e.value.code == F.FILL_ENOTSPD
    plan = F.Plan(64, 64, mask, P)
    dd = dev(d)
    with pytest.raises(F.FillError) as e:
        plan.realize(dd, 0, 0.0)
    assert e.value.code == F.FILL_EINVAL
    with pytest.raises(F.FillError) as e:
        F.fill_realize(plan.handle, dd.data_ptr(), 0, dd.data_ptr(), 1e-8)
    assert e.value.code == F.FILL_EINVAL
    plan.set_max_iter(3)
    with pytest.raises(F.FillError) as e:
        plan.realize(dd, 0, 1e-12)
    assert e.value.code == F.FILL_ENOCONV
    st = plan.stats()
    assert st["iters_inner"] == 3 and st["status"] == F.FILL_ENOCONV
    x = plan.realize(dd, 0, 1e-12, allow_noconv=True)
    assert np.all(np.isfinite(host(x)))
