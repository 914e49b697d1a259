"""GPU: the block preconditioner (FILL_PRECOND_BLOCK) against the oracle.

* M^-1 applied on the GPU (FILL_OP_MINV) equals the oracle's block
  preconditioner element by element: a short band (no truncation), a tall
  band (truncated Toeplitz per kx), two band runs in one problem, holes
  across the periodic edges, a piece
  cut into cells, a fully masked row that is not a band, and the 256^2 / 512^2
  band + holes workloads; FP64 to 1e-9, FP32 to the bar below;
* the fill with it reaches the oracle's solution (1e-9 FP64 at rtol 1e-12,
  1e-5 mixed) on grids of several tiles with ragged masks, and the 2048^2
  workload meets its FP64 residual by the oracle;
* far fewer iterations than M^-1 = Px C Px;
* its CG coefficients equal the oracle's block PCG's over the first steps;
* graph replays are bitwise equal to direct launches; a new spectrum rebuilds
  it; a fully masked grid returns the unconstrained draw;
* a batched plan (own masks and spectra per problem) matches the oracle;
* a batched plan of identical problems (one shared set of factors and
  inverses) gives each problem exactly what a plan of its own gives, holds
  the set once, and one differing problem in it gets its own;
* errors: spectra not symmetric in ky, FILL_OP_MINV without it.

FP32 bar for M^-1: the band factors and block inverses are rounded to FP32
and the substitutions run in FP32, so the result carries a relative error of
about kappa(T_kx) * 2^-24 on the worst-conditioned frequencies; 2e-3 relative
L2 on the masked pixels covers the cases here with a margin (measured values
are printed).
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle.block_precond as B
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


def disk(mask, cy, cx, r):
    ny, nx = mask.shape
    y, x = np.mgrid[:ny, :nx]
    dy = (y - cy + ny // 2) % ny - ny // 2
    dx = (x - cx + nx // 2) % nx - nx // 2
    mask[dy * dy + dx * dx <= r * r] = 1


def case(name):
    if name == "short":
        ny, nx = 128, 32
        P = W.damped_power_law(nx, ny, 2.0, 5.0, 1e-6)
        m = np.zeros((ny, nx), np.uint8)
        m[10:17] = 1
        disk(m, 40, 16, 3)
        return m, P
    if name == "mix":
        ny, nx = 256, 128
        P = W.damped_power_law(nx, ny, 2.0, 12.0, 1e-6)
        m = np.zeros((ny, nx), np.uint8)
        m[90:141] = 1          # 51-row band (> 32: truncated)
        disk(m, 142, 10, 4)    # touches the band
        disk(m, 0, 0, 3)       # across the corner
        m[180:230, 50:100] = 1  # 2500 pixels: cut into cells
        m[5, :127] = 1         # a row that is masked but for one pixel
        return m, P
    if name == "two":
        # two band runs in one problem (a tall one and a short one) and a hole
        # between them: the second run's factor streams follow the first's
        ny, nx = 256, 64
        P = W.damped_power_law(nx, ny, 2.0, 10.0, 1e-6)
        m = np.zeros((ny, nx), np.uint8)
        m[20:60] = 1
        m[150:170] = 1
        disk(m, 100, 30, 5)
        return m, P
    p = W.make_problem("grid2048", n=int(name))
    return p.mask, p.P


def plan_block(F, mask, P, prec):
    ny, nx = mask.shape
    plan = F.Plan(nx, ny, mask, P, prec=prec)
    plan.set_precond(F.FILL_PRECOND_BLOCK)
    return plan


@pytest.mark.parametrize("name", ["short", "mix", "two", "256", "512"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 2e-3)])
def test_minv_matches_oracle(F, name, prec, tol):
    mask, P = case(name)
    M = B.BlockPrecond(mask, P, pivot_min=B.PIVOT_MIN if prec == 0 else B.PIVOT_MIN_F32, halo="auto")
    if name == "two":
        assert M.runs == [(20, 40), (150, 20)]
    rng = np.random.default_rng(11)
    r = np.where(mask != 0, rng.standard_normal(mask.shape), 0.0)
    ref = M.apply(r)
    plan = plan_block(F, mask, P, prec)
    info = plan.block_info()
    # the library's default halo is the oracle's choice (step 6 of its definition)
    assert info["halo_min"] == info["halo_max"] == M.halo
    assert info["blocks"] == len(M.blocks) and info["block_entries"] == B.block_entries(M.blocks)
    got = host(plan.apply(F.FILL_OP_MINV, dev(r)))
    m = mask != 0
    err = rel(got, ref, m)
    print(f"M^-1 {name} prec {prec}: rel err {err:.2e}")
    assert err < tol
    assert np.all(got[~m] == 0.0)


@pytest.mark.parametrize("halo", [0, 8, 12, 14])
def test_minv_fixed_halo_matches_oracle(F, halo):
    mask, P = case("mix")
    M = B.BlockPrecond(mask, P, halo=halo)
    r = np.where(mask != 0, np.random.default_rng(12).standard_normal(mask.shape), 0.0)
    plan = plan_block(F, mask, P, 0)
    plan.set_block_halo(halo)  # rebuilds the built preconditioner
    info = plan.block_info()
    assert info["halo_min"] == info["halo_max"] == halo and info["blocks"] == len(M.blocks)
    assert info["block_entries"] == B.block_entries(M.blocks)
    err = rel(host(plan.apply(F.FILL_OP_MINV, dev(r))), M.apply(r), mask != 0)
    print(f"M^-1 halo {halo}: rel err {err:.2e}")
    assert err < 1e-9
    for bad in (-2, 15):
        with pytest.raises(F.FillError):
            plan.set_block_halo(bad)
    assert plan.block_info() == info


@pytest.mark.parametrize("nx,ny,seed", [(256, 256, 71), (768, 512, 72), (1024, 128, 73), (384, 1536, 74)])
@pytest.mark.parametrize("prec,tol,rtol", [(0, 1e-9, 1e-12), (1, 1e-5, 1e-10)])
def test_fill_matches_oracle(F, nx, ny, seed, prec, tol, rtol):
    P = W.damped_power_law(nx, ny, 4.0, min(nx, ny) / 8, 1e-7)
    mask = W.band_holes_mask(nx, ny, W.band_rows(ny, 0.1), 15, 2.0, 9.0, seed)
    d = W.observed_map(P, nx, ny, seed + 1, mask)
    ref = OF.fill_realize(d, mask, P, 7, 1e-13)
    plan = plan_block(F, mask, P, prec)
    x = host(plan.realize(dev(d), 7, rtol))
    m = mask != 0
    assert plan.stats()["status"] == 0
    assert rel(x, ref.x_out, m) < tol
    assert np.array_equal(x[~m].view(np.uint64), d[~m].view(np.uint64))


@pytest.mark.parametrize("prec", [0, 1])
def test_far_fewer_iterations_than_cxx(F, prec):
    p = W.make_problem("grid2048", n=512)
    dd = dev(p.d_obs)
    it = {}
    for pc in (2, 3):
        plan = F.Plan(p.nx, p.ny, p.mask, p.P, prec=prec)
        plan.set_precond(pc)
        plan.realize(dd, p.seed, 1e-8)
        st = plan.stats()
        assert st["status"] == 0 and st["rel_resid"] <= 1e-8
        it[pc] = st["iters_inner"]
    print("iterations cxx / block:", it)
    assert it[3] * 4 <= it[2], it


def test_coefficients_match_oracle(F):
    p = W.make_problem("grid64")
    s = OF.unconstrained_realization(p.P, p.seed)
    v = OF.rhs(np.where(p.mask != 0, 0.0, p.d_obs - s), p.mask, p.P)
    _, info = B.pcg_block(v, p.mask, p.P, 1e-12)
    plan = plan_block(F, p.mask, p.P, 0)
    plan.set_lanczos(4096)
    plan.realize(dev(p.d_obs), p.seed, 1e-12)
    al, be = plan.lanczos()
    k = min(6, len(info.alphas))
    assert len(al) >= k
    assert np.abs(al[:k] - info.alphas[:k]).max() <= 1e-8 * np.abs(info.alphas[:k]).max()
    assert np.abs(be[:k - 1] - info.betas[:k - 1]).max() <= 1e-8 * np.abs(info.betas[:k - 1]).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_bitwise(F, prec):
    mask, P = case("256")
    d = W.observed_map(P, 256, 256, 5, mask)
    dd = dev(d)
    ref_plan = plan_block(F, mask, P, prec)
    ref_plan.set_graph(False)
    g_plan = plan_block(F, mask, P, prec)
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


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_2048_workload_residual(F, prec):
    p = W.make_problem("grid2048")
    plan = plan_block(F, p.mask, p.P, prec)
    x = host(plan.realize(dev(p.d_obs), p.seed, p.rtol))
    st = plan.stats()
    m = p.mask != 0
    s = OF.unconstrained_realization(p.P, p.seed)
    v = OF.rhs(np.where(m, 0.0, p.d_obs - s), p.mask, p.P)
    u = np.where(m, x - s, 0.0)
    res = np.linalg.norm(v - OF.apply_A(u, p.mask, p.P)) / np.linalg.norm(v)
    print("2048^2 block:", st)
    assert st["status"] == 0 and res < 1.5 * p.rtol
    assert np.array_equal(x[~m].view(np.uint64), p.d_obs[~m].view(np.uint64))


def test_new_spectrum_rebuilds(F):
    mask, P = case("256")
    d = W.observed_map(P, 256, 256, 9, mask)
    plan = plan_block(F, mask, P, 0)
    info = plan.block_info()
    plan.set_pk(P.copy())  # the same spectrum: a no-op
    assert plan.block_info() == info
    x = host(plan.realize(dev(d), 3, 1e-12))
    assert rel(x, OF.fill_realize(d, mask, P, 3, 1e-13).x_out, mask != 0) < 1e-9
    P2 = W.damped_power_law(256, 256, 1.0, 40.0, 1e-6)
    plan.set_pk(P2)
    x = host(plan.realize(dev(d), 3, 1e-12))
    ref = OF.fill_realize(d, mask, P2, 3, 1e-13)
    assert rel(x, ref.x_out, mask != 0) < 1e-9
    got = host(plan.apply(F.FILL_OP_MINV, dev(np.where(mask != 0, 1.0, 0.0))))
    want = B.BlockPrecond(mask, P2, halo="auto").apply(np.where(mask != 0, 1.0, 0.0))
    assert rel(got, want, mask != 0) < 1e-9


def test_all_masked_returns_unconstrained_draw(F):
    n = 128
    P = W.damped_power_law(n, n, 4.0, 16.0, 1e-7)
    mask = np.ones((n, n), np.uint8)
    plan = plan_block(F, mask, P, 0)
    d = np.zeros((n, n))
    x = host(plan.realize(dev(d), 4, 1e-10))
    s = host(plan.realize_unconstrained(4))
    assert rel(x, s) < 1e-9


@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 1e-5)])
def test_batch_matches_oracle(F, prec, tol):
    # three problems of one size, own masks (one with a band, one holes only,
    # one fully masked row set plus a large piece), per-problem spectra
    n = 256
    masks, Ps, ds = [], [], []
    for i in range(3):
        P = W.damped_power_law(n, n, 2.0 + i, n / (6 + 2 * i), 1e-7)
        if i == 0:
            m = W.band_holes_mask(n, n, W.band_rows(n, 0.12), 12, 2.0, 8.0, 90)
        elif i == 1:
            m = W.band_holes_mask(n, n, None, 20, 2.0, 8.0, 91)
        else:
            m = np.zeros((n, n), np.uint8)
            m[100:130] = 1
            m[180:230, 40:90] = 1
        masks.append(m)
        Ps.append(P)
        ds.append(W.observed_map(P, n, n, 95 + i, m))
    bp = F.BatchPlan(n, n, np.stack(masks), np.stack(Ps), prec=prec)
    bp.set_precond(F.FILL_PRECOND_BLOCK)
    xb = host(bp.realize(dev(np.stack(ds)), [4, 5, 6], 1e-12 if prec == 0 else 1e-10))
    for i in range(3):
        ref = OF.fill_realize(ds[i], masks[i], Ps[i], 4 + i, 1e-13)
        assert rel(xb[i], ref.x_out, masks[i] != 0) < tol, i
    st = bp.stats()
    assert all(s["status"] == 0 for s in st)
    assert max(s["iters_inner"] for s in st) < 60


@pytest.mark.parametrize("prec", [0, 1])
def test_identical_problems_share(F, prec):
    # problems 0, 1, 3 identical (mask and spectrum), problem 2 with its own
    # mask: the shared set must serve 0, 1, 3 exactly as their own plans do;
    # the default halos differ (8 and 14): each problem keeps its own
    n = 256
    P = W.damped_power_law(n, n, 3.0, n / 8, 1e-7)
    m0 = W.band_holes_mask(n, n, W.band_rows(n, 0.15), 14, 2.0, 8.0, 120)
    m2 = W.band_holes_mask(n, n, W.band_rows(n, 0.08), 9, 2.0, 8.0, 129)
    assert B.auto_halo(m0) == 8 and B.auto_halo(m2) == 14
    masks = np.stack([m0, m0, m2, m0])
    ds = [W.observed_map(P, n, n, 130 + i, masks[i]) for i in range(4)]
    seeds = [11, 12, 13, 14]
    rtol = 1e-12 if prec == 0 else 1e-10
    bp = F.BatchPlan(n, n, masks, P, prec=prec)
    bp.set_precond(F.FILL_PRECOND_BLOCK)
    xb = host(bp.realize(dev(np.stack(ds)), seeds, rtol))
    ib = bp.block_info()
    st = bp.stats()
    bp.close()
    infos = []
    for i in range(4):
        pl = F.Plan(n, n, masks[i], P, prec)
        pl.set_precond(F.FILL_PRECOND_BLOCK)
        xi = host(pl.realize(dev(ds[i]), seeds[i], rtol))
        infos.append(pl.block_info())
        sti = pl.stats()
        pl.close()
        assert st[i]["iters_inner"] == sti["iters_inner"], i
        assert np.array_equal(xb[i], xi), (i, float(np.max(np.abs(xb[i] - xi))))
    assert [v["halo_min"] for v in infos] == [v["halo_max"] for v in infos] == [8, 8, 14, 8]
    assert ib["halo_min"] == 8 and ib["halo_max"] == 14
    # logical sizes add up over the problems; the stored set counts once
    assert ib["block_entries"] == sum(v["block_entries"] for v in infos)
    assert ib["band_stream_values"] == sum(v["band_stream_values"] for v in infos)
    assert ib["bytes"] < infos[0]["bytes"] * 2 + infos[2]["bytes"]


def test_errors(F):
    mask, P = case("short")
    ny, nx = mask.shape
    Pa = P.copy()
    Pa[1, 3] *= 1.5  # P(kx, ky) != P(kx, -ky)
    plan = F.Plan(nx, ny, mask, Pa)
    with pytest.raises(Exception):
        plan.set_precond(F.FILL_PRECOND_BLOCK)
    plan2 = F.Plan(nx, ny, mask, P)
    with pytest.raises(Exception):
        plan2.apply(F.FILL_OP_MINV, dev(np.zeros((ny, nx))))
