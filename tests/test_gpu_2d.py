"""GPU parity of the 2D HIP path against the FP64 oracle (through the C ABI).

Stage tests feed both sides the same inputs.  The elliptic solves are
iterative on both sides: they agree to about cond(A) * tol, so the GPU solves
to a tolerance tight enough for the FP64 bar (relative L2 <= 1e-10) and the
FP32 + FP64-refinement bar (<= 1e-6).  At the full 2048 x 2048 size the
predictor and the mask are compared cell by cell and the solve is checked by
the oracle's own residual of the GPU pressure."""
import numpy as np
import pytest

import oracle as O
import swe_inputs as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17025_amd import swe_nh
    return swe_nh


def dt_(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def rel(g, r):
    g = g.detach().cpu().numpy() if hasattr(g, "detach") else np.asarray(g)
    return np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)


def case(nx=70, ny=37, seed=3):
    return S.random_case_2d(nx, ny, seed=seed, dx=0.5, dy=0.4)


def test_predictor_stage_parity(B):
    c = case()
    ctx = B.context_2d(c, crit=S.CRIT_GLOBAL, tol=1e-12, max_iter=2000)
    out = [torch.empty((c.ny, c.nx), dtype=torch.float64, device=DEV) for _ in range(4)]
    t0, dt = 0.13, 0.02
    ctx.predict(dt_(c.h), dt_(c.hu), dt_(c.hv), dt_(c.hw), t0, dt, *out)
    assert ctx.sync_stats()["status"] == 0
    ref = O.predict_2d(c.ds, c.dx, c.dy, c.body, O.phys_struct(), t0, dt, c.h, c.hu, c.hv, c.hw)
    for g, r in zip(out, ref):
        assert rel(g, r) <= 1e-13


def _safe_knh(ind, k):
    while np.min(np.abs(ind - k)) <= 1e-9 * k:
        k *= 1.0 + 1e-6
    return k


@pytest.mark.parametrize("crit", range(8))
@pytest.mark.parametrize("e", [0, 1, 3])
def test_mask_stage_bit_exact(B, crit, e):
    c = case(seed=5)
    t1 = 0.4
    ind = O.indicator_2d(c.ds, c.dx, c.dy, c.body, O.phys_struct(crit=min(crit, 5)), t1, c.h, c.hu,
                         c.hv, c.hw)
    k = float(np.percentile(ind, 80)) if crit < 6 else 1e-3
    if crit < 6:
        k = _safe_knh(ind, k)
    ctx = B.context_2d(c, crit=crit, k_nh=k, enlarge=e, tol=1e-10, max_iter=100)
    m = torch.zeros((c.ny, c.nx), dtype=torch.uint8, device=DEV)
    na = ctx.mask(dt_(c.h), dt_(c.hu), dt_(c.hv), dt_(c.hw), t1, 0, m)
    ref, cnt = O.mask_2d(c.ds, c.dx, c.dy, c.body, O.phys_struct(crit=crit, k_nh=k, enlarge=e), t1,
                         c.h, c.hu, c.hv, c.hw)
    assert np.array_equal(m.cpu().numpy(), ref)
    assert na == cnt


def _mask(c, seed):
    rng = np.random.default_rng(seed)
    m = (rng.random((c.ny, c.nx)) < 0.2).astype(np.uint8)
    m[5:30, 10:60] = 1
    m[0:4, 0:6] = 1   # a patch at the corner walls
    m[20, :] = 1      # a row spanning every tile column
    return m


@pytest.mark.parametrize("precision,tol,bar", [(0, 1e-13, 1e-10), (1, 1e-10, 1e-6)])
def test_pressure_and_projection_stage_parity(B, precision, tol, bar):
    c = case(seed=7)
    m = _mask(c, 1)
    t0, dt = 0.2, 0.01
    ctx = B.context_2d(c, crit=S.CRIT_ETA_D, precision=precision, tol=tol, max_iter=20000, warm=0)
    p = torch.full((c.ny, c.nx), 3.0, dtype=torch.float64, device=DEV)
    args = (dt_(c.h), dt_(c.hu), dt_(c.hv), dt_(c.hw))
    it, rr = ctx.solve_pressure(*args, torch.tensor(m, device=DEV), t0, dt, p)
    st = ctx.sync_stats()
    assert st["status"] == 0, st
    assert rr <= tol and it > 0
    ph = O.phys_struct()
    cell, xf, yf = O.nh_coeffs_2d(c.ds, c.dx, c.dy, c.body, ph, t0 + dt, dt, c.h, c.hu, c.hv, c.hw)
    rhs = O.nh_rhs_2d(cell, xf, yf, m)
    pref, _, _ = O.cg_2d(cell, xf, yf, m, rhs, tol=1e-14)
    assert rel(p, pref) <= bar
    assert np.all(p.cpu().numpy()[m == 0] == 0.0)
    mref, nref, kref = O.nh_correct_2d(cell, xf, yf, dt, 1000.0, c.hu, c.hv, c.hw, m, pref)
    outs = [torch.empty_like(args[0]) for _ in range(3)]
    ctx.correct(*args, torch.tensor(m, device=DEV), dt_(pref), t0, dt, *outs)
    assert ctx.sync_stats()["status"] == 0
    assert rel(outs[0], mref) <= 1e-12
    assert rel(outs[1], nref) <= 1e-12
    assert rel(outs[2] - args[3], kref - c.hw) <= 1e-11


def run2d(B, c, nsteps, **kw):
    ctx = B.context_2d(c, **kw)
    ctx.set_time(c.t0)
    h, hu, hv, hw = dt_(c.h), dt_(c.hu), dt_(c.hv), dt_(c.hw)
    p = torch.zeros_like(h)
    m = torch.zeros((c.ny, c.nx), dtype=torch.uint8, device=DEV)
    ctx.step(h, hu, hv, hw, p, m, nsteps=nsteps)
    return ctx, ctx.sync_stats(), h, hu, hv, hw, p, m


@pytest.mark.parametrize("crit", [S.CRIT_GLOBAL, S.CRIT_ETA_D, S.CRIT_NONE])
@pytest.mark.parametrize("precision", [0, 1])
def test_steps_parity(B, crit, precision):
    c = case(nx=66, ny=50, seed=11)
    tol = 1e-13 if precision == 0 else 1e-11
    kw = dict(crit=crit, k_nh=4e-3, enlarge=1, cfl=0.4, precision=precision, tol=tol,
              max_iter=20000, warm=1)
    ctx, st, h, hu, hv, hw, p, m = run2d(B, c, 8, **kw)
    assert st["status"] == 0, st
    ref = O.Sim2D(c, O.phys_struct(crit=crit, k_nh=4e-3, enlarge=1, tol=1e-14), cfl=0.4).step(8)
    assert np.array_equal(m.cpu().numpy(), ref.mask)
    assert st["n_active"] == ref.last_active
    bar = 1e-10 if precision == 0 else 1e-6
    for g, r in ((h - dt_(c.ds), ref.h - c.ds), (hu, ref.hu), (hv, ref.hv), (hw, ref.hw)):
        assert rel(g, r) <= bar
    if crit != S.CRIT_NONE:
        assert rel(p, ref.p) <= bar


def test_shelf_reduced_fp32_refinement(B):
    """the 2D shelf with a moving mound, reduced to 256 x 256 (same dx, depth
    statistics and mound), adaptive |eta/d|, FP32 PCG + FP64 refinement"""
    c = S.shelf_case_2d(nx=256, ny=256, x0=60.0, y0=128.0, amp=3.0, width=60.0 / 4)
    kw = dict(crit=S.CRIT_ETA_D, k_nh=1e-3, enlarge=1, cfl=0.5, precision=1, tol=1e-10,
              max_iter=20000, warm=1)
    ctx, st, h, hu, hv, hw, p, m = run2d(B, c, 20, **kw)
    assert st["status"] == 0, st
    ref = O.Sim2D(c, O.phys_struct(crit=S.CRIT_ETA_D, k_nh=1e-3, enlarge=1, tol=1e-13),
                  cfl=0.5).step(20)
    assert np.array_equal(m.cpu().numpy(), ref.mask) and ref.last_active > 0
    for g, r in ((h - dt_(c.ds), ref.h - c.ds), (hu, ref.hu), (hv, ref.hv), (hw, ref.hw), (p, ref.p)):
        assert rel(g, r) <= 1e-6


def test_full_size_shelf_properties(B):
    """2048 x 2048 shelf, in the benchmark's launch configuration: predictor
    and mask cell by cell against the oracle, the pressure through the
    oracle's residual, mass conservation"""
    c = S.shelf_case_2d()
    kw = dict(crit=S.CRIT_ETA_D, k_nh=1e-3, enlarge=1, cfl=0.5, precision=1, tol=1e-10,
              max_iter=20000, warm=1)
    ctx = B.context_2d(c, **kw)
    ctx.set_time(c.t0)
    h, hu, hv, hw = dt_(c.h), dt_(c.hu), dt_(c.hv), dt_(c.hw)
    p = torch.zeros_like(h)
    m = torch.zeros((c.ny, c.nx), dtype=torch.uint8, device=DEV)
    ctx.step(h, hu, hv, hw, p, m, nsteps=30)
    st = ctx.sync_stats()
    assert st["status"] == 0, st
    t = float(ctx.get_time()[0])
    # one more step driven stage by stage from the same state
    hs, hus, hvs, hws = (a.cpu().numpy() for a in (h, hu, hv, hw))
    mass0 = hs.sum()
    dtv = 0.5 / O.max_rate_2d(hs, hus, hvs, c.dx, c.dy)
    outs = [torch.empty_like(h) for _ in range(4)]
    ctx.predict(h, hu, hv, hw, t, dtv, *outs)
    ref = O.predict_2d(c.ds, c.dx, c.dy, c.body, O.phys_struct(), t, dtv, hs, hus, hvs, hws)
    for g, r in zip(outs, ref):
        assert rel(g, r) <= 1e-13
    ht, mt, nt, kt = ref
    ph = O.phys_struct(crit=S.CRIT_ETA_D, k_nh=1e-3, enlarge=1)
    mref, cnt = O.mask_2d(c.ds, c.dx, c.dy, c.body, ph, t + dtv, ht, mt, nt, kt)
    mg = torch.zeros_like(m)
    na = ctx.mask(*[dt_(a) for a in ref], t + dtv, 0, mg)
    assert na == cnt > 0 and np.array_equal(mg.cpu().numpy(), mref)
    pg = torch.zeros_like(h)
    it, rr = ctx.solve_pressure(*[dt_(a) for a in ref], mg, t, dtv, pg)
    assert rr <= 1e-10
    cell, xf, yf = O.nh_coeffs_2d(c.ds, c.dx, c.dy, c.body, ph, t + dtv, dtv, ht, mt, nt, kt)
    rhs = O.nh_rhs_2d(cell, xf, yf, mref)
    r = rhs - O.nh_apply_2d(cell, xf, yf, mref, pg.cpu().numpy())
    assert np.linalg.norm(r[mref == 1]) <= 1.01e-10 * np.linalg.norm(rhs[mref == 1])
    # the projection of the full-size state with that pressure, cell by cell
    outs = [torch.empty_like(h) for _ in range(3)]
    ctx.correct(*[dt_(a) for a in ref], mg, pg, t, dtv, *outs)
    assert ctx.sync_stats()["status"] == 0
    mc, nc, kc = O.nh_correct_2d(cell, xf, yf, dtv, 1000.0, mt, nt, kt, mref, pg.cpu().numpy())
    assert rel(outs[0], mc) <= 1e-12 and rel(outs[1], nc) <= 1e-12
    assert rel(outs[2] - dt_(kt), kc - kt) <= 1e-11
    assert abs(hs.sum() - c.h.sum()) <= 1e-12 * c.h.sum()
    assert abs(mass0 - c.h.sum()) <= 1e-12 * c.h.sum()


def test_step_with_device_time_2d(B):
    """swe_nh_step_t in 2D: the bits of swe_nh_step and the time after it"""
    c = case(nx=66, ny=50, seed=11)
    kw = dict(crit=S.CRIT_ETA_D, k_nh=4e-3, enlarge=1, cfl=0.4, precision=0, tol=1e-12,
              max_iter=5000, warm=1)
    ctx, st, h, hu, hv, hw, p, m = run2d(B, c, 3, **kw)
    ctx2 = B.context_2d(c, **kw)
    h2, hu2, hv2, hw2 = dt_(c.h), dt_(c.hu), dt_(c.hv), dt_(c.hw)
    p2 = torch.zeros_like(h2)
    t_dev = torch.tensor([c.t0], dtype=torch.float64, device=DEV)
    for _ in range(3):
        st2 = ctx2.step_t(h2, hu2, hv2, hw2, p2, t_dev)
        assert st2["status"] == 0
    for x, y in ((h, h2), (hu, hu2), (hv, hv2), (hw, hw2), (p, p2)):
        assert torch.equal(x, y)
    assert float(t_dev.item()) == float(ctx.get_time()[0]) > c.t0


def test_deterministic_2d(B):
    c = case(nx=80, ny=64, seed=2)
    kw = dict(crit=S.CRIT_ETA_D, k_nh=4e-3, cfl=0.4, precision=1, tol=1e-10, max_iter=5000)
    a = run2d(B, c, 5, **kw)
    b = run2d(B, c, 5, **kw)
    for x, y in zip(a[2:], b[2:]):
        assert torch.equal(x, y)


@pytest.mark.parametrize("precision", [0, 1])
def test_many_tiles_per_solver_block(B, precision):
    """global extension on 1536 x 510 cells (1536 tiles, more than the
    solver's blocks): every block of the persistent solver walks several
    tiles (the Chronopoulos-Gear form with a neighbour-tile sync).  The odd
    extent after one halving keeps the grid off the multigrid solver."""
    c = S.random_case_2d(1536, 510, seed=41, dx=1.0, dy=1.0, h0=10.0)
    tol = 1e-13 if precision == 0 else 1e-11
    kw = dict(crit=S.CRIT_GLOBAL, cfl=0.4, precision=precision, tol=tol, max_iter=5000, warm=1)
    ctx, st, h, hu, hv, hw, p, m = run2d(B, c, 1, **kw)
    assert st["status"] == 0, st
    ref = O.Sim2D(c, O.phys_struct(crit=S.CRIT_GLOBAL, tol=1e-14), cfl=0.4).step(1)
    bar = 1e-10 if precision == 0 else 1e-6
    for g, r in ((h - dt_(c.ds), ref.h - c.ds), (hu, ref.hu), (hv, ref.hv), (hw, ref.hw), (p, ref.p)):
        assert rel(g, r) <= bar


@pytest.mark.parametrize("nx,ny", [(256, 254), (288, 254), (100, 41)])
@pytest.mark.parametrize("precision", [0, 1])
def test_solver_around_the_coarse_space_limit(B, nx, ny, precision):
    """global extension with 128 active tiles (the most the solver's coarse
    space takes), 144 (the pipelined solver without it) and a few ragged
    tiles: same results as the oracle (grids that do not halve evenly to
    1024 cells, so the tile solver runs, not the multigrid one)"""
    c = S.random_case_2d(nx, ny, seed=43, dx=1.0, dy=1.0, h0=10.0)
    tol = 1e-13 if precision == 0 else 1e-11
    kw = dict(crit=S.CRIT_GLOBAL, cfl=0.4, precision=precision, tol=tol, max_iter=5000, warm=1)
    ctx, st, h, hu, hv, hw, p, m = run2d(B, c, 2, **kw)
    assert st["status"] == 0, st
    ref = O.Sim2D(c, O.phys_struct(crit=S.CRIT_GLOBAL, tol=1e-14), cfl=0.4).step(2)
    bar = 1e-10 if precision == 0 else 1e-6
    for g, r in ((h - dt_(c.ds), ref.h - c.ds), (hu, ref.hu), (hv, ref.hv), (hw, ref.hw), (p, ref.p)):
        assert rel(g, r) <= bar


def test_iteration_total_accumulates(B):
    """stats.iters_total sums the PCG iterations of every solve since init
    (what the benchmark divides by the steps of one multi-step call)"""
    c = case(nx=80, ny=64, seed=5)
    kw = dict(crit=S.CRIT_ETA_D, k_nh=4e-3, cfl=0.4, precision=1, tol=1e-10, max_iter=5000)
    ctx = B.context_2d(c, **kw)
    ctx.set_time(c.t0)
    h, hu, hv, hw = dt_(c.h), dt_(c.hu), dt_(c.hv), dt_(c.hw)
    p = torch.zeros_like(h)
    assert ctx.sync_stats()["iters_total"] == 0
    per_step = []
    for _ in range(4):
        ctx.step(h, hu, hv, hw, p)
        st = ctx.sync_stats()
        assert st["status"] == 0, st
        per_step.append(st["iters"])
    assert st["iters_total"] == sum(per_step) and sum(per_step) > 0


@pytest.mark.parametrize("nx,ny", [(200, 80), (256, 192), (320, 288), (512, 512)])
@pytest.mark.parametrize("precision", [0, 1])
def test_global_multigrid_steps(B, nx, ny, precision):
    """global extension on grids that halve evenly down to at most 4096
    cells (1 to 3 coarsenings; tiles of the smoothing kernels ragged at
    200 x 80 and 320 x 288): the CG with the multigrid preconditioner gives
    the oracle's steps, in a few dozen iterations"""
    c = S.random_case_2d(nx, ny, seed=47, dx=1.0, dy=1.0, h0=10.0)
    tol = 1e-13 if precision == 0 else 1e-11
    kw = dict(crit=S.CRIT_GLOBAL, cfl=0.4, precision=precision, tol=tol, max_iter=5000, warm=1)
    ctx, st, h, hu, hv, hw, p, m = run2d(B, c, 2, **kw)
    print("multigrid CG iterations of the last step", st["iters"])
    assert st["status"] == 0, st
    assert 0 < st["iters"] <= 64 and st["rel_res"] <= tol, st
    ref = O.Sim2D(c, O.phys_struct(crit=S.CRIT_GLOBAL, tol=1e-14), cfl=0.4).step(2)
    bar = 1e-10 if precision == 0 else 1e-6
    for g, r in ((h - dt_(c.ds), ref.h - c.ds), (hu, ref.hu), (hv, ref.hv), (hw, ref.hw), (p, ref.p)):
        assert rel(g, r) <= bar


def test_global_multigrid_solve_stage(B):
    """the multigrid solve through the pressure stage on a full mask: the
    oracle's CG pressure to 1e-10, zero guess and a warm guess"""
    c = case(nx=192, ny=128, seed=9)
    m = np.ones((c.ny, c.nx), np.uint8)
    t0, dt = 0.2, 0.01
    ph = O.phys_struct()
    cell, xf, yf = O.nh_coeffs_2d(c.ds, c.dx, c.dy, c.body, ph, t0 + dt, dt, c.h, c.hu, c.hv, c.hw)
    rhs = O.nh_rhs_2d(cell, xf, yf, m)
    pref, _, _ = O.cg_2d(cell, xf, yf, m, rhs, tol=1e-14)
    args = (dt_(c.h), dt_(c.hu), dt_(c.hv), dt_(c.hw))
    its = []
    for warm, p0 in ((0, 3.0), (1, None)):
        ctx = B.context_2d(c, crit=S.CRIT_GLOBAL, precision=1, tol=1e-13, max_iter=5000, warm=warm)
        p = (torch.full((c.ny, c.nx), p0, dtype=torch.float64, device=DEV) if p0 is not None
             else dt_(pref * (1.0 + 1e-6)))
        it, rr = ctx.solve_pressure(*args, torch.tensor(m, device=DEV), t0, dt, p)
        assert ctx.sync_stats()["status"] == 0
        assert rr <= 1e-13 and 0 < it <= 64
        assert rel(p, pref) <= 1e-10
        its.append(it)
    assert its[1] < its[0], its


@pytest.mark.parametrize("precision", [0, 1])
def test_global_multigrid_continued_by_the_tile_solver(B, precision):
    """cells four times wider than high (the point smoother leaves the
    anisotropic error's smooth-along-x part, ~65 multigrid iterations from a
    zero guess), so the multigrid CG uses its per-step budget of 32
    iterations: the tile solver continues from its iterate, the step meets
    the tolerance, counts the iterations of both and matches the oracle"""
    c = S.random_case_2d(200, 80, seed=47, dx=1.0, dy=0.25, h0=10.0)
    tol = 1e-13 if precision == 0 else 1e-11
    kw = dict(crit=S.CRIT_GLOBAL, cfl=0.4, precision=precision, tol=tol, max_iter=20000,
              warm=0)
    ctx, st, h, hu, hv, hw, p, m = run2d(B, c, 1, **kw)
    print("iterations", st["iters"], "rel_res", st["rel_res"])
    assert st["status"] == 0, st
    assert st["iters"] > 32 and st["rel_res"] <= tol, st
    ref = O.Sim2D(c, O.phys_struct(crit=S.CRIT_GLOBAL, tol=1e-14), cfl=0.4).step(1)
    bar = 1e-10 if precision == 0 else 1e-6
    for g, r in ((hu, ref.hu), (hv, ref.hv), (hw, ref.hw), (p, ref.p)):
        assert rel(g, r) <= bar


def test_global_multigrid_no_convergence_status(B):
    """an iteration cap below what the tolerance needs: the step reports
    no convergence (status code), the pressure is the last iterate"""
    c = S.random_case_2d(256, 192, seed=47, dx=1.0, dy=1.0, h0=10.0)
    kw = dict(crit=S.CRIT_GLOBAL, cfl=0.4, precision=0, tol=1e-14, max_iter=2, warm=0)
    ctx, st, h, hu, hv, hw, p, m = run2d(B, c, 1, **kw)
    assert st["status"] == B.ENOCONV
    assert st["iters"] == 2 and st["rel_res"] > 1e-14
    assert torch.isfinite(p).all()


def test_status_codes_2d(B):
    """a non-finite value in the state gives ENAN, a cell whose depth is not
    positive gives EDRY (both in a whole step); the state stays finite where
    it was"""
    c = case(nx=96, ny=64, seed=13)
    kw = dict(crit=S.CRIT_ETA_D, k_nh=4e-3, cfl=0.0, dt_fixed=0.005, precision=0, tol=1e-12,
              max_iter=2000)
    for mutate, want in ((lambda h: h.__setitem__((10, 20), np.nan), B.ENAN),
                         (lambda h: h.__setitem__((30, 40), -0.5), B.EDRY)):
        hh = c.h.copy()
        mutate(hh)
        ctx = B.context_2d(c, **kw)
        ctx.set_time(c.t0)
        h, hu, hv, hw = dt_(hh), dt_(c.hu), dt_(c.hv), dt_(c.hw)
        p = torch.zeros_like(h)
        ctx.step(h, hu, hv, hw, p, nsteps=1)
        assert ctx.sync_stats()["status"] == want


@pytest.mark.parametrize("precision", [0, 1])
def test_adaptive_multigrid_on_the_active_box(B, precision):
    """an adaptive step whose marked area (a disc of ~113k cells, 251 active
    tiles: more than the 128 up to which the tile solver keeps its coarse
    space) sends the solve to the multigrid CG on the active tiles'
    bounding box, with identity rows on the box's unmarked tiles: the
    oracle's masks and fields, in multigrid's few dozen iterations"""
    c = S.hump_case_2d(640, 512, seed=5, amp=0.01, radius=125.0)
    tol = 1e-13 if precision == 0 else 1e-11
    kw = dict(crit=S.CRIT_ETA_D, k_nh=1e-3, enlarge=1, cfl=0.4, precision=precision, tol=tol,
              max_iter=20000, warm=1)
    # the first call of a context steps with the tile solver (the host has
    # not seen an active-tile count yet); the second, after the first one's
    # count (251 tiles) is back, with the multigrid graph
    ctx, st, h, hu, hv, hw, p, m = run2d(B, c, 1, **kw)
    assert st["iters"] > 32, st  # the tile solver's count
    ctx.step(h, hu, hv, hw, p, m, nsteps=2)
    st = ctx.sync_stats()
    print("active", st["n_active"], "iterations", st["iters"], "rel_res", st["rel_res"])
    assert st["status"] == 0, st
    assert st["n_active"] > 128 * 512 and st["iters"] <= 32, st
    ref = O.Sim2D(c, O.phys_struct(crit=S.CRIT_ETA_D, k_nh=1e-3, enlarge=1, tol=1e-14),
                  cfl=0.4).step(3)
    assert np.array_equal(m.cpu().numpy(), ref.mask)
    bar = 1e-10 if precision == 0 else 1e-6
    for g, r in ((h - dt_(c.ds), ref.h - c.ds), (hu, ref.hu), (hv, ref.hv), (hw, ref.hw), (p, ref.p)):
        assert rel(g, r) <= bar
    # a second context gives the same bits (the box leaves cells of the
    # coarsest level outside it, whose LDS values the sweeps must not read)
    again = run2d(B, c, 1, **kw)
    again[0].step(*again[2:8], nsteps=2)
    for x, y in zip((h, hu, hv, hw, p), again[2:7]):
        assert torch.equal(x, y)
