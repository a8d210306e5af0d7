"""Pins of the 2D FP64 oracle.  The paper is one-dimensional and names 2D as
future work, so the 2D reading is pinned by reductions and invariants only:
y-invariant data reproduces the 1D oracle, x <-> y transposition, lake at
rest, mass conservation, SPD operator and dense solve, and the 2D linear
dispersion relation of the Green-Naghdi equations."""
import math

import numpy as np
import pytest

import oracle as O
import swe_inputs as S


def _yinv_case(case1d, ny=5, dy=0.3):
    t = lambda a: np.tile(np.asarray(a)[None, :], (ny, 1)).copy()
    return S.Case2D(nx=case1d.n, ny=ny, dx=case1d.dx, dy=dy, ds=t(case1d.ds), h=t(case1d.h),
                    hu=t(case1d.hu), hv=np.zeros((ny, case1d.n)), hw=t(case1d.hw),
                    body=case1d.body, t0=case1d.t0)


def test_y_invariant_hydrostatic_part_is_exactly_1d():
    c1 = S.random_case_1d(120, seed=31, amp=0.01, mom=0.02, vert=0.01)
    ph = O.phys_struct(crit=S.CRIT_NONE)
    a = O.Sim1D(c1, ph, cfl=0.0, dt_fixed=2e-3).step(6)
    b = O.Sim2D(_yinv_case(c1), ph, cfl=0.0, dt_fixed=2e-3).step(6)
    for j in range(b.ny):
        assert np.allclose(b.h[j], a.h, rtol=0, atol=1e-13)
        assert np.allclose(b.hu[j], a.hu, rtol=0, atol=1e-13)
        assert np.allclose(b.hw[j], a.hw, rtol=0, atol=1e-13)
    assert np.abs(b.hv).max() == 0.0


@pytest.mark.parametrize("crit", [S.CRIT_GLOBAL, S.CRIT_ETA_D, S.CRIT_ETA_X, S.CRIT_U, S.CRIT_U_X,
                                  S.CRIT_W, S.CRIT_W_X])
def test_y_invariant_data_reproduces_1d(crit):
    """zero Dirichlet p also holds at the y-walls, which the 1D problem does
    not have; their influence decays like exp(-dist sqrt(3) / h), so rows far
    from the y-walls (in units of h / sqrt(3)) must equal the 1D oracle"""
    c1 = S.random_case_1d(120, seed=31, amp=0.01, mom=0.02, vert=0.01)
    ny = 31
    c2 = _yinv_case(c1, ny=ny, dy=2.0)
    k = {S.CRIT_ETA_D: 4e-3, S.CRIT_ETA_X: 1e-2, S.CRIT_U: 5e-3, S.CRIT_U_X: 2e-2,
         S.CRIT_W: 3e-3, S.CRIT_W_X: 2e-2}.get(crit, 1e-3)
    ph = O.phys_struct(crit=crit, k_nh=k, tol=1e-15)
    a = O.Sim1D(c1, ph, cfl=0.0, dt_fixed=2e-3).step(6)
    b = O.Sim2D(c2, ph, cfl=0.0, dt_fixed=2e-3).step(6)
    assert 0 < a.last_active
    for j in range(ny // 2 - 3, ny // 2 + 4):
        assert np.array_equal(b.mask[j], a.mask)
        assert np.allclose(b.h[j], a.h, rtol=0, atol=1e-12)
        assert np.allclose(b.hu[j], a.hu, rtol=0, atol=1e-10)
        assert np.allclose(b.hw[j], a.hw, rtol=0, atol=1e-10)
        assert np.allclose(b.p[j], a.p, rtol=0, atol=1e-8 * np.abs(a.p).max())
        assert np.abs(b.hv[j]).max() < 1e-12


def test_transpose_symmetry():
    c = S.random_case_2d(18, 14, seed=2, body=S.Body())
    T = lambda a: np.ascontiguousarray(a.T)
    ct = S.Case2D(nx=c.ny, ny=c.nx, dx=c.dy, dy=c.dx, ds=T(c.ds), h=T(c.h), hu=T(c.hv), hv=T(c.hu),
                  hw=T(c.hw), body=S.Body())
    ph = O.phys_struct(crit=S.CRIT_ETA_D, k_nh=2e-3, tol=1e-14)
    a = O.Sim2D(c, ph, cfl=0.4).step(5)
    b = O.Sim2D(ct, ph, cfl=0.4).step(5)
    assert np.array_equal(a.mask, b.mask.T)
    assert np.allclose(a.h, b.h.T, rtol=0, atol=1e-12)
    assert np.allclose(a.hu, b.hv.T, rtol=0, atol=1e-11)
    assert np.allclose(a.hv, b.hu.T, rtol=0, atol=1e-11)
    assert np.allclose(a.hw, b.hw.T, rtol=0, atol=1e-11)


def test_lake_at_rest_and_mass_2d():
    rng = np.random.default_rng(7)
    nx, ny = 24, 20
    ds = 2.0 + 0.3 * S.gaussian_field_2d(nx, ny, 0.5, 0.5, 1.0, 1.5, 11)
    z = np.zeros((ny, nx))
    c = S.Case2D(nx=nx, ny=ny, dx=0.5, dy=0.5, ds=ds, h=ds.copy(), hu=z, hv=z, hw=z, body=S.Body())
    s = O.Sim2D(c, O.phys_struct(crit=S.CRIT_GLOBAL), cfl=0.4).step(100)
    assert np.abs(s.h - ds).max() < 1e-12
    assert max(np.abs(s.hu).max(), np.abs(s.hv).max(), np.abs(s.hw).max()) < 1e-12
    c2 = S.random_case_2d(20, 16, seed=9)
    s2 = O.Sim2D(c2, O.phys_struct(crit=S.CRIT_ETA_D, tol=1e-12), cfl=0.4)
    m0 = s2.h.sum()
    s2.step(40)
    assert abs(s2.h.sum() - m0) <= 1e-13 * m0


def test_operator_symmetric_positive_definite_and_cg_matches_dense():
    c = S.random_case_2d(9, 7, seed=4)
    ph = O.phys_struct()
    cell, xf, yf = O.nh_coeffs_2d(c.ds, c.dx, c.dy, c.body, ph, 0.2, 0.01, c.h, c.hu, c.hv, c.hw)
    mask = np.ones((7, 9), dtype=np.uint8)
    mask[3, 2:5] = 0
    mask[0, 8] = 0
    idx = np.argwhere(mask.ravel()).ravel()
    N = 63
    A = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        A[:, k] = O.nh_apply_2d(cell, xf, yf, mask, e.reshape(7, 9)).ravel()
    As = A[np.ix_(idx, idx)]
    assert np.allclose(As, As.T, rtol=1e-13, atol=1e-13 * np.abs(As).max())
    np.linalg.cholesky(As)
    rhs = O.nh_rhs_2d(cell, xf, yf, mask)
    x, it, rr = O.cg_2d(cell, xf, yf, mask, rhs, tol=1e-14)
    ref = np.zeros(N)
    ref[idx] = np.linalg.solve(As, rhs.ravel()[idx])
    assert np.allclose(x.ravel(), ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
    assert rr <= 1e-14 * 1.01
    assert np.all(x.ravel()[mask.ravel() == 0] == 0.0)


def test_dispersion_2d_box_mode():
    """cos(kx x) cos(ky y) standing mode on a flat bottom, |k| d = 1:
    omega^2 = g d |k|^2 / (1 + (|k| d)^2 / 3)"""
    g, d, a = 9.81, 1.0, 1e-4
    kk = 1.0
    kx = ky = kk / math.sqrt(2)
    Lx, Ly = 2 * math.pi / kx, 2 * math.pi / ky
    n = 48
    dx, dy = Lx / n, Ly / n
    x = (np.arange(n) + 0.5) * dx
    y = (np.arange(n) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    mode = np.cos(kx * X) * np.cos(ky * Y)
    z = np.zeros((n, n))
    c = S.Case2D(nx=n, ny=n, dx=dx, dy=dy, ds=np.full((n, n), d), h=d + a * mode, hu=z, hv=z, hw=z,
                 body=S.Body())
    w = math.sqrt(g * d * kk * kk / (1 + kk * kk / 3))
    sim = O.Sim2D(c, O.phys_struct(crit=S.CRIT_GLOBAL, tol=1e-12), cfl=0.3)
    proj = lambda: 4.0 / (n * n) * np.sum((sim.h - d) * mode)
    tp, ap = 0.0, proj()
    while True:
        sim.step()
        an = proj()
        if an <= 0:
            tq = tp + (sim.time - tp) * ap / (ap - an)
            break
        tp, ap = sim.time, an
    assert abs(tq - 0.5 * math.pi / w) < 0.015 * (0.5 * math.pi / w)
