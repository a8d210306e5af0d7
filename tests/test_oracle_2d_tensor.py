"""Pins of the oracle's exact-tensor 2D operator (the 7-point stencil).

The flux correction at the faces is the tensor S12^{-1} applied to the face
gradients of p; the diagonal (5-point) form keeps its diagonal only.  The
off-diagonal entries couple an x-face with a y-face, paired by owner cell (the
x-face east of a cell with the y-face north of it), which gives each cell two
more neighbours: (i-1, j+1) and (i+1, j-1).  Pinned here against what the
continuous operator fixes:

* the pair's 2 x 2 block is the inverse of S12 = (rho / (dt h))(I + grad d
  grad d^T / 4) on a planar bottom under uniform depth (computed here with a
  matrix inverse, not from the oracle's formula);
* on a planar bottom, with uniform depth and a linear pressure field, the
  discrete operator is exact: A p = (s22 + s11^T S12^{-1} s11) p with
  s11 = -3 grad d / (2 h), i.e. (3 dt / (rho h))(1 + 3 |grad d|^2 / alpha) p,
  the same for every direction of the slope; the diagonal form is not
  (it misses by ~1e-4 relative on a diagonal slope of 1/4);
* the correction of a constant pressure is S12^{-1} (-s11) p, parallel to
  grad d: (6 dt / (rho alpha)) grad d p in hu, hv and 6 dt p / (rho alpha)
  in hw;
* y-invariant data gives no pair coupling, so the step equals the diagonal
  form's (and with it the 1D reductions of test_oracle_2d.py);
* the operator is symmetric positive definite with the 7-point pattern, CG
  matches a dense solve, and a step is symmetric under x <-> y transposition."""
import math

import numpy as np
import pytest

import oracle as O
import swe_inputs as S

RHO = 1000.0


def planar(nx, ny, dx, dy, sx, sy, h0=5.0, d0=6.0):
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    ds = d0 + sx * X + sy * Y
    return X, Y, ds, np.full((ny, nx), h0)


def system(nx, ny, dx, dy, ds, h, dt, t1=0.0):
    z = np.zeros_like(h)
    ph = O.phys_struct()
    cell, xf, yf = O.nh_coeffs_2d(ds, dx, dy, S.Body(), ph, t1, dt, h, z, z, z)
    kxy = O.nh_pairs_2d(ds, dx, dy, S.Body(), t1, xf, yf)
    return cell, xf, yf, kxy


SLOPES = [(0.25 * math.cos(a), 0.25 * math.sin(a)) for a in (0.0, math.pi / 6, math.pi / 4,
                                                             2 * math.pi / 3, -math.pi / 3)]


@pytest.mark.parametrize("sx,sy", SLOPES + [(0.6, -0.45), (-0.05, 0.02)])
def test_pair_block_is_the_inverse_of_s12(sx, sy):
    nx, ny, dx, dy, dt, h0 = 12, 10, 0.5, 0.4, 0.02, 5.0
    _, _, ds, h = planar(nx, ny, dx, dy, sx, sy, h0=h0)
    _, xf, yf, kxy = system(nx, ny, dx, dy, ds, h, dt)
    g = np.array([sx, sy])
    S12 = RHO / (dt * h0) * (np.eye(2) + np.outer(g, g) / 4.0)
    Kt = np.linalg.inv(S12)
    for j in range(2, ny - 2):
        for i in range(2, nx - 2):
            blk = np.array([[xf[0, j, i + 1], kxy[j, i]], [kxy[j, i], yf[0, j + 1, i]]])
            assert np.allclose(blk, Kt, rtol=1e-12, atol=1e-12 * np.abs(Kt).max()), (i, j)
    # walls: the pairs with a wall face carry no coupling
    assert np.all(kxy[:, nx - 1] == 0.0) and np.all(kxy[ny - 1, :] == 0.0)


@pytest.mark.parametrize("sx,sy", SLOPES)
def test_operator_on_linear_pressure_is_exact_and_isotropic(sx, sy):
    nx, ny, dx, dy, dt, h0 = 14, 12, 0.5, 0.4, 0.02, 5.0
    X, Y, ds, h = planar(nx, ny, dx, dy, sx, sy, h0=h0)
    cell, xf, yf, kxy = system(nx, ny, dx, dy, ds, h, dt)
    p = 2.0 + 0.3 * X - 0.7 * Y
    mask = np.ones((ny, nx), dtype=np.uint8)
    s2 = sx * sx + sy * sy
    al = 4.0 + s2
    want = 3.0 * dt / (RHO * h0) * (1.0 + 3.0 * s2 / al) * p
    A7 = O.nh_apply_2d(cell, xf, yf, mask, p, kxy=kxy)
    A5 = O.nh_apply_2d(cell, xf, yf, mask, p)
    sl = (slice(2, ny - 2), slice(2, nx - 2))
    e7 = np.abs(A7[sl] / want[sl] - 1.0).max()
    e5 = np.abs(A5[sl] / want[sl] - 1.0).max()
    assert e7 < 1e-11, e7
    if abs(sx * sy) > 1e-3:  # the diagonal form misses the cross term 2 k s11x s11y
        assert e5 > 5e-5, e5
    else:
        assert e5 < 1e-11, e5


@pytest.mark.parametrize("sx,sy", SLOPES)
def test_correction_of_constant_pressure_follows_the_slope(sx, sy):
    nx, ny, dx, dy, dt, h0 = 12, 11, 0.5, 0.4, 0.02, 5.0
    X, Y, ds, h = planar(nx, ny, dx, dy, sx, sy, h0=h0)
    cell, xf, yf, kxy = system(nx, ny, dx, dy, ds, h, dt)
    rng = np.random.default_rng(3)
    mt, nt, kt = (rng.standard_normal((ny, nx)) * 0.1 for _ in range(3))
    mask = np.ones((ny, nx), dtype=np.uint8)
    P0 = 1500.0
    a = O.nh_correct_2d(cell, xf, yf, dt, RHO, mt, nt, kt, mask, np.full((ny, nx), P0), kxy=kxy)
    b = O.nh_correct_2d(cell, xf, yf, dt, RHO, mt, nt, kt, mask, np.zeros((ny, nx)), kxy=kxy)
    al = 4.0 + sx * sx + sy * sy
    c = 6.0 * dt / (RHO * al) * P0
    sl = (slice(2, ny - 2), slice(2, nx - 2))
    tol = 1e-11 * c
    assert np.allclose((a[0] - b[0])[sl], c * sx, rtol=0, atol=tol)
    assert np.allclose((a[1] - b[1])[sl], c * sy, rtol=0, atol=tol)
    assert np.allclose((a[2] - b[2])[sl], c, rtol=0, atol=tol)


def test_y_invariant_data_has_no_pair_coupling():
    c1 = S.random_case_1d(60, seed=5, amp=0.01, mom=0.02, vert=0.01)
    ny = 7
    t = lambda a: np.tile(np.asarray(a)[None, :], (ny, 1)).copy()
    c2 = S.Case2D(nx=c1.n, ny=ny, dx=c1.dx, dy=0.4, ds=t(c1.ds), h=t(c1.h), hu=t(c1.hu),
                  hv=np.zeros((ny, c1.n)), hw=t(c1.hw), body=c1.body, t0=c1.t0)
    a = O.Sim2D(c2, O.phys_struct(crit=S.CRIT_GLOBAL, tol=1e-14), cfl=0.4).step(4)
    b = O.Sim2D(c2, O.phys_struct(crit=S.CRIT_GLOBAL, tol=1e-14, tensor=1), cfl=0.4).step(4)
    for x, y in ((a.h, b.h), (a.hu, b.hu), (a.hv, b.hv), (a.hw, b.hw), (a.p, b.p)):
        assert np.array_equal(x, y)


def dense(cell, xf, yf, kxy, mask):
    ny, nx = mask.shape
    N = nx * ny
    A = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        A[:, k] = O.nh_apply_2d(cell, xf, yf, mask, e.reshape(ny, nx), kxy=kxy).ravel()
    return A


def test_operator_spd_seven_point_and_cg_matches_dense():
    nx, ny = 9, 8
    c = S.random_case_2d(nx, ny, seed=4)
    c.ds[:] += 0.4 * np.add.outer(np.arange(ny) * c.dy, -0.7 * np.arange(nx) * c.dx)  # steep
    c.h[:] += 0.4 * np.add.outer(np.arange(ny) * c.dy, -0.7 * np.arange(nx) * c.dx)
    ph = O.phys_struct()
    t1, dt = 0.2, 0.01
    cell, xf, yf = O.nh_coeffs_2d(c.ds, c.dx, c.dy, c.body, ph, t1, dt, c.h, c.hu, c.hv, c.hw)
    kxy = O.nh_pairs_2d(c.ds, c.dx, c.dy, c.body, t1, xf, yf)
    assert np.abs(kxy).max() > 1e-3 * np.abs(xf[0]).max()
    mask = np.ones((ny, nx), dtype=np.uint8)
    mask[3, 2:5] = 0
    mask[0, 8] = 0
    mask[6, 6] = 0
    A = dense(cell, xf, yf, kxy, mask)
    idx = np.argwhere(mask.ravel()).ravel()
    As = A[np.ix_(idx, idx)]
    assert np.allclose(As, As.T, rtol=1e-13, atol=1e-13 * np.abs(As).max())
    np.linalg.cholesky(As)
    # the stencil: the cell, its four neighbours, (i-1, j+1) and (i+1, j-1)
    allowed = {(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (-1, 1), (1, -1)}
    seen = set()
    for r in idx:
        jr, ir = divmod(r, nx)
        for cc in np.nonzero(A[r])[0]:
            jc, ic = divmod(cc, nx)
            assert (ic - ir, jc - jr) in allowed, (ir, jr, ic, jc)
            seen.add((ic - ir, jc - jr))
    assert seen == allowed
    rhs = O.nh_rhs_2d(cell, xf, yf, mask)
    x, it, rr = O.cg_2d(cell, xf, yf, mask, rhs, tol=1e-14, kxy=kxy)
    ref = np.zeros(nx * ny)
    ref[idx] = np.linalg.solve(As, rhs.ravel()[idx])
    assert np.allclose(x.ravel(), ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
    assert rr <= 1e-14 * 1.01


def test_tensor_step_transpose_symmetry():
    c = S.random_case_2d(18, 14, seed=2, body=S.Body())
    ny, nx = c.ds.shape
    c.ds[:] += 0.3 * np.add.outer(np.arange(ny) * c.dy, 0.5 * np.arange(nx) * c.dx)
    c.h[:] += 0.3 * np.add.outer(np.arange(ny) * c.dy, 0.5 * np.arange(nx) * c.dx)
    T = lambda a: np.ascontiguousarray(a.T)
    ct = S.Case2D(nx=c.ny, ny=c.nx, dx=c.dy, dy=c.dx, ds=T(c.ds), h=T(c.h), hu=T(c.hv), hv=T(c.hu),
                  hw=T(c.hw), body=S.Body())
    ph = O.phys_struct(crit=S.CRIT_ETA_D, k_nh=2e-3, tol=1e-14, tensor=1)
    a = O.Sim2D(c, ph, cfl=0.4).step(5)
    b = O.Sim2D(ct, ph, cfl=0.4).step(5)
    assert a.last_active > 0
    ref = O.Sim2D(c, O.phys_struct(crit=S.CRIT_ETA_D, k_nh=2e-3, tol=1e-14), cfl=0.4).step(5)
    assert np.abs(ref.hu - a.hu).max() > 1e-9  # the pair coupling changed the step
    assert np.array_equal(a.mask, b.mask.T)
    assert np.allclose(a.h, b.h.T, rtol=0, atol=1e-12)
    assert np.allclose(a.hu, b.hv.T, rtol=0, atol=1e-11)
    assert np.allclose(a.hv, b.hu.T, rtol=0, atol=1e-11)
    assert np.allclose(a.hw, b.hw.T, rtol=0, atol=1e-11)
