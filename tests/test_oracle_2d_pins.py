"""Pins of the 2D oracle's moving-bottom, cross-derivative and y-direction
terms, which y-invariant data (every y term zero) and x <-> y transposition
(the body moves along x only) cannot reach.

* d_t, d_tt, d_xt, d_yt of the forcing against centred differences of the
  oracle's own d(x, y, t) evaluated at single points (a 1 x 1 grid whose cell
  centre is the point).
* phi (vector form of Eq. 5): alpha phi / (rho h) is minus the second time
  derivative of the bottom elevation d seen along a path that starts at the
  cell with the flow velocity and accelerates with the hydrostatic -g grad eta:
  d2/dtau2 d(X(tau), t + tau) = d_tt + 2 u . grad d_t + u^T (grad grad d) u
  + X'' . grad d.  The path derivative is taken by a centred difference in tau
  of point values of d, so it shares none of the oracle's spatial stencils;
  the oracle's central differences converge to it at second order.
* The face coefficient K = (dt h / rho) (1 - d_n^2 / alpha): the diagonal
  entry of (I - grad d grad d^T / alpha), which equals the inverse of
  I + grad d grad d^T / 4 (computed here with a 2 x 2 matrix inverse).
* f2 with the same independent ingredients.
* Every 2D criterion: closed forms on linear fields, and transposition on
  random fields (non-square grid, dx != dy, walls included)."""
import math

import numpy as np
import pytest

import oracle as O
import swe_inputs as S

G, RHO = 9.81, 1000.0
LX, LY = 12.0, 9.0


def ds_fn(x, y):  # static depth with strong slopes in both directions
    return 6.0 + 0.5 * x - 0.4 * y + 0.3 * np.sin(0.5 * x) * np.cos(0.4 * y)


def eta_fn(x, y):
    return 0.15 * np.sin(0.45 * x + 0.3) * np.cos(0.35 * y - 0.2) + 0.05 * y / LY


def u_fn(x, y):
    return 0.9 + 0.4 * np.sin(0.3 * y)


def v_fn(x, y):
    return -0.7 + 0.3 * np.cos(0.25 * x)


def w_fn(x, y):
    return 0.05 * np.cos(0.2 * x + 0.3 * y)


def body(t_ramp=3.0):
    """Gaussian mound offset in y from the grid's centre line, on a
    sinusoidal ramp (X'' != 0 at the times used)"""
    return S.Body(kind=S.BODY_GAUSS, law=S.LAW_SIN_RAMP, amp=1.2, length=2.5, x0=4.0, y0=3.2,
                  dir=1.0, q=(5.0, t_ramp, 0.0, 0.0, 0.0))


def d_point(x, y, t, b):
    """the oracle's d at the point (x, y) and time t: a 1 x 1 grid centred there"""
    d, *_ = O.forcing_2d(np.array([[ds_fn(x, y)]]), 2.0 * x, 2.0 * y, b, t)
    return float(d[0, 0])


def grid(n):
    nx, ny = n, int(round(n * LY / LX * 1.25))  # dy != dx, non-square
    dx, dy = LX / nx, LY / ny
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    return nx, ny, dx, dy, X, Y


def state(X, Y, b, t1):
    d, *_ = O.forcing_2d(ds_fn(X, Y), X[0, 1] - X[0, 0], Y[1, 0] - Y[0, 0], b, t1)
    h = d + eta_fn(X, Y)
    return h, h * u_fn(X, Y), h * v_fn(X, Y), h * w_fn(X, Y)


def grad_fn(f, x, y, e=1e-5):
    return ((f(x + e, y) - f(x - e, y)) / (2 * e), (f(x, y + e) - f(x, y - e)) / (2 * e))


def interior(ny, nx, m):
    s = np.zeros((ny, nx), bool)
    s[m:ny - m, m:nx - m] = True
    return s


def test_forcing_2d_time_and_mixed_derivatives():
    b = body()
    n = 24
    nx, ny, dx, dy, X, Y = grid(n)
    t = 1.1
    d, d_t, d_tt, d_xt, d_yt = O.forcing_2d(ds_fn(X, Y), dx, dy, b, t)
    e = 1e-4
    rng = np.random.default_rng(3)
    for _ in range(40):
        j, i = rng.integers(0, ny), rng.integers(0, nx)
        x, y = X[j, i], Y[j, i]
        P = lambda dxp, dyp, dtp: d_point(x + dxp, y + dyp, t + dtp, b)
        ft = (P(0, 0, e) - P(0, 0, -e)) / (2 * e)
        ftt = (P(0, 0, e) - 2 * P(0, 0, 0) + P(0, 0, -e)) / (e * e)
        fxt = (P(e, 0, e) - P(e, 0, -e) - P(-e, 0, e) + P(-e, 0, -e)) / (4 * e * e)
        fyt = (P(0, e, e) - P(0, e, -e) - P(0, -e, e) + P(0, -e, -e)) / (4 * e * e)
        assert abs(d[j, i] - P(0, 0, 0)) <= 1e-14 * abs(d[j, i])
        assert abs(d_t[j, i] - ft) <= 1e-7 * max(1.0, abs(ft))
        assert abs(d_tt[j, i] - ftt) <= 2e-5 * max(1.0, abs(ftt))
        assert abs(d_xt[j, i] - fxt) <= 2e-5 * max(1.0, abs(fxt))
        assert abs(d_yt[j, i] - fyt) <= 2e-5 * max(1.0, abs(fyt))
    # the mound's y-offset makes d_yt non-trivial on this grid
    assert np.abs(d_yt).max() > 0.1 * np.abs(d_xt).max()


def path_targets(X, Y, b, t1, mask):
    """-d2/dtau2 d along the hydrostatic particle path, at the masked cells"""
    T = np.full(X.shape, np.nan)
    tau = 2e-3
    for j, i in zip(*np.nonzero(mask)):
        x, y = X[j, i], Y[j, i]
        u, v = u_fn(x, y), v_fn(x, y)
        ex, ey = grad_fn(eta_fn, x, y)
        ax, ay = -G * ex, -G * ey
        P = lambda s: d_point(x + u * s + 0.5 * ax * s * s, y + v * s + 0.5 * ay * s * s, t1 + s, b)
        T[j, i] = -(P(tau) - 2.0 * P(0.0) + P(-tau)) / (tau * tau)
    return T


def exact_grad_d(x, y, b, t1, e=1e-5):
    return ((d_point(x + e, y, t1, b) - d_point(x - e, y, t1, b)) / (2 * e),
            (d_point(x, y + e, t1, b) - d_point(x, y - e, t1, b)) / (2 * e))


def phi_and_f2_errors(n, t1=1.3, dt=0.01):
    b = body()
    nx, ny, dx, dy, X, Y = grid(n)
    h, m, nn, k = state(X, Y, b, t1)
    ph = O.phys_struct(g=G, rho=RHO)
    cell, xf, yf = O.nh_coeffs_2d(ds_fn(X, Y), dx, dy, b, ph, t1, dt, h, m, nn, k)
    # the same physical points at every resolution: every (n/12)-th cell
    # centre at n = 12 q lies on a fixed lattice when n is a multiple of 12
    sel = np.zeros((ny, nx), bool)
    step_x, step_y = n // 12, ny // 15
    for jj in range(3, 12):
        for ii in range(3, 9):
            sel[jj * step_y + step_y // 2, ii * step_x + step_x // 2] = True
    T = path_targets(X, Y, b, t1, sel)
    al, phi, f2 = cell[2], cell[3], cell[5]
    got = al * phi / (RHO * h)
    e_phi = np.nanmax(np.abs(got - T)[sel]) / np.nanmax(np.abs(T[sel]))
    # f2 = -2 d_t - 2 k / h - grad d . m / (2 h) - dt alpha phi / (2 rho h)
    ref = np.full(X.shape, np.nan)
    e = 1e-5
    for j, i in zip(*np.nonzero(sel)):
        x, y = X[j, i], Y[j, i]
        gx, gy = exact_grad_d(x, y, b, t1)
        a = 4.0 + gx * gx + gy * gy
        phx = T[j, i] * RHO * h[j, i] / a
        d_t = (d_point(x, y, t1 + e, b) - d_point(x, y, t1 - e, b)) / (2 * e)
        ref[j, i] = (-2.0 * d_t - 2.0 * k[j, i] / h[j, i] - (gx * m[j, i] + gy * nn[j, i]) /
                     (2.0 * h[j, i]) - dt * a * phx / (2.0 * RHO * h[j, i]))
    e_f2 = np.nanmax(np.abs(f2 - ref)[sel]) / np.nanmax(np.abs(ref[sel]))
    return e_phi, e_f2, T[sel]


def test_phi_and_f2_match_the_particle_path_at_second_order():
    c1, f1, T = phi_and_f2_errors(48)
    c2, f2, _ = phi_and_f2_errors(96)
    # every term of phi contributes on this data
    assert np.abs(T).max() > 0.5
    assert c2 < 3e-3 and f2 < 3e-3, (c1, c2, f1, f2)
    assert 2.8 < c1 / c2 < 5.5, (c1, c2)
    assert 2.8 < f1 / f2 < 5.5, (f1, f2)


def face_K_error(n, t1=1.3, dt=0.01):
    b = body()
    nx, ny, dx, dy, X, Y = grid(n)
    h, m, nn, k = state(X, Y, b, t1)
    ph = O.phys_struct(g=G, rho=RHO)
    cell, xf, yf = O.nh_coeffs_2d(ds_fn(X, Y), dx, dy, b, ph, t1, dt, h, m, nn, k)
    errs = []
    for jj in range(3, 12):
        for ii in range(3, 9):
            j = jj * (ny // 15) + (ny // 15) // 2
            f = ii * (n // 12)  # x-face between cells f-1 and f
            xfc, yfc = f * dx, Y[j, 0]
            hf = 0.5 * (h[j, f - 1] + h[j, f])
            D = np.array(exact_grad_d(xfc, yfc, b, t1))
            Minv = np.linalg.inv(np.eye(2) + np.outer(D, D) / 4.0)
            errs.append(abs(xf[0, j, f] * RHO / (dt * hf) - Minv[0, 0]))
            # y-face between rows j-1 and j, at column i
            i = ii * (n // 12) + (n // 12) // 2
            yfc2 = j * dy
            hf = 0.5 * (h[j - 1, i] + h[j, i])
            D = np.array(exact_grad_d(X[0, i], yfc2, b, t1))
            Minv = np.linalg.inv(np.eye(2) + np.outer(D, D) / 4.0)
            errs.append(abs(yf[0, j, i] * RHO / (dt * hf) - Minv[1, 1]))
    return max(errs)


def test_face_coefficient_is_the_inverse_tensor_diagonal():
    e1, e2 = face_K_error(48), face_K_error(96)
    assert e2 < 5e-4, (e1, e2)
    assert 2.8 < e1 / e2 < 5.5, (e1, e2)


# ------------------------------------------------------------ criteria ----

def lin_case(nx=14, ny=11, dx=0.7, dy=0.45):
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    return nx, ny, dx, dy, X, Y


CLOSED_FORMS = {
    # crit: (eta, u, v, w) as functions of (X, Y), indicator in the interior
    S.CRIT_ETA_X: (lambda X, Y: 0.02 * X - 0.035 * Y, None, None, None, math.hypot(0.02, 0.035)),
    S.CRIT_U: (None, lambda X, Y: 0.3 + 0 * X, lambda X, Y: -0.4 + 0 * X, None, 0.5),
    S.CRIT_U_X: (None, lambda X, Y: 0.03 * X + 0.05 * Y, lambda X, Y: -0.02 * X + 0.07 * Y, None,
                 math.sqrt(0.03 ** 2 + 0.05 ** 2 + 0.02 ** 2 + 0.07 ** 2)),
    S.CRIT_W: (None, None, None, lambda X, Y: -0.012 + 0 * X, 0.012),
    S.CRIT_W_X: (None, None, None, lambda X, Y: 0.004 * X - 0.009 * Y, math.hypot(0.004, 0.009)),
}


@pytest.mark.parametrize("crit", sorted(CLOSED_FORMS))
def test_criteria_closed_forms_on_linear_fields(crit):
    nx, ny, dx, dy, X, Y = lin_case()
    fe, fu, fv, fw, val = CLOSED_FORMS[crit]
    ds = 2.0 + 0.1 * X + 0.05 * Y
    z = np.zeros_like(X)
    eta = fe(X, Y) if fe else z
    h = ds + eta
    u, v, w = (f(X, Y) if f else z for f in (fu, fv, fw))
    ind = O.indicator_2d(ds, dx, dy, S.Body(), O.phys_struct(crit=crit), 0.0, h, h * u, h * v,
                         h * w)
    inn = interior(ny, nx, 1)
    assert np.allclose(ind[inn], val, rtol=1e-12, atol=0)


def test_eta_d_criterion_closed_form():
    nx, ny, dx, dy, X, Y = lin_case()
    b = body()
    ds = 2.0 + 0.1 * X + 0.05 * Y
    d, *_ = O.forcing_2d(ds, dx, dy, b, 0.7)
    eta = 0.03 * np.sin(X) * np.cos(Y)
    h = d + eta
    z = np.zeros_like(X)
    ind = O.indicator_2d(ds, dx, dy, b, O.phys_struct(crit=S.CRIT_ETA_D), 0.7, h, z, z, z)
    assert np.allclose(ind, np.abs(eta / d), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("crit", [S.CRIT_ETA_D, S.CRIT_ETA_X, S.CRIT_U, S.CRIT_U_X, S.CRIT_W,
                                  S.CRIT_W_X])
def test_every_criterion_transposes(crit):
    """walls included: u is odd across x-walls and v across y-walls"""
    c = S.random_case_2d(13, 9, seed=21 + crit, body=S.Body())
    c.hu[:] += 0.3 * c.h * np.linspace(-1, 1, c.nx)[None, :]
    c.hv[:] -= 0.2 * c.h * np.linspace(-1, 1, c.ny)[:, None] ** 2
    T = lambda a: np.ascontiguousarray(np.asarray(a).T)
    ph = O.phys_struct(crit=crit, k_nh=1e-3)
    a = O.indicator_2d(c.ds, c.dx, c.dy, S.Body(), ph, 0.0, c.h, c.hu, c.hv, c.hw)
    b = O.indicator_2d(T(c.ds), c.dy, c.dx, S.Body(), ph, 0.0, T(c.h), T(c.hv), T(c.hu), T(c.hw))
    assert np.allclose(a, b.T, rtol=1e-13, atol=1e-300)
    assert np.abs(a).max() > 0
    # the y-parts matter: the indicator changes when only the y-data change
    c2hv = c.hv.copy()
    c2hv[:, 3] *= 1.7
    if crit in (S.CRIT_U, S.CRIT_U_X):
        a2 = O.indicator_2d(c.ds, c.dx, c.dy, S.Body(), ph, 0.0, c.h, c.hu, c2hv, c.hw)
        assert np.abs(a2 - a).max() > 1e-6 * np.abs(a).max()
