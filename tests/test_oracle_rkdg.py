"""Pins of the oracle of the paper's own 1D discretisation (oracle/rkdg1d.py:
RKDG-P1 predictor, Sec. 3.1; LDG-P1 elliptic solve with the flip-flop flux,
Sec. 3.2).

* The paper's solitary-wave run at its own resolution (Sec. 4.1, dx = 4 m,
  dt = 0.1 s, T = 30 s) against its printed RMSE and correlation
  (tests/golden/solitary_paper.json).
* The LDG solve against a manufactured solution of the first-order system
  with variable coefficients: second-order convergence of p and hu.
* The hydrostatic predictor: exact mass conservation between walls, and
  second-order convergence to the linear standing wave of the shallow water
  equations.
* The whole non-hydrostatic step: the Green-Naghdi dispersion relation
  c^2 = g d / (1 + (kd)^2 / 3) of a standing wave.
* The moving-bottom terms: the sliding-block flume of Sec. 4.3 run with this
  discretisation and with the finite-volume oracle agree as both are refined."""
import dataclasses
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import swe_inputs as S
from oracle import rkdg1d as R

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_solitary_wave_at_its_own_resolution():
    g = json.load(open(os.path.join(GOLD, "solitary_paper.json")))
    st, pr = g["setup"], g["printed"]
    a, d, L, dx, dt, T = st["a"], st["d"], st["L"], st["dx"], st["dt"], st["T"]
    n = int(round(L / dx))
    Q = R.solitary_initial(n, dx, a, d, st["x0_over_L"] * L)
    m0 = Q[0].sum()
    Q, p, t = R.run(Q, d, S.Body(), 0.0, dt, int(round(T / dt)), dx)
    assert abs(t - T) < 1e-9
    x = R.node_x(n, dx)
    ex, _, _ = S.solitary_exact(x, t, a, d, st["x0_over_L"] * L)
    eta = Q[0] - d
    rmse = np.sqrt(np.mean((eta - ex) ** 2))
    r = np.corrcoef(eta.ravel(), ex.ravel())[0, 1]
    # the printed values: RMSE 0.0108 (this reading gives 0.0111) and r 0.9997
    assert abs(rmse - pr["rmse"]) <= 0.05 * pr["rmse"], rmse
    assert round(r, 4) == pr["r"], r
    assert abs(Q[0].sum() - m0) <= 1e-12 * m0


def _manufactured(n, L=3.0):
    P = lambda x: np.sin(np.pi * x / L) * (1 + 0.3 * x / L)
    Pd = lambda x: (np.pi / L * np.cos(np.pi * x / L) * (1 + 0.3 * x / L)
                    + np.sin(np.pi * x / L) * 0.3 / L)
    Qf = lambda x: np.cos(2 * x / L) + 0.5
    Qd = lambda x: -2 / L * np.sin(2 * x / L)
    dx = L / n
    x = R.node_x(n, dx)
    s11 = 0.4 * np.sin(x) + 0.2
    s12 = 1.5 + 0.5 * np.cos(x)
    s22 = 0.8 + 0.3 * x
    f1 = Pd(x) + s11 * P(x) + s12 * Qf(x)
    f2 = Qd(x) - s11 * Qf(x) + s22 * P(x)
    p, q = R.ldg_solve(s11, s12, -s11, s22, f1, f2, dx)
    return np.abs(p - P(x)).max(), np.abs(q - Qf(x)).max()


def test_ldg_solve_converges_at_second_order():
    e = [_manufactured(n) for n in (20, 40, 80)]
    for (p1, q1), (p2, q2) in zip(e, e[1:]):
        assert 3.6 < p1 / p2 < 4.4 and 3.6 < q1 / q2 < 4.4, e
    assert e[-1][0] < 2e-4 and e[-1][1] < 1e-4


def test_predictor_conserves_mass_between_walls():
    rng = np.random.default_rng(3)
    n, dx = 64, 0.5
    x = R.node_x(n, dx)
    Q = np.stack([2.0 + 0.1 * np.sin(0.3 * x) + 0.01 * rng.standard_normal((n, 2)),
                  0.2 * np.cos(0.2 * x), 0.05 * np.sin(x)])
    m0 = Q[0].sum()
    body = S.Body(kind=S.BODY_GAUSS, law=S.LAW_CONST_VEL, amp=0.2, length=2.0, x0=10.0,
                  q=(0.5, 0, 0, 0, 0))
    t = 0.0
    for _ in range(50):
        Q = R.predict(Q, 2.0, body, t, 0.02, dx)
        t += 0.02
    assert abs(Q[0].sum() - m0) <= 1e-13 * m0


def _standing_wave_error(n, L=20.0, d=1.0, a=1e-7, T=4.0):
    """hydrostatic predictor alone on eta = a cos(k x), k = pi / L (one
    half-wavelength between the walls); exact linear solution
    eta = a cos(k x) cos(w t), w = k sqrt(g d)"""
    dx = L / n
    x = R.node_x(n, dx)
    k = math.pi / L
    Q = np.stack([d + a * np.cos(k * x), np.zeros_like(x), np.zeros_like(x)])
    dt = 0.2 * dx / math.sqrt(9.81 * d)
    steps = int(round(T / dt))
    t = 0.0
    for _ in range(steps):
        Q = R.predict(Q, d, S.Body(), t, dt, dx)
        t += dt
    w = k * math.sqrt(9.81 * d)
    return np.abs(Q[0] - d - a * np.cos(k * x) * math.cos(w * t)).max() / a


def test_predictor_converges_to_the_linear_standing_wave():
    e1, e2 = _standing_wave_error(40), _standing_wave_error(80)
    # second order (a / d = 1e-7 keeps the nonlinear terms below the errors)
    assert e2 < 2e-4 and 3.6 < e1 / e2 < 4.4, (e1, e2)


def test_nonhydrostatic_step_gives_the_green_naghdi_dispersion():
    """standing wave cos(k x) between walls with kd = 1: the mode's first
    zero crossing comes at a quarter period of w^2 = g d k^2 / (1 + (kd)^2 / 3)"""
    d, a, kd = 1.0, 1e-4, 1.0
    k = kd / d
    L = math.pi / k * 4          # four half-wavelengths between the walls
    n = 160
    dx = L / n
    x = R.node_x(n, dx)
    mode = np.cos(k * x)
    Q = np.stack([d + a * mode, np.zeros_like(x), np.zeros_like(x)])
    w = math.sqrt(9.81 * d * k * k / (1 + kd * kd / 3))
    dt = 0.2 * dx / math.sqrt(9.81 * d)  # Courant 0.2: P1 with Heun is stable below about 1/3
    proj = lambda Q: np.sum((Q[0] - d) * mode) / np.sum(mode * mode)
    t, ap = 0.0, proj(Q)
    while True:
        Q, p = R.step(Q, d, S.Body(), t, dt, dx)
        an = proj(Q)
        if an <= 0:
            tq = t + dt * ap / (ap - an)
            break
        t, ap = t + dt, an
    assert abs(tq - 0.5 * math.pi / w) < 0.01 * (0.5 * math.pi / w), (tq, 0.5 * math.pi / w)
    # the hydrostatic quarter period is 13% shorter: the test tells them apart
    assert abs(0.5 * math.pi / (k * math.sqrt(9.81 * d)) - tq) > 0.1 * tq


def _flume_body():
    """the flume of Sec. 4.3 (Fr = 0.25 law of Eq. 21) with a smooth Gaussian
    body of the quartic block's height: the quartic's slope jumps at its
    ends, where the bottom's second derivative is a delta that point
    evaluation at nodes and centred differences treat differently"""
    base = S.whittaker_case(fr_index=1)
    return dataclasses.replace(base.body, kind=S.BODY_GAUSS, amp=0.026, length=0.15)


def _fv_flume(body, dx, dt, T, length=30.0, h0=0.175):
    n = int(round(length / dx))
    ds = np.full(n, h0)
    d0, *_ = O.forcing_1d(ds, dx, body, 0.0)
    c = S.Case1D(n=n, dx=dx, ds=ds, h=d0.copy(), hu=np.zeros(n), hw=np.zeros(n), body=body)
    sim = O.Sim1D(c, O.phys_struct(crit=S.CRIT_GLOBAL), cfl=0.0, dt_fixed=dt)
    sim.step(int(round(T / dt)))
    d_end, *_ = O.forcing_1d(ds, dx, body, sim.time)
    return (np.arange(n) + 0.5) * dx, sim.h - d_end, sim.time


def test_moving_bottom_terms_agree_with_the_finite_volume_reading():
    """a body moved by the law of Eq. 21 in the global model for 1.5 s: the
    RKDG/LDG oracle approaches the finite-volume oracle on a fine grid as it
    is refined, to within the finite-volume grid's own error (3-6%: its
    minmod slopes converge slowly at the wave's crests)"""
    body, T = _flume_body(), 1.5
    xf, ef, tf = _fv_flume(body, 0.009375, 0.000625, T)
    assert np.abs(ef).max() > 2e-3  # the body has made a wave
    errs = []
    for n, dt in ((400, 0.005), (800, 0.0025)):
        dx = 30.0 / n
        x = R.node_x(n, dx)
        Q = np.stack([R.bottom(0.175, body, x, 0.0)[0], np.zeros_like(x), np.zeros_like(x)])
        Q, p, t = R.run(Q, 0.175, body, 0.0, dt, int(round(T / dt)), dx)
        assert abs(t - tf) < 1e-9
        eta = Q[0] - R.bottom(0.175, body, x, t)[0]
        ref = np.interp(x.mean(axis=1), xf, ef)
        errs.append(np.linalg.norm(eta.mean(axis=1) - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.6 * errs[0] and errs[1] < 0.05, errs


def test_predictor_stage_two_sees_the_bottom_at_the_new_time():
    """still water over a moving body at time t is balanced by the bottom at
    t, so the first Heun stage leaves it unchanged; the second stage sees
    the bottom at t + dt (Heun as printed), which has moved: the momentum it
    adds scales with dt^2 (the slope change times dt / 2)"""
    body = _flume_body()
    n, dx, t = 400, 0.075, 0.8
    x = R.node_x(n, dx)
    Q = np.stack([R.bottom(0.175, body, x, t)[0], np.zeros_like(x), np.zeros_like(x)])
    assert np.abs(R.operator(Q, dx, R.p1_slope(Q[0], dx))).max() < 1e-12
    m = [np.abs(R.predict(Q, 0.175, body, t, dt, dx)[1]).max() for dt in (2e-3, 1e-3)]
    assert m[1] > 1e-8 and 3.6 < m[0] / m[1] < 4.4, m
