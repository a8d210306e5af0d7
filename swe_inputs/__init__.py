"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package holds no arithmetic of the method itself: only grids, static
depth fields, initial states, body parameters and random numbers.  Both the
HIP path and the CPU oracle receive the arrays it produces.

Workloads (shapes and distributions follow the paper's test problems and the
synthetic configurations described in the design notes):
  * solitary wave over a flat bottom (Sec. 4.1, Eq. 18), exact Serre solution;
  * 1D moving-bottom slide: quartic block (Eq. 20) sliding down a slope;
  * ensemble of uneven-length 1D slide channels with seeded parameters;
  * 2D shelf with a seeded Gaussian-correlated bathymetry perturbation and a
    translating Gaussian mound;
  * Whittaker-type slide with the piecewise law of Eq. 21 (Table 2 parameters).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

G = 9.81
RHO = 1000.0

# criterion codes (Sec. 5.1), shared numbering of the public interface
CRIT_ETA_D, CRIT_ETA_X, CRIT_U, CRIT_U_X, CRIT_W, CRIT_W_X, CRIT_GLOBAL, CRIT_NONE = range(8)
CRIT_NAMES = {"eta_d": 0, "eta_x": 1, "u": 2, "u_x": 3, "w": 4, "w_x": 5, "global": 6, "none": 7}

BODY_NONE, BODY_QUARTIC, BODY_GAUSS = 0, 1, 2
LAW_FIXED, LAW_CONST_VEL, LAW_SIN_RAMP, LAW_PIECEWISE = 0, 1, 2, 3


@dataclasses.dataclass
class Body:
    """Rigid body carried by the bottom: d(x,t) = d_s(x) - B(x - X(t)),
    X(t) = x0 + dir * s(t)."""
    kind: int = BODY_NONE
    law: int = LAW_FIXED
    amp: float = 0.0
    length: float = 1.0
    x0: float = 0.0
    y0: float = 0.0
    dir: float = 1.0
    q: tuple = (0.0, 0.0, 0.0, 0.0, 0.0)


@dataclasses.dataclass
class Case1D:
    n: int
    dx: float
    ds: np.ndarray
    h: np.ndarray
    hu: np.ndarray
    hw: np.ndarray
    body: Body
    t0: float = 0.0


@dataclasses.dataclass
class Case2D:
    nx: int
    ny: int
    dx: float
    dy: float
    ds: np.ndarray   # [ny, nx]
    h: np.ndarray
    hu: np.ndarray
    hv: np.ndarray
    hw: np.ndarray
    body: Body
    t0: float = 0.0


# ----------------------------------------------------------------------------
# solitary wave (Sec. 4.1, Eq. 18)
# ----------------------------------------------------------------------------

def solitary_params(a: float, d: float, g: float = G):
    """celerity c = sqrt(g (d + a)) and scaling K = sqrt(3a / (4 d^2 (d + a)))"""
    c = math.sqrt(g * (d + a))
    K = math.sqrt(3.0 * a / (4.0 * d * d * (d + a)))
    return c, K


def solitary_exact(x, t, a, d, x0, g: float = G):
    """Serre solitary wave: eta, u, and hw from the divergence constraint
    (Eq. 4 over a flat static bottom gives hw = -(c d / 2) eta_x)."""
    c, K = solitary_params(a, d, g)
    xi = K * (np.asarray(x, dtype=np.float64) - c * t - x0)
    sech2 = 1.0 / np.cosh(xi) ** 2
    eta = a * sech2
    u = c * eta / (d + eta)
    eta_x = -2.0 * a * K * sech2 * np.tanh(xi)
    hw = -0.5 * c * d * eta_x
    return eta, u, hw


def solitary_case(n=2000, length=200.0, d=1.0, a=0.2, x0=None, g: float = G) -> Case1D:
    dx = length / n
    x = (np.arange(n) + 0.5) * dx
    if x0 is None:
        x0 = length / 4.0
    eta, u, hw = solitary_exact(x, 0.0, a, d, x0, g)
    h = d + eta
    return Case1D(n=n, dx=dx, ds=np.full(n, d), h=h, hu=h * u, hw=hw, body=Body())


# ----------------------------------------------------------------------------
# 1D moving-bottom slide
# ----------------------------------------------------------------------------

def slope_depth(n, dx, h0=0.4, d_wall=0.10, theta_deg=15.0):
    """static depth rising linearly from d_wall at the x = 0 wall to h0"""
    x = (np.arange(n) + 0.5) * dx
    return np.minimum(h0, d_wall + x * math.tan(math.radians(theta_deg)))


def slide_body(theta_deg=15.0, length=0.4, height=0.05, x_start=0.25, s_final=1.0, t_ramp=2.0):
    """quartic block (Eq. 20) centred at x_start, displaced along the slope by
    s(t) = (s_f / 2)(1 - cos(pi t / T_s)) (sinusoidal ramp), X = x0 + cos(theta) s"""
    return Body(kind=BODY_QUARTIC, law=LAW_SIN_RAMP, amp=height, length=length, x0=x_start,
                dir=math.cos(math.radians(theta_deg)), q=(s_final, t_ramp, 0.0, 0.0, 0.0))


def slide_case(n=32768, dx=0.005, h0=0.4, theta_deg=15.0, length=0.4, height=0.05) -> Case1D:
    ds = slope_depth(n, dx, h0=h0, theta_deg=theta_deg)
    body = slide_body(theta_deg=theta_deg, length=length, height=height)
    # lake at rest over the body at t = 0: eta = 0 -> h = d(x, 0)
    h = ds - _body_profile_1d(n, dx, body, 0.0)
    return Case1D(n=n, dx=dx, ds=ds, h=h, hu=np.zeros(n), hw=np.zeros(n), body=body)


def _body_profile_1d(n, dx, body: Body, t: float, x=None):
    """B(x - X(0)) for the quartic body at rest at its start position (used
    only to lay down the still-water initial state; the solvers evaluate the
    moving bottom themselves); x: the points (default: cell centres)"""
    if x is None:
        x = (np.arange(n) + 0.5) * dx
    assert t == 0.0
    xi = np.asarray(x, dtype=np.float64) - body.x0
    if body.kind == BODY_QUARTIC:
        z = 2.0 * xi / body.length
        return np.where(np.abs(xi) < 0.5 * body.length, body.amp * (1.0 - z ** 4), 0.0)
    if body.kind == BODY_GAUSS:
        return body.amp * np.exp(-(xi * xi) / body.length ** 2)
    return np.zeros(np.shape(xi))


def whittaker_case(fr_index=1, n=None, dx=0.075, h0=0.175, length_domain=30.0) -> Case1D:
    """flat flume with a quartic slide moved by the piecewise law of Eq. 21;
    Table 2 gives (a0, u_t, t1, t2, t3) for Fr = 0.125, 0.25, 0.375."""
    table = [(1.5, 0.163, 0.109, 2.109, 2.218),
             (1.5, 0.327, 0.218, 2.218, 2.436),
             (1.5, 0.491, 0.327, 2.327, 2.654)]
    if n is None:
        n = int(round(length_domain / dx))
    body = Body(kind=BODY_QUARTIC, law=LAW_PIECEWISE, amp=0.026, length=0.5, x0=2.0, dir=1.0,
                q=table[fr_index])
    ds = np.full(n, h0)
    h = ds - _body_profile_1d(n, dx, body, 0.0)
    return Case1D(n=n, dx=dx, ds=ds, h=h, hu=np.zeros(n), hw=np.zeros(n), body=body)


# ----------------------------------------------------------------------------
# node values [3, n, 2] (h, hu, hw at the two ends of each P1 element
# [i dx, (i + 1) dx]) for the paper's own discretisation
# ----------------------------------------------------------------------------

def dg_nodes(n, dx):
    x0 = np.arange(n) * dx
    return np.stack([x0, x0 + dx], axis=1)


def dg_solitary_state(n, dx, a, d, x0, g: float = G):
    """the Serre solitary wave at t = 0 at the element nodes"""
    eta, u, hw = solitary_exact(dg_nodes(n, dx), 0.0, a, d, x0, g)
    h = d + eta
    return np.stack([h, h * u, hw])


def dg_still_water_state(n, dx, h0, body: Body):
    """still water over the body at rest at its start position, flat static
    depth h0"""
    x = dg_nodes(n, dx)
    h = h0 - _body_profile_1d(n, dx, body, 0.0, x=x)
    return np.stack([h, np.zeros_like(h), np.zeros_like(h)])


@dataclasses.dataclass
class Ensemble:
    channels: List[Case1D]

    @property
    def lengths(self):
        return [c.n for c in self.channels]

    @property
    def offsets(self):
        return np.concatenate([[0], np.cumsum(self.lengths)]).astype(np.int64)

    def packed(self, name):
        return np.concatenate([getattr(c, name) for c in self.channels])


def ensemble_case(n_channels=512, n_min=4096, n_max=65536, seed=17026, dx=0.005, h0=0.4) -> Ensemble:
    """independent slide channels with lengths ~ U{n_min..n_max} and
    L_s ~ U[0.2, 0.6], H_s ~ U[0.02, 0.08], theta ~ U[10, 20] degrees"""
    rng = np.random.default_rng(seed)
    lens = rng.integers(n_min, n_max + 1, size=n_channels)
    Ls = rng.uniform(0.2, 0.6, size=n_channels)
    Hs = rng.uniform(0.02, 0.08, size=n_channels)
    th = rng.uniform(10.0, 20.0, size=n_channels)
    chans = []
    for c in range(n_channels):
        n = int(lens[c])
        ds = slope_depth(n, dx, h0=h0, theta_deg=float(th[c]))
        body = slide_body(theta_deg=float(th[c]), length=float(Ls[c]), height=float(Hs[c]),
                          x_start=0.25 + 0.5 * float(Ls[c]))
        h = ds - _body_profile_1d(n, dx, body, 0.0)
        chans.append(Case1D(n=n, dx=dx, ds=ds, h=h, hu=np.zeros(n), hw=np.zeros(n), body=body))
    return Ensemble(chans)


# ----------------------------------------------------------------------------
# 2D shelf with a Gaussian-correlated perturbation and a moving mound
# ----------------------------------------------------------------------------

def gaussian_field_2d(nx, ny, dx, dy, sigma, ell, seed):
    """white noise convolved periodically with a Gaussian kernel so that the
    covariance is exp(-r^2 / (2 ell^2)), rescaled to sample std sigma"""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, nx))
    kx = np.fft.fftfreq(nx, d=dx) * 2.0 * math.pi
    ky = np.fft.fftfreq(ny, d=dy) * 2.0 * math.pi
    KX, KY = np.meshgrid(kx, ky)
    # kernel with std ell / sqrt(2): its self-convolution has std ell
    s = ell / math.sqrt(2.0)
    filt = np.exp(-0.5 * (KX ** 2 + KY ** 2) * s * s)
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))
    f -= f.mean()
    sd = f.std()
    return f * (sigma / sd) if sd > 0 else f


def mound_body(amp=3.0, width=60.0, x0=400.0, y0=1024.0, speed=8.0):
    return Body(kind=BODY_GAUSS, law=LAW_CONST_VEL, amp=amp, length=width, x0=x0, y0=y0, dir=1.0,
                q=(speed, 0.0, 0.0, 0.0, 0.0))


def shelf_case_2d(nx=2048, ny=2048, dx=1.0, dy=1.0, h0=50.0, sigma=2.0, ell=40.0, seed=17025,
                  amp=3.0, width=60.0, x0=None, y0=None, speed=8.0) -> Case2D:
    ds = h0 + gaussian_field_2d(nx, ny, dx, dy, sigma, ell, seed)
    if x0 is None:
        x0 = 400.0 * nx / 2048.0
    if y0 is None:
        y0 = 0.5 * ny * dy
    body = mound_body(amp=amp, width=width, x0=x0, y0=y0, speed=speed)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    B = amp * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / width ** 2)
    h = ds - B
    z = np.zeros((ny, nx))
    return Case2D(nx=nx, ny=ny, dx=dx, dy=dy, ds=ds, h=h, hu=z.copy(), hv=z.copy(), hw=z.copy(),
                  body=body)


# ----------------------------------------------------------------------------
# generic random smooth states for stage-level parity tests
# ----------------------------------------------------------------------------

def smooth_noise(n, rng, scale, corr=8.0):
    w = rng.standard_normal(n + 64)
    k = np.exp(-0.5 * (np.arange(-32, 33) / corr) ** 2)
    f = np.convolve(w, k / k.sum(), mode="same")[32:32 + n]
    return scale * f / max(np.abs(f).max(), 1e-300)


def random_case_1d(n, seed, dx=0.05, h0=1.0, amp=0.05, mom=0.05, vert=0.01, body=None,
                   bottom=0.1) -> Case1D:
    rng = np.random.default_rng(seed)
    ds = h0 + smooth_noise(n, rng, bottom * h0)
    eta = smooth_noise(n, rng, amp * h0)
    h = ds + eta
    hu = smooth_noise(n, rng, mom) * h
    hw = smooth_noise(n, rng, vert) * h
    if body is None:
        body = Body(kind=BODY_QUARTIC, law=LAW_SIN_RAMP, amp=0.05 * h0, length=30 * dx,
                    x0=0.4 * n * dx, dir=0.97, q=(10 * dx, 0.5, 0, 0, 0))
    return Case1D(n=n, dx=dx, ds=ds, h=h, hu=hu, hw=hw, body=body, t0=0.1)


def random_case_2d(nx, ny, seed, dx=0.5, dy=0.5, h0=2.0, amp=0.05, mom=0.05, vert=0.01,
                   body=None) -> Case2D:
    rng = np.random.default_rng(seed)
    ds = h0 + 0.05 * h0 * gaussian_field_2d(nx, ny, dx, dy, 1.0, 4 * dx, int(rng.integers(1 << 30)))
    eta = amp * h0 * gaussian_field_2d(nx, ny, dx, dy, 1.0, 3 * dx, int(rng.integers(1 << 30)))
    h = ds + eta
    hu = mom * gaussian_field_2d(nx, ny, dx, dy, 1.0, 3 * dx, int(rng.integers(1 << 30))) * h
    hv = mom * gaussian_field_2d(nx, ny, dx, dy, 1.0, 3 * dx, int(rng.integers(1 << 30))) * h
    hw = vert * gaussian_field_2d(nx, ny, dx, dy, 1.0, 3 * dx, int(rng.integers(1 << 30))) * h
    if body is None:
        body = Body(kind=BODY_GAUSS, law=LAW_CONST_VEL, amp=0.05 * h0, length=4 * dx,
                    x0=0.4 * nx * dx, y0=0.5 * ny * dy, dir=1.0, q=(1.0, 0, 0, 0, 0))
    return Case2D(nx=nx, ny=ny, dx=dx, dy=dy, ds=ds, h=h, hu=hu, hv=hv, hw=hw, body=body, t0=0.05)


def hump_case_2d(nx, ny, seed, dx=1.0, h0=10.0, amp=0.01, radius=100.0, cx=None, cy=None,
                 body=None) -> Case2D:
    """a Gaussian hump of water, eta = amp h0 exp(-r^2 / radius^2), at rest
    over a seeded, gently perturbed bottom (2% of h0, correlation 4 dx): the
    non-hydrostatic area is a disc whose bounding box leaves much of the
    grid outside"""
    rng = np.random.default_rng(seed)
    ds = h0 + 0.02 * h0 * gaussian_field_2d(nx, ny, dx, dx, 1.0, 4 * dx, int(rng.integers(1 << 30)))
    cx = 0.4 * nx * dx if cx is None else cx
    cy = 0.55 * ny * dx if cy is None else cy
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(x, y)
    eta = amp * h0 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / radius ** 2)
    h = ds + eta
    z = np.zeros_like(h)
    if body is None:
        body = Body()
    return Case2D(nx=nx, ny=ny, dx=dx, dy=dx, ds=ds, h=h, hu=z, hv=z.copy(), hw=z.copy(),
                  body=body, t0=0.0)


def warm_start_case_2d(seed, n=1024, dx=2.0, h0=50.0) -> Case2D:
    """2D slide scenario for the learned warm start: the shelf of the 2D
    benchmark (50 m, Gaussian-correlated perturbation with std 2 m and
    correlation length 40 m) on an n x n grid of spacing dx, with a Gaussian
    mound (3 m, e-folding width 60 m, 8 m/s) whose start position and the
    bathymetry vary with the seed"""
    rng = np.random.default_rng(seed)
    L = n * dx
    x0 = float(rng.uniform(0.15, 0.35)) * L
    y0 = float(rng.uniform(0.35, 0.65)) * L
    return shelf_case_2d(nx=n, ny=n, dx=dx, dy=dx, h0=h0, sigma=2.0, ell=40.0, seed=seed,
                         amp=3.0, width=60.0, x0=x0, y0=y0, speed=8.0)
