"""Plain FP64 CPU oracle of the adaptive non-hydrostatic SWE step.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports it, and it
shares no code with the HIP library.  Each function wraps one routine of
oracle/swe_oracle.c; see that file for the paper passages each one follows.

Parity status: every function here is pinned by the CPU test suite
(tests/test_oracle_*.py) against closed forms, invariants, brute force or the
paper's printed values, except the 2D extension, which the paper does not
contain: its pins are reductions (y-invariant data equals the 1D oracle,
x<->y transpose symmetry, lake at rest, mass, dense solve, the 2D linear
dispersion relation).  oracle/rkdg1d.py is the paper's own discretisation
(RKDG-P1 predictor, LDG-P1 elliptic solve) in NumPy, pinned by
tests/test_oracle_rkdg.py.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build_oracle

_LIB = None

OK, EINVAL, ENOCONV, EDRY, ENAN = 0, -1, -2, -3, -4


class OrcBody(C.Structure):
    _fields_ = [("kind", C.c_int32), ("law", C.c_int32), ("amp", C.c_double), ("len", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("dir", C.c_double),
                ("q", C.c_double * 5)]


class OrcPhys(C.Structure):
    _fields_ = [("g", C.c_double), ("rho", C.c_double), ("k_nh", C.c_double),
                ("crit", C.c_int32), ("enlarge", C.c_int32), ("first_global", C.c_int32),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("tensor", C.c_int32)]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(build_oracle.LIB):
            build_oracle.build()
        _LIB = C.CDLL(build_oracle.LIB)
        _LIB.orc_max_speed_1d.restype = C.c_double
        _LIB.orc_max_rate_2d.restype = C.c_double
    return _LIB


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def body_struct(body) -> OrcBody:
    b = OrcBody()
    b.kind, b.law = int(body.kind), int(body.law)
    b.amp, b.len, b.x0, b.y0, b.dir = body.amp, body.length, body.x0, body.y0, body.dir
    for i in range(5):
        b.q[i] = float(body.q[i])
    return b


def phys_struct(g=9.81, rho=1000.0, k_nh=1e-3, crit=6, enlarge=1, first_global=1, tol=1e-13,
                max_iter=100000, tensor=0) -> OrcPhys:
    return OrcPhys(g, rho, k_nh, int(crit), int(enlarge), int(first_global), tol, int(max_iter),
                   int(tensor))


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where} returned status {code}")
        self.code = code


def _check(code, where):
    if code < 0:
        raise OracleError(code, where)
    return code


# ---------------------------------------------------------------- forcing ---

def body_motion(body, t):
    X, Xd, Xdd = C.c_double(), C.c_double(), C.c_double()
    b = body_struct(body)
    lib().orc_body_motion(C.byref(b), C.c_double(t), C.byref(X), C.byref(Xd), C.byref(Xdd))
    return X.value, Xd.value, Xdd.value


def forcing_1d(ds, dx, body, t):
    ds = _f64(ds)
    n = ds.size
    out = [np.empty(n) for _ in range(4)]
    b = body_struct(body)
    lib().orc_forcing_1d(C.c_int32(n), C.c_double(dx), _p(ds), C.byref(b), C.c_double(t),
                         *[_p(o) for o in out])
    return tuple(out)  # d, d_t, d_tt, d_xt


def forcing_2d(ds, dx, dy, body, t):
    ds = _f64(ds)
    ny, nx = ds.shape
    out = [np.empty((ny, nx)) for _ in range(5)]
    b = body_struct(body)
    lib().orc_forcing_2d(C.c_int32(nx), C.c_int32(ny), C.c_double(dx), C.c_double(dy), _p(ds),
                         C.byref(b), C.c_double(t), *[_p(o) for o in out])
    return tuple(out)  # d, d_t, d_tt, d_xt, d_yt


# --------------------------------------------------------------------- 1D ---

def max_speed_1d(h, hu, g=9.81):
    h, hu = _f64(h), _f64(hu)
    return lib().orc_max_speed_1d(C.c_int32(h.size), _p(h), _p(hu), C.c_double(g))


def operator_1d(d, h, hu, hw, dx, g=9.81):
    d, h, hu, hw = map(_f64, (d, h, hu, hw))
    n = h.size
    L = [np.empty(n) for _ in range(3)]
    _check(lib().orc_operator_1d(C.c_int32(n), C.c_double(dx), C.c_double(g), _p(d), _p(h), _p(hu),
                                 _p(hw), *[_p(x) for x in L]), "operator_1d")
    return tuple(L)


def predict_1d(case_or_ds, dx, body, phys, t, dt, h, hu, hw):
    ds = _f64(case_or_ds)
    h, hu, hw = map(_f64, (h, hu, hw))
    n = h.size
    out = [np.empty(n) for _ in range(3)]
    b = body_struct(body)
    _check(lib().orc_predict_1d(C.c_int32(n), C.c_double(dx), _p(ds), C.byref(b), C.byref(phys),
                                C.c_double(t), C.c_double(dt), _p(h), _p(hu), _p(hw),
                                *[_p(o) for o in out]), "predict_1d")
    return tuple(out)


def indicator_1d(ds, dx, body, phys, t1, ht, mt, kt):
    ds, ht, mt, kt = map(_f64, (ds, ht, mt, kt))
    ind = np.empty(ht.size)
    b = body_struct(body)
    _check(lib().orc_indicator_1d(C.c_int32(ht.size), C.c_double(dx), _p(ds), C.byref(b),
                                  C.byref(phys), C.c_double(t1), _p(ht), _p(mt), _p(kt), _p(ind)),
           "indicator_1d")
    return ind


def mask_1d(ds, dx, body, phys, t1, ht, mt, kt, first_step=False):
    ds, ht, mt, kt = map(_f64, (ds, ht, mt, kt))
    mask = np.zeros(ht.size, dtype=np.uint8)
    b = body_struct(body)
    cnt = _check(lib().orc_mask_1d(C.c_int32(ht.size), C.c_double(dx), _p(ds), C.byref(b),
                                   C.byref(phys), C.c_double(t1), C.c_int32(int(first_step)),
                                   _p(ht), _p(mt), _p(kt), _p(mask)), "mask_1d")
    return mask, cnt


def nh_coeffs_1d(ds, dx, body, phys, t1, dt, ht, mt, kt):
    ds, ht, mt, kt = map(_f64, (ds, ht, mt, kt))
    n = ht.size
    cell = np.empty((8, n))
    face = np.empty((8, n + 1))
    b = body_struct(body)
    _check(lib().orc_nh_coeffs_1d(C.c_int32(n), C.c_double(dx), _p(ds), C.byref(b), C.byref(phys),
                                  C.c_double(t1), C.c_double(dt), _p(ht), _p(mt), _p(kt), _p(cell),
                                  _p(face)), "nh_coeffs_1d")
    names_c = ["D", "alpha", "phi", "s22", "f2", "d_t", "eta_x", "u"]
    names_f = ["h", "D", "s11", "K", "a", "b", "qpred", "fd"]
    return ({k: cell[i] for i, k in enumerate(names_c)}, {k: face[i] for i, k in enumerate(names_f)})


def nh_system_1d(ds, dx, body, phys, t1, dt, ht, mt, kt, mask):
    ds, ht, mt, kt = map(_f64, (ds, ht, mt, kt))
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    n = ht.size
    dg, up, rh = np.empty(n), np.empty(n), np.empty(n)
    b = body_struct(body)
    _check(lib().orc_nh_system_1d(C.c_int32(n), C.c_double(dx), _p(ds), C.byref(b), C.byref(phys),
                                  C.c_double(t1), C.c_double(dt), _p(ht), _p(mt), _p(kt),
                                  _p(mask), _p(dg), _p(up), _p(rh)), "nh_system_1d")
    return dg, up, rh


def tridiag_solve(diag, upper, rhs):
    diag, upper, rhs = map(_f64, (diag, upper, rhs))
    x = np.empty(diag.size)
    _check(lib().orc_tridiag_solve(C.c_int32(diag.size), _p(diag), _p(upper), _p(rhs), _p(x)),
           "tridiag_solve")
    return x


def nh_correct_1d(ds, dx, body, phys, t1, dt, ht, mt, kt, mask, p):
    ds, ht, mt, kt, p = map(_f64, (ds, ht, mt, kt, p))
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    n = ht.size
    mo, ko = np.empty(n), np.empty(n)
    b = body_struct(body)
    _check(lib().orc_nh_correct_1d(C.c_int32(n), C.c_double(dx), _p(ds), C.byref(b), C.byref(phys),
                                   C.c_double(t1), C.c_double(dt), _p(ht), _p(mt), _p(kt),
                                   _p(mask), _p(p), _p(mo), _p(ko)), "nh_correct_1d")
    return mo, ko


class Sim1D:
    """time loop over orc_step_1d; state arrays are updated in place"""

    def __init__(self, case, phys, cfl=0.5, dt_fixed=0.0):
        self.n, self.dx = case.n, case.dx
        self.ds = _f64(case.ds).copy()
        self.h, self.hu, self.hw = _f64(case.h).copy(), _f64(case.hu).copy(), _f64(case.hw).copy()
        self.p = np.zeros(self.n)
        self.mask = np.zeros(self.n, dtype=np.uint8)
        self.body = body_struct(case.body)
        self.phys = phys
        self.cfl, self.dt_fixed = cfl, dt_fixed
        self.t = C.c_double(case.t0)
        self.step_index = 0
        self.last_dt = 0.0
        self.last_active = 0

    def step(self, nsteps=1):
        dt, na = C.c_double(), C.c_int32()
        for _ in range(nsteps):
            _check(lib().orc_step_1d(C.c_int32(self.n), C.c_double(self.dx), _p(self.ds),
                                     C.byref(self.body), C.byref(self.phys), C.c_double(self.cfl),
                                     C.c_double(self.dt_fixed), C.c_int32(self.step_index),
                                     C.byref(self.t), _p(self.h), _p(self.hu), _p(self.hw),
                                     _p(self.p), _p(self.mask), C.byref(dt), C.byref(na)),
                   "step_1d")
            self.step_index += 1
            self.last_dt, self.last_active = dt.value, na.value
        return self

    @property
    def time(self):
        return self.t.value


# --------------------------------------------------------------------- 2D ---

def max_rate_2d(h, hu, hv, dx, dy, g=9.81):
    h, hu, hv = map(_f64, (h, hu, hv))
    ny, nx = h.shape
    return lib().orc_max_rate_2d(C.c_int32(nx), C.c_int32(ny), C.c_double(dx), C.c_double(dy),
                                 _p(h), _p(hu), _p(hv), C.c_double(g))


def operator_2d(d, h, hu, hv, hw, dx, dy, g=9.81):
    d, h, hu, hv, hw = map(_f64, (d, h, hu, hv, hw))
    ny, nx = h.shape
    L = [np.empty((ny, nx)) for _ in range(4)]
    _check(lib().orc_operator_2d(C.c_int32(nx), C.c_int32(ny), C.c_double(dx), C.c_double(dy),
                                 C.c_double(g), _p(d), _p(h), _p(hu), _p(hv), _p(hw),
                                 *[_p(x) for x in L]), "operator_2d")
    return tuple(L)


def predict_2d(ds, dx, dy, body, phys, t, dt, h, hu, hv, hw):
    ds, h, hu, hv, hw = map(_f64, (ds, h, hu, hv, hw))
    ny, nx = h.shape
    out = [np.empty((ny, nx)) for _ in range(4)]
    b = body_struct(body)
    _check(lib().orc_predict_2d(C.c_int32(nx), C.c_int32(ny), C.c_double(dx), C.c_double(dy),
                                _p(ds), C.byref(b), C.byref(phys), C.c_double(t), C.c_double(dt),
                                _p(h), _p(hu), _p(hv), _p(hw), *[_p(o) for o in out]),
           "predict_2d")
    return tuple(out)


def indicator_2d(ds, dx, dy, body, phys, t1, ht, mt, nt, kt):
    ds, ht, mt, nt, kt = map(_f64, (ds, ht, mt, nt, kt))
    ny, nx = ht.shape
    ind = np.empty((ny, nx))
    b = body_struct(body)
    _check(lib().orc_indicator_2d(C.c_int32(nx), C.c_int32(ny), C.c_double(dx), C.c_double(dy),
                                  _p(ds), C.byref(b), C.byref(phys), C.c_double(t1), _p(ht),
                                  _p(mt), _p(nt), _p(kt), _p(ind)), "indicator_2d")
    return ind


def mask_2d(ds, dx, dy, body, phys, t1, ht, mt, nt, kt, first_step=False):
    ds, ht, mt, nt, kt = map(_f64, (ds, ht, mt, nt, kt))
    ny, nx = ht.shape
    mask = np.zeros((ny, nx), dtype=np.uint8)
    b = body_struct(body)
    cnt = _check(lib().orc_mask_2d(C.c_int32(nx), C.c_int32(ny), C.c_double(dx), C.c_double(dy),
                                   _p(ds), C.byref(b), C.byref(phys), C.c_double(t1),
                                   C.c_int32(int(first_step)), _p(ht), _p(mt), _p(nt), _p(kt),
                                   _p(mask)), "mask_2d")
    return mask, cnt


def nh_coeffs_2d(ds, dx, dy, body, phys, t1, dt, ht, mt, nt, kt):
    ds, ht, mt, nt, kt = map(_f64, (ds, ht, mt, nt, kt))
    ny, nx = ht.shape
    cell = np.empty((7, ny, nx))
    xf = np.empty((5, ny, nx + 1))
    yf = np.empty((5, ny + 1, nx))
    b = body_struct(body)
    _check(lib().orc_nh_coeffs_2d(C.c_int32(nx), C.c_int32(ny), C.c_double(dx), C.c_double(dy),
                                  _p(ds), C.byref(b), C.byref(phys), C.c_double(t1),
                                  C.c_double(dt), _p(ht), _p(mt), _p(nt), _p(kt), _p(cell),
                                  _p(xf), _p(yf)), "nh_coeffs_2d")
    return cell, xf, yf


def nh_pairs_2d(ds, dx, dy, body, t1, xf, yf):
    """the exact-tensor operator's off-diagonal entry per owner cell [ny, nx]"""
    ds = _f64(ds)
    ny, nx = ds.shape
    kxy = np.empty((ny, nx))
    b = body_struct(body)
    _check(lib().orc_nh_pairs_2d(C.c_int32(nx), C.c_int32(ny), C.c_double(dx), C.c_double(dy),
                                 _p(ds), C.byref(b), C.c_double(t1), _p(_f64(xf)), _p(_f64(yf)),
                                 _p(kxy)), "nh_pairs_2d")
    return kxy


def nh_apply_2d(cell, xf, yf, mask, p, kxy=None):
    """A p; kxy (from nh_pairs_2d) selects the exact-tensor operator"""
    ny, nx = mask.shape
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    p = _f64(p)
    out = np.empty((ny, nx))
    kxy = None if kxy is None else _f64(kxy)
    lib().orc_nh_apply7_2d(C.c_int32(nx), C.c_int32(ny), _p(cell), _p(xf), _p(yf), _p(kxy),
                           _p(mask), _p(p), _p(out))
    return out


def nh_rhs_2d(cell, xf, yf, mask):
    ny, nx = mask.shape
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.empty((ny, nx))
    lib().orc_nh_rhs_2d(C.c_int32(nx), C.c_int32(ny), _p(cell), _p(xf), _p(yf), _p(mask), _p(out))
    return out


def cg_2d(cell, xf, yf, mask, rhs, tol=1e-13, max_iter=100000, x0=None, kxy=None):
    ny, nx = mask.shape
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    rhs = _f64(rhs)
    x = np.zeros((ny, nx)) if x0 is None else _f64(x0).copy()
    it, rr = C.c_int32(), C.c_double()
    kxy = None if kxy is None else _f64(kxy)
    _check(lib().orc_cg7_2d(C.c_int32(nx), C.c_int32(ny), _p(cell), _p(xf), _p(yf), _p(kxy),
                            _p(mask), _p(rhs), C.c_double(tol), C.c_int32(max_iter), _p(x),
                            C.byref(it), C.byref(rr)), "cg_2d")
    return x, it.value, rr.value


def nh_correct_2d(cell, xf, yf, dt, rho, mt, nt, kt, mask, p, kxy=None):
    mt, nt, kt, p = map(_f64, (mt, nt, kt, p))
    ny, nx = mt.shape
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    mo, no, ko = np.empty((ny, nx)), np.empty((ny, nx)), np.empty((ny, nx))
    kxy = None if kxy is None else _f64(kxy)
    lib().orc_nh_correct7_2d(C.c_int32(nx), C.c_int32(ny), _p(cell), _p(xf), _p(yf), _p(kxy),
                             C.c_double(dt), C.c_double(rho), _p(mt), _p(nt), _p(kt), _p(mask),
                             _p(p), _p(mo), _p(no), _p(ko))
    return mo, no, ko


class Sim2D:
    def __init__(self, case, phys, cfl=0.5, dt_fixed=0.0):
        self.nx, self.ny, self.dx, self.dy = case.nx, case.ny, case.dx, case.dy
        self.ds = _f64(case.ds).copy()
        self.h, self.hu, self.hv, self.hw = (_f64(a).copy() for a in (case.h, case.hu, case.hv, case.hw))
        self.p = np.zeros((self.ny, self.nx))
        self.mask = np.zeros((self.ny, self.nx), dtype=np.uint8)
        self.body = body_struct(case.body)
        self.phys = phys
        self.cfl, self.dt_fixed = cfl, dt_fixed
        self.t = C.c_double(case.t0)
        self.step_index = 0
        self.last_dt = 0.0
        self.last_active = 0
        self.last_iters = 0
        self.last_res = 0.0

    def step(self, nsteps=1):
        dt, na, it, rr = C.c_double(), C.c_int32(), C.c_int32(), C.c_double()
        for _ in range(nsteps):
            _check(lib().orc_step_2d(C.c_int32(self.nx), C.c_int32(self.ny), C.c_double(self.dx),
                                     C.c_double(self.dy), _p(self.ds), C.byref(self.body),
                                     C.byref(self.phys), C.c_double(self.cfl),
                                     C.c_double(self.dt_fixed), C.c_int32(self.step_index),
                                     C.byref(self.t), _p(self.h), _p(self.hu), _p(self.hv),
                                     _p(self.hw), _p(self.p), _p(self.mask), C.byref(dt),
                                     C.byref(na), C.byref(it), C.byref(rr)), "step_2d")
            self.step_index += 1
            self.last_dt, self.last_active = dt.value, na.value
            self.last_iters, self.last_res = it.value, rr.value
        return self

    @property
    def time(self):
        return self.t.value
