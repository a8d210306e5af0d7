"""Pins of the 1D FP64 oracle against facts that do not come from the oracle
itself: closed forms, invariants, textbook solutions, brute force, dense
linear algebra, and the values the paper prints."""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle as O
import swe_inputs as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ forcing --

@pytest.mark.parametrize("body", [
    S.slide_body(theta_deg=15.0, length=0.4, height=0.05, s_final=1.0, t_ramp=2.0),
    S.Body(kind=S.BODY_GAUSS, law=S.LAW_CONST_VEL, amp=0.1, length=0.3, x0=1.0, q=(0.7, 0, 0, 0, 0)),
    S.Body(kind=S.BODY_QUARTIC, law=S.LAW_PIECEWISE, amp=0.026, length=0.5, x0=1.5,
           q=(1.5, 0.327, 0.218, 2.218, 2.436)),
])
@pytest.mark.parametrize("t", [0.05, 0.3, 1.0, 2.3])
def test_forcing_chain_rule_matches_finite_differences(body, t):
    """d_t, d_tt, d_xt of the moving bottom vs centred differences of d(x,t)"""
    n, dx = 4000, 0.001
    ds = np.full(n, 0.4)
    eps = 1e-4
    d0, dt_, dtt, dxt = O.forcing_1d(ds, dx, body, t)
    dp, *_ = O.forcing_1d(ds, dx, body, t + eps)
    dm, *_ = O.forcing_1d(ds, dx, body, t - eps)
    fd_t = (dp - dm) / (2 * eps)
    fd_tt = (dp - 2 * d0 + dm) / eps ** 2
    scale = max(np.abs(dt_).max(), 1e-12)
    # smooth part only: stay away from the body edges where B is not C^2
    X, _, _ = O.body_motion(body, t)
    x = (np.arange(n) + 0.5) * dx
    inner = np.abs(x - X) < 0.45 * body.length
    assert np.abs(fd_t - dt_)[inner].max() <= 1e-6 * scale + 1e-12
    if np.abs(dtt).max() > 0:
        assert np.abs(fd_tt - dtt)[inner].max() <= 1e-3 * np.abs(dtt).max() + 1e-7
    fd_xt = np.gradient(dt_, dx)
    assert np.abs(fd_xt - dxt)[inner][2:-2].max() <= 1e-3 * max(np.abs(dxt).max(), 1e-12) + 1e-9


def test_piecewise_law_is_continuous_and_stops():
    """Eq. 21 with Table 2 rows: s(t) continuous, and s' = 0 after t3"""
    for row in [(1.5, 0.163, 0.109, 2.109, 2.218), (1.5, 0.327, 0.218, 2.218, 2.436),
                (1.5, 0.491, 0.327, 2.327, 2.654)]:
        body = S.Body(kind=S.BODY_QUARTIC, law=S.LAW_PIECEWISE, amp=0.026, length=0.5, x0=0.0, q=row)
        for tk in row[2:]:
            a = O.body_motion(body, tk - 1e-9)[0]
            b = O.body_motion(body, tk + 1e-9)[0]
            assert abs(a - b) < 1e-8
        # acceleration a0 reaches the coasting speed: a0 t1 = u_t (Table 2)
        assert abs(row[0] * row[2] - row[1]) < 2e-3
        assert abs(O.body_motion(body, row[4] + 0.5)[1]) == 0.0
        assert abs(O.body_motion(body, row[2])[1] - row[0] * row[2]) < 1e-12


# ---------------------------------------------------------------- predictor --

def test_lake_at_rest_is_preserved():
    """hydrostatic reconstruction: still water over an uneven static bottom
    stays still, NH extension on everywhere (then phi = 0 and RHS = 0)"""
    rng = np.random.default_rng(1)
    n = 400
    ds = 1.0 + 0.3 * S.smooth_noise(n, rng, 1.0, corr=3.0)
    case = S.Case1D(n=n, dx=0.05, ds=ds, h=ds.copy(), hu=np.zeros(n), hw=np.zeros(n), body=S.Body())
    sim = O.Sim1D(case, O.phys_struct(crit=S.CRIT_GLOBAL), cfl=0.5).step(500)
    assert np.abs(sim.h - ds).max() < 1e-12
    assert np.abs(sim.hu).max() < 1e-12
    assert np.abs(sim.hw).max() < 1e-12


def test_mass_is_conserved_with_moving_bottom():
    """h is never corrected (Sec. 3.2) and wall fluxes vanish, so sum(h) dx is
    constant even with a moving body and an adaptive NH area"""
    case = S.random_case_1d(600, seed=3)
    for crit in (S.CRIT_GLOBAL, S.CRIT_ETA_D, S.CRIT_NONE):
        sim = O.Sim1D(case, O.phys_struct(crit=crit), cfl=0.45)
        m0 = sim.h.sum()
        sim.step(300)
        assert abs(sim.h.sum() - m0) <= 1e-13 * m0


def stoker(x, t, hl, hr, x0, g=9.81):
    """exact dam break over a flat wet bottom (rarefaction + shock)"""
    cl = math.sqrt(g * hl)

    def f(hm):
        um_r = 2.0 * (cl - math.sqrt(g * hm))
        um_s = (hm - hr) * math.sqrt(0.5 * g * (hm + hr) / (hm * hr))
        return um_r - um_s

    hm = brentq(f, hr, hl)
    um = 2.0 * (cl - math.sqrt(g * hm))
    s = hm * um / (hm - hr)
    xi = (x - x0) / t
    h = np.where(xi < -cl, hl, 0.0)
    rare = (xi >= -cl) & (xi < um - math.sqrt(g * hm))
    h = np.where(rare, (2.0 * cl - xi) ** 2 / (9.0 * g), h)
    h = np.where((xi >= um - math.sqrt(g * hm)) & (xi < s), hm, h)
    h = np.where(xi >= s, hr, h)
    return h


def test_stoker_dam_break_converges():
    """NH off: the predictor alone must converge to the textbook solution"""
    errs = []
    for n in (200, 400, 800):
        L = 100.0
        dx = L / n
        x = (np.arange(n) + 0.5) * dx
        h = np.where(x < 50.0, 2.0, 1.0)
        case = S.Case1D(n=n, dx=dx, ds=np.full(n, 1.0), h=h, hu=np.zeros(n), hw=np.zeros(n),
                        body=S.Body())
        sim = O.Sim1D(case, O.phys_struct(crit=S.CRIT_NONE), cfl=0.4)
        while sim.time < 5.0 - 1e-12:
            sim.step()
        ex = stoker(x, sim.time, 2.0, 1.0, 50.0)
        errs.append(np.abs(sim.h - ex).mean())
    assert errs[0] < 0.02
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1]


def test_mirror_symmetry():
    """reflecting the data (x -> L - x, hu -> -hu) reflects the step"""
    case = S.random_case_1d(300, seed=5, body=S.Body())
    mir = S.Case1D(n=case.n, dx=case.dx, ds=case.ds[::-1].copy(), h=case.h[::-1].copy(),
                   hu=-case.hu[::-1].copy(), hw=case.hw[::-1].copy(), body=S.Body())
    a = O.Sim1D(case, O.phys_struct(crit=S.CRIT_GLOBAL), cfl=0.4).step(20)
    b = O.Sim1D(mir, O.phys_struct(crit=S.CRIT_GLOBAL), cfl=0.4).step(20)
    assert np.allclose(a.h, b.h[::-1], rtol=0, atol=1e-12)
    assert np.allclose(a.hu, -b.hu[::-1], rtol=0, atol=1e-12)
    assert np.allclose(a.hw, b.hw[::-1], rtol=0, atol=1e-12)
    assert np.allclose(a.p, b.p[::-1], rtol=1e-9, atol=1e-9)


# ----------------------------------------------------------------- criteria --

def test_solitary_mask_closed_form():
    g = json.load(open(os.path.join(GOLD, "solitary_mask.json")))
    st, ex = g["setup"], g["expected"]
    a, d, n, L, x0 = st["a"], st["d"], st["n"], st["L"], st["x0"]
    _, K = S.solitary_params(a, d)
    half = math.acosh(math.sqrt(a / (1e-3 * d))) / K
    assert abs(half - ex["half_width_m"]) < 1e-5
    case = S.solitary_case(n=n, length=L, d=d, a=a, x0=x0)
    x = (np.arange(n) + 0.5) * case.dx
    inside = np.nonzero(np.abs(x - x0) < half)[0]
    for e, cnt in ((0, ex["count"]), (1, ex["count_enlarged_1"])):
        mask, c = O.mask_1d(case.ds, case.dx, case.body, O.phys_struct(crit=S.CRIT_ETA_D, enlarge=e),
                            0.0, case.h, case.hu, case.hw)
        assert c == cnt
        idx = np.nonzero(mask)[0]
        assert idx[0] == inside[0] - e == ex["first"] - e and idx[-1] == inside[-1] + e == ex["last"] + e


def brute_mask(ds, dx, body, t1, ht, mt, kt, crit, k_nh, e):
    """criterion definitions of Sec. 5.1 written out with Python loops"""
    n = len(ht)
    d, *_ = O.forcing_1d(ds, dx, body, t1)
    X, _, _ = O.body_motion(body, t1)

    def val(q, i):  # q: 'eta' 'u' 'w' with mirrored ghosts (u odd)
        if i < 0:
            j, s = -1 - i, -1.0
        elif i >= n:
            j, s = 2 * n - 1 - i, -1.0
        else:
            j, s = i, 1.0
        if q == "eta":
            return ht[j] - d[j]
        if q == "u":
            return s * mt[j] / ht[j]
        return kt[j] / ht[j]

    raw = []
    for i in range(n):
        if crit == S.CRIT_ETA_D:
            v = abs((ht[i] - d[i]) / d[i])
        elif crit == S.CRIT_ETA_X:
            v = abs(val("eta", i + 1) - val("eta", i - 1)) / (2 * dx)
        elif crit == S.CRIT_U:
            v = abs(mt[i] / ht[i])
        elif crit == S.CRIT_U_X:
            v = abs(val("u", i + 1) - val("u", i - 1)) / (2 * dx)
        elif crit == S.CRIT_W:
            v = abs(kt[i] / ht[i])
        else:
            v = abs(val("w", i + 1) - val("w", i - 1)) / (2 * dx)
        raw.append(v > k_nh)
    out = np.zeros(n, dtype=np.uint8)
    for i in range(n):
        out[i] = any(raw[j] for j in range(max(0, i - e), min(n, i + e + 1)))
    return out


@pytest.mark.parametrize("crit", range(6))
@pytest.mark.parametrize("e", [0, 1, 3])
def test_mask_matches_brute_force(crit, e):
    case = S.random_case_1d(150, seed=10 + crit, amp=0.003, mom=0.004, vert=0.002)
    k_nh = {0: 1e-3, 1: 2e-3, 2: 1.5e-3, 3: 3e-3, 4: 8e-4, 5: 2e-3}[crit]
    ph = O.phys_struct(crit=crit, enlarge=e, k_nh=k_nh)
    t1 = 0.37
    mask, cnt = O.mask_1d(case.ds, case.dx, case.body, ph, t1, case.h, case.hu, case.hw)
    ref = brute_mask(case.ds, case.dx, case.body, t1, case.h, case.hu, case.hw, crit, k_nh, e)
    assert np.array_equal(mask, ref)
    assert cnt == int(ref.sum())
    assert 0 < cnt < case.n  # the case exercises both sides of the threshold


def test_first_step_global_rule_for_w_criteria():
    """Sec. 5.1.2: with hw = 0 initially, |w| and |w_x| start with one global step"""
    case = S.slide_case(n=800, dx=0.005)
    for crit in (S.CRIT_W, S.CRIT_W_X):
        sim = O.Sim1D(case, O.phys_struct(crit=crit), cfl=0.5)
        sim.step()
        assert sim.last_active == case.n
        sim.step()
        assert sim.last_active < case.n
        off = O.Sim1D(case, O.phys_struct(crit=crit, first_global=0), cfl=0.5).step()
        assert off.last_active < case.n


def test_threshold_limits_reduce_to_global_and_hydrostatic():
    case = S.random_case_1d(200, seed=8)
    glob = O.Sim1D(case, O.phys_struct(crit=S.CRIT_GLOBAL), cfl=0.4).step(15)
    every = O.Sim1D(case, O.phys_struct(crit=S.CRIT_ETA_D, k_nh=-1.0, enlarge=0), cfl=0.4).step(15)
    none = O.Sim1D(case, O.phys_struct(crit=S.CRIT_NONE), cfl=0.4).step(15)
    never = O.Sim1D(case, O.phys_struct(crit=S.CRIT_ETA_D, k_nh=1e300), cfl=0.4).step(15)
    for q in ("h", "hu", "hw", "p"):
        assert np.array_equal(getattr(glob, q), getattr(every, q))
        assert np.array_equal(getattr(none, q), getattr(never, q))
    assert np.abs(none.p).max() == 0.0 and np.abs(glob.p).max() > 0.0


# ----------------------------------------------------------- elliptic part --

def _faces_from_paper(case, t1, dt, ht, mt, kt, rho=1000.0, g=9.81):
    """coefficients of Eqs. 12-13 evaluated literally (cells and faces), with
    the same reading of the derivatives: central differences at cells,
    two-point differences and means at faces, mirrored ghosts at walls"""
    n, dx = case.n, case.dx
    d, d_t, d_tt, d_xt = O.forcing_1d(case.ds, dx, case.body, t1)
    ext = lambda a, odd=False: np.concatenate([[-a[0] if odd else a[0]], a, [-a[-1] if odd else a[-1]]])
    de, he, me = ext(d), ext(ht), ext(mt, odd=True)
    ee = he - de
    dxc = (de[2:] - de[:-2]) / (2 * dx)
    dxx = (de[2:] - 2 * de[1:-1] + de[:-2]) / dx ** 2
    exc = (ee[2:] - ee[:-2]) / (2 * dx)
    u = mt / ht
    al = 4 + dxc ** 2
    phi = rho * ht / al * (g * dxc * exc - d_tt - 2 * u * d_xt - u ** 2 * dxx)
    phie = ext(phi)
    hf = 0.5 * (he[:-1] + he[1:])
    Df = (de[1:] - de[:-1]) / dx
    hxf = (he[1:] - he[:-1]) / dx
    phif = 0.5 * (phie[:-1] + phie[1:])
    mtf = 0.5 * (me[:-1] + me[1:])
    alf = 4 + Df ** 2
    s11 = (2 * hxf - 3 * Df) / (2 * hf)                                   # Eq. 12
    s12 = rho * alf / (4 * dt * hf)                                        # Eq. 12
    f1 = alf / (4 * hf) * (phif * Df + rho / dt * mtf)                    # Eq. 12
    s22 = 3 * dt / (rho * ht)                                              # Eq. 13
    f2 = -2 * d_t - 2 * kt / ht - dxc * mt / (2 * ht) - dt * al / (2 * rho * ht) * phi  # Eq. 13
    return dict(s11=s11, s12=s12, f1=f1, s22=s22, f2=f2, mtf=mtf, al=al, phi=phi, dxc=dxc)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_elliptic_solve_equals_dense_first_order_system(seed):
    """Schur complement + Thomas == dense solve of the first-order system of
    Eqs. 14-15 with the flip-flop fluxes (p* = p+, (hu)* = (hu)-) at degree
    zero: unknowns p on NH cells, hu on every face touching an NH cell.  The
    corrected hu and hw are then checked against Eqs. 10, 11 and 5 solved
    cell by cell as a 2x2 system in the unknowns (h p)_x and P_b."""
    rng = np.random.default_rng(seed)
    n = 14
    case = S.random_case_1d(n, seed=seed, dx=0.07, amp=0.05, mom=0.1, vert=0.05,
                            body=S.Body(kind=S.BODY_QUARTIC, law=S.LAW_SIN_RAMP, amp=0.08,
                                        length=0.6, x0=0.5, dir=0.96, q=(0.4, 0.8, 0, 0, 0)))
    mask = (rng.random(n) < 0.65).astype(np.uint8)
    mask[[3, 4, 5, 9]] = [1, 1, 1, 0]
    mask[0] = 1  # a run touching the wall
    t1, dt, rho = 0.21, 0.004, 1000.0
    ph = O.phys_struct(crit=S.CRIT_GLOBAL)
    ht, mt, kt = case.h, case.hu, case.hw
    C = _faces_from_paper(case, t1, dt, ht, mt, kt)
    cells = [i for i in range(n) if mask[i]]
    faces = sorted({f for i in cells for f in (i, i + 1)})
    ip = {c: k for k, c in enumerate(cells)}
    iq = {f: len(cells) + k for k, f in enumerate(faces)}
    M = np.zeros((len(cells) + len(faces),) * 2)
    b = np.zeros(M.shape[0])
    dx = case.dx
    for f in faces:  # Eq. 14 on face f: p_x + s11 p + s12 hu = f1, p = 0 off the NH area
        r = iq[f]
        for c, coef in ((f - 1, -1.0 / dx + 0.5 * C["s11"][f]), (f, 1.0 / dx + 0.5 * C["s11"][f])):
            if c in ip:
                M[r, ip[c]] += coef
        M[r, iq[f]] += C["s12"][f]
        b[r] = C["f1"][f]
    for i in cells:  # Eq. 15 on cell i with s21 = -s11 at the faces
        r = ip[i]
        M[r, iq[i + 1]] += 1.0 / dx - 0.5 * C["s11"][i + 1]
        M[r, iq[i]] += -1.0 / dx - 0.5 * C["s11"][i]
        M[r, ip[i]] += C["s22"][i]
        b[r] = C["f2"][i]
    sol = np.linalg.solve(M, b)
    p_dense = np.zeros(n)
    for c in cells:
        p_dense[c] = sol[ip[c]]

    dg, up, rh = O.nh_system_1d(case.ds, dx, case.body, ph, t1, dt, ht, mt, kt, mask)
    p = O.tridiag_solve(dg, up, rh)
    assert np.allclose(p, p_dense, rtol=1e-10, atol=1e-10 * np.abs(p_dense).max())

    mo, ko = O.nh_correct_1d(case.ds, dx, case.body, ph, t1, dt, ht, mt, kt, mask, p)
    for i in range(n):
        if not mask[i]:
            assert mo[i] == mt[i] and ko[i] == kt[i]
            continue
        dm = 0.5 * ((sol[iq[i]] - C["mtf"][i]) + (sol[iq[i + 1]] - C["mtf"][i + 1]))
        assert abs(mo[i] - (mt[i] + dm)) <= 1e-9 * (abs(mt[i]) + abs(dm) + 1e-12)
        # Eqs. 10, 11 with P_b of Eq. 5: unknowns X = (h p)_x and P
        D, al, phi = C["dxc"][i], C["al"][i], C["phi"][i]
        A2 = np.array([[-1.0, D], [D / al, -1.0]])
        r2 = np.array([rho * dm / dt, -6.0 * p_dense[i] / al - phi])
        X, P = np.linalg.solve(A2, r2)
        assert abs(ko[i] - (kt[i] + dt * P / rho)) <= 1e-9 * (abs(kt[i]) + abs(dt * P / rho) + 1e-12)


def test_elliptic_matrix_is_spd():
    """s11 + s21 = 0 and s12 > 0 (Sec. 3.2) make A symmetric positive definite"""
    case = S.random_case_1d(80, seed=21, amp=0.1, mom=0.2, vert=0.05)
    ph = O.phys_struct()
    mask = np.ones(80, dtype=np.uint8)
    mask[[10, 11, 40]] = 0
    dg, up, rh = O.nh_system_1d(case.ds, case.dx, case.body, ph, 0.3, 0.01, case.h, case.hu,
                                case.hw, mask)
    A = np.diag(dg) + np.diag(up[:-1], 1) + np.diag(up[:-1], -1)
    np.linalg.cholesky(A)
    assert np.all(up[~mask.astype(bool)] == 0.0)


def test_thomas_matches_dense():
    rng = np.random.default_rng(4)
    n = 50
    up = rng.uniform(-1, 1, n)
    up[-1] = 0
    dg = np.abs(up) + np.abs(np.concatenate([[0], up[:-1]])) + rng.uniform(0.1, 1, n)
    rh = rng.standard_normal(n)
    A = np.diag(dg) + np.diag(up[:-1], 1) + np.diag(up[:-1], -1)
    assert np.allclose(O.tridiag_solve(dg, up, rh), np.linalg.solve(A, rh), rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------ whole steps --

def test_solitary_wave_matches_serre_exact_solution():
    """Sec. 4.1: the global NH model follows the Serre solitary wave.  The
    paper reports RMSE 0.0108 for a = 2 (RMSE / a = 5.4e-3) and r = 0.9997;
    the same normalised bounds are required on the a/h0 = 0.2 case, while the
    hydrostatic SWE alone fails them."""
    case = S.solitary_case(n=2000, length=200.0, d=1.0, a=0.2)
    x = (np.arange(case.n) + 0.5) * case.dx
    res = {}
    for crit in (S.CRIT_GLOBAL, S.CRIT_ETA_D, S.CRIT_NONE):
        sim = O.Sim1D(case, O.phys_struct(crit=crit, enlarge=1), cfl=0.5).step(1000)
        ex, _, _ = S.solitary_exact(x, sim.time, 0.2, 1.0, 50.0)
        eta = sim.h - 1.0
        res[crit] = (np.sqrt(np.mean((eta - ex) ** 2)) / 0.2, np.corrcoef(eta, ex)[0, 1])
    for crit in (S.CRIT_GLOBAL, S.CRIT_ETA_D):
        assert res[crit][0] < 5.4e-3 and res[crit][1] > 0.9997
    assert res[S.CRIT_NONE][0] > 5 * res[S.CRIT_GLOBAL][0] and res[S.CRIT_NONE][1] < 0.99


def test_solitary_wave_error_decreases_with_resolution():
    errs = []
    for n in (500, 1000, 2000):
        case = S.solitary_case(n=n, length=200.0, d=1.0, a=0.2)
        sim = O.Sim1D(case, O.phys_struct(crit=S.CRIT_GLOBAL), cfl=0.5)
        while sim.time < 4.0 - 1e-12:
            sim.step()
        x = (np.arange(n) + 0.5) * case.dx
        ex, _, _ = S.solitary_exact(x, sim.time, 0.2, 1.0, 50.0)
        errs.append(np.sqrt(np.mean((sim.h - 1.0 - ex) ** 2)))
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]


def test_paper_solitary_setup_reaches_printed_accuracy():
    g = json.load(open(os.path.join(GOLD, "solitary_paper.json")))
    st, pr = g["setup"], g["printed"]
    n = int(round(st["L"] / 1.0))
    case = S.solitary_case(n=n, length=st["L"], d=st["d"], a=st["a"], x0=st["x0_over_L"] * st["L"])
    dt = st["dt"] * (st["L"] / n) / st["dx"]
    sim = O.Sim1D(case, O.phys_struct(crit=S.CRIT_GLOBAL), cfl=0.0, dt_fixed=dt)
    sim.step(int(round(st["T"] / dt)))
    x = (np.arange(n) + 0.5) * case.dx
    ex, _, _ = S.solitary_exact(x, sim.time, st["a"], st["d"], st["x0_over_L"] * st["L"])
    eta = sim.h - st["d"]
    assert abs(sim.time - st["T"]) < 1e-9
    assert np.sqrt(np.mean((eta - ex) ** 2)) <= pr["rmse"]
    assert np.corrcoef(eta, ex)[0, 1] >= pr["r"]


def _standing_wave_quarter_period(kd, crit, n_per_wl=128):
    d, a = 1.0, 1e-4
    k = kd / d
    L = 2 * math.pi / k
    n = n_per_wl
    dx = L / n
    x = (np.arange(n) + 0.5) * dx
    eta = a * np.cos(k * x)
    case = S.Case1D(n=n, dx=dx, ds=np.full(n, d), h=d + eta, hu=np.zeros(n), hw=np.zeros(n),
                    body=S.Body())
    sim = O.Sim1D(case, O.phys_struct(crit=crit), cfl=0.25)
    proj = lambda: 2.0 / n * np.sum((sim.h - d) * np.cos(k * x))
    t_prev, a_prev = 0.0, proj()
    while True:
        sim.step()
        a_now = proj()
        if a_now <= 0.0:
            return t_prev + (sim.time - t_prev) * a_prev / (a_prev - a_now)
        t_prev, a_prev = sim.time, a_now


@pytest.mark.parametrize("kd", [0.5, 1.0])
def test_linear_dispersion_is_green_naghdi(kd):
    """flat bottom: the model is equivalent to Green-Naghdi / Serre, whose
    linear dispersion is omega^2 = g d k^2 / (1 + (kd)^2 / 3); the hydrostatic
    SWE gives omega^2 = g d k^2"""
    g, d = 9.81, 1.0
    k = kd / d
    w_gn = math.sqrt(g * d * k * k / (1 + kd * kd / 3))
    w_swe = math.sqrt(g * d) * k
    tq = _standing_wave_quarter_period(kd, S.CRIT_GLOBAL)
    assert abs(tq - 0.5 * math.pi / w_gn) < 0.01 * (0.5 * math.pi / w_gn)
    tq_h = _standing_wave_quarter_period(kd, S.CRIT_NONE)
    assert abs(tq_h - 0.5 * math.pi / w_swe) < 0.01 * (0.5 * math.pi / w_swe)


# ------------------------------------------------------------ error codes --

def test_status_codes():
    case = S.random_case_1d(64, seed=2)
    h = case.h.copy()
    h[10] = -0.1
    bad = S.Case1D(n=64, dx=case.dx, ds=case.ds, h=h, hu=case.hu, hw=case.hw, body=case.body)
    with pytest.raises(O.OracleError) as e:
        O.Sim1D(bad, O.phys_struct(), cfl=0.0, dt_fixed=1e-4).step()
    assert e.value.code == O.EDRY
    h = case.h.copy()
    h[5] = np.nan
    bad = S.Case1D(n=64, dx=case.dx, ds=case.ds, h=h, hu=case.hu, hw=case.hw, body=case.body)
    with pytest.raises(O.OracleError) as e:
        O.Sim1D(bad, O.phys_struct(), cfl=0.5).step()
    assert e.value.code == O.ENAN
