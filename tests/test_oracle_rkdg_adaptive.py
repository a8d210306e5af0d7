"""Pins of the adaptive model in the oracle of the paper's own 1D
discretisation (oracle/rkdg1d.py, Sec. 5: criterion on the predictor,
elliptic solve and correction on the marked elements only, optional
enlargement of the marked set by Sec. 5.2).

* Every element marked is the global model; no element marked is the
  hydrostatic predictor alone.
* The restricted LDG solve: exterior p = 0 and hu = hu~ exactly, and the
  whole vector satisfies the global system's rows of the marked unknowns.
* The element criterion: the strict threshold, the derivative criteria on the
  element's slope, the widening by e elements, the first step global.
* The paper's solitary-wave tables at its own resolution (Table 4 without
  enlargement, Table 8 with enlargement by one element;
  tests/golden/solitary_adaptive_paper.json): the value criteria and every
  enlarged run within 10 % of the printed RMSE; the derivative criteria
  without enlargement degraded as printed, |w_x| by far the worst."""
import json
import os

import numpy as np
import pytest

import swe_inputs as S
from oracle import rkdg1d as R

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NAMES = ["eta/d", "eta_x", "u", "u_x", "w", "w_x"]


def solitary_setup():
    st = json.load(open(os.path.join(GOLD, "solitary_paper.json")))["setup"]
    a, d, L, dx, dt, T = st["a"], st["d"], st["L"], st["dx"], st["dt"], st["T"]
    n = int(round(L / dx))
    x0 = st["x0_over_L"] * L
    return a, d, dx, dt, int(round(T / dt)), n, x0, R.solitary_initial(n, dx, a, d, x0)


def test_every_element_marked_is_the_global_model():
    a, d, dx, dt, _, n, x0, Q0 = solitary_setup()
    Qg, pg, tg = R.run(Q0, d, S.Body(), 0.0, dt, 25, dx)
    Qa, pa, ta, cnt = R.run_adaptive(Q0, d, S.Body(), 0.0, dt, 25, dx, R.CRIT_GLOBAL)
    assert cnt == [n] * 25 and ta == tg
    assert np.allclose(Qa, Qg, rtol=0, atol=1e-12 * np.abs(Qg).max())
    assert np.allclose(pa, pg, rtol=0, atol=1e-10 * np.abs(pg).max())


def test_no_element_marked_is_the_predictor():
    a, d, dx, dt, _, n, x0, Q0 = solitary_setup()
    Qa, pa, ta, cnt = R.run_adaptive(Q0, d, S.Body(), 0.0, dt, 10, dx, R.CRIT_NONE)
    Q, t = Q0, 0.0
    for _ in range(10):
        Q = R.predict(Q, d, S.Body(), t, dt, dx)
        t += dt
    assert cnt == [0] * 10 and np.array_equal(Qa, Q) and not pa.any()


def test_restricted_solve_fixes_the_exterior_and_meets_the_marked_rows():
    n, dx = 40, 0.5
    rng = np.random.default_rng(11)
    x = R.node_x(n, dx)
    c = dict(s11=0.3 * np.sin(x), s12=1.2 + 0.4 * np.cos(x), s22=0.9 + 0.1 * x,
             f1=rng.standard_normal((n, 2)), f2=rng.standard_normal((n, 2)))
    c["s21"] = -c["s11"]
    qt = rng.standard_normal((n, 2))
    mask = np.zeros(n, dtype=bool)
    mask[0:4] = True     # touches the left wall
    mask[10:17] = True
    mask[22] = True      # an isolated element
    mask[33:] = True     # touches the right wall
    p, q = R.ldg_solve_masked(c, qt, mask, dx)
    assert not p[~mask].any() and np.array_equal(q[~mask], qt[~mask])
    A = R.ldg_matrix(c["s11"], c["s12"], c["s21"], c["s22"], dx).tocsr()
    b = R.ldg_rhs(c["f1"], c["f2"], dx)
    z = np.concatenate([p.ravel(), q.ravel()])
    node = np.repeat(mask, 2)
    I = np.flatnonzero(np.concatenate([node, node]))
    res = (A @ z - b)[I]
    assert np.abs(res).max() <= 1e-12 * (np.abs(b).max() + np.abs(A).max() * np.abs(z).max())
    # the exterior values enter: a different hu~ outside changes the solution
    p2, q2 = R.ldg_solve_masked(c, qt + 1.0 * (~mask)[:, None], mask, dx)
    assert np.abs(p2 - p)[mask].max() > 1e-6
    # and with everything marked, the global solve
    pg, qg = R.ldg_solve(c["s11"], c["s12"], c["s21"], c["s22"], c["f1"], c["f2"], dx)
    pa, qa = R.ldg_solve_masked(c, qt, np.ones(n, dtype=bool), dx)
    assert np.allclose(pa, pg, rtol=0, atol=1e-12) and np.allclose(qa, qg, rtol=0, atol=1e-12)


def test_element_criterion_threshold_slope_and_enlargement():
    n, dx, d = 12, 2.0, 10.0
    Qt = np.zeros((3, n, 2))
    Qt[0] = d
    Qt[1] = 0.0
    k = 1e-3
    Qt[0, 3, 1] = d + k * d          # |eta/d| = k at one node: not marked (strict)
    Qt[0, 6, 0] = d + 1.5 * k * d    # above at one node
    ind = R.element_indicator(Qt, d, S.Body(), 0.0, dx, R.CRIT_ETA_D)
    assert ind[3] == pytest.approx(k) and ind[6] == pytest.approx(1.5 * k)
    m0 = R.element_mask(Qt, d, S.Body(), 0.0, dx, R.CRIT_ETA_D, k, 0, False)
    assert np.flatnonzero(m0).tolist() == [6]
    m2 = R.element_mask(Qt, d, S.Body(), 0.0, dx, R.CRIT_ETA_D, k, 2, False)
    assert np.flatnonzero(m2).tolist() == [4, 5, 6, 7, 8]
    # the slope criterion: element 6 has slope 1.5 k d / dx in eta
    sl = R.element_indicator(Qt, d, S.Body(), 0.0, dx, R.CRIT_ETA_X)
    assert sl[6] == pytest.approx(1.5 * k * d / dx) and sl[3] == pytest.approx(k * d / dx)
    assert sl[0] == 0.0
    # |w| and |w_x| global on the first step when asked, not otherwise
    for crit in (R.CRIT_W, R.CRIT_W_X):
        assert R.element_mask(Qt, d, S.Body(), 0.0, dx, crit, k, 0, True).all()
        assert not R.element_mask(Qt, d, S.Body(), 0.0, dx, crit, k, 0, True,
                                  first_global=False).any()
        assert not R.element_mask(Qt, d, S.Body(), 0.0, dx, crit, k, 0, False).any()


def _score(Q, t, a, d, dx, n, x0):
    x = R.node_x(n, dx)
    ex, _, _ = S.solitary_exact(x, t, a, d, x0)
    eta = Q[0] - d
    return float(np.sqrt(np.mean((eta - ex) ** 2))), float(np.corrcoef(eta.ravel(), ex.ravel())[0, 1])


def test_paper_adaptive_solitary_tables():
    gold = json.load(open(os.path.join(GOLD, "solitary_adaptive_paper.json")))
    a, d, dx, dt, steps, n, x0, Q0 = solitary_setup()
    got = {}
    for e, key in ((0, "no_enlargement"), (1, "enlarged_by_one")):
        for crit, name in enumerate(NAMES):
            Q, p, t, cnt = R.run_adaptive(Q0, d, S.Body(), 0.0, dt, steps, dx, crit,
                                          gold["k_nh"], e, first_global=False)
            assert 0 < np.mean(cnt) < 0.5 * n  # a local correction
            got[key, name] = _score(Q, t, a, d, dx, n, x0)
    tab4, tab8 = gold["no_enlargement"], gold["enlarged_by_one"]
    # Table 8: with the enlargement every criterion matches the printed RMSE
    # and r (this reading: 0.0109 - 0.0115 against 0.0108 - 0.0118)
    for name in NAMES:
        rmse, r = got["enlarged_by_one", name]
        assert abs(rmse - tab8[name][1]) <= 0.1 * tab8[name][1], (name, rmse)
        assert abs(r - tab8[name][2]) <= 2e-4, (name, r)
    # Table 4: the value criteria likewise
    for name in ("eta/d", "u", "w"):
        rmse, r = got["no_enlargement", name]
        assert abs(rmse - tab4[name][1]) <= 0.1 * tab4[name][1], (name, rmse)
        assert abs(r - tab4[name][2]) <= 2e-4, (name, r)
    # the slope criteria without enlargement lose accuracy at the interfaces
    # (printed 1.3x and 1.5x the |eta/d| RMSE; this reading 2.9x and 3.1x:
    # above the printed values, within a factor 3 of them)
    base = got["no_enlargement", "eta/d"][0]
    for name in ("eta_x", "u_x"):
        rmse, r = got["no_enlargement", name]
        assert tab4[name][1] <= rmse <= 3.0 * tab4[name][1], (name, rmse)
        assert rmse > 1.2 * base and r < tab4["eta/d"][2]
    # |w_x| without enlargement is by far the worst, with its isolated
    # elements (printed RMSE 0.1146, r 0.9606)
    rmse, r = got["no_enlargement", "w_x"]
    assert rmse > 4 * max(got["no_enlargement", k][0] for k in NAMES[:5])  # printed 7x
    assert rmse > 10 * base  # printed 11x
    assert tab4["w_x"][1] / 1.5 <= rmse <= 1.5 * tab4["w_x"][1], rmse
    assert r < 0.98
    # the enlargement improves every slope criterion
    for name in ("eta_x", "u_x", "w_x"):
        assert got["enlarged_by_one", name][0] < got["no_enlargement", name][0]
