"""GPU parity of the adaptive model on the paper's own 1D discretisation
(Sec. 5 with the RKDG-P1 predictor and the LDG-P1 solve restricted to the
marked elements) against its FP64 oracle (oracle/rkdg1d.py run_adaptive),
through the C ABI.

The element masks are integer results and are compared exactly, step by
step (both sides take the criterion in FP64 on states that agree to
rounding); the states are held to the global model's bar (<= 1e-10 over
whole runs)."""
import json
import os

import numpy as np
import pytest

import swe_inputs as S
from oracle import rkdg1d as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
GOLD = os.path.join(os.path.dirname(__file__), "golden")
NAMES = ["eta/d", "eta_x", "u", "u_x", "w", "w_x"]


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17025_amd import swe_nh
    return swe_nh


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def rel(g, r):
    return np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)


def gpu_run(B, Q, n, dx, dt, d_static, body, t0, nsteps, **kw):
    h, hu, hw = dev(Q[0]), dev(Q[1]), dev(Q[2])
    p = torch.zeros_like(h)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    marked = torch.full((max(nsteps, 1),), -1, dtype=torch.int32, device=DEV)
    print(f"dg1d adaptive n={n} steps={nsteps} {kw}", flush=True)
    rc = B.dg1d_run(n, dx, dt, d_static, body, t0, nsteps, h, hu, hw, p, status, marked=marked,
                    **kw)
    return (rc, np.stack([a.cpu().numpy() for a in (h, hu, hw)]), p.cpu().numpy(),
            marked.cpu().numpy()[:nsteps].tolist())


def solitary():
    st = json.load(open(os.path.join(GOLD, "solitary_paper.json")))["setup"]
    a, d, L, dx, dt, T = st["a"], st["d"], st["L"], st["dx"], st["dt"], st["T"]
    n = int(round(L / dx))
    x0 = st["x0_over_L"] * L
    return a, d, dx, dt, int(round(T / dt)), n, x0, S.dg_solitary_state(n, dx, a, d, x0)


@pytest.mark.parametrize("enlarge", [0, 1])
@pytest.mark.parametrize("crit", range(6))
def test_paper_adaptive_solitary_matches_the_oracle(B, crit, enlarge):
    """the runs behind Tables 4 and 8 (Sec. 5, k_nh = 0.001, 300 steps):
    the same elements marked in every step, the same final state, and so the
    same RMSE against the exact wave"""
    a, d, dx, dt, steps, n, x0, Q0 = solitary()
    rc, Qg, pg, mg = gpu_run(B, Q0, n, dx, dt, d, S.Body(), 0.0, steps, crit=crit, k_nh=1e-3,
                             enlarge=enlarge)
    assert rc == B.OK
    Qr, pr, t, mr = R.run_adaptive(Q0, d, S.Body(), 0.0, dt, steps, dx, crit, 1e-3, enlarge,
                                   first_global=False)
    assert mg == mr
    assert 0 < np.mean(mr) < n
    assert rel(Qg[0] - d, Qr[0] - d) <= 1e-10
    for k in (1, 2):
        assert rel(Qg[k], Qr[k]) <= 1e-10, k
    assert rel(pg, pr) <= 1e-10
    x = R.node_x(n, dx)
    ex, _, _ = S.solitary_exact(x, t, a, d, x0)
    rm = lambda e: np.sqrt(np.mean((e - ex) ** 2))
    assert abs(rm(Qg[0] - d) - rm(Qr[0] - d)) <= 1e-9


@pytest.mark.parametrize("crit,enlarge,first_global", [(S.CRIT_ETA_D, 1, False),
                                                      (S.CRIT_W, 0, True),
                                                      (S.CRIT_W_X, 2, True)])
def test_adaptive_sliding_block_matches_the_oracle(B, crit, enlarge, first_global):
    """the flume of Sec. 4.3 (water at rest over the moving quartic block,
    400 elements): |w| and |w_x| need the first step global (Sec. 5.1.2),
    without it nothing is ever marked"""
    body = S.whittaker_case(fr_index=1).body
    n, dt, steps, d = 400, 0.005, 300, 0.175
    dx = 30.0 / n
    x = R.node_x(n, dx)
    Q0 = S.dg_still_water_state(n, dx, d, body)
    rc, Qg, pg, mg = gpu_run(B, Q0, n, dx, dt, d, body, 0.0, steps, crit=crit, k_nh=1e-3,
                             enlarge=enlarge, first_global=first_global)
    assert rc == B.OK
    Qr, pr, _, mr = R.run_adaptive(Q0, d, body, 0.0, dt, steps, dx, crit, 1e-3, enlarge,
                                   first_global=first_global)
    assert mg == mr
    assert 0 < np.mean(mr) < n
    d_end = R.bottom(d, body, x, steps * dt)[0]
    assert rel(Qg[0] - d_end, Qr[0] - d_end) <= 1e-10
    for k in (1, 2):
        assert rel(Qg[k], Qr[k]) <= 1e-10, k
    assert rel(pg, pr) <= 1e-10


def threshold_at(ind, frac):
    """a k_nh that marks about the fraction frac of the elements, halfway
    between two indicator values that differ by far more than rounding"""
    v = np.sort(ind)
    j = min(max(int(round((1.0 - frac) * len(v))), 0), len(v))
    if j == 0:
        return 0.5 * v[0]
    if j == len(v):
        return 2.0 * v[-1]
    while j < len(v) and v[j] - v[j - 1] <= 1e-9 * v[j]:
        j += 1
    return 0.5 * (v[j - 1] + v[j]) if j < len(v) else 2.0 * v[-1]


@pytest.mark.parametrize("n", [1, 2, 7, 64, 512, 513])
@pytest.mark.parametrize("frac", [0.0, 0.3, 0.7])
def test_one_adaptive_step_on_a_rough_state(B, n, frac):
    """one step from a rough state (every field varying node by node over a
    moving Gaussian mound) with a threshold that marks about the fraction
    frac of the elements by |eta/d|: scattered sets with isolated elements,
    segments at either wall, the first element marked and not, and the
    empty set; the oracle's restricted solve"""
    rng = np.random.default_rng(300 + n)
    dx, dt, t0 = 0.5, 0.02, 0.37
    x = R.node_x(n, dx)
    Q0 = np.stack([2.0 + 0.1 * np.sin(0.3 * x) + 0.03 * rng.standard_normal((n, 2)),
                   0.2 * np.cos(0.2 * x) + 0.01 * rng.standard_normal((n, 2)),
                   0.05 * np.sin(x) + 0.01 * rng.standard_normal((n, 2))])
    body = S.Body(kind=S.BODY_GAUSS, law=S.LAW_CONST_VEL, amp=0.2, length=2.0,
                  x0=0.3 * n * dx, q=(0.5, 0, 0, 0, 0))
    Qt = R.predict(Q0, 2.0, body, t0, dt, dx)
    k_nh = threshold_at(R.element_indicator(Qt, 2.0, body, t0 + dt, dx, S.CRIT_ETA_D), frac)
    rc, Qg, pg, mg = gpu_run(B, Q0, n, dx, dt, 2.0, body, t0, 1, crit=S.CRIT_ETA_D, k_nh=k_nh)
    assert rc == B.OK
    Qr, pr, _, mr = R.run_adaptive(Q0, 2.0, body, t0, dt, 1, dx, S.CRIT_ETA_D, k_nh, 0)
    assert mg == mr
    assert abs(mr[0] - frac * n) <= 1 + 0.02 * n
    assert rel(Qg[0] - 2.0, Qr[0] - 2.0) <= 1e-13
    for g_, r_ in ((Qg[1], Qr[1]), (Qg[2], Qr[2])):
        assert rel(g_, r_) <= 1e-10
    if mr[0]:
        assert rel(pg, pr) <= 1e-10
    else:
        assert not pg.any() and not pr.any()


def test_global_and_none_criteria(B):
    """SWE_NH_CRIT_GLOBAL through the adaptive path is the global model bit
    for bit; SWE_NH_CRIT_NONE is the predictor alone (p = 0)"""
    a, d, dx, dt, _, n, x0, Q0 = solitary()
    h, hu, hw = dev(Q0[0]), dev(Q0[1]), dev(Q0[2])
    p = torch.zeros_like(h)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    assert B.dg1d_run(n, dx, dt, d, S.Body(), 0.0, 40, h, hu, hw, p, st) == B.OK
    rc, Qg, pg, mg = gpu_run(B, Q0, n, dx, dt, d, S.Body(), 0.0, 40, crit=S.CRIT_GLOBAL)
    assert rc == B.OK and mg == [n] * 40
    for u, v in zip((h, hu, hw, p), (Qg[0], Qg[1], Qg[2], pg)):
        assert np.array_equal(u.cpu().numpy(), v)
    rc, Qg, pg, mg = gpu_run(B, Q0, n, dx, dt, d, S.Body(), 0.0, 40, crit=S.CRIT_NONE)
    assert rc == B.OK and mg == [0] * 40 and not pg.any()
    Qr, _, _, _ = R.run_adaptive(Q0, d, S.Body(), 0.0, dt, 40, dx, S.CRIT_NONE)
    for k in range(3):
        assert rel(Qg[k], Qr[k]) <= 1e-12


def test_adaptive_argument_checks(B):
    """a criterion outside the enumeration, an enlargement beyond
    SWE_NH_DG_MAX_ENLARGE or a negative threshold give EINVAL and leave the
    state untouched"""
    n, dx = 16, 0.5
    for kw in (dict(crit=8), dict(crit=-1), dict(crit=0, enlarge=B.DG_MAX_ENLARGE + 1),
               dict(crit=0, enlarge=-1), dict(crit=0, k_nh=-1e-3)):
        h = dev(np.full((n, 2), 2.0))
        z = torch.zeros_like(h)
        st = torch.zeros(1, dtype=torch.int32, device=DEV)
        assert B.dg1d_run(n, dx, 0.01, 2.0, S.Body(), 0.0, 1, h, z, z.clone(), z.clone(), st,
                          **kw) == B.EINVAL, kw
        assert torch.all(h == 2.0)
