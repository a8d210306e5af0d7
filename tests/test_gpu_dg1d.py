"""GPU parity of the paper's own 1D discretisation (RKDG-P1 predictor, Sec.
3.1; LDG-P1 elliptic solve with the alternating flux, Sec. 3.2; correction of
Eqs. 10-11) against its FP64 oracle (oracle/rkdg1d.py), through the C ABI.

Both sides are FP64 and take the same steps; the elliptic solves differ in
their elimination order only (sparse LU with pivoting in the oracle, per-
element condensation and cyclic reduction of the interface pairs on the
GPU), so one step agrees to rounding and whole runs to <= 1e-10."""
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


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17025_amd import swe_nh
    return swe_nh


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def rel(g, r):
    g = g.cpu().numpy() if hasattr(g, "cpu") else np.asarray(g)
    return np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)


def gpu_run(B, Q, n, dx, dt, d_static, body, t0, nsteps):
    h, hu, hw = dev(Q[0]), dev(Q[1]), dev(Q[2])
    p = torch.zeros_like(h)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    rc = B.dg1d_run(n, dx, dt, d_static, body, t0, nsteps, h, hu, hw, p, status)
    return rc, np.stack([a.cpu().numpy() for a in (h, hu, hw)]), p.cpu().numpy()


def test_paper_solitary_wave_matches_the_oracle(B):
    """the paper's solitary run (Sec. 4.1: a = 2 m, d = 10 m, dx = 4 m,
    dt = 0.1 s, 300 steps): the GPU state is the oracle's, and so is its
    error against the exact solitary wave (RMSE 0.0110 against the printed
    0.0108)"""
    g = json.load(open(os.path.join(GOLD, "solitary_paper.json")))
    st = g["setup"]
    a, d, L, dx, dt, T = st["a"], st["d"], st["L"], st["dx"], st["dt"], st["T"]
    n, steps = int(round(L / dx)), int(round(T / dt))
    Q0 = S.dg_solitary_state(n, dx, a, d, st["x0_over_L"] * L)
    rc, Qg, pg = gpu_run(B, Q0, n, dx, dt, d, S.Body(), 0.0, steps)
    assert rc == B.OK
    Qr, pr, t = R.run(Q0, d, S.Body(), 0.0, dt, steps, dx)
    for a_ in range(3):
        assert rel(Qg[a_], Qr[a_]) <= 1e-10, a_
    assert rel(pg, pr) <= 1e-10
    x = R.node_x(n, dx)
    ex, _, _ = S.solitary_exact(x, t, a, d, st["x0_over_L"] * L)
    rm = lambda e: np.sqrt(np.mean((e - ex) ** 2))
    assert abs(rm(Qg[0] - d) - rm(Qr[0] - d)) <= 1e-9
    assert abs(rm(Qg[0] - d) - g["printed"]["rmse"]) <= 0.05 * g["printed"]["rmse"]


@pytest.mark.parametrize("n,dt,steps", [(400, 0.005, 300), (800, 0.0025, 120)])
def test_sliding_block_flume_matches_the_oracle(B, n, dt, steps):
    """the flume of Sec. 4.3: the quartic block of Eq. 20 moved by the law of
    Eq. 21 (Fr = 0.25) under still water 0.175 m deep, 30 m long; 800
    elements run on the 1024-thread workgroup"""
    body = S.whittaker_case(fr_index=1).body
    dx = 30.0 / n
    x = R.node_x(n, dx)
    Q0 = S.dg_still_water_state(n, dx, 0.175, body)
    rc, Qg, pg = gpu_run(B, Q0, n, dx, dt, 0.175, body, 0.0, steps)
    assert rc == B.OK
    Qr, pr, _ = R.run(Q0, 0.175, body, 0.0, dt, steps, dx)
    assert np.abs(Qr[1]).max() > 1e-4  # the block has moved water
    d_end = R.bottom(0.175, body, x, steps * dt)[0]
    assert rel(Qg[0] - d_end, Qr[0] - d_end) <= 1e-10  # eta
    for a_ in (1, 2):
        assert rel(Qg[a_], Qr[a_]) <= 1e-10, a_
    assert rel(pg, pr) <= 1e-10


@pytest.mark.parametrize("n", [1, 2, 3, 64, 511, 512, 513])
def test_one_step_on_a_rough_state(B, n):
    """one step from a state with every field varying node by node over a
    moving Gaussian mound (the sizes straddle the 512-thread workgroup and
    include one and two elements).  The LDG matrix is badly scaled (its
    2-norm condition number is ~1e8 here: s12 = rho alpha / (4 dt h) against
    O(1) entries), so the pressure and the corrected hu are held to a
    normwise backward error of 1e-14 in the oracle's own system (a forward
    bar of cond * eps would be ~4e-8); the predictor's h to rounding"""
    rng = np.random.default_rng(100 + n)
    dx, dt, t0 = 0.5, 0.02, 0.37
    x = R.node_x(n, dx)
    Q0 = np.stack([2.0 + 0.1 * np.sin(0.3 * x) + 0.01 * rng.standard_normal((n, 2)),
                   0.2 * np.cos(0.2 * x) + 0.01 * rng.standard_normal((n, 2)),
                   0.05 * np.sin(x) + 0.01 * rng.standard_normal((n, 2))])
    body = S.Body(kind=S.BODY_GAUSS, law=S.LAW_CONST_VEL, amp=0.2, length=2.0,
                  x0=0.3 * n * dx, q=(0.5, 0, 0, 0, 0))
    rc, Qg, pg = gpu_run(B, Q0, n, dx, dt, 2.0, body, t0, 1)
    assert rc == B.OK
    Qr, pr, _ = R.run(Q0, 2.0, body, t0, dt, 1, dx)
    assert rel(Qg[0] - 2.0, Qr[0] - 2.0) <= 1e-13
    Qt = R.predict(Q0, 2.0, body, t0, dt, dx)
    c = R.nh_coefficients(Qt, 2.0, body, t0 + dt, dt, dx)
    A = R.ldg_matrix(c["s11"], c["s12"], c["s21"], c["s22"], dx)
    b = R.ldg_rhs(c["f1"], c["f2"], dx)
    z = np.concatenate([pg.ravel(), Qg[1].ravel()])
    berr = np.linalg.norm(A @ z - b) / (np.linalg.norm(A.toarray(), 2) * np.linalg.norm(z) +
                                        np.linalg.norm(b))
    assert berr <= 1e-14, berr
    for g_, r_ in ((pg, pr), (Qg[1], Qr[1]), (Qg[2], Qr[2])):
        assert rel(g_, r_) <= 1e-10


def test_status_codes(B):
    """a node depth <= 0 entering a predictor stage gives EDRY; element
    counts outside 1 .. 1024 give EINVAL and leave the state untouched"""
    n, dx = 32, 0.5
    x = R.node_x(n, dx)
    Q0 = np.stack([2.0 + 0.0 * x, 0.0 * x, 0.0 * x])
    Q0[0][5, 1] = -0.1
    rc, _, _ = gpu_run(B, Q0, n, dx, 0.01, 2.0, S.Body(), 0.0, 1)
    assert rc == B.EDRY
    for bad in (0, B.DG_MAX_ELEMS + 1):
        h = dev(np.full((max(bad, 1), 2), 2.0))
        z = torch.zeros_like(h)
        st = torch.zeros(1, dtype=torch.int32, device=DEV)
        assert B.dg1d_run(bad, dx, 0.01, 2.0, S.Body(), 0.0, 1, h, z, z.clone(), z.clone(),
                          st) == B.EINVAL
        assert torch.all(h == 2.0)
