"""GPU tests of the learned warm start on grids larger than the network's
256 x 256 window: the window is placed over the active tiles and clamped to
the grid, the network computes only the active tiles' box widened by 16
cells, and marked cells outside the window start from 0.  The pressure solve
still iterates to the tolerance, so the state after the steps must match the
FP64 oracle; on a grid whose active tiles fit in the window the guess must
equal the network evaluated on the whole grid (same solve from the same
start: same iteration count, same pressure)."""
import numpy as np
import pytest

import oracle as O
import swe_inputs as S
from oracle import cnn as OC

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
NX, NY, DX, H0 = 320, 288, 2.0, 50.0
SCALES, P_SCALE = [0.05, 1.0, 1.0, 0.1], 100.0
KW = dict(crit=S.CRIT_ETA_D, k_nh=2e-3, enlarge=1, cfl=0.4, precision=0, tol=1e-13,
          max_iter=50000)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17025_amd import swe_nh
    return swe_nh


def humps_case(centres, seed=3):
    """flat-ish 50 m shelf with Gaussian surface humps at the given cell centres"""
    rng = np.random.default_rng(seed)
    x = (np.arange(NX) + 0.5) * DX
    y = (np.arange(NY) + 0.5) * DX
    X, Y = np.meshgrid(x, y)
    ds = H0 + 0.5 * S.gaussian_field_2d(NX, NY, DX, DX, 1.0, 20.0, int(rng.integers(1 << 30)))
    eta = np.zeros_like(X)
    for (ci, cj) in centres:
        eta += 0.6 * np.exp(-((X - (ci + 0.5) * DX) ** 2 + (Y - (cj + 0.5) * DX) ** 2) / 16.0 ** 2)
    h = ds + eta
    z = np.zeros_like(X)
    return S.Case2D(nx=NX, ny=NY, dx=DX, dy=DX, ds=ds, h=h, hu=z.copy(), hv=z.copy(), hw=z.copy(),
                    body=S.Body(), t0=0.0)


def net_params(seed):
    rng = np.random.default_rng(seed)
    p = OC.init_params(seed).astype(np.float64)
    o = 0
    for (nw, nb) in OC.layer_sizes():
        p[o + nw:o + nw + nb] = 0.05 * rng.standard_normal(nb)
        o += nw + nb
    return torch.tensor(p.astype(np.float32), device=DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def run(B, c, warm, nsteps, pt=None, p0=None):
    ctx = B.context_2d(c, warm=warm, **KW)
    if pt is not None:
        ctx.set_warm_start_net(pt, SCALES, P_SCALE)
    ctx.set_time(c.t0)
    f = lambda a: torch.tensor(a, dtype=torch.float64, device=DEV)
    h, hu, hv, hw = f(c.h), f(c.hu), f(c.hv), f(c.hw)
    p = torch.zeros_like(h) if p0 is None else p0.clone()
    m = torch.zeros((NY, NX), dtype=torch.uint8, device=DEV)
    ctx.step(h, hu, hv, hw, p, m, nsteps=nsteps)
    st = ctx.sync_stats()
    assert st["status"] == 0, st
    return ctx, (h, hu, hv, hw, p, m), st


@pytest.mark.parametrize("name,centres", [
    ("corner", [(22, 270)]),                 # active tiles against two walls
    ("wide", [(24, 40), (300, 250)]),        # active box wider and taller than the window
])
def test_windowed_guess_keeps_the_solution(B, name, centres):
    print(f"warm window case {name}: {NX}x{NY}, humps at {centres}", flush=True)
    c = humps_case(centres)
    _, (h, hu, hv, hw, p, m), st = run(B, c, 2, 3, pt=net_params(9))
    ref = O.Sim2D(c, O.phys_struct(crit=S.CRIT_ETA_D, k_nh=2e-3, enlarge=1, tol=1e-14),
                  cfl=0.4).step(3)
    assert st["n_active"] == ref.last_active > 0
    assert np.array_equal(m.cpu().numpy(), ref.mask)
    cols = np.nonzero(ref.mask.any(axis=0))[0]
    rows = np.nonzero(ref.mask.any(axis=1))[0]
    if name == "wide":  # the marked area does not fit in one window
        assert cols[-1] - cols[0] > 256 and rows[-1] - rows[0] > 200
    for g, r in ((h, ref.h), (hu, ref.hu), (hv, ref.hv), (hw, ref.hw), (p, ref.p)):
        assert rel(g.cpu().numpy(), r) <= 1e-10


def test_windowed_guess_equals_whole_grid_network(B):
    """one step from t0: the guess the step builds on its window must be the
    network on the whole grid, scaled, on the marked cells"""
    c = humps_case([(22, 270)])
    pt = net_params(11)
    ctxA, (_, _, _, _, pA, mA), stA = run(B, c, 2, 1, pt=pt)
    dt = stA["dt"]
    f = lambda a: torch.tensor(a, dtype=torch.float64, device=DEV)
    ht, mt, nt, kt = (torch.empty((NY, NX), dtype=torch.float64, device=DEV) for _ in range(4))
    ctxA.predict(f(c.h), f(c.hu), f(c.hv), f(c.hw), c.t0, dt, ht, mt, nt, kt)
    feat = torch.empty((NY, NX, 16), dtype=torch.int16, device=DEV)
    ctxA.features(ht, mt, nt, mA, c.t0 + dt, SCALES, feat)
    out = torch.empty((1, NY, NX), dtype=torch.float32, device=DEV)
    B.Net(1, NY, NX, device=DEV).forward(pt, feat, out)
    guess = P_SCALE * out[0].double() * mA.double()
    assert guess.abs().max().item() > 0
    _, (_, _, _, _, pB, mB), stB = run(B, c, 1, 1, p0=guess)
    assert torch.equal(mA, mB)
    assert stB["iters"] == stA["iters"], (stA["iters"], stB["iters"])
    assert rel(pA.cpu().numpy(), pB.cpu().numpy()) <= 1e-14
