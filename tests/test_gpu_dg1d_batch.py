"""GPU tests of the batched form of the paper's own 1D discretisation
(swe_nh_dg1d_run_batch: one workgroup per channel, each channel with its own
config, global or adaptive), through the C ABI.

Each channel of a batch is the single-channel run of the same config (the
same arithmetic; held to 1e-13, since the batch may run a channel in the
other kernel variant), and so the oracle's run (<= 1e-10, as the single-
channel tests); the per-step marked counts of adaptive channels are exact."""
import numpy as np
import pytest

import swe_inputs as S
from oracle import rkdg1d as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17025_amd import swe_nh
    return swe_nh


def rel(g, r):
    return np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)


def channel(kind, n, seed):
    """(n, dx, dt, d_static, body, Q0, adaptive kwargs) of a test channel"""
    rng = np.random.default_rng(seed)
    if kind == "solitary":
        a, d = rng.uniform(0.5, 2.0), 10.0
        dx = 800.0 / n
        return n, dx, 0.025 * dx, d, S.Body(), S.dg_solitary_state(n, dx, a, d, 0.25 * n * dx)
    if kind == "flume":
        body = S.whittaker_case(fr_index=int(rng.integers(0, 3))).body
        dx = 30.0 / n
        return n, dx, 0.005 * (400.0 / n), 0.175, body, S.dg_still_water_state(n, dx, 0.175, body)
    dx = 0.5  # rough state over a moving mound
    x = R.node_x(n, dx)
    Q0 = np.stack([2.0 + 0.1 * np.sin(0.3 * x) + 0.01 * rng.standard_normal((n, 2)),
                   0.2 * np.cos(0.2 * x) + 0.01 * rng.standard_normal((n, 2)),
                   0.05 * np.sin(x) + 0.01 * rng.standard_normal((n, 2))])
    body = S.Body(kind=S.BODY_GAUSS, law=S.LAW_CONST_VEL, amp=0.2, length=2.0,
                  x0=0.3 * n * dx, q=(0.5, 0, 0, 0, 0))
    return n, dx, 0.01, 2.0, body, Q0


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def run_batch(B, chans, nsteps):
    """chans: list of (n, dx, dt, ds, body, Q0, kw); returns (rc, per-channel
    (Q, p, marked))"""
    h = dev(np.concatenate([c[5][0] for c in chans]))
    hu = dev(np.concatenate([c[5][1] for c in chans]))
    hw = dev(np.concatenate([c[5][2] for c in chans]))
    p = torch.zeros_like(h)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    marks, cfgs = [], []
    for n, dx, dt, ds, body, Q0, kw in chans:
        m = torch.full((nsteps,), -1, dtype=torch.int32, device=DEV) if kw else None
        marks.append(m)
        cfgs.append(B.dg1d_config(n, dx, dt, ds, body, marked=m, nsteps=nsteps, **kw))
    print(f"dg1d batch nch={len(chans)} steps={nsteps} elements={sum(c[0] for c in chans)}",
          flush=True)
    rc = B.dg1d_run_batch(cfgs, 0.0, nsteps, h, hu, hw, p, status)
    out, e0 = [], 0
    H, HU, HW, P = (t.cpu().numpy() for t in (h, hu, hw, p))
    for (n, *_), m in zip(chans, marks):
        sl = slice(e0, e0 + n)
        out.append((np.stack([H[sl], HU[sl], HW[sl]]), P[sl],
                    None if m is None else m.cpu().numpy().tolist()))
        e0 += n
    return rc, out


def run_single(B, ch, nsteps):
    n, dx, dt, ds, body, Q0, kw = ch
    h, hu, hw = dev(Q0[0]), dev(Q0[1]), dev(Q0[2])
    p = torch.zeros_like(h)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    m = torch.full((nsteps,), -1, dtype=torch.int32, device=DEV) if kw else None
    rc = B.dg1d_run(n, dx, dt, ds, body, 0.0, nsteps, h, hu, hw, p, status, marked=m, **kw)
    assert rc == B.OK
    return (np.stack([a.cpu().numpy() for a in (h, hu, hw)]), p.cpu().numpy(),
            None if m is None else m.cpu().numpy().tolist())


def mixed(big=False):
    E = dict(crit=S.CRIT_ETA_D, k_nh=1e-3, enlarge=1)
    chans = [channel("solitary", 200, 1) + ({},),
             channel("solitary", 200, 2) + (E,),
             channel("flume", 400, 3) + ({},),
             channel("flume", 400, 4) + (dict(crit=S.CRIT_W, k_nh=1e-3, first_global=True),),
             channel("rough", 7, 5) + ({},),
             channel("rough", 1, 6) + (dict(crit=S.CRIT_ETA_D, k_nh=0.05),),
             channel("rough", 64, 7) + (dict(crit=S.CRIT_U_X, k_nh=0.02, enlarge=3),)]
    if big:
        chans.insert(3, channel("flume", 800, 8) + (E,))
    return chans


@pytest.mark.parametrize("big", [False, True])
def test_mixed_batch_equals_single_runs_and_the_oracle(B, big):
    """global and adaptive channels of 1 to 400 (and 800: the 1024-thread
    variant) elements in one launch"""
    chans, nsteps = mixed(big), 80
    rc, got = run_batch(B, chans, nsteps)
    assert rc == B.OK
    for k, (ch, (Qb, pb, mb)) in enumerate(zip(chans, got)):
        Qs, ps, ms = run_single(B, ch, nsteps)
        assert mb == ms, k
        for a in range(3):
            assert rel(Qb[a], Qs[a]) <= 1e-13, (k, a)
        assert rel(pb, ps) <= 1e-13 or (not pb.any() and not ps.any()), k
        n, dx, dt, ds, body, Q0, kw = ch
        if kw:
            Qr, pr, _, mr = R.run_adaptive(Q0, ds, body, 0.0, dt, nsteps, dx, kw["crit"],
                                           kw.get("k_nh", 1e-3), kw.get("enlarge", 0),
                                           first_global=kw.get("first_global", False))
            assert mb == mr, k
        else:
            Qr, pr, _ = R.run(Q0, ds, body, 0.0, dt, nsteps, dx)
        d_end = R.bottom(ds, body, R.node_x(n, dx), nsteps * dt)[0]
        assert rel(Qb[0] - d_end, Qr[0] - d_end) <= 1e-10, k
        for a in (1, 2):
            assert rel(Qb[a], Qr[a]) <= 1e-10 or np.abs(Qr[a]).max() < 1e-300, (k, a)


def test_batch_of_many_channels(B):
    """600 channels (more than one workgroup per compute unit) of 50 to 512
    elements, a third adaptive: a sample equals its single-channel runs"""
    rng = np.random.default_rng(42)
    chans = []
    for c in range(600):
        n = int(rng.integers(50, 513))
        kw = dict(crit=int(rng.integers(0, 6)), k_nh=1e-3, enlarge=int(rng.integers(0, 3))) \
            if c % 3 == 0 else {}
        chans.append(channel("solitary", n, 100 + c) + (kw,))
    nsteps = 40
    rc, got = run_batch(B, chans, nsteps)
    assert rc == B.OK
    for k in list(range(0, 600, 37)) + [599]:
        Qs, ps, ms = run_single(B, chans[k], nsteps)
        Qb, pb, mb = got[k]
        assert mb == ms, k
        for a in range(3):
            assert rel(Qb[a], Qs[a]) <= 1e-13, (k, a)


def test_batch_argument_checks(B):
    """an empty batch, one invalid config among valid ones, or a missing array
    give EINVAL and leave the state untouched"""
    chans = mixed()[:3]
    good = [B.dg1d_config(c[0], c[1], c[2], c[3], c[4]) for c in chans]
    bad = B.dg1d_config(chans[1][0], chans[1][1], -1.0, chans[1][3], chans[1][4])
    tot = sum(c[0] for c in chans)
    h = dev(np.full((tot, 2), 3.0))
    z = torch.zeros_like(h)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    assert B.dg1d_run_batch([good[0], bad, good[2]], 0.0, 5, h, z, z.clone(), z.clone(),
                            st) == B.EINVAL
    assert B.dg1d_run_batch([], 0.0, 5, h, z, z.clone(), z.clone(), st) == B.EINVAL
    assert torch.all(h == 3.0)


@pytest.mark.parametrize("adaptive", [False, True])
def test_batch_of_one_is_the_single_run_bit_for_bit(B, adaptive):
    """a batch of one channel runs the same kernel variant as the single-
    channel call (same thread count, same model): the same bits"""
    kw = dict(crit=S.CRIT_ETA_D, k_nh=1e-3, enlarge=1) if adaptive else {}
    ch = channel("solitary", 200, 11) + (kw,)
    rc, got = run_batch(B, [ch], 60)
    assert rc == B.OK
    Qs, ps, ms = run_single(B, ch, 60)
    Qb, pb, mb = got[0]
    assert np.array_equal(Qb, Qs) and np.array_equal(pb, ps) and mb == ms


def test_batch_reports_a_dry_channel(B):
    """a node depth <= 0 in one channel of a batch gives EDRY for the call"""
    chans = [channel("rough", 32, 21) + ({},), channel("rough", 32, 22) + ({},),
             channel("rough", 32, 23) + ({},)]
    Q = chans[1][5].copy()
    Q[0][5, 1] = -0.1
    chans[1] = chans[1][:5] + (Q, {})
    rc, _ = run_batch(B, chans, 2)
    assert rc == B.EDRY
