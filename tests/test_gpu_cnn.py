"""GPU parity of the warm-start network kernels (BF16 matrix cores, FP32
accumulation) against the FP64 NumPy oracle, and of the learned-warm-start
solve against the FP64 solver oracle.

Two bars for the network: (1) against the oracle evaluated with the same
storage roundings as the kernels (BF16 weights, activations and input
gradients), relative L2 <= 1e-2 (only the FP32 summation order differs);
(2) against the exact FP64 oracle, relative L2 <= 3e-2 for the output and
<= 0.1 for the weight gradients: the BF16 input gradients lose about 1% per
layer of depth (0.3% at the last layer, 7% at the first for this case)."""
import numpy as np
import pytest

import oracle as O
import swe_inputs as S
from oracle import cnn as OC

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17025_amd import swe_nh
    return swe_nh


def bf16_bits(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def round_weights(p):
    """BF16 weights (the kernels round them), FP32 biases (added in FP32)"""
    q = np.array(p, dtype=np.float64)
    o = 0
    for (nw, nb) in OC.layer_sizes():
        q[o:o + nw] = bf16_value(bf16_bits(q[o:o + nw]))
        o += nw + nb
    return q


def inputs(n, h, w, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, h, w, 16), np.float32)
    x[..., :5] = rng.standard_normal((n, h, w, 5))
    xb = bf16_bits(x)
    return xb, bf16_value(xb)


def params(seed):
    rng = np.random.default_rng(seed)
    p = OC.init_params(seed).astype(np.float64)
    o = 0
    for (nw, nb) in OC.layer_sizes():
        p[o + nw:o + nw + nb] = 0.05 * rng.standard_normal(nb)
        o += nw + nb
    return p.astype(np.float32)


def emulated(pr, xv, G):
    """the oracle's convolutions with the kernels' storage roundings"""
    rb = lambda a: bf16_value(bf16_bits(a))
    L = OC.unpack(pr)
    a, acts = xv, []
    for l, (W, b) in enumerate(L):
        z = OC.conv3x3(a, W, b)
        a = rb(np.maximum(z, 0.0)) if l < 5 else z
        acts.append(a)
    ins = [xv] + acts[:-1]
    g = rb(G[..., None].astype(np.float64))
    grads = [None] * 6
    n, h, w = G.shape
    for l in range(5, -1, -1):
        W, b = L[l]
        ap = np.pad(ins[l], ((0, 0), (1, 1), (1, 1), (0, 0)))
        dW = np.zeros_like(W)
        for ky in range(3):
            for kx in range(3):
                dW[:, ky, kx, :] = np.einsum("nyxo,nyxc->oc", g, ap[:, ky:ky + h, kx:kx + w, :])
        grads[l] = (dW, g.sum(axis=(0, 1, 2)))
        if l > 0:
            gp = np.pad(g, ((0, 0), (1, 1), (1, 1), (0, 0)))
            dx = np.zeros_like(ins[l])
            for ky in range(3):
                for kx in range(3):
                    dx += gp[:, 2 - ky:2 - ky + h, 2 - kx:2 - kx + w, :] @ W[:, ky, kx, :]
            g = rb(dx * (ins[l] > 0.0))
    return acts[-1][..., 0], OC.pack(grads)


def test_forward_backward_match_oracle(B):
    n, h, w = 2, 32, 48
    xb, xv = inputs(n, h, w, 1)
    p = params(2)
    net = B.Net(n, h, w)
    pt = torch.tensor(p, device=DEV)
    xt = torch.tensor(xb.view(np.int16), device=DEV)
    out = torch.empty((n, h, w), dtype=torch.float32, device=DEV)
    net.forward(pt, xt, out)
    pr = round_weights(p)
    ref = OC.forward(pr, xv)[-1][..., 0]
    rng = np.random.default_rng(5)
    G = rng.standard_normal((n, h, w)).astype(np.float32)
    emu_out, emu_g = emulated(pr, xv, G)
    o_gpu = out.cpu().numpy()
    assert rel(o_gpu, emu_out) <= 1e-2
    assert rel(o_gpu, ref) <= 3e-2
    grad = torch.empty_like(pt)
    net.backward(pt, xt, torch.tensor(G, device=DEV), grad)
    gref = OC.backward(pr, xv, G[..., None].astype(np.float64))
    g = grad.cpu().numpy()
    o = 0
    for l, (nw, nb) in enumerate(OC.layer_sizes()):
        if l == 0:  # input channels 5..15 are zero: their weights get no gradient
            W = g[o:o + nw].reshape(32, 3, 3, 16)
            assert np.all(W[..., 5:] == 0.0)
        assert rel(g[o:o + nw], emu_g[o:o + nw]) <= 1e-2, l
        assert rel(g[o + nw:o + nw + nb], emu_g[o + nw:o + nw + nb]) <= 1e-2, l
        assert rel(g[o:o + nw], gref[o:o + nw]) <= 0.1, l
        assert rel(g[o + nw:o + nw + nb], gref[o + nw:o + nw + nb]) <= 0.1, l
        o += nw + nb


def test_adam_and_mse(B):
    n, h, w = 1, 16, 32
    net = B.Net(n, h, w)
    rng = np.random.default_rng(7)
    p = rng.standard_normal(OC.param_count()).astype(np.float32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pt, mt, vt = (torch.tensor(a, device=DEV) for a in (p, m, v))
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.standard_normal(p.size).astype(np.float32)
        net.adam(pt, mt, vt, torch.tensor(g, device=DEV), step, 1e-2)
        pr, mr, vr = OC.adam(pr, mr, vr, g.astype(np.float64), step, 1e-2)
    assert rel(pt.cpu().numpy(), pr) <= 1e-6
    o = rng.standard_normal((n, h, w)).astype(np.float32)
    t = rng.standard_normal((n, h, w)).astype(np.float32)
    wt = (rng.random((n, h, w)) < 0.3).astype(np.float32)
    dout = torch.empty((n, h, w), dtype=torch.float32, device=DEV)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    net.mse(*(torch.tensor(a, device=DEV) for a in (o, t, wt)), dout, loss)
    ls = np.sum(wt * (o - t) ** 2, dtype=np.float64) / wt.sum()
    assert abs(loss.item() - ls) <= 1e-6 * ls
    assert rel(dout.cpu().numpy(), 2 * wt * (o - t) / wt.sum()) <= 1e-6


def test_features(B):
    c = S.random_case_2d(48, 32, seed=4, dx=2.0, dy=2.0, h0=50.0)
    ctx = B.context_2d(c, crit=0, tol=1e-10, max_iter=1000)
    rng = np.random.default_rng(1)
    mask = (rng.random((32, 48)) < 0.5).astype(np.uint8)
    out = torch.empty((32, 48, 16), dtype=torch.int16, device=DEV)
    t1, h0 = 0.37, 50.0
    c0 = np.sqrt(9.81 * h0)
    sc = [h0 * 1e-3, h0 * c0 * 1e-2, h0 * c0 * 2e-2, c0 * 1e-2]
    f = lambda a: torch.tensor(a, dtype=torch.float64, device=DEV)
    ctx.features(f(c.h), f(c.hu), f(c.hv), torch.tensor(mask, device=DEV), t1, sc, out)
    got = bf16_value(out.cpu().numpy().view(np.uint16))
    d, d_t, *_ = O.forcing_2d(c.ds, c.dx, c.dy, c.body, t1)
    ref = np.stack([(c.h - d) / sc[0], c.hu / sc[1], c.hv / sc[2], -d_t / sc[3],
                    mask.astype(np.float64)], axis=-1)
    # one BF16 rounding on each side: equal to within one unit in the last place
    assert np.all(np.abs(got[..., :5] - ref) <= 2.0 ** -7 * np.abs(ref) + 1e-30)
    assert np.all(got[..., 5:] == 0.0)


def test_network_guess_keeps_the_solution(B):
    """warm = 2: the PCG from the network's guess converges to the same
    pressure (the guess changes iteration counts only)"""
    c = S.random_case_2d(64, 48, seed=6, dx=2.0, dy=2.0, h0=50.0)
    kw = dict(crit=S.CRIT_ETA_D, k_nh=2e-3, enlarge=1, cfl=0.4, precision=0, tol=1e-13,
              max_iter=50000)
    ctx = B.context_2d(c, warm=2, **kw)
    pt = torch.tensor(params(9), device=DEV)
    ctx.set_warm_start_net(pt, [0.05, 1.0, 1.0, 0.1], 100.0)
    ctx.set_time(c.t0)
    f = lambda a: torch.tensor(a, dtype=torch.float64, device=DEV)
    h, hu, hv, hw = f(c.h), f(c.hu), f(c.hv), f(c.hw)
    p = torch.zeros_like(h)
    m = torch.zeros((48, 64), dtype=torch.uint8, device=DEV)
    ctx.step(h, hu, hv, hw, p, m, nsteps=5)
    st = ctx.sync_stats()
    assert st["status"] == 0, st
    ref = O.Sim2D(c, O.phys_struct(crit=S.CRIT_ETA_D, k_nh=2e-3, enlarge=1, tol=1e-14),
                  cfl=0.4).step(5)
    assert st["n_active"] == ref.last_active > 0
    for g, r in ((h, ref.h), (hu, ref.hu), (hv, ref.hv), (hw, ref.hw), (p, ref.p)):
        assert rel(g.cpu().numpy(), r) <= 1e-10
