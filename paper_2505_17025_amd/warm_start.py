"""Learned warm start of the 2D pressure solve: data generation with the
solver itself, training with the project's HIP network kernels (forward,
backward, Adam), and evaluation of the PCG iterations it saves.

Everything numeric runs in libswe_nh.so; this module only moves tensors:
random crops of the solver's fields, batching, and the training loop.
"""
from __future__ import annotations

import numpy as np
import torch

from . import swe_nh as B

RHO, G = 1000.0, 9.81


def he_init(seed):
    """He-normal weights (std sqrt(2 / fan_in)) and zero biases, in the
    network's parameter layout"""
    rng = np.random.default_rng(seed)
    cin = [16, 32, 32, 32, 32, 32]
    cout = [32, 32, 32, 32, 32, 1]
    parts = []
    for ci, co in zip(cin, cout):
        parts.append((rng.standard_normal(co * 9 * ci) * np.sqrt(2.0 / (9 * ci))).astype(np.float32))
        parts.append(np.zeros(co, np.float32))
    p = np.concatenate(parts)
    assert p.size == B.Net.param_count()
    return p


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def snapshots(case, nsteps, every, scales, tol=1e-8, precision=1):
    """run the solver on `case` and yield (features bf16 [ny,nx,16] as int16,
    pressure [ny,nx] FP32 in Pa, mask uint8, time, predictor state) of the
    predictor state of every `every`-th step, the pressure solved to `tol`"""
    ctx = B.context_2d(case, crit=0, k_nh=1e-3, enlarge=1, cfl=0.5, precision=precision, tol=tol,
                       max_iter=100000, warm=1)
    ctx.set_time(case.t0)
    h, hu, hv, hw = (_dev(a) for a in (case.h, case.hu, case.hv, case.hw))
    p = torch.zeros_like(h)
    ht, mt, nt, kt = (torch.empty_like(h) for _ in range(4))
    mask = torch.zeros(h.shape, dtype=torch.uint8, device="cuda")
    feat = torch.empty(h.shape + (16,), dtype=torch.int16, device="cuda")
    pk = torch.zeros_like(h)
    for k in range(1, nsteps + 1):
        if k % every == 0:
            st = ctx.sync_stats()
            t = float(ctx.get_time()[0])
            dt = st["dt"] if st["dt"] > 0 else 0.01
            # the stage calls reproduce the step's predictor and pressure
            ctx.predict(h, hu, hv, hw, t, dt, ht, mt, nt, kt)
            na = ctx.mask(ht, mt, nt, kt, t + dt, 0, mask)
            if na > 0:
                pk.zero_()
                ctx.solve_pressure(ht, mt, nt, kt, mask, t, dt, pk)
                ctx.features(ht, mt, nt, mask, t + dt, scales, feat)
                yield feat.clone(), pk.float().clone(), mask.clone(), (ctx, t, dt, ht, mt, nt, kt, p)
        ctx.step(h, hu, hv, hw, p)
    st = ctx.sync_stats()
    if st["status"] != 0:
        raise RuntimeError(f"data run failed: {st}")


def bf16_to_float(x):
    return (x.to(torch.int32) << 16).view(torch.float32)


def estimate_scales(case, nsteps, every, tol=1e-8):
    """standard deviations of eta, hu, hv and -d_t on the marked cells"""
    acc = torch.zeros(4, dtype=torch.float64, device="cuda")
    cnt = 0.0
    for f, _, m, _ in snapshots(case, nsteps, every, [1.0, 1.0, 1.0, 1.0], tol=tol):
        v = bf16_to_float(f[..., :4].contiguous()).double()
        w = m.double()[..., None]
        acc += (v * v * w).sum(dim=(0, 1))
        cnt += float(m.sum())
    s = torch.sqrt(acc / max(cnt, 1.0)).cpu().numpy()
    return [float(x) if x > 0 else 1.0 for x in s]


def crops(feat, p, mask, ncrop, size, rng):
    """random size x size crops centred near marked cells"""
    ny, nx = mask.shape
    idx = torch.nonzero(mask).cpu().numpy()
    out = []
    for _ in range(ncrop):
        cy, cx = idx[rng.integers(len(idx))] + rng.integers(-size // 4, size // 4 + 1, size=2)
        y0 = int(np.clip(cy - size // 2, 0, ny - size))
        x0 = int(np.clip(cx - size // 2, 0, nx - size))
        out.append((feat[y0:y0 + size, x0:x0 + size], p[y0:y0 + size, x0:x0 + size],
                    mask[y0:y0 + size, x0:x0 + size]))
    return out


def dataset(seeds, scales, n=1024, dx=4.0, nsteps=200, every=10, crops_per=16, size=128, tol=1e-8,
            seed=0, make_case=None):
    import swe_inputs as S
    make_case = make_case or (lambda s: S.warm_start_case_2d(s, n=n, dx=dx))
    rng = np.random.default_rng(seed)
    X, P, M = [], [], []
    for s in seeds:
        for f, p, m, _ in snapshots(make_case(s), nsteps, every, scales, tol=tol):
            for a, b, c in crops(f, p, m, crops_per, size, rng):
                X.append(a)
                P.append(b)
                M.append(c)
    X = torch.stack(X).contiguous()
    P = torch.stack(P).contiguous()
    M = torch.stack(M).float().contiguous()
    return X, P, M


def train(X, P, M, iters=1000, batch=16, lr=1e-3, seed=0, log_every=0):
    """fit the network to the normalised pressure; returns (params, p_scale, losses)"""
    n, h, w = P.shape
    scale = float(torch.sqrt((P.double() ** 2 * M).sum() / M.sum().clamp(min=1.0)))
    T = (P / scale).contiguous()
    params = torch.tensor(he_init(seed), device="cuda")
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    net = B.Net(batch, h, w)
    out = torch.empty((batch, h, w), dtype=torch.float32, device="cuda")
    dout = torch.empty_like(out)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    run = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for it in range(1, iters + 1):
        sel = torch.randint(0, n, (batch,), generator=g).cuda()
        xb = X.index_select(0, sel).contiguous()
        tb = T.index_select(0, sel).contiguous()
        wb = M.index_select(0, sel).contiguous()
        net.forward(params, xb, out)
        net.mse(out, tb, wb, dout, loss)
        net.backward(params, xb, dout, grad)
        rate = lr * (0.1 ** (it / iters))  # exponential decay to lr / 10
        net.adam(params, m, v, grad, it, rate)
        run += loss
        if log_every and it % log_every == 0:
            losses.append(float(run.item()) / log_every)
            run.zero_()
    return params, scale, losses


def guess(params, p_scale, feat, mask):
    """network guess (Pa) for one field"""
    ny, nx = mask.shape
    net = B.Net(1, ny, nx)
    out = torch.empty((1, ny, nx), dtype=torch.float32, device="cuda")
    net.forward(params, feat.reshape(1, ny, nx, 16).contiguous(), out)
    return (out[0].double() * p_scale) * mask.double()


def evaluate(params, p_scale, scales, case, nsteps, every, tol=1e-8):
    """PCG iterations to tol from the zero guess, the network's guess and the
    previous step's pressure, on the predictor states of a held-out run"""
    res = {"zero": [], "learned": [], "previous": []}
    for f, _, m, (ctx, t, dt, ht, mt, nt, kt, p) in snapshots(case, nsteps, every, scales, tol=tol):
        for name, g0 in (("zero", torch.zeros_like(p)), ("learned", guess(params, p_scale, f, m)),
                         ("previous", p * m.double())):
            pk = g0.contiguous().clone()
            it, rr = ctx.solve_pressure(ht, mt, nt, kt, m, t, dt, pk)
            res[name].append(it)
    return res
