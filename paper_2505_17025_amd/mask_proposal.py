"""Learned proposal of the non-hydrostatic area: the warm-start network's
architecture (six 3x3 BF16 convolutions on the matrix cores) trained as a
per-cell classifier of the criterion's marked set (|eta/d| > k_nh widened by
the enlargement, Sec. 5.1-5.2) from the predictor state alone (the mask
channel of the input is left at zero), with the weighted binary cross-entropy
of its logits.  A proposal is the set of cells with a positive logit; the
stage entry points solve the pressure on it like on the criterion's set.

Everything numeric runs in libswe_nh.so; this module only moves tensors:
snapshots of the solver's own runs, random crops, batching and the training
loop.
"""
from __future__ import annotations

import numpy as np
import torch

from . import swe_nh as B
from .warm_start import _dev, bf16_to_float, he_init


def snapshots(case, nsteps, every, scales, k_nh=1e-3, enlarge=1, cover=0, tol=1e-8):
    """run the adaptive solver (|eta/d|) on `case`; for the predictor state
    of every `every`-th step yield (features bf16 [ny,nx,16] as int16 with a
    zero mask channel, the criterion's mask uint8 widened by `cover` more
    cells of enlargement, (ctx, t, dt, ht, mt, nt, kt, p, criterion mask))"""
    ctx = B.context_2d(case, crit=0, k_nh=k_nh, enlarge=enlarge, cfl=0.5, precision=1, tol=tol,
                       max_iter=100000, warm=1)
    wide = (B.context_2d(case, crit=0, k_nh=k_nh, enlarge=enlarge + cover, cfl=0.5, precision=1,
                         tol=tol, max_iter=100000, warm=1) if cover else None)
    ctx.set_time(case.t0)
    h, hu, hv, hw = (_dev(a) for a in (case.h, case.hu, case.hv, case.hw))
    p = torch.zeros_like(h)
    ht, mt, nt, kt = (torch.empty_like(h) for _ in range(4))
    mask = torch.zeros(h.shape, dtype=torch.uint8, device="cuda")
    target = torch.zeros_like(mask)
    none = torch.zeros_like(mask)
    feat = torch.empty(h.shape + (16,), dtype=torch.int16, device="cuda")
    for k in range(1, nsteps + 1):
        if k % every == 0:
            st = ctx.sync_stats()
            t = float(ctx.get_time()[0])
            dt = st["dt"] if st["dt"] > 0 else 0.01
            ctx.predict(h, hu, hv, hw, t, dt, ht, mt, nt, kt)
            na = ctx.mask(ht, mt, nt, kt, t + dt, 0, mask)
            if na > 0:
                if wide is not None:
                    wide.mask(ht, mt, nt, kt, t + dt, 0, target)
                else:
                    target.copy_(mask)
                ctx.features(ht, mt, nt, none, t + dt, scales, feat)
                yield feat.clone(), target.clone(), (ctx, t, dt, ht, mt, nt, kt, p, mask.clone())
        ctx.step(h, hu, hv, hw, p)
    st = ctx.sync_stats()
    if st["status"] != 0:
        raise RuntimeError(f"data run failed: {st}")


def crops(feat, mask, ncrop, size, rng, near=0.75):
    """size x size crops: a fraction `near` centred near marked cells, the
    rest anywhere (so that the unmarked far field is seen too)"""
    ny, nx = mask.shape
    idx = torch.nonzero(mask).cpu().numpy()
    out = []
    for _ in range(ncrop):
        if rng.random() < near:
            cy, cx = idx[rng.integers(len(idx))] + rng.integers(-size // 4, size // 4 + 1, size=2)
        else:
            cy, cx = rng.integers(0, ny), rng.integers(0, nx)
        y0 = int(np.clip(cy - size // 2, 0, ny - size))
        x0 = int(np.clip(cx - size // 2, 0, nx - size))
        out.append((feat[y0:y0 + size, x0:x0 + size], mask[y0:y0 + size, x0:x0 + size]))
    return out


def dataset(seeds, scales, make_case, nsteps=100, every=10, crops_per=16, size=64, seed=0,
            cover=0):
    rng = np.random.default_rng(seed)
    X, M = [], []
    for s in seeds:
        for f, m, _ in snapshots(make_case(s), nsteps, every, scales, cover=cover):
            for a, b in crops(f, m, crops_per, size, rng):
                X.append(a)
                M.append(b)
    return torch.stack(X).contiguous(), torch.stack(M).float().contiguous()


def train(X, M, iters=1000, batch=16, lr=2e-3, seed=0, log_every=0):
    """fit the network's logits to the marked set; returns (params, losses)"""
    n, h, w = M.shape
    params = torch.tensor(he_init(seed), device="cuda")
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    net = B.Net(batch, h, w)
    out = torch.empty((batch, h, w), dtype=torch.float32, device="cuda")
    dout = torch.empty_like(out)
    wt = torch.ones((batch, h, w), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    run = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for it in range(1, iters + 1):
        sel = torch.randint(0, n, (batch,), generator=g).cuda()
        xb = X.index_select(0, sel).contiguous()
        tb = M.index_select(0, sel).contiguous()
        net.forward(params, xb, out)
        net.bce(out, tb, wt, dout, loss)
        net.backward(params, xb, dout, grad)
        net.adam(params, m, v, grad, it, lr * (0.1 ** (it / iters)))
        run += loss
        if log_every and it % log_every == 0:
            losses.append(float(run.item()) / log_every)
            run.zero_()
    return params, losses


def propose(params, feat):
    """the proposed marked set (uint8 [ny, nx]): cells with a positive logit"""
    ny, nx = feat.shape[:2]
    net = B.Net(1, ny, nx)
    out = torch.empty((1, ny, nx), dtype=torch.float32, device="cuda")
    net.forward(params, feat.reshape(1, ny, nx, 16).contiguous(), out)
    return (out[0] > 0).to(torch.uint8)


def scores(pred, true):
    """intersection over union, precision and recall of a proposed set"""
    p, t = pred.bool(), true.bool()
    inter = float((p & t).sum())
    union = float((p | t).sum())
    return {"iou": inter / max(union, 1.0), "precision": inter / max(float(p.sum()), 1.0),
            "recall": inter / max(float(t.sum()), 1.0)}


def evaluate(params, scales, case, nsteps, every, cover=0, tol=1e-8):
    """on the predictor states of a held-out run: the proposal's scores
    against its training target (the criterion's set widened by `cover`
    cells) and its recall of the criterion's own set; the pressure solved on
    the criterion's set, on the proposed set and on the whole grid (the
    global model), each adaptive pressure's relative L2 difference from the
    global one over the criterion's set, and the iteration counts"""
    rows = []
    for f, tgt, (ctx, t, dt, ht, mt, nt, kt, p, crit) in snapshots(case, nsteps, every, scales,
                                                                   cover=cover, tol=tol):
        prop = propose(params, f)
        row = scores(prop, tgt)
        row["recall_of_criterion"] = scores(prop, crit)["recall"]
        pres = {}
        for name, mk in (("criterion", crit), ("proposal", prop),
                         ("global", torch.ones_like(crit))):
            pk = torch.zeros_like(p)
            it, _ = ctx.solve_pressure(ht, mt, nt, kt, mk.contiguous(), t, dt, pk)
            pres[name] = (pk, it)
        sel = crit.bool()
        g = pres["global"][0][sel]
        for name in ("criterion", "proposal"):
            row[f"{name}_vs_global"] = float(torch.linalg.norm(pres[name][0][sel] - g) /
                                             torch.linalg.norm(g).clamp(min=1e-300))
        row["iters"] = {k: v[1] for k, v in pres.items()}
        row["marked"] = int(crit.sum())
        rows.append(row)
    return rows
