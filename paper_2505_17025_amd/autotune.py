"""Launch-shape autotuner.

The 1D stencil, criterion and compaction kernels work on tiles whose LDS
windows hold 128, 256 or 512 cells; which tile is fastest depends on the packed
length and on how the tiles spread over the 256 compute units (short channels
favour small tiles, long ensembles large ones).  The fused step (either
precision) widens a tile by 6 + e cells on each side (e = enlargement), so for each capacity the
tile of capacity - 2 (6 + e) cells, whose window fills whole wavefronts, is a
candidate beside the full capacity.  `tune_1d` times whole steps for every
candidate on a copy of the caller's state and returns the fastest; results are
kept per (cells, channels, precision, criterion, enlargement, steps timed) in a
JSON table so that a later run on the same device skips the sweep.  The span of
steps matters: the marked region grows during a run, and a tile that is best
while few tiles are marked can lose later (its level-1 system outgrows one
wavefront sooner), so the span should cover the run being tuned for.

All timing goes through the library's own step entry point; this module only
picks the knob.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import swe_nh as B

CAPACITIES_1D = (128, 256, 512)
FUSED_MAX_ENLARGE = 8  # largest enlargement the fused step handles


def candidates_1d(kw):
    """tile lengths worth timing for the context options `kw`"""
    e = int(kw.get("enlarge", 1))
    fused = e <= FUSED_MAX_ENLARGE
    out = []
    for cap in CAPACITIES_1D:
        if fused:
            out.append(cap - 2 * (6 + e))
        out.append(cap)
    return tuple(out)


def _key(dev_name, cells, batch, kw, warmup, nsteps):
    return (f"{dev_name}|1d|cells={cells}|batch={batch}|prec={kw.get('precision', 0)}"
            f"|crit={kw.get('crit', 0)}|e={kw.get('enlarge', 1)}|steps={warmup}+{nsteps}")


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _save(path, table):
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_steps(case, kw, state, t0, nsteps, warmup):
    ctx = B.context_1d(case, **kw)
    ctx.set_time(t0)
    h, hu, hw = (a.clone() for a in state)
    p = torch.zeros_like(h)
    ctx.step(h, hu, None, hw, p, nsteps=warmup)
    torch.cuda.synchronize()
    s = time.perf_counter()
    ctx.step(h, hu, None, hw, p, nsteps=nsteps)
    torch.cuda.synchronize()
    el = time.perf_counter() - s
    st = ctx.sync_stats()
    if st["status"] != 0:
        raise RuntimeError(f"autotune run failed: {st}")
    return el / nsteps


def tune_1d(case, kw, state, t0, nsteps=200, warmup=20, table_path=None, candidates=None):
    """fastest tile1d for `case` with the context options `kw`; `state` is the
    (h, hu, hw) device tensors (copied, never written) and `t0` the start
    time(s).  Returns (tile, {tile: seconds per step})."""
    if candidates is None:
        candidates = candidates_1d(kw)
    cells = int(state[0].numel())
    batch = len(case.channels) if hasattr(case, "channels") else 1
    key = _key(torch.cuda.get_device_name(0), cells, batch, kw, warmup, nsteps)
    table = _load(table_path)
    if key in table:
        e = table[key]
        return int(e["tile"]), {int(k): v for k, v in e["s_per_step"].items()}
    times = {}
    for t in candidates:
        times[t] = _time_steps(case, dict(kw, tile1d=t), state, t0, nsteps, warmup)
    best = min(times, key=times.get)
    table[key] = {"tile": best, "s_per_step": {str(k): v for k, v in times.items()}}
    _save(table_path, table)
    return best, times
