"""Autotuner for the persistent Sign kernel's schedule.

The schedule has two knobs (dil_ctx_set_param):
  persist.hmax  tasks a workgroup holds at once; with G = 64 / l candidate
                slots per batch, each held task gets G / hmax consecutive
                nonces per batch (hmax = G: no speculation until tasks retire);
  persist.grid  workgroups launched (at most the number the GPU keeps
                resident; fewer concentrate tasks into fewer, fuller groups).
Small hmax fills the GPU with speculative nonces and shortens the tail but
wastes work on iterations after the first valid one; large hmax wastes none
but leaves the GPU underfilled for small batches.  The best point depends on
the batch size, the level and the GPU, so it is measured: every candidate runs
the caller's own batch (Sign is deterministic, so every candidate produces the
same signatures) and the fastest median wins.
"""
from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np


def slots_per_batch(level: int) -> int:
    return 64 // {2: 4, 3: 5, 5: 7}[level]


def candidates(level: int, count: int, resident_groups: int) -> List[tuple]:
    g = slots_per_batch(level)
    hm = sorted({h for h in (1, 2, 3, 4, 6, 8, 12, 16) if h <= g} | {g})
    out = []
    for h in hm:
        need = -(-count // h)
        for frac in (1.0, 0.5):
            grid = max(1, min(int(resident_groups * frac), need))
            if (h, grid) not in out:
                out.append((h, grid))
    return out


def tune_sign(ctx, level: int, run, resident_groups: int, reps: int = 3,
              cands: Optional[List[tuple]] = None, count: Optional[int] = None) -> Dict:
    """Time `run()` (one Sign call on ctx) for each (hmax, grid) candidate; leave the best set on ctx.

    run: callable issuing the Sign batch on the current stream.
    resident_groups: workgroups the GPU keeps resident for the persistent kernel.
    """
    import torch
    cands = cands or candidates(level, count, resident_groups)
    table = []
    for h, grid in cands:
        ctx.set_param("persist.hmax", h)
        ctx.set_param("persist.grid", grid)
        run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            run()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        ev, seq = ctx.sign_stats()
        table.append({"hmax": h, "grid": grid, "ms": float(np.median(ts)), "evaluated": ev, "sequential": seq})
    best = min(table, key=lambda r: r["ms"])
    ctx.set_param("persist.hmax", best["hmax"])
    ctx.set_param("persist.grid", best["grid"])
    return {"best": best, "table": table}
