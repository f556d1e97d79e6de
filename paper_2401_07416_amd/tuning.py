"""Tile shapes of the half-step kernels chosen by measurement.

``tune_table.json`` maps "<nx>x<ny>x<nz>:<precision>" to the tile (the
keyword arguments of ``Sim.set_tile``: two-pass rows/waves/zc, one-pass
fused/fused_rows/fused_zc) that a sweep on the MI355X found fastest for that
grid.  Grids absent from the table run the library's defaults.  ``autotune``
re-measures a grid in place.
"""
from __future__ import annotations

import json
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tune_table.json")


def _key(nx, ny, nz, precision):
    return f"{nx}x{ny}x{nz}:{precision}"


def load_table() -> dict:
    if not os.path.exists(TABLE):
        return {}
    with open(TABLE) as f:
        return json.load(f)


def tile_for(w, precision: str) -> Optional[dict]:
    t = load_table().get(_key(w.nx, w.ny, w.nz, precision))
    return dict(t["tile"]) if t else None


def candidates(nz: int):
    """Two-pass tiles, one-pass tiles, then two-step sweep tiles, as set_tile
    keyword dicts."""
    for rows in (1, 2, 4):
        for waves in (1, 2, 4):
            for zc in (1, 2, 4, 8, 16, 32, 64, 128, 256):
                if zc <= nz:
                    yield dict(fused=0, two_step=0, rows=rows, waves=waves, zc=zc)
    for ft in (256, 128, 64):
        for fr in (2, 3, 4):
            for zc in (1, 2, 4, 8, 16, 32, 64, 128):
                if zc <= nz:
                    yield dict(fused=1, two_step=0, fused_rows=fr, fused_zc=zc, fused_prefetch=0,
                               fused_threads=ft)
    for fr in (2, 3):
        for zc in (16, 64):
            if zc <= nz:
                yield dict(fused=1, two_step=0, fused_rows=fr, fused_zc=zc, fused_prefetch=1,
                           fused_threads=256)
    for tx in (16, 24, 32, 40, 56, 64, 120):
        for rows, threads in ((2, 256), (1, 512), (2, 512), (1, 1024)):
            for zc in (32, 64, 128):
                if zc <= nz:
                    yield dict(fused=1, two_step=1, two_step_tx=tx, two_step_rows=rows,
                               two_step_zc=zc, two_step_prefetch=1, two_step_threads=threads)


def autotune(sim, steps: int = 20, reps: int = 3, cands=None):
    """Time each candidate tile on a live simulation (the state advances;
    use a scratch simulation).  Tiles the grid cannot take are skipped.
    Returns [(ms_per_step, tile)] sorted."""
    import torch

    from .tdse import TdseError
    res = []
    if cands is None:
        # the library's own default for this grid (its cost-model choice of
        # the two-step tile) is timed with the list
        t = sim.get_tile()
        cur = dict(fused=t.fused, two_step=t.two_step)
        if t.two_step:
            cur.update(two_step_tx=t.two_step_tx, two_step_rows=t.two_step_rows,
                       two_step_zc=t.two_step_zc, two_step_prefetch=t.two_step_prefetch,
                       two_step_threads=t.two_step_threads)
        cands = list(candidates(sim.desc.nz)) + [cur]
    # one-time costs (first launches, code loading) land here, not on the
    # first candidate
    sim.step(4)
    torch.cuda.synchronize()
    for tile in cands:
        try:
            sim.set_tile(**tile)
        except TdseError:
            continue
        sim.step(2)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            sim.step(steps)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / steps)
        res.append((best, tile))
    res.sort()
    return res


def autotune_batch(batch, intervals: int = 2, cands=None):
    """Time batch tiles (the members advance; use a scratch batch).  A
    candidate is ("one-pass", fused_rows, fused_zc, prefetch, threads) or
    ("two-step", tx, rows, zc, threads); returns [(ms_per_step, candidate)]
    sorted, and leaves the batch prepared with the best."""
    import torch

    from .tdse import TdseError

    def apply(c):
        if c[0] == "two-step":
            _, tx, rows, zc, threads = c
            batch.set_two_step(True, tx=tx, zc=zc, prefetch=True, rows=rows, threads=threads)
        else:
            _, m, zc, pf, ft = c
            batch.set_two_step(False)
            batch.set_tile(m, zc, pf, ft)

    if cands is None:
        cands = [("two-step", tx, rows, zc, nt) for tx in (32, 56, 64)
                 for rows, nt in ((1, 512), (2, 256), (1, 1024)) for zc in (32, 64, 128)]
        cands += [("one-pass", m, zc, 0, 256) for m in (2, 3) for zc in (16, 32, 64)]
    res = []
    interval = None
    for c in cands:
        try:
            apply(c)
            batch.prepare()
        except TdseError:
            continue
        if interval is None:
            w = batch.members[0].desc.record_every
            interval = int(w) if w > 0 else 64
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(batch.stream)
        batch.run(intervals * interval)
        e1.record(batch.stream)
        e1.synchronize()
        res.append((e0.elapsed_time(e1) / (intervals * interval), c))
    res.sort()
    if res:
        apply(res[0][1])
        batch.prepare()
    return res
