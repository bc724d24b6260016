"""Tile-shape autotuner.

The particle and rank kernels take one block per tile of cells, one wavefront per tile row.
The tile shape sets the particles per block, the LDS per block and the balance between
blocks; the context's default comes from a rule of thumb (about 1024 particles per tile row
and species).  The tuner times whole cycles for candidate shapes on a live context
(pic_set_tiles, then HIP-event timing of a few cycles) and leaves the fastest shape applied.
Re-tiling does not change results beyond the order of floating-point atomic additions, but the
timed cycles do advance the context: tune before the cycles that matter, or on a copy.
"""
from __future__ import annotations

from . import binding

# (0, 0) is the library's own choice from the load.
CANDIDATES = [(0, 0), (4, 4), (8, 4), (16, 4), (32, 4), (8, 2), (16, 2), (32, 2), (16, 1),
              (32, 1), (8, 8), (16, 8)]


def tune_tiles(ctx, candidates=CANDIDATES, cycles=4, warmup=1, repeats=2):
    """Time `cycles` cycles (after `warmup` untimed ones), `repeats` times, for every candidate
    tile shape that fits in LDS, keep each shape's best repeat (timings of a few cycles vary
    by several per cent), and apply and return the fastest.  Returns {"best": (tx, tz),
    "ms_per_cycle": {(tx, tz): ms}, "cycles_used": n}."""
    timings = {}
    used = 0
    for tile in candidates:
        try:
            ctx.set_tiles(*tile)
        except binding.PicError:
            continue  # its LDS accumulators do not fit
        shape = tuple(ctx.get_info()["tile"])   # (0, 0) resolves to the library's choice
        ctx.step(warmup)
        ctx.sync()
        used += warmup
        best = timings.get(shape, float("inf"))
        for _ in range(repeats):
            ctx.profile_enable(True)
            ctx.step(cycles)
            ctx.sync()
            prof = ctx.profile_read()
            ctx.profile_enable(False)
            used += cycles
            best = min(best, prof["step_ms"] / max(prof["steps"], 1))
        timings[shape] = best
    if not timings:
        raise RuntimeError("no candidate tile shape fits")
    best = min(timings, key=timings.get)
    ctx.set_tiles(*best)
    return {"best": best, "ms_per_cycle": timings, "cycles_used": used}


# Shapes tried for a whole batch; (0, 0) is the library's own choice per run.
BATCH_CANDIDATES = [(0, 0), (32, 4), (16, 4), (32, 2), (16, 8), (8, 4), (64, 2), (64, 4)]


def tune_batch(batch, ctxs, candidates=BATCH_CANDIDATES, cycles=4, warmup=1, repeats=2):
    """Time whole batch cycles for every candidate shape, applied to every member at once
    ((0, 0): each run's own default), and leave the fastest applied.  A small run stepped
    alone cannot fill the GPU and prefers small tiles (more blocks); in a full batch the
    per-tile work decides, so the batch is timed as a whole (best of `repeats` timings per
    shape).  A member whose LDS does not take a shape keeps its previous one.  The timed cycles
    advance every member.  Returns
    {"best": (tx, tz), "ms_per_cycle": {(tx, tz): ms}, "cycles_used": n}."""
    import time
    timings = {}
    used = 0
    for tile in candidates:
        for c in ctxs:
            try:
                c.set_tiles(*tile)
            except binding.PicError:
                pass
        batch.step(warmup)
        batch.sync()
        used += warmup
        best = float("inf")
        for _ in range(repeats):
            t0 = time.perf_counter()
            batch.step(cycles)
            batch.sync()
            best = min(best, (time.perf_counter() - t0) / cycles * 1e3)
            used += cycles
        timings[tuple(tile)] = best
    best = min(timings, key=timings.get)
    for c in ctxs:
        try:
            c.set_tiles(*best)
        except binding.PicError:
            pass
    return {"best": best, "ms_per_cycle": timings, "cycles_used": used}
