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

CANDIDATES = [(4, 4), (8, 4), (16, 4), (32, 4), (8, 2), (16, 2), (32, 2), (16, 1), (32, 1),
              (8, 8), (16, 8)]


def tune_tiles(ctx, candidates=CANDIDATES, cycles=4, warmup=1):
    """Time `cycles` cycles (after `warmup` untimed ones) for every candidate tile shape that
    fits in LDS; apply and return the fastest.  Returns {"best": (tx, tz), "ms_per_cycle":
    {(tx, tz): ms}, "cycles_used": n}."""
    timings = {}
    used = 0
    for tile in candidates:
        try:
            ctx.set_tiles(*tile)
        except binding.PicError:
            continue  # its LDS accumulators do not fit
        ctx.step(warmup)
        ctx.sync()
        ctx.profile_enable(True)
        ctx.step(cycles)
        ctx.sync()
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        used += warmup + cycles
        timings[tuple(tile)] = prof["step_ms"] / max(prof["steps"], 1)
    if not timings:
        raise RuntimeError("no candidate tile shape fits")
    best = min(timings, key=timings.get)
    ctx.set_tiles(*best)
    return {"best": best, "ms_per_cycle": timings, "cycles_used": used}
