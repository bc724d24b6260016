#!/usr/bin/env python3
"""Benchmark of the implicit 2D3V PIC particle stage on one MI355X.

A step is one full cycle of the hot path on the resident workload: field solve, fused
gather-push-deposit, and the stable cell sort.  The workload defaults to the
particle-dominated foil (1024 x 512 cells, absorbing x, periodic z, 40-cell slab at 100 n_c,
64 particles per cell and species, about 2.6M particles, FP64).  Inputs are generated
in host memory, loaded once, and are resident in HBM before the timed region starts.

Prints one JSON line with the throughput (alive particles x steps / s over whole cycles),
the roofline position of the dominant kernel (the fused particle kernel) measured with HIP
events on the stream the kernels run on, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import picgen  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the fused particle kernel: each particle's state is read and written
# once (FP64: 2 positions + 3 momenta = 40 B, twice), and per node E-bar, H^{n+1/2},
# H^{n+3/2} (3 x 24 B) are read and 12 + S moment planes (8 B each) written once.
BYTES_PER_PARTICLE = {"f64": 80}


def bytes_per_node(S):
    return 72 + 8 * (12 + S)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="foil",
                    help="foil | foil_cm | lowdensity | uniform64a | uniform64b")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget for the CPU oracle baseline (0 disables it)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB before the timed region "
                         "(reference dispatch for scaling HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(wl, budget_s):
    """The oracle as it is (single-threaded C), on the same workload, for whole cycles until
    the budget is used (at least one cycle)."""
    from oracle import OracleSim
    o = OracleSim(wl.grid)
    for s, sp in enumerate(wl.species):
        o.load_species(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    steps = 0
    ps = 0
    t0 = time.perf_counter()
    while True:
        n = sum(sp.n for sp in o.species if sp is not None)
        o.step(1)
        steps += 1
        ps += n
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 50:
            break
    return {"value": ps / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} full cycles of the same workload ({wl.name}) on one host core, "
                      f"{el:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "strip decomposition is not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1308_2590_amd import binding

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    wl = picgen.named(args.workload)
    S = wl.grid.n_species
    ctx = binding.Context(wl.grid, track_ids=False, tile=(args.tile, args.tile))
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    ctx.step(args.warmup)
    ctx.sync()
    torch.cuda.synchronize()
    info0 = ctx.get_info()
    n_alive0 = sum(info0["alive"])

    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    info1 = ctx.get_info()
    n_alive1 = sum(info1["alive"])
    if info1["overflow_flags"]:
        print(f"overflow flags raised: {info1['overflow_flags']}", file=sys.stderr)
        sys.exit(3)

    # particles processed per cycle: the alive count entering each cycle (bounded by these)
    n_mean = 0.5 * (n_alive0 + n_alive1)
    value = n_mean * args.steps / wall
    part_ms = prof["particle_ms"] / max(prof["particle_launches"], 1)
    alg_bytes = BYTES_PER_PARTICLE["f64"] * n_mean + bytes_per_node(S) * wl.grid.n_nodes
    achieved = alg_bytes / (part_ms * 1e-3) / 1e9
    out = {
        "metric": "implicit particle push+deposit/s (FP64 vs mixed); batched p50/p99 step ms",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": wl.name,
            "grid": [wl.grid.nx, wl.grid.nz],
            "particles": int(n_alive0),
            "species": S,
            "precision": "fp64",
            "tile": list(info1["tile"]),
            "note": wl.note,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_particles<true> (fused gather-push-deposit)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_ms": part_ms,
        },
        "breakdown_ms_per_step": {
            "field_solve": prof["field_ms"] / max(prof["field_launches"], 1),
            "particles": part_ms,
            "sort": prof["sort_ms"] / max(prof["sort_launches"], 1),
            "events_step": prof["step_ms"] / max(prof["steps"], 1),
        },
    }
    ctx.close()
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
