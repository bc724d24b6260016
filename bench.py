#!/usr/bin/env python3
"""Benchmark of the implicit 2D3V PIC particle stage on one MI355X.

A step is one full cycle of the hot path on the resident workload: field solve, fused
gather-push-deposit, and the stable cell sort.  The workload defaults to the largest
single-GPU configuration, the field-dominated run (2048 x 2048 cells, absorbing x, periodic
z, uniform 0.1 n_c, 4 particles per cell and species: 33.6M particles, FP64).  Inputs are
generated in host memory, loaded once, and are resident in HBM before the timed region starts.

Prints one JSON line with the throughput (alive particles x steps / s over whole cycles),
the roofline position of the dominant kernel (the fused particle kernel) measured with HIP
events on the stream the kernels run on, and the CPU oracle timed on a bounded sample (one
thread, and independent copies on all cores the job may use).  The line also carries the
particle-dominated foil (1024 x 512 cells, 40-cell slab at 100 n_c, 64 particles per cell and
species) with its own roofline, and the FP64 / mixed-precision comparison on the foil, the
dense foil (200 n_c, 128 particles per cell and species) and the count-matched dense foil
(160-cell slab, 21.0M particles).
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

KERNEL_SOURCE = os.path.join(ROOT, "paper_1308_2590_amd", "csrc", "pic_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def parse_tile(text):
    if "x" in str(text):
        tx, tz = str(text).split("x")
        return int(tx), int(tz)
    return int(text), int(text)


def measured_traffic(workload, precision, tile):
    """HBM bytes per launch of the particle kernel from the committed counter summary of this
    workload, precision and tile shape, if it was taken on the current kernel source (else
    None)."""
    import hashlib
    path = os.path.join(PROFILES, f"k_particles_{workload}_{precision}_{tile[0]}x{tile[1]}_traffic.md")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the fused particle kernel: each particle's state is read and written
# once (FP64: 2 positions + 3 momenta = 40 B, twice; mixed: int32 cell + 2 FP32 offsets +
# 3 FP32 momenta = 24 B, twice), and per node E-bar, H^{n+1/2}, H^{n+3/2} (3 x 24 B) are read
# and 12 + S FP64 moment planes (8 B each) written once.
BYTES_PER_PARTICLE = {"fp64": 80, "mixed": 48}


# the sort's ranker (pic_set_rank_mode): automatic unless --rank says otherwise
RANK_MODE = 0
RANK_NAMES = {0: "auto", 1: "rows", 2: "cells"}


def bytes_per_node(S):
    return 72 + 8 * (12 + S)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="lowdensity",
                    help="lowdensity | foil | foil_cm | foil_dense | foil_dense_cm | uniform64a | uniform64b")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget for the CPU oracle baseline (0 disables it)")
    ap.add_argument("--tile", default="0",
                    help="tile shape 'TXxTZ' or square side 'N'; 0 = the library's automatic choice")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: time candidate tile shapes during warmup and keep the fastest")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--rank", choices=["auto", "rows", "cells"], default="auto",
                    help="ranker of the cell sort: automatic, tile rows, or one thread per cell")
    ap.add_argument("--compare-steps", type=int, default=20,
                    help="timed cycles of each FP64 / mixed comparison run (0 skips them)")
    ap.add_argument("--drift-steps", type=int, default=500,
                    help="cycles of the FP64 / mixed drift comparison on the dense foil (0 skips it)")
    ap.add_argument("--foil-steps", type=int, default=50,
                    help="timed cycles of the particle-dominated foil section (0 skips it)")
    ap.add_argument("--cpu-cores", type=int, default=16,
                    help="most host cores the all-cores oracle baseline may use")
    ap.add_argument("--cpu-worker", default="",
                    help=argparse.SUPPRESS)
    ap.add_argument("--mover-steps", type=int, default=1000,
                    help="cycles of the warm-plasma energy comparison of the mover options "
                         "(0 skips the mover-option section)")
    ap.add_argument("--batch-runs", type=int, default=32,
                    help="runs of the batched FP64 / mixed comparison (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=50,
                    help="timed cycles of the batched FP64 / mixed comparison")
    ap.add_argument("--serve-runs", type=int, default=256,
                    help="requests of the batched serving stream (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="request arrivals per second")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the workload, run one elementwise kernel that reads and writes "
                         "this many MiB (the reference dispatch for scaling HBM byte counters)")
    return ap.parse_args()


def cpu_sample(name):
    """The bounded sample of a workload that the oracle runs: the field-dominated run as a
    2048 x 64 strip (its full row length, cells, particles per cell, temperatures and laser,
    1,048,576 particles), every other workload as it is."""
    if name == "lowdensity":
        return picgen.low_density(nz=64), "a 2048 x 64 strip of the 2048 x 2048 run (1,048,576 particles)"
    wl = picgen.named(name)
    return wl, f"the whole workload ({wl.n_particles} particles)"


def cpu_run(name, budget_s):
    """The oracle as it is (single-threaded C) on the sample of a workload: whole cycles until
    the budget is used (at least one).  Returns (particle-steps, seconds, cycles)."""
    from oracle import OracleSim
    wl, _ = cpu_sample(name)
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
        if el >= budget_s or steps >= 200:
            break
    return ps, el, steps


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, budget_s, max_cores):
    """The oracle timed on the host cores of this job: one thread in this process, then
    independent copies of the same sample in child processes, one per core (at most
    max_cores, and no more than the cores this process may run on), at the same time.  The
    value is the all-cores aggregate; the one-thread figure is beside it."""
    import subprocess
    _, what = cpu_sample(name)
    ps, el, steps = cpu_run(name, budget_s)
    one = ps / el
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    ncores = max(1, min(max_cores, avail))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", name,
           "--cpu-seconds", str(budget_s)]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    t0 = time.perf_counter()
    procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=env, text=True)
             for _ in range(ncores)]
    rates = []
    for p in procs:
        out, _ = p.communicate()
        if p.returncode == 0 and out.strip():
            r = json.loads(out.strip().splitlines()[-1])
            rates.append(r["particle_steps"] / r["seconds"])
    wall = time.perf_counter() - t0
    return {"value": sum(rates) if rates else one, "unit": "particle-steps/s",
            "cores": len(rates) if rates else 1, "kind": "oracle",
            "sample": f"{what} of the {name} workload: the plain FP64 oracle, one thread per "
                      f"process, whole cycles for about {budget_s:.0f} s; {len(rates)} copies ran "
                      f"at once ({wall:.1f} s wall) for the all-cores value",
            "single_thread_value": one, "single_thread_cycles": steps,
            "single_thread_seconds": el, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "cores_available": avail}


PROFILE_EVERY = 4


def run_gpu(binding, torch, wl, precision, steps, warmup, tile, autotune=False):
    """Load the workload, run warmup cycles (and the tile autotuner, whose cycles come before
    the timed ones), then time `steps` cycles (wall clock around the whole batch, HIP events
    per kernel group).  Returns the measurements."""
    S = wl.grid.n_species
    prec = picgen.PREC_MIXED if precision == "mixed" else picgen.PREC_FP64
    ctx = binding.Context(wl.grid, track_ids=False, tile=tile, precision=prec)
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    ctx.set_rank_mode(RANK_MODE)
    tuned = None
    if autotune:
        from paper_1308_2590_amd import autotune as at
        tuned = at.tune_tiles(ctx)
    ctx.step(warmup)
    ctx.sync()
    torch.cuda.synchronize()
    info0 = ctx.get_info()
    n_alive0 = sum(info0["alive"])

    # kernel times from HIP events on every PROFILE_EVERY-th timed cycle (the events leave the
    # GPU idle between kernels, so the other cycles run without them)
    ctx.profile_enable(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    info1 = ctx.get_info()
    # nodes the deposit reached (any moment plane nonzero): the node part of the kernel's work
    M = ctx.read_moments()
    touched = int(np.count_nonzero(np.any(M != 0.0, axis=0)))
    del M
    ctx.close()
    if info1["overflow_flags"]:
        print(f"overflow flags raised: {info1['overflow_flags']}", file=sys.stderr)
        sys.exit(3)
    n_alive1 = sum(info1["alive"])
    # particles processed per cycle: the alive count entering each cycle (bounded by these)
    n_mean = 0.5 * (n_alive0 + n_alive1)
    part_ms = prof["particle_ms"] / max(prof["particle_launches"], 1)
    alg_bytes = BYTES_PER_PARTICLE[precision] * n_mean + bytes_per_node(S) * wl.grid.n_nodes
    alg_bytes_touched = BYTES_PER_PARTICLE[precision] * n_mean + bytes_per_node(S) * touched
    achieved = alg_bytes / (part_ms * 1e-3) / 1e9
    return {
        "autotune": None if tuned is None else {
            "best": list(tuned["best"]),
            "ms_per_cycle": {f"{k[0]}x{k[1]}": v for k, v in tuned["ms_per_cycle"].items()},
            "cycles_used": tuned["cycles_used"]},
        "value": n_mean * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "particles": int(n_alive0),
        "tile": list(info1["tile"]),
        "rank": RANK_NAMES[info1["rank_mode"]],
        "part_ms": part_ms,
        "alg_bytes": alg_bytes,
        "alg_bytes_touched": alg_bytes_touched,
        "nodes_touched": touched,
        "achieved": achieved,
        "achieved_touched": alg_bytes_touched / (part_ms * 1e-3) / 1e9,
        "breakdown": {
            "field_solve": prof["field_ms"] / max(prof["field_launches"], 1),
            "particles": part_ms,
            "sort": prof["sort_ms"] / max(prof["sort_launches"], 1),
            "events_step": prof["step_ms"] / max(prof["steps"], 1),
        },
    }


def precision_pair(wl, mf, mm):
    """The FP64 and mixed measurements of one workload side by side."""
    r = {}
    for prec, m in (("fp64", mf), ("mixed", mm)):
        r[prec] = {"particle_steps_per_s": m["value"], "ms_per_step": m["ms_per_step"],
                   "particle_kernel_ms": m["part_ms"], "particle_kernel_GBps": m["achieved"],
                   "particle_kernel_frac_hbm": m["achieved"] / HBM_PEAK_GBS,
                   "particle_kernel_frac_hbm_touched_nodes": m["achieved_touched"] / HBM_PEAK_GBS,
                   "tile": m["tile"]}
    r["speedup_mixed_over_fp64"] = r["mixed"]["particle_steps_per_s"] / r["fp64"]["particle_steps_per_s"]
    r["particle_kernel_speedup"] = r["fp64"]["particle_kernel_ms"] / r["mixed"]["particle_kernel_ms"]
    r["workload"] = wl.name
    r["particles"] = wl.n_particles
    return r


def comparison(binding, torch, wl, steps, warmup, tile, autotune):
    mf = run_gpu(binding, torch, wl, "fp64", steps, warmup, tile, autotune)
    mm = run_gpu(binding, torch, wl, "mixed", steps, warmup, tile, autotune)
    return precision_pair(wl, mf, mm)


def drift(binding, steps, name="foil_dense"):
    """After `steps` cycles from the same loaded state: each moment plane and field of the mixed
    run against the FP64 run (relative L2 and max-norm errors), beside two controls:
    - two FP64 runs that differ only in tile shape (the run-to-run spread from the order of
      floating-point atomic additions, amplified by the particle dynamics over many cycles);
    - an FP64 run started from the inputs rounded to the mixed form (the amplification of the
      rounding at load alone).  The mixed run is also compared with this one."""
    import numpy as np
    wl = picgen.named(name)
    wl32 = picgen.fp32_representable(wl)
    runs = {}
    for key, prec, tile, w in (("fp64", 0, (32, 1), wl), ("fp64_other_tiles", 0, (16, 4), wl),
                               ("fp64_rounded_inputs", 0, (32, 1), wl32), ("mixed", 1, (4, 4), wl)):
        ctx = binding.Context(w.grid, precision=prec, tile=tile)
        for s, sp in enumerate(w.species):
            ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
        ctx.step(steps)
        M = ctx.read_moments()
        E, H = ctx.read_fields()
        runs[key] = (M, E, H)
        ctx.close()
    names = ["S_xx", "S_xy", "S_xz", "S_yx", "S_yy", "S_yz", "S_zx", "S_zy", "S_zz",
             "dj_x", "dj_y", "dj_z"] + [f"n_{s}" for s in range(wl.grid.n_species)]

    def errs(a, b):
        out = {}
        for p, nm in enumerate(names):
            d = a[0][p] - b[0][p]
            out[nm] = {"l2": float(np.linalg.norm(d) / max(np.linalg.norm(b[0][p]), 1e-300)),
                       "max": float(np.max(np.abs(d)) / max(np.max(np.abs(b[0][p])), 1e-300))}
        for f, (ia, nm) in enumerate(((1, "E"), (2, "H"))):
            for r in range(3):
                d = a[ia][r] - b[ia][r]
                out[f"{nm}{'xyz'[r]}"] = {
                    "l2": float(np.linalg.norm(d) / max(np.linalg.norm(b[ia][r]), 1e-300)),
                    "max": float(np.max(np.abs(d)) / max(np.max(np.abs(b[ia][r])), 1e-300))}
        return out

    return {"workload": wl.name, "cycles": steps,
            "mixed_vs_fp64": errs(runs["mixed"], runs["fp64"]),
            "fp64_vs_fp64_other_tiles": errs(runs["fp64_other_tiles"], runs["fp64"]),
            "fp64_rounded_inputs_vs_fp64": errs(runs["fp64_rounded_inputs"], runs["fp64"]),
            "mixed_vs_fp64_rounded_inputs": errs(runs["mixed"], runs["fp64_rounded_inputs"])}


def roofline(m, workload, precision):
    """The roofline object of the particle kernel from a run_gpu measurement: algorithmic bytes
    with every grid node (the moments are defined on the whole grid), and with the nodes the
    deposit reached (the kernel touches only the tiles holding particles)."""
    return {
        "bound": "hbm",
        "kernel": "k_particles (fused gather-push-deposit)",
        "achieved": m["achieved"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": m["achieved"] / HBM_PEAK_GBS,
        "traffic": measured_traffic(workload, precision, m["tile"]),
        "alg_bytes_per_launch": m["alg_bytes"],
        "avg_launch_ms": m["part_ms"],
        "alg_bytes_per_launch_touched_nodes": m["alg_bytes_touched"],
        "nodes_touched": m["nodes_touched"],
        "achieved_touched_nodes": m["achieved_touched"],
        "frac_touched_nodes": m["achieved_touched"] / HBM_PEAK_GBS,
    }


def particle_dominated(binding, torch, steps, warmup, auto):
    """The particle-dominated foil (1024 x 512 cells, 40-cell slab at 100 n_c, 64 particles per
    cell and species: 2.62M particles) in FP64: throughput, cycle breakdown and the particle
    kernel's roofline."""
    wl = picgen.named("foil")
    m = run_gpu(binding, torch, wl, "fp64", steps, warmup, (0, 0), autotune=auto)
    return {"workload": wl.name, "particles": m["particles"], "steps": steps,
            "particle_steps_per_s": m["value"], "ms_per_step": m["ms_per_step"], "tile": m["tile"],
            "breakdown_ms_per_step": m["breakdown"], "roofline": roofline(m, "foil", "fp64"),
            "autotune": m["autotune"]}


def warm_plasma(temperature_kev, nx=128, nz=128, ppc=16):
    """Periodic two-species plasma with thermal electrons at temperature_kev (cold ions, m_i/m_e
    = 1836), density 1, dx = dz = 1.25, dt = 0.5 (omega_p dt = 0.5), uniform B_z = 0.5, E = 0."""
    import numpy as np
    ci, ck = np.meshgrid(np.arange(nx), np.arange(nz))
    el = picgen.make_species(np.random.default_rng(71), ci.ravel(), ck.ravel(), ppc, q=-1.0,
                             m=1.0, density=1.0, temperature_kev=temperature_kev, quiet=False)
    io = picgen.make_species(np.random.default_rng(72), ci.ravel(), ck.ravel(), ppc, q=1.0,
                             m=picgen.ION_MASS, density=1.0, temperature_kev=0.0, quiet=False)
    g = picgen.Grid(nx=nx, nz=nz, dx=1.25, dz=1.25, dt=0.5, h0=(0.0, 0.0, 0.5))
    return picgen.Workload(name=f"warm{nx}x{nz}_Te{temperature_kev:g}keV_ppc{ppc}", grid=g,
                           species=[el, io], steps=0, note="periodic warm plasma")


def mover_options(binding, torch, steps):
    """The mover options (the Lorentz-factor predictor gamma(u^n + beta E^n), bilinear B, both)
    against the default mover: relative change of the total energy of periodic warm plasmas over
    `steps` cycles (the diagnostic for choosing between the readings; a periodic plasma without
    sources should keep its energy), and the cycle time on the foil (the per-particle kernel of
    the options against the tile kernel)."""
    names = {0: "default", 1: "gamma_predict", 2: "b_bilinear", 3: "both"}
    res = {"energy": [], "foil_ms_per_cycle": {}}
    for te in (1.0, 50.0):
        wl = warm_plasma(te)
        row = {"workload": wl.name, "cycles": steps, "particles": wl.n_particles}
        for opt, nm in names.items():
            ctx = binding.Context(wl.grid)
            for s, sp in enumerate(wl.species):
                ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
            ctx.set_mover(opt)
            E0 = ctx.energy()
            W0, K0 = sum(E0), sum(E0[1:])
            worst = 0.0
            done = 0
            while done < steps:
                k = min(100, steps - done)
                ctx.step(k)
                done += k
                worst = max(worst, abs(sum(ctx.energy()) - W0) / K0)
            W1 = ctx.energy()
            # the uniform B_z holds most of the field energy: changes are given relative to the
            # initial kinetic energy as well as to the total
            row[nm] = {"energy_start": E0, "energy_end": W1,
                       "total_change_over_total": (sum(W1) - W0) / W0,
                       "total_change_over_kinetic0": (sum(W1) - W0) / K0,
                       "max_abs_change_over_kinetic0": worst,
                       "kinetic_end_over_kinetic0": sum(W1[1:]) / K0}
            ctx.close()
        res["energy"].append(row)
    wl = picgen.named("foil")
    for opt, nm in names.items():
        ctx = binding.Context(wl.grid, tile=(32, 2))
        for s, sp in enumerate(wl.species):
            ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
        ctx.set_mover(opt)
        ctx.step(2)
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(10)
        ctx.sync()
        res["foil_ms_per_cycle"][nm] = 1e3 * (time.perf_counter() - t0) / 10
        ctx.close()
    return res


def batched(binding, torch, nruns, steps, warmup, autotune=False):
    """The batched form in both precisions: `nruns` independent foil runs of uneven size (drawn
    like the serving stream: sides log-uniform in [32, 512], slab 5-15 % of x, density 10-200
    n_c, 8-64 particles per cell) stepped together by the persistent batch kernels with graph
    replay, first all in FP64, then all in mixed precision: aggregate particle-steps/s of each
    (particles alive, averaged over the timed cycles) and the speedup of the mixed batch.  With
    autotune, the tile shape is tuned on the whole batch (every member takes the candidate
    shape at once, whole batch cycles are timed)."""
    from paper_1308_2590_amd import autotune as at
    reqs = picgen.serving_stream(nruns, seed=11)
    res = {"runs": nruns, "cycles": steps, "graph": True, "tiles": "tuned on the batch" if autotune
           else "library default per run"}
    for name, prec in (("fp64", picgen.PREC_FP64), ("mixed", picgen.PREC_MIXED)):
        b = binding.Batch(0, prec)
        ctxs = []
        for r in reqs:
            wl = picgen.request_workload(r, precision=prec)
            ctx = binding.Context(wl.grid, precision=prec)
            for s, sp in enumerate(wl.species):
                ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
            b.add(ctx)
            ctxs.append(ctx)
        b.set_graph(True)
        if autotune:
            tuned = at.tune_batch(b, ctxs)
            res.setdefault("tuning", {})[name] = {
                "best": list(tuned["best"]),
                "ms_per_cycle": {f"{k[0]}x{k[1]}": v for k, v in tuned["ms_per_cycle"].items()}}
        b.step(warmup)
        b.sync()
        alive = lambda: sum(sum(c.get_info()["alive"]) for c in ctxs)
        n0 = alive()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        b.sync()
        dt = time.perf_counter() - t0
        n1 = alive()
        shapes = {}
        for c in ctxs:
            key = "x".join(str(v) for v in c.get_info()["tile"])
            shapes[key] = shapes.get(key, 0) + 1
        res[name] = {"particles": n0, "ms_per_step": dt / steps * 1e3,
                     "particle_steps_per_s": 0.5 * (n0 + n1) * steps / dt, "tile_shapes": shapes}
        b.close()
        for c in ctxs:
            c.close()
    res["speedup_mixed_over_fp64"] = (res["mixed"]["particle_steps_per_s"]
                                      / res["fp64"]["particle_steps_per_s"])
    return res


def serving(args):
    """The batched serving stream: independent foil runs arriving Poisson at serve_rate per
    second (grid sides log-uniform in [32, 512], slab 5-15 % of x, density 10-200 n_c,
    8-64 particles per cell, a0 in [0.5, 10], 100-1000 cycles each), mixed precision, admitted
    into one batch by slots and device-memory footprint and stepped together."""
    from paper_1308_2590_amd import serve
    reqs = picgen.serving_stream(args.serve_runs, rate_per_s=args.serve_rate)
    srv = serve.Server(picgen.request_workload, precision=picgen.PREC_MIXED, max_slots=256,
                       budget_bytes=64 << 30, graph=True)
    done = [0]

    def progress(req, ctx):
        done[0] += 1
        if done[0] % 32 == 0:
            print(f"[bench] serving: {done[0]} of {len(reqs)} runs done", file=sys.stderr, flush=True)

    try:
        st = srv.run(reqs, realtime=True, on_finish=progress)
    finally:
        srv.close()
    out = st.summary()
    out.update({"arrival_rate_per_s": args.serve_rate, "precision": "mixed", "graph": True,
                "offered_particle_steps": float(sum(
                    2 * r.slab_cells * r.nz * r.ppc * r.steps for r in reqs))})
    return out


def main():
    args = parse()
    global RANK_MODE
    RANK_MODE = {"auto": 0, "rows": 1, "cells": 2}[args.rank]
    if args.cpu_worker:
        # child of cpu_baseline: one copy of the oracle on its sample, no GPU
        ps, el, steps = cpu_run(args.cpu_worker, args.cpu_seconds)
        print(json.dumps({"particle_steps": ps, "seconds": el, "cycles": steps}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has "
              "no multi-GPU path (the strip decomposition across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1308_2590_amd import binding

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    wl = picgen.named(args.workload)
    S = wl.grid.n_species
    tile = parse_tile(args.tile)
    auto = bool(args.autotune) and tile == (0, 0)
    m = run_gpu(binding, torch, wl, args.precision, args.steps, args.warmup, tile, autotune=auto)
    print(f"[bench] {wl.name} {args.precision}: {m['value']:.4g} particle-steps/s, "
          f"{m['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
    out = {
        "metric": "implicit particle push+deposit/s (FP64 vs mixed); batched p50/p99 step ms",
        "value": m["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": wl.name,
            "grid": [wl.grid.nx, wl.grid.nz],
            "particles": m["particles"],
            "species": S,
            "precision": args.precision,
            "tile": m["tile"],
            "rank": m["rank"],
            "note": wl.note,
        },
        "roofline": roofline(m, args.workload, args.precision),
        "breakdown_ms_per_step": m["breakdown"],
        "autotune": m["autotune"],
    }
    if args.foil_steps > 0 and args.workload != "foil":
        out["particle_dominated"] = particle_dominated(binding, torch, args.foil_steps,
                                                       args.warmup, bool(args.autotune))
        print("[bench] particle-dominated foil done", file=sys.stderr, flush=True)
    if args.compare_steps > 0:
        pairs = []
        if args.precision == "fp64":
            # the headline workload in the mixed form, beside the FP64 run measured above
            mm = run_gpu(binding, torch, wl, "mixed", args.steps, args.warmup, tile, autotune=auto)
            pairs.append(precision_pair(wl, m, mm))
        pairs += [comparison(binding, torch, picgen.named(name), args.compare_steps, args.warmup,
                             (0, 0), bool(args.autotune))
                  for name in ("foil", "foil_dense", "foil_dense_cm")]
        out["fp64_vs_mixed"] = pairs
        print("[bench] comparison done", file=sys.stderr, flush=True)
    if args.drift_steps > 0:
        out["precision_drift"] = drift(binding, args.drift_steps)
        print("[bench] drift done", file=sys.stderr, flush=True)
    if args.mover_steps > 0:
        out["mover_options"] = mover_options(binding, torch, args.mover_steps)
        print("[bench] mover options done", file=sys.stderr, flush=True)
    if args.batch_runs > 0:
        out["batched_fp64_vs_mixed"] = batched(binding, torch, args.batch_runs, args.batch_steps,
                                               args.warmup, bool(args.autotune))
        print("[bench] batched comparison done", file=sys.stderr, flush=True)
    if args.serve_runs > 0:
        out["serving"] = serving(args)
        print("[bench] serving done", file=sys.stderr, flush=True)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds, args.cpu_cores)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
