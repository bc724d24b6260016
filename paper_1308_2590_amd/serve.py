"""Continuous batching of independent runs on one GPU.

Requests (independent simulations) arrive over time.  A request is admitted as soon as it has
arrived, a slot is free and its device-memory footprint fits in the budget.  Admitted requests
are loaded (context created, particles placed and sorted, moments deposited) by a loader
thread, off the cycle path, and join the batch at the next cycle once loaded.  All members
are stepped together, with one launch of each kernel per cycle.  Particles and fields stay
resident on the device from admission to completion.  A run leaves the batch after the cycles
it asked for, which frees its slot and memory for waiting requests.

Two latencies are recorded per cycle: the GPU time of the batch step (launch to completion),
and the cycle time a resident run sees, from the end of the previous cycle to the end of this
one, which also holds whatever the cycle thread did in between (joining loaded runs, which
rebuilds the batch tables and recaptures its graph, and retiring finished runs).

The arithmetic all happens in the library's kernels.  This module only schedules: it decides
admission, creates and loads contexts, steps the batch and retires finished runs.
"""
from __future__ import annotations

import collections
import concurrent.futures
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding


def footprint_bytes(nx, nz, bc_x, n_species, n_particles, precision, *, per_particle_w=False,
                    track_ids=False):
    """Upper bound of the device bytes a run's context holds once its particles are loaded:
    two time levels of E and H, the moment planes, per species the two state copies (with
    per-particle densities and labels when used), two permutations, two cell-start arrays,
    move codes, nine move counts and the arrivals per cell, plus the tile flags and lists for
    tiles of at least one cell.  Checked against the library's own count in the tests."""
    nxn = nx + (1 if bc_x == 1 else 0)
    nodes, cells = nxn * nz, nx * nz
    grid = 8 * nodes * (3 * 2 + 12 + n_species) + 8 * cells * 3 * 2 + 4 + 12 * 8
    state = 24 if precision == 1 else 40
    if per_particle_w:
        state += 4 if precision == 1 else 8
    if track_ids:
        state += 8
    # both state copies, two permutations (8 entries of padding each), the move codes
    per_particle = 2 * state + 2 * 4 + 4
    per_species = 2 * 4 * (cells + 1) + 4 * 9 * cells + 4 * cells + 4 * (cells // 1024 + 1) + 2 * 4 * 8
    tiles = 2 * (cells + 4 * (cells + 1)) + cells + 64
    per_alloc = 256   # allocation granularity, per block
    n_allocs = 16 + n_species * 20
    return int(grid + n_species * per_species + n_particles * per_particle + tiles
               + per_alloc * n_allocs)


@dataclass
class ServeStats:
    """Counters of one serving run.  particle_steps counts, for every cycle, the particles each
    active run was loaded with; step_s holds the GPU time of every batch step and cycle_s the
    cycle time the resident runs saw (host work between steps included)."""
    runs: int = 0
    cycles: int = 0
    particle_steps: float = 0.0
    wall_s: float = 0.0
    step_s: list = field(default_factory=list)
    cycle_s: list = field(default_factory=list)
    max_concurrent: int = 0
    admit_wait_s: list = field(default_factory=list)
    join_wait_s: list = field(default_factory=list)
    max_device_bytes: int = 0
    footprint_checks: list = field(default_factory=list)

    def summary(self):
        def pct(v, q, scale=1.0):
            return float(np.percentile(np.array(v) * scale, q)) if v else 0.0
        return {
            "runs": self.runs,
            "cycles": self.cycles,
            "particle_steps_per_s": self.particle_steps / self.wall_s if self.wall_s > 0 else 0.0,
            "gpu_particle_steps_per_s": self.particle_steps / max(float(np.sum(self.step_s)), 1e-12),
            "step_ms_p50": pct(self.step_s, 50, 1e3),
            "step_ms_p99": pct(self.step_s, 99, 1e3),
            "step_ms_mean": float(np.mean(self.step_s) * 1e3) if self.step_s else 0.0,
            "cycle_ms_p50": pct(self.cycle_s, 50, 1e3),
            "cycle_ms_p99": pct(self.cycle_s, 99, 1e3),
            "cycle_ms_max": float(np.max(self.cycle_s) * 1e3) if self.cycle_s else 0.0,
            "wall_s": self.wall_s,
            "max_concurrent": self.max_concurrent,
            "admission_wait_s_p50": pct(self.admit_wait_s, 50),
            "admission_wait_s_p99": pct(self.admit_wait_s, 99),
            "join_wait_s_p50": pct(self.join_wait_s, 50),
            "join_wait_s_p99": pct(self.join_wait_s, 99),
            # read only when the server checks the budget
            "max_device_bytes": self.max_device_bytes if self.footprint_checks else None,
        }


class Server:
    """Admit runs into one batch as slots and memory allow, step them together, retire them.

    make_workload(request) returns the run's workload (grid, species); the request needs the
    attributes rid, arrival_s and steps.  With realtime=True arrivals follow the wall clock
    (the server sleeps when it has nothing to run).  With realtime=False each cycle advances a
    virtual clock by cycle_s and loaded runs join in admission order, which makes admission
    deterministic (used by the tests).  check_budget=True reads the device bytes every member
    holds after each join and raises if their sum exceeds the budget (it waits for the batch,
    so it is for tests).
    """

    def __init__(self, make_workload, *, precision=1, max_slots=64, budget_bytes=64 << 30,
                 graph=True, device=0, tile=(0, 0), track_ids=False, check_budget=False):
        self.make_workload = make_workload
        self.precision = precision
        self.max_slots = max_slots
        self.budget = budget_bytes
        self.device = device
        self.tile = tile
        self.track_ids = track_ids
        self.check_budget = check_budget
        self.batch = binding.Batch(device, precision)
        self.batch.set_graph(graph)
        self._loader = concurrent.futures.ThreadPoolExecutor(max_workers=1)
        self._cache = {}

    def _workload(self, req):
        wl = self._cache.pop(req.rid, None)
        return wl if wl is not None else self.make_workload(req)

    def _need(self, req):
        wl = self._cache.get(req.rid)
        if wl is None:
            wl = self._cache[req.rid] = self.make_workload(req)
        g = wl.grid
        pw = any(np.ndim(sp.w) > 0 for sp in wl.species)
        return footprint_bytes(g.nx, g.nz, g.bc_x, g.n_species, wl.n_particles, self.precision,
                               per_particle_w=pw, track_ids=self.track_ids)

    def _load(self, req, wl):
        """Loader thread: create the run's context and load its particles (on the context's own
        stream; the batch is not touched here)."""
        ctx = binding.Context(wl.grid, precision=self.precision, device=self.device,
                              tile=self.tile, track_ids=self.track_ids)
        try:
            for s, sp in enumerate(wl.species):
                ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
            ctx.sync()
        except Exception:
            ctx.close()
            raise
        return ctx

    def run(self, requests, *, realtime=True, cycle_s=1e-3, on_finish=None):
        loading = collections.deque()   # admitted, being loaded: (run record, future)
        active = []
        try:
            return self._run(requests, realtime, cycle_s, on_finish, loading, active)
        except BaseException:
            # leave nothing behind: wait for the loads under way and release every context
            for _, fut in loading:
                try:
                    fut.result().close()
                except Exception:
                    pass
            for r in active:
                try:
                    self.batch.remove(r["ctx"])
                except Exception:
                    pass
                r["ctx"].close()
            raise

    def _run(self, requests, realtime, cycle_s, on_finish, loading, active):
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        used = 0
        st = ServeStats()
        vclock = 0.0
        t0 = time.perf_counter()
        last_end = None

        def now():
            return time.perf_counter() - t0 if realtime else vclock

        while pending or loading or active:
            t = now()
            # admission: slots and memory are reserved at once, the load runs on the loader
            while pending and pending[0].arrival_s <= t and len(active) + len(loading) < self.max_slots:
                r = pending[0]
                need = self._need(r)
                if used > 0 and used + need > self.budget:
                    break   # waits for running requests to free memory
                pending.popleft()
                wl = self._workload(r)
                run = {"req": r, "left": int(r.steps), "n": wl.n_particles, "bytes": need,
                       "admitted": t}
                loading.append((run, self._loader.submit(self._load, r, wl)))
                used += need
                st.admit_wait_s.append(max(0.0, t - r.arrival_s))
                st.runs += 1
            # loaded runs join the batch (in admission order; on the virtual clock every load is
            # awaited, in real time only the finished ones join)
            joined = False
            while loading and (not realtime or loading[0][1].done() or not active):
                run, fut = loading.popleft()
                run["ctx"] = fut.result()
                self.batch.add(run["ctx"])
                st.join_wait_s.append(max(0.0, now() - run["admitted"]))
                active.append(run)
                joined = True
            if joined and self.check_budget:
                held = sum(r["ctx"].get_info()["device_bytes"] for r in active)
                st.max_device_bytes = max(st.max_device_bytes, held)
                for r in active:
                    st.footprint_checks.append((r["bytes"], r["ctx"].get_info()["device_bytes"]))
                if held > self.budget:
                    raise RuntimeError(f"members hold {held} device bytes, over the budget "
                                       f"{self.budget}")
            st.max_concurrent = max(st.max_concurrent, len(active))
            if not active:
                last_end = None
                if pending and not loading:
                    if realtime:
                        time.sleep(max(0.0, pending[0].arrival_s - now()))
                    else:
                        vclock = max(vclock, pending[0].arrival_s)
                continue
            ta = time.perf_counter()
            self.batch.step(1)
            self.batch.sync()
            tb = time.perf_counter()
            st.step_s.append(tb - ta)
            st.cycle_s.append(tb - (last_end if last_end is not None else ta))
            last_end = tb
            st.cycles += 1
            st.particle_steps += sum(r["n"] for r in active)
            vclock += cycle_s
            keep = []
            for r in active:
                r["left"] -= 1
                if r["left"] > 0:
                    keep.append(r)
                    continue
                if on_finish is not None:
                    on_finish(r["req"], r["ctx"])
                self.batch.remove(r["ctx"])
                r["ctx"].close()
                used -= r["bytes"]
            active[:] = keep
        st.wall_s = time.perf_counter() - t0
        return st

    def close(self):
        self._loader.shutdown(wait=True)
        self.batch.close()
