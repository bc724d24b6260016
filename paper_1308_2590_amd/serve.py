"""Continuous batching of independent runs on one GPU.

Requests (independent simulations) arrive over time.  A request is admitted as soon as it has
arrived, a slot is free and its device-memory footprint fits in the budget.  All admitted
runs are stepped together by one batch, with one launch of each kernel per cycle.  Particles
and fields stay resident on the device from admission to completion.  A run leaves the batch
after the cycles it asked for, which frees its slot and memory for waiting requests.  The
latency of every batch cycle is recorded.

The arithmetic all happens in the library's kernels.  This module only schedules: it decides
admission, creates and loads contexts, steps the batch and retires finished runs.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding


def footprint_bytes(nx, nz, bc_x, n_species, n_particles, precision):
    """Device bytes a run will hold (the library's allocations, rounded up by 10 %)."""
    nxn = nx + (1 if bc_x == 1 else 0)
    nodes, cells = nxn * nz, nx * nz
    grid = 8 * nodes * (3 * 2 + 12 + n_species) + 8 * cells * 3 * 2
    per_species_cells = 4 * cells * (9 + 1 + 2) + 8
    per_particle = 2 * (24 if precision == 1 else 40) + 2 * 4 + 4
    tiles = 4 * cells  # tile flags, lists and maps, generously
    return int(1.1 * (grid + n_species * per_species_cells + n_particles * per_particle + tiles))


@dataclass
class ServeStats:
    """Counters of one serving run.  particle_steps counts, for every cycle, the particles each
    active run was loaded with; step_s holds the wall time of every batch cycle (launch to
    completion)."""
    runs: int = 0
    cycles: int = 0
    particle_steps: float = 0.0
    wall_s: float = 0.0
    step_s: list = field(default_factory=list)
    max_concurrent: int = 0
    admit_wait_s: list = field(default_factory=list)

    def summary(self):
        lat = np.array(self.step_s) * 1e3 if self.step_s else np.zeros(1)
        wait = np.array(self.admit_wait_s) if self.admit_wait_s else np.zeros(1)
        return {
            "runs": self.runs,
            "cycles": self.cycles,
            "particle_steps_per_s": self.particle_steps / self.wall_s if self.wall_s > 0 else 0.0,
            "gpu_particle_steps_per_s": self.particle_steps / max(float(np.sum(self.step_s)), 1e-12),
            "step_ms_p50": float(np.percentile(lat, 50)),
            "step_ms_p99": float(np.percentile(lat, 99)),
            "step_ms_mean": float(np.mean(lat)),
            "wall_s": self.wall_s,
            "max_concurrent": self.max_concurrent,
            "admission_wait_s_p50": float(np.percentile(wait, 50)),
            "admission_wait_s_p99": float(np.percentile(wait, 99)),
        }


class Server:
    """Admit runs into one batch as slots and memory allow, step them together, retire them.

    make_workload(request) returns the run's workload (grid, species); the request needs the
    attributes rid, arrival_s and steps.  With realtime=True arrivals follow the wall clock
    (the server sleeps when it has nothing to run).  With realtime=False each cycle advances a
    virtual clock by cycle_s, which makes admission deterministic (used by the tests).
    """

    def __init__(self, make_workload, *, precision=1, max_slots=64, budget_bytes=64 << 30,
                 graph=True, device=0, tile=(0, 0)):
        self.make_workload = make_workload
        self.precision = precision
        self.max_slots = max_slots
        self.budget = budget_bytes
        self.device = device
        self.tile = tile
        self.batch = binding.Batch(device, precision)
        self.batch.set_graph(graph)
        self._cache = {}

    def _workload(self, req):
        wl = self._cache.pop(req.rid, None)
        return wl if wl is not None else self.make_workload(req)

    def _need(self, req):
        wl = self._cache.get(req.rid)
        if wl is None:
            wl = self._cache[req.rid] = self.make_workload(req)
        g = wl.grid
        return footprint_bytes(g.nx, g.nz, g.bc_x, g.n_species, wl.n_particles, self.precision)

    def _admit(self, req):
        need = self._need(req)
        wl = self._workload(req)
        g = wl.grid
        ctx = binding.Context(g, precision=self.precision, device=self.device, tile=self.tile)
        for s, sp in enumerate(wl.species):
            ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
        self.batch.add(ctx)
        return {"req": req, "ctx": ctx, "left": int(req.steps), "n": wl.n_particles, "bytes": need}

    def run(self, requests, *, realtime=True, cycle_s=1e-3, on_finish=None):
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        active = []
        used = 0
        st = ServeStats()
        vclock = 0.0
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0 if realtime else vclock

        while pending or active:
            t = now()
            while pending and pending[0].arrival_s <= t and len(active) < self.max_slots:
                r = pending[0]
                if used > 0 and used + self._need(r) > self.budget:
                    break   # waits for running requests to free memory
                pending.popleft()
                run = self._admit(r)
                used += run["bytes"]
                st.admit_wait_s.append(max(0.0, t - r.arrival_s))
                active.append(run)
                st.runs += 1
            st.max_concurrent = max(st.max_concurrent, len(active))
            if not active:
                if pending:
                    if realtime:
                        time.sleep(max(0.0, pending[0].arrival_s - now()))
                    else:
                        vclock = max(vclock, pending[0].arrival_s)
                continue
            ta = time.perf_counter()
            self.batch.step(1)
            self.batch.sync()
            dt = time.perf_counter() - ta
            st.step_s.append(dt)
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
            active = keep
        st.wall_s = time.perf_counter() - t0
        return st

    def close(self):
        self.batch.close()
