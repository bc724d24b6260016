"""Serving: runs admitted into one batch as they arrive and retired when done.

Each served run's final state must equal the same run stepped alone (a context of its own,
pic_step), within the mixed-precision tolerance of the batch tests (1e-6: only the order of the
FP32 partial sums and FP64 atomic additions differs), whatever else shared the batch.  Runs
carry particle labels, so the two are compared particle by particle: the cell-sorted order of
the labels is the same except for a particle that sits within rounding of a face, and every
particle's position and momentum agree.  The serving loop runs on a virtual clock here, so
admissions are deterministic; it checks after every join that the members' device memory
stays within the budget, and that the footprint it reserved for each run bounds what the run's
context holds.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import picgen

pytestmark = pytest.mark.gpu

TOL = 1e-6
FACE = 1e-5   # cells: a particle this close to a face may take the other side


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_2590_amd import binding
    binding.load_library()
    return binding


def rel(a, b):
    s = float(np.max(np.abs(b))) if b.size else 0.0
    d = float(np.max(np.abs(a - b))) if a.size else 0.0
    return d / s if s > 0 else d


def snapshot(ctx, nsp):
    E, H = ctx.read_fields()
    return {"M": ctx.read_moments(), "E": E, "H": H,
            "P": [ctx.read_particles(s, ids=True) for s in range(nsp)], "info": ctx.get_info()}


def compare_particles(got, solo, rid, s):
    """Particle by particle through the labels."""
    ig, io = got["id"], solo["id"]
    assert np.array_equal(np.sort(ig), np.sort(io)), (rid, s, "different particles alive")
    pg = np.argsort(ig, kind="stable")
    po = np.argsort(io, kind="stable")
    for k in ("xi_x", "xi_z", "ux", "uy", "uz", "w"):
        a, b = got[k][pg], solo[k][po]
        assert np.all(np.abs(a - b) <= TOL * (1.0 + np.abs(b))), (rid, s, k)
    # the order: identical apart from particles on a face
    if not np.array_equal(ig, io):
        bad = np.nonzero(ig != io)[0]
        x, z = got["xi_x"][bad], got["xi_z"][bad]
        near = (np.abs(x - np.round(x)) <= FACE) | (np.abs(z - np.round(z)) <= FACE)
        assert np.all(near), (rid, s, "order differs away from a face")


@pytest.mark.parametrize("slots,budget", [(3, 64 << 30), (8, 6 << 20)])
def test_served_runs_equal_solo_runs(pic, slots, budget):
    from paper_1308_2590_amd import serve
    reqs = picgen.serving_stream(10, rate_per_s=400.0, seed=9, nx_range=(24, 64),
                                 nz_range=(16, 48), ppc_range=(4, 12), steps_range=(5, 30))
    _say(f"serve {len(reqs)} requests slots={slots} budget={budget}")
    results = {}

    def done(req, ctx):
        results[req.rid] = snapshot(ctx, 2)

    srv = serve.Server(picgen.request_workload, precision=1, max_slots=slots, budget_bytes=budget,
                       track_ids=True, check_budget=True)
    st = srv.run(reqs, realtime=False, cycle_s=2e-3, on_finish=done)
    srv.close()
    summ = st.summary()
    _say(f"served: {summ}")
    assert st.runs == len(reqs) and len(results) == len(reqs)
    assert 1 < st.max_concurrent <= slots
    assert 0 < st.max_device_bytes <= budget
    assert st.footprint_checks and all(est >= held for est, held in st.footprint_checks)
    assert len(st.cycle_s) == len(st.step_s) and min(st.cycle_s) > 0
    for req in reqs:
        wl = picgen.request_workload(req)
        ctx = pic.Context(wl.grid, precision=1, track_ids=True)
        for s, sp in enumerate(wl.species):
            ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
        ctx.step(req.steps)
        solo = snapshot(ctx, 2)
        ctx.close()
        got = results[req.rid]
        assert got["info"]["step"] == req.steps == solo["info"]["step"]
        assert got["info"]["alive"] == solo["info"]["alive"]
        assert got["info"]["overflow_flags"] == 0
        for p in range(solo["M"].shape[0]):
            assert rel(got["M"][p], solo["M"][p]) <= TOL, (req.rid, p)
        assert rel(got["E"], solo["E"]) <= TOL and rel(got["H"], solo["H"]) <= TOL
        for s in range(2):
            compare_particles(got["P"][s], solo["P"][s], req.rid, s)


def test_serving_realtime_loader(pic):
    """Real-time arrivals with the loader thread: every request is served to completion, the
    cycle time seen by resident runs is recorded beside the GPU step time, and no run starts
    before it has arrived."""
    from paper_1308_2590_amd import serve
    reqs = picgen.serving_stream(12, rate_per_s=200.0, seed=4, nx_range=(24, 96),
                                 nz_range=(16, 64), ppc_range=(4, 16), steps_range=(10, 60))
    _say(f"serve {len(reqs)} requests in real time")
    finished = []
    srv = serve.Server(picgen.request_workload, precision=1, max_slots=6, track_ids=False)
    st = srv.run(reqs, realtime=True, on_finish=lambda r, c: finished.append(r.rid))
    srv.close()
    assert sorted(finished) == sorted(r.rid for r in reqs)
    assert st.cycles >= max(r.steps for r in reqs)
    summ = st.summary()
    _say(f"real-time serving: {summ}")
    assert summ["cycle_ms_p99"] >= summ["step_ms_p50"] > 0
