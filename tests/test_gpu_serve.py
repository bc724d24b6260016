"""Serving: runs admitted into one batch as they arrive and retired when done.

Each served run's final state must equal the same run stepped alone (a context of its own,
pic_step), within the mixed-precision tolerance of the batch tests (1e-6: only the order of the
FP32 partial sums and FP64 atomic additions differs), whatever else shared the batch.  The
serving loop runs on a virtual clock here, so admissions are deterministic.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import picgen

pytestmark = pytest.mark.gpu

TOL = 1e-6


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
            "P": [ctx.read_particles(s) for s in range(nsp)], "info": ctx.get_info()}


@pytest.mark.parametrize("slots,budget", [(3, 64 << 30), (8, 6 << 20)])
def test_served_runs_equal_solo_runs(pic, slots, budget):
    from paper_1308_2590_amd import serve
    reqs = picgen.serving_stream(10, rate_per_s=400.0, seed=9, nx_range=(24, 64),
                                 nz_range=(16, 48), ppc_range=(4, 12), steps_range=(5, 30))
    _say(f"serve {len(reqs)} requests slots={slots} budget={budget}")
    results = {}

    def done(req, ctx):
        results[req.rid] = snapshot(ctx, 2)

    srv = serve.Server(picgen.request_workload, precision=1, max_slots=slots, budget_bytes=budget)
    st = srv.run(reqs, realtime=False, cycle_s=2e-3, on_finish=done)
    srv.close()
    summ = st.summary()
    _say(f"served: {summ}")
    assert st.runs == len(reqs) and len(results) == len(reqs)
    assert 1 < st.max_concurrent <= slots
    for req in reqs:
        wl = picgen.request_workload(req)
        ctx = pic.Context(wl.grid, precision=1)
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
        # the cell order could differ for a particle within rounding of a face, so each
        # component is compared as a sorted set of values
        for s in range(2):
            for k in ("xi_x", "xi_z", "ux", "uy", "uz"):
                a, b = np.sort(got["P"][s][k]), np.sort(solo["P"][s][k])
                assert rel(a, b) <= TOL, (req.rid, s, k)
