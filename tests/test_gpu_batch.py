"""Batches: many runs stepped by one launch of each kernel per cycle (pic_batch_*).

Every run of a batch must give the result of stepping it alone (pic_step): the cycle is the
same, only the order of the floating-point atomic additions of the deposit can differ.  So
FP64 runs agree with their solo copies to 1e-12 in max-norm relative error per array, and the
sorted order (labels) is identical; the solo path itself matches the oracle to 1e-10
(test_gpu_parity).  Mixed-precision runs agree with their solo copies to 1e-6 (FP32 partial
sums in a different order).  Runs join and leave at different cycles, so their buffer parities
differ; replays of a captured cycle are checked after every replay, with host reads in between.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import picgen
from oracle import OracleSim

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOLMIX = 1e-6


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


def workloads(precision=picgen.PREC_FP64):
    shapes = [(7, 5, 0, 3), (20, 17, 1, 2), (33, 6, 1, 4), (9, 1, 0, 6), (40, 24, 0, 3)]
    out = []
    for seed, (nx, nz, bc, ppc) in enumerate(shapes):
        wl = picgen.random_small(30 + seed, nx=nx, nz=nz, ppc=ppc, bc_x=bc, dx=0.5, dz=0.4, dt=0.3)
        if precision == picgen.PREC_MIXED:
            wl = picgen.fp32_representable(wl)
        out.append(wl)
    return out


def make(pic, wl, precision, seed, step0=0):
    ctx = pic.Context(wl.grid, track_ids=True, precision=precision)
    ctx.load_fields(*picgen.random_fields(200 + seed, wl.grid))
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    if step0:
        ctx.set_step(step0)
    return ctx


def compare(a, b, nsp, tol):
    Ma, Mb = a.read_moments(), b.read_moments()
    for p in range(Ma.shape[0]):
        assert rel(Ma[p], Mb[p]) <= tol, f"moment plane {p}: {rel(Ma[p], Mb[p]):.2e}"
    Ea, Ha = a.read_fields()
    Eb, Hb = b.read_fields()
    assert rel(Ea, Eb) <= tol and rel(Ha, Hb) <= tol
    for s in range(nsp):
        pa, pb = a.read_particles(s, ids=True), b.read_particles(s, ids=True)
        assert np.array_equal(pa["id"], pb["id"]), f"species {s}: order differs"
        for k in ("xi_x", "xi_z", "ux", "uy", "uz", "w"):
            assert rel(pa[k], pb[k]) <= tol, f"species {s} {k}: {rel(pa[k], pb[k]):.2e}"
    ia, ib = a.get_info(), b.get_info()
    assert ia["step"] == ib["step"] and ia["alive"] == ib["alive"]
    assert ia["overflow_flags"] == 0 and ib["overflow_flags"] == 0


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_solo_fp64(pic, graph):
    wls = workloads()
    _say(f"batch fp64 graph={graph}")
    solo = [make(pic, wl, 0, i) for i, wl in enumerate(wls)]
    mem = [make(pic, wl, 0, i) for i, wl in enumerate(wls)]
    # both rankers of the sort, in the batch and alone (the order is the same)
    for i in range(len(wls)):
        mem[i].set_rank_mode(1 + i % 2)
        solo[i].set_rank_mode(2 - i % 2)
    b = pic.Batch(0, 0)
    b.set_graph(graph)
    for c in mem:
        b.add(c)
    assert b.size() == len(mem)
    for rnd in range(3):
        b.step(2)
        for c in solo:
            c.step(2)
        for i, wl in enumerate(wls):   # reads between cycles (and between graph replays)
            compare(mem[i], solo[i], len(wl.species), TOL64)
    b.close()
    for c in solo + mem:
        c.close()


def test_batch_member_matches_oracle(pic):
    wl = workloads()[1]
    _say("batch member vs oracle")
    ctx = make(pic, wl, 0, 1)
    other = make(pic, workloads()[4], 0, 4)
    orc = OracleSim(wl.grid)
    orc.load_fields(*picgen.random_fields(201, wl.grid))
    for s, sp in enumerate(wl.species):
        orc.load_species(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    b = pic.Batch(0, 0)
    b.add(ctx)
    b.add(other)
    b.step(4)
    orc.step(4)
    M, Mo = ctx.read_moments(), orc.moments()
    for p in range(M.shape[0]):
        assert rel(M[p], Mo[p]) <= 1e-10
    E, H = ctx.read_fields()
    assert rel(E, orc.E) <= 1e-10 and rel(H, orc.H) <= 1e-10
    for s in range(len(wl.species)):
        g, o = ctx.read_particles(s, ids=True), orc.particles(s)
        assert np.array_equal(g["id"], o["id"])
        assert rel(g["ux"], o["ux"]) <= 1e-10
    b.close()
    ctx.close()
    other.close()


def test_batch_staggered_membership(pic):
    """Runs join and leave at different cycles (different buffer parities and step counts),
    one with a laser so the device-side step counter sets the source time."""
    wls = workloads()
    laser = picgen.random_small(77, nx=24, nz=10, ppc=3, bc_x=1, dx=0.5, dz=0.4, dt=0.3,
                                laser_a0=2.0)
    wls = wls[:3] + [laser]
    _say("batch staggered membership")
    solo = [make(pic, wl, 0, i, step0=(40 if i == 3 else 0)) for i, wl in enumerate(wls)]
    mem = [make(pic, wl, 0, i, step0=(40 if i == 3 else 0)) for i, wl in enumerate(wls)]
    b = pic.Batch(0, 0)
    b.set_graph(True)
    b.add(mem[0])
    b.step(3)
    solo[0].step(3)
    b.add(mem[1])
    b.add(mem[3])
    b.step(2)
    for i in (0, 1, 3):
        solo[i].step(2)
    b.remove(mem[0])
    mem[2].step(1)       # a context stepped alone before it joins
    solo[2].step(1)
    b.add(mem[2])
    b.step(5)
    for i in (1, 2, 3):
        solo[i].step(5)
    for i, wl in enumerate(wls):
        compare(mem[i], solo[i], len(wl.species), TOL64)
    assert np.max(np.abs(mem[3].read_fields()[0][1])) > 1e-3   # the source injected a field
    # a member removed from the batch steps alone again
    mem[0].step(2)
    solo[0].step(2)
    compare(mem[0], solo[0], len(wls[0].species), TOL64)
    b.close()
    for c in solo + mem:
        c.close()


def test_batch_mixed(pic):
    wls = workloads(picgen.PREC_MIXED)
    _say("batch mixed")
    solo = [make(pic, wl, 1, i) for i, wl in enumerate(wls)]
    mem = [make(pic, wl, 1, i) for i, wl in enumerate(wls)]
    b = pic.Batch(0, 1)
    b.set_graph(True)
    for c in mem:
        b.add(c)
    b.step(4)
    for c in solo:
        c.step(4)
    for i, wl in enumerate(wls):
        compare(mem[i], solo[i], len(wl.species), TOLMIX)
    b.close()
    for c in solo + mem:
        c.close()


def test_batch_reload_member(pic):
    """Loading new particles into a member between batch steps takes effect at the next step."""
    wls = workloads()
    _say("batch reload member")
    a, a_solo = make(pic, wls[0], 0, 0), make(pic, wls[0], 0, 0)
    c, c_solo = make(pic, wls[2], 0, 2), make(pic, wls[2], 0, 2)
    b = pic.Batch(0, 0)
    b.add(a)
    b.add(c)
    b.step(2)
    a_solo.step(2)
    c_solo.step(2)
    new = picgen.random_small(99, nx=wls[2].grid.nx, nz=wls[2].grid.nz, ppc=5, bc_x=1,
                              dx=0.5, dz=0.4, dt=0.3).species[0]
    for ctx in (c, c_solo):
        ctx.load_particles(0, new.q, new.m, new.w, new.xi_x, new.xi_z, new.ux, new.uy, new.uz)
    b.step(3)
    a_solo.step(3)
    c_solo.step(3)
    compare(a, a_solo, 2, TOL64)
    compare(c, c_solo, 2, TOL64)
    b.close()
    for ctx in (a, a_solo, c, c_solo):
        ctx.close()


def test_batch_rules(pic):
    wls = workloads()
    ctx = make(pic, wls[0], 0, 0)
    mixed = make(pic, workloads(picgen.PREC_MIXED)[0], 1, 0)
    b = pic.Batch(0, 0)
    b.add(ctx)
    with pytest.raises(pic.PicError) as e:
        b.add(ctx)
    assert e.value.status == 1
    with pytest.raises(pic.PicError) as e:
        b.add(mixed)
    assert e.value.status == 1
    with pytest.raises(pic.PicError) as e:
        ctx.step(1)
    assert e.value.status == 4
    with pytest.raises(pic.PicError) as e:
        b.remove(mixed)
    assert e.value.status == 1
    b.step(0)
    b.remove(ctx)
    ctx.step(1)   # alone again
    empty = pic.Batch(0, 1)
    empty.step(3)   # no members: nothing to do
    assert empty.size() == 0
    empty.close()
    b.close()
    ctx.close()
    mixed.close()


def test_set_tiles_and_autotune(pic):
    """Re-tiling mid-run changes nothing but the order of atomic additions; the autotuner
    leaves a valid shape applied; a shape too large for LDS is refused and the old one kept."""
    from paper_1308_2590_amd import autotune
    wl = workloads()[4]
    a, b = make(pic, wl, 0, 4), make(pic, wl, 0, 4)
    a.step(2)
    b.step(2)
    b.set_tiles(8, 2)
    assert b.get_info()["tile"] == (8, 2)
    a.step(3)
    b.step(3)
    compare(b, a, 2, TOL64)
    with pytest.raises(pic.PicError) as e:
        b.set_tiles(64, 64)
    assert e.value.status == 1 and b.get_info()["tile"] == (8, 2)
    res = autotune.tune_tiles(b, cycles=2, warmup=1)
    assert tuple(b.get_info()["tile"]) == tuple(res["best"])
    a.step(res["cycles_used"])
    compare(b, a, 2, TOL64)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [picgen.PREC_FP64, picgen.PREC_MIXED])
def test_batch_with_per_particle_densities(pic, precision):
    """Members carrying per-particle densities next to members with one density per species:
    the batch runs the kernel with per-particle densities for all and matches the solo runs."""
    wls = workloads(precision)
    wls = [picgen.with_particle_densities(wl, seed=i) if i % 2 == 0 else wl
           for i, wl in enumerate(wls)]
    if precision == picgen.PREC_MIXED:
        wls = [picgen.fp32_representable(wl) for wl in wls]
    tol = TOL64 if precision == picgen.PREC_FP64 else TOLMIX
    _say(f"batch with per-particle densities precision={precision}")
    solo = [make(pic, wl, precision, i) for i, wl in enumerate(wls)]
    mem = [make(pic, wl, precision, i) for i, wl in enumerate(wls)]
    b = pic.Batch(0, precision)
    b.set_graph(True)
    for c in mem:
        b.add(c)
    for _ in range(2):
        b.step(2)
        for c in solo:
            c.step(2)
        for i, wl in enumerate(wls):
            compare(mem[i], solo[i], len(wl.species), tol)
    b.close()
    for c in solo + mem:
        c.close()
