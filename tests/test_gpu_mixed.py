"""Parity of the mixed-precision form (PIC_PREC_MIXED) with the FP64 oracle.

The mixed form keeps each particle as an int32 cell key, FP32 in-cell offsets and FP32
momenta; the gather, the push and the per-particle moments run in FP32, and FP32 register and
LDS partial sums are folded into the FP64 moment planes.  The field solve stays FP64.  Inputs
are made exactly representable in that form (picgen.fp32_representable), so the two sides
start from the same state and every difference is FP32 rounding.

Tolerances, with the FP32 unit roundoff u = 2^-24 = 6.0e-8:
  moments    per plane, max |GPU - oracle| <= MOM_TOL * A_p, where A_p is the largest node
             value of the deposit of |contribution| (so cancelling planes such as delta-j are
             measured against the size of their terms).  One particle's compact moments take
             about 25 FP32 operations (relative error <= ~25 u), the corner weights and the
             expansion of S-hat with B a few more, and a node sums its contributions in FP32
             partials before the FP64 fold; for the few hundred contributions a node receives
             here the bound is of order 1e-5 and the observed error far below it.
  momenta    |u_GPU - u_oracle| <= U_TOL (1 + |u|): the push is ~40 FP32 operations on FP32
             fields (the FP64 E-bar and H are rounded once when staged).
  positions  |x_GPU - x_oracle| <= X_TOL cells: one FP32 add of a step of at most one cell to
             an offset in [0, 1), i.e. an absolute error of about u per cycle.
  fields     after one cycle, E and H differ only through the moments that enter the FP64
             solve; max-norm error relative to the field's largest value <= FIELD_TOL.
Integer results are exact where they are defined by the GPU's own positions: the cell-sorted
order equals the stable sort of the previous order by each particle's new cell.  A particle
can change cell relative to the oracle only when it is within X_TOL of a face; such particles
are counted and allowed.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import picgen
from oracle import OracleSim
from tests.order_match import align_sorted, cell_keys, near_face
from tests.pic_checks import abs_deposit_scale

pytestmark = pytest.mark.gpu

MOM_TOL = 1e-5
U_TOL = 2e-5
X_TOL = 1e-6
FIELD_TOL = 1e-6


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


def setup_both(pic, wl, *, fields=None, tile=(0, 0), track_ids=True):
    ctx = pic.Context(wl.grid, track_ids=track_ids, tile=tile, precision=picgen.PREC_MIXED)
    orc = OracleSim(wl.grid)
    if fields is not None:
        ctx.load_fields(*fields)
        orc.load_fields(*fields)
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
        orc.load_species(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    return ctx, orc


def species_tuples(wl, parts):
    """(q, m, w, positions, momenta) per species; the densities come with the particle lists
    (one per particle, in their order)."""
    return [(sp.q, sp.m, p["w"], p["xi_x"], p["xi_z"], p["ux"], p["uy"], p["uz"])
            for sp, p in zip(wl.species, parts)]


def moment_errors(M, Mo, scale):
    out = []
    for p in range(M.shape[0]):
        d = float(np.max(np.abs(M[p] - Mo[p]))) if M[p].size else 0.0
        out.append(d / scale[p] if scale[p] > 0 else d)
    return np.array(out)


def check_moments_vs(M, Mo, scale, tol=MOM_TOL, what=""):
    e = moment_errors(M, Mo, scale)
    _say(f"{what} moment errors (max over planes) {e.max():.2e}; per plane "
         + " ".join(f"{v:.1e}" for v in e))
    bad = np.nonzero(e > tol)[0]
    assert bad.size == 0, f"{what} planes {bad.tolist()} exceed {tol}: {e[bad]}"
    return e


def field_errors(ctx, orc):
    E, H = ctx.read_fields()
    errs = {}
    for name, A, B in (("E", E, orc.E), ("H", H, orc.H)):
        for r in range(3):
            s = float(np.max(np.abs(B[r])))
            d = float(np.max(np.abs(A[r] - B[r])))
            errs[f"{name}{'xyz'[r]}"] = d / s if s > 0 else d
    return errs


def mixed_small():
    out = []
    for seed, (nx, nz, bc, ppc) in enumerate([(7, 5, 0, 3), (13, 9, 1, 5), (20, 17, 0, 2),
                                              (33, 6, 1, 4), (1, 8, 0, 6), (9, 1, 0, 6)]):
        wl = picgen.random_small(seed, nx=nx, nz=nz, ppc=ppc, bc_x=bc, dx=0.5, dz=0.4, dt=0.3)
        out.append(picgen.fp32_representable(wl))
    return out


SMALL = mixed_small()


@pytest.mark.parametrize("tile", [(0, 0), (1, 1), (4, 4), (8, 2), (16, 8)])
@pytest.mark.parametrize("wi", range(len(SMALL)))
def test_mixed_load_and_deposit(pic, wi, tile):
    """Load: order and state exactly the oracle's; deposit within MOM_TOL."""
    wl = SMALL[wi]
    _say(f"mixed load/deposit {wl.name} tile={tile}")
    fields = picgen.random_fields(wi, wl.grid)
    ctx, orc = setup_both(pic, wl, fields=fields, tile=tile)
    for s in range(len(wl.species)):
        g = ctx.read_particles(s)
        o = orc.particles(s)
        assert np.array_equal(g["id"], o["id"])
        for k in ("xi_x", "xi_z", "ux", "uy", "uz"):
            assert np.array_equal(g[k], o[k]), k
    parts = [orc.particles(s) for s in range(len(wl.species))]
    scale = abs_deposit_scale(wl.grid.nx, wl.grid.nz, wl.grid.bc_x, wl.grid.dt,
                              species_tuples(wl, parts), orc.H)
    check_moments_vs(ctx.read_moments(), orc.moments(), scale, what="load")
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()


def compare_step(ctx, orc, wl, prev_ids):
    """After one cycle from identical state: per-particle state by label, the order, the
    moments (against the oracle's deposit of the GPU's own new state) and the fields."""
    nx, nz = wl.grid.nx, wl.grid.nz
    E, H = ctx.read_fields()
    gparts = []
    n_face = 0
    for s in range(len(wl.species)):
        g = ctx.read_particles(s, ids=True)
        o = orc.particles(s)
        gparts.append(g)
        # order: stable sort of the previous order by the new cell of each particle
        kg = np.floor(g["xi_z"]).astype(np.int64) * nx + np.floor(g["xi_x"]).astype(np.int64)
        assert np.all(np.diff(kg) >= 0)
        prev = prev_ids[s]
        rank_prev = np.zeros(int(max(prev.max(initial=-1), g["id"].max(initial=-1))) + 1, dtype=np.int64)
        rank_prev[prev] = np.arange(prev.size)
        if g["id"].size:
            key = kg * (prev.size + 1) + rank_prev[g["id"]]
            assert np.all(np.diff(key) > 0), "order is not stable by (cell, previous slot)"
        # state by label (labels are 0 .. n-1 from the load)
        nlab = int(max(prev.max(initial=-1), o["id"].max(initial=-1), g["id"].max(initial=-1))) + 1
        pos_o = np.full(nlab, -1, dtype=np.int64)
        pos_o[o["id"]] = np.arange(o["id"].size)
        pos_g = np.full(nlab, -1, dtype=np.int64)
        pos_g[g["id"]] = np.arange(g["id"].size)
        jg = np.nonzero(pos_o[g["id"]] >= 0)[0]
        jo = pos_o[g["id"][jg]]
        # alive sets may differ only by particles within X_TOL of an absorbing face
        only_g = np.nonzero((pos_g >= 0) & (pos_o < 0))[0]
        only_o = np.nonzero((pos_o >= 0) & (pos_g < 0))[0]
        xg = g["xi_x"][pos_g[only_g]]
        assert np.all(np.minimum(xg, nx - xg) <= X_TOL), f"species {s}: alive only on the GPU at x={xg}"
        xo = o["xi_x"][pos_o[only_o]]
        assert np.all(np.minimum(xo, nx - xo) <= X_TOL), f"species {s}: alive only in the oracle at x={xo}"
        if jg.size:
            for k, span in (("xi_x", nx), ("xi_z", nz)):
                d = np.abs(g[k][jg] - o[k][jo])
                d = np.minimum(d, span - d)
                assert float(d.max()) <= X_TOL, f"species {s} {k}: {d.max():.2e}"
            for k in ("ux", "uy", "uz"):
                d = np.abs(g[k][jg] - o[k][jo]) / (1.0 + np.abs(o[k][jo]))
                assert float(d.max()) <= U_TOL, f"species {s} {k}: {d.max():.2e}"
            ko = (np.floor(o["xi_z"][jo]).astype(np.int64) * nx
                  + np.floor(o["xi_x"][jo]).astype(np.int64))
            n_face += int(np.sum(kg[jg] != ko))
    _say(f"particles changing cell relative to the oracle (within {X_TOL} of a face): {n_face}")
    check_fields_and_moments(ctx, orc, wl, gparts, E, H)
    return n_face


def check_fields_and_moments(ctx, orc, wl, gparts, E, H):
    """Fields within FIELD_TOL of the oracle's; the GPU's moments within MOM_TOL of the
    oracle's deposit of the GPU's own new state with the GPU's fields."""
    nx, nz = wl.grid.nx, wl.grid.nz
    fe = field_errors(ctx, orc)
    _say("field errors " + " ".join(f"{k}={v:.1e}" for k, v in fe.items()))
    for k, v in fe.items():
        assert v <= FIELD_TOL, f"{k}: {v:.2e}"
    # moments of the GPU's new state, deposited by the oracle with the GPU's fields
    ref = OracleSim(wl.grid)
    ref.load_fields(E, H)
    for s, (sp, g) in enumerate(zip(wl.species, gparts)):
        ref.load_species(s, sp.q, sp.m, g["w"], g["xi_x"], g["xi_z"], g["ux"], g["uy"], g["uz"])
    scale = abs_deposit_scale(nx, nz, wl.grid.bc_x, wl.grid.dt, species_tuples(wl, gparts), H)
    check_moments_vs(ctx.read_moments(), ref.moments(), scale, what="step")
    # and against the oracle's own step (different by the FP32 push; cells can change)
    e = moment_errors(ctx.read_moments(), orc.moments(), scale)
    _say(f"moments vs the oracle's own step: max {e.max():.2e}")


def compare_step_unlabelled(ctx, orc, wl):
    """compare_step for a context without particle labels (the kernel instantiation the
    benchmark runs): both cell-sorted lists are matched slot by slot (same cell, positions
    within X_TOL, momenta within U_TOL (1 + |u|)); a particle may be out of place only when it
    lies within X_TOL of a face on both sides.  Then fields and moments as in compare_step."""
    nx, nz = wl.grid.nx, wl.grid.nz
    E, H = ctx.read_fields()
    gparts = []
    n_face = 0
    for s in range(len(wl.species)):
        g = ctx.read_particles(s, ids=False)
        o = orc.particles(s)
        gparts.append(g)
        assert np.all(np.diff(cell_keys(g, nx)) >= 0), f"species {s}: GPU order not sorted by cell"

        def close(a, b):
            ok = np.ones(a.size, dtype=bool)
            for k, span in (("xi_x", nx), ("xi_z", nz)):
                d = np.abs(g[k][a] - o[k][b])
                ok &= np.minimum(d, span - d) <= X_TOL
            for k in ("ux", "uy", "uz"):
                ok &= np.abs(g[k][a] - o[k][b]) <= U_TOL * (1.0 + np.abs(o[k][b]))
            ok &= g["w"][a] == o["w"][b]   # FP32-representable densities travel unchanged
            return ok

        jg, jo, eg, eo = align_sorted(g, o, nx, close)
        bad_g = eg[~near_face(g, eg, X_TOL, nx)]
        bad_o = eo[~near_face(o, eo, X_TOL, nx)]
        assert bad_g.size == 0 and bad_o.size == 0, (
            f"species {s}: {bad_g.size} GPU / {bad_o.size} oracle particles out of place or beyond "
            f"tolerance and not within {X_TOL} of a face (GPU slots {bad_g[:5].tolist()}, oracle "
            f"slots {bad_o[:5].tolist()}; {jg.size} matched of {len(g['xi_x'])} / {len(o['xi_x'])})")
        n_face += max(eg.size, eo.size)
    _say(f"particles out of place (within {X_TOL} of a face): {n_face}")
    check_fields_and_moments(ctx, orc, wl, gparts, E, H)
    return n_face


@pytest.mark.parametrize("rank", [1, 2])
@pytest.mark.parametrize("tile", [(0, 0), (4, 4), (8, 2)])
@pytest.mark.parametrize("wi", range(len(SMALL)))
def test_mixed_one_step(pic, wi, tile, rank):
    wl = SMALL[wi]
    _say(f"mixed step {wl.name} tile={tile} rank={rank}")
    fields = picgen.random_fields(100 + wi, wl.grid)
    ctx, orc = setup_both(pic, wl, fields=fields, tile=tile)
    ctx.set_rank_mode(rank)
    prev = [ctx.read_particles(s, ids=True)["id"] for s in range(len(wl.species))]
    ctx.step(1)
    orc.step(1)
    compare_step(ctx, orc, wl, prev)
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()


@pytest.mark.parametrize("tile", [(0, 0), (8, 2), (4, 4)])
@pytest.mark.parametrize("wi", range(len(SMALL)))
def test_mixed_without_labels_vs_oracle(pic, wi, tile):
    """The mixed kernel without particle labels (the instantiation the benchmark runs) against
    the FP64 oracle: one cycle from identical state, both sorted lists compared slot by slot."""
    wl = SMALL[wi]
    _say(f"mixed without labels {wl.name} tile={tile}")
    fields = picgen.random_fields(100 + wi, wl.grid)
    ctx, orc = setup_both(pic, wl, fields=fields, tile=tile, track_ids=False)
    ctx.step(1)
    orc.step(1)
    compare_step_unlabelled(ctx, orc, wl)
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()


def test_mixed_laser_absorbing(pic):
    wl = picgen.random_small(11, nx=24, nz=10, ppc=4, bc_x=1, dx=0.5, dz=0.4, dt=0.3,
                             laser_a0=2.0)
    wl = picgen.fp32_representable(wl)
    _say(f"mixed laser {wl.name}")
    ctx, orc = setup_both(pic, wl)
    ctx.set_step(40)
    orc.t = 40 * wl.grid.dt
    orc.step_count = 40
    prev = [ctx.read_particles(s, ids=True)["id"] for s in range(len(wl.species))]
    ctx.step(1)
    orc.step(1)
    compare_step(ctx, orc, wl, prev)
    ctx.close()


def test_mixed_face_particles(pic):
    """Particles on cell faces with tiny velocities towards the lower face: the mixed carry
    keeps every offset in [0, 1) and positions within X_TOL of the FP64 result."""
    nx, nz = 6, 5
    g = picgen.Grid(nx=nx, nz=nz, dx=0.5, dz=0.5, dt=0.25, bc_x=picgen.BC_ABSORBING,
                    n_species=1, precision=picgen.PREC_MIXED)
    xs, zs, ux, uz = [], [], [], []
    for i in range(nx):
        for k in range(nz):
            for v in (-1e-9, -1e-7, 0.0, 1e-9, -0.3):
                xs.append(float(i))
                zs.append(float(k))
                ux.append(v)
                uz.append(v)
    xs, zs = np.array(xs), np.array(zs)
    ux = np.array(ux, dtype=np.float32).astype(np.float64)
    uz = np.array(uz, dtype=np.float32).astype(np.float64)
    uy = np.zeros_like(ux)
    sp = picgen.Species(q=-1.0, m=1.0, w=0.0, xi_x=xs, xi_z=zs, ux=ux, uy=uy, uz=uz)
    wl = picgen.Workload(name="faces", grid=g, species=[sp], steps=1)
    ctx, orc = setup_both(pic, wl)
    prev = [ctx.read_particles(0, ids=True)["id"]]
    ctx.step(1)
    orc.step(1)
    p = ctx.read_particles(0, ids=True)
    for k in ("xi_x", "xi_z"):
        f = p[k] - np.floor(p[k])
        assert np.all((f >= 0.0) & (f < 1.0))
    compare_step(ctx, orc, wl, prev)
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()


def test_mixed_empty_and_all_absorbed(pic):
    g = picgen.Grid(nx=8, nz=4, dx=0.5, dz=0.5, dt=0.4, bc_x=picgen.BC_ABSORBING, n_species=3,
                    precision=picgen.PREC_MIXED)
    ctx = pic.Context(g, track_ids=True, precision=picgen.PREC_MIXED)
    e = np.zeros(0)
    ctx.load_particles(0, -1.0, 1.0, 0.5, e, e, e, e, e)
    # species 1 runs out through x = 0 in two cycles
    n = 12
    xs = np.linspace(0.05, 0.6, n)
    zs = np.linspace(0.1, 3.9, n)
    ux = np.full(n, -50.0)
    ctx.load_particles(1, -1.0, 1.0, 0.5, xs, zs, ux, np.zeros(n), np.zeros(n))
    ctx.load_particles(2, 1.0, 4.0, 0.5, np.array([3.5]), np.array([2.5]), np.zeros(1),
                       np.zeros(1), np.zeros(1))
    ctx.step(3)
    inf = ctx.get_info()
    assert inf["alive"][:3] == [0, 0, 1]
    assert inf["absorbed"][:3] == [0, n, 0]
    assert inf["overflow_flags"] == 0
    M = ctx.read_moments()
    assert np.isclose(M[12 + 2].sum(), 0.5, rtol=0, atol=1e-12)
    ctx.close()


def test_mixed_charge_conserved_many_cycles(pic):
    """Partition of unity: each species' density plane sums to its total weight, every cycle,
    to FP32 rounding of the partial sums."""
    wl = picgen.fp32_representable(picgen.named("uniform64b"))
    ctx = pic.Context(wl.grid, precision=picgen.PREC_MIXED)
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    for _ in range(10):
        ctx.step(1)
        M = ctx.read_moments()
        for s, sp in enumerate(wl.species):
            tot = sp.w * sp.n
            assert abs(M[12 + s].sum() - tot) <= 1e-6 * tot
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()


def test_mixed_full_size_foil_dense(pic):
    """The mixed-precision foil workload (1024 x 512, 128 particles per cell and species in a
    40-cell slab of density 200): one cycle from identical state against the oracle, at the
    tile shape the benchmark runs."""
    wl = picgen.fp32_representable(picgen.named("foil_dense"))
    _say(f"mixed full size {wl.name}: {wl.n_particles} particles")
    ctx, orc = setup_both(pic, wl, fields=picgen.random_fields(4, wl.grid), track_ids=True)
    ctx.set_step(300)
    orc.t = 300 * wl.grid.dt
    orc.step_count = 300
    prev = [ctx.read_particles(s, ids=True)["id"] for s in range(len(wl.species))]
    ctx.step(1)
    orc.step(1)
    compare_step(ctx, orc, wl, prev)
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()


@pytest.mark.parametrize("name", ["foil_dense", "foil_dense_cm", "lowdensity"])
def test_mixed_full_size_unlabelled(pic, name):
    """The mixed-precision workloads at full size in the launch configuration the benchmark
    times (automatic tiles, no particle labels): the geometry-literal dense foil (40-cell slab,
    5.24M particles), the count-matched one (160-cell slab, 21.0M particles) and the 2048 x 2048
    run (33.6M particles, the chunk-of-2 form with its direct deposit), one cycle from
    identical state against the FP64 oracle, both sorted lists compared slot by slot."""
    wl = picgen.fp32_representable(picgen.named(name))
    _say(f"mixed full size unlabelled {wl.name}: {wl.n_particles} particles")
    ctx, orc = setup_both(pic, wl, fields=picgen.random_fields(4, wl.grid), track_ids=False)
    ctx.set_step(300)
    orc.t = 300 * wl.grid.dt
    orc.step_count = 300
    ctx.step(1)
    orc.step(1)
    compare_step_unlabelled(ctx, orc, wl)
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()


@pytest.mark.parametrize("labels", [True, False])
@pytest.mark.parametrize("wi", [0, 1, 3])
def test_mixed_per_particle_densities(pic, wi, labels):
    """Per-particle densities in the mixed form (stored as FP32; the inputs are FP32
    representable): one cycle from identical state against the FP64 oracle."""
    wl = picgen.fp32_representable(picgen.with_particle_densities(SMALL[wi], seed=40 + wi))
    _say(f"mixed per-particle densities {wl.name} labels={labels}")
    fields = picgen.random_fields(100 + wi, wl.grid)
    ctx, orc = setup_both(pic, wl, fields=fields, tile=(8, 2), track_ids=labels)
    prev = [ctx.read_particles(s, ids=True)["id"] for s in range(len(wl.species))] if labels else None
    ctx.step(1)
    orc.step(1)
    if labels:
        compare_step(ctx, orc, wl, prev)
    else:
        compare_step_unlabelled(ctx, orc, wl)
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()
