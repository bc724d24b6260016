"""Mover options (pic_set_mover) and the energy diagnostic (pic_energy) against the oracle.

Each option set (the Boris-style Lorentz-factor predictor, bilinear B, both) runs the cycle in
the per-particle kernel; the oracle runs the same options (pinned in test_oracle_pins).
Tolerances as in test_gpu_parity: FP64 arrays to 1e-10 in max-norm relative error, the sorted
order (labels) identical.  Energies: 1e-12 relative (FP64 sums in another order); the mixed
kinetic energy to 1e-6 (FP32 momenta).
"""
from __future__ import annotations

import numpy as np
import pytest

import picgen
from oracle import OracleSim
from tests.test_gpu_parity import (SMALL, _say, check_fields, check_moments, check_particles,
                                   rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_2590_amd import binding
    binding.load_library()
    return binding


def _setup(pic, wl, options, seed):
    fields = picgen.random_fields(300 + seed, wl.grid)
    ctx = pic.Context(wl.grid, track_ids=True)
    orc = OracleSim(wl.grid, mode=options)
    ctx.load_fields(*fields)
    orc.load_fields(*fields)
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
        orc.load_species(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    ctx.set_mover(options)
    return ctx, orc


@pytest.mark.parametrize("options", [1, 2, 3])
@pytest.mark.parametrize("wi", [0, 1, 3, 4])
def test_mover_options_match_oracle(pic, wi, options):
    wl = SMALL[wi]
    _say(f"mover options {options} workload {wi}")
    ctx, orc = _setup(pic, wl, options, wi)
    check_moments(ctx, orc)          # the deposit of the loaded state with the options
    for _ in range(2):
        ctx.step(2)
        orc.step(2)
        check_fields(ctx, orc)
        check_moments(ctx, orc)
        check_particles(ctx, orc, wl)
    info = ctx.get_info()
    assert info["overflow_flags"] == 0
    ctx.close()


@pytest.mark.parametrize("options", [1, 3])
def test_mover_options_dense_cells_per_particle_densities(pic, options):
    """The options kernel sums each value over the lanes that deposit into one cell before its
    global atomics.  100 particles per cell and species make runs of equal cells that fill
    whole wavefronts and cross wavefront and block edges; three species with per-particle
    densities and an absorbing x boundary (particles leave, the counts skip them)."""
    base = picgen.random_small(77, nx=9, nz=6, ppc=100, bc_x=1, masses=(1.0, 25.0, 4.0),
                               charges=(-1.0, 1.0, 2.0), temps=(20.0, 0.5, 2.0),
                               density=(0.8, 0.4, 0.2))
    wl = picgen.with_particle_densities(base, 77)
    _say(f"mover options {options}, dense cells, per-particle densities")
    ctx, orc = _setup(pic, wl, options, 77)
    check_moments(ctx, orc)
    for _ in range(2):
        ctx.step(2)
        orc.step(2)
        check_fields(ctx, orc)
        check_moments(ctx, orc)
        check_particles(ctx, orc, wl)
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()


def test_mover_switch_mid_run(pic):
    """Options on for three cycles, then back to the default tile kernel (and the oracle's
    default mover) for three more."""
    wl = SMALL[1]
    _say("mover switch")
    ctx, orc = _setup(pic, wl, 3, 1)
    ctx.step(3)
    orc.step(3)
    ctx.set_mover(0)
    orc.mode = 0
    check_moments(ctx, orc)
    ctx.step(3)
    orc.step(3)
    check_fields(ctx, orc)
    check_moments(ctx, orc)
    check_particles(ctx, orc, wl)
    ctx.close()


def test_energy_matches_oracle(pic):
    wl = SMALL[3]
    _say("energy")
    ctx, orc = _setup(pic, wl, 0, 3)
    for k in range(3):
        We, Wo = ctx.energy(), orc.energy()
        assert len(We) == 1 + wl.grid.n_species
        for a, b in zip(We, Wo):
            assert abs(a - b) <= 1e-12 * max(abs(b), 1e-300), (k, We, Wo)
        ctx.step(2)
        orc.step(2)
    ctx.close()
    # mixed: kinetic energy from FP32 momenta
    wlm = picgen.fp32_representable(SMALL[0])
    ctx = pic.Context(wlm.grid, precision=1)
    orc = OracleSim(wlm.grid)
    for s, sp in enumerate(wlm.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
        orc.load_species(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    We, Wo = ctx.energy(), orc.energy()
    assert abs(We[0] - Wo[0]) <= 1e-12 * max(Wo[0], 1e-300)
    for a, b in zip(We[1:], Wo[1:]):
        assert abs(a - b) <= 1e-6 * b
    ctx.close()


def test_mover_option_rules(pic):
    wl = SMALL[0]
    ctx = pic.Context(wl.grid)
    with pytest.raises(pic.PicError) as e:
        ctx.set_mover(4)
    assert e.value.status == 1
    with pytest.raises(pic.PicError) as e:
        ctx._check(ctx.lib.pic_energy(ctx.h, None, 0))
    assert e.value.status == 1
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    ctx.set_mover(pic.MOVER_B_BILINEAR)
    b = pic.Batch(0, 0)
    with pytest.raises(pic.PicError) as e:
        b.add(ctx)
    assert e.value.status == 1
    ctx.set_mover(0)
    b.add(ctx)
    with pytest.raises(pic.PicError) as e:
        ctx.set_mover(1)
    assert e.value.status == 4
    b.close()
    ctx.close()
    wlm = picgen.fp32_representable(wl)
    m = pic.Context(wlm.grid, precision=1)
    with pytest.raises(pic.PicError) as e:
        m.set_mover(1)
    assert e.value.status == 1
    m.set_mover(0)
    m.close()


def test_mover_options_full_foil_one_cycle(pic):
    """The 1024 x 512 foil (2.6 M particles) with both options: the deposit of the loaded state
    and one full cycle (fields, moments, sorted particles) against the oracle."""
    wl = picgen.named("foil")
    _say("mover options, full foil")
    ctx = pic.Context(wl.grid, track_ids=True)
    orc = OracleSim(wl.grid, mode=3)
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
        orc.load_species(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    ctx.set_mover(3)
    check_moments(ctx, orc)
    ctx.step(1)
    orc.step(1)
    check_fields(ctx, orc)
    check_moments(ctx, orc)
    check_particles(ctx, orc, wl)
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()


def test_mover_options_field_dominated_full_size_one_cycle(pic):
    """The 2048 x 2048 run (33.6M particles at 4 per cell and species, the laser entering
    through the absorbing x = 0 boundary) with both options: the deposit of the loaded state and
    one full cycle against the oracle.  Runs of equal cells are short here (about four lanes),
    the opposite of the foil's."""
    wl = picgen.named("lowdensity")
    _say(f"mover options, field-dominated full size {wl.n_particles} particles")
    ctx = pic.Context(wl.grid, track_ids=False)
    orc = OracleSim(wl.grid, mode=3)
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
        orc.load_species(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    ctx.set_mover(3)
    check_moments(ctx, orc)
    ctx.step(1)
    orc.step(1)
    check_fields(ctx, orc)
    check_moments(ctx, orc)
    check_particles(ctx, orc, wl, ids=False)
    assert ctx.get_info()["overflow_flags"] == 0
    ctx.close()
