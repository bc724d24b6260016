"""The energy entry point that allocates no device memory (pic_energy_noalloc) against
pic_energy, through the C ABI.

Two calls in a row on different contexts, the second on a smaller input (fewer cells,
particles and species slots in use than the first left in the fixed buffer), each compared
with pic_energy of the same state to 1e-12 relative (the two differ only in the order of the
FP64 additions).  With an
allocator hook counting the library's device allocations, pic_energy_noalloc takes none,
while pic_energy takes its reduction buffer; and repeated calls on one state give the same
bits (the sums are added in a fixed order).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import picgen

pytestmark = pytest.mark.gpu


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


def _context(pic, wl, precision, seed):
    ctx = pic.Context(wl.grid, precision=precision)
    ctx.load_fields(*picgen.random_fields(seed, wl.grid))
    for s, sp in enumerate(wl.species):
        ctx.load_particles(s, sp.q, sp.m, sp.w, sp.xi_x, sp.xi_z, sp.ux, sp.uy, sp.uz)
    return ctx


def _close(a, b, tol=1e-12):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert abs(x - y) <= tol * max(abs(y), 1e-300), (a, b)


@pytest.mark.parametrize("precision", [picgen.PREC_FP64, picgen.PREC_MIXED])
def test_energy_noalloc_matches_energy(pic, precision):
    import torch
    big = picgen.with_particle_densities(picgen.random_small(61, nx=40, nz=33, ppc=6, bc_x=1), 3)
    small = picgen.random_small(62, nx=9, nz=5, ppc=2, bc_x=0)
    if precision == picgen.PREC_MIXED:
        big, small = picgen.fp32_representable(big), picgen.fp32_representable(small)
    counted = {"alloc": 0}

    def alloc(nbytes, device):
        counted["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=device)

    def free(ptr, nbytes, device):
        torch.cuda.caching_allocator_delete(int(ptr))

    try:
        pic.set_allocator(alloc, free)
        for name, wl, seed in (("larger", big, 5), ("smaller", small, 6)):
            _say(f"energy without allocation, {name} input, precision={precision}")
            ctx = _context(pic, wl, precision, seed)
            ctx.step(2)
            counted["alloc"] = 0
            e1 = ctx.energy_noalloc()
            e2 = ctx.energy_noalloc()
            assert counted["alloc"] == 0, "pic_energy_noalloc allocated device memory"
            assert e1 == e2, "repeated calls on one state differ"
            ref = ctx.energy()
            assert counted["alloc"] >= 1   # pic_energy takes its buffer through the hook
            _close(e1, ref)
            assert len(e1) == 1 + wl.grid.n_species and e1[0] > 0 and all(v >= 0 for v in e1)
            ctx.close()
    finally:
        pic.set_allocator(None, None)
