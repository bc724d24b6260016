"""CPU checks of the C ABI: the library loads, exports every function include/pic.h declares,
and rejects invalid descriptors before touching a device (no compute calls here)."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import pytest

import picgen
from paper_1308_2590_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("pic_init_grid", "pic_load_particles", "pic_step", "pic_read_moments",
                     "pic_read_fields"):
        assert required in names
    assert sorted(binding.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpic.so not built")
    lib = C.CDLL(binding.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors have the size and field offsets gcc gives the C structs."""
    structs = {"pic_grid_desc": binding.GridDesc, "pic_info": binding.Info,
               "pic_profile": binding.Profile}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pic.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, f"{cname}.{f}"


def _desc(**kw):
    g = picgen.Grid(nx=8, nz=8, dx=1.0, dz=1.0, dt=0.5)
    d = binding.make_desc(g)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("field,value,msg", [
    ("dt", 2.0, "dt must not exceed"),
    ("nx", 0, "nx and nz"),
    ("nx", 1 << 22, "below 2^22"),
    ("bc_z", 1, "bc_z must be periodic"),
    ("precision", 7, "precision"),
    ("n_species", 9, "n_species"),
    ("allow_cfl_violation", 1, "dt must not exceed"),
    ("tile_x", 3, "tile_x, tile_z"),
])
def test_invalid_descriptor_rejected_before_device_use(field, value, msg):
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpic.so not built")
    lib = binding.load_library()
    d = _desc(**{field: value})
    h = C.c_void_p()
    st = lib.pic_init_grid(C.byref(d), C.byref(h))
    assert st == 1  # PIC_ERR_ARG
    assert h.value is None
    assert msg in lib.pic_last_error(None).decode()


def test_laser_needs_absorbing_axis():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpic.so not built")
    lib = binding.load_library()
    d = _desc(laser_a0=1.0, laser_sigma_z=1.0, laser_fwhm_t=1.0)
    h = C.c_void_p()
    assert lib.pic_init_grid(C.byref(d), C.byref(h)) == 1
    assert "absorbing" in lib.pic_last_error(None).decode()


def test_batch_argument_errors_without_device():
    """The batch calls reject bad arguments before touching a device."""
    import ctypes as C
    from paper_1308_2590_amd import binding
    lib = binding.load_library()
    h = C.c_void_p()
    assert lib.pic_batch_create(0, 7, C.byref(h)) == 1      # precision
    assert b"precision" in lib.pic_batch_last_error(None)
    assert lib.pic_batch_create(0, 0, None) == 1            # out is NULL
    assert lib.pic_batch_step(None, 1) == 1
    assert lib.pic_batch_add(None, None) == 1
    assert lib.pic_batch_remove(None, None) == 1
    assert lib.pic_batch_sync(None) == 1
    n = C.c_int32(-1)
    assert lib.pic_batch_size(None, C.byref(n)) == 1
    assert lib.pic_batch_set_graph(None, 1) == 1
    lib.pic_batch_destroy(None)


def test_set_allocator_rejects_half_a_pair_without_device():
    """pic_set_allocator takes both functions or neither; it touches no device."""
    lib = binding.load_library()
    null_a = C.cast(None, binding.ALLOC_FN)
    null_f = C.cast(None, binding.FREE_FN)
    hook = binding.ALLOC_FN(lambda n, d, u: None)
    assert lib.pic_set_allocator(hook, null_f, None) == 1
    assert b"both" in lib.pic_last_error(None)
    assert lib.pic_set_allocator(null_a, null_f, None) == 0


def test_load_particles_argument_errors_without_device():
    """pic_load_particles refuses a NULL context before touching a device."""
    lib = binding.load_library()
    assert lib.pic_load_particles(None, 0, -1.0, 1.0, 0, None, None, None, None, None, None, 1.0) == 1


def test_rank_mode_argument_errors_without_device():
    lib = binding.load_library()
    assert lib.pic_set_rank_mode(None, binding.RANK_CELLS) == 1
    assert b"NULL" in lib.pic_last_error(None)
