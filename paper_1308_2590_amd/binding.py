"""Thin ctypes binding of include/pic.h (argument marshalling only).

Every computation happens in the HIP library ``libpic.so`` built in-tree by ``build.py``.
There is no fallback: if the library is missing or fails to load, every call raises.
PyTorch is imported first so that the library and torch share one HIP runtime in the
process; it is otherwise only used to pass a torch stream to ``set_stream``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpic.so")

PIC_OK = 0
STATUS = {0: "PIC_OK", 1: "PIC_ERR_ARG", 2: "PIC_ERR_OOM", 3: "PIC_ERR_DEVICE",
          4: "PIC_ERR_STATE", 5: "PIC_ERR_RANGE", 6: "PIC_ERR_OVERFLOW"}
MAX_SPECIES = 8
MOVER_GAMMA_PREDICT = 1   # gamma-bar = gamma(u^n + beta E^n) (Boris-style predictor)
MOVER_B_BILINEAR = 2      # B interpolated from the four surrounding cell centres
RANK_AUTO, RANK_ROWS, RANK_CELLS = 0, 1, 2   # rankers of the cell sort (pic_set_rank_mode)
EXPORTED = ["pic_init_grid", "pic_load_particles", "pic_load_fields", "pic_set_tiles",
            "pic_set_rank_mode", "pic_set_step", "pic_step",
            "pic_read_moments", "pic_read_fields", "pic_read_particles", "pic_get_info",
            "pic_set_stream", "pic_sync", "pic_profile_enable", "pic_profile_read",
            "pic_set_mover", "pic_energy", "pic_energy_noalloc", "pic_set_allocator",
            "pic_last_error", "pic_destroy",
            "pic_batch_create", "pic_batch_add", "pic_batch_remove", "pic_batch_step",
            "pic_batch_set_graph", "pic_batch_sync", "pic_batch_size", "pic_batch_last_error",
            "pic_batch_destroy"]


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("dx", C.c_double), ("dz", C.c_double),
                ("dt", C.c_double), ("bc_x", C.c_int32), ("bc_z", C.c_int32),
                ("precision", C.c_int32), ("n_species", C.c_int32),
                ("e0", C.c_double * 3), ("h0", C.c_double * 3),
                ("laser_a0", C.c_double), ("laser_omega", C.c_double),
                ("laser_sigma_z", C.c_double), ("laser_z_center", C.c_double),
                ("laser_fwhm_t", C.c_double), ("laser_t_center", C.c_double),
                ("allow_cfl_violation", C.c_int32), ("track_ids", C.c_int32),
                ("tile_x", C.c_int32), ("tile_z", C.c_int32), ("device", C.c_int32),
                ("reserved", C.c_int32 * 7)]


class Info(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("n_species", C.c_int32),
                ("nodes_x", C.c_int32), ("nodes_z", C.c_int32), ("cells_x", C.c_int32),
                ("cells_z", C.c_int32), ("tile_x", C.c_int32), ("tile_z", C.c_int32),
                ("precision", C.c_int32), ("alive", C.c_int64 * MAX_SPECIES),
                ("absorbed", C.c_int64 * MAX_SPECIES), ("overflow_flags", C.c_uint32),
                ("rank_mode", C.c_int32), ("device_bytes", C.c_int64)]


class Profile(C.Structure):
    _fields_ = [("steps", C.c_int64), ("particle_launches", C.c_int64),
                ("particle_ms", C.c_double), ("field_launches", C.c_int64),
                ("field_ms", C.c_double), ("sort_launches", C.c_int64), ("sort_ms", C.c_double),
                ("step_ms", C.c_double)]


# Device-memory hook types of pic_set_allocator.
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_int32, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_uint64, C.c_int32, C.c_void_p)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpic.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1308_2590_amd/build.py "
                           "(or __graft_entry__.build())")
    try:
        import torch  # noqa: F401  -- one HIP runtime per process, shared with torch
    except ImportError:
        pass
    lib = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "pic_init_grid": ([C.POINTER(GridDesc), C.POINTER(P)], C.c_int),
        "pic_load_particles": ([P, I32, D, D, I64, P, P, P, P, P, P, D], C.c_int),
        "pic_load_fields": ([P, P, P], C.c_int),
        "pic_set_tiles": ([P, I32, I32], C.c_int),
        "pic_set_rank_mode": ([P, I32], C.c_int),
        "pic_set_step": ([P, I64], C.c_int),
        "pic_step": ([P, I32], C.c_int),
        "pic_read_moments": ([P, P, I64], C.c_int),
        "pic_read_fields": ([P, P, P], C.c_int),
        "pic_read_particles": ([P, I32, C.POINTER(I64), P, P, P, P, P, P, P], C.c_int),
        "pic_get_info": ([P, C.POINTER(Info)], C.c_int),
        "pic_set_stream": ([P, P], C.c_int),
        "pic_sync": ([P], C.c_int),
        "pic_profile_enable": ([P, I32], C.c_int),
        "pic_profile_read": ([P, C.POINTER(Profile)], C.c_int),
        "pic_set_mover": ([P, I32], C.c_int),
        "pic_energy": ([P, P, I32], C.c_int),
        "pic_energy_noalloc": ([P, P, I32], C.c_int),
        "pic_set_allocator": ([ALLOC_FN, FREE_FN, P], C.c_int),
        "pic_last_error": ([P], C.c_char_p),
        "pic_destroy": ([P], None),
        "pic_batch_create": ([I32, I32, C.POINTER(P)], C.c_int),
        "pic_batch_add": ([P, P], C.c_int),
        "pic_batch_remove": ([P, P], C.c_int),
        "pic_batch_step": ([P, I32], C.c_int),
        "pic_batch_set_graph": ([P, I32], C.c_int),
        "pic_batch_sync": ([P], C.c_int),
        "pic_batch_size": ([P, C.POINTER(I32)], C.c_int),
        "pic_batch_last_error": ([P], C.c_char_p),
        "pic_batch_destroy": ([P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_desc(grid, *, track_ids=False, tile=(0, 0), device=0, precision=None) -> GridDesc:
    """pic_grid_desc from any object with the grid attributes (nx, nz, dx, dz, dt, bc_x, ...)."""
    d = GridDesc()
    d.nx, d.nz = int(grid.nx), int(grid.nz)
    d.dx, d.dz, d.dt = float(grid.dx), float(grid.dz), float(grid.dt)
    d.bc_x, d.bc_z = int(grid.bc_x), int(grid.bc_z)
    d.precision = int(getattr(grid, "precision", 0) if precision is None else precision)
    d.n_species = int(grid.n_species)
    for r in range(3):
        d.e0[r] = float(grid.e0[r])
        d.h0[r] = float(grid.h0[r])
    d.laser_a0, d.laser_omega = float(grid.laser_a0), float(grid.laser_omega)
    d.laser_sigma_z, d.laser_z_center = float(grid.laser_sigma_z), float(grid.laser_z_center)
    d.laser_fwhm_t, d.laser_t_center = float(grid.laser_fwhm_t), float(grid.laser_t_center)
    d.allow_cfl_violation = int(getattr(grid, "allow_cfl_violation", 0))
    d.track_ids = 1 if track_ids else 0
    d.tile_x, d.tile_z = int(tile[0]), int(tile[1])
    d.device = int(device)
    return d


class Context:
    """One pic_ctx.  Method names follow the C ABI without the ``pic_`` prefix."""

    def __init__(self, grid, *, track_ids=False, tile=(0, 0), device=0, precision=None):
        self.lib = load_library()
        self.desc = make_desc(grid, track_ids=track_ids, tile=tile, device=device,
                              precision=precision)
        h = C.c_void_p()
        st = self.lib.pic_init_grid(C.byref(self.desc), C.byref(h))
        if st != PIC_OK:
            raise PicError(st, self.lib.pic_last_error(None).decode())
        self.h = h
        self.S = self.desc.n_species
        self.nxn = self.desc.nx + (1 if self.desc.bc_x == 1 else 0)
        self.nzn = self.desc.nz
        self.nx, self.nz = self.desc.nx, self.desc.nz

    def _check(self, st):
        if st != PIC_OK:
            raise PicError(st, self.lib.pic_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.pic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the ABI --------------------------------------------------------------------------
    def load_particles(self, s, q, m, w, xi_x, xi_z, ux, uy, uz):
        """w: one density for the whole species (a number) or one per particle (an array)."""
        arrs = [_f64(a) for a in (xi_x, xi_z, ux, uy, uz)]
        n = arrs[0].shape[0]
        if any(a.shape[0] != n for a in arrs):
            raise ValueError("particle arrays differ in length")
        if np.ndim(w) == 0:
            wa, wu = None, float(w)
        else:
            wa, wu = _f64(w), 0.0
            if wa.shape[0] != n:
                raise ValueError("w has another length than the particle arrays")
        self._check(self.lib.pic_load_particles(self.h, int(s), float(q), float(m), n,
                                                *[_p(a) for a in arrs], _p(wa), wu))

    def load_fields(self, e=None, h=None):
        e = None if e is None else _f64(e).reshape(-1)
        h = None if h is None else _f64(h).reshape(-1)
        if e is not None and e.size != 3 * self.nxn * self.nzn:
            raise ValueError("E must have 3 * nodes values")
        if h is not None and h.size != 3 * self.nx * self.nz:
            raise ValueError("H must have 3 * cells values")
        self._check(self.lib.pic_load_fields(self.h, _p(e), _p(h)))

    def set_tiles(self, tile_x, tile_z):
        self._check(self.lib.pic_set_tiles(self.h, int(tile_x), int(tile_z)))

    def set_rank_mode(self, mode):
        """RANK_AUTO, RANK_ROWS or RANK_CELLS (the sort's ranker; same order either way)."""
        self._check(self.lib.pic_set_rank_mode(self.h, int(mode)))

    def set_mover(self, options):
        """MOVER_* bits (0: the default mover); FP64 contexts only."""
        self._check(self.lib.pic_set_mover(self.h, int(options)))

    def energy(self):
        """[field energy, kinetic energy of species 0, 1, ...] of the current state."""
        out = np.zeros(1 + self.S)
        self._check(self.lib.pic_energy(self.h, _p(out), len(out)))
        return [float(v) for v in out]

    def energy_noalloc(self):
        """energy() through the entry point that allocates no device memory."""
        out = np.zeros(1 + self.S)
        self._check(self.lib.pic_energy_noalloc(self.h, _p(out), len(out)))
        return [float(v) for v in out]

    def set_step(self, step):
        self._check(self.lib.pic_set_step(self.h, int(step)))

    def step(self, nsteps=1):
        self._check(self.lib.pic_step(self.h, int(nsteps)))

    def read_moments(self):
        out = np.empty((12 + self.S, self.nzn, self.nxn))
        self._check(self.lib.pic_read_moments(self.h, _p(out), out.size))
        return out

    def read_fields(self):
        e = np.empty((3, self.nzn, self.nxn))
        h = np.empty((3, self.nz, self.nx))
        self._check(self.lib.pic_read_fields(self.h, _p(e), _p(h)))
        return e, h

    def read_particles(self, s, ids=None):
        if ids is None:
            ids = bool(self.desc.track_ids)
        info = self.get_info()
        n = int(info["alive"][s])
        cap = C.c_int64(n)
        out = {k: np.empty(n) for k in ("xi_x", "xi_z", "ux", "uy", "uz", "w")}
        idv = np.empty(n, dtype=np.int64) if ids else None
        self._check(self.lib.pic_read_particles(self.h, int(s), C.byref(cap), _p(out["xi_x"]),
                                                _p(out["xi_z"]), _p(out["ux"]), _p(out["uy"]),
                                                _p(out["uz"]), _p(out["w"]), _p(idv)))
        if idv is not None:
            out["id"] = idv
        return out

    def get_info(self):
        inf = Info()
        self._check(self.lib.pic_get_info(self.h, C.byref(inf)))
        S = inf.n_species
        return {"step": inf.step, "t": inf.t, "n_species": S, "nodes_x": inf.nodes_x,
                "nodes_z": inf.nodes_z, "cells_x": inf.cells_x, "cells_z": inf.cells_z,
                "tile": (inf.tile_x, inf.tile_z), "precision": inf.precision,
                "alive": [inf.alive[s] for s in range(S)],
                "absorbed": [inf.absorbed[s] for s in range(S)],
                "overflow_flags": inf.overflow_flags, "rank_mode": inf.rank_mode,
                "device_bytes": inf.device_bytes}

    def set_stream(self, stream=None):
        """stream: a torch.cuda.Stream, a raw hipStream_t as int, or None (own stream)."""
        ptr = None
        if stream is not None:
            ptr = int(getattr(stream, "cuda_stream", stream))
        self._check(self.lib.pic_set_stream(self.h, C.c_void_p(ptr) if ptr else None))

    def sync(self):
        self._check(self.lib.pic_sync(self.h))

    def profile_enable(self, on=True, every=1):
        """Start (on) or stop per-kernel event timing; with every = n only every n-th cycle is
        timed, the first one included."""
        self._check(self.lib.pic_profile_enable(self.h, int(every) if on else 0))

    def profile_read(self):
        p = Profile()
        self._check(self.lib.pic_profile_read(self.h, C.byref(p)))
        return {f: getattr(p, f) for f, _ in Profile._fields_}


class Batch:
    """One pic_batch: member Contexts stepped together.  Names follow the C ABI without the
    ``pic_batch_`` prefix."""

    def __init__(self, device=0, precision=0):
        self.lib = load_library()
        h = C.c_void_p()
        st = self.lib.pic_batch_create(int(device), int(precision), C.byref(h))
        if st != 0:
            raise PicError(st, self.lib.pic_batch_last_error(None).decode())
        self.h = h
        self.members = []

    def _check(self, st):
        if st != 0:
            raise PicError(st, self.lib.pic_batch_last_error(self.h).decode())

    def add(self, ctx):
        self._check(self.lib.pic_batch_add(self.h, ctx.h))
        self.members.append(ctx)

    def remove(self, ctx):
        self._check(self.lib.pic_batch_remove(self.h, ctx.h))
        self.members.remove(ctx)

    def step(self, nsteps=1):
        self._check(self.lib.pic_batch_step(self.h, int(nsteps)))

    def set_graph(self, on=True):
        self._check(self.lib.pic_batch_set_graph(self.h, 1 if on else 0))

    def sync(self):
        self._check(self.lib.pic_batch_sync(self.h))

    def size(self):
        n = C.c_int32()
        self._check(self.lib.pic_batch_size(self.h, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.pic_batch_destroy(self.h)
            self.h = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_grid(grid, **kw) -> Context:
    return Context(grid, **kw)


# Every callback pair ever installed: contexts and batches keep calling the pair they were
# created with after another one is installed, so none may be released.
_hooks = []


def set_allocator(alloc=None, free=None):
    """pic_set_allocator with Python callables alloc(bytes, device) -> int address (0 when it
    cannot) and free(address, bytes, device); None for both restores hipMalloc / hipFree.
    Contexts and batches created afterwards use them."""
    lib = load_library()
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        st = lib.pic_set_allocator(C.cast(None, ALLOC_FN), C.cast(None, FREE_FN), None)
        if st != PIC_OK:
            raise PicError(st, lib.pic_last_error(None).decode())
        return

    def _a(nbytes, device, _user):
        try:
            return int(alloc(int(nbytes), int(device))) or None
        except Exception:
            return None

    def _f(ptr, nbytes, device, _user):
        free(int(ptr), int(nbytes), int(device))

    hooks = (ALLOC_FN(_a), FREE_FN(_f))
    _hooks.append(hooks)
    st = lib.pic_set_allocator(hooks[0], hooks[1], None)
    if st != PIC_OK:
        raise PicError(st, lib.pic_last_error(None).decode())


def use_torch_allocator():
    """Back the library's device memory with PyTorch's caching allocator (on torch's current
    stream of each device), so the library and torch share one pool."""
    import torch

    def alloc(nbytes, device):
        return torch.cuda.caching_allocator_alloc(nbytes, device=device)

    def free(ptr, nbytes, device):
        torch.cuda.caching_allocator_delete(ptr)

    set_allocator(alloc, free)
