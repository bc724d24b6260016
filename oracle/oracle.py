"""ctypes binding and cycle driver for the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.c")
LIB = os.path.join(HERE, "liborc.so")

PERIODIC = 0
ABSORBING = 1
GAMMA_PREDICT = 1   # mover option: gamma-bar = gamma(u^n + beta E^n) (reading R1's alternative)
B_BILINEAR = 2      # mover option: B interpolated from the four cell centres (R5's alternative)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, IEEE semantics."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("dx", C.c_double), ("dz", C.c_double),
                ("dt", C.c_double), ("bc_x", C.c_int32), ("bc_z", C.c_int32),
                ("n_species", C.c_int32), ("laser_a0", C.c_double), ("laser_omega", C.c_double),
                ("laser_sigma_z", C.c_double), ("laser_z_center", C.c_double),
                ("laser_fwhm_t", C.c_double), ("laser_t_center", C.c_double)]


class Species(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("n", C.c_int64),
                ("xi_x", C.c_void_p), ("xi_z", C.c_void_p), ("ux", C.c_void_p),
                ("uy", C.c_void_p), ("uz", C.c_void_p), ("w", C.c_void_p), ("id", C.c_void_p)]


_lib = None


def load_library():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB)
        P = C.c_void_p
        lib.orc_nodes_x.restype = C.c_int32
        lib.orc_nodes_z.restype = C.c_int32
        lib.orc_response.argtypes = [C.c_double, C.c_double, C.c_double, P, P, P, P]
        lib.orc_response_g.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, P, P]
        lib.orc_deposit.argtypes = [P, C.c_int32, P, P, P, C.c_int32, P]
        lib.orc_gather.argtypes = [P, P, C.c_int32, C.c_int64, P, P, P]
        lib.orc_particle_B.argtypes = [P, P, C.c_int32, C.c_int64, P, P, P]
        lib.orc_incident_ey.argtypes = [P, C.c_double, C.c_double, C.c_double]
        lib.orc_incident_ey.restype = C.c_double
        lib.orc_field_solve.argtypes = [P, C.c_double, P, P, P, P, P, P]
        lib.orc_push.argtypes = [P, P, P, P, P, C.c_int32, P]
        lib.orc_sort.argtypes = [P, P, P, P]
        lib.orc_sort.restype = C.c_int64
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_grid(g) -> Grid:
    """Oracle grid from any object with the grid attributes (nx, nz, dx, dz, dt, bc_x, ...)."""
    return Grid(nx=int(g.nx), nz=int(g.nz), dx=float(g.dx), dz=float(g.dz), dt=float(g.dt),
                bc_x=int(g.bc_x), bc_z=int(g.bc_z), n_species=int(g.n_species),
                laser_a0=float(g.laser_a0), laser_omega=float(g.laser_omega),
                laser_sigma_z=float(g.laser_sigma_z), laser_z_center=float(g.laser_z_center),
                laser_fwhm_t=float(g.laser_fwhm_t), laser_t_center=float(g.laser_t_center))


class _Sp:
    def __init__(self, q, m, xi_x, xi_z, ux, uy, uz, w, ids):
        self.q, self.m = float(q), float(m)
        f = lambda a: np.ascontiguousarray(np.array(a, dtype=np.float64, copy=True))
        self.xi_x, self.xi_z, self.ux, self.uy, self.uz, self.w = (
            f(xi_x), f(xi_z), f(ux), f(uy), f(uz), f(w))
        self.id = np.ascontiguousarray(np.array(ids, dtype=np.int64, copy=True))
        self.n = int(self.xi_x.shape[0])

    def struct(self) -> Species:
        return Species(q=self.q, m=self.m, n=self.n, xi_x=self.xi_x.ctypes.data,
                       xi_z=self.xi_z.ctypes.data, ux=self.ux.ctypes.data, uy=self.uy.ctypes.data,
                       uz=self.uz.ctypes.data, w=self.w.ctypes.data, id=self.id.ctypes.data)

    def truncate(self, n):
        self.n = int(n)
        for name in ("xi_x", "xi_z", "ux", "uy", "uz", "w", "id"):
            setattr(self, name, np.ascontiguousarray(getattr(self, name)[:n]))


class OracleSim:
    """One simulation held in numpy arrays, advanced by the C oracle.

    State after k cycles: positions x^{k+1/2} (cell units), momenta u^k, E^k on nodes,
    H^{k+1/2} at cell centres and t = k dt.  mode selects the mover options (GAMMA_PREDICT,
    B_BILINEAR; 0 = the defaults).
    """

    def __init__(self, grid, mode=0):
        self.mode = int(mode)
        self.lib = load_library()
        self.g = make_grid(grid)
        if self.g.bc_z != PERIODIC:
            raise ValueError("the oracle supports a periodic z axis only")
        self.nxn = self.lib.orc_nodes_x(C.byref(self.g))
        self.nzn = self.lib.orc_nodes_z(C.byref(self.g))
        self.S = int(self.g.n_species)
        e0 = getattr(grid, "e0", (0.0, 0.0, 0.0))
        h0 = getattr(grid, "h0", (0.0, 0.0, 0.0))
        self.E = np.zeros((3, self.nzn, self.nxn))
        self.H = np.zeros((3, self.g.nz, self.g.nx))
        for r in range(3):
            self.E[r] = e0[r]
            self.H[r] = h0[r]
        self.species = [None] * self.S
        self.t = 0.0
        self.step_count = 0
        self.absorbed = [0] * self.S

    # -- state set-up ---------------------------------------------------------------------
    def load_species(self, s, q, m, w, xi_x, xi_z, ux, uy, uz, ids=None):
        n = len(xi_x)
        wa = np.full(n, float(w)) if np.ndim(w) == 0 else w
        ids = np.arange(n, dtype=np.int64) if ids is None else ids
        sp = _Sp(q, m, xi_x, xi_z, ux, uy, uz, wa, ids)
        st = sp.struct()
        n_new = self.lib.orc_sort(C.byref(self.g), C.byref(st), None, None)
        sp.truncate(n_new)
        self.species[s] = sp
        self.absorbed[s] = 0

    def load_fields(self, E, H):
        self.E = np.ascontiguousarray(np.array(E, dtype=np.float64).reshape(3, self.nzn, self.nxn))
        self.H = np.ascontiguousarray(np.array(H, dtype=np.float64).reshape(3, self.g.nz, self.g.nx))

    # -- the pieces of one cycle ----------------------------------------------------------
    def moments(self, H=None, E=None):
        """M^{k+1/2}: S-hat (9), delta-j (3) and S densities on the nodes."""
        H = self.H if H is None else H
        E = self.E if E is None else E
        M = np.zeros((12 + self.S, self.nzn, self.nxn))
        for s, sp in enumerate(self.species):
            if sp is None or sp.n == 0:
                continue
            st = sp.struct()
            self.lib.orc_deposit(C.byref(self.g), s, C.byref(st), _ptr(np.ascontiguousarray(H)),
                                 _ptr(np.ascontiguousarray(E)), self.mode, _ptr(M))
        return M

    def field_solve(self, M):
        E_new = np.zeros_like(self.E)
        Ebar = np.zeros_like(self.E)
        H_new = np.zeros_like(self.H)
        self.lib.orc_field_solve(C.byref(self.g), self.t, _ptr(M), _ptr(self.E), _ptr(self.H),
                                 _ptr(E_new), _ptr(Ebar), _ptr(H_new))
        return E_new, Ebar, H_new

    def push(self, s, Ebar, H, E=None):
        sp = self.species[s]
        E = self.E if E is None else E
        alive = np.ones(sp.n, dtype=np.uint8)
        st = sp.struct()
        self.lib.orc_push(C.byref(self.g), C.byref(st), _ptr(np.ascontiguousarray(Ebar)),
                          _ptr(np.ascontiguousarray(H)), _ptr(np.ascontiguousarray(E)), self.mode,
                          _ptr(alive))
        return alive

    def sort(self, s, alive=None):
        sp = self.species[s]
        st = sp.struct()
        perm = np.zeros(max(sp.n, 1), dtype=np.int64)
        n_new = self.lib.orc_sort(C.byref(self.g), C.byref(st), _ptr(alive), _ptr(perm))
        self.absorbed[s] += sp.n - n_new
        sp.truncate(n_new)
        return perm[:n_new]

    def step(self, nsteps=1):
        for _ in range(nsteps):
            M = self.moments()
            E_new, Ebar, H_new = self.field_solve(M)
            for s, sp in enumerate(self.species):
                if sp is None:
                    continue
                alive = self.push(s, Ebar, self.H)
                self.sort(s, alive)
            self.E, self.H = E_new, H_new
            self.t += self.g.dt
            self.step_count += 1

    # -- read-back ------------------------------------------------------------------------
    def particles(self, s):
        sp = self.species[s]
        return {"xi_x": sp.xi_x.copy(), "xi_z": sp.xi_z.copy(), "ux": sp.ux.copy(),
                "uy": sp.uy.copy(), "uz": sp.uz.copy(), "w": sp.w.copy(), "id": sp.id.copy()}

    def gather(self, F, xi_x, xi_z):
        F = np.ascontiguousarray(F, dtype=np.float64)
        ncomp = F.shape[0]
        n = len(xi_x)
        out = np.zeros((ncomp, n))
        self.lib.orc_gather(C.byref(self.g), _ptr(F), ncomp, n,
                            _ptr(np.ascontiguousarray(xi_x, dtype=np.float64)),
                            _ptr(np.ascontiguousarray(xi_z, dtype=np.float64)), _ptr(out))
        return out

    def particle_B(self, H, xi_x, xi_z, mode=None):
        """B at the given positions as the mover sees it (this simulation's mode by default)."""
        H = np.ascontiguousarray(H, dtype=np.float64)
        n = len(xi_x)
        out = np.zeros((3, n))
        self.lib.orc_particle_B(C.byref(self.g), _ptr(H), self.mode if mode is None else int(mode),
                                n, _ptr(np.ascontiguousarray(xi_x, dtype=np.float64)),
                                _ptr(np.ascontiguousarray(xi_z, dtype=np.float64)), _ptr(out))
        return out

    def energy(self):
        """Energies of the current state (the plain definitions): [field, kinetic of species
        0, 1, ...] with field = (1/2)(sum over nodes of |E^k|^2 + sum over cells of
        |H^{k+1/2}|^2) dx dz and kinetic = sum over particles of w m (gamma(u^k) - 1) dx dz."""
        area = float(self.g.dx) * float(self.g.dz)
        out = [0.5 * (float(np.sum(self.E * self.E)) + float(np.sum(self.H * self.H))) * area]
        for sp in self.species:
            if sp is None or sp.n == 0:
                out.append(0.0)
                continue
            gam = np.sqrt(1.0 + sp.ux * sp.ux + sp.uy * sp.uy + sp.uz * sp.uz)
            out.append(float(np.sum(sp.w * sp.m * (gam - 1.0))) * area)
        return out

    def incident_ey(self, t, x, z):
        return self.lib.orc_incident_ey(C.byref(self.g), float(t), float(x), float(z))


def response_g(q, m, dt, gamma, B):
    """R of one particle for a given gamma-bar (exposed for the tests)."""
    lib = load_library()
    B = np.ascontiguousarray(B, dtype=np.float64)
    R = np.zeros(9)
    lib.orc_response_g(float(q), float(m), float(dt), float(gamma), _ptr(B), _ptr(R))
    return R.reshape(3, 3)


def response(q, m, dt, u, B):
    """R and gamma-bar of one particle (exposed for the tests)."""
    lib = load_library()
    u = np.ascontiguousarray(u, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    R = np.zeros(9)
    gam = C.c_double(0.0)
    lib.orc_response(float(q), float(m), float(dt), _ptr(u), _ptr(B), _ptr(R), C.byref(gam))
    return R.reshape(3, 3), gam.value
