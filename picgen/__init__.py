"""Seeded synthetic inputs for the implicit 2D3V particle-in-cell particle stage.

This module only *draws* inputs: grid and laser parameters of each workload, particle
positions (cell units) and momenta u = p/(m c).  It contains none of the method's
arithmetic (no shape functions, no mover, no field update), so the GPU library and the
CPU oracle can both be fed from it without sharing any computation.

Units follow the normalisation c = eps0 = mu0 = 1: time in 1/omega_r, length in c/omega_r,
momentum in m_s c, fields in m_e c omega_r / e, density in eps0 m_e omega_r^2 / e^2,
charge in e and mass in m_e.  omega_r is the plasma frequency for the uniform-plasma
workloads and the laser frequency omega_0 for the foil and low-density workloads.

Workload shapes follow the paper's two regimes (Sec. 4): a dense slab in an otherwise
empty box ("particle dominated") and a large grid with few particles per cell ("field
dominated").  The paper's own foil runs need its ionisation and material model, so these
synthetic inputs stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

ME_C2_KEV = 510.99895  # electron rest energy in keV
ION_MASS = 1836.0      # proton-to-electron mass ratio used by every workload

BC_PERIODIC = 0
BC_ABSORBING = 1
PREC_FP64 = 0
PREC_MIXED = 1

SEED_BASE = 13082590


@dataclass
class Grid:
    nx: int
    nz: int
    dx: float
    dz: float
    dt: float
    bc_x: int = BC_PERIODIC
    bc_z: int = BC_PERIODIC
    n_species: int = 2
    e0: tuple = (0.0, 0.0, 0.0)
    h0: tuple = (0.0, 0.0, 0.0)
    laser_a0: float = 0.0
    laser_omega: float = 1.0
    laser_sigma_z: float = 1.0
    laser_z_center: float = 0.0
    laser_fwhm_t: float = 1.0
    laser_t_center: float = 0.0
    allow_cfl_violation: int = 0
    precision: int = PREC_FP64

    @property
    def nodes_x(self) -> int:
        return self.nx + (1 if self.bc_x == BC_ABSORBING else 0)

    @property
    def nodes_z(self) -> int:
        return self.nz + (1 if self.bc_z == BC_ABSORBING else 0)

    @property
    def n_nodes(self) -> int:
        return self.nodes_x * self.nodes_z

    @property
    def n_cells(self) -> int:
        return self.nx * self.nz


@dataclass
class Species:
    q: float
    m: float
    w: object  # density carried by each macro-particle: one number, or one per particle
    xi_x: np.ndarray
    xi_z: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray

    @property
    def n(self) -> int:
        return int(self.xi_x.shape[0])

    def copy(self) -> "Species":
        w = self.w.copy() if isinstance(self.w, np.ndarray) else self.w
        return replace(self, w=w, xi_x=self.xi_x.copy(), xi_z=self.xi_z.copy(),
                       ux=self.ux.copy(), uy=self.uy.copy(), uz=self.uz.copy())


@dataclass
class Workload:
    name: str
    grid: Grid
    species: list
    steps: int
    note: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return sum(s.n for s in self.species)


def sigma_u(temperature_kev: float, mass: float) -> float:
    """Standard deviation of each momentum component of a Maxwellian, in units of m c."""
    return math.sqrt(temperature_kev / (mass * ME_C2_KEV))


def load_cells(rng, cells_i, cells_k, ppc, *, quiet=False):
    """Exactly ``ppc`` particles in each listed cell; offsets U[0,1)^2, or a centred lattice.

    Returns positions in cell units, ordered cell by cell in the order given.
    """
    cells_i = np.asarray(cells_i, dtype=np.int64).ravel()
    cells_k = np.asarray(cells_k, dtype=np.int64).ravel()
    nc = cells_i.shape[0]
    if quiet:
        side = int(round(math.sqrt(ppc)))
        if side * side != ppc:
            raise ValueError("quiet start needs a square number of particles per cell")
        lat = (np.arange(side) + 0.5) / side
        ox, oz = np.meshgrid(lat, lat, indexing="xy")
        ox = np.tile(ox.ravel(), nc)
        oz = np.tile(oz.ravel(), nc)
    else:
        ox = rng.random(nc * ppc)
        oz = rng.random(nc * ppc)
    xi_x = np.repeat(cells_i, ppc).astype(np.float64) + ox
    xi_z = np.repeat(cells_k, ppc).astype(np.float64) + oz
    return xi_x, xi_z


def make_species(rng, cells_i, cells_k, ppc, *, q, m, density, temperature_kev,
                 quiet=False, shuffle=False, drift=(0.0, 0.0, 0.0)):
    xi_x, xi_z = load_cells(rng, cells_i, cells_k, ppc, quiet=quiet)
    n = xi_x.shape[0]
    if temperature_kev > 0.0:
        s = sigma_u(temperature_kev, m)
        ux = rng.normal(0.0, s, n)
        uy = rng.normal(0.0, s, n)
        uz = rng.normal(0.0, s, n)
    else:
        ux = np.zeros(n)
        uy = np.zeros(n)
        uz = np.zeros(n)
    ux += drift[0]
    uy += drift[1]
    uz += drift[2]
    if shuffle:
        p = rng.permutation(n)
        xi_x, xi_z, ux, uy, uz = xi_x[p], xi_z[p], ux[p], uy[p], uz[p]
    w = density / ppc if ppc > 0 else 0.0
    return Species(q=q, m=m, w=w, xi_x=np.ascontiguousarray(xi_x), xi_z=np.ascontiguousarray(xi_z),
                   ux=np.ascontiguousarray(ux), uy=np.ascontiguousarray(uy),
                   uz=np.ascontiguousarray(uz))


def _all_cells(nx, nz):
    k, i = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    return i.ravel(), k.ravel()


def _slab_cells(nx, nz, i_lo, i_hi):
    k, i = np.meshgrid(np.arange(nz), np.arange(i_lo, i_hi), indexing="ij")
    return i.ravel(), k.ravel()


def _seed(config_id: int, species: int) -> int:
    return SEED_BASE + 100 * config_id + species


def uniform_plasma(variant="a", *, ppc=16, nx=64, nz=64, quiet=False, shuffle=True):
    """Uniform two-species periodic plasma in a uniform B_z (the 64x64 oracle-size case).

    variant "a": dx = dz = 0.05 c/omega_p, dt = 0.02/omega_p (Courant number 0.4);
    variant "b": dx = dz = 1.25, dt = 0.5 (keeps omega_p dt = 0.5);
    variant "literal": dx = 0.05, dt = 0.5, which violates dt <= min(dx, dz).
    Density 1, electrons Maxwellian at 1 keV, ions cold with m_i/m_e = 1836, B_z = 0.5, E = 0.
    """
    dx, dt, allow = {"a": (0.05, 0.02, 0), "b": (1.25, 0.5, 0), "literal": (0.05, 0.5, 1)}[variant]
    cid = 1
    ci, ck = _all_cells(nx, nz)
    el = make_species(np.random.Generator(np.random.PCG64(_seed(cid, 0))), ci, ck, ppc,
                      q=-1.0, m=1.0, density=1.0, temperature_kev=1.0, quiet=quiet, shuffle=shuffle)
    io = make_species(np.random.Generator(np.random.PCG64(_seed(cid, 1))), ci, ck, ppc,
                      q=1.0, m=ION_MASS, density=1.0, temperature_kev=0.0, quiet=quiet, shuffle=shuffle)
    g = Grid(nx=nx, nz=nz, dx=dx, dz=dx, dt=dt, h0=(0.0, 0.0, 0.5), allow_cfl_violation=allow)
    steps = 3 if variant == "literal" else 10
    return Workload(name=f"uniform{nx}x{nz}_{variant}", grid=g, species=[el, io], steps=steps,
                    note="uniform periodic plasma, n=1, ppc=%d/species, Te=1 keV, cold ions, Bz=0.5" % ppc)


FOIL_DX = math.pi / 20.0   # lambda_0 / 40 with omega_0 = 1
FOIL_DT = math.pi / 50.0   # 0.01 lambda_0 / c


def foil(*, slab_cells=40, density=100.0, ppc=64, nx=1024, nz=512, a0=5.0, sigma_cells=64,
         steps=500, precision=PREC_FP64, config_id=2, shuffle=False):
    """Particle-dominated foil: a dense slab centred in x, absorbing x, periodic z, laser at x = 0.

    Electrons Maxwellian at 1 keV, ions cold.  Grid spacing lambda_0/40 and time step
    0.01 lambda_0/c, as in the paper's runs (Sec. 4).  The laser is an E_y plane wave with a
    Gaussian transverse profile (sigma in cells) and a Gaussian temporal envelope of intensity
    FWHM 200 steps centred at 400 steps.
    """
    i_lo = nx // 2 - slab_cells // 2
    i_hi = i_lo + slab_cells
    ci, ck = _slab_cells(nx, nz, i_lo, i_hi)
    el = make_species(np.random.Generator(np.random.PCG64(_seed(config_id, 0))), ci, ck, ppc,
                      q=-1.0, m=1.0, density=density, temperature_kev=1.0, shuffle=shuffle)
    io = make_species(np.random.Generator(np.random.PCG64(_seed(config_id, 1))), ci, ck, ppc,
                      q=1.0, m=ION_MASS, density=density, temperature_kev=0.0, shuffle=shuffle)
    g = Grid(nx=nx, nz=nz, dx=FOIL_DX, dz=FOIL_DX, dt=FOIL_DT, bc_x=BC_ABSORBING, bc_z=BC_PERIODIC,
             laser_a0=a0, laser_omega=1.0, laser_sigma_z=sigma_cells * FOIL_DX,
             laser_z_center=0.5 * nz * FOIL_DX, laser_fwhm_t=200 * FOIL_DT,
             laser_t_center=400 * FOIL_DT, precision=precision)
    name = f"foil{nx}x{nz}_slab{slab_cells}_n{density:g}_ppc{ppc}"
    return Workload(name=name, grid=g, species=[el, io], steps=steps,
                    note=f"slab cells [{i_lo},{i_hi}) x all z, n={density:g} n_c, ppc={ppc}/species",
                    meta={"slab": (i_lo, i_hi), "ppc": ppc})


def low_density(*, nx=2048, nz=2048, ppc=4, density=0.1, a0=1.0, sigma_cells=256, steps=200,
                shuffle=False):
    """Field-dominated run: large grid, uniform low-density plasma, few particles per cell."""
    cid = 3
    ci, ck = _all_cells(nx, nz)
    el = make_species(np.random.Generator(np.random.PCG64(_seed(cid, 0))), ci, ck, ppc,
                      q=-1.0, m=1.0, density=density, temperature_kev=0.1, shuffle=shuffle)
    io = make_species(np.random.Generator(np.random.PCG64(_seed(cid, 1))), ci, ck, ppc,
                      q=1.0, m=ION_MASS, density=density, temperature_kev=0.0, shuffle=shuffle)
    g = Grid(nx=nx, nz=nz, dx=FOIL_DX, dz=FOIL_DX, dt=FOIL_DT, bc_x=BC_ABSORBING, bc_z=BC_PERIODIC,
             laser_a0=a0, laser_omega=1.0, laser_sigma_z=sigma_cells * FOIL_DX,
             laser_z_center=0.5 * nz * FOIL_DX, laser_fwhm_t=200 * FOIL_DT,
             laser_t_center=400 * FOIL_DT)
    return Workload(name=f"lowdensity{nx}x{nz}_ppc{ppc}", grid=g, species=[el, io], steps=steps,
                    note=f"uniform n={density:g} n_c, ppc={ppc}/species, Te=100 eV")


def named(name: str) -> Workload:
    """The workloads used by the tests and the benchmark, by name."""
    table = {
        "uniform64a": lambda: uniform_plasma("a"),
        "uniform64b": lambda: uniform_plasma("b"),
        "uniform64_literal": lambda: uniform_plasma("literal"),
        "foil": lambda: foil(),
        "foil_cm": lambda: foil(slab_cells=80),
        "lowdensity": lambda: low_density(),
        "foil_dense": lambda: foil(density=200.0, ppc=128, precision=PREC_MIXED, config_id=4),
        "foil_dense_cm": lambda: foil(slab_cells=160, density=200.0, ppc=128,
                                      precision=PREC_MIXED, config_id=4),
    }
    return table[name]()


def random_small(seed, *, nx=7, nz=5, ppc=3, bc_x=BC_PERIODIC, dx=0.5, dz=0.4, dt=0.3,
                 h0=(0.2, -0.3, 0.7), e0=(0.05, -0.02, 0.03), temps=(5.0, 0.5), density=(0.8, 0.8),
                 masses=(1.0, 25.0), charges=(-1.0, 1.0), shuffle=True, laser_a0=0.0):
    """Small irregular grids (ragged against any tile size) with random thermal species."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 7 * seed + 3))
    ci, ck = _all_cells(nx, nz)
    sp = []
    for s in range(len(masses)):
        sp.append(make_species(rng, ci, ck, ppc, q=charges[s], m=masses[s], density=density[s],
                               temperature_kev=temps[s], shuffle=shuffle))
    g = Grid(nx=nx, nz=nz, dx=dx, dz=dz, dt=dt, bc_x=bc_x, e0=e0, h0=h0, n_species=len(masses),
             laser_a0=laser_a0, laser_sigma_z=nz * dz / 4, laser_z_center=nz * dz / 2,
             laser_fwhm_t=20 * dt, laser_t_center=10 * dt)
    return Workload(name=f"random{nx}x{nz}_s{seed}", grid=g, species=sp, steps=5)


def random_fields(seed, grid: Grid, amp_e=0.1, amp_h=0.3):
    """Random E on nodes [3][nodes_z][nodes_x] and H at cell centres [3][nz][nx]."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 11 * seed + 5))
    e = amp_e * rng.standard_normal((3, grid.nodes_z, grid.nodes_x))
    h = amp_h * rng.standard_normal((3, grid.nz, grid.nx))
    return np.ascontiguousarray(e), np.ascontiguousarray(h)


def with_particle_densities(wl: Workload, seed: int, spread=(0.2, 2.0)) -> Workload:
    """Copy of a workload in which every particle carries its own density: the species'
    density times a factor drawn uniformly from ``spread`` (seeded)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 13 * seed + 7))
    out = []
    for sp in wl.species:
        c = sp.copy()
        c.w = float(np.mean(sp.w)) * rng.uniform(spread[0], spread[1], sp.n)
        out.append(c)
    return replace(wl, species=out, name=wl.name + "_pw")


def fp32_representable(wl: Workload) -> Workload:
    """Copy of a workload whose particle state is exactly representable in the mixed form:
    in-cell offsets and momenta rounded to the nearest float32 (an offset that rounds up to 1
    becomes the largest float32 below 1), so both precisions start from the same state."""
    out = []
    for sp in wl.species:
        c = sp.copy()
        for k in ("xi_x", "xi_z"):
            v = getattr(c, k)
            i = np.floor(v)
            f = (v - i).astype(np.float32)
            f = np.where(f >= np.float32(1.0), np.nextafter(np.float32(1.0), np.float32(0.0)), f)
            setattr(c, k, i + f.astype(np.float64))
        for k in ("ux", "uy", "uz"):
            setattr(c, k, getattr(c, k).astype(np.float32).astype(np.float64))
        if isinstance(c.w, np.ndarray):   # per-particle densities are stored as FP32 too
            c.w = c.w.astype(np.float32).astype(np.float64)
        out.append(c)
    return replace(wl, species=out, grid=replace(wl.grid, precision=PREC_MIXED))


@dataclass
class Request:
    """One run of a serving stream: its arrival time, the cycles it asks for, and the
    parameters its foil workload is drawn from."""
    rid: int
    arrival_s: float
    steps: int
    nx: int
    nz: int
    slab_cells: int
    density: float
    ppc: int
    a0: float
    seed: int


def serving_stream(n=256, rate_per_s=20.0, seed=5, *, nx_range=(32, 512), nz_range=(32, 512),
                   slab_frac=(0.05, 0.15), density_range=(10.0, 200.0), ppc_range=(8, 64),
                   a0_range=(0.5, 10.0), steps_range=(100, 1000)):
    """A stream of independent foil runs: Poisson arrivals (exponential gaps) at rate_per_s;
    grid sides log-uniform in nx_range / nz_range; slab width a uniform fraction of nx;
    density log-uniform; particles per cell and cycles uniform integers; a0 uniform."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 100 * 5 + seed))
    t = 0.0
    out = []
    for r in range(n):
        t += float(rng.exponential(1.0 / rate_per_s))
        nx = int(round(math.exp(rng.uniform(math.log(nx_range[0]), math.log(nx_range[1])))))
        nz = int(round(math.exp(rng.uniform(math.log(nz_range[0]), math.log(nz_range[1])))))
        slab = max(1, int(round(rng.uniform(*slab_frac) * nx)))
        dens = float(math.exp(rng.uniform(math.log(density_range[0]), math.log(density_range[1]))))
        ppc = int(rng.integers(ppc_range[0], ppc_range[1] + 1))
        a0 = float(rng.uniform(*a0_range))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        out.append(Request(rid=r, arrival_s=t, steps=steps, nx=nx, nz=nz, slab_cells=slab,
                           density=dens, ppc=ppc, a0=a0, seed=r))
    return out


def request_workload(req: Request, precision=PREC_MIXED) -> Workload:
    """The foil workload of one request: slab centred in x, laser sigma = nz / 8 cells."""
    nx, nz = req.nx, req.nz
    i_lo = nx // 2 - req.slab_cells // 2
    i_hi = i_lo + req.slab_cells
    ci, ck = _slab_cells(nx, nz, i_lo, i_hi)
    base = SEED_BASE + 100 * 5 + 1000 * (req.seed + 1)
    el = make_species(np.random.Generator(np.random.PCG64(base)), ci, ck, req.ppc,
                      q=-1.0, m=1.0, density=req.density, temperature_kev=1.0)
    io = make_species(np.random.Generator(np.random.PCG64(base + 1)), ci, ck, req.ppc,
                      q=1.0, m=ION_MASS, density=req.density, temperature_kev=0.0)
    g = Grid(nx=nx, nz=nz, dx=FOIL_DX, dz=FOIL_DX, dt=FOIL_DT, bc_x=BC_ABSORBING,
             bc_z=BC_PERIODIC, laser_a0=req.a0, laser_omega=1.0,
             laser_sigma_z=(nz / 8.0) * FOIL_DX, laser_z_center=0.5 * nz * FOIL_DX,
             laser_fwhm_t=200 * FOIL_DT, laser_t_center=400 * FOIL_DT, precision=precision)
    return Workload(name=f"req{req.rid}_{nx}x{nz}", grid=g, species=[el, io], steps=req.steps,
                    note=f"slab {req.slab_cells} cells, n={req.density:.1f}, ppc={req.ppc}, a0={req.a0:.2f}")
