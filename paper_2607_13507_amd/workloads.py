"""Seeded synthetic inputs for the PIC hot path.

This module only draws random numbers and lays out particle lists and initial fields; it
holds none of the method's arithmetic (no shape function, push, deposit or field solve), so
both the HIP path and the FP64 oracle can take their inputs from it.

Units are normalised (c = eps0 = m_e = e = 1); for laser workloads the reference frequency
is the laser's, so the wavelength is 2*pi, the critical density is 1 and a0 is the peak
field.  A macro-particle carries the weight w = n / ppc (a density), positions are absolute
FP64 coordinates, momenta are u = gamma v.

Recipes (configuration names follow the workloads they model):
  thermal_2d      2D3V periodic uniform electron plasma on a fixed ion background,
                  Gaussian momenta sigma = sqrt(T/m) per component, random in-cell positions
  laser_slab_2d   2D3V fully ionised hydrogen slab (electrons + protons) with a linearly
                  polarised Gaussian pulse initialised in the vacuum region in front of it
  thermal_3d      3D3V periodic uniform electron plasma on a fixed ion background
  ensemble_2d     many independent laser-slab runs of mixed sizes drawn from one seed
  wakefield_2d    underdense electron plasma filling a long box, fixed ions, Gaussian pulse
  cold_langmuir   cold electron lattice with a sinusoidal velocity perturbation
  vacuum_mode     one Fourier mode of the vacuum field, no particles
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

M_PROTON = 1836.15267343
LAMBDA = 2.0 * math.pi          # laser wavelength in units of c / omega_L
T_1KEV = 1.0 / 510.99895        # 1 keV in units of m_e c^2


@dataclass
class SpeciesInit:
    name: str
    q: float
    m: float
    order: int                  # 1 = CIC, 2 = quadratic
    x: np.ndarray
    y: np.ndarray
    z: Optional[np.ndarray]
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    w: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Workload:
    name: str
    ndim: int
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    dt: float
    rho_bg: float
    species: List[SpeciesInit]
    fields: Dict[str, np.ndarray] = field(default_factory=dict)   # initial E, B (flat, x fastest)
    steps: int = 1
    meta: dict = field(default_factory=dict)
    open_x: bool = False                  # open (absorbing) x ends instead of periodic
    laser: Optional[dict] = None          # antenna: pol, ia, a0, omega, waist, yc, zc, t0, tau
    pml: Optional[dict] = None            # open x ends: CPML layers (cells, order, sigma_max,
                                          # kappa_max, a_max) instead of the Mur condition

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * (self.nz if self.ndim == 3 else 1)

    @property
    def nparticles(self) -> int:
        return sum(s.n for s in self.species)

    def box(self):
        return (self.nx * self.dx, self.ny * self.dy, self.nz * self.dz)


def cfl_dt(eta: float, *h: float) -> float:
    """Time step eta / (c sqrt(sum h^-2)), the CFL form stated in Sec. 3.2."""
    return eta / math.sqrt(sum(1.0 / (v * v) for v in h))


# ----------------------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------------------
def _random_in_cells(rng, cells_x, cells_y, cells_z, ppc, dx, dy, dz):
    """ppc particles uniformly at random inside each listed cell (C-order cell lists)."""
    nc = cells_x.shape[0]

    def axis(cells, h):
        v = rng.random(nc * ppc)
        v.reshape(nc, ppc)[...] += cells.astype(np.float64)[:, None]
        v *= h
        return v

    x = axis(cells_x, dx)
    y = axis(cells_y, dy)
    z = axis(cells_z, dz) if cells_z is not None else None
    # a draw of exactly 1.0 cannot happen (rng.random is in [0, 1)), but rounding of
    # (i + r) * dx at the top cell can reach the box edge: fold it back
    return x, y, z


def _cell_lists_2d(x0, x1, y0, y1):
    jj, ii = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
    return ii.reshape(-1), jj.reshape(-1)


def _thermal_species(rng, name, q, m, order, x, y, z, T, density, ppc):
    n = x.shape[0]
    sig = math.sqrt(T / m) if T > 0 else 0.0
    ux = rng.normal(0.0, sig, n) if sig > 0 else np.zeros(n)
    uy = rng.normal(0.0, sig, n) if sig > 0 else np.zeros(n)
    uz = rng.normal(0.0, sig, n) if sig > 0 else np.zeros(n)
    w = np.full(n, density / ppc)
    return SpeciesInit(name, q, m, order, x, y, z, ux, uy, uz, w)


def _fold(a, L):
    a = np.where(a >= L, a - L, a)
    return np.where(a < 0, a + L, a)


def gaussian_pulse_fields(nx, ny, dx, dy, a0, x_lo, x_hi, waist, y_centre):
    """Linearly polarised (E mostly along y) pulse moving in +x, laid out on the Yee stagger
    with a discretely divergence-free E.  With the profile
        f(x, y) = a0 sin^2(pi (x - x_lo)/(x_hi - x_lo)) exp(-((y - yc)/waist)^2)
    (zero outside [x_lo, x_hi)), a stream function psi = f cos(x) sits at the Bz points
    (i+1/2, j+1/2); Ey = -d psi/dx and Ex = d psi/dy are its one-cell differences, so the
    discrete div E vanishes at every node and Ey ~ f sin(x).  Bz = f sin(x) at its own
    points (B has only a z component in this 2D layout, so div B = 0 as well)."""
    def env(xs, ys):
        inside = (xs >= x_lo) & (xs < x_hi)
        e = np.where(inside, np.sin(math.pi * (xs - x_lo) / (x_hi - x_lo)) ** 2, 0.0)
        return a0 * e * np.exp(-((ys - y_centre) / waist) ** 2)

    i = np.arange(nx)
    j = np.arange(ny)
    Y, X = np.meshgrid((j + 0.5) * dy, (i + 0.5) * dx, indexing="ij")   # Bz points [j, i]
    f = env(X, Y)
    psi = f * np.cos(X)
    bz = f * np.sin(X)
    # Ey at (i, j+1/2): -(psi[i+1/2] - psi[i-1/2]) / dx;  Ex at (i+1/2, j): (psi[j+1/2] -
    # psi[j-1/2]) / dy, with periodic neighbours
    ey = -(psi - np.roll(psi, 1, axis=1)) / dx
    ex = (psi - np.roll(psi, 1, axis=0)) / dy
    return {"ex": ex.reshape(-1), "ey": ey.reshape(-1), "bz": bz.reshape(-1)}


# ----------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------
def thermal_2d(nx=64, ny=64, dx=0.05, ppc=16, T=0.01, density=1.0, order=1, seed=1,
               eta=0.95, steps=100, name="thermal_2d") -> Workload:
    """2D3V periodic uniform electrons on a fixed neutralising ion background (defaults:
    64x64, dx = dy = 0.05 c/omega_p, 16 ppc, T = 0.01 m c^2, CIC, 100 steps)."""
    rng = np.random.default_rng(seed)
    cx, cy = _cell_lists_2d(0, nx, 0, ny)
    x, y, _ = _random_in_cells(rng, cx, cy, None, ppc, dx, dx, None)
    x, y = _fold(x, nx * dx), _fold(y, ny * dx)
    e = _thermal_species(rng, "electron", -1.0, 1.0, order, x, y, None, T, density, ppc)
    dt = cfl_dt(eta, dx, dx)
    return Workload(name, 2, nx, ny, 1, dx, dx, 1.0, dt, +density, [e], {}, steps,
                    dict(ppc=ppc, T=T, density=density, order=order, seed=seed))


def laser_slab_2d(nx=2048, ny=1024, cells_per_lambda=32, slab=(512, 768), density=20.0,
                  ppc=32, T=T_1KEV, a0=10.0, order=2, seed=2, eta=0.95, steps=2000,
                  pulse_cells=None, waist_lambda=6.25, inject=True, duration_lambda=25.0,
                  pml_cells=0, name="laser_slab_2d") -> Workload:
    """2D3V hydrogen slab (electrons + protons, `ppc` each) of `density` n_c in cells
    [slab[0], slab[1]) over the whole y extent, and a linearly polarised (E along y)
    Gaussian laser of peak a0, waist `waist_lambda` wavelengths.
    inject=True: open x ends and a laser antenna 4 cells from the left end, sin^2 envelope
    of full duration `duration_lambda` wavelengths (the setup of Sec. 4.2); y periodic.
    pml_cells > 0 (with inject): graded PML layers of that many cells at both x ends
    instead of the Mur condition, the antenna 4 cells inside the left layer's inner face.
    inject=False: periodic box with the pulse placed in the vacuum in front of the slab
    (x in [0, pulse_cells) cells, sin^2 envelope over that span).
    Electrons sit uniformly at random in their cells, each proton on an electron, so the
    plasma starts neutral node by node; momenta are drawn independently per species."""
    rng = np.random.default_rng(seed)
    dx = LAMBDA / cells_per_lambda
    cx, cy = _cell_lists_2d(slab[0], slab[1], 0, ny)
    xs, ys, _ = _random_in_cells(rng, cx, cy, None, ppc, dx, dx, None)
    xs, ys = _fold(xs, nx * dx), _fold(ys, ny * dx)
    e = _thermal_species(rng, "electron", -1.0, 1.0, order, xs, ys, None, T, density, ppc)
    # each proton starts on an electron: zero net charge at every node at t = 0
    p = _thermal_species(rng, "proton", +1.0, M_PROTON, order, xs.copy(), ys.copy(), None, T,
                         density, ppc)
    dt = cfl_dt(eta, dx, dx)
    if inject:
        laser = dict(pol=1, ia=pml_cells + 4, a0=a0, omega=1.0, waist=waist_lambda * LAMBDA,
                     yc=0.5 * ny * dx, zc=0.0, t0=0.0, tau=duration_lambda * LAMBDA)
        return Workload(name, 2, nx, ny, 1, dx, dx, 1.0, dt, 0.0, [e, p], {}, steps,
                        dict(ppc=ppc, T=T, density=density, order=order, seed=seed, a0=a0,
                             slab=slab, inject=True, pml_cells=pml_cells), open_x=True,
                        laser=laser, pml=dict(cells=pml_cells) if pml_cells else None)
    if pulse_cells is None:
        pulse_cells = min(slab[0], nx)
    flds = {}
    if a0 > 0 and pulse_cells > 0:
        flds = gaussian_pulse_fields(nx, ny, dx, dx, a0, 0.0, pulse_cells * dx,
                                     waist_lambda * LAMBDA, 0.5 * ny * dx)
    return Workload(name, 2, nx, ny, 1, dx, dx, 1.0, dt, 0.0, [e, p], flds, steps,
                    dict(ppc=ppc, T=T, density=density, order=order, seed=seed, a0=a0,
                         slab=slab, pulse_cells=pulse_cells, inject=False))


def thermal_3d(n=256, dx=0.1, ppc=8, T=0.05, density=1.0, order=2, seed=3, eta=0.95,
               steps=200, name="thermal_3d") -> Workload:
    """3D3V periodic uniform electrons on a fixed ion background (defaults 256^3, 8 ppc,
    T = 0.05 m c^2, quadratic)."""
    rng = np.random.default_rng(seed)
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    x, y, z = _random_in_cells(rng, ii.reshape(-1), jj.reshape(-1), kk.reshape(-1), ppc,
                               dx, dx, dx)
    L = n * dx
    x, y, z = _fold(x, L), _fold(y, L), _fold(z, L)
    e = _thermal_species(rng, "electron", -1.0, 1.0, order, x, y, z, T, density, ppc)
    dt = cfl_dt(eta, dx, dx, dx)
    return Workload(name, 3, n, n, n, dx, dx, dx, dt, +density, [e], {}, steps,
                    dict(ppc=ppc, T=T, density=density, order=order, seed=seed))


def ensemble_2d(seed=4, members=64, max_scale=1, sizes_x=(128, 256, 512, 1024),
                sizes_y=(128, 256, 512), cells_per_lambda=32, eta=0.95, steps=20):
    """Independent 2D3V laser-slab runs drawn from one seed: nx >= ny from the listed sizes,
    ppc per species from {4, 8, 16, 32}, slab density log-uniform in [0.1, 10] n_c filling
    the right half (up to 8 cells from the open right end), a0 log-uniform in [0.5, 20]
    injected from the left, CIC or quadratic with probability 1/2.  All members share
    dx = lambda/32 and hence dt."""
    rng = np.random.default_rng(seed)
    params = []
    for r in range(members):
        while True:
            nx = int(rng.choice(sizes_x))
            ny = int(rng.choice(sizes_y))
            if nx >= ny:
                break
        nx //= max_scale
        ny //= max_scale
        ppc = int(rng.choice([4, 8, 16, 32]))
        dens = float(10 ** rng.uniform(-1, 1))
        a0 = float(10 ** rng.uniform(math.log10(0.5), math.log10(20)))
        order = int(rng.choice([1, 2]))
        sub = int(rng.integers(0, 2 ** 31 - 1))
        params.append(dict(nx=nx, ny=ny, cells_per_lambda=cells_per_lambda,
                           slab=(nx // 2, nx - 8), density=dens, ppc=ppc, a0=a0, order=order,
                           seed=sub, eta=eta, steps=steps, pulse_cells=nx // 2,
                           waist_lambda=min(6.25, 0.2 * ny / cells_per_lambda),
                           name=f"ensemble_member_{r}"))
    return [laser_slab_2d(**kw) for kw in params]


def wakefield_2d(nx=8192, ny=512, cells_per_lambda=40, density=0.01, ppc=4, a0=2.0,
                 waist_lambda=8.0, order=2, seed=5, eta=0.95, steps=20000, T=0.0,
                 pulse_cells=None, moving=False, spare=1 << 20,
                 name="wakefield_2d") -> Workload:
    """Underdense electrons (fixed ions) filling the box ahead of an in-box Gaussian pulse.

    moving=False: a static periodic box, electrons random in their cells.
    moving=True: the box has open x ends and is meant to move with the pulse at c
    (meta["window"]: cells per step and the plasma to inject at the leading edge); the
    electrons sit on a sqrt(ppc) x sqrt(ppc) lattice in every cell, as the injected plasma
    will, and `spare` dead slots follow them for the injected particles."""
    rng = np.random.default_rng(seed)
    dx = LAMBDA / cells_per_lambda
    if pulse_cells is None:
        pulse_cells = min(nx // 4, 20 * cells_per_lambda)
    dt = cfl_dt(eta, dx, dx)
    meta = dict(ppc=ppc, density=density, order=order, seed=seed, a0=a0)
    if moving:
        side = int(round(math.sqrt(ppc)))
        assert side * side == ppc, "a moving window injects a square lattice"
        lo, hi = max(pulse_cells, 3), nx - 3          # between the open ends' margins
        cx, cy = _cell_lists_2d(lo, hi, 0, ny)
        sub = (np.arange(side) + 0.5) / side
        oy, ox = np.meshgrid(sub, sub, indexing="ij")
        xs = ((cx[:, None] + ox.reshape(1, -1)) * dx).reshape(-1)
        ys = ((cy[:, None] + oy.reshape(1, -1)) * dx).reshape(-1)
        dead = np.full(spare, -1.0)
        xs, ys = np.concatenate([xs, dead]), np.concatenate([ys, dead])
        e = _thermal_species(rng, "electron", -1.0, 1.0, order, xs, ys, None, T, density, ppc)
        e.w[-spare:] = 0.0
        meta["window"] = dict(cells_per_step=dt / dx,
                              plasma=dict(species=0, ppc_x=side, ppc_y=side, density=density))
    else:
        cx, cy = _cell_lists_2d(pulse_cells, nx, 0, ny)
        xs, ys, _ = _random_in_cells(rng, cx, cy, None, ppc, dx, dx, None)
        xs, ys = _fold(xs, nx * dx), _fold(ys, ny * dx)
        e = _thermal_species(rng, "electron", -1.0, 1.0, order, xs, ys, None, T, density, ppc)
    flds = gaussian_pulse_fields(nx, ny, dx, dx, a0, 0.0, pulse_cells * dx,
                                 waist_lambda * LAMBDA, 0.5 * ny * dx)
    return Workload(name, 2, nx, ny, 1, dx, dx, 1.0, dt, +density, [e], flds, steps, meta,
                    open_x=moving)


def cold_langmuir(nx=64, ny=64, dx=0.05, lattice=4, amp=1e-3, order=1, eta=0.95, steps=1000,
                  density=1.0, name="cold_langmuir") -> Workload:
    """Cold electron lattice (lattice x lattice per cell, at sub-cell centres) on a fixed
    ion background with u_x = amp sin(2 pi x / L)."""
    cx, cy = _cell_lists_2d(0, nx, 0, ny)
    sub = (np.arange(lattice) + 0.5) / lattice
    oy, ox = np.meshgrid(sub, sub, indexing="ij")
    ox = ox.reshape(-1)
    oy = oy.reshape(-1)
    ppc = lattice * lattice
    x = (np.repeat(cx, ppc) + np.tile(ox, cx.shape[0])) * dx
    y = (np.repeat(cy, ppc) + np.tile(oy, cy.shape[0])) * dx
    L = nx * dx
    n = x.shape[0]
    ux = amp * np.sin(2 * math.pi * x / L)
    e = SpeciesInit("electron", -1.0, 1.0, order, x, y, None, ux, np.zeros(n), np.zeros(n),
                    np.full(n, density / ppc))
    dt = cfl_dt(eta, dx, dx)
    return Workload(name, 2, nx, ny, 1, dx, dx, 1.0, dt, +density, [e], {}, steps,
                    dict(amp=amp, lattice=lattice, order=order))


def vacuum_mode(nx=64, ny=64, dx=0.05, mx=1, my=1, amp=1.0, eta=0.95, steps=1000,
                name="vacuum_mode") -> Workload:
    """Standing mode Ez = amp cos(kx x) cos(ky y), B = 0 (kx = 2 pi mx / Lx, same in y)."""
    L = nx * dx
    kx = 2 * math.pi * mx / L
    ky = 2 * math.pi * my / (ny * dx)
    Y, X = np.meshgrid(np.arange(ny) * dx, np.arange(nx) * dx, indexing="ij")
    ez = amp * np.cos(kx * X) * np.cos(ky * Y)
    dt = cfl_dt(eta, dx, dx)
    return Workload(name, 2, nx, ny, 1, dx, dx, 1.0, dt, 0.0, [], {"ez": ez.reshape(-1)},
                    steps, dict(kx=kx, ky=ky, amp=amp))


def gaussian_pulse_vacuum(nx=2048, ny=1024, cells_per_lambda=32, a0=10.0, steps=1000,
                          eta=0.95, name="pulse_vacuum") -> Workload:
    """Vacuum Gaussian pulse on the laser-slab grid (no particles)."""
    dx = LAMBDA / cells_per_lambda
    flds = gaussian_pulse_fields(nx, ny, dx, dx, a0, 0.0, min(nx, 16 * cells_per_lambda) * dx,
                                 6.25 * LAMBDA, 0.5 * ny * dx)
    dt = cfl_dt(eta, dx, dx)
    return Workload(name, 2, nx, ny, 1, dx, dx, 1.0, dt, 0.0, [], flds, steps, dict(a0=a0))


def random_fields(ncell, seed, scale=1.0, names=("ex", "ey", "ez", "bx", "by", "bz")):
    """Uniform random field values in [-scale, scale) for unit-level kernel checks."""
    rng = np.random.default_rng(seed)
    return {k: scale * (2 * rng.random(ncell) - 1) for k in names}


def deterministic_ensemble(steps=1000):
    """Independent 2D boxes of mixed sizes whose evolution is deterministic (no thermal
    noise): vacuum standing modes, a vacuum Gaussian pulse, and cold electron lattices
    (CIC and quadratic) on fixed ions with a velocity perturbation along x or y."""
    members = [
        vacuum_mode(nx=64, ny=64, dx=0.05, mx=2, my=1, steps=steps, name="ens_vacuum_64x64"),
        vacuum_mode(nx=48, ny=32, dx=0.05, mx=1, my=2, amp=0.5, steps=steps,
                    name="ens_vacuum_48x32"),
        gaussian_pulse_vacuum(nx=256, ny=64, cells_per_lambda=32, a0=2.0, steps=steps,
                              name="ens_pulse_256x64"),
        cold_langmuir(nx=64, ny=16, dx=0.05, lattice=4, amp=1e-2, order=1, steps=steps,
                      name="ens_cold_cic_64x16"),
        cold_langmuir(nx=32, ny=32, dx=0.05, lattice=2, amp=2e-2, order=2, steps=steps,
                      name="ens_cold_quad_32x32"),
        cold_langmuir(nx=128, ny=16, dx=0.05, lattice=2, amp=5e-3, order=2, steps=steps,
                      name="ens_cold_quad_128x16"),
    ]
    # the last lattice oscillates along y instead of x: same plasma, axes exchanged in u
    s = members[-1].species[0]
    s.ux, s.uy = np.zeros_like(s.ux), 5e-3 * np.sin(2 * math.pi * s.y / (16 * 0.05))
    members[-1].meta["perturbed_axis"] = "y"
    return members


def _directions(rng, n):
    """n isotropic unit vectors."""
    v = rng.normal(size=(3, n))
    return v / np.linalg.norm(v, axis=0)


def qed_beam(ndim=2, n=24, dx=0.1, ppc=1, gamma=(500.0, 2000.0), b0=300.0, noise=0.2,
             order=2, seed=7, eta=0.95, name="qed_beam") -> Workload:
    """Electrons of Lorentz factor uniform in `gamma` with isotropic directions in a strong
    uniform magnetic field b0 (along z) with a random perturbation of relative size `noise`
    on every E and B component: quantum parameters ~0.1-3 at hbar_omega ~ 2e-6, the
    regime where the emission of Sec. 3.4 happens within a few steps."""
    rng = np.random.default_rng(seed)
    if ndim == 2:
        cx, cy = _cell_lists_2d(0, n, 0, n)
        cz, nz = None, 1
    else:
        kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        cx, cy, cz, nz = ii.reshape(-1), jj.reshape(-1), kk.reshape(-1), n
    x, y, z = _random_in_cells(rng, cx, cy, cz, ppc, dx, dx, dx)
    L = n * dx
    x, y = _fold(x, L), _fold(y, L)
    z = _fold(z, L) if z is not None else None
    m = x.shape[0]
    g = rng.uniform(gamma[0], gamma[1], m)
    u = _directions(rng, m) * np.sqrt(g * g - 1.0)
    e = SpeciesInit("electron", -1.0, 1.0, order, x, y, z, u[0], u[1], u[2],
                    rng.uniform(0.5, 1.5, m))
    ncell = n * n * nz
    f = random_fields(ncell, seed + 1, noise * b0)
    f["bz"] = f["bz"] + b0
    dt = cfl_dt(eta, dx, dx) if ndim == 2 else cfl_dt(eta, dx, dx, dx)
    return Workload(name, ndim, n, n, nz, dx, dx, dx if ndim == 3 else 1.0, dt, 0.0, [e], f, 1,
                    dict(ppc=ppc, gamma=gamma, b0=b0, noise=noise, order=order, seed=seed))


def qed_photons(wl: Workload, n, k=(1000.0, 4000.0), seed=9):
    """n photons spread over the box of wl cell by cell in storage order (as photons emitted
    by tile-sorted leptons lie), with momenta |k| uniform in `k` (units of m c) and isotropic
    directions: positions x, y, z, momenta kx, ky, kz and weights."""
    rng = np.random.default_rng(seed)
    ncell = wl.ncell
    cell = (np.arange(n, dtype=np.int64) * ncell) // n        # non-decreasing cell index
    ix = cell % wl.nx
    iy = (cell // wl.nx) % wl.ny
    iz = cell // (wl.nx * wl.ny)
    pos = [(ix + rng.random(n)) * wl.dx, (iy + rng.random(n)) * wl.dy,
           (iz + rng.random(n)) * wl.dz if wl.ndim == 3 else np.zeros(n)]
    Lx, Ly, Lz = wl.box()
    pos = [_fold(pos[0], Lx), _fold(pos[1], Ly), _fold(pos[2], Lz) if wl.ndim == 3 else pos[2]]
    kv = _directions(rng, n) * rng.uniform(k[0], k[1], n)
    return pos, kv, rng.uniform(0.5, 1.5, n)
