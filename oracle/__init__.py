"""Plain FP64 CPU oracle of the lambda-PIC timestep (arXiv 2607.13507).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It wraps ``oracle.c``
(plain C, FP64, single threaded) through ctypes and shares no code with the HIP library.

Parity status of every function is recorded in the test suite (``tests/test_oracle_pins.py``):
each is pinned by a closed form, an invariant or a brute-force case, except the laser-plasma
physics of the large workloads, which is pinned only through continuity, the Gauss invariant
and energy balance.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_SRCS = (_SRC, os.path.join(_HERE, "qed.c"))

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile oracle.c and qed.c with gcc (IEEE semantics: no fast-math)."""
    if force or not os.path.exists(_SO):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fopenmp", "-shared", "-fPIC",
                               "-o", _SO + ".tmp", *_SRCS, "-lm"])
        os.replace(_SO + ".tmp", _SO)
    return _SO


class Pml(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int32), ("order", ctypes.c_int32),
                ("a_order", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("sigma_max", ctypes.c_double), ("kappa_max", ctypes.c_double),
                ("a_max", ctypes.c_double), ("psi", _dp)]


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dz", ctypes.c_double), ("dt", ctypes.c_double), ("rho_bg", ctypes.c_double),
                ("open_x", ctypes.c_int32), ("pml", ctypes.POINTER(Pml))]


def pml_defaults(pml, dx):
    """The layer parameters with their defaults filled in: order 3, a_order 1, sigma_max =
    0.8 (m + 1) / dx (the usual choice for a graded layer, normalised impedance 1),
    kappa_max 1, a_max 0."""
    m = int(pml.get("order", 3))
    sigma = pml.get("sigma_max")
    return dict(cells=int(pml["cells"]), order=m, a_order=int(pml.get("a_order", 1)),
                sigma_max=float(0.8 * (m + 1) / dx if sigma is None or sigma < 0 else sigma),
                kappa_max=float(pml.get("kappa_max", 1.0)), a_max=float(pml.get("a_max", 0.0)))


class Laser(ctypes.Structure):
    _fields_ = [("pol", ctypes.c_int32), ("ia", ctypes.c_int32), ("a0", ctypes.c_double),
                ("omega", ctypes.c_double), ("waist", ctypes.c_double), ("yc", ctypes.c_double),
                ("zc", ctypes.c_double), ("t0", ctypes.c_double), ("tau", ctypes.c_double)]


OPEN_MARGIN = 3   # cells at each open x end where particles are removed (oracle.h)


class Fields(ctypes.Structure):
    _fields_ = [(n, _dp) for n in ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz",
                                   "rho0", "rho1")]


class Species(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("q", ctypes.c_double), ("m", ctypes.c_double),
                ("order", ctypes.c_int32), ("x", _dp), ("y", _dp), ("z", _dp),
                ("ux", _dp), ("uy", _dp), ("uz", _dp), ("w", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(f)
                                          for f in _SRCS):
            build()
        L = ctypes.CDLL(_SO)
        L.orc_shape.restype = ctypes.c_double
        L.orc_shape.argtypes = [ctypes.c_int32, ctypes.c_double]
        L.orc_boris.argtypes = [_dp, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_gather.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields), ctypes.c_int32,
                                 _dp, _dp, _dp]
        L.orc_yee_e.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields), ctypes.c_double]
        L.orc_yee_b.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields), ctypes.c_double]
        L.orc_deposit_particle.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                           ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                           _dp, _dp, ctypes.c_double]
        L.orc_deposit_rho.argtypes = [ctypes.POINTER(Grid), _dp, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_double, _dp]
        L.orc_push_deposit.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                       ctypes.POINTER(Species), ctypes.c_int32, _dp, _dp, _dp]
        L.orc_gather_push.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                      ctypes.POINTER(Species)]
        L.orc_step.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                               ctypes.POINTER(Species), ctypes.c_int32, ctypes.POINTER(Laser),
                               ctypes.c_double]
        L.orc_step_threads.restype = ctypes.c_int32
        L.orc_step_threads.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                       ctypes.POINTER(Species), ctypes.c_int32,
                                       ctypes.POINTER(Laser), ctypes.c_double, ctypes.c_int32]
        L.orc_laser_source.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                       ctypes.POINTER(Laser), ctypes.c_double]
        L.orc_field_energy.restype = ctypes.c_double
        L.orc_field_energy.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields)]
        L.orc_kinetic_energy.restype = ctypes.c_double
        L.orc_kinetic_energy.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Species)]
        L.orc_continuity.restype = ctypes.c_double
        L.orc_continuity.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields)]
        L.orc_gauss.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields), _dp]
        L.orc_div_b.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields), _dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


FIELD_NAMES = ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz")


class OracleSpecies:
    """FP64 particle arrays of one species (absolute positions)."""

    def __init__(self, q, m, order, x, y, z, ux, uy, uz, w):
        f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).copy()
        self.q, self.m, self.order = float(q), float(m), int(order)
        self.x, self.y, self.z = f64(x), f64(y), f64(z)
        self.ux, self.uy, self.uz, self.w = f64(ux), f64(uy), f64(uz), f64(w)

    @property
    def n(self):
        return self.x.shape[0]

    def struct(self):
        return Species(self.n, self.q, self.m, self.order, _ptr(self.x), _ptr(self.y),
                       _ptr(self.z), _ptr(self.ux), _ptr(self.uy), _ptr(self.uz), _ptr(self.w))


class OracleSim:
    """One periodic run: grid, FP64 fields (flat, x fastest) and species."""

    def __init__(self, ndim, nx, ny, nz, dx, dy, dz, dt, rho_bg=0.0, species=(), fields=None,
                 with_rho=True, open_x=False, laser=None, pml=None):
        self.grid = Grid(ndim, nx, ny, nz if ndim == 3 else 1, dx, dy, dz if ndim == 3 else 1.0,
                         dt, rho_bg, int(bool(open_x)), None)
        self.pml = None
        if pml:
            assert open_x, "a PML needs open x ends"
            p = pml_defaults(pml, dx)
            assert p["cells"] >= 1 and 2 * p["cells"] < nx
            self.psi = np.zeros(4 * 2 * p["cells"] * ny * (nz if ndim == 3 else 1))
            self.pml = Pml(p["cells"], p["order"], p["a_order"], 0, p["sigma_max"],
                           p["kappa_max"], p["a_max"], _ptr(self.psi))
            self.grid.pml = ctypes.pointer(self.pml)
        self.laser = None if laser is None else Laser(**laser)
        self.ncell = nx * ny * (nz if ndim == 3 else 1)
        self.f = {k: np.zeros(self.ncell) for k in FIELD_NAMES}
        if fields:
            for k, v in fields.items():
                self.f[k] = np.ascontiguousarray(v, dtype=np.float64).reshape(-1).copy()
        self.rho0 = np.zeros(self.ncell) if with_rho else None
        self.rho1 = np.zeros(self.ncell) if with_rho else None
        self.species = list(species)
        self.t = 0.0
        self.nstep = 0

    @classmethod
    def from_workload(cls, wl, with_rho=True):
        sp = [OracleSpecies(s.q, s.m, s.order, s.x, s.y, s.z, s.ux, s.uy, s.uz, s.w)
              for s in wl.species]
        return cls(wl.ndim, wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.dt, wl.rho_bg, sp,
                   wl.fields, with_rho, getattr(wl, "open_x", False), getattr(wl, "laser", None),
                   getattr(wl, "pml", None))

    def fields_struct(self):
        f = self.f
        return Fields(*(_ptr(f[k]) for k in FIELD_NAMES), _ptr(self.rho0), _ptr(self.rho1))

    # --- single operations -------------------------------------------------------------
    def yee_e(self, frac=0.5):
        fs = self.fields_struct()
        lib().orc_yee_e(ctypes.byref(self.grid), ctypes.byref(fs), frac)

    def yee_b(self, frac=0.5):
        fs = self.fields_struct()
        lib().orc_yee_b(ctypes.byref(self.grid), ctypes.byref(fs), frac)

    def gather(self, order, pos):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        E = np.zeros(3)
        B = np.zeros(3)
        fs = self.fields_struct()
        lib().orc_gather(ctypes.byref(self.grid), ctypes.byref(fs), order, _ptr(pos), _ptr(E),
                         _ptr(B))
        return E, B

    def gather_push(self, s: OracleSpecies):
        fs = self.fields_struct()
        st = s.struct()
        lib().orc_gather_push(ctypes.byref(self.grid), ctypes.byref(fs), ctypes.byref(st))

    def push_deposit(self, s: OracleSpecies, deposit=True):
        """Push one species and deposit its current; returns the deposit path starts."""
        n = s.n
        xs, ys, zs = np.zeros(n), np.zeros(n), np.zeros(n)
        fs = self.fields_struct()
        st = s.struct()
        lib().orc_push_deposit(ctypes.byref(self.grid), ctypes.byref(fs), ctypes.byref(st),
                               int(deposit), _ptr(xs), _ptr(ys), _ptr(zs))
        return xs, ys, zs

    def deposit_particle(self, order, q, w, p0, p1, vz_bar=0.0):
        fs = self.fields_struct()
        a0 = np.ascontiguousarray(p0, dtype=np.float64)
        a1 = np.ascontiguousarray(p1, dtype=np.float64)
        lib().orc_deposit_particle(ctypes.byref(self.grid), ctypes.byref(fs), order, q, w,
                                   _ptr(a0), _ptr(a1), vz_bar)

    def deposit_rho(self, rho, order, q, w, pos):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        lib().orc_deposit_rho(ctypes.byref(self.grid), _ptr(rho), order, q, w, _ptr(pos))

    def zero_currents(self):
        for k in ("jx", "jy", "jz"):
            self.f[k][:] = 0.0
        if self.rho0 is not None:
            self.rho0[:] = 0.0
            self.rho1[:] = 0.0

    # --- Algorithm 1 ---------------------------------------------------------------------
    def step(self, n=1):
        fs = self.fields_struct()
        arr = (Species * max(1, len(self.species)))(*[s.struct() for s in self.species])
        las = ctypes.byref(self.laser) if self.laser is not None else None
        for _ in range(n):
            lib().orc_step(ctypes.byref(self.grid), ctypes.byref(fs), arr, len(self.species),
                           las, (self.nstep + 1) * self.grid.dt)
            self.t += self.grid.dt
            self.nstep += 1

    def step_threads(self, n=1, threads=None):
        """The same steps with the particle loop on `threads` host threads (all logical
        CPUs by default): a timing mode, equal to step() up to the order of the current
        sums.  Returns the number of threads used."""
        threads = int(threads or os.cpu_count() or 1)
        fs = self.fields_struct()
        arr = (Species * max(1, len(self.species)))(*[s.struct() for s in self.species])
        las = ctypes.byref(self.laser) if self.laser is not None else None
        used = 1
        for _ in range(n):
            used = lib().orc_step_threads(ctypes.byref(self.grid), ctypes.byref(fs), arr,
                                          len(self.species), las,
                                          (self.nstep + 1) * self.grid.dt, threads)
            if used < 1:
                raise MemoryError("orc_step_threads could not allocate its private arrays")
            self.t += self.grid.dt
            self.nstep += 1
        return used

    # --- moving window (open x ends, 2D) -------------------------------------------------
    def window_shift(self, m, plasma=None):
        """Move the box m cells in +x between two steps: every field array moves m columns
        to the left and the m columns entering at the right start at zero; particles keep
        their place in the lab, so their box coordinate drops by m dx, and those that fall
        behind the box's left end are removed (x = -1); with `plasma` (dict: species index,
        ppc_x, ppc_y, density, ux, uy, uz), the m columns just inside the right-hand margin
        (box columns nx - 3 - m .. nx - 4) get ppc_x x ppc_y macro-particles per cell at the
        lattice points ((l + 1/2)/ppc) of each cell, weight density / (ppc_x ppc_y), in the
        order column, row, lattice point (x fastest)."""
        g = self.grid
        assert g.ndim == 2 and g.open_x, "a moving window needs a 2D box with open x ends"
        assert self.pml is None, "a moving window keeps the Mur condition"
        nx, ny = g.nx, g.ny
        arrays = [self.f[k] for k in FIELD_NAMES] + [a for a in (self.rho0, self.rho1)
                                                     if a is not None]
        for a in arrays:
            v = a.reshape(ny, nx)
            v[:, :nx - m] = v[:, m:].copy()
            v[:, nx - m:] = 0.0
        for s in self.species:
            alive = s.x >= 0.0
            s.x[alive] -= m * g.dx
            gone = alive & (s.x < 0.0)
            s.x[gone] = -1.0
            s.y[gone] = -1.0
        self.shifted = getattr(self, "shifted", 0) + m
        if plasma:
            s = self.species[plasma["species"]]
            px, py = int(plasma["ppc_x"]), int(plasma["ppc_y"])
            xs, ys = [], []
            for col in range(m):
                c = nx - OPEN_MARGIN - m + col
                for j in range(ny):
                    for l in range(px * py):
                        lx, ly = l % px, l // px
                        xs.append((c + (2 * lx + 1) / (2 * px)) * g.dx)
                        ys.append((j + (2 * ly + 1) / (2 * py)) * g.dy)
            k = len(xs)
            s.x = np.concatenate([s.x, np.array(xs)])
            s.y = np.concatenate([s.y, np.array(ys)])
            s.ux = np.concatenate([s.ux, np.full(k, float(plasma.get("ux", 0.0)))])
            s.uy = np.concatenate([s.uy, np.full(k, float(plasma.get("uy", 0.0)))])
            s.uz = np.concatenate([s.uz, np.full(k, float(plasma.get("uz", 0.0)))])
            s.w = np.concatenate([s.w, np.full(k, plasma["density"] / (px * py))])

    def laser_source(self, t):
        fs = self.fields_struct()
        lib().orc_laser_source(ctypes.byref(self.grid), ctypes.byref(fs),
                               ctypes.byref(self.laser), t)

    # --- diagnostics ---------------------------------------------------------------------
    def field_energy(self):
        fs = self.fields_struct()
        return lib().orc_field_energy(ctypes.byref(self.grid), ctypes.byref(fs))

    def kinetic_energy(self):
        tot = 0.0
        for s in self.species:
            st = s.struct()
            tot += lib().orc_kinetic_energy(ctypes.byref(self.grid), ctypes.byref(st))
        return tot

    def continuity(self):
        fs = self.fields_struct()
        return lib().orc_continuity(ctypes.byref(self.grid), ctypes.byref(fs))

    def gauss(self):
        out = np.zeros(self.ncell)
        fs = self.fields_struct()
        lib().orc_gauss(ctypes.byref(self.grid), ctypes.byref(fs), _ptr(out))
        return out

    def div_b(self):
        out = np.zeros(self.ncell)
        fs = self.fields_struct()
        lib().orc_div_b(ctypes.byref(self.grid), ctypes.byref(fs), _ptr(out))
        return out


def shape(order, xi):
    return lib().orc_shape(int(order), float(xi))


def boris(u, E, B, q, m, dt):
    u = np.array(u, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lib().orc_boris(_ptr(u), _ptr(E), _ptr(B), q, m, dt)
    return u
