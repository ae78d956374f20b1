"""Python harness over the C ABI: device memory as torch tensors, named-stage hooks.

``Simulation`` owns the field and particle tensors of one box or an ensemble of boxes and
drives ``lpic_step`` (Algorithm 1 of the paper, Sec. 3.3).  Callbacks follow the paper's
callback system (Sec. 2.2): a function attached to a named stage with an interval (whole
steps, simulation time, or a predicate) that sees the full state, here as torch tensors on
the GPU.  Every step of the hot path runs in the HIP library; this module only marshals.
"""
from __future__ import annotations

import ctypes
from typing import Callable, Dict, List, Optional, Sequence, Union

import numpy as np
import torch

from . import lpic as L
from .workloads import Workload

FIELD_NAMES = ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz")


def torch_dtype(prec):
    return torch.float32 if prec == L.F32_CELLOFS else torch.float64


def grid_struct(wl: Workload) -> L.Grid:
    return L.Grid(wl.ndim, wl.nx, wl.ny, wl.nz if wl.ndim == 3 else 1, wl.dx, wl.dy,
                  wl.dz if wl.ndim == 3 else 1.0, wl.dt, wl.rho_bg,
                  int(bool(getattr(wl, "open_x", False))), 0)


class DeviceFields:
    """Yee arrays of one box (flat, x fastest) plus rho at the start / end of a step."""

    def __init__(self, wl: Workload, prec, device="cuda", with_rho=True):
        dt = torch_dtype(prec)
        n = wl.ncell
        self.t: Dict[str, torch.Tensor] = {k: torch.zeros(n, dtype=dt, device=device)
                                           for k in FIELD_NAMES}
        for k, v in wl.fields.items():
            self.t[k].copy_(torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(dt))
        self.rho0 = torch.zeros(n, dtype=dt, device=device) if with_rho else None
        self.rho1 = torch.zeros(n, dtype=dt, device=device) if with_rho else None

    def struct(self) -> L.Fields:
        return L.Fields(*[L.ptr(self.t[k]) for k in FIELD_NAMES], L.ptr(self.rho0),
                        L.ptr(self.rho1))

    def numpy(self) -> Dict[str, np.ndarray]:
        out = {k: v.detach().double().cpu().numpy() for k, v in self.t.items()}
        if self.rho0 is not None:
            out["rho0"] = self.rho0.double().cpu().numpy()
            out["rho1"] = self.rho1.double().cpu().numpy()
        return out


class DeviceSpecies:
    """Structure-of-arrays particle storage of one species on the GPU."""

    def __init__(self, ndim, n, q, m, order, prec, device="cuda"):
        self.ndim, self.n, self.q, self.m, self.order, self.prec = ndim, n, q, m, order, prec
        dt = torch_dtype(prec)
        e = lambda d: torch.empty(n, dtype=d, device=device)
        self.a: Dict[str, torch.Tensor] = {}
        if prec == L.F32_CELLOFS:
            self.a["cell"] = e(torch.int32)
            for k in ("ox", "oy", "oz")[:ndim]:
                self.a[k] = e(torch.float32)
        else:
            for k in ("x", "y", "z")[:ndim]:
                self.a[k] = e(torch.float64)
        for k in ("ux", "uy", "uz", "w"):
            self.a[k] = e(dt)

    @classmethod
    def from_init(cls, grid: L.Grid, s, prec, device="cuda", stream=None):
        d = cls(grid.ndim, s.n, s.q, s.m, s.order, prec, device)
        dt = torch_dtype(prec)
        for k in ("ux", "uy", "uz", "w"):
            d.a[k].copy_(torch.from_numpy(np.ascontiguousarray(getattr(s, k), dtype=np.float64)).to(dt))
        d.load_positions(grid, s.x, s.y, s.z, stream)
        return d

    def like(self):
        return DeviceSpecies(self.ndim, self.n, self.q, self.m, self.order, self.prec,
                             next(iter(self.a.values())).device)

    def struct(self) -> L.Species:
        g = lambda k: L.ptr(self.a.get(k))
        return L.Species(self.n, self.q, self.m, self.order, 0, g("cell"), g("ox"), g("oy"),
                         g("oz"), g("x"), g("y"), g("z"), g("ux"), g("uy"), g("uz"), g("w"))

    def load_positions(self, grid, x, y, z=None, stream=None):
        if self.n == 0:
            return
        dev = next(iter(self.a.values())).device
        t = [torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(dev)
             if v is not None else None for v in (x, y, z)]
        L.lpic_load_positions(grid, self.struct(), L.ptr(t[0]), L.ptr(t[1]), L.ptr(t[2]),
                              self.prec, stream)
        torch.cuda.current_stream().synchronize()

    def positions(self, grid, stream=None) -> List[np.ndarray]:
        """Absolute FP64 positions (dead particles: -1)."""
        if self.n == 0:
            return [np.zeros(0)] * self.ndim
        dev = next(iter(self.a.values())).device
        t = [torch.empty(self.n, dtype=torch.float64, device=dev) for _ in range(self.ndim)]
        t3 = t + [None] * (3 - self.ndim)
        L.lpic_store_positions(grid, self.struct(), L.ptr(t3[0]), L.ptr(t3[1]), L.ptr(t3[2]),
                               self.prec, stream)
        return [v.cpu().numpy() for v in t]

    def numpy(self, k) -> np.ndarray:
        return self.a[k].detach().cpu().numpy()


# ------------------------------------------------------------------------------------------
# callbacks (Sec. 2.2)
# ------------------------------------------------------------------------------------------
class Callback:
    """Stateful callback: subclass, set `stage` and `interval`, implement __call__(sim)."""

    stage: str = "LOOP_END"
    interval: Union[int, float, Callable, None] = 1

    def __call__(self, sim: "Simulation"):
        raise NotImplementedError

    def due(self, sim: "Simulation") -> bool:
        iv = self.interval
        if iv is None:
            return True
        if callable(iv):
            return bool(iv(sim))
        if isinstance(iv, int):
            return sim.nstep % iv == 0
        # simulation-time interval: fire on the first step at or past each multiple
        k = int(np.floor(sim.time / iv + 1e-9))
        if k > getattr(self, "_last_k", -1):
            self._last_k = k
            return True
        return False


def callback(stage="LOOP_END", interval: Union[int, float, Callable, None] = 1):
    """Decorator: attach a plain function f(sim) to a named stage with an interval."""

    def wrap(fn):
        class _Fn(Callback):
            pass

        cb = _Fn()
        cb.stage = stage
        cb.interval = interval
        cb.__call__ = None
        cb.fn = fn
        cb.__name__ = getattr(fn, "__name__", "callback")
        return cb

    return wrap


def _run_cb(cb, sim):
    fn = getattr(cb, "fn", None)
    return fn(sim) if fn is not None else cb(sim)


# ------------------------------------------------------------------------------------------
class Simulation:
    """One box or an ensemble of independent boxes advanced by lpic_step."""

    def __init__(self, workloads: Union[Workload, Sequence[Workload]], prec=L.F32_CELLOFS,
                 tiling=(16, 16, 8), halo=5, chunk=2048, sort_interval=10, diag_interval=0,
                 use_graph=True, device="cuda", with_rho=True, stream=None, flags=0):
        wls = [workloads] if isinstance(workloads, Workload) else list(workloads)
        self.workloads = wls
        self.prec = prec
        self.ndim = wls[0].ndim
        self.stream = stream
        self.grids = [grid_struct(w) for w in wls]
        self.fields = [DeviceFields(w, prec, device, with_rho) for w in wls]
        self.species: List[DeviceSpecies] = []
        self.alt: List[DeviceSpecies] = []
        self.species_run: List[int] = []
        for r, w in enumerate(wls):
            for s in w.species:
                d = DeviceSpecies.from_init(self.grids[r], s, prec, device, stream)
                self.species.append(d)
                self.alt.append(d.like())
                self.species_run.append(r)
        self.options = L.Options(L.Tiling(tiling[0], tiling[1], tiling[2] if self.ndim == 3 else 1,
                                          halo, chunk, flags),
                                 sort_interval, diag_interval, int(use_graph), 0)
        self.h = L.lpic_sim_create(self.grids, [f.struct() for f in self.fields],
                                   [s.struct() for s in self.species], self.species_run,
                                   [a.struct() for a in self.alt], prec, self.options, stream)
        self._hook_refs = []
        self._callbacks: List[Callback] = []
        self.nstep = 0
        self.dt = wls[0].dt
        for r, w in enumerate(wls):   # laser antennas (GaussianLaser, Sec. 2.2)
            if getattr(w, "laser", None):
                self.set_laser(r, w.laser)
            if getattr(w, "pml", None):
                self.set_pml(r, w.pml)

    def species_of_run(self, r) -> List[int]:
        """Global indices of run r's species, in the order its workload lists them."""
        return [i for i, rr in enumerate(self.species_run) if rr == r]

    def set_laser(self, r, laser):
        """Attach the antenna `laser` (dict with the fields of lpic_laser) to run r, or
        remove it with None."""
        L.lpic_set_laser(self.h, r, L.Laser(**laser) if laser else None)

    def set_pml(self, r, pml):
        """Convolutional PML layers at run r's open x ends (dict: cells, order=3, a_order=1,
        sigma_max=-1 for 0.8 (order + 1) / dx, kappa_max=1, a_max=0), or None for Mur."""
        p = None
        if pml:
            sigma = pml.get("sigma_max")
            p = L.Pml(int(pml["cells"]), int(pml.get("order", 3)), int(pml.get("a_order", 1)),
                      0, -1.0 if sigma is None else float(sigma),
                      float(pml.get("kappa_max", 1.0)), float(pml.get("a_max", 0.0)))
        L.lpic_set_pml(self.h, r, p)

    def window_shift(self, r, m, plasma=None):
        """Move box r's window by m cells in +x (open x ends).  plasma: dict(species=global
        species index, ppc_x, ppc_y, density, ux=0, uy=0, uz=0) for the fresh columns."""
        pl = None
        if plasma:
            pl = L.Plasma(plasma["species"], plasma["ppc_x"], plasma["ppc_y"], 0,
                          plasma["density"], plasma.get("ux", 0.0), plasma.get("uy", 0.0),
                          plasma.get("uz", 0.0))
        L.lpic_window_shift(self.h, r, m, pl)

    def window_info(self, r=0):
        """(cells box r has moved, fresh particles dropped for lack of slots)"""
        return L.lpic_window_info(self.h, r)

    def box_fields(self, r=0):
        """Field arrays of box r in the box frame (column 0 = the window's left end), as
        float64 numpy arrays shaped (nz,) ny, nx."""
        import numpy as np
        shift = self.window_info(r)[0] % self.grids[r].nx
        g = self.grids[r]
        shape = (g.nz, g.ny, g.nx) if self.ndim == 3 else (g.ny, g.nx)
        return {k: np.roll(v.reshape(shape).astype(np.float64), -shift, axis=-1)
                for k, v in self.fields[r].numpy().items()}

    # -- state ------------------------------------------------------------------------------
    @property
    def time(self):
        return self.nstep * self.dt

    def current(self, i) -> DeviceSpecies:
        """The buffer that holds species i now (the sort alternates two buffers)."""
        cur = L.lpic_get_species(self.h, i)
        a = self.species[i]
        key = "cell" if self.prec == L.F32_CELLOFS else "x"
        if a.n == 0 or cur.ux == L.ptr(a.a["ux"]):
            return a
        b = self.alt[i]
        assert cur.ux == L.ptr(b.a["ux"]) and (getattr(cur, key) == L.ptr(b.a[key]))
        return b

    def positions(self, i):
        """Absolute FP64 positions of species i in its box's frame (dead particles: -1)."""
        r = self.species_run[i]
        pos = self.current(i).positions(self.grids[r], self.stream)
        shift = self.window_info(r)[0] % self.grids[r].nx if self.ndim == 2 else 0
        if shift:   # the arrays' frame of a moved window: box x = array x - x0 dx (mod L)
            g = self.grids[r]
            x = pos[0]
            alive = x >= 0.0
            xb = x[alive] - shift * g.dx
            x[alive] = np.where(xb < 0.0, xb + g.nx * g.dx, xb)
        return pos

    def step(self, n=1):
        start = self.nstep
        L.lpic_step(self.h, n)
        self.nstep = start + n

    def diagnostics(self, r=0):
        d = L.lpic_get_diagnostics(self.h, r)
        return dict(field_energy=d[0], kinetic_energy=d[1], continuity=d[2], gauss=d[3],
                    step=int(d[4]))

    def stats(self):
        s = L.lpic_get_stats(self.h)
        return dict(steps=s.steps, sorts=s.sorts, fused=bool(s.fused), graph=bool(s.graph),
                    fused_ms=s.fused_ms, fused_launches=s.fused_launches,
                    halo_escapes=s.halo_escapes,
                    field_tile=(s.field_tile[0], s.field_tile[1]))

    def set_timing(self, on):
        L.lpic_set_timing(self.h, on)

    def set_options(self, **kw):
        o = self.options
        t = o.tiling
        tiling = kw.get("tiling", (t.tx, t.ty, t.tz))
        self.options = L.Options(L.Tiling(tiling[0], tiling[1], tiling[2] if self.ndim == 3 else 1,
                                          kw.get("halo", t.halo), kw.get("chunk", t.chunk),
                                          kw.get("flags", t.flags)),
                                 kw.get("sort_interval", o.sort_interval),
                                 kw.get("diag_interval", o.diag_interval),
                                 int(kw.get("use_graph", o.use_graph)), 0)
        L.lpic_set_options(self.h, self.options)

    def autotune(self, candidates: Sequence[dict], steps_each=3):
        opts = []
        for c in candidates:
            t = c.get("tiling", (16, 16, 8))
            opts.append(L.Options(L.Tiling(t[0], t[1], t[2] if self.ndim == 3 else 1,
                                           c.get("halo", 5), c.get("chunk", 2048),
                                           c.get("flags", self.options.tiling.flags)),
                                  c.get("sort_interval", self.options.sort_interval),
                                  c.get("diag_interval", self.options.diag_interval),
                                  int(c.get("use_graph", self.options.use_graph)), 0))
        before = L.lpic_get_stats(self.h).steps
        best = L.lpic_autotune(self.h, opts, steps_each)
        self.nstep += L.lpic_get_stats(self.h).steps - before
        self.options = best
        t = best.tiling
        return dict(tiling=(t.tx, t.ty, t.tz), halo=t.halo, chunk=t.chunk,
                    sort_interval=best.sort_interval, use_graph=bool(best.use_graph))

    def autotune_search(self, tile=((8, 8, 1), (32, 32, 1)), halo=(3, 7), chunk=(512, 4096),
                        sort_interval=(10, 80), rebin=2, steps_each=40, max_trials=24):
        """lpic_autotune_search over the given (min, max) ranges (rebin: the re-binned
        escape path off 0, on 1, both tried 2); the simulation advances while it tunes.
        Returns the chosen options and every trial (options, ms per step)."""
        sp = L.TuneSpace((ctypes.c_int32 * 3)(*tile[0]), (ctypes.c_int32 * 3)(*tile[1]),
                         halo[0], halo[1], chunk[0], chunk[1], sort_interval[0],
                         sort_interval[1], rebin, steps_each, max_trials)
        before = L.lpic_get_stats(self.h).steps
        best, rep = L.lpic_autotune_search(self.h, sp)
        self.nstep += L.lpic_get_stats(self.h).steps - before
        self.options = best

        def od(o):
            t = o.tiling
            return dict(tiling=(t.tx, t.ty, t.tz), halo=t.halo, chunk=t.chunk,
                        sort_interval=o.sort_interval, flags=t.flags,
                        rebin=bool(t.flags & L.ESCAPE_REBIN))
        trials = [dict(od(rep.trial[i]), ms_per_step=round(rep.ms_per_step[i], 4))
                  for i in range(rep.ntrials)]
        return dict(od(best), use_graph=bool(best.use_graph)), trials

    # -- hooks and callbacks --------------------------------------------------------------
    def register_hook(self, stage: str, fn: Callable[["Simulation", str, int], Optional[int]]):
        """Raw hook: fn(sim, stage_name, step) -> 0/None to continue, non-zero to stop."""
        def c_hook(h, st, step, user):
            try:
                self.nstep = int(step)
                rc = fn(self, L.STAGES[st], int(step))
                return int(rc or 0)
            except Exception:  # a Python error stops the step with LPIC_EHOOK
                import traceback
                traceback.print_exc()
                return 1
        cf = L.HOOK_FN(c_hook)
        self._hook_refs.append(cf)
        L.lpic_register_hook(self.h, L.STAGE[stage], cf, None)

    def add_callback(self, cb: Callback):
        self._callbacks.append(cb)

        def hook(sim, stage, step):
            if cb.due(sim):
                return _run_cb(cb, sim)
            return 0
        self.register_hook(cb.stage, hook)

    def clear_hooks(self):
        L.lpic_clear_hooks(self.h)
        self._hook_refs.clear()
        self._callbacks.clear()

    def close(self):
        if getattr(self, "h", None):
            L.lpic_sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
