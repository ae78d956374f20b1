"""Shared helpers of the GPU parity tests: build the same seeded state on the GPU (through
the C ABI) and in the FP64 oracle, and compare."""
import numpy as np
import torch

from oracle import OracleSim, OracleSpecies
from paper_2607_13507_amd import lpic as L
from paper_2607_13507_amd import workloads as W
from paper_2607_13507_amd.simulation import DeviceFields, DeviceSpecies, grid_struct

FIELDS = ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz")
TOL = {L.F64_ABS: 1e-11, L.F32_CELLOFS: 2e-5}


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def device_state(wl, prec, random_fields_seed=None, field_scale=1.0):
    """GPU fields + species for workload wl, and the oracle with the same inputs."""
    if random_fields_seed is not None:
        wl.fields = W.random_fields(wl.ncell, random_fields_seed, field_scale)
    grid = grid_struct(wl)
    F = DeviceFields(wl, prec)
    S = [DeviceSpecies.from_init(grid, s, prec) for s in wl.species]
    torch.cuda.synchronize()
    orc = OracleSim.from_workload(wl)
    if prec == L.F32_CELLOFS:
        # the oracle starts from exactly the FP32-rounded fields the GPU holds
        for k, v in F.numpy().items():
            if k in orc.f:
                orc.f[k][:] = v
        # and from the positions / momenta as the GPU stores them
        for s, d in zip(orc.species, S):
            pos = d.positions(grid)
            s.x[:] = pos[0]
            s.y[:] = pos[1]
            if wl.ndim == 3:
                s.z[:] = pos[2]
            for k in ("ux", "uy", "uz", "w"):
                getattr(s, k)[:] = d.numpy(k)
    return grid, F, S, orc


def periodic_diff(a, b, L_):
    d = a - b
    return d - L_ * np.round(d / L_)


def compare_particles(grid, dspec, ospec, prec, tol_pos=None, tol_u=None, what=""):
    pos = dspec.positions(grid)
    Ls = (grid.nx * grid.dx, grid.ny * grid.dy, grid.nz * grid.dz)
    oxyz = (ospec.x, ospec.y, ospec.z)
    tol_pos = tol_pos if tol_pos is not None else (1e-11 if prec == L.F64_ABS else 2e-5)
    tol_u = tol_u if tol_u is not None else (1e-11 if prec == L.F64_ABS else 2e-5)
    h = (grid.dx, grid.dy, grid.dz)
    for d in range(grid.ndim):
        alive = oxyz[0] >= 0
        err = np.abs(periodic_diff(pos[d][alive], oxyz[d][alive], Ls[d])).max(initial=0) / h[d]
        assert err <= tol_pos, f"{what} position axis {d}: {err} cells"
    for k in ("ux", "uy", "uz"):
        g = dspec.numpy(k).astype(np.float64)
        o = getattr(ospec, k)
        scale = max(1.0, np.abs(o).max(initial=0))
        err = np.abs(g - o).max(initial=0) / scale
        assert err <= tol_u, f"{what} {k}: {err}"


def compare_fields(F, orc, prec, keys=FIELDS, tol=None, what="", floor=None):
    """Max error of each component relative to its largest magnitude (or to floor[k] when
    that is larger: a component that is nearly zero everywhere is compared against the
    scale it would have in a non-trivial state)."""
    tol = tol if tol is not None else TOL[prec]
    g = F.numpy()
    worst = {}
    for k in keys:
        o = orc.f[k] if k in orc.f else getattr(orc, k)
        scale = max(1e-300, np.abs(o).max(initial=0), (floor or {}).get(k, 0.0))
        err = np.abs(g[k] - o).max(initial=0) / scale
        worst[k] = err
        assert err <= tol, f"{what} {k}: rel err {err} (scale {scale})"
    return worst
