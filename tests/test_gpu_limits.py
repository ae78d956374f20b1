"""Boxes at the limits of the packed cell coordinate of the FP32 path (2D: nx = 65536 or
ny = 32768; 3D: nx or ny = 2048, nz = 512), thin in the other directions so that the oracle
stays quick: whole steps (sorts, diagnostics, periodic wrap across the largest index)
against the FP64 oracle, for the FP64 path (1e-10 of each component's largest value) and
the FP32 path (tracking, 1e-4)."""
import numpy as np
import pytest
import torch

from gpu_helpers import banner, compare_fields, compare_particles
from oracle import OracleSim
from paper_2607_13507_amd import lpic as L
from paper_2607_13507_amd import workloads as W
from paper_2607_13507_amd.simulation import Simulation

pytestmark = pytest.mark.gpu

SHAPES = [(2, 65536, 4, 1), (2, 8, 32768, 1), (3, 2048, 4, 4), (3, 4, 2048, 4),
          (3, 4, 4, 512)]


def _box(ndim, nx, ny, nz, seed):
    """Uniform electrons (1 per cell in 2D, 2 in 3D), T = 0.1 (they cross many cell edges in
    a few steps), quadratic shape, weights tagged (uniquely in FP32) so that particles can be
    followed through the sorts."""
    rng = np.random.default_rng(seed)
    dx = 0.1
    ncell = nx * ny * (nz if ndim == 3 else 1)
    n = (2 if ndim == 3 else 1) * ncell
    x = rng.uniform(0, nx * dx, n)
    y = rng.uniform(0, ny * dx, n)
    z = rng.uniform(0, nz * dx, n) if ndim == 3 else None
    u = rng.normal(0.0, np.sqrt(0.1), (3, n))
    # unique tags in FP32 too: (1 + i 2^-20) is exact in 21 mantissa bits for i < 2^19,
    # and ncell / n is a power of two
    assert n <= 1 << 19
    w = (ncell / n) * (1.0 + np.arange(n) * 2.0 ** -20)
    e = W.SpeciesInit("electron", -1.0, 1.0, 2, x, y, z, u[0], u[1], u[2], w)
    h = (dx, dx, dx) if ndim == 3 else (dx, dx)
    wl = W.Workload(f"limit_{nx}x{ny}x{nz}", ndim, nx, ny, nz if ndim == 3 else 1, dx, dx,
                    dx, W.cfl_dt(0.9, *h), 1.0, [e], {}, 4, {})
    wl.fields = W.random_fields(wl.ncell, seed + 1, 0.2)
    return wl


def _oracle_like(sim, wl):
    orc = OracleSim.from_workload(wl)
    for k, v in sim.fields[0].numpy().items():
        if k in orc.f:
            orc.f[k][:] = v
    s, pos, cur = orc.species[0], sim.positions(0), sim.current(0)
    s.x[:], s.y[:] = pos[0], pos[1]
    if wl.ndim == 3:
        s.z[:] = pos[2]
    for k in ("ux", "uy", "uz", "w"):
        getattr(s, k)[:] = cur.numpy(k)
    return orc


def _follow_gpu_order(orc_s, sim):
    tags = sim.current(0).numpy("w").astype(np.float64)
    idx = np.argsort(orc_s.w)
    perm = idx[np.searchsorted(orc_s.w[idx], tags)]
    for k in ("x", "y", "z", "ux", "uy", "uz", "w"):
        a = getattr(orc_s, k)
        if a is not None:
            a[:] = a[perm]


@pytest.mark.parametrize("prec", [L.F64_ABS, L.F32_CELLOFS], ids=["f64", "f32"])
@pytest.mark.parametrize("ndim,nx,ny,nz", SHAPES,
                         ids=[f"{d}d-{a}x{b}x{c}" for d, a, b, c in SHAPES])
def test_box_at_the_cell_packing_limit(prec, ndim, nx, ny, nz):
    banner(f"packing limit {ndim}D {nx}x{ny}x{nz} prec={'f64' if prec == L.F64_ABS else 'f32'}")
    wl = _box(ndim, nx, ny, nz, seed=101 + nx + 7 * ny + 13 * nz)
    tiling, halo = ((8, 8, 1), 4) if ndim == 2 else ((8, 4, 4), 3)
    sim = Simulation(wl, prec=prec, tiling=tiling, halo=halo, chunk=256, sort_interval=2,
                     diag_interval=2, use_graph=True)
    orc = _oracle_like(sim, wl)
    sim.step(4)
    orc.step(4)
    torch.cuda.synchronize()
    f64 = prec == L.F64_ABS
    compare_fields(sim.fields[0], orc, prec, tol=1e-10 if f64 else 1e-4, what="fields")
    _follow_gpu_order(orc.species[0], sim)
    tol = 1e-10 if f64 else 1e-4
    compare_particles(sim.grids[0], sim.current(0), orc.species[0], prec, tol_pos=tol,
                      tol_u=tol)
    d = sim.diagnostics(0)
    assert d["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-10 if f64 else 1e-4)
    assert d["continuity"] < (1e-12 if f64 else 1e-5)
    sim.close()
