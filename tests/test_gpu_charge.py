"""The charge density of diagnostic steps (rho0 and rho1 at the two ends of each deposited
path, Sec. 3.1 shapes on the integer lattice) against the oracle, node by node, in 2D and 3D.

The fused pass deposits the charge of a particle on its exact (ORDER + 1)^DIM stencils in
LDS; a particle that has left its tile's staged region goes through global memory (window
form), or, with the re-binned escape path, through the second pass.  The boxes (96 x 80 and
24^3) are hot (T = 0.5 m c^2) and sorted only at the first step, so by the compared step a
large part of the particles has left its region and every branch deposits charge.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import banner, compare_fields
from oracle import OracleSim
from paper_2607_13507_amd import lpic as L
from paper_2607_13507_amd import workloads as W
from paper_2607_13507_amd.simulation import Simulation

pytestmark = pytest.mark.gpu


def _oracle_from(sim, wl):
    """The oracle from the GPU's present state (FP32 rounding included)."""
    orc = OracleSim.from_workload(wl)
    for k, v in sim.fields[0].numpy().items():
        if k in orc.f:
            orc.f[k][:] = v
    for i, s in enumerate(orc.species):
        pos = sim.positions(i)
        s.x[:], s.y[:] = pos[0], pos[1]
        if wl.ndim == 3:
            s.z[:] = pos[2]
        cur = sim.current(i)
        for k in ("ux", "uy", "uz", "w"):
            getattr(s, k)[:] = cur.numpy(k)
    return orc


@pytest.mark.parametrize("rebin", [False, True], ids=["escape", "rebin"])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("prec", [L.F64_ABS, L.F32_CELLOFS], ids=["f64", "f32"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_charge_matches_oracle(ndim, prec, order, rebin):
    banner(f"charge ndim={ndim} prec={prec} order={order} rebin={rebin}")
    if ndim == 2:
        wl = W.thermal_2d(nx=96, ny=80, dx=0.05, ppc=8, T=0.5, order=order, seed=11)
        tiling = (8, 8, 1)
    else:
        wl = W.thermal_3d(n=24, dx=0.1, ppc=4, T=0.5, order=order, seed=11)
        tiling = (8, 4, 4)
    sim = Simulation(wl, prec=prec, tiling=tiling, halo=3, chunk=256, sort_interval=1000,
                     diag_interval=1, use_graph=False,
                     flags=L.ESCAPE_REBIN if rebin else 0)
    sim.step(12)
    torch.cuda.synchronize()
    e0 = sim.stats()["halo_escapes"]
    # one more (diagnostic) step from the GPU's state, in the oracle too
    orc = _oracle_from(sim, wl)
    sim.step(1)
    orc.step(1)
    torch.cuda.synchronize()
    esc = (sim.stats()["halo_escapes"] - e0) / wl.species[0].n
    banner(f"escapes in the compared step: {esc:.3f} of the particles")
    assert esc > 0.1, esc
    tol = 1e-10 if prec == L.F64_ABS else 2e-5
    compare_fields(sim.fields[0], orc, prec, keys=("rho0", "rho1", "jx", "jy", "jz"), tol=tol,
                   what="charge vs oracle")
    d = sim.diagnostics(0)
    assert d["continuity"] < (1e-12 if prec == L.F64_ABS else 1e-5), d
    assert d["gauss"] == pytest.approx(np.abs(orc.gauss()).max(), rel=1e-8 if prec == L.F64_ABS else 1e-4)
    sim.close()


@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
@pytest.mark.parametrize("rebin", [False, True], ids=["escape", "rebin"])
@pytest.mark.parametrize("box,prec,sort_interval",
                         [("3d", L.F32_CELLOFS, 1000), ("3d", L.F32_CELLOFS, 10),
                          ("3d", L.F32_CELLOFS, 11), ("3d_open", L.F32_CELLOFS, 1000),
                          ("2d_open", L.F32_CELLOFS, 1000), ("2d_open", L.F64_ABS, 1000)],
                         ids=["3d-f32", "3d-f32-sort_before", "3d-f32-sort_on_diag",
                              "3d_open-f32", "2d_open-f32", "2d_open-f64"])
def test_chained_charge_matches_oracle(box, prec, sort_interval, rebin, graph):
    """Inside one call, the step before a diagnostic step accumulates the charge at its
    paths' ends into rho0, leaving out the particles that leave the box, and the diagnostic
    step its own into rho1 (chained charge, 3D FP32 with 8 x 4 x 4 tiles and halo 3): a hot
    periodic box, and a hot box with open x ends, where particles leave through the ends at
    every step.  Against the oracle stepped from the GPU's state through the same two steps,
    and against the same run taken one step per call (no chain: the diagnostic step
    accumulates both planes).  With a sort interval of 10 or 11 the particles are re-sorted
    on the step before the diagnostic step or on the diagnostic step itself.  The 2D cases
    (FP32 and FP64 keep both planes on the diagnostic step) check the same quantities
    through the same calls."""
    banner(f"chained charge box={box} prec={prec} rebin={rebin} graph={graph}")
    if box.startswith("3d"):
        wl = W.thermal_3d(n=24, dx=0.1, ppc=4, T=0.5, order=2, seed=13)
        wl.open_x = box == "3d_open"
        tiling = (8, 4, 4)
    else:
        wl = W.thermal_2d(nx=96, ny=80, dx=0.05, ppc=8, T=0.5, order=2, seed=13)
        wl.open_x = True
        tiling = (8, 8, 1)
    kw = dict(prec=prec, tiling=tiling, halo=3, chunk=256, sort_interval=sort_interval,
              diag_interval=4, use_graph=graph, flags=L.ESCAPE_REBIN if rebin else 0)
    sim = Simulation(wl, **kw)
    one = Simulation(wl, **kw)
    sim.step(10)                       # steps 0-9 (diagnostics after steps 3 and 7)
    for _ in range(10):
        one.step(1)
    torch.cuda.synchronize()
    orc = _oracle_from(sim, wl)
    alive0 = int((orc.species[0].x >= 0).sum())
    sim.step(2)                        # step 10 (before a diagnostic step) and step 11
    for _ in range(2):
        one.step(1)
    orc.step(2)
    torch.cuda.synchronize()
    if box != "3d":                    # particles have left through the open ends
        assert int((orc.species[0].x >= 0).sum()) < alive0
    assert sim.diagnostics(0)["step"] == 12
    tol = 1e-10 if prec == L.F64_ABS else 2e-5
    compare_fields(sim.fields[0], orc, prec, keys=("rho0", "rho1", "jx", "jy", "jz"), tol=tol,
                   what="chained charge vs oracle")
    d, d1 = sim.diagnostics(0), one.diagnostics(0)
    cmax = 1e-12 if prec == L.F64_ABS else 1e-5
    assert d["continuity"] < cmax and d1["continuity"] < cmax, (d, d1)
    a, b = sim.fields[0].numpy(), one.fields[0].numpy()
    for k in ("rho0", "rho1"):
        err = np.abs(a[k].astype(np.float64) - b[k]).max() / np.abs(b[k]).max()
        assert err < (1e-12 if prec == L.F64_ABS else 1e-5), (k, err)
    assert d["gauss"] == pytest.approx(d1["gauss"], rel=1e-8 if prec == L.F64_ABS else 1e-4)
    assert d["kinetic_energy"] == pytest.approx(d1["kinetic_energy"],
                                                rel=1e-12 if prec == L.F64_ABS else 1e-6)
    sim.close()
    one.close()
