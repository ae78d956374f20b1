"""Open x ends (first-order Mur, particle loss) and the laser antenna on the GPU, against
the FP64 oracle through the C ABI: single kernels, then whole steps with particles leaving
through both ends while the antenna drives a pulse in.  Tolerances as in
test_gpu_kernels.py (FP64: rounding order only; FP32: a few ulps per operation)."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import banner, compare_fields, compare_particles, device_state
from oracle import Laser, OracleSim
from paper_2607_13507_amd import lpic as L
from paper_2607_13507_amd import workloads as W
from paper_2607_13507_amd.simulation import Simulation

pytestmark = pytest.mark.gpu

PRECS = [L.F64_ABS, L.F32_CELLOFS]
PNAME = {L.F64_ABS: "f64", L.F32_CELLOFS: "f32"}


def _open(wl):
    wl.open_x = True
    return wl


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
@pytest.mark.parametrize("ndim", [2, 3])
def test_yee_with_open_x_ends(prec, ndim):
    banner(f"open yee prec={PNAME[prec]} ndim={ndim}")
    wl = W.thermal_2d(nx=40, ny=36, dx=0.1, ppc=1) if ndim == 2 else \
        W.thermal_3d(n=20, dx=0.1, ppc=1)
    wl.species = []
    _open(wl)
    grid, F, S, orc = device_state(wl, prec, random_fields_seed=11)
    assert grid.open_x == 1 and orc.grid.open_x == 1
    rng = np.random.default_rng(12)
    for k in ("jx", "jy", "jz"):
        F.t[k].copy_(torch.from_numpy(rng.uniform(-1, 1, wl.ncell)))
        orc.f[k][:] = F.t[k].double().cpu().numpy()
    for which, frac in ((0, 0.5), (1, 0.5), (0, 1.0), (1, 0.25)):
        L.lpic_yee_update_EB(grid, F.struct(), which, frac, 0, prec)
        (orc.yee_e if which == 0 else orc.yee_b)(frac)
        compare_fields(F, orc, prec, what=f"which={which} frac={frac}")


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
@pytest.mark.parametrize("ndim,pol", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_laser_source_matches_oracle(prec, ndim, pol):
    banner(f"laser source prec={PNAME[prec]} ndim={ndim} pol={pol}")
    wl = W.thermal_2d(nx=40, ny=36, dx=0.1, ppc=1) if ndim == 2 else \
        W.thermal_3d(n=20, dx=0.1, ppc=1)
    wl.species = []
    _open(wl)
    grid, F, S, orc = device_state(wl, prec)
    las = dict(pol=pol, ia=5, a0=3.0, omega=2.0, waist=0.8, yc=1.7, zc=1.1, t0=0.3, tau=4.0)
    orc.laser = Laser(**las)
    for t in (0.1, 0.9, 2.3, 4.2):   # before, inside and after the envelope
        L.lpic_laser_source(grid, F.struct(), L.Laser(**las), t, prec)
        orc.laser_source(t)
    compare_fields(F, orc, prec, keys=("jx", "jy", "jz"), what="antenna J")
    J = F.numpy()["jy" if pol == 1 else "jz"].reshape(-1, wl.nx)
    assert np.count_nonzero(J[:, :5]) == 0 and np.count_nonzero(J[:, 6:]) == 0


def _open_laser_box(order, ndim, seed=21):
    if ndim == 2:
        wl = W.thermal_2d(nx=48, ny=40, dx=0.1, ppc=4, T=0.2, order=order, seed=seed)
        las = dict(pol=1, ia=3, a0=2.0, omega=4.0, waist=1.2, yc=2.0, zc=0.0, t0=0.0, tau=3.0)
    else:
        wl = W.thermal_3d(n=16, dx=0.1, ppc=2, T=0.2, order=order, seed=seed)
        las = dict(pol=2, ia=3, a0=2.0, omega=4.0, waist=0.6, yc=0.8, zc=0.8, t0=0.0, tau=3.0)
    wl.open_x = True
    wl.laser = las
    for s in wl.species:   # unique weights: the tests follow particles through sorts
        s.w = s.w * (1.0 + 1e-3 * np.arange(s.n) / s.n)
    return wl


def _oracle_like(sim, wl):
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


def _follow_gpu_order(orc_s, sim, i):
    tags = sim.current(i).numpy("w").astype(np.float64)
    idx = np.argsort(orc_s.w)
    perm = idx[np.searchsorted(orc_s.w[idx], tags)]
    for k in ("x", "y", "z", "ux", "uy", "uz", "w"):
        a = getattr(orc_s, k)
        if a is not None:
            a[:] = a[perm]


@pytest.mark.parametrize("ndim,order", [(2, 1), (2, 2), (3, 2)])
@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_open_x_laser_steps_match_oracle(ndim, order, graph):
    banner(f"open + laser f64 steps ndim={ndim} order={order} graph={graph}")
    wl = _open_laser_box(order, ndim)
    tiling, halo = ((8, 8, 1), 4) if ndim == 2 else ((8, 4, 4), 3)
    sim = Simulation(wl, prec=L.F64_ABS, tiling=tiling, halo=halo, chunk=128, sort_interval=4,
                     diag_interval=2, use_graph=graph)
    orc = _oracle_like(sim, wl)
    n0 = sum(int((s.x >= 0).sum()) for s in orc.species)
    nsteps = 16
    sim.step(nsteps)
    orc.step(nsteps)
    torch.cuda.synchronize()
    compare_fields(sim.fields[0], orc, L.F64_ABS, tol=1e-10, what="fields")
    _follow_gpu_order(orc.species[0], sim, 0)
    dead_gpu = sim.positions(0)[0] < 0
    dead_orc = orc.species[0].x < 0
    np.testing.assert_array_equal(dead_gpu, dead_orc)
    assert dead_orc.sum() > 0 and sum(int((s.x >= 0).sum()) for s in orc.species) < n0
    compare_particles(sim.grids[0], sim.current(0), orc.species[0], L.F64_ABS, tol_pos=1e-10,
                      tol_u=1e-10)
    d = sim.diagnostics(0)
    assert d["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-10)
    assert d["kinetic_energy"] == pytest.approx(orc.kinetic_energy(), rel=1e-10)
    assert d["continuity"] < 1e-12
    assert orc.field_energy() > 0.1   # the antenna did inject a pulse
    sim.close()


def test_open_x_laser_fp32_tracks_oracle_and_conserves_charge():
    banner("open + laser f32 steps")
    wl = _open_laser_box(2, 2)
    sim = Simulation(wl, prec=L.F32_CELLOFS, tiling=(16, 16, 1), halo=4, chunk=256,
                     sort_interval=4, diag_interval=1, use_graph=True)
    orc = _oracle_like(sim, wl)
    for n in range(1, 9):
        sim.step(1)
        orc.step(1)
        d = sim.diagnostics(0)
        assert d["continuity"] < 1e-5, (n, d)
        if n <= 4:
            compare_fields(sim.fields[0], orc, L.F32_CELLOFS, tol=1e-4, what=f"step {n}")
            assert d["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-4)
    sim.close()


def test_antenna_pulse_leaves_through_the_open_end():
    """Vacuum: the antenna's pulse crosses the box and leaves; what stays is far below what
    passed (FP32, graph replay, many steps in one call)."""
    banner("antenna pulse leaves")
    nx, ny = 256, 16
    dx = 2 * math.pi / 32
    dt = 0.95 * dx / math.sqrt(2)
    wl = W.Workload("vacuum_open", 2, nx, ny, 1, dx, dx, 1.0, dt, 0.0, [], {}, 1, {},
                    open_x=True,
                    laser=dict(pol=1, ia=4, a0=1.0, omega=1.0, waist=1e9, yc=0.0, zc=0.0,
                               t0=0.0, tau=20.0))
    sim = Simulation(wl, prec=L.F32_CELLOFS, tiling=(16, 16, 1), halo=4, chunk=256,
                     sort_interval=10, diag_interval=1, use_graph=True)
    peak = 0.0
    for _ in range(16):
        sim.step(40)
        peak = max(peak, sim.diagnostics(0)["field_energy"])
    final = sim.diagnostics(0)["field_energy"]
    assert peak > 1.0 and final < 2e-3 * peak, (peak, final)
    sim.close()


def test_laser_attached_after_some_steps_keeps_the_clock():
    """An antenna attached after steps without one starts from the simulation's clock
    (t = (step + 1) dt), eager and graph replay alike."""
    banner("laser attached late")
    for graph in (False, True):
        wl = _open_laser_box(2, 2, seed=23)
        las = wl.laser
        wl.laser = None
        sim = Simulation(wl, prec=L.F64_ABS, tiling=(8, 8, 1), halo=4, chunk=128,
                         sort_interval=4, diag_interval=0, use_graph=graph)
        orc = _oracle_like(sim, wl)
        sim.step(5)
        orc.step(5)
        sim.set_laser(0, dict(las, t0=0.2))
        orc.laser = Laser(**dict(las, t0=0.2))
        sim.step(7)
        orc.step(7)
        torch.cuda.synchronize()
        compare_fields(sim.fields[0], orc, L.F64_ABS, tol=1e-10, what=f"graph={graph}")
        assert orc.field_energy() > 0.01
        sim.close()
