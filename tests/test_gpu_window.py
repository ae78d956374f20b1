"""Moving window on the GPU (lpic_window_shift) against the oracle (OracleSim.window_shift),
through the C ABI: an open-ended 2D box with a thermal plasma and fields moves by a few
cells every few steps, fresh cold plasma filling the columns that enter at the right, for
FP64 (eager and graph replay: tolerance as for the FP64 steps, 1e-10 of each component's
largest value) and FP32 (tracking, 1e-4, charge continuity 1e-5).  The GPU's arrays are in
the array frame (circular x with the window's origin); `Simulation.box_fields` rolls them
back to the box frame the oracle uses.  Particles are compared as sets: the originals carry
unique weights, the fresh ones sit on a lattice.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import banner
from oracle import OracleSim
from paper_2607_13507_amd import lpic as L
from paper_2607_13507_amd import workloads as W
from paper_2607_13507_amd.simulation import Simulation

pytestmark = pytest.mark.gpu

PNAME = {L.F64_ABS: "f64", L.F32_CELLOFS: "f32"}
PLASMA = dict(species=0, ppc_x=2, ppc_y=2, density=0.5)
FIELDS = ("ex", "ey", "ez", "bx", "by", "bz")


def _box(pad, seed=61):
    wl = W.thermal_2d(nx=64, ny=16, dx=0.1, ppc=4, T=0.01, order=2, seed=seed)
    wl.open_x = True
    wl.fields = W.random_fields(wl.ncell, seed + 1, 0.05)
    s = wl.species[0]
    s.w = s.w * (1.0 + 1e-3 * np.arange(s.n) / s.n)   # unique tags
    # dead slots for the fresh plasma
    dead = np.full(pad, -1.0)
    s.x, s.y = np.concatenate([s.x, dead]), np.concatenate([s.y, dead])
    for k in ("ux", "uy", "uz", "w"):
        setattr(s, k, np.concatenate([getattr(s, k), np.zeros(pad)]))
    return wl


def _oracle_like(sim, wl):
    orc = OracleSim.from_workload(wl)
    for k, v in sim.fields[0].numpy().items():
        if k in orc.f:
            orc.f[k][:] = v
    s, pos, cur = orc.species[0], sim.positions(0), sim.current(0)
    s.x[:], s.y[:] = pos[0], pos[1]
    for k in ("ux", "uy", "uz", "w"):
        getattr(s, k)[:] = cur.numpy(k)
    return orc


def _alive_set(x, y, ux, uy, uz, w, dx):
    keep = x >= 0
    x, y, ux, uy, uz, w = (np.asarray(a, dtype=np.float64)[keep] for a in (x, y, ux, uy, uz, w))
    order = np.lexsort((y, np.round(x / dx * 1e4), w))
    return np.stack([x, y, ux, uy, uz, w])[:, order]


def _compare(sim, orc, wl, tol, what):
    bf = sim.box_fields(0)
    for k in FIELDS:
        o = orc.f[k].reshape(wl.ny, wl.nx)
        err = np.abs(bf[k] - o).max() / max(1e-300, np.abs(o).max())
        assert err <= tol, f"{what} {k}: {err}"
    pos, cur = sim.positions(0), sim.current(0)
    g = _alive_set(pos[0], pos[1], cur.numpy("ux"), cur.numpy("uy"), cur.numpy("uz"),
                   cur.numpy("w"), wl.dx)
    s = orc.species[0]
    o = _alive_set(s.x, s.y, s.ux, s.uy, s.uz, s.w, wl.dx)
    assert g.shape == o.shape, (what, g.shape, o.shape)
    assert np.abs(g[:2] - o[:2]).max() / wl.dx <= tol * 10, what        # positions, cells
    assert np.abs(g[2:5] - o[2:5]).max() <= tol * 10, what               # momenta
    np.testing.assert_allclose(g[5], o[5], rtol=1e-6)                     # weights


def _run(sim, orc, shifts, every):
    for m in shifts:
        sim.step(every)
        orc.step(every)
        sim.window_shift(0, m, PLASMA)
        orc.window_shift(m, PLASMA)
    sim.step(every)
    orc.step(every)
    torch.cuda.synchronize()


@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_moving_window_fp64_matches_oracle(graph):
    banner(f"moving window f64 graph={graph}")
    wl = _box(pad=2048)
    sim = Simulation(wl, prec=L.F64_ABS, tiling=(8, 8, 1), halo=4, chunk=128, sort_interval=3,
                     diag_interval=3, use_graph=graph)
    orc = _oracle_like(sim, wl)
    shifts = (3, 1, 5, 2, 4)
    _run(sim, orc, shifts, every=3)
    assert sim.window_info(0) == (sum(shifts), 0)
    assert sim.stats()["field_tile"] == (0, 0)   # separate field kernels once a window moved
    _compare(sim, orc, wl, 1e-10, "fp64")
    d = sim.diagnostics(0)
    assert d["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-10)
    assert d["kinetic_energy"] == pytest.approx(orc.kinetic_energy(), rel=1e-10)
    assert d["continuity"] < 1e-12
    sim.close()


def test_moving_window_fp32_tracks_oracle():
    banner("moving window f32")
    wl = _box(pad=2048, seed=63)
    sim = Simulation(wl, prec=L.F32_CELLOFS, tiling=(8, 8, 1), halo=4, chunk=128,
                     sort_interval=2, diag_interval=2, use_graph=True)
    orc = _oracle_like(sim, wl)
    _run(sim, orc, (2, 3, 1), every=2)
    _compare(sim, orc, wl, 1e-4, "fp32")
    d = sim.diagnostics(0)
    assert d["continuity"] < 1e-5
    assert d["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-4)
    sim.close()


def test_moving_window_drops_what_does_not_fit():
    """With fewer dead slots than fresh particles the surplus is counted, not written, and
    the box keeps stepping."""
    banner("moving window, no room")
    wl = _box(pad=40, seed=65)
    sim = Simulation(wl, prec=L.F32_CELLOFS, tiling=(8, 8, 1), halo=4, chunk=128,
                     sort_interval=2, diag_interval=2, use_graph=False)
    sim.step(2)
    sim.window_shift(0, 2, PLASMA)   # 2 columns x 16 rows x 4 = 128 fresh, room for 40 + the
    sim.step(2)                      # particles of the 2 columns that left (after a sort)
    shifted, dropped = sim.window_info(0)
    assert shifted == 2 and dropped == 128 - 40
    cur = sim.current(0)
    assert (cur.numpy("cell") >= 0).sum() <= cur.n
    assert sim.diagnostics(0)["continuity"] < 1e-5
    sim.close()
