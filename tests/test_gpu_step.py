"""Whole-step parity (Algorithm 1 through lpic_step) against the FP64 oracle, plus the
equivalences the orchestration must keep: graph vs eager, fused vs split (hooks), ensemble
member vs the same box alone, sort interval; hooks fire in stage order.

Tolerances as in test_gpu_kernels.py; FP32 runs are compared only over a few steps (thermal
PIC is chaotic, so FP32 and FP64 trajectories separate), and through the invariants
(continuity, Gauss) and deterministic workloads over long runs.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import banner, compare_fields, compare_particles
from oracle import OracleSim
from paper_2607_13507_amd import lpic as L
from paper_2607_13507_amd import workloads as W
from paper_2607_13507_amd.simulation import Callback, Simulation, callback

pytestmark = pytest.mark.gpu

FIELDS = ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz")


def _wl(order=2, nx=40, ny=36, ppc=4, T=0.05, seed=8):
    return W.thermal_2d(nx=nx, ny=ny, dx=0.05, ppc=ppc, T=T, order=order, seed=seed)


def _oracle_like_gpu(sim, wl):
    """Oracle starting from exactly the GPU's initial state (FP32 rounding included)."""
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


def _order_like(orc_s, sim, i):
    """The sort permutes particles: reorder the oracle's arrays to the GPU's order using the
    unique weight tags set by the test."""
    cur = sim.current(i)
    tags = cur.numpy("w").astype(np.float64)
    idx = np.argsort(orc_s.w)
    perm = idx[np.searchsorted(orc_s.w[idx], tags)]
    for k in ("x", "y", "z", "ux", "uy", "uz", "w"):
        a = getattr(orc_s, k)
        if a is not None:
            a[:] = a[perm]


def _tag_weights(wl):
    for s in wl.species:
        s.w = s.w * (1.0 + 1e-3 * np.arange(s.n) / s.n)   # unique, still ~n/ppc


@pytest.mark.parametrize("ndim,order", [(2, 1), (2, 2), (3, 2)])
@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_fp64_steps_match_oracle(ndim, order, graph):
    banner(f"f64 steps ndim={ndim} order={order} graph={graph}")
    wl = _wl(order) if ndim == 2 else W.thermal_3d(n=12, dx=0.1, ppc=2, T=0.05, order=order, seed=4)
    _tag_weights(wl)
    nsteps = 12
    tiling, halo = ((8, 8, 1), 4) if ndim == 2 else ((8, 4, 4), 3)
    sim = Simulation(wl, prec=L.F64_ABS, tiling=tiling, halo=halo, chunk=128, sort_interval=5,
                     diag_interval=3, use_graph=graph)
    orc = _oracle_like_gpu(sim, wl)
    sim.step(nsteps)
    orc.step(nsteps)
    torch.cuda.synchronize()
    compare_fields(sim.fields[0], orc, L.F64_ABS, tol=1e-10, what="fields")
    _order_like(orc.species[0], sim, 0)
    compare_particles(sim.grids[0], sim.current(0), orc.species[0], L.F64_ABS, tol_pos=1e-10,
                      tol_u=1e-10)
    d = sim.diagnostics(0)
    assert d["step"] == 12
    assert d["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-10)
    assert d["kinetic_energy"] == pytest.approx(orc.kinetic_energy(), rel=1e-10)
    assert d["continuity"] < 1e-12
    st = sim.stats()
    assert st["steps"] == nsteps and st["sorts"] == 3 and st["fused"]
    assert st["graph"] == graph
    sim.close()


@pytest.mark.parametrize("order", [1, 2])
def test_fp32_steps_track_oracle_and_conserve_charge(order):
    banner(f"f32 steps order={order}")
    wl = _wl(order, nx=48, ny=40, ppc=8, T=0.01)
    sim = Simulation(wl, prec=L.F32_CELLOFS, tiling=(16, 16, 1), halo=4, chunk=256,
                     sort_interval=4, diag_interval=1, use_graph=True)
    orc = _oracle_like_gpu(sim, wl)
    g1 = None
    for n in range(1, 21):
        sim.step(1)
        orc.step(1)
        d = sim.diagnostics(0)
        assert d["continuity"] < 1e-5, (n, d)             # charge conservation, FP32
        if n == 1:
            g1 = d["gauss"]
        if n <= 5:
            compare_fields(sim.fields[0], orc, L.F32_CELLOFS, tol=1e-4, what=f"step {n}")
            assert d["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-4)
            assert d["kinetic_energy"] == pytest.approx(orc.kinetic_energy(), rel=1e-5)
    # Gauss invariant: div E - (rho^n + rho^{n+1})/2 stays at its step-1 value per node
    f = sim.fields[0].numpy()
    ref = OracleSim(2, wl.nx, wl.ny, 1, wl.dx, wl.dy, 1.0, wl.dt, wl.rho_bg, [],
                    {k: f[k] for k in FIELDS})
    ref.rho0[:], ref.rho1[:] = f["rho0"], f["rho1"]
    assert abs(np.abs(ref.gauss()).max() - g1) < 1e-4 * max(1.0, g1)
    sim.close()


def test_vacuum_mode_fp32_energy_1000_steps():
    """Deterministic vacuum mode: FP32 field energy within 1e-4 of the FP64 oracle after
    1000 steps (normalised by the oracle's maximum field energy)."""
    banner("vacuum mode 1000 steps")
    wl = W.vacuum_mode(nx=64, ny=64, dx=0.05, mx=2, my=1, steps=1000)
    sim = Simulation(wl, prec=L.F32_CELLOFS, diag_interval=100, use_graph=True)
    orc = OracleSim.from_workload(wl)
    emax = 0.0
    for _ in range(10):
        sim.step(100)
        orc.step(100)
        e = orc.field_energy()
        emax = max(emax, e)
        assert abs(sim.diagnostics(0)["field_energy"] - e) <= 1e-4 * emax
    sim.close()


def test_cold_plasma_fp32_1000_steps():
    """Deterministic cold Langmuir oscillation: FP32 field energy within 1e-4 of the FP64
    oracle over 1000 steps (normalised by the oracle's maximum)."""
    banner("cold plasma 1000 steps")
    wl = W.cold_langmuir(nx=64, ny=4, dx=0.05, lattice=4, amp=1e-2, order=1, steps=1000)
    sim = Simulation(wl, prec=L.F32_CELLOFS, tiling=(16, 4, 1), halo=3, chunk=256,
                     sort_interval=20, diag_interval=50, use_graph=True)
    orc = _oracle_like_gpu(sim, wl)
    emax, worst = 0.0, 0.0
    for _ in range(20):
        sim.step(50)
        orc.step(50)
        e = orc.field_energy()
        emax = max(emax, e)
        worst = max(worst, abs(sim.diagnostics(0)["field_energy"] - e))
    assert worst <= 1e-4 * emax, worst / emax
    sim.close()


def test_split_path_and_hook_order():
    """A hook at an intermediate particle stage switches to the split kernels; the result
    equals the fused path's, and every stage fires in Algorithm 1 order."""
    banner("hooks / split path")
    wl = _wl(2)
    _tag_weights(wl)
    a = Simulation(wl, prec=L.F64_ABS, tiling=(8, 8, 1), chunk=64, sort_interval=3,
                   diag_interval=2, use_graph=True)
    b = Simulation(wl, prec=L.F64_ABS, tiling=(8, 8, 1), chunk=64, sort_interval=3,
                   diag_interval=2, use_graph=True)
    seen = []
    for st in L.STAGES:
        b.register_hook(st, lambda sim, stage, step: seen.append((step, stage)))
    a.step(4)
    b.step(4)
    torch.cuda.synchronize()
    fa, fb = a.fields[0].numpy(), b.fields[0].numpy()
    for k in FIELDS:
        scale = max(1e-300, np.abs(fa[k]).max())
        assert np.abs(fa[k] - fb[k]).max() / scale < 1e-12, k
    sa, sb = a.stats(), b.stats()
    assert sa["fused"] and sa["graph"] and not sb["fused"] and not sb["graph"]
    one_step = ["LOOP_START", "MAXWELL_1", "PUSH_POSITION_1", "INTERPOLATOR", "PUSH_MOMENTUM",
                "PUSH_POSITION_2", "CURRENT_DEPOSITION", "QED_CREATE", "MAXWELL_2", "LOOP_END"]
    stages = [s for _, s in seen]
    assert stages[0] == "START" and stages[-1] == "FINISH"
    assert stages[1:-1] == one_step * 4
    assert a.diagnostics(0)["field_energy"] == pytest.approx(b.diagnostics(0)["field_energy"], rel=1e-12)
    a.close()
    b.close()


def test_hook_can_modify_state_and_stop():
    banner("hook modifies / stops")
    wl = _wl(1)
    sim = Simulation(wl, prec=L.F32_CELLOFS, tiling=(8, 8, 1), chunk=64, use_graph=True)

    @callback(stage="LOOP_END", interval=2)
    def kick(s):
        s.fields[0].t["bz"].add_(1.0)

    sim.add_callback(kick)
    sim.step(4)
    torch.cuda.synchronize()
    assert sim.stats()["graph"]           # LOOP_END hooks run between graph launches
    # a stateful callback that fails stops the step with LPIC_EHOOK
    class Stop(Callback):
        stage = "MAXWELL_2"
        interval = 1

        def __call__(self, s):
            return 3

    sim.add_callback(Stop())
    with pytest.raises(L.LpicError) as e:
        sim.step(1)
    assert e.value.status == -5
    sim.close()


def test_ensemble_members_match_standalone_runs():
    banner("ensemble")
    members = W.ensemble_2d(seed=4, members=4, max_scale=8, steps=6)
    for m in members:
        _tag_weights(m)
    ens = Simulation(members, prec=L.F64_ABS, tiling=(8, 8, 1), halo=4, chunk=256,
                     sort_interval=3, diag_interval=2, use_graph=True)
    ens.step(6)
    torch.cuda.synchronize()
    for r, m in enumerate(members):
        orc = OracleSim.from_workload(m)
        orc.step(6)
        F = ens.fields[r]
        g = F.numpy()
        for k in FIELDS:
            scale = max(1e-300, np.abs(orc.f[k]).max())
            assert np.abs(g[k] - orc.f[k]).max() / scale < 1e-10, (r, k)
        d = ens.diagnostics(r)
        assert d["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-10)
        assert d["kinetic_energy"] == pytest.approx(orc.kinetic_energy(), rel=1e-10)
        assert d["continuity"] < 1e-12
    ens.close()


def test_sort_interval_does_not_change_physics():
    banner("sort interval")
    wl = _wl(2, T=0.2)
    runs = []
    for k in (1, 7):
        s = Simulation(wl, prec=L.F64_ABS, tiling=(8, 8, 1), halo=3, chunk=100, sort_interval=k,
                       use_graph=False)
        s.step(10)
        runs.append(s.fields[0].numpy())
        s.close()
    for k in FIELDS:
        scale = max(1e-300, np.abs(runs[0][k]).max())
        assert np.abs(runs[0][k] - runs[1][k]).max() / scale < 1e-12, k


def test_autotune_picks_a_candidate_and_keeps_physics():
    banner("autotune")
    wl = _wl(2)
    sim = Simulation(wl, prec=L.F64_ABS, use_graph=False, diag_interval=1)
    best = sim.autotune([dict(tiling=(8, 8, 1), chunk=64, sort_interval=2),
                         dict(tiling=(16, 16, 1), chunk=512, sort_interval=4),
                         dict(tiling=(128, 128, 1), chunk=512)], steps_each=2)
    assert best["tiling"] in [(8, 8, 1), (16, 16, 1)]       # the LDS-infeasible one is skipped
    n_done = sim.nstep
    orc = OracleSim.from_workload(wl)
    orc.step(n_done)
    sim.step(1)
    orc.step(1)
    assert sim.diagnostics(0)["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-10)
    sim.close()


def test_autotune_search_stays_in_its_space_and_keeps_physics():
    """lpic_autotune_search walks tile, halo, chunk, sort interval and the re-binned escape
    path inside the given bounds, times no option set twice, keeps the fastest, and the simulation it tuned goes
    on taking exactly the oracle's steps."""
    banner("autotune search")
    wl = _wl(2)
    sim = Simulation(wl, prec=L.F64_ABS, tiling=(16, 16, 1), halo=4, chunk=256,
                     sort_interval=4, use_graph=True, diag_interval=2)
    best, trials = sim.autotune_search(tile=((8, 8, 1), (16, 16, 1)), halo=(3, 5),
                                       chunk=(64, 512), sort_interval=(2, 8), steps_each=4,
                                       max_trials=12)
    assert 2 <= len(trials) <= 12
    keys = [(t["tiling"], t["halo"], t["chunk"], t["sort_interval"], t["rebin"]) for t in trials]
    assert len(set(keys)) == len(keys)
    for t in trials:
        assert t["tiling"][0] in (8, 16) and t["tiling"][1] in (8, 16)
        assert 3 <= t["halo"] <= 5 and 64 <= t["chunk"] <= 512 and 2 <= t["sort_interval"] <= 8
    fastest = min((t for t in trials if t["ms_per_step"] >= 0), key=lambda t: t["ms_per_step"])
    assert (best["tiling"], best["halo"], best["chunk"], best["sort_interval"]) == (
        fastest["tiling"], fastest["halo"], fastest["chunk"], fastest["sort_interval"])
    n_done = sim.nstep
    orc = OracleSim.from_workload(wl)
    orc.step(n_done)
    sim.step(2)
    orc.step(2)
    assert sim.diagnostics(0)["field_energy"] == pytest.approx(orc.field_energy(), rel=1e-10)
    sim.close()


@pytest.mark.parametrize("prec", [L.F64_ABS, L.F32_CELLOFS], ids=["f64", "f32"])
def test_small_thermal_configuration_100_steps_vs_oracle(prec):
    """The small thermal configuration as stated (64 x 64, dx = 0.05, 16 ppc, T = 0.01, CIC,
    100 steps, 65,536 electrons on a fixed ion background), all 100 steps in one call with
    graphs, against the oracle's 100 steps from the same state: fields element by element,
    field and kinetic energy, continuity (FP64: 1e-8 after 100 steps of round-off growth;
    FP32: 1e-4 tracking)."""
    banner(f"thermal 64x64 100 steps prec={'f64' if prec == L.F64_ABS else 'f32'}")
    wl = W.thermal_2d()
    assert wl.nparticles == 65_536 and wl.steps == 100
    sim = Simulation(wl, prec=prec, tiling=(16, 16, 1), halo=4, chunk=512, sort_interval=10,
                     diag_interval=100, use_graph=True)
    orc = _oracle_like_gpu(sim, wl)
    sim.step(100)
    orc.step(100)
    torch.cuda.synchronize()
    f64 = prec == L.F64_ABS
    tol = 1e-8 if f64 else 1e-4
    compare_fields(sim.fields[0], orc, prec, tol=tol, what="fields after 100 steps")
    d = sim.diagnostics(0)
    assert d["step"] == 100
    assert d["field_energy"] == pytest.approx(orc.field_energy(), rel=tol)
    assert d["kinetic_energy"] == pytest.approx(orc.kinetic_energy(), rel=tol)
    assert d["continuity"] < (1e-12 if f64 else 1e-5)
    sim.close()
