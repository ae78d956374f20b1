"""Throughput of the PIC hot path on one MI355X: particle pushes per second.

A step is one full pass of Algorithm 1 (Sec. 3.3) through lpic_step: field half updates,
tile sort (every K steps), fused gather + Boris push + Esirkepov deposit over all species,
field half updates, FP64 diagnostics every 10 steps.  A push is one alive macro-particle
advanced through gather + push + deposit.

Headline workload (default): the batched ensemble of 64 independent 2D3V laser-slab runs
drawn from seed 4 (grids 128x128 .. 1024x512, ppc 4-32 per species, slab density 0.1-10
n_c, a0 0.5-20 injected from the left, CIC or quadratic, 179,609,600 particles), all of them
advanced by one launch per kernel and one captured graph per step, options chosen by the
library's autotuner.  It is the largest configuration of the metric that fits one GPU.

Also measured, each with its own roofline and CPU baseline (keys of "extra"):
  laser_slab              2D3V 2048x1024, H slab 20 n_c, e- + p+ 32 ppc (16,777,216), quadratic,
                          a0 = 10 antenna inside a 16-cell PML layer: the first steps;
  laser_slab_interaction  the same box timed from step 1200, when the pulse is inside the
                          slab (relativistic hot electrons, particles leaving their tiles);
                          the escape path is chosen again for this phase (the re-binned
                          path on and off, tried on a copy advanced to the same step);
  thermal_3d              3D3V periodic 256^3, 8 ppc (134,217,728), T = 0.05, quadratic, sort
                          every 20 steps as the configuration states;
  wakefield               2D3V 8192x512, 0.01 n_c at 4 ppc, a0 = 2, window moving with light;
  qed                     the QED event Monte-Carlo of Sec. 3.4 at the laser-slab scale:
                          16,777,216 electrons (gamma 500-2000, isotropic) on 2048x2048 cells
                          in a 300 m_e w c / e magnetic field with 20% random E and B
                          (quantum parameters ~0.1-3), one emission gather-push launch per
                          step, and 16,777,216 photons (|k| 1000-4000 m_e c) in a 2000-unit
                          field for the pair push, the converted photons compacted out
                          between launches; launches timed with HIP events, records
                          written to caller buffers.

Every configuration runs the FP32 cell+offset path (`value`) and the plain FP64 path beside
it.  Timing: after the warmup steps (and alignment to a sort period), K steps run eagerly
with HIP events around every fused launch (the kernel's average launch time for the
roofline), then, after one untimed period that captures every step variant, the same K
steps replay from the captured graphs, the library's default mode: that pass is the rate.

Output: one JSON line.  The benchmark runs on one GPU; with --gpus > 1 it exits (the
multi-GPU decomposition is a design, not implemented).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
VALU_PEAK = 614.4e9            # wave64 VALU instructions/s: 256 CUs x 4 SIMDs x 2.4 GHz / 4
KERNEL_SOURCES = ("paper_2607_13507_amd/csrc/lpic_device.hpp",
                  "paper_2607_13507_amd/csrc/lpic_fused.hip")
METRIC = "particle-pushes/sec (gather+push+deposit) FP32 vs FP64, % HBM roofline"
WORKLOADS = ("ensemble", "laser_slab", "thermal_3d", "wakefield")
INTERACTION_STEP = 1200        # the laser slab's pulse is inside the slab by then


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_push(ndim, prec_f32, ppc_tot):
    """Bytes the method must move per push (particle state in and out once; E, B read and J
    written once per cell, amortised over the particles per cell)."""
    if prec_f32:
        part = 52 if ndim == 2 else 60
        grid = 36
    else:
        part = 88 if ndim == 2 else 104
        grid = 72
    return part + grid / ppc_tot


def read_summary(name, key):
    """A value from a committed PMC summary (profiles/fused_<name>_pmc.md), if it was taken
    on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"fused_{name}_pmc.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------------------------------------------
# workloads
# ------------------------------------------------------------------------------------------
def build_workload(name):
    """(list of runs, description, ndim, particles per occupied cell of each run)."""
    from paper_2607_13507_amd import workloads as W
    if name == "laser_slab":
        wl = W.laser_slab_2d(pml_cells=16)
        desc = ("laser_slab_2d 2048x1024 dx=lambda/32, H slab 20 n_c cells x in [512,768), "
                f"e- + p+ 32 ppc each ({wl.nparticles} particles), T=1 keV, quadratic, a0=10 "
                "laser injected at the open left end (antenna, waist 6.25 lambda, 25 lambda "
                "sin^2), open x ends with 16-cell graded PML layers, FP32 cell+offset")
        return [wl], desc, 2, [64]
    if name == "thermal_3d":
        wl = W.thermal_3d()
        desc = (f"thermal_3d 256^3 dx=0.1 c/omega_p, electrons 8 ppc ({wl.nparticles} "
                "particles) on a fixed ion background, T=0.05, quadratic, periodic, sort every "
                "20 steps, FP32 cell+offset")
        return [wl], desc, 3, [8]
    if name == "wakefield":
        wl = W.wakefield_2d(moving=True)
        alive0 = int((wl.species[0].x >= 0).sum())
        desc = (f"wakefield_2d 8192x512 dx=lambda/40, electrons 0.01 n_c 4 ppc on a 2x2 "
                f"lattice ({alive0} at start) on fixed ions, a0=2 waist 8 lambda pulse, "
                "window moving with light (open x ends; fresh plasma injected at the leading "
                "edge at every sort), quadratic, FP32 cell+offset")
        return [wl], desc, 2, [4]
    members = W.ensemble_2d(seed=4, members=64)
    n = sum(m.nparticles for m in members)
    desc = (f"ensemble_2d 64 independent laser-slab runs from seed 4 ({n} particles), grids "
            "128^2..1024x512, ppc 4-32 per species, density 0.1-10 n_c, a0 0.5-20 injected "
            "from the left, CIC/quadratic, one launch per kernel for all runs, FP32 cell+offset")
    return members, desc, 2, [2 * m.meta["ppc"] for m in members]


def tune_space(name, ndim, f32):
    """Search space of the autotuner (lpic_autotune_search) per workload: tile edges, halo,
    chunk, sort interval and the re-binned escape path (tried on and off)."""
    if ndim == 3:   # sort every 20 steps, as the 3D configuration states
        return dict(tile=((4, 4, 4), (8, 8, 8)), halo=(3, 5 if f32 else 4), chunk=(1024, 4096),
                    sort_interval=(20, 20), rebin=2, steps_each=20, max_trials=10)
    return dict(tile=((8, 8, 1), (32, 32, 1)), halo=(3, 7), chunk=(512, 4096),
                sort_interval=(10, 80), rebin=2, steps_each=40, max_trials=24 if f32 else 12)


def start_options(ndim, f32):
    """The autotuner's starting point (and the options of --no-autotune)."""
    from paper_2607_13507_amd import lpic as L
    if ndim == 3:   # halo 3: two workgroups per CU; at 20 steps per sort ~11% of the pushes
        # leave their tile's margin and go through the re-binned second pass
        return dict(tiling=(8, 4, 4), halo=3, chunk=2048, sort_interval=20,
                    flags=L.ESCAPE_REBIN)
    return dict(tiling=(16, 16, 1), halo=5, chunk=1024, sort_interval=20, flags=0)


def alive(sim):
    """Alive macro-particles of all species (dead slots excluded)."""
    from paper_2607_13507_amd import lpic as L
    n = 0
    for i in range(len(sim.species)):
        cur = sim.current(i)
        key = "cell" if sim.prec == L.F32_CELLOFS else "x"
        n += int((cur.a[key] >= 0).sum().item())
    return n


def advance(sim, wl, n):
    """n steps; a box with a moving window moves with light at every sort boundary (its
    fresh plasma then meets the regular sort), by the whole cells light has gained."""
    win = wl[0].meta.get("window") if len(wl) == 1 else None
    if not win:
        sim.step(n)
        return
    k = sim.options.sort_interval
    while n > 0:
        take = min(n, k - sim.nstep % k)
        sim.step(take)
        n -= take
        if sim.nstep % k == 0:
            m = int(sim.nstep * win["cells_per_step"]) - sim.window_info(0)[0]
            if m >= 1:
                sim.window_shift(0, m, win["plasma"])


# ------------------------------------------------------------------------------------------
# GPU measurement
# ------------------------------------------------------------------------------------------
def timed_window(sim, wl, steps, graph):
    """K steps eagerly with HIP events around every fused launch, then (graph) one untimed
    period in graph mode and the same K steps replayed from the captured graphs."""
    import torch
    k = sim.options.sort_interval
    period = k // math.gcd(k, 10) * 10
    sim.set_timing(True)
    n0 = alive(sim)
    e0 = sim.stats()["halo_escapes"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(sim, wl, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sim.stats()
    sim.set_timing(False)
    n = 0.5 * (n0 + alive(sim))   # pushes per step (a moving window adds particles)
    res = dict(eager_ms_per_step=1e3 * (t1 - t0) / steps, eager_pushes_per_s=n * steps / (t1 - t0),
               alive=int(n), fused_ms=st["fused_ms"] / max(1, st["fused_launches"]),
               fused_launches=st["fused_launches"],
               halo_escapes_per_push=(st["halo_escapes"] - e0) / max(1.0, n * steps))
    res["ms_per_step"], res["pushes_per_s"] = res["eager_ms_per_step"], res["eager_pushes_per_s"]
    if graph:
        advance(sim, wl, period + (-(sim.nstep + period)) % period)
        torch.cuda.synchronize()
        ng0 = alive(sim)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        advance(sim, wl, steps)
        torch.cuda.synchronize()
        g1 = time.perf_counter()
        ng = 0.5 * (ng0 + alive(sim))
        res["ms_per_step"] = 1e3 * (g1 - g0) / steps
        res["pushes_per_s"] = ng * steps / (g1 - g0)
    res["step_at_end"] = sim.nstep
    res["diagnostics"] = sim.diagnostics(0)
    return res


def run_gpu(name, wl, ndim, prec, args, steps, warmup, tune, interaction=False):
    import torch
    from paper_2607_13507_amd import lpic as L
    from paper_2607_13507_amd.simulation import Simulation

    f32 = prec == L.F32_CELLOFS
    opt = start_options(ndim, f32)
    if args.tile:
        opt["tiling"] = tuple(args.tile)
    for key in ("halo", "chunk", "sort_interval"):
        if getattr(args, key) is not None:
            opt[key] = getattr(args, key)
    if args.rebin is not None:
        opt["flags"] = L.ESCAPE_REBIN if args.rebin else 0
    tuned, trials = None, []
    if tune:
        # lpic_autotune_search advances the simulation it tunes, so it runs on a copy and
        # the measured run starts from the workload's initial state
        tsim = Simulation(wl, prec=prec, tiling=opt["tiling"], halo=opt["halo"],
                          chunk=opt["chunk"], sort_interval=opt["sort_interval"],
                          diag_interval=10, use_graph=True, flags=opt["flags"])
        tuned, trials = tsim.autotune_search(**tune_space(name, ndim, f32))
        tsim.close()
        del tsim
        torch.cuda.empty_cache()
        opt = dict(tiling=tuned["tiling"], halo=tuned["halo"], chunk=tuned["chunk"],
                   sort_interval=tuned["sort_interval"], flags=tuned["flags"])
    sim = Simulation(wl, prec=prec, tiling=opt["tiling"], halo=opt["halo"], chunk=opt["chunk"],
                     sort_interval=opt["sort_interval"], diag_interval=10,
                     use_graph=not args.no_graph, flags=opt["flags"])
    advance(sim, wl, warmup)
    # the timed steps start where a sort and a diagnostics step fall together, so that the
    # window holds at least its proportional share of both (whole periods: exactly)
    k = sim.options.sort_interval
    period = k // math.gcd(k, 10) * 10
    advance(sim, wl, (-sim.nstep) % period)
    def opts_now():
        t = sim.options.tiling
        return dict(tiling=[t.tx, t.ty, t.tz], halo=t.halo, chunk=t.chunk,
                    sort_interval=sim.options.sort_interval,
                    escape_rebin=bool(t.flags & L.ESCAPE_REBIN))

    out = dict(start=timed_window(sim, wl, steps, not args.no_graph))
    out["start"]["options"] = opts_now()
    if interaction:
        advance(sim, wl, max(0, INTERACTION_STEP - sim.nstep))
        advance(sim, wl, (-sim.nstep) % period)
        if tune:
            # the escape path is chosen again for this phase (particles now leave their
            # tiles): a copy advanced to the same step tries it on and off, and the measured
            # run takes the faster setting
            t = sim.options.tiling
            tsim = Simulation(wl, prec=prec, tiling=(t.tx, t.ty, t.tz), halo=t.halo,
                              chunk=t.chunk, sort_interval=k, diag_interval=10,
                              use_graph=True, flags=t.flags)
            advance(tsim, wl, sim.nstep)
            tuned_i, trials_i = tsim.autotune_search(
                tile=((t.tx, t.ty, t.tz), (t.tx, t.ty, t.tz)), halo=(t.halo, t.halo),
                chunk=(t.chunk, t.chunk), sort_interval=(k, k), rebin=2, steps_each=k,
                max_trials=2)
            tsim.close()
            del tsim
            torch.cuda.empty_cache()
            out["interaction_tuned"] = dict(tuned_i, trials=trials_i)
            if tuned_i["flags"] != t.flags:
                sim.set_options(flags=tuned_i["flags"])
                advance(sim, wl, period)      # settle: the new options sort first
        out["interaction"] = timed_window(sim, wl, steps, not args.no_graph)
        out["interaction"]["options"] = opts_now()
    out["tuned"] = tuned
    out["tune_trials"] = trials
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def copy_calibration(mib):
    """A plain elementwise copy of known size (read mib MiB, write mib MiB), launched three
    times, against which the HBM byte counters of a profiler pass are scaled."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    return dict(kernel="elementwise mul by 1 (float32)", bytes_read=n * 4, bytes_written=n * 4,
                launches=3)


def copy_bandwidth(mib=1024, reps=5):
    """GB/s of a plain device-to-device copy of mib MiB (bytes read + bytes written per
    second), timed with events: the practical HBM rate beside the 8 TB/s peak."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(gbs, 1)


# ------------------------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host
# ------------------------------------------------------------------------------------------
def host_cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def host_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_sample(wls, target):
    """Oracle simulations holding about `target` particles of the workload: whole boxes in
    order, the last one (or a single box) cut to its first particles of every species (the
    generators lay particles out cell by cell, so a cut keeps whole cells)."""
    import numpy as np
    import oracle
    sims, taken = [], 0
    for wl in wls:
        if taken >= target:
            break
        orc = oracle.OracleSim.from_workload(wl, with_rho=False)
        if taken + wl.nparticles > target:
            frac = (target - taken) / wl.nparticles
            for s in orc.species:
                m = max(1, int(s.n * frac))
                for k in ("x", "y", "z", "ux", "uy", "uz", "w"):
                    a = getattr(s, k)
                    if a is not None:
                        setattr(s, k, np.ascontiguousarray(a[:m]))
        alive_n = sum(int((s.x >= 0).sum()) for s in orc.species)
        sims.append(orc)
        taken += alive_n
    return sims, taken


def cpu_baseline(name, wls):
    """The FP64 oracle as it is, one step of a bounded sample of the workload: once on one
    thread (the parity mode) and once with its particle loop on every host thread
    (orc_step_threads: private current arrays per thread, added afterwards)."""
    nthreads = host_threads()
    single_target = 3_000_000 if name == "thermal_3d" else 12_000_000
    multi_target = min(sum(w.nparticles for w in wls),
                       (4_000_000 if name == "thermal_3d" else 16_000_000) * max(1, nthreads // 2))
    sims, n1 = _oracle_sample(wls, single_target)
    t0 = time.perf_counter()
    for s in sims:
        s.step(1)
    t1 = time.perf_counter() - t0
    del sims
    sims, nm = _oracle_sample(wls, multi_target)
    used = 1
    t0 = time.perf_counter()
    for s in sims:
        used = s.step_threads(1, nthreads)
    tm = time.perf_counter() - t0
    del sims
    what = "boxes" if len(wls) > 1 else "particles"
    return dict(value=round(nm / tm, 1), unit="particle-pushes/s", cores=used, kind="oracle",
                sample=f"one step of {nm} {name} particles ({what} taken in order up to that "
                       f"count, full grids), FP64, particle loop on {used} threads of "
                       f"{host_cpu()} ({nthreads} usable), {tm:.1f} s",
                single_thread=dict(value=round(n1 / t1, 1), cores=1,
                                   sample=f"one step of {n1} particles, one thread, {t1:.1f} s"))


# ------------------------------------------------------------------------------------------
# QED event Monte-Carlo (Sec. 3.4)
# ------------------------------------------------------------------------------------------
QED_HW = 2e-6                  # hbar w_r / (m_e c^2)
QED_SOURCES = ("paper_2607_13507_amd/csrc/lpic_qed.hip", "paper_2607_13507_amd/csrc/lpic_internal.hpp",
               "paper_2607_13507_amd/csrc/lpic_device.hpp")


def qed_traffic(kernel):
    """HBM bytes per launch of a QED kernel from the committed counter summary
    (profiles/qed_beam_stats.md, already divided by the copy calibration), if it was taken
    on the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", "qed_beam_stats.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in QED_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    text = open(path).read()
    if f"qed_source_sha256: {h.hexdigest()[:16]}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(f"- {kernel}: fetch "):
            parts = line.split()
            return int((float(parts[3]) + float(parts[6])) * 1e6)
    return None
QED_PAIR_HW = 2.5e-6


def qed_bytes(kind, events_per_push, per_cell):
    """Algorithmic bytes of one push of the QED kernels (FP32 cell+offset leptons, FP64
    records): particle words in and out, the optical depth in and out, E and B once per
    cell (per_cell particles share a cell), and the records the events write (76 B each:
    seven FP64 words and the source index)."""
    fields = 6 * 4 / per_cell
    if kind == "emit":   # read cell, 2 offsets, u, w; write cell, offsets, u, old state
        return 28 + 24 + 12 + 16 + fields + 76 * events_per_push
    # photons: read x, y, k, w, tau; write x, y, tau; two records per pair event
    return 56 + 24 + fields + 2 * 76 * events_per_push


class _QedBuf:
    def __init__(self, cap):
        import torch
        self.cap = cap
        self.t = {k: torch.zeros(cap, dtype=torch.float64, device="cuda")
                  for k in ("x", "y", "ux", "uy", "uz", "w", "tau")}
        self.src = torch.zeros(cap, dtype=torch.int32, device="cuda")
        self.count = torch.zeros(1, dtype=torch.int32, device="cuda")

    def struct(self):
        from paper_2607_13507_amd import lpic as L
        t = self.t
        return L.QedBuffer(self.cap, self.count.data_ptr(), t["x"].data_ptr(), t["y"].data_ptr(),
                           None, t["ux"].data_ptr(), t["uy"].data_ptr(), t["uz"].data_ptr(),
                           t["w"].data_ptr(), t["tau"].data_ptr(), self.src.data_ptr())


def measure_qed(args, want_cpu):
    import numpy as np
    import torch
    from paper_2607_13507_amd import lpic as L
    from paper_2607_13507_amd import workloads as W
    from paper_2607_13507_amd.simulation import DeviceFields, DeviceSpecies, grid_struct
    print("[bench] qed: building inputs", file=sys.stderr, flush=True)
    F32 = L.F32_CELLOFS
    launches = max(3, min(args.steps, 10))
    warm = 2
    tabs = L.lpic_qed_tables_create(1)
    stream = torch.cuda.current_stream()
    st = stream.cuda_stream

    def timed(launch, reset):
        ms = []
        for i in range(warm + launches):
            reset()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            launch(i)
            b.record(stream)
            b.synchronize()
            if i >= warm:
                ms.append(a.elapsed_time(b))
        return sum(ms) / len(ms)

    # emission: electrons in the strong field
    wl = W.qed_beam(ndim=2, n=2048, ppc=4, order=2, seed=11)
    grid = grid_struct(wl)
    F = DeviceFields(wl, F32, with_rho=False)
    sp = DeviceSpecies.from_init(grid, wl.species[0], F32)
    n = sp.n
    tau = torch.empty(n, dtype=torch.float64, device="cuda")
    L.lpic_qed_init_tau(tau.data_ptr(), n, 1, 0)
    ph = _QedBuf(n)
    old = torch.empty(L.lpic_old_state_bytes(2, n, F32), dtype=torch.uint8, device="cuda")
    counts = []

    def emit(i):
        L.lpic_qed_gather_push(grid, F.struct(), sp.struct(), tau.data_ptr(), tabs,
                               L.QedParams(QED_HW, 1, 1 + i), ph.struct(), old.data_ptr(),
                               old.numel(), F32, stream=st)

    def emit_reset():
        if ph.count.item() > 0:
            counts.append(int(ph.count.item()))
        ph.count.zero_()

    ms_emit = timed(emit, emit_reset)
    emit_reset()
    ev_emit = sum(counts[-launches:]) / launches / n

    def plain(i):   # the same particles through the gather-push without QED, for context
        L.lpic_gather_push(grid, F.struct(), sp.struct(), old.data_ptr(), old.numel(), F32,
                           stream=st)

    ms_plain = timed(plain, lambda: None)
    fields_f = F
    del ph, old, tau, sp
    # pairs: photons in a stronger field
    wl2 = W.qed_beam(ndim=2, n=2048, dx=0.5, b0=2000.0, ppc=1, order=2, seed=12)
    wl2.species = []
    grid2 = grid_struct(wl2)
    F2 = DeviceFields(wl2, F32, with_rho=False)
    m = n
    pos, kv, w = W.qed_photons(wl2, m, seed=13)
    phot = _QedBuf(m)
    for k, v in (("x", pos[0]), ("y", pos[1]), ("ux", kv[0]), ("uy", kv[1]), ("uz", kv[2]),
                 ("w", w)):
        phot.t[k].copy_(torch.from_numpy(np.ascontiguousarray(v)))
    phot.count.fill_(m)
    L.lpic_qed_init_tau(phot.t["tau"].data_ptr(), m, 2, 0)
    pairs = _QedBuf(m)
    spare = _QedBuf(m)
    ws = torch.empty(L.lpic_qed_compact_ws_bytes(m), dtype=torch.uint8, device="cuda")
    alive, pcounts, compact_ms = [], [], []
    bufs = [phot, spare]

    def pair(i):
        L.lpic_qed_photon_push(grid2, F2.struct(), 2, bufs[0].struct(), tabs,
                               L.QedParams(QED_PAIR_HW, 2, 1 + i), pairs.struct(), F32,
                               stream=st)

    def pair_reset():
        # the converted photons leave the buffer (stable compaction, timed on its own), so
        # every launch pushes live photons only
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        L.lpic_qed_compact(bufs[0].struct(), bufs[1].struct(), 2, ws.data_ptr(), ws.numel(),
                           stream=st)
        b.record(stream)
        b.synchronize()
        compact_ms.append(a.elapsed_time(b))
        bufs.reverse()
        alive.append(int(bufs[0].count.item()))
        if pairs.count.item() > 0:
            pcounts.append(int(pairs.count.item()) // 2)
        pairs.count.zero_()

    ms_pair = timed(pair, pair_reset)
    pair_reset()
    live = sum(alive[warm:warm + launches]) / launches
    ev_pair = sum(pcounts[-launches:]) / launches / live
    ms_compact = sum(compact_ms[warm:warm + launches]) / launches
    del phot, spare, pairs, bufs, ws, F2, fields_f, F
    L.lpic_qed_tables_destroy(tabs)

    def roof(kind, npush, ms, ev, kernel):
        b = qed_bytes(kind, ev, 4.0)
        gbs = b * npush / (ms * 1e-3) / 1e9
        return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(gbs / HBM_PEAK_GBS, 4),
                    traffic=qed_traffic(kernel.split("::")[1].split("<")[0]), kernel=kernel,
                    bytes_per_push=round(b, 3), avg_launch_ms=round(ms, 4), launches=launches)

    out = dict(workload="qed_beam 2048x2048 f32, 16,777,216 electrons; 16,777,216 photons",
               value=round(n / (ms_emit * 1e-3), 1), unit="particle-pushes/s",
               emission=dict(pushes_per_s=round(n / (ms_emit * 1e-3), 1),
                             avg_launch_ms=round(ms_emit, 4),
                             events_per_push=round(ev_emit, 5), hbar_omega=QED_HW,
                             plain_gather_push_ms=round(ms_plain, 4),
                             roofline=roof("emit", n, ms_emit, ev_emit, "lpic::k_qed_push<float,2>")),
               pairs=dict(pushes_per_s=round(live / (ms_pair * 1e-3), 1),
                          avg_launch_ms=round(ms_pair, 4), live_photons=int(live),
                          compaction_ms=round(ms_compact, 4),
                          events_per_push=round(ev_pair, 5), hbar_omega=QED_PAIR_HW,
                          roofline=roof("pair", live, ms_pair, ev_pair,
                                        "lpic::k_qed_photons<float,2>")))
    out["roofline"] = out["emission"]["roofline"]
    if want_cpu:
        out["cpu_baseline"] = qed_cpu_baseline(wl, wl2)
    return out


def qed_cpu_baseline(wl, wl2):
    """The oracle's QED push (single-threaded, each rate and quantile from its integrals)
    on the first 2000 electrons of the same workload and on 1000 photons."""
    import numpy as np
    import oracle
    from oracle import qed as Q
    from paper_2607_13507_amd import workloads as W
    print("[bench] qed: CPU baseline (oracle)", file=sys.stderr, flush=True)
    m = 2000
    orc = oracle.OracleSim.from_workload(wl, with_rho=False)
    s = orc.species[0]
    for k in ("x", "y", "ux", "uy", "uz", "w"):
        setattr(s, k, np.ascontiguousarray(getattr(s, k)[:m]))
    tau = Q.init_tau(m, 1, 0)
    buf = Q.QedBuf(m)
    t0 = time.perf_counter()
    Q.qed_gather_push(orc, s, tau, QED_HW, 1, 1, buf)
    t_emit = time.perf_counter() - t0
    del orc
    orc2 = oracle.OracleSim.from_workload(wl2, with_rho=False)
    k = 1000
    pos, kv, w = W.qed_photons(wl2, k, seed=13)
    ph = Q.QedBuf(k, count=k)
    ph.x[:], ph.y[:] = pos[0], pos[1]
    ph.ux[:], ph.uy[:], ph.uz[:] = kv
    ph.w[:] = w
    ph.tau[:] = Q.init_tau(k, 2, 0)
    pairs = Q.QedBuf(2 * k)
    t0 = time.perf_counter()
    Q.qed_photon_push(orc2, 2, ph, QED_PAIR_HW, 2, 1, pairs)
    t_pair = time.perf_counter() - t0
    return dict(value=round(m / t_emit, 1), unit="particle-pushes/s", cores=1, kind="oracle",
                sample=f"one emission gather-push of the first {m} electrons ({buf.count} "
                       f"events), FP64, one thread of {host_cpu()}, {t_emit:.1f} s",
                pairs=dict(value=round(k / t_pair, 1), cores=1,
                           sample=f"one photon push of {k} photons ({pairs.count // 2} pairs), "
                                  f"{t_pair:.1f} s"))


# ------------------------------------------------------------------------------------------
def roofline_of(name, ndim, wls, ppc_tot, res, launch_key="start"):
    """HBM roofline of the dominant kernel (k_fused, FP32) for one configuration."""
    w = res[launch_key]
    slots = sum(x.nparticles for x in wls)
    nparticles = w["alive"]
    launch_bytes = sum(algorithmic_bytes_per_push(ndim, True, p) * x.nparticles
                       for x, p in zip(wls, ppc_tot)) * nparticles / slots
    achieved = launch_bytes / (w["fused_ms"] * 1e-3) / 1e9
    key = name if launch_key == "start" else f"{name}_{launch_key}"
    traffic = read_summary(key, "per_launch_bytes")
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=f"lpic::k_fused<float,{ndim}>",
                bytes_per_push=round(launch_bytes / nparticles, 3),
                bytes_per_launch=int(launch_bytes), avg_launch_ms=round(w["fused_ms"], 4),
                launches=w["fused_launches"], kernel_source_sha256=kernel_source_hash())
    valu = read_summary(key, "valu_insts_per_launch")
    if valu:
        rate = valu / (w["fused_ms"] * 1e-3)
        roof["valu_issue"] = dict(insts_per_launch=int(valu), achieved=round(rate / 1e9, 1),
                                  peak=VALU_PEAK / 1e9, unit="G wave-instructions/s",
                                  frac=round(rate / VALU_PEAK, 4))
    return roof


def fp64_entry(ndim, wls, ppc_tot, r64, key="start"):
    w = r64[key]
    slots = sum(x.nparticles for x in wls)
    launch_bytes = sum(algorithmic_bytes_per_push(ndim, False, p) * x.nparticles
                       for x, p in zip(wls, ppc_tot)) * w["alive"] / slots
    gbs = launch_bytes / (w["fused_ms"] * 1e-3) / 1e9
    return dict(pushes_per_s=round(w["pushes_per_s"], 1), ms_per_step=round(w["ms_per_step"], 4),
                fused_avg_ms=round(w["fused_ms"], 4), kernel=f"lpic::k_fused<double,{ndim}>",
                bytes_per_push=round(launch_bytes / w["alive"], 3),
                fused_hbm_gbs=round(gbs, 1), fused_frac=round(gbs / HBM_PEAK_GBS, 4),
                halo_escapes_per_push=w["halo_escapes_per_push"], diagnostics=w["diagnostics"])


def measure(name, args, want_cpu):
    """Every number of one configuration: FP32 and FP64 paths, roofline, CPU baseline."""
    import gc
    from paper_2607_13507_amd import lpic as L
    wls, desc, ndim, ppc_tot = build_workload(name)
    tune = not args.no_autotune
    inter = name == "laser_slab" and not args.no_interaction
    print(f"[bench] {name}: FP32", file=sys.stderr, flush=True)
    r32 = run_gpu(name, wls, ndim, L.F32_CELLOFS, args, args.steps, args.warmup, tune, inter)
    r64 = None
    if not args.no_fp64:
        print(f"[bench] {name}: FP64", file=sys.stderr, flush=True)
        s64 = max(5, args.steps // 5)
        r64 = run_gpu(name, wls, ndim, L.F64_ABS, args, s64, max(2, args.warmup // 5), tune,
                      inter)
    windows = ["start"] + (["interaction"] if inter else [])
    entries = {}
    for key in windows:
        w = r32[key]
        e = dict(workload=desc + (f"; timed from step {INTERACTION_STEP}, the pulse inside the "
                                  "slab" if key == "interaction" else ""),
                 value=round(w["pushes_per_s"], 1), unit="particle-pushes/s",
                 ms_per_step=round(w["ms_per_step"], 4), particles=w["alive"], runs=len(wls),
                 last_timed_step=w["step_at_end"] - 1,
                 roofline=roofline_of(name, ndim, wls, ppc_tot, r32, key),
                 fused_pushes_per_s=round(w["alive"] / (w["fused_ms"] * 1e-3), 1),
                 eager_mode=dict(ms_per_step=round(w["eager_ms_per_step"], 4),
                                 pushes_per_s=round(w["eager_pushes_per_s"], 1)),
                 halo_escapes_per_push=w["halo_escapes_per_push"],
                 options=w["options"], diagnostics_fp32=w["diagnostics"])
        if r64:
            e["fp64"] = fp64_entry(ndim, wls, ppc_tot, r64, key)
            e["fp32_over_fp64"] = round(w["pushes_per_s"] / r64[key]["pushes_per_s"], 3)
        entries[key] = e
    head = entries["start"]
    if r32["tuned"]:
        head["autotuned"] = dict(r32["tuned"], trials=len(r32["tune_trials"]))
    if r64 and r64["tuned"]:
        head["autotuned_fp64"] = dict(r64["tuned"], trials=len(r64["tune_trials"]))
    if "interaction" in entries:
        for r, k in ((r32, "autotuned"), (r64, "autotuned_fp64")):
            if r and r.get("interaction_tuned"):
                it = r["interaction_tuned"]
                entries["interaction"][k] = dict(
                    {x: v for x, v in it.items() if x != "trials"},
                    trials=[dict(rebin=t["rebin"], ms_per_step=t["ms_per_step"])
                            for t in it["trials"]])
    gc.collect()
    return wls, entries, want_cpu


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default=None, choices=WORKLOADS,
                    help="measure one configuration only (it becomes the headline); default: "
                         "the ensemble as headline and the others as extra keys")
    ap.add_argument("--extra", default="laser_slab,thermal_3d,wakefield,qed",
                    help="comma-separated configurations measured beside the headline")
    ap.add_argument("--tile", type=int, nargs="+", default=None, metavar="T",
                    help="start (or, with --no-autotune, fixed) tile edges x y [z]")
    ap.add_argument("--halo", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=None)
    ap.add_argument("--sort-interval", type=int, default=None)
    ap.add_argument("--rebin", type=int, default=None, choices=(0, 1),
                    help="start (or fixed) setting of the re-binned escape path")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the start / given options instead of the autotuner's pick")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-interaction", action="store_true",
                    help="laser_slab: skip the window timed from step 1200")
    ap.add_argument("--no-graph", action="store_true",
                    help="eager launches only (profiler passes)")
    ap.add_argument("--qed-only", action="store_true",
                    help="measure the QED kernels only and print their entry (profiler runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain copy of this many MiB (profiler byte calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not implemented", file=sys.stderr)
        sys.exit(2)

    from paper_2607_13507_amd import lpic as L
    L.lib()   # the HIP library must be there; no fallback
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.qed_only:
        out = dict(qed=measure_qed(args, not args.no_cpu_baseline))
        if args.copy_calibration > 0:
            out["copy_calibration"] = copy_calibration(args.copy_calibration)
        print(json.dumps(out), flush=True)
        return
    head_name = args.workload or "ensemble"
    extras = [] if args.workload else [e for e in args.extra.split(",") if e]
    want_qed = "qed" in extras
    extras = [e for e in extras if e != "qed"]
    copy_gbs = copy_bandwidth()
    results, pending_cpu = {}, []
    for name in [head_name] + extras:
        wls, entries, _ = measure(name, args, not args.no_cpu_baseline)
        results[name] = entries
        if not args.no_cpu_baseline:
            pending_cpu.append((name, wls))   # oracle timings after all GPU work
        else:
            del wls
    for name, wls in pending_cpu:
        print(f"[bench] {name}: CPU baseline (oracle)", file=sys.stderr, flush=True)
        results[name]["start"]["cpu_baseline"] = cpu_baseline(name, wls)
    pending_cpu.clear()

    head = results[head_name]["start"]
    head["roofline"]["copy_gbs"] = copy_gbs
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": head["workload"], "particles": head["particles"],
                   "runs": head["runs"], "diag_interval": 10, "options": head["options"]},
        "roofline": head["roofline"],
        "cpu_baseline": head.get("cpu_baseline"),
        "timed_mode": "eager" if args.no_graph else "graph replay",
    }
    for k in ("fp64", "fp32_over_fp64", "fused_pushes_per_s", "eager_mode",
              "halo_escapes_per_push", "diagnostics_fp32", "autotuned", "autotuned_fp64"):
        if k in head:
            out[k] = head[k]
    extra = {}
    for key, e in results[head_name].items():
        if key != "start":
            extra[f"{head_name}_{key}"] = e
    for name in extras:
        for key, e in results[name].items():
            extra[name if key == "start" else f"{name}_{key}"] = e
    if want_qed:
        extra["qed"] = measure_qed(args, not args.no_cpu_baseline)
    if extra:
        out["extra"] = extra
    if args.copy_calibration > 0:
        out["copy_calibration"] = copy_calibration(args.copy_calibration)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
