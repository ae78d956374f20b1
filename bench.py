"""Throughput of the PIC hot path on one MI355X: particle pushes per second.

A step is one full pass of Algorithm 1 (Sec. 3.3) through lpic_step: field half updates,
tile sort (every K steps), fused gather + Boris push + Esirkepov deposit over all species,
field half updates, FP64 diagnostics every 10 steps.  A push is one alive macro-particle
advanced through gather + push + deposit.

Workload (default): 2D3V 2048x1024 Yee grid, dx = lambda/32, fully ionised hydrogen slab of
20 n_c in cells x in [512, 768), electrons + protons at 32 ppc each (16,777,216 particles),
T = 1 keV, quadratic shape, linearly polarised a0 = 10 Gaussian laser (waist 6.25 lambda,
sin^2 envelope of 25 lambda / c) injected by an antenna 4 cells inside the left absorbing
layer, open x ends with 16-cell graded convolutional PML layers (the absorbing boundaries
of Sec. 3.2; --pml 0: first-order Mur ends), periodic y, seeded synthetic data.  The FP32 cell+offset path is `value`;
the plain FP64 path is reported beside it.

Timing: after the warmup steps (and alignment to a sort period), K steps run eagerly with HIP
events around every fused launch (the kernel's average launch time for the roofline), then,
after one untimed period that captures every step variant, the same K steps replay from the
captured graphs, the library's default mode: that pass is `value` and `ms_per_step`
(`eager_mode` reports the first one; --no-graph makes it `value`).

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
KERNEL_SOURCES = ("paper_2607_13507_amd/csrc/lpic_device.hpp",
                  "paper_2607_13507_amd/csrc/lpic_fused.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "fused_laser_slab_2048x1024_pmc.md")


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


def read_traffic(launch_bytes_key="per_launch_bytes"):
    """HBM bytes per fused launch from the committed PMC summary, if it was taken on the
    current kernel source (else None)."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    vals = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals[launch_bytes_key])
    except (KeyError, ValueError):
        return None


def build_workload(args):
    """(list of runs, description, ndim, particles per occupied cell of each run)."""
    from paper_2607_13507_amd import workloads as W
    if args.workload == "laser_slab":
        wl = W.laser_slab_2d(nx=args.nx, ny=args.ny, slab=(args.nx // 4, args.nx * 3 // 8),
                             ppc=args.ppc, steps=args.steps, pml_cells=args.pml)
        ends = (f"open x ends with {args.pml}-cell graded PML layers" if args.pml else
                "open x ends (first-order Mur)")
        desc = (f"laser_slab_2d {args.nx}x{args.ny} dx=lambda/32, H slab 20 n_c cells x in "
                f"[{args.nx // 4},{args.nx * 3 // 8}), e- + p+ {args.ppc} ppc each "
                f"({wl.nparticles} particles), T=1 keV, quadratic, a0=10 laser injected at the "
                f"open left end (antenna, waist 6.25 lambda, 25 lambda sin^2), {ends}, "
                "FP32 cell+offset")
        return [wl], desc, 2, [2 * args.ppc]
    if args.workload == "thermal_3d":
        wl = W.thermal_3d()
        desc = (f"thermal_3d 256^3 dx=0.1 c/omega_p, electrons 8 ppc ({wl.nparticles} "
                "particles) on a fixed ion background, T=0.05, quadratic, periodic, "
                "FP32 cell+offset")
        return [wl], desc, 3, [8]
    if args.workload == "wakefield":
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
            "128^2..1024x512, ppc 4-32, CIC/quadratic, lasers from the left, one step of all "
            "of them per launch, FP32 cell+offset")
    return members, desc, 2, [2 * m.meta["ppc"] for m in members]


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


def run_gpu(wl, prec, args, steps, warmup, tune):
    import torch
    from paper_2607_13507_amd import lpic as L
    from paper_2607_13507_amd.simulation import Simulation

    ty, halo = args.tile, args.halo
    if wl[0].ndim == 3:   # a 3D region with its charge planes must fit one CU's LDS
        ty = max(1, args.tile // 2)
        if prec == L.F64_ABS:
            halo = max(3, halo - 1)
    tiling, chunk, sort_interval = (args.tile, ty, args.tile_z), args.chunk, args.sort_interval
    tuned = None
    if tune:
        # the autotuner (lpic_autotune) times each candidate over whole sort and diagnostics
        # periods and keeps the fastest per step; it advances the simulation it tunes, so it
        # runs on a copy and the measured run starts from the workload's initial state
        if wl[0].ndim == 2:
            cands = [dict(tiling=(16, 16, 1), halo=5, chunk=ch, sort_interval=k, use_graph=True)
                     for k in (20, 40) for ch in (1024, 2048)]
            cands.append(dict(tiling=(16, 16, 1), halo=6, chunk=1024, sort_interval=40,
                              use_graph=True))
        else:   # a 3D tile region with its charge planes fills most of one CU's LDS
            cands = [dict(tiling=(8, 4, 4), halo=halo, chunk=2048, sort_interval=k,
                          use_graph=True) for k in (5, 10, 20)]
        tsim = Simulation(wl, prec=prec, tiling=tiling, halo=halo, chunk=chunk,
                          sort_interval=sort_interval, diag_interval=10, use_graph=True)
        tuned = tsim.autotune(cands, steps_each=40 if wl[0].ndim == 2 else 10)
        tsim.close()
        del tsim
        torch.cuda.empty_cache()
        tiling, halo, chunk, sort_interval = (tuned["tiling"], tuned["halo"], tuned["chunk"],
                                              tuned["sort_interval"])
    sim = Simulation(wl, prec=prec, tiling=tiling, halo=halo, chunk=chunk,
                     sort_interval=sort_interval, diag_interval=10, use_graph=not args.no_graph)
    advance(sim, wl, warmup)
    # the timed steps start where a sort and a diagnostics step fall together, so that the
    # window holds at least its proportional share of both (whole periods: exactly)
    k = sim.options.sort_interval
    period = k // math.gcd(k, 10) * 10
    advance(sim, wl, (-sim.nstep) % period)
    torch.cuda.synchronize()
    # timed region: eager launches with HIP events around every fused launch
    sim.set_timing(True)
    n0 = alive(sim)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(sim, wl, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sim.stats()
    sim.set_timing(False)
    n = 0.5 * (n0 + alive(sim))   # pushes per step (a moving window adds particles)
    # the same number of steps again as captured graphs (no per-kernel events), after one
    # untimed sort period in graph mode so that every step variant is already captured
    if not args.no_graph:
        advance(sim, wl, period + (-(sim.nstep + period)) % period)
    torch.cuda.synchronize()
    ng0 = alive(sim)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    if not args.no_graph:
        advance(sim, wl, steps)
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    ng = 0.5 * (ng0 + alive(sim))
    diag = sim.diagnostics(0)
    stg = sim.stats()
    res = dict(ms_per_step=1e3 * (t1 - t0) / steps,
               pushes_per_s=n * steps / (t1 - t0),
               alive=int(n),
               ms_per_step_graph=None if args.no_graph else 1e3 * (g1 - g0) / steps,
               pushes_per_s_graph=None if args.no_graph else ng * steps / (g1 - g0),
               fused_ms=st["fused_ms"] / max(1, st["fused_launches"]),
               fused_launches=st["fused_launches"],
               halo_escapes_per_push=stg["halo_escapes"] / max(1, n * stg["steps"]),
               window_cells=sim.window_info(0)[0] if wl[0].ndim == 2 else 0,
               graph=stg["graph"], diagnostics=diag, tuned=tuned,
               options=dict(tile=sim.options.tiling.tx, halo=sim.options.tiling.halo,
                            chunk=sim.options.tiling.chunk,
                            sort_interval=sim.options.sort_interval))
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return res


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


def host_cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(wl):
    """The FP64 oracle (single thread) on one full step of the same workload."""
    import oracle
    orc = oracle.OracleSim.from_workload(wl)
    t0 = time.perf_counter()
    orc.step(1)
    dt = time.perf_counter() - t0
    return dict(value=wl.nparticles / dt, unit="particle-pushes/s", cores=1, kind="oracle",
                sample=f"one full step (all {wl.nparticles} particles, {wl.nx}x{wl.ny} grid) "
                       f"of the benchmark workload, FP64, single thread on {host_cpu()} "
                       f"({os.cpu_count()} logical CPUs visible), {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=2048)
    ap.add_argument("--ny", type=int, default=1024)
    ap.add_argument("--ppc", type=int, default=32)
    ap.add_argument("--workload", default="laser_slab",
                    choices=("laser_slab", "thermal_3d", "wakefield", "ensemble"),
                    help="laser_slab (default, the headline configuration); the others are "
                         "extra measurements")
    ap.add_argument("--pml", type=int, default=16, metavar="CELLS",
                    help="laser_slab: graded PML layers of CELLS cells at the open x ends, "
                         "the antenna 4 cells inside the left one (0: first-order Mur ends, "
                         "the antenna 4 cells from the left end)")
    ap.add_argument("--tile", type=int, default=None)
    ap.add_argument("--tile-z", type=int, default=None)
    ap.add_argument("--halo", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=2048)
    ap.add_argument("--sort-interval", type=int, default=None)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the fixed tile / halo / chunk / sort interval instead of the "
                         "autotuner's pick")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="eager launches only (profiler passes)")
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

    wl, desc, ndim, ppc_tot = build_workload(args)
    if args.tile is None:
        args.tile = 16 if ndim == 2 else 8
    if args.tile_z is None:
        args.tile_z = 1 if ndim == 2 else 4
    if args.halo is None:
        args.halo = 5 if ndim == 2 else 4
    if args.sort_interval is None:
        args.sort_interval = 20   # the sort interval the 3D thermal configuration fixes
    nparticles = sum(w.nparticles for w in wl)
    tune = not args.no_autotune
    f32 = run_gpu(wl, L.F32_CELLOFS, args, args.steps, args.warmup, tune)
    f64 = None
    if not args.no_fp64:
        s64 = max(5, args.steps // 5)
        f64 = run_gpu(wl, L.F64_ABS, args, s64, max(2, args.warmup // 5), tune)

    slots = nparticles
    nparticles = f32["alive"]   # alive macro-particles per timed step (dead slots excluded)

    def launch_bytes_of(f32_path):
        # particle state in and out once per particle; E, B in and J out once per occupied cell
        return sum(algorithmic_bytes_per_push(ndim, f32_path, p) * w.nparticles
                   for w, p in zip(wl, ppc_tot)) * nparticles / slots
    launch_bytes = launch_bytes_of(True)
    bpp = launch_bytes / nparticles
    achieved = launch_bytes / (f32["fused_ms"] * 1e-3) / 1e9
    traffic = read_traffic() if args.workload == "laser_slab" else None
    valu = read_traffic("valu_insts_per_launch") if args.workload == "laser_slab" else None
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=f"lpic::k_fused<float,{ndim}>", bytes_per_push=round(bpp, 3),
                bytes_per_launch=int(launch_bytes), avg_launch_ms=round(f32["fused_ms"], 4),
                launches=f32["fused_launches"], kernel_source_sha256=kernel_source_hash())
    roof["copy_gbs"] = copy_bandwidth()   # measured, for context (not the peak)
    if valu:
        # the unit that binds this kernel: VALU issue.  A wave64 VALU instruction occupies a
        # SIMD for 4 cycles; 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G wave-instructions/s
        rate = valu / (f32["fused_ms"] * 1e-3)
        roof["valu_issue"] = dict(insts_per_launch=int(valu), achieved=round(rate / 1e9, 1),
                                  peak=614.4, unit="G wave-instructions/s",
                                  frac=round(rate / 614.4e9, 4))
    cpu = None
    if not args.no_cpu_baseline and args.workload == "laser_slab":
        cpu = cpu_baseline(wl[0])
    # `value` is the simulation as it runs by default: K steps replayed from captured graphs
    # (the eager pass before them records HIP events around every fused launch for the
    # roofline, which costs launch time of its own); --no-graph reports the eager pass
    graph = not args.no_graph
    key = "_graph" if graph else ""
    out = {
        "metric": "particle-pushes/sec (gather+push+deposit) FP32 vs FP64, % HBM roofline",
        "value": round(f32["pushes_per_s" + key], 1),
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step" + key], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc,
                   "particles": nparticles, "runs": len(wl),
                   "grid": [wl[0].nx, wl[0].ny] + ([wl[0].nz] if ndim == 3 else []),
                   "sort_interval": f32["options"]["sort_interval"],
                   "diag_interval": 10, "tiling": f32["options"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fused_pushes_per_s": round(nparticles / (f32["fused_ms"] * 1e-3), 1),
        "timed_mode": "graph replay" if graph else "eager",
        "eager_mode": {"ms_per_step": round(f32["ms_per_step"], 4),
                       "pushes_per_s": round(f32["pushes_per_s"], 1),
                       "note": "the same K steps launched one by one, with HIP events around "
                               "every fused launch (the source of avg_launch_ms)"},
        "halo_escapes_per_push": f32["halo_escapes_per_push"],
        "diagnostics_fp32": f32["diagnostics"],
    }
    if f64:
        out["fp64"] = {"pushes_per_s": round(f64["pushes_per_s" + key], 1),
                       "ms_per_step": round(f64["ms_per_step" + key], 4),
                       "fused_avg_ms": round(f64["fused_ms"], 4),
                       "fused_hbm_gbs": round(launch_bytes_of(False) /
                                              (f64["fused_ms"] * 1e-3) / 1e9, 1),
                       "eager_pushes_per_s": round(f64["pushes_per_s"], 1),
                       "fp32_over_fp64": round(f32["pushes_per_s" + key] /
                                               f64["pushes_per_s" + key], 3),
                       "diagnostics": f64["diagnostics"]}
    if f32["tuned"]:
        out["autotuned"] = f32["tuned"]
    if f32.get("window_cells"):
        out["config"]["window_cells_moved"] = f32["window_cells"]
    if args.copy_calibration > 0:
        out["copy_calibration"] = copy_calibration(args.copy_calibration)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
