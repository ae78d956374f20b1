"""Writes the stored expected values of the long-run GPU tests, from the FP64 oracle only.

Each golden file holds what the oracle computes for a seeded synthetic input; nothing in
it comes from the HIP library.  Run from the repository root:

    python tests/golden/make_goldens.py [name ...]

Goldens:
  pulse_vacuum_2048x1024  The vacuum Gaussian pulse on the laser-slab grid (2048 x 1024,
                          dx = lambda/32, a0 = 10, periodic), started from its initial
                          fields rounded to FP32 (the values the FP32 path holds), stepped
                          1000 times by Algorithm 1: the field energy at every 100th step
                          and Ex, Ey, Bz at 64 seeded nodes after the last step.
  ensemble_deterministic  Every member of workloads.deterministic_ensemble() (vacuum
                          modes, a vacuum pulse, cold lattices, CIC and quadratic), started
                          from its inputs as the FP32 path holds them (fields, momenta and
                          weights rounded to FP32, positions as FP32 offsets in their
                          cells), stepped 1000 times: the field energy at every 100th step.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import OracleSim  # noqa: E402
from paper_2607_13507_amd import workloads as W  # noqa: E402


def pulse_vacuum_2048x1024():
    wl = W.gaussian_pulse_vacuum(nx=2048, ny=1024, a0=10.0, steps=1000)
    # the FP32 path starts from the initial fields rounded to FP32
    wl.fields = {k: v.astype(np.float32).astype(np.float64) for k, v in wl.fields.items()}
    orc = OracleSim.from_workload(wl, with_rho=False)
    energy = [orc.field_energy()]
    t0 = time.time()
    for k in range(10):
        orc.step(100)
        energy.append(orc.field_energy())
        print(f"  step {orc.nstep}: field energy {energy[-1]:.12e} ({time.time() - t0:.0f} s)",
              flush=True)
    rng = np.random.default_rng(1000)
    nodes = rng.choice(wl.ncell, 64, replace=False)
    # and the nodes where the pulse is strongest at the end
    nodes = np.concatenate([nodes, np.argsort(np.abs(orc.f["ey"]))[-64:]])
    return dict(workload="gaussian_pulse_vacuum(nx=2048, ny=1024, a0=10.0), initial fields "
                         "rounded to FP32, periodic, no particles",
                steps_per_record=100, field_energy=energy,
                sample_nodes=[int(i) for i in nodes],
                sample_final={k: [float(orc.f[k][i]) for i in nodes] for k in ("ex", "ey", "bz")},
                amplitude={k: float(np.abs(orc.f[k]).max()) for k in ("ex", "ey", "bz")})


def _as_fp32_inputs(wl):
    """The workload's inputs as the FP32 cell+offset path stores them."""
    f32 = lambda a: np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
    wl.fields = {k: f32(v) for k, v in wl.fields.items()}
    h = (wl.dx, wl.dy, wl.dz)
    for s in wl.species:
        for k in ("ux", "uy", "uz", "w"):
            setattr(s, k, f32(getattr(s, k)))
        for d, k in enumerate(("x", "y", "z")[:wl.ndim]):
            X = getattr(s, k) / h[d]
            cell = np.floor(X)
            setattr(s, k, (cell + f32(X - cell)) * h[d])
    return wl


def ensemble_deterministic():
    out = []
    for wl in W.deterministic_ensemble(steps=1000):
        orc = OracleSim.from_workload(_as_fp32_inputs(wl))
        energy = [orc.field_energy()]
        for k in range(10):
            orc.step(100)
            energy.append(orc.field_energy())
        print(f"  {wl.name}: {wl.nparticles} particles, field energy {energy[0]:.6e} -> "
              f"{energy[-1]:.6e}", flush=True)
        out.append(dict(name=wl.name, nx=wl.nx, ny=wl.ny, particles=wl.nparticles,
                        field_energy=energy))
    return dict(workload="deterministic_ensemble(steps=1000), inputs rounded as the FP32 "
                         "path holds them", steps_per_record=100, members=out)


GOLDENS = {"pulse_vacuum_2048x1024": pulse_vacuum_2048x1024,
           "ensemble_deterministic": ensemble_deterministic}


def main(names):
    for name in names or list(GOLDENS):
        print(f"golden {name}", flush=True)
        out = GOLDENS[name]()
        out["written_by"] = "tests/golden/make_goldens.py " + name
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(out, fh, indent=1)
            fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
