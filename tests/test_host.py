"""Host-side logic on the CPU: the seeded input recipes (sizes, placement, neutrality,
reproducibility), the benchmark's byte model and its refusal of several GPUs."""
import math
import os
import subprocess
import sys

import numpy as np

from paper_2607_13507_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_laser_slab_recipe():
    wl = W.laser_slab_2d(nx=256, ny=64, slab=(64, 96), ppc=8, pml_cells=16)
    e, p = wl.species
    assert wl.nparticles == 2 * 8 * 32 * 64
    # the slab's cells only, and each proton on an electron (neutral node by node)
    assert e.x.min() >= 64 * wl.dx and e.x.max() < 96 * wl.dx
    np.testing.assert_array_equal(e.x, p.x)
    np.testing.assert_array_equal(e.y, p.y)
    assert e.q == -1.0 and p.q == 1.0 and p.m > 1836
    assert np.allclose(e.w, 20.0 / 8)
    assert wl.dx == W.LAMBDA / 32 and wl.dt <= W.cfl_dt(1.0, wl.dx, wl.dy)
    # PML layers of 16 cells, the antenna 4 cells inside the left one's inner face
    assert wl.open_x and wl.pml == dict(cells=16) and wl.laser["ia"] == 20
    assert W.laser_slab_2d(nx=256, ny=64, slab=(64, 96), ppc=8).laser["ia"] == 4


def test_recipes_are_reproducible_from_their_seed():
    a = W.ensemble_2d(seed=7, members=5, max_scale=16)
    b = W.ensemble_2d(seed=7, members=5, max_scale=16)
    c = W.ensemble_2d(seed=8, members=5, max_scale=16)
    for x, y in zip(a, b):
        assert (x.nx, x.ny) == (y.nx, y.ny)
        for s, t in zip(x.species, y.species):
            np.testing.assert_array_equal(s.x, t.x)
            np.testing.assert_array_equal(s.ux, t.ux)
    assert any((x.nx, x.ny, x.nparticles) != (y.nx, y.ny, y.nparticles) for x, y in zip(a, c))
    for m in a:   # every member: nx >= ny, a laser from the left, open x ends
        assert m.nx >= m.ny and m.open_x and m.laser is not None


def test_thermal_recipes():
    wl = W.thermal_3d(n=8, ppc=2, T=0.05, seed=3)
    s = wl.species[0]
    assert wl.nparticles == 8 ** 3 * 2 and wl.ndim == 3
    assert s.x.min() >= 0 and s.x.max() < 8 * wl.dx and s.z.max() < 8 * wl.dz
    # Maxwellian momenta: the variance of each component is about T (non-relativistic T)
    assert abs(np.var(s.ux) / 0.05 - 1.0) < 0.2
    assert wl.dt <= W.cfl_dt(1.0, wl.dx, wl.dy, wl.dz)


def test_wakefield_moving_window_recipe():
    wl = W.wakefield_2d(nx=512, ny=64, moving=True, spare=1000)
    s = wl.species[0]
    alive = s.x >= 0
    assert (~alive).sum() == 1000 and np.all(s.w[~alive] == 0)
    assert wl.open_x and "window" in wl.meta
    assert wl.meta["window"]["cells_per_step"] == wl.dt / wl.dx


def test_algorithmic_bytes_per_push():
    # FP32 2D: 28 bytes in and 24 out per particle, 36 per cell amortised over 64 particles
    assert bench.algorithmic_bytes_per_push(2, True, 64) == 52 + 36 / 64
    assert bench.algorithmic_bytes_per_push(2, False, 64) == 88 + 72 / 64
    assert math.isclose(bench.algorithmic_bytes_per_push(3, True, 8), 60 + 36 / 8)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
