"""The oracle's multi-threaded timing mode (orc_step_threads) takes the same steps as the
single-threaded parity mode: only the order of the current sums differs, so fields, charge
and particles agree to FP64 round-off.  Cases: a periodic thermal box (CIC, charge planes),
a laser slab with open ends, an antenna and PML layers (quadratic, two species, particles
leaving), and a 3D thermal box."""
import numpy as np
import pytest

from oracle import OracleSim
from paper_2607_13507_amd import workloads as W


def _pair(wl):
    return OracleSim.from_workload(wl), OracleSim.from_workload(wl)


def _same(a, b, tol=1e-12):
    for k in a.f:
        scale = max(1e-300, np.abs(a.f[k]).max())
        assert np.abs(a.f[k] - b.f[k]).max() <= tol * scale, k
    for k in ("rho0", "rho1"):
        x, y = getattr(a, k), getattr(b, k)
        assert np.abs(x - y).max() <= tol * max(1e-300, np.abs(x).max()), k
    for s, t in zip(a.species, b.species):
        for k in ("x", "y", "z", "ux", "uy", "uz"):
            u, v = getattr(s, k), getattr(t, k)
            if u is None:
                continue
            assert np.abs(u - v).max() <= tol * max(1.0, np.abs(u).max()), k


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_threads_equal_single_thread_thermal(threads):
    wl = W.thermal_2d(nx=32, ny=32, ppc=8, order=1, seed=11)
    a, b = _pair(wl)
    a.step(3)
    used = b.step_threads(3, threads)
    assert used == threads
    _same(a, b)


def test_threads_equal_single_thread_laser_slab_with_pml():
    wl = W.laser_slab_2d(nx=128, ny=64, slab=(48, 96), ppc=4, pml_cells=8, a0=5.0,
                         duration_lambda=2.0)
    a, b = _pair(wl)
    a.step(40)
    b.step_threads(40, 4)
    assert (a.species[0].x < 0).sum() == (b.species[0].x < 0).sum()
    _same(a, b, tol=1e-11)


def test_threads_equal_single_thread_3d():
    wl = W.thermal_3d(n=8, ppc=2, T=0.05, seed=12)
    a, b = _pair(wl)
    a.step(2)
    b.step_threads(2, 5)
    _same(a, b)
