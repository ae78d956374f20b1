"""Pins of the oracle's moving window (CPU).  A window is a bookkeeping move of the box, so
its pins are physical statements that a wrong column offset, sign or injection place
breaks:

- a light pulse in vacuum, moving at c, stays put in a window that moves at c (it crosses
  the box when the window stands still), with its energy unchanged;
- a cold, neutral, uniform plasma stays exactly uniform through window moves that inject
  the same plasma: every column between the margins keeps ppc x ny particles, no field
  appears, and the particles that fall behind the left end are removed.
"""
import math

import numpy as np
import pytest

from oracle import OPEN_MARGIN, OracleSim, OracleSpecies
from paper_2607_13507_amd import workloads as W


def _pulse_box(nx=256, ny=16):
    dx = 2 * math.pi / 32
    flds = W.gaussian_pulse_fields(nx, ny, dx, dx, 1.0, 64 * dx, 128 * dx, 1e9, 0.5 * ny * dx)
    return OracleSim(2, nx, ny, 1, dx, dx, 1.0, W.cfl_dt(0.95, dx, dx), 0.0, [], flds,
                     open_x=True)


def _centroid(orc):
    e = (orc.f["ey"] ** 2 + orc.f["bz"] ** 2).reshape(orc.grid.ny, orc.grid.nx).sum(axis=0)
    return float((e * np.arange(orc.grid.nx)).sum() / e.sum())


def test_pulse_stays_in_a_window_moving_at_c():
    still, moving = _pulse_box(), _pulse_box()
    c0, e0 = _centroid(moving), moving.field_energy()
    cells_per_step = moving.grid.dt / moving.grid.dx
    done, nsteps = 0, 150
    for n in range(1, nsteps + 1):
        still.step(1)
        moving.step(1)
        due = int(math.floor(n * cells_per_step)) - done
        if due > 0:
            moving.window_shift(due)
            done += due
    assert done == int(math.floor(nsteps * cells_per_step)) > 90
    # the still box sees the pulse travel about c t (~100 cells; the discrete pulse lags a
    # few cells); in the moving one it stays within those few cells of where it started,
    # and the two boxes hold the same pulse, `done` cells apart
    assert _centroid(still) - c0 == pytest.approx(nsteps * cells_per_step, abs=4)
    assert abs(_centroid(moving) - c0) < 4.0
    nx, ny = still.grid.nx, still.grid.ny
    es = (still.f["ey"] ** 2 + still.f["bz"] ** 2).reshape(ny, nx).sum(axis=0)
    pulse = np.where(es > 1e-3 * es.max())[0]
    pulse = pulse[pulse >= done]
    for k in ("ey", "bz"):
        a = still.f[k].reshape(ny, nx)[:, pulse]
        b = moving.f[k].reshape(ny, nx)[:, pulse - done]
        assert np.abs(a - b).max() < 1e-3 * np.abs(a).max(), k
    # what the moving box lost is the ~1% of the start-up field that runs backwards
    assert 0.98 * e0 < moving.field_energy() <= e0 * (1 + 1e-6)


def test_uniform_plasma_stays_uniform_through_window_moves():
    nx, ny, px, py, dx = 48, 8, 2, 2, 0.1
    dens = 1.0
    cols = np.arange(OPEN_MARGIN, nx - OPEN_MARGIN)
    xs, ys = [], []
    for c in cols:
        for j in range(ny):
            for l in range(px * py):
                xs.append((c + (2 * (l % px) + 1) / (2 * px)) * dx)
                ys.append((j + (2 * (l // px) + 1) / (2 * py)) * dx)
    n = len(xs)
    e = OracleSpecies(-1.0, 1.0, 2, np.array(xs), np.array(ys), None, np.zeros(n), np.zeros(n),
                      np.zeros(n), np.full(n, dens / (px * py)))
    orc = OracleSim(2, nx, ny, 1, dx, dx, 1.0, W.cfl_dt(0.9, dx, dx), dens, [e], open_x=True)
    plasma = dict(species=0, ppc_x=px, ppc_y=py, density=dens)
    for m in (1, 5, 2, 7, 3):
        orc.step(2)
        orc.window_shift(m, plasma)
    orc.step(2)
    s = orc.species[0]
    alive = s.x >= 0
    counts = np.bincount(np.floor(s.x[alive] / dx).astype(int), minlength=nx)
    assert np.all(counts[OPEN_MARGIN:nx - OPEN_MARGIN] == ppc_total(px, py, ny))
    assert counts[:OPEN_MARGIN].sum() == 0 and counts[nx - OPEN_MARGIN:].sum() == 0
    assert (~alive).sum() == 18 * px * py * ny   # the 1+5+2+7+3 columns that fell behind
    for k in ("ex", "ey", "ez", "bx", "by", "bz"):
        assert np.abs(orc.f[k]).max() < 1e-12, k
    assert np.abs(s.ux[alive]).max() < 1e-12


def ppc_total(px, py, ny):
    return px * py * ny
