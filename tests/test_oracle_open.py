"""Pins of the oracle's open x ends and laser antenna (CPU only).

- Mur outgoing-wave condition: a plane pulse leaving through either x end takes its energy
  with it (a periodic box keeps it), both directions.
- Antenna: a current sheet J = -2 E_inc / dx radiates E_inc to each side (the field of a
  surface current K in these units is -K/2 on both sides), so the field right of the antenna
  is E_inc at the retarded time, and the left-going half leaves through the open end
  without coming back.
- Particles: removed when their new position enters the margin of an open end; charge
  continuity holds node by node in every step, including the one in which they leave.
"""
import math

import numpy as np
import pytest

from oracle import OPEN_MARGIN, OracleSim, OracleSpecies

DX = 2 * math.pi / 32                 # laser units: lambda = 2 pi, 32 cells per lambda
DT = 0.95 * DX / math.sqrt(2)


def _plane_pulse(direction, open_x, nx=512, ny=4):
    o = OracleSim(2, nx, ny, 1, DX, DX, 1.0, DT, open_x=open_x)
    xc, sig = 0.5 * nx * DX, 3.0
    g = lambda x: np.exp(-((x - xc) / sig) ** 2) * np.sin(x)
    o.f["ey"][:] = np.tile(g(np.arange(nx) * DX), ny)                      # Ey at (i, j+1/2)
    o.f["bz"][:] = np.tile(direction * g((np.arange(nx) + 0.5) * DX), ny)  # Bz at (i+1/2, j+1/2)
    return o


@pytest.mark.parametrize("direction", [+1, -1], ids=["to_right", "to_left"])
def test_mur_lets_a_plane_pulse_leave(direction):
    o = _plane_pulse(direction, open_x=True)
    e0 = o.field_energy()
    o.step(int(0.75 * o.grid.nx * DX / DT))
    assert o.field_energy() / e0 < 2e-4          # ~0.6% amplitude reflection at 32 cells/lambda
    p = _plane_pulse(direction, open_x=False)     # control: a periodic box keeps the pulse
    p.step(int(0.75 * p.grid.nx * DX / DT))
    assert p.field_energy() / e0 == pytest.approx(1.0, abs=1e-4)


def _einc(las, t):
    t = np.asarray(t, dtype=np.float64) - las["t0"]
    env = np.where((t >= 0) & (t <= las["tau"]), np.sin(math.pi * t / las["tau"]) ** 2, 0.0)
    return las["a0"] * las["omega"] * env * np.sin(las["omega"] * t)


def test_antenna_radiates_the_incident_field_both_ways():
    nx, ny, ia = 600, 4, 40
    las = dict(pol=1, ia=ia, a0=1.0, omega=1.0, waist=1e9, yc=0.0, zc=0.0, t0=0.0, tau=120.0)
    o = OracleSim(2, nx, ny, 1, DX, DX, 1.0, DT, open_x=True, laser=las)
    n = int(100.0 / DT)
    o.step(n)
    t = n * DT
    x = np.arange(nx) * DX
    ey = o.f["ey"].reshape(ny, nx)[0]
    # right of the antenna, near it (little grid dispersion): the retarded incident field
    near = (x > (ia + 2) * DX) & (x < (ia + 80) * DX)
    np.testing.assert_allclose(ey[near], _einc(las, t - (x[near] - ia * DX)), atol=0.02)
    # the peak amplitude everywhere on the right is the incident one
    right = (x > (ia + 2) * DX) & (x < (nx - 10) * DX)
    assert abs(ey[right]).max() == pytest.approx(abs(_einc(las, t - (x[right] - ia * DX))).max(),
                                                 rel=0.01)
    # left of it: the left-going half, with nothing reflected from the open end
    left = (x > 5 * DX) & (x < (ia - 2) * DX)
    np.testing.assert_allclose(ey[left], _einc(las, t - (ia * DX - x[left])), atol=0.01)
    # a z-polarised antenna gives the same field in Ez
    las_z = dict(las, pol=2)
    oz = OracleSim(2, nx, ny, 1, DX, DX, 1.0, DT, open_x=True, laser=las_z)
    oz.step(n)
    np.testing.assert_allclose(oz.f["ez"].reshape(ny, nx)[0][near], ey[near], atol=0.02)


def test_gaussian_antenna_profile_across_y():
    nx, ny, ia = 200, 64, 20
    las = dict(pol=1, ia=ia, a0=2.0, omega=1.0, waist=10 * DX, yc=32 * DX, zc=0.0, t0=0.0,
               tau=60.0)
    o = OracleSim(2, nx, ny, 1, DX, DX, 1.0, DT, open_x=True, laser=las)
    jy = np.zeros(nx * ny)
    o.laser_source(30.0)
    jy = o.f["jy"].reshape(ny, nx)
    y = (np.arange(ny) + 0.5) * DX
    expect = -2.0 * _einc(las, 30.0) * np.exp(-((y - las["yc"]) / las["waist"]) ** 2) / DX
    np.testing.assert_allclose(jy[:, ia], expect, rtol=1e-12, atol=1e-300)
    assert np.count_nonzero(jy) == ny        # one column only
    o.zero_currents()
    o.laser_source(61.0)                     # after the pulse: nothing
    assert not o.f["jy"].any()


def test_open_x_particles_leave_and_charge_is_conserved():
    nx, ny = 48, 8
    xs = np.array([(nx - OPEN_MARGIN - 1.5) * DX, (OPEN_MARGIN + 1.5) * DX, 20.3 * DX])
    ys = np.array([2.2, 3.7, 4.1]) * DX
    ux = np.array([2.0, -2.0, 0.1])          # the first two head for the x ends at ~0.9 c
    sp = OracleSpecies(-1.0, 1.0, 2, xs, ys, None, ux, np.zeros(3), np.zeros(3), np.full(3, 0.3))
    o = OracleSim(2, nx, ny, 1, DX, DX, 1.0, DT, species=[sp], open_x=True)
    alive = []
    for n in range(8):
        o.step(1)
        assert o.continuity() < 1e-12
        alive.append((sp.x >= 0).copy())
    assert not alive[-1][0] and not alive[-1][1] and alive[-1][2]
    # they leave exactly when their new position enters the margin
    left_at = [int(np.argmax(~np.array(alive)[:, k])) for k in range(2)]
    assert all(1 <= s <= 4 for s in left_at)
