"""Pins of the oracle's convolutional PML (CPML) at open x ends (CPU).

The layer replaces every x derivative of the curls by D/kappa + psi, psi following a
recursive convolution (the form of Roden and Gedney).  Its pins are statements of the
continuous stretched-coordinate theory that a wrong coefficient, sign, time step or index
breaks:

- lossless parameters (sigma = 0, kappa = 1) leave the Yee update of a periodic box
  unchanged, bit for bit, in 2D and 3D;
- in a uniform layer (grading orders 0) a wave travelling along x with the stretch
  s = kappa + sigma / (a + i omega) keeps its shape and loses energy at the rate
  2 sigma / kappa per unit time when a = 0 (any frequency), and at 2 alpha v_g with
  alpha = sigma omega^2 / (a^2 + omega^2), v_g = 1 / (dk/domega) when a > 0, which the
  scheme approaches as dt shrinks (the recursion is first order in dt in that term);
- a graded layer of 12 cells reflects less than 1e-6 of an incident packet's energy at
  normal, 45 and 60 degree incidence, while the first-order Mur condition reflects its
  theoretical ((1 - cos t) / (1 + cos t))^2 there (so the measurement itself is pinned).
"""
import math

import numpy as np
import pytest

from oracle import OracleSim
from paper_2607_13507_amd import workloads as W

DX = 2 * math.pi / 32          # lambda / 32 with omega = 1
KEYS = ("ex", "ey", "ez", "bx", "by", "bz")


def _envelope(x, x_lo, x_hi):
    s = np.clip((x - x_lo) / (x_hi - x_lo), 0.0, 1.0)
    return np.sin(math.pi * s) ** 2


def _packet_2d(nx, ny, n_y, x_lo, x_hi):
    """A plane-wave packet with E along z, wave vector (kx, ky), |k| = 1, ky = 2 pi n_y /
    (ny dy) (periodic in y), travelling towards +x, sin^2 envelope on [x_lo, x_hi) along x.
    B is the discrete curl of A_z (div B = 0 exactly), E = -dA_z/dt of the plane wave."""
    ky = 2 * math.pi * n_y / (ny * DX)
    kx = math.sqrt(1.0 - ky * ky)
    i = np.arange(nx)[None, :] * DX
    j = np.arange(ny)[:, None] * DX
    ph = kx * (i - x_lo) + ky * j
    az = -_envelope(i, x_lo, x_hi) * np.cos(ph)
    ez = _envelope(i, x_lo, x_hi) * np.sin(ph)
    return {"ez": ez.ravel(), "bx": ((np.roll(az, -1, axis=0) - az) / DX).ravel(),
            "by": (-(np.roll(az, -1, axis=1) - az) / DX).ravel()}, kx


def _pulse_3d(nx, ny, nz, x_lo, x_hi):
    """A plane pulse along x (E along y, B along z; B the discrete curl of A_y)."""
    i = np.arange(nx) * DX
    ay = -_envelope(i, x_lo, x_hi) * np.cos(i - x_lo)
    ey = _envelope(i, x_lo, x_hi) * np.sin(i - x_lo)
    bz = (np.roll(ay, -1) - ay) / DX
    rep = lambda a: np.broadcast_to(a, (nz, ny, nx)).ravel().copy()
    return {"ey": rep(ey), "bz": rep(bz)}


def _sim(nx, ny, fields, pml, eta=0.95, open_x=True, ndim=2, nz=1):
    h = (DX, DX, DX) if ndim == 3 else (DX, DX)
    return OracleSim(ndim, nx, ny, nz, DX, DX, DX, W.cfl_dt(eta, *h), 0.0, [], fields,
                     open_x=open_x, pml=pml)


def _layer_energy(o, lo, hi):
    g = o.grid
    nz = g.nz if g.ndim == 3 else 1
    e = sum((o.f[k].reshape(nz, g.ny, g.nx)[:, :, lo:hi] ** 2).sum() for k in KEYS)
    return 0.5 * e


def _decay_rate(nx, L, pml, x_lo, x_hi, d1, d2, eta=0.95, ny=2, ndim=2, nz=1):
    """Energy decay rate (per unit time) inside the right layer [nx - L, nx) between the
    moments the pulse has moved d1 and d2 cells (at c) from its start."""
    if ndim == 3:
        flds = _pulse_3d(nx, ny, nz, x_lo * DX, x_hi * DX)
    else:
        flds = W.gaussian_pulse_fields(nx, ny, DX, DX, 1.0, x_lo * DX, x_hi * DX, 1e9,
                                       0.5 * ny * DX)
    o = _sim(nx, ny, flds, pml, eta, ndim=ndim, nz=nz)
    dt = o.grid.dt
    t1, t2 = int(round(d1 * DX / dt)), int(round(d2 * DX / dt))
    o.step(t1)
    u1 = _layer_energy(o, nx - L, nx)
    o.step(t2 - t1)
    u2 = _layer_energy(o, nx - L, nx)
    return math.log(u1 / u2) / ((t2 - t1) * dt)


def _uniform(L, **kw):
    return dict(cells=L, order=0, a_order=0, **kw)


@pytest.mark.parametrize("ndim", [2, 3])
def test_lossless_layer_is_the_plain_yee_update(ndim):
    nx, ny, nz = 40, 12, (6 if ndim == 3 else 1)
    rng = np.random.default_rng(71)
    flds = {k: rng.standard_normal(nx * ny * nz) for k in KEYS}
    a = _sim(nx, ny, flds, dict(cells=8, order=3, sigma_max=0.0, kappa_max=1.0, a_max=0.3),
             ndim=ndim, nz=nz)
    b = _sim(nx, ny, flds, None, open_x=False, ndim=ndim, nz=nz)
    a.step(25)
    b.step(25)
    for k in KEYS:
        np.testing.assert_array_equal(a.f[k], b.f[k])
    assert not a.psi.any()


def test_uniform_layer_loses_energy_at_twice_sigma():
    """kappa = 1, a = 0: rate 2 sigma, whatever the pulse's spectrum."""
    sigma = 0.03
    r = _decay_rate(1400, 560, _uniform(560, sigma_max=sigma), 600, 640, 400 * 0.672,
                    1000 * 0.672)
    assert r == pytest.approx(2 * sigma, rel=5e-3)


def test_uniform_layer_with_kappa_slows_the_wave_and_the_loss():
    """kappa = 2: the pulse crosses the layer at c / kappa, so the rate is 2 sigma / kappa."""
    sigma = 0.03
    r = _decay_rate(1400, 560, _uniform(560, sigma_max=sigma, kappa_max=2.0), 600, 640,
                    400 * 0.672, 1000 * 0.672)
    assert r == pytest.approx(sigma, rel=5e-3)


def test_uniform_layer_in_3d():
    sigma = 0.03
    r = _decay_rate(1400, 560, _uniform(560, sigma_max=sigma), 600, 640, 400 * 0.672,
                    1000 * 0.672, ndim=3, ny=2, nz=2, eta=0.95)
    assert r == pytest.approx(2 * sigma, rel=5e-3)


def test_frequency_shift_term_converges_to_the_stretched_coordinate_rate():
    """a = omega = 1: alpha = sigma / 2 and v_g = 1, so the rate is sigma.  At a finite dt
    the recursion lags (first order in dt); halving dt must bring the rate closer, and the
    first-order extrapolation must land within 2% of sigma."""
    sigma = 0.03
    pml = _uniform(800, sigma_max=sigma, a_max=1.0)
    r1 = _decay_rate(2000, 800, pml, 830, 1086, 400, 880, eta=0.95)
    r2 = _decay_rate(2000, 800, pml, 830, 1086, 400, 880, eta=0.475)
    assert abs(r2 - sigma) < abs(r1 - sigma) < 0.08 * sigma
    assert (2 * r2 - r1) == pytest.approx(sigma, rel=0.02)


def _reflection(n_y, ny, pml, L):
    """Energy reflected into the interior, from the difference with the same packet in a
    periodic box wide enough that nothing comes back within the time, relative to the
    packet's energy; measured once the packet has moved nx cells in x."""
    nx, pad = 400, 300
    c0 = 0.5 * nx * DX
    f, kx = _packet_2d(nx, ny, n_y, c0 - 64 * DX, c0 + 64 * DX)
    fr, _ = _packet_2d(nx + 2 * pad, ny, n_y, c0 + (pad - 64) * DX, c0 + (pad + 64) * DX)
    o = _sim(nx, ny, f, pml)
    r = _sim(nx + 2 * pad, ny, fr, None, open_x=False)
    e0 = o.field_energy()
    steps = int(nx * DX / (kx * o.grid.dt))
    o.step(steps)
    r.step(steps)
    d = sum(((o.f[k].reshape(ny, nx)[:, L:nx - L]
              - r.f[k].reshape(ny, nx + 2 * pad)[:, pad + L:pad + nx - L]) ** 2).sum()
            for k in KEYS)
    return 0.5 * d * DX * DX / e0, kx


@pytest.mark.parametrize("n_y,ny", [(0, 4), (1, 45), (1, 37)], ids=["0deg", "45deg", "60deg"])
def test_graded_layer_reflects_far_less_than_mur(n_y, ny):
    r_pml, kx = _reflection(n_y, ny, dict(cells=12), 12)
    assert r_pml < 1e-6
    r_mur, _ = _reflection(n_y, ny, None, 3)
    if n_y:
        theory = ((1 - kx) / (1 + kx)) ** 2
        assert r_mur == pytest.approx(theory, rel=0.25)
    assert r_mur > 1e3 * r_pml


def _einc(las, t):
    """The antenna's incident field on its axis (the definition in the oracle's header)."""
    t = np.asarray(t, dtype=np.float64) - las["t0"]
    env = np.where((t >= 0) & (t <= las["tau"]), np.sin(np.pi * t / las["tau"]) ** 2, 0.0)
    return las["a0"] * las["omega"] * env * np.sin(las["omega"] * t)


@pytest.mark.parametrize("pol", [1, 2])
def test_antenna_between_layers_in_3d(pol):
    """3D, plane antenna (huge waist) between two graded layers: right of it the field is the
    retarded incident field, left of it the left-going half, and once the pulse has left
    through both layers (nothing comes back from them) the box is empty."""
    nx, ny, nz, ia, Lc = 400, 2, 2, 40, 12
    las = dict(pol=pol, ia=ia, a0=1.0, omega=1.0, waist=1e9, yc=0.0, zc=0.0, t0=0.0, tau=40.0)
    dt = W.cfl_dt(0.95, DX, DX, DX)
    o = OracleSim(3, nx, ny, nz, DX, DX, DX, dt, 0.0, [], None, open_x=True, laser=las,
                  pml=dict(cells=Lc))
    n = int(60.0 / dt)
    o.step(n)
    t = n * dt
    x = np.arange(nx) * DX
    comp = "ey" if pol == 1 else "ez"
    e = o.f[comp].reshape(nz, ny, nx)[0, 0]
    near = (x > (ia + 2) * DX) & (x < (ia + 60) * DX)
    np.testing.assert_allclose(e[near], _einc(las, t - (x[near] - ia * DX)), atol=0.02)
    left = (x >= Lc * DX) & (x < (ia - 2) * DX)
    np.testing.assert_allclose(e[left], _einc(las, t - (ia * DX - x[left])), atol=0.02)
    # both halves leave: the pulse is 40/dx ~ 200 cells long, the box 400; after it has
    # crossed the right layer nothing of it is left
    peak = o.field_energy()
    o.step(int(70.0 / dt))
    assert o.field_energy() < 1e-6 * peak
