"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one part of the oracle against something other than the oracle itself: a
closed-form solution of the discrete scheme, an exact invariant, or a moment identity of the
B-spline shapes.  The paper prints no worked numeric example, so there is no golden table.

P1  Boris, pure B: |u| conserved; discrete rotation angle 2 atan(|q| B dt / (2 m gamma)) per
    step; the trapezoidal orbit is a circle of radius (dt/2) |v| cot(theta/2).
P2  Boris, pure E: u advances by q E dt / m exactly; hyperbolic motion converges at O(dt^2).
P3  Boris, crossed E and B: mean velocity over whole gyro-periods equals E x B / B^2.
P4  Gather: constant and linear fields reproduced exactly at every staggered location;
    second moment of the shape (dx^2/4 quadratic, dx^2 o(1-o) CIC).
P5  Esirkepov: discrete continuity at every node; first moments of J; zero current at rest;
    no transverse current for axial motion; 2D Jz equals the z-integral of 3D Jz.
P6  Yee: vacuum standing modes follow A cos(omega n dt) with the discrete dispersion
    sin(omega dt/2) = (dt/2) K; div B is preserved.
P7  Whole step: the Gauss invariant div E - (rho^n + rho^{n+1})/2 is constant per node.
P8  Cold plasma oscillation at omega_p.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import OracleSim, OracleSpecies
from paper_2607_13507_amd import workloads as W


def _sim2(nx=16, ny=16, dx=0.1, dy=0.1, dt=0.05, **kw):
    return OracleSim(2, nx, ny, 1, dx, dy, 1.0, dt, **kw)


def _sim3(n=12, dx=0.1, dt=0.04, **kw):
    return OracleSim(3, n, n, n, dx, dx, dx, dt, **kw)


def _single(q, m, order, pos, u, w=0.0):
    z = None if len(pos) == 2 else [pos[2]]
    return OracleSpecies(q, m, order, [pos[0]], [pos[1]], z, [u[0]], [u[1]], [u[2]], [w])


# ---------------------------------------------------------------------------------- P1
def test_p1_boris_pure_b_rotation_angle():
    q, m, dt, B0 = -1.0, 1.0, 0.05, 2.0
    u = np.array([0.3, 0.0, 0.1])
    gam = math.sqrt(1 + u @ u)
    theta = 2 * math.atan(abs(q) * B0 * dt / (2 * m * gam))
    uperp = 0.3
    for n in range(1, 10001):
        u = oracle.boris(u, [0, 0, 0], [0, 0, B0], q, m, dt)
        if n % 2500 == 0:
            # negative charge in +z field rotates counter-clockwise
            assert u[0] == pytest.approx(uperp * math.cos(n * theta), abs=1e-11)
            assert u[1] == pytest.approx(uperp * math.sin(n * theta), abs=1e-11)
            assert u[2] == 0.1
            assert math.sqrt(u @ u) == pytest.approx(math.sqrt(0.1), rel=1e-13)


@pytest.mark.parametrize("order", [1, 2])
def test_p1_gyration_orbit_through_grid(order):
    """Uniform Bz on the grid: gather is exact, and the trapezoidal position push closes a
    circle of radius (dt/2)|v| cot(theta/2) around the closed-form centre."""
    dt, B0 = 0.05, 1.5
    sim = _sim2(nx=32, ny=32, dx=0.2, dy=0.2, dt=dt)
    sim.f["bz"][:] = B0
    u0 = np.array([0.4, 0.0, 0.0])
    s = _single(-1.0, 1.0, order, [3.2, 3.2], u0)
    gam = math.sqrt(1 + u0 @ u0)
    v = 0.4 / gam
    theta = 2 * math.atan(B0 * dt / (2 * gam))
    x0 = complex(3.2, 3.2)
    for n in range(1, 401):
        sim.gather_push(s)
        # x^n - x^0 = -i (dt/2) v cot(theta/2) (e^{i n theta} - 1) for counter-clockwise
        # rotation of a velocity that starts along +x
        pred = x0 + (-1j) * 0.5 * dt * v / math.tan(theta / 2) * (np.exp(1j * n * theta) - 1)
        assert s.x[0] == pytest.approx(pred.real, abs=1e-11)
        assert s.y[0] == pytest.approx(pred.imag, abs=1e-11)


# ---------------------------------------------------------------------------------- P2
def test_p2_pure_e_kick_exact():
    E = np.array([0.3, -0.2, 0.7])
    u = np.array([0.1, 0.2, -0.3])
    q, m, dt = -1.0, 1836.15267343, 0.07
    for _ in range(50):
        un = oracle.boris(u, E, [0, 0, 0], q, m, dt)
        np.testing.assert_allclose(un, u + q * E * dt / m, rtol=0, atol=1e-15)
        u = un


def _hyperbolic_error(dt, order=2, E0=1.0, T=5.0):
    sim = _sim2(nx=64, ny=8, dx=0.5, dy=0.5, dt=dt)
    sim.f["ex"][:] = E0
    s = _single(1.0, 1.0, order, [1.0, 1.0], [0.0, 0.0, 0.0])
    nsteps = int(round(T / dt))
    for _ in range(nsteps):
        sim.gather_push(s)
    exact = 1.0 + (math.sqrt(1 + (E0 * T) ** 2) - 1) / E0
    assert s.ux[0] == pytest.approx(E0 * T, rel=1e-12)
    return abs(s.x[0] - exact)


def test_p2_hyperbolic_motion_second_order():
    e1 = _hyperbolic_error(0.1)
    e2 = _hyperbolic_error(0.05)
    e3 = _hyperbolic_error(0.025)
    assert math.log2(e1 / e2) == pytest.approx(2.0, abs=0.1)
    assert math.log2(e2 / e3) == pytest.approx(2.0, abs=0.1)


# ---------------------------------------------------------------------------------- P3
def test_p3_exb_drift_over_whole_periods():
    dt, P = 0.1, 100                       # P steps per discrete gyro-period
    theta = 2 * math.pi / P
    B0 = 2 * math.tan(theta / 2) / dt      # rotation angle 2 atan(q B dt / 2m) = theta
    E0 = 1e-3 * B0
    sim = _sim2(nx=16, ny=16, dx=1.0, dy=1.0, dt=dt)
    sim.f["ey"][:] = E0
    sim.f["bz"][:] = B0
    s = _single(1.0, 1.0, 1, [8.0, 8.0], [0.0, 0.0, 0.0])
    x = 8.0
    nper = 10
    for _ in range(P * nper):
        xold = s.x[0]
        sim.gather_push(s)
        dxs = s.x[0] - xold
        if dxs < -8:
            dxs += 16
        x += dxs
    vmean = (x - 8.0) / (P * nper * dt)
    assert vmean == pytest.approx(E0 / B0, rel=1e-5)


# ---------------------------------------------------------------------------------- P4
STAG2 = {"ex": (0.5, 0, 0), "ey": (0, 0.5, 0), "ez": (0, 0, 0),
         "bx": (0, 0.5, 0), "by": (0.5, 0, 0), "bz": (0.5, 0.5, 0)}
STAG3 = {"ex": (0.5, 0, 0), "ey": (0, 0.5, 0), "ez": (0, 0, 0.5),
         "bx": (0, 0.5, 0.5), "by": (0.5, 0, 0.5), "bz": (0.5, 0.5, 0)}
COMPS = ("ex", "ey", "ez", "bx", "by", "bz")


def _node_coords(sim, comp):
    g = sim.grid
    st = (STAG3 if g.ndim == 3 else STAG2)[comp]
    nz = g.nz if g.ndim == 3 else 1
    k, j, i = np.meshgrid(np.arange(nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
    X = ((i + st[0]) * g.dx).reshape(-1)
    Y = ((j + st[1]) * g.dy).reshape(-1)
    Z = ((k + st[2]) * g.dz).reshape(-1)
    return X, Y, Z


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("order", [1, 2])
def test_p4_gather_linear_fields_exact(ndim, order):
    rng = np.random.default_rng(11)
    sim = _sim2(nx=16, ny=16, dx=0.13, dy=0.07) if ndim == 2 else _sim3(n=12, dx=0.11)
    coef = {}
    for c in COMPS:
        a, b, cc, d = rng.normal(size=4)
        if ndim == 2:
            d = 0.0
        coef[c] = (a, b, cc, d)
        X, Y, Z = _node_coords(sim, c)
        sim.f[c][:] = a + b * X + cc * Y + d * Z
    g = sim.grid
    for _ in range(40):
        # stay 4 cells away from the box edge so the linear field is not wrapped
        pos = [g.dx * rng.uniform(4, g.nx - 4), g.dy * rng.uniform(4, g.ny - 4),
               g.dz * rng.uniform(4, max(5, g.nz - 4)) if ndim == 3 else 0.0]
        E, B = sim.gather(order, pos)
        got = dict(zip(COMPS, list(E) + list(B)))
        for c in COMPS:
            a, b, cc, d = coef[c]
            exp = a + b * pos[0] + cc * pos[1] + d * pos[2]
            assert got[c] == pytest.approx(exp, abs=1e-12), c


@pytest.mark.parametrize("order", [1, 2])
def test_p4_gather_second_moment(order):
    """sum_k (x_k)^2 S(x_k - x) = x^2 + var, var = dx^2/4 (quadratic) or dx^2 o (1 - o) (CIC)
    with o the offset of x from the component's node lattice."""
    rng = np.random.default_rng(12)
    sim = _sim2(nx=24, ny=24, dx=0.1, dy=0.1)
    for c in COMPS:
        X, _, _ = _node_coords(sim, c)
        sim.f[c][:] = X ** 2
    for _ in range(30):
        pos = [rng.uniform(0.6, 1.8), rng.uniform(0.6, 1.8), 0.0]
        E, B = sim.gather(order, pos)
        got = dict(zip(COMPS, list(E) + list(B)))
        for c in COMPS:
            sx = STAG2[c][0]
            Xc = pos[0] / 0.1 - sx
            o = Xc - math.floor(Xc)
            var = 0.25 if order == 2 else o * (1 - o)
            assert got[c] == pytest.approx(pos[0] ** 2 + var * 0.01, abs=1e-13), c


def test_p4_shape_partition_and_symmetry():
    for order in (1, 2):
        for xi in np.linspace(-0.999, 0.999, 37):
            tot = sum(oracle.shape(order, k - xi) for k in range(-3, 4))
            assert tot == pytest.approx(1.0, abs=1e-15)
            assert oracle.shape(order, xi) == oracle.shape(order, -xi)
    assert oracle.shape(2, 0.0) == 0.75 and oracle.shape(2, 1.0) == 0.125
    assert oracle.shape(2, 1.5) == 0.0 and oracle.shape(1, 1.0) == 0.0


# ---------------------------------------------------------------------------------- P5
def _divj(sim):
    g = sim.grid
    if g.ndim == 2:
        sh = (g.ny, g.nx)
        jx, jy = sim.f["jx"].reshape(sh), sim.f["jy"].reshape(sh)
        return ((jx - np.roll(jx, 1, axis=1)) / g.dx + (jy - np.roll(jy, 1, axis=0)) / g.dy)
    sh = (g.nz, g.ny, g.nx)
    jx, jy, jz = (sim.f[k].reshape(sh) for k in ("jx", "jy", "jz"))
    return ((jx - np.roll(jx, 1, axis=2)) / g.dx + (jy - np.roll(jy, 1, axis=1)) / g.dy +
            (jz - np.roll(jz, 1, axis=0)) / g.dz)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("order", [1, 2])
def test_p5_esirkepov_continuity_and_moments(ndim, order):
    rng = np.random.default_rng(20 + ndim * 3 + order)
    sim = _sim2(nx=10, ny=9, dx=0.1, dy=0.13, dt=0.05) if ndim == 2 else _sim3(n=8, dt=0.04)
    g = sim.grid
    h = np.array([g.dx, g.dy, g.dz])
    L = np.array([g.nx * g.dx, g.ny * g.dy, g.nz * g.dz])
    for trial in range(25):
        sim.zero_currents()
        q, w = rng.choice([-1.0, 1.0]), rng.uniform(0.1, 2.0)
        p0 = rng.uniform(0, 1, 3) * L
        if trial < 6:      # start right at the box edge to exercise the periodic wrap
            p0[trial % ndim] = L[trial % ndim] * (1 - 1e-3 * trial)
        disp = rng.uniform(-0.67, 0.67, 3) * h
        if ndim == 2:
            p0[2] = disp[2] = 0.0
        p1 = p0 + disp
        vz = rng.normal()
        sim.deposit_particle(order, q, w, p0, p1, vz)
        sim.deposit_rho(sim.rho0, order, q, w, p0)
        sim.deposit_rho(sim.rho1, order, q, w, p1)
        shp = (g.ny, g.nx) if ndim == 2 else (g.nz, g.ny, g.nx)
        res = sim.rho1.reshape(shp) - sim.rho0.reshape(shp) + g.dt * _divj(sim)
        assert np.abs(res).max() <= 1e-13 * w
        assert sim.continuity() <= 1e-13
        # first moments: sum of J along an axis = q w displacement / dt
        for d, k in enumerate(("jx", "jy", "jz")[:ndim]):
            assert sim.f[k].sum() == pytest.approx(q * w * disp[d] / g.dt, abs=1e-12)
        if ndim == 2:
            assert sim.f["jz"].sum() == pytest.approx(q * w * vz, abs=1e-12)


@pytest.mark.parametrize("order", [1, 2])
def test_p5_particle_at_rest_and_axial_motion(order):
    sim = _sim2(nx=8, ny=8, dx=0.1, dy=0.1, dt=0.05)
    sim.deposit_particle(order, -1.0, 1.0, [0.33, 0.41, 0], [0.33, 0.41, 0], 0.0)
    for k in ("jx", "jy", "jz"):
        assert np.abs(sim.f[k]).max() == 0.0
    sim.zero_currents()
    sim.deposit_particle(order, -1.0, 1.0, [0.33, 0.41, 0], [0.37, 0.41, 0], 0.0)
    assert np.abs(sim.f["jy"]).max() == 0.0
    # Jx rows are proportional to the y shape at the (unchanged) y position
    jx = sim.f["jx"].reshape(8, 8)
    rows = jx.sum(axis=1)
    Y = 0.41 / 0.1
    expect = np.array([sum(oracle.shape(order, jj + 8 * m - Y) for m in (-1, 0, 1))
                       for jj in range(8)])
    np.testing.assert_allclose(rows / rows.sum(), expect, atol=1e-14)


@pytest.mark.parametrize("order", [1, 2])
def test_p5_2d_jz_is_z_integral_of_3d(order):
    rng = np.random.default_rng(7)
    dt, dx = 0.04, 0.1
    s2 = OracleSim(2, 8, 8, 1, dx, dx, 1.0, dt)
    s3 = OracleSim(3, 8, 8, 8, dx, dx, dx, dt)
    for _ in range(10):
        s2.zero_currents()
        s3.zero_currents()
        p0 = np.array([rng.uniform(0.2, 0.6), rng.uniform(0.2, 0.6), 0.43])
        d = rng.uniform(-0.05, 0.05, 3)
        s3.deposit_particle(order, 1.0, 0.7, p0, p0 + d, 0.0)
        s2.deposit_particle(order, 1.0, 0.7, [p0[0], p0[1], 0], [p0[0] + d[0], p0[1] + d[1], 0],
                            d[2] / dt)
        jz3 = s3.f["jz"].reshape(8, 8, 8).sum(axis=0) * dx   # integral over z
        jz2 = s2.f["jz"].reshape(8, 8) * dx                    # one cell thick
        np.testing.assert_allclose(jz3, jz2, atol=1e-13)


# ---------------------------------------------------------------------------------- P6
def test_p6_vacuum_tm_mode_closed_form():
    wl = W.vacuum_mode(nx=32, ny=24, dx=0.05, mx=2, my=1, steps=1000)
    sim = OracleSim.from_workload(wl)
    kx, ky = wl.meta["kx"], wl.meta["ky"]
    K2 = 4 * math.sin(kx * wl.dx / 2) ** 2 / wl.dx ** 2 + 4 * math.sin(ky * wl.dy / 2) ** 2 / wl.dy ** 2
    omega = 2 / wl.dt * math.asin(wl.dt * math.sqrt(K2) / 2)
    ez0 = sim.f["ez"].copy()
    for n in range(1, 1001):
        sim.step()
        if n % 250 == 0:
            np.testing.assert_allclose(sim.f["ez"], ez0 * math.cos(omega * n * wl.dt),
                                       atol=2e-12)


def test_p6_vacuum_te_mode_closed_form():
    nx, ny, dx, dy = 20, 16, 0.07, 0.05
    dt = W.cfl_dt(0.95, dx, dy)
    sim = OracleSim(2, nx, ny, 1, dx, dy, 1.0, dt)
    kx, ky = 2 * math.pi * 3 / (nx * dx), 2 * math.pi * 2 / (ny * dy)
    X, Y, _ = _node_coords(sim, "bz")
    sim.f["bz"][:] = np.cos(kx * X) * np.cos(ky * Y)
    b0 = sim.f["bz"].copy()
    K2 = 4 * math.sin(kx * dx / 2) ** 2 / dx ** 2 + 4 * math.sin(ky * dy / 2) ** 2 / dy ** 2
    omega = 2 / dt * math.asin(dt * math.sqrt(K2) / 2)
    for n in range(1, 401):
        sim.step()
        if n % 100 == 0:
            np.testing.assert_allclose(sim.f["bz"], b0 * math.cos(omega * n * dt), atol=2e-12)


@pytest.mark.parametrize("ndim", [2, 3])
def test_p6_div_b_preserved(ndim):
    sim = _sim2(nx=12, ny=10) if ndim == 2 else _sim3(n=8)
    rng = np.random.default_rng(5)
    for k in COMPS + ("jx", "jy", "jz"):
        sim.f[k][:] = rng.normal(size=sim.ncell)
    d0 = sim.div_b()
    for _ in range(20):
        sim.yee_e(0.5)
        sim.yee_b(0.5)
    np.testing.assert_allclose(sim.div_b(), d0, atol=1e-10)


# ---------------------------------------------------------------------------------- P7
@pytest.mark.parametrize("ndim,order", [(2, 1), (2, 2), (3, 2), (3, 1)])
def test_p7_gauss_invariant_whole_step(ndim, order):
    if ndim == 2:
        wl = W.thermal_2d(nx=12, ny=10, dx=0.1, ppc=4, T=0.05, order=order, seed=3)
    else:
        wl = W.thermal_3d(n=6, dx=0.1, ppc=2, T=0.05, order=order, seed=3)
    sim = OracleSim.from_workload(wl)
    sim.step()
    g1 = sim.gauss()
    assert np.abs(g1).max() > 1e-3        # the random loading leaves a non-zero invariant
    for _ in range(20):
        sim.step()
        assert sim.continuity() < 1e-12
    np.testing.assert_allclose(sim.gauss(), g1, atol=1e-11)


# ---------------------------------------------------------------------------------- P8
def test_p8_cold_plasma_oscillation_frequency():
    wl = W.cold_langmuir(nx=64, ny=2, dx=0.05, lattice=4, amp=1e-3, order=1, steps=400)
    sim = OracleSim.from_workload(wl)
    probe = 16 * 1 + 0      # node i = 16 (quarter wavelength), row 0: Ex at its peak there
    series = []
    for _ in range(wl.steps):
        sim.step()
        series.append(sim.f["ex"][probe])
    s = np.array(series)
    t = (np.arange(len(s)) + 1) * wl.dt
    crossings = []
    for a in range(len(s) - 1):
        if s[a] == 0 or s[a] * s[a + 1] < 0:
            crossings.append(t[a] - s[a] * (t[a + 1] - t[a]) / (s[a + 1] - s[a]))
    assert len(crossings) >= 4
    omega = math.pi * (len(crossings) - 1) / (crossings[-1] - crossings[0])
    assert omega == pytest.approx(1.0, rel=5e-3)


# ------------------------------------------------------------- P1/P5 (general geometry)
def _rodrigues(v, axis, ang):
    k = axis / np.linalg.norm(axis)
    return (v * math.cos(ang) + np.cross(k, v) * math.sin(ang) +
            k * (k @ v) * (1 - math.cos(ang)))


@pytest.mark.parametrize("q", [-1.0, 1.0])
def test_p1_boris_rotation_about_oblique_field(q):
    """Pure B along an arbitrary axis: u turns about B by 2 atan(|q| |B| dt / (2 m gamma))
    per step, in the sense of -q B (right-handed rotation for negative charge)."""
    B = np.array([0.3, -0.5, 0.8]) * 1.7
    u0 = np.array([0.2, 0.4, -0.1])
    dt, m = 0.03, 1.0
    gam = math.sqrt(1 + u0 @ u0)
    theta = 2 * math.atan(abs(q) * np.linalg.norm(B) * dt / (2 * m * gam))
    u = u0.copy()
    for n in range(1, 2001):
        u = oracle.boris(u, [0, 0, 0], B, q, m, dt)
    exp = _rodrigues(u0, -q * B, n * theta)
    np.testing.assert_allclose(u, exp, atol=1e-11)


@pytest.mark.parametrize("order", [1, 2])
def test_p5_esirkepov_anisotropic_3d(order):
    rng = np.random.default_rng(31)
    sim = OracleSim(3, 7, 6, 5, 0.11, 0.07, 0.13, 0.03)
    g = sim.grid
    h = np.array([g.dx, g.dy, g.dz])
    for _ in range(15):
        sim.zero_currents()
        p0 = rng.uniform(0, 1, 3) * np.array([7 * 0.11, 6 * 0.07, 5 * 0.13])
        disp = rng.uniform(-0.5, 0.5, 3) * h
        sim.deposit_particle(order, -1.0, 0.9, p0, p0 + disp, 0.0)
        sim.deposit_rho(sim.rho0, order, -1.0, 0.9, p0)
        sim.deposit_rho(sim.rho1, order, -1.0, 0.9, p0 + disp)
        res = (sim.rho1 - sim.rho0).reshape(5, 6, 7) + g.dt * _divj(sim)
        assert np.abs(res).max() <= 1e-13
        for d, k in enumerate(("jx", "jy", "jz")):
            assert sim.f[k].sum() == pytest.approx(-0.9 * disp[d] / g.dt, abs=1e-12)


@pytest.mark.parametrize("order", [1, 2])
def test_p5_2d_jz_matches_3d_push_in_uniform_fields(order):
    """A full push in uniform fields: the 3D trapezoidal z displacement fixes the 2D Jz
    (z-integrated 3D Jz equals the one-cell-thick 2D Jz)."""
    dx, dt = 0.1, 0.04
    E = {"ex": 0.2, "ey": -0.3, "ez": 0.9}
    B = {"bx": 0.7, "by": 0.4, "bz": -0.5}
    s2 = OracleSim(2, 8, 8, 1, dx, dx, 1.0, dt)
    s3 = OracleSim(3, 8, 8, 8, dx, dx, dx, dt)
    for s in (s2, s3):
        for k, v in {**E, **B}.items():
            s.f[k][:] = v
    p = [0.41, 0.37, 0.43]
    u = [0.3, -0.6, 0.8]
    a2 = _single(-1.0, 1.0, order, p[:2], u, w=0.5)
    a3 = _single(-1.0, 1.0, order, p, u, w=0.5)
    s2.push_deposit(a2)
    s3.push_deposit(a3)
    np.testing.assert_allclose([a2.ux[0], a2.uy[0], a2.uz[0]], [a3.ux[0], a3.uy[0], a3.uz[0]],
                               atol=1e-15)
    jz3 = s3.f["jz"].reshape(8, 8, 8).sum(axis=0) * dx
    jz2 = s2.f["jz"].reshape(8, 8) * dx
    np.testing.assert_allclose(jz3, jz2, atol=1e-13)


# ------------------------------------------------------------------ energy diagnostics
def test_kinetic_energy_special_values():
    sim = OracleSim(2, 4, 4, 1, 0.2, 0.3, 1.0, 0.05)
    sim.species = [_single(1.0, W.M_PROTON, 1, [0.1, 0.1], [0.3, 0.0, 0.4], w=2.0),
                   _single(-1.0, 1.0, 2, [0.1, 0.1], [0.0, 3.0, 0.0], w=0.5)]
    exp = (2.0 * W.M_PROTON * (math.sqrt(1.25) - 1) + 0.5 * (math.sqrt(10.0) - 1)) * 0.2 * 0.3
    assert sim.kinetic_energy() == pytest.approx(exp, rel=1e-14)
    sim.f["ez"][:] = 2.0
    sim.f["bx"][:] = 1.0
    assert sim.field_energy() == pytest.approx(0.5 * 16 * 5.0 * 0.2 * 0.3, rel=1e-14)


def test_cold_plasma_energy_is_bounded():
    """With the current of each step taken on the path x^{n+1/2} -> x^{n+1/2} + dt v^{n+1}
    (J at the whole time level, Eq. 3), a cold plasma mode evolves under the map
        v' = v + a dt F,   F' = F - b dt v'          (a b = omega_p^2)
    of determinant 1: the oscillation energy has no secular trend.  (The path x^n -> x^{n+1}
    would give determinant 1 + (omega_p dt)^2 / 2 and exponential growth.)"""
    wl = W.cold_langmuir(nx=32, ny=2, dx=0.05, lattice=2, amp=1e-2, order=2, steps=600)
    sim = OracleSim.from_workload(wl)
    k0 = sim.kinetic_energy()
    tot, fe = [], []
    for _ in range(wl.steps):
        sim.step()
        fe.append(sim.field_energy())
        tot.append(fe[-1] + sim.kinetic_energy())
    assert max(fe) > 0.9 * k0              # nearly all kinetic energy passes into the field
    slope = np.polyfit(np.arange(1, wl.steps + 1), np.log(np.array(tot) / k0), 1)[0]
    assert abs(slope) < 0.02 * math.log(1 + 0.5 * wl.dt ** 2)
    assert (max(tot) - min(tot)) < 2e-3 * k0


def test_cold_plasma_leapfrog_dispersion_at_large_omega_dt():
    """At omega_p dt = 0.6 the time-centred scheme oscillates at the leapfrog frequency
    (2/dt) asin(omega_p dt / 2) = 1.0157 omega_p (the other path choice gives 0.963)."""
    dx = 0.05
    dt = W.cfl_dt(0.95, dx, dx)
    wp = 0.6 / dt
    wl = W.cold_langmuir(nx=64, ny=2, dx=dx, lattice=4, amp=1e-4, order=1, steps=400,
                         density=wp * wp)
    sim = OracleSim.from_workload(wl)
    series = []
    for _ in range(wl.steps):
        sim.step()
        series.append(sim.f["ex"][16])
    s_ = np.array(series)
    t = (np.arange(len(s_)) + 1) * dt
    cr = [t[a] - s_[a] * (t[a + 1] - t[a]) / (s_[a + 1] - s_[a])
          for a in range(len(s_) - 1) if s_[a] * s_[a + 1] < 0]
    omega = math.pi * (len(cr) - 1) / (cr[-1] - cr[0])
    assert omega / wp == pytest.approx(2 / (wp * dt) * math.asin(wp * dt / 2), rel=5e-3)
