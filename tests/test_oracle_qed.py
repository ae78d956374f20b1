"""Pins of the oracle's QED event Monte-Carlo (Sec. 3.4) to what the mathematics and the
physics fix: the Bessel functions against SciPy, the emission spectrum's classical
(synchrotron) limits -- photon number rate 5 chi / (2 sqrt 3) and the Larmor power
(2/3) chi^2 with its known quantum (Gaunt) corrections 1 - (55 sqrt3 / 16) chi + 48 chi^2 --,
the pair rate's small-chi asymptote (3/16) sqrt(3/2) chi exp(-8 / (3 chi)) (the saddle point
of the spectrum at xi = 1/2), the pair spectrum's symmetry, the quantum parameters of
simple field configurations (Lorentz invariants), the published SplitMix64 output, the
optical-depth statistics of a population, and momentum and energy conservation of every
event."""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import kv

from oracle import OracleSim, OracleSpecies
from oracle import qed as Q

HW = 1e-6          # hbar omega / (m c^2): w_r = 1.52e15 rad/s, a 1.24 um wavelength


def test_bessel_k_matches_scipy():
    for nu in (1 / 3, 2 / 3, 5 / 3):
        for x in (1e-9, 1e-6, 1e-3, 0.1, 1.0, 5.0, 50.0, 300.0):
            assert Q.bessel_k(nu, x) == pytest.approx(kv(nu, x), rel=1e-12)
    for x in (1e-3, 0.5, 3.0, 40.0):
        ref = quad(lambda s: kv(1 / 3, s), x, np.inf, epsabs=0, epsrel=1e-12, limit=200)[0]
        assert Q.bessel_k_tail(1 / 3, x) == pytest.approx(ref, rel=1e-10)
    # int_0^inf K_nu = pi / (2 cos(nu pi / 2)); the tail from 1e-12 misses ~x^(2/3)
    assert Q.bessel_k_tail(1 / 3, 1e-12) == pytest.approx(math.pi / math.sqrt(3), rel=1e-7)


def test_compton_classical_limits():
    for chi in (1e-4, 1e-3):
        h = Q.compton_rate(chi)
        assert h / (5 * chi / (2 * math.sqrt(3))) == pytest.approx(1.0, abs=2 * chi)
        gaunt = 1 - 55 * math.sqrt(3) / 16 * chi + 48 * chi ** 2
        assert Q.compton_moment(chi) / (2 / 3 * chi ** 2) == pytest.approx(gaunt, abs=600 * chi ** 3)
    # the spectrum falls with chi beyond the classical limit, never above it
    h = [Q.compton_rate(c) / c for c in (0.01, 0.1, 1.0, 10.0)]
    assert all(a > b for a, b in zip(h, h[1:]))
    # the cdf reaches the total at xi = 1 and the spectrum vanishes outside (0, 1)
    assert Q.compton_cdf(0.3, 1.0) == Q.compton_rate(0.3)
    assert Q.compton_spectrum(0.3, 0.0) == 0.0 and Q.compton_spectrum(0.3, 1.0) == 0.0


def test_compton_sampler():
    chi = 1e-3
    r = (np.arange(200) + 0.5) / 200
    xi = np.array([Q.compton_sample(chi, v) for v in r])
    assert np.all(np.diff(xi) > 0) and xi[0] > 0 and xi[-1] < 1
    # classical mean energy fraction: (2/3 chi^2) / (5 chi / (2 sqrt 3)) = 4 sqrt3 chi / 15
    assert xi.mean() == pytest.approx(4 * math.sqrt(3) / 15 * chi, rel=0.03)
    for chi, v in ((0.05, 0.3), (2.0, 0.97)):
        x = Q.compton_sample(chi, v)
        assert Q.compton_cdf(chi, x) / Q.compton_rate(chi) == pytest.approx(v, abs=1e-9)


def test_breit_wheeler_asymptote_and_symmetry():
    def ratio(chi):
        return Q.bw_rate(chi) / (3 / 16 * math.sqrt(1.5) * chi * math.exp(-8 / (3 * chi)))
    r1, r2 = ratio(0.01), ratio(0.005)
    assert abs(1 - r2) < 2e-3
    assert 1.7 < (1 - r1) / (1 - r2) < 2.3          # the correction is linear in chi
    for chi in (0.3, 3.0):
        for xi in (0.1, 0.27, 0.45):
            assert Q.bw_spectrum(chi, xi) == pytest.approx(Q.bw_spectrum(chi, 1 - xi), rel=1e-12)
        for v in (0.05, 0.3):
            assert Q.bw_sample(chi, v) + Q.bw_sample(chi, 1 - v) == pytest.approx(1.0, abs=1e-9)
    # small chi: a Gaussian around 1/2 of variance 1 / (8 y0), y0 = 8 / (3 chi)
    chi = 0.02
    r = (np.arange(200) + 0.5) / 200
    xi = np.array([Q.bw_sample(chi, v) for v in r])
    assert xi.mean() == pytest.approx(0.5, abs=1e-9)
    assert xi.var() == pytest.approx(3 * chi / 64, rel=0.1)


def test_quantum_parameters():
    u = np.array([30.0, -40.0, 0.0])                      # |u| = 50
    B = np.array([0.0, 0.0, 2.0])
    assert Q.chi_lepton(u, [0, 0, 0], B, HW) == pytest.approx(HW * 50 * 2, rel=1e-14)
    E = np.array([0.6, -0.8, 0.0])                        # along u, |E| = 1
    assert Q.chi_lepton(u, E, [0, 0, 0], HW) == pytest.approx(HW, rel=1e-12)
    assert Q.chi_lepton([0, 0, 0], [1.0, 2.0, 2.0], [0, 0, 0], HW) == pytest.approx(3 * HW)
    # crossed field |E| = |B| with the particle along E x B: chi = hw |E| (gamma - |u|)
    ux = 20.0
    g = math.sqrt(1 + ux * ux)
    c = Q.chi_lepton([ux, 0, 0], [0, 5.0, 0], [0, 0, 5.0], HW)
    assert c == pytest.approx(HW * 5.0 * (g - ux), rel=1e-9)
    # head-on: gamma + |u|
    c = Q.chi_lepton([-ux, 0, 0], [0, 5.0, 0], [0, 0, 5.0], HW)
    assert c == pytest.approx(HW * 5.0 * (g + ux), rel=1e-12)
    k = np.array([0.0, 300.0, 400.0])
    assert Q.chi_photon(k, [0, 3.0, 4.0], [0, 0, 0], HW) == 0.0   # along E
    assert Q.chi_photon(k, [0, 0, 0], [7.0, 0, 0], HW) == pytest.approx(HW * 500 * 7, rel=1e-14)


def test_splitmix64_published_output():
    # the first outputs of SplitMix64 seeded with 1234567
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    assert [Q.splitmix64(1234567, k) for k in range(5)] == ref
    v = [Q.uniform(7, 3, i, d) for i in range(50) for d in range(4)]
    assert len(set(v)) == len(v) and min(v) > 0 and max(v) < 1


def _uniform_box(B=(0.0, 0.0, 0.0), E=(0.0, 0.0, 0.0), ndim=2):
    n = 16
    sim = OracleSim(ndim, n, n, n if ndim == 3 else 1, 0.1, 0.1, 0.1, 0.05)
    for k, v in zip(("ex", "ey", "ez", "bx", "by", "bz"), (*E, *B)):
        sim.f[k][:] = v
    return sim


def _beam(n, u, q=-1.0, seed=1):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1.6, n)
    y = rng.uniform(0, 1.6, n)
    return OracleSpecies(q, 1.0, 2, x, y, None, np.full(n, u[0]), np.full(n, u[1]),
                         np.full(n, u[2]), rng.uniform(0.5, 1.5, n))


def test_emission_statistics_and_conservation():
    """q = 0 keeps the Boris push out of the way: every event must conserve momentum
    exactly, and the share of emitters must follow 1 - exp(-W dt) for optical depths drawn
    as -ln U."""
    Bz = 5.0
    ux = 2000.0
    sim = _uniform_box(B=(0, 0, Bz))
    hw = 0.5 / (ux * Bz)                      # chi = hw |u x B| = 0.5
    s = _beam(1000, (ux, 0, 0), q=0.0)
    u0 = s.ux.copy()
    tau0 = Q.init_tau(s.n, seed=5, step=0)
    tau = tau0.copy()
    ph = Q.QedBuf(2000)
    x0 = s.x.copy()
    Q.qed_gather_push(sim, s, tau, hw, seed=5, step=1, photons=ph)
    g0 = math.sqrt(1 + ux * ux)
    W = 7.2973525693e-3 * Q.compton_rate(0.5) / (g0 * hw)
    dtau = W * sim.grid.dt
    emit = tau0 - dtau <= 0
    n_ev = int(emit.sum())
    assert ph.count == n_ev
    p = 1 - math.exp(-dtau)
    assert abs(n_ev - 1000 * p) < 4 * math.sqrt(1000 * p * (1 - p)), (n_ev, p)
    np.testing.assert_allclose(tau[~emit], tau0[~emit] - dtau, rtol=0, atol=1e-12)
    idx = ph.src[:n_ev]
    assert sorted(idx) == list(np.nonzero(emit)[0])
    # momentum conservation, photon along u, energy fraction xi gamma in (0, gamma)
    np.testing.assert_allclose(s.ux[idx] + ph.ux[:n_ev], u0[idx], rtol=1e-14)
    assert np.all(ph.uy[:n_ev] == 0) and np.all(ph.ux[:n_ev] > 0)
    assert np.all(ph.ux[:n_ev] < g0)
    np.testing.assert_allclose(ph.w[:n_ev], s.w[idx], rtol=0)
    # the photon starts at x^{n+1/2}; the new depths come from draws 1 and 2
    np.testing.assert_allclose(ph.x[:n_ev], (x0[idx] + 0.5 * sim.grid.dt * ux / g0) % 1.6,
                               rtol=1e-14)
    for j, i in enumerate(idx[:20]):
        assert ph.tau[j] == -math.log(Q.uniform(5, 1, int(i), 2))
        assert tau[i] == -math.log(Q.uniform(5, 1, int(i), 1))
    # non-emitters move ballistically with q = 0
    np.testing.assert_allclose(s.x[~emit], (x0[~emit] + sim.grid.dt * ux / g0) % 1.6, rtol=1e-13)


def test_classical_depth_decrement():
    """At chi << 1 the depth falls by the classical photon number rate: W = 5 alpha chi /
    (2 sqrt3 gamma hbar_omega)."""
    Bz, ux = 5.0, 200.0
    sim = _uniform_box(B=(0, 0, Bz))
    hw = 1e-4 / (ux * Bz)                    # chi = 1e-4
    s = _beam(50, (ux, 0, 0), q=0.0)
    tau = np.full(s.n, 30.0)
    ph = Q.QedBuf(10)
    Q.qed_gather_push(sim, s, tau, hw, seed=1, step=0, photons=ph)
    g0 = math.sqrt(1 + ux * ux)
    W = 7.2973525693e-3 * 5 * 1e-4 / (2 * math.sqrt(3) * g0 * hw)
    assert ph.count == 0
    np.testing.assert_allclose(30.0 - tau, W * sim.grid.dt, rtol=3e-4)


def test_pair_statistics_and_conservation():
    Bx = 4.0
    km = 1000.0
    hw = 1.0 / (km * Bx)                      # chi_gamma = 1 for k perpendicular to B
    sim = _uniform_box(B=(Bx, 0, 0))
    n = 500
    ph = Q.QedBuf(n, count=n)
    rng = np.random.default_rng(3)
    ph.x[:] = rng.uniform(0, 1.6, n)
    ph.y[:] = rng.uniform(0, 1.6, n)
    ph.uy[:] = km
    ph.w[:] = rng.uniform(0.5, 1.5, n)
    ph.tau[:] = Q.init_tau(n, seed=9, step=0)
    tau0, x0, y0 = ph.tau.copy(), ph.x.copy(), ph.y.copy()
    pairs = Q.QedBuf(2 * n)
    Q.qed_photon_push(sim, 2, ph, hw, seed=9, step=1, pairs=pairs)
    dtau = 7.2973525693e-3 * Q.bw_rate(1.0) / (km * hw) * sim.grid.dt
    conv = tau0 - dtau <= 0
    m = int(conv.sum())
    p = 1 - math.exp(-dtau)
    assert abs(m - n * p) < 4 * math.sqrt(n * p * (1 - p)), (m, p)
    assert pairs.count == 2 * m
    assert np.all(ph.x[conv] == -1.0)
    e, q = slice(0, 2 * m, 2), slice(1, 2 * m, 2)
    np.testing.assert_array_equal(pairs.src[e], pairs.src[q])
    np.testing.assert_array_equal(pairs.src[e], np.nonzero(conv)[0])
    ge = np.sqrt(1 + pairs.uy[e] ** 2)
    gp = np.sqrt(1 + pairs.uy[q] ** 2)
    np.testing.assert_allclose(ge + gp, km, rtol=1e-12)        # energy shared by the pair
    assert np.all(pairs.ux[:2 * m] == 0) and np.all(pairs.uz[:2 * m] == 0)
    np.testing.assert_allclose(pairs.y[e], (y0[conv] + 0.5 * sim.grid.dt) % 1.6, rtol=1e-14)
    # survivors move by c dt along k
    np.testing.assert_allclose(ph.y[~conv], (y0[~conv] + sim.grid.dt) % 1.6, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(ph.x[~conv], x0[~conv])
    np.testing.assert_allclose(ph.tau[~conv], tau0[~conv] - dtau, atol=1e-12)


@pytest.mark.parametrize("ndim,order", [(2, 1), (2, 2), (3, 2)])
def test_push_without_events_is_the_plain_push(ndim, order):
    """With hbar_omega -> 0 there is no event, and the QED push is the oracle's push."""
    n = 12
    rng = np.random.default_rng(4)
    sim = OracleSim(ndim, n, n, n if ndim == 3 else 1, 0.1, 0.12, 0.09, 0.04)
    for k in ("ex", "ey", "ez", "bx", "by", "bz"):
        sim.f[k][:] = rng.uniform(-2, 2, sim.ncell)
    m = 300
    L = (n * 0.1, n * 0.12, n * 0.09)
    args = [rng.uniform(0, L[0], m), rng.uniform(0, L[1], m),
            rng.uniform(0, L[2], m) if ndim == 3 else None] + \
           [rng.normal(0, 3, m) for _ in range(3)] + [rng.uniform(0.5, 1, m)]
    a = OracleSpecies(-1.0, 1.0, order, *args)
    b = OracleSpecies(-1.0, 1.0, order, *args)
    sim.gather_push(a)
    tau = np.full(m, 1.0)
    ph = Q.QedBuf(4)
    Q.qed_gather_push(sim, b, tau, 1e-30, seed=1, step=0, photons=ph)
    assert ph.count == 0
    for k in ("x", "y", "z", "ux", "uy", "uz"):
        if getattr(a, k) is not None:
            np.testing.assert_array_equal(getattr(a, k), getattr(b, k))
