"""Pins for the oracle's phase-space generator (RAMBO family, Sec. 2.4)."""
import math

import numpy as np
import pytest
from scipy import integrate as si

import oracle as O

M = 173.0


def minkowski(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def test_massless_volume_closed_form():
    # (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!) evaluated by hand
    assert abs(O.massless_volume(2, 7.0) - 1 / (8 * math.pi)) < 1e-17
    assert abs(O.massless_volume(3, 1.0) - 1 / (256 * math.pi**3)) < 1e-19
    assert abs(O.massless_volume(4, 1.0) - 1 / (24576 * math.pi**5)) < 1e-22
    assert abs(O.massless_volume(3, 1.0) / 1.25983e-4 - 1) < 1e-5
    assert abs(O.massless_volume(4, 2.0) / (1.32966e-7 * 4) - 1) < 1e-5


@pytest.mark.parametrize("n_f", [2, 3, 4, 5])
def test_momentum_conservation_and_mass_shell(n_f):
    rng = np.random.default_rng(n_f)
    masses = [M, M] + [0.0] * (n_f - 2)
    for _ in range(300):
        rs = 2 * M + rng.exponential(400.0) + 1e-3
        k, w, st = O.phase_space(n_f, masses, rs, rng.random(3 * n_f - 4))
        assert st == 0 and w > 0
        tot = k.sum(axis=0)
        assert abs(tot[0] - rs) < 1e-12 * rs
        assert np.all(np.abs(tot[1:]) < 1e-12 * rs)
        for i in range(n_f):
            assert abs(minkowski(k[i], k[i]) - masses[i] ** 2) < 1e-10 * rs**2
            assert k[i][0] > 0


def test_two_body_massive_weight_is_beta_over_8pi():
    rng = np.random.default_rng(2)
    for _ in range(200):
        rs = 2 * M + rng.exponential(300.0) + 1e-6
        k, w, st = O.phase_space(2, [M, M], rs, rng.random(2))
        beta = math.sqrt(1 - 4 * M * M / rs**2)
        assert abs(w / (beta / (8 * math.pi)) - 1) < 1e-13
        assert abs(math.sqrt(k[0][1] ** 2 + k[0][2] ** 2 + k[0][3] ** 2) - beta * rs / 2) < 1e-12 * rs


@pytest.mark.parametrize("n_f", [3, 4, 5])
def test_massless_generator_is_flat(n_f):
    """Flat massless phase space: <s_ij> = 2 s/(n(n-1)) for every pair; for n = 3
    the Dalitz plot is uniform so <s_ij^2> = s^2 / 6."""
    rng = np.random.default_rng(10 + n_f)
    N = 20000
    s_ij = np.zeros((N, n_f, n_f))
    for e in range(N):
        k, w, st = O.phase_space(n_f, [0.0] * n_f, 1.0, rng.random(3 * n_f - 4))
        assert abs(w - O.massless_volume(n_f, 1.0)) < 1e-18
        for i in range(n_f):
            for j in range(i + 1, n_f):
                s_ij[e, i, j] = 2 * minkowski(k[i], k[j])
    expect = 2.0 / (n_f * (n_f - 1))
    for i in range(n_f):
        for j in range(i + 1, n_f):
            v = s_ij[:, i, j]
            assert abs(v.mean() - expect) < 5 * v.std() / math.sqrt(N)
            if n_f == 3:
                assert abs((v**2).mean() - 1 / 6) < 5 * (v**2).std() / math.sqrt(N)


@pytest.mark.parametrize("n_f", [3, 4, 5])
def test_massless_single_particle_energy_spectrum(n_f):
    """In flat massless n-body phase space the remaining n - 1 particles have
    invariant mass squared s (1 - x), x = 2E/sqrt(s), and their phase space
    grows like that to the power n - 3, so x of every particle follows
    x (1 - x)^(n - 3): Beta(2, n - 2).  Each particle is generated at a
    different step of the sequential construction (the mass-ratio equations
    of degree 1 .. n - 2), so each slot tests one of them."""
    from scipy import stats
    rng = np.random.default_rng(40 + n_f)
    N = 6000
    x = np.zeros((N, n_f))
    for e in range(N):
        k, w, st = O.phase_space(n_f, [0.0] * n_f, 1.0, rng.random(3 * n_f - 4))
        x[e] = 2 * k[:, 0]
    for i in range(n_f):
        assert stats.kstest(x[:, i], stats.beta(2, n_f - 2).cdf).pvalue > 1e-4, i


def test_three_body_massive_volume_matches_dalitz_quadrature():
    """Phi_3 = (1/(128 pi^3 s)) x (Dalitz-plot area in (m12^2, m23^2))."""
    rs, m1, m2, m3 = 1000.0, M, M, 0.0
    s = rs * rs

    def m23_range(m12sq):
        m12 = math.sqrt(m12sq)
        e2 = (m12sq - m1 * m1 + m2 * m2) / (2 * m12)
        e3 = (s - m12sq - m3 * m3) / (2 * m12)
        p2 = math.sqrt(max(e2 * e2 - m2 * m2, 0.0))
        p3 = math.sqrt(max(e3 * e3 - m3 * m3, 0.0))
        return (e2 + e3) ** 2 - (p2 + p3) ** 2, (e2 + e3) ** 2 - (p2 - p3) ** 2

    area, _ = si.quad(lambda m12sq: np.subtract(*m23_range(m12sq)[::-1]),
                      (m1 + m2) ** 2, (rs - m3) ** 2, epsabs=0, epsrel=1e-12, limit=200)
    exact = area / (128 * math.pi**3 * s)
    rng = np.random.default_rng(99)
    N = 40000
    ws = np.array([O.phase_space(3, [m1, m2, m3], rs, rng.random(5))[1] for _ in range(N)])
    assert abs(ws.mean() - exact) < 4 * ws.std() / math.sqrt(N)
    assert abs(exact - 74.856) < 0.01


def test_newton_failure_is_reported():
    k, w, st = O.phase_space(3, [M, M, 0.0], 600.0, np.full(5, 0.3), max_newton=0)
    assert st == 1 and w == 0.0


def test_newton_condition_number_closed_forms(pdf_table):
    """kappa_N = sqrt(s_hat) / (xi F'(xi)) of the mass-rescaling root.  For
    t tbar it is 1 / beta^2 = s_hat / (s_hat - 4 m^2) (both momenta have
    |k| = beta sqrt(s_hat) / 2 and E = sqrt(s_hat) / 2); for (nearly)
    massless tops the rescaling is the identity and kappa_N -> 1 for any
    number of particles, so a dropped or doubled term of the sum shows."""
    grid4 = np.tile(np.arange(51) / 50, (4, 1))
    seen = 0
    for e in range(400):
        _, ev = O.event_weight(O.Process(n_g=2), 13000.0, pdf_table, grid4, 11, 0, e)
        if not ev.pass_threshold or ev.newton_fail:
            assert ev.newton_kappa == 0.0 or ev.pass_threshold
            continue
        beta2 = 1.0 - 4.0 * 173.0**2 / ev.shat
        assert ev.newton_kappa == pytest.approx(1.0 / beta2, rel=1e-9 / beta2)
        seen += 1
    assert seen > 100
    for n_g in (2, 3, 4):
        D = 3 * n_g - 2
        grid = np.tile(np.arange(51) / 50, (D, 1))
        p = O.Process(n_g=n_g, m_top=1e-3)
        for e in range(50):
            _, ev = O.event_weight(p, 13000.0, pdf_table, grid, 5, 0, e)
            if ev.pass_threshold and not ev.newton_fail:
                # m^2 / E^2 corrections only
                assert abs(ev.newton_kappa - 1.0) < 1e-6, (n_g, e, ev.newton_kappa)


def test_newton_condition_number_flag(pdf_table):
    """Bit 6 of the event flags marks kappa_N > 1e3, and event_weights
    returns the same kappa_N as the single-event call."""
    grid4 = np.tile(np.arange(51) / 50, (4, 1))
    ids = np.arange(3000)
    w, fl, kap = O.event_weights(O.Process(n_g=2), 13000.0, pdf_table, grid4, 0, 0, ids,
                                 return_kappa=True)
    for e in (0, 7, 1234):
        _, ev = O.event_weight(O.Process(n_g=2), 13000.0, pdf_table, grid4, 0, 0, e)
        assert kap[e] == ev.newton_kappa
    assert np.array_equal((fl & 64) != 0, kap > 1e3)
