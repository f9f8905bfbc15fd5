"""Pins for the oracle's tree-level |M|^2 (helicity amplitudes + colour sum)."""
import math

import numpy as np
import pytest

import oracle as O

M = 173.0
AS = 0.118
GS2 = 4 * math.pi * AS


def esw(shat, c, m=M):
    """Averaged LO |M|^2 / g^4 for g g -> t tbar (Glueck-Owens-Reya 1978;
    Ellis-Stirling-Webber, QCD and Collider Physics)."""
    rho = 4 * m * m / shat
    b = math.sqrt(1 - rho)
    t1, t2 = (1 - b * c) / 2, (1 + b * c) / 2
    return (1 / (6 * t1 * t2) - 3 / 8) * (t1 * t1 + t2 * t2 + rho - rho * rho / (4 * t1 * t2))


def sigma_hat_ttx(shat, m=M, alpha_s=AS):
    """Closed-form LO partonic cross section in GeV^-2."""
    rho = 4 * m * m / shat
    b = math.sqrt(1 - rho)
    return math.pi * alpha_s**2 / (3 * shat) * (
        (1 + rho + rho * rho / 16) * math.log((1 + b) / (1 - b)) - b * (7 / 4 + 31 * rho / 16))


def ttx_momenta(rs, c, phi=0.0, m=M):
    E = rs / 2
    k = math.sqrt(E * E - m * m)
    s = math.sqrt(1 - c * c)
    kt = [E, k * s * math.cos(phi), k * s * math.sin(phi), k * c]
    kb = [E, -kt[1], -kt[2], -kt[3]]
    return np.array([kt, kb, [-E, 0, 0, -E], [-E, 0, 0, E]])


def random_momenta(n_g, rs, rng):
    nf = n_g
    kk, w, st = O.phase_space(nf, [M, M] + [0.0] * (nf - 2), rs, rng.random(3 * nf - 4))
    E = rs / 2
    return np.array([kk[0], kk[1], [-E, 0, 0, -E], [-E, 0, 0, E]] + [kk[i] for i in range(2, nf)])


def avg(n_g, p, width=0.0):
    return O.me2_sum(n_g, p, M, width) / (4 * 64 * math.factorial(n_g - 2))


@pytest.mark.parametrize("rs,c", [(500.0, 0.3), (400.0, -0.9), (2000.0, 0.99), (350.0, 0.0),
                                  (13000.0, -0.5)])
def test_ttx_matches_closed_form(rs, c):
    p = ttx_momenta(rs, c, phi=0.7)
    assert abs(avg(2, p) / esw(rs * rs, c) - 1) < 1e-13


def test_ttx_worked_point_value():
    p = ttx_momenta(500.0, 0.3)
    assert abs(avg(2, p) * GS2**2 - 0.54344845155) < 1e-10


def test_sigma_hat_by_quadrature_of_the_amplitude():
    """(1/(2s)) int dPhi_2 |M|^2 = sigma_hat: with dPhi_2 = beta/(32 pi^2) dOmega
    and Gauss-Legendre in cos(theta) the amplitude reproduces the closed form."""
    rs = 500.0
    s = rs * rs
    beta = math.sqrt(1 - 4 * M * M / s)
    xs, ws = np.polynomial.legendre.leggauss(64)
    integral = sum(w * avg(2, ttx_momenta(rs, c)) for c, w in zip(xs, ws)) * GS2**2
    sig = integral * 2 * math.pi * beta / (32 * math.pi**2) / (2 * s)
    assert abs(sig / sigma_hat_ttx(s) - 1) < 1e-12
    assert abs(sigma_hat_ttx(s) - 4.60349428e-8) < 1e-15
    assert abs(sigma_hat_ttx(s) * 0.3893793721e9 - 17.9250571) < 1e-6


@pytest.mark.parametrize("n_g", [2, 3])
def test_colour_decomposition_matches_colour_dressed_feynman_rules(n_g):
    rng = np.random.default_rng(20 + n_g)
    for _ in range(2):
        p = random_momenta(n_g, 900.0, rng)
        h = O.all_helicities(n_g)
        a = O.me2_sum_hel(n_g, p, M, 1.5, h)
        b = O.me2_sum_fullcolour(n_g, p, M, 1.5, h)
        assert abs(a / b - 1) < 1e-12


def test_colour_decomposition_ttgg_selected_helicities():
    rng = np.random.default_rng(40)
    p = random_momenta(4, 1100.0, rng)
    h = O.all_helicities(4)[[0, 13, 38, 63]]
    a = O.me2_sum_hel(4, p, M, 1.5, h)
    b = O.me2_sum_fullcolour(4, p, M, 1.5, h)
    assert abs(a / b - 1) < 1e-12


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_ward_identity_per_partial_amplitude(n_g):
    rng = np.random.default_rng(60 + n_g)
    for _ in range(3):
        p = random_momenta(n_g, 1000.0, rng)
        hel = rng.integers(0, 2, n_g + 2)
        ref = np.abs(O.partial_amplitudes(n_g, p, M, 0.0, hel)).max()
        for g in range(n_g):
            A = O.partial_amplitudes(n_g, p, M, 0.0, hel, ward_gluon=g)
            # the gauge term carries the momentum scale in place of a unit vector
            scale = ref * max(abs(p[2 + g][0]), 1.0)
            assert np.abs(A).max() < 1e-11 * scale


def lorentz(p, rng):
    """Random boost followed by a random rotation, applied to all momenta."""
    b = rng.normal(size=3)
    b *= 0.8 * rng.random() / np.linalg.norm(b)
    g = 1 / math.sqrt(1 - b @ b)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = g * b
    L[1:, 1:] += (g - 1) * np.outer(b, b) / (b @ b)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    R = np.eye(4)
    R[1:, 1:] = q
    return p @ (R @ L).T


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_lorentz_invariance(n_g):
    """Exact at zero width.  A finite top width breaks the Ward identity at
    O(m Gamma / (p^2 - m^2)), so the sum over polarisations transverse in a
    given frame picks up a frame dependence of that order (checked below);
    every evaluation here uses the partonic centre-of-mass frame."""
    rng = np.random.default_rng(80 + n_g)
    p = random_momenta(n_g, 1200.0, rng)
    ref = O.me2_sum(n_g, p, M, 0.0)
    for _ in range(2):
        q = lorentz(p, rng)
        assert abs(O.me2_sum(n_g, q, M, 0.0) / ref - 1) < 1e-11
    q = lorentz(p, rng)
    assert abs(O.me2_sum(n_g, q, M, 1.5) / O.me2_sum(n_g, p, M, 1.5) - 1) < 1e-4


def test_bose_symmetry():
    rng = np.random.default_rng(5)
    p = random_momenta(4, 1000.0, rng)
    ref = O.me2_sum(4, p, M, 1.5)
    swapped_final = p[[0, 1, 2, 3, 5, 4]]
    swapped_initial = p[[0, 1, 3, 2, 4, 5]]
    assert abs(O.me2_sum(4, swapped_final, M, 1.5) / ref - 1) < 1e-12
    assert abs(O.me2_sum(4, swapped_initial, M, 1.5) / ref - 1) < 1e-12
    p3 = random_momenta(3, 1000.0, rng)
    assert abs(O.me2_sum(3, p3[[0, 1, 3, 2, 4]], M, 1.5) / O.me2_sum(3, p3, M, 1.5) - 1) < 1e-12


def test_charge_conjugation_symmetry():
    """Swapping top and antitop momenta leaves the helicity- and colour-summed
    |M|^2 unchanged (C invariance of QCD)."""
    rng = np.random.default_rng(6)
    for n_g in (2, 3, 4):
        p = random_momenta(n_g, 1000.0, rng)
        q = p.copy()
        q[[0, 1]] = p[[1, 0]]
        assert abs(O.me2_sum(n_g, q, M, 1.5) / O.me2_sum(n_g, p, M, 1.5) - 1) < 1e-11


def test_width_effect_is_small():
    p = ttx_momenta(600.0, 0.4)
    a0, a1 = avg(2, p, 0.0), avg(2, p, 1.5)
    assert 0 < abs(a1 / a0 - 1) < 1e-4


def test_soft_gluon_limit_scaling():
    """A soft final gluon of energy E makes |M|^2 grow like 1/E^2 (eikonal
    factorisation), so E^2 |M|^2 tends to a constant.  Momenta are built to
    conserve exactly: tops at +/-q - E n/2, beams balancing the energy."""
    q = np.array([110.0, -40.0, 150.0])
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    vals = []
    for E in (1e-1, 1e-2, 1e-3):
        kt = q - E * n / 2
        kb = -q - E * n / 2
        Et = math.sqrt(M * M + kt @ kt)
        Eb = math.sqrt(M * M + kb @ kb)
        P0 = Et + Eb + E
        p = np.array([[Et, *kt], [Eb, *kb], [-P0 / 2, 0, 0, -P0 / 2], [-P0 / 2, 0, 0, P0 / 2],
                      [E, *(E * n)]])
        assert np.all(np.abs(p.sum(axis=0)) < 1e-12 * P0)
        vals.append(O.me2_sum(3, p, M, 0.0) * E * E)
    d1 = abs(vals[1] / vals[0] - 1)
    d2 = abs(vals[2] / vals[1] - 1)
    assert d2 < 1e-3 and d2 < 0.3 * d1 + 1e-9
