"""Pins for the oracle's full integrand and integration loop."""
import math

import numpy as np
import pytest
from scipy import integrate as si

import oracle as O
import workloads as W

M = 173.0
SQRT_S = 13000.0


def proc(n_g=2, **kw):
    d = dict(n_g=n_g, m_top=M, w_top=1.5, alpha_s=0.118, mu_f=173.0)
    d.update(kw)
    return O.Process(**d)


def sigma_hat(shat, m, alpha_s=0.118):
    rho = 4 * m * m / shat
    if rho >= 1:
        return 0.0
    b = math.sqrt(1 - rho)
    return math.pi * alpha_s**2 / (3 * shat) * (
        (1 + rho + rho * rho / 16) * math.log((1 + b) / (1 - b)) - b * (7 / 4 + 31 * rho / 16))


def gluon(x, q2=173.0**2):
    return x**-1.2 * (1 - x) ** 5 * (1 + 0.1 * math.log(q2))


def sigma_quadrature(m):
    """sigma = int dx1 dx2 g(x1) g(x2) sigma_hat(x1 x2 s), in pb, with the
    analytic synthetic gluon density, in logarithmic variables."""
    s = SQRT_S**2
    tau0 = 4 * m * m / s

    def inner(l1):
        x1 = math.exp(l1)
        lo = math.log(tau0 / x1)
        f = lambda l2: gluon(math.exp(l2)) * math.exp(l2) * sigma_hat(x1 * math.exp(l2) * s, m)
        return si.quad(f, lo, 0.0, epsabs=0, epsrel=1e-11, limit=200)[0] * gluon(x1) * x1

    v = si.quad(inner, math.log(tau0), 0.0, epsabs=0, epsrel=1e-10, limit=200)[0]
    return v * 0.3893793721e9


@pytest.fixture(scope="module")
def quad_sigma():
    return {m: sigma_quadrature(m) for m in (172.9, 173.0, 173.1)}


def test_quadrature_reference_values(quad_sigma):
    assert abs(quad_sigma[173.0] - 913.4845) < 2e-3


def test_ttx_hadronic_cross_section_matches_quadrature(pdf_table, quad_sigma):
    """The five-iteration VEGAS estimate of the g g -> t tbar hadronic cross
    section agrees with the 2-D quadrature of the closed form within its MC
    error, plus 5e-4 for PDF interpolation and the top width."""
    r = O.integrate(proc(), SQRT_S, pdf_table, 100_000, 5, seed=0)
    ref = quad_sigma[173.0]
    assert abs(r.sigma - ref) < 4 * r.sigma_err + 5e-4 * ref
    assert r.sigma_err / r.sigma < 5e-3
    assert r.chi2_dof < 5
    assert r.n_newton_fail == 0
    # VEGAS adaptation must reduce the variance
    assert r.iter_var[-1] < 0.5 * r.iter_var[0]


def test_iteration_sums_are_compensated(pdf_table):
    n = 50_000
    r = O.integrate(proc(), SQRT_S, pdf_table, n, 2, seed=3)
    exact = math.fsum(r.weights_last)
    assert abs(r.iter_sigma[-1] * n - exact) <= 4e-16 * abs(exact)
    assert O.neumaier_sum(r.weights_last) == exact or \
        abs(O.neumaier_sum(r.weights_last) - exact) <= 2.3e-16 * abs(exact)


def test_deterministic_and_thread_count_independent(pdf_table):
    a = O.integrate(proc(), SQRT_S, pdf_table, 20_000, 3, seed=1, n_threads=4)
    b = O.integrate(proc(), SQRT_S, pdf_table, 20_000, 3, seed=1, n_threads=4)
    c = O.integrate(proc(), SQRT_S, pdf_table, 20_000, 3, seed=1, n_threads=1)
    assert a.sigma == b.sigma and np.array_equal(a.grid, b.grid)
    # the per-thread histograms are added in a different order, so grids after
    # the first refinement differ at the rounding level only
    np.testing.assert_allclose(a.weights_last, c.weights_last, rtol=1e-12, atol=0)
    assert abs(a.sigma / c.sigma - 1) < 1e-13
    a1 = O.integrate(proc(), SQRT_S, pdf_table, 20_000, 1, seed=1, n_threads=4)
    c1 = O.integrate(proc(), SQRT_S, pdf_table, 20_000, 1, seed=1, n_threads=1)
    assert np.array_equal(a1.weights_last, c1.weights_last)


def test_resume_from_grid_is_identical(pdf_table):
    full = O.integrate(proc(), SQRT_S, pdf_table, 10_000, 4, seed=2, n_threads=2)
    first = O.integrate(proc(), SQRT_S, pdf_table, 10_000, 2, seed=2, n_threads=2)
    rest = O.integrate(proc(), SQRT_S, pdf_table, 10_000, 2, seed=2, n_threads=2,
                       grid=first.grid, start_iter=2)
    assert np.array_equal(full.grid, rest.grid)
    assert np.array_equal(full.iter_sigma[2:], rest.iter_sigma)
    assert np.array_equal(full.weights_last, rest.weights_last)


def test_alpha_s_scaling_is_exact(pdf_table):
    grid = np.tile(np.arange(51) / 50, (7, 1))
    for e in range(50):
        w1, ev = O.event_weight(proc(3, ptmin_g=20.0), SQRT_S, pdf_table, grid, 0, 0, e)
        w2, _ = O.event_weight(proc(3, ptmin_g=20.0, alpha_s=0.118 * 1.01), SQRT_S, pdf_table,
                               grid, 0, 0, e)
        assert abs(w2 - w1 * 1.01**3) <= 1e-14 * abs(w1) + 1e-300


def esw_weight(y, m, pdf_table, grid):
    """Event weight of g g -> t tbar from the closed-form |M|^2 (zero width)."""
    _, ev = O.event_weight_y(proc(m_top=m, w_top=0.0), SQRT_S, pdf_table, grid, y)
    x1, x2 = ev.x[0], ev.x[1]
    s = x1 * x2 * SQRT_S**2
    rho = 4 * m * m / s
    if rho >= 1:
        return 0.0
    b = math.sqrt(1 - rho)
    c = 2 * ev.x[2] - 1
    t1, t2 = (1 - b * c) / 2, (1 + b * c) / 2
    F = (1 / (6 * t1 * t2) - 3 / 8) * (t1 * t1 + t2 * t2 + rho - rho * rho / (4 * t1 * t2))
    g4 = (4 * math.pi * 0.118) ** 2
    return ev.jac * b / (8 * math.pi) * ev.f1 * ev.f2 * g4 * F / (2 * s) * 0.3893793721e9


def test_analytic_mt_gradient_matches_finite_differences(pdf_table):
    rng = np.random.default_rng(12)
    grid = np.tile(np.arange(51) / 50, (4, 1))
    checked = 0
    for y in rng.random((300, 4)):
        g, w = O.ttx_dweight_dmt_analytic(proc(w_top=0.0), SQRT_S, pdf_table, grid, y)
        if w == 0.0:
            continue
        h = 1e-4 * M
        # finite differences of the amplitude-based oracle weight at zero width
        wp, _ = O.event_weight_y(proc(m_top=M + h, w_top=0.0), SQRT_S, pdf_table, grid, y)
        wm, _ = O.event_weight_y(proc(m_top=M - h, w_top=0.0), SQRT_S, pdf_table, grid, y)
        if wm == 0.0 or wp == 0.0:
            continue
        fd = (wp - wm) / (2 * h)
        assert abs(fd - g) < 1e-6 * abs(g) + 1e-9 * abs(w)
        # and of the closed-form weight
        fd2 = (esw_weight(y, M + h, pdf_table, grid) - esw_weight(y, M - h, pdf_table, grid)) / (2 * h)
        assert abs(fd2 - g) < 1e-6 * abs(g) + 1e-9 * abs(w)
        assert abs(esw_weight(y, M, pdf_table, grid) / w - 1) < 1e-13
        checked += 1
    assert checked > 250


def test_integrated_mt_gradient_matches_quadrature(pdf_table, quad_sigma):
    """Mean of the analytic per-event gradient over uniform samples of the unit
    cube (uniform grid) vs the central difference of the quadrature."""
    rng = np.random.default_rng(21)
    grid = np.tile(np.arange(51) / 50, (4, 1))
    ys = rng.random((40_000, 4))
    gs = np.array([O.ttx_dweight_dmt_analytic(proc(w_top=0.0), SQRT_S, pdf_table, grid, y)[0]
                   for y in ys])
    est, err = gs.mean(), gs.std() / math.sqrt(len(gs))
    ref = (quad_sigma[173.1] - quad_sigma[172.9]) / 0.2
    assert abs(ref - (-17.738)) < 0.01
    assert abs(est - ref) < 5 * err + 1e-3 * abs(ref)
