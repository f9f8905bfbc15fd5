"""Pins for the oracle's log-bicubic PDF interpolation."""
import math

import numpy as np
from scipy import integrate as si
from scipy.special import beta as beta_fn

import oracle as O
import workloads


def test_knot_values_reproduced(pdf_table):
    t = pdf_table
    for m in (0, 1, 24, 25, 48, 49):
        for k in (0, 1, 37, 97, 98):
            v = O.pdf_xf(t, math.exp(t.log_x[k]), math.exp(t.log_q2[m]))
            assert abs(v - t.xf[m, k]) <= 1e-13 * abs(t.xf[m, k])


def test_exact_for_quadratics_in_logs():
    """With uniform log spacing the centred secant mean is the exact slope of a
    quadratic, so a table quadratic in ln x times quadratic in ln Q^2 is
    reproduced exactly away from the first and last intervals."""
    base = workloads.synthetic_pdf()
    lx, lq = base.log_x, base.log_q2
    f = lambda a, b: (3.0 + 0.3 * a + 0.02 * a * a) * (2.0 - 0.1 * b + 0.004 * b * b)
    tab = workloads.PdfTable(lx, lq, np.ascontiguousarray(f(lx[None, :], lq[:, None])))
    rng = np.random.default_rng(4)
    for _ in range(400):
        a = rng.uniform(lx[1], lx[-2])
        b = rng.uniform(lq[1], lq[-2])
        v = O.pdf_xf(tab, math.exp(a), math.exp(b))
        assert abs(v - f(a, b)) < 1e-12 * abs(f(a, b))


def test_momentum_integral_matches_beta_function(pdf_table):
    """int_0^1 x g(x) dx = B(0.8, 6)(1 + 0.1 ln Q^2) for the synthetic table."""
    q2 = 173.0**2
    val, _ = si.quad(lambda lnx: O.pdf_xf(pdf_table, math.exp(lnx), q2) * math.exp(lnx),
                     math.log(1e-7), 0.0, limit=400, epsrel=1e-10)
    exact = beta_fn(0.8, 6.0) * (1 + 0.1 * math.log(q2))
    assert abs(exact - 0.5713) < 1e-3
    assert abs(val / exact - 1) < 2e-4


def test_interpolation_error_is_small_over_the_physical_range(pdf_table):
    """Above x ~ 0.3 the factor (1 - x)^5 changes by tens of percent between
    knots 7/99 decades apart and the relative error grows; the weight there is
    negligible.  Over the threshold-to-0.3 range the error stays below 5e-4."""
    q2 = 173.0**2
    for x in np.geomspace(7e-4, 0.3, 200):
        exact = x**-0.2 * (1 - x) ** 5 * (1 + 0.1 * math.log(q2))
        assert abs(O.pdf_xf(pdf_table, x, q2) / exact - 1) < 5e-4


def test_interpolant_overshoot_is_flagged_ill_conditioned(pdf_table):
    """The cubic in the last x interval overshoots below zero (the one-sided
    end slope misses the (1 - x)^5 flatness at x = 1); near its zero crossing
    the relative value is ill-conditioned and the event is flagged."""
    q2 = 173.0**2
    xs = np.linspace(0.70, 0.999, 3000)
    vals = np.array([O.pdf_xf(pdf_table, x, q2) for x in xs])
    assert vals.min() < 0 < vals.max()
    x0 = xs[np.argmin(np.abs(vals))]
    grid = np.tile(np.arange(51) / 50, (4, 1))
    y_bad = np.array([0.1, x0, 0.3, 0.4])
    y_bad[0] = 0.5
    _, ev = O.event_weight_y(O.Process(n_g=2), 13000.0, pdf_table, grid, y_bad)
    assert ev.pass_cuts and ev.ill_conditioned
    _, ev = O.event_weight_y(O.Process(n_g=2), 13000.0, pdf_table, grid, np.array([0.05, 0.1, 0.3, 0.4]))
    assert ev.pass_cuts and not ev.ill_conditioned
