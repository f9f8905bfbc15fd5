"""Pins for the oracle's iteration estimates, their combination and the cuts.

* The combination of iterations (inverse-variance weighted mean, its error
  and chi^2/dof) against exact rational arithmetic and 50-digit square roots.
* V_j = [(1/N) sum w^2 - I_j^2] / (N - 1), the variance of the iteration
  estimate with the N - 1 denominator, against the two-pass form
  sum (w - I_j)^2 / (N (N - 1)) of the oracle's own per-event weights,
  summed with math.fsum.
* The fiducial cuts (pT, lab |eta|, Delta R with the azimuthal difference
  folded into [0, pi]) against an independent numpy evaluation from the
  momenta (arcsinh for the rapidity, the modulo fold for the azimuth), on
  both sides of every cut.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle as O

SQRT_S = 13000.0


# ---------------------------------------------------------------- combination

def exact_combine(I, V):
    """sigma, sigma_err, chi^2/dof of the iterations with V_j > 0, from the
    exact rationals of the given doubles (sqrt at 50 digits)."""
    used = [(Fraction(i), Fraction(v)) for i, v in zip(I, V) if v > 0]
    if not used:
        return float(I[-1]), 0.0, 0.0
    s_inv = sum(1 / v for _, v in used)
    mean = sum(i / v for i, v in used) / s_inv
    mpmath.mp.dps = 50
    err = mpmath.mpf(1) / mpmath.sqrt(mpmath.mpf(s_inv.numerator) / s_inv.denominator)
    chi = Fraction(0)
    if len(used) > 1:
        chi = sum((i - mean) ** 2 / v for i, v in used) / (len(used) - 1)
    return float(mean), float(err), float(chi)


def check(I, V, tol_chi=1e-13):
    s, e, c = O.combine(np.array(I, float), np.array(V, float))
    rs, re_, rc = exact_combine(I, V)
    assert s == pytest.approx(rs, rel=1e-15, abs=0), (s, rs)
    assert e == pytest.approx(re_, rel=1e-15, abs=0), (e, re_)
    assert c == pytest.approx(rc, rel=tol_chi, abs=1e-300), (c, rc)
    return s, e, c


def test_combine_hand_example():
    # sum 1/V = 15, sum I/V = 14.25: sigma = 0.95, err = 15^-1/2,
    # chi^2/dof = (0.05^2 4 + 0.55^2 2 + 0.2^2 8 + 0.3^2) / 3 = 1.025 / 3
    s, e, c = check([1.0, 1.5, 0.75, 1.25], [0.25, 0.5, 0.125, 1.0])
    assert s == pytest.approx(0.95, rel=1e-15)
    assert e == pytest.approx(1 / math.sqrt(15), rel=1e-15)
    assert c == pytest.approx(1.025 / 3, rel=1e-14)
    # the plausible mistakes give other numbers
    assert abs(e - 1 / 15) > 0.1 and abs(c - 1.025 / 4) > 0.05


def test_combine_skips_zero_variance_and_single_iteration():
    s, e, c = check([2.0, 3.0, 5.0], [0.0, 0.5, 0.5])
    assert (s, e, c) == (4.0, 0.5, 4.0)
    s, e, c = check([7.0], [0.09])
    assert s == pytest.approx(7.0, rel=1e-15) and e == pytest.approx(0.3, rel=1e-15) and c == 0.0
    # no iteration with a variance: the last estimate, no error
    assert O.combine(np.array([1.0, 2.0]), np.array([0.0, 0.0])) == (2.0, 0.0, 0.0)


@pytest.mark.parametrize("n_iter", [2, 5, 10, 300])
def test_combine_random_against_exact(n_iter):
    rng = np.random.default_rng(n_iter)
    I = 900.0 + 10.0 * rng.standard_normal(n_iter)
    V = (1.0 + rng.exponential(size=n_iter)) * 25.0
    check(list(I), list(V))


# ------------------------------------------------------------ iteration variance

@pytest.mark.parametrize("n_events,n_g", [(2, 2), (3, 2), (5000, 2), (400, 3)])
def test_iteration_variance_two_pass(pdf_table, n_events, n_g):
    kw = dict(ptmin_g=20.0, etamax_g=2.5) if n_g == 3 else {}
    r = O.integrate(O.Process(n_g=n_g, **kw), SQRT_S, pdf_table, n_events, 1, seed=11)
    w = r.weights_last
    N = len(w)
    I = math.fsum(w) / N
    V = math.fsum((x - I) ** 2 for x in w) / (N * (N - 1))
    assert r.iter_sigma[0] == pytest.approx(I, rel=1e-15, abs=0)
    assert r.iter_var[0] == pytest.approx(V, rel=1e-11, abs=1e-300)
    # with N in place of N - 1 the estimate would be off by N/(N-1)
    if N < 10:
        assert abs(r.iter_var[0] * N / (N - 1) - V) > 1e-3 * V
    # the combination of one iteration reports sqrt(V) as its error
    assert r.sigma_err == pytest.approx(math.sqrt(V), rel=1e-11)
    assert r.w_max == max(w)


def test_two_event_variance_closed_form(pdf_table):
    # N = 2: V = (w0 - w1)^2 / 4
    r = O.integrate(O.Process(n_g=2), SQRT_S, pdf_table, 2, 1, seed=3)
    w0, w1 = r.weights_last
    assert r.iter_var[0] == pytest.approx((w0 - w1) ** 2 / 4, rel=1e-14)


def test_integrate_rejects_more_than_256_iterations(pdf_table):
    with pytest.raises(ValueError):
        O.integrate(O.Process(n_g=2), SQRT_S, pdf_table, 10, 257, seed=0)


# --------------------------------------------------------------------- cuts

def gluon(pt, eta, phi):
    return [pt * math.cosh(eta), pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta)]


def numpy_cuts(k, y_boost, ptmin, etamax, drmin):
    """(pass, near) from the gluon momenta k[2:], written independently."""
    g = np.asarray(k[2:], dtype=float)
    pt = np.hypot(g[:, 1], g[:, 2])
    eta = np.arcsinh(g[:, 3] / pt)
    phi = np.arctan2(g[:, 2], g[:, 1])
    ok, near = True, False
    rel = lambda v, c: abs(v - c) < 1e-9 * abs(c)
    for i in range(len(g)):
        if ptmin > 0:
            ok &= bool(pt[i] > ptmin)
            near |= rel(pt[i], ptmin)
        if etamax > 0:
            a = abs(eta[i] + y_boost)
            ok &= bool(a < etamax)
            near |= rel(a, etamax)
    if drmin > 0:
        for i in range(len(g)):
            for j in range(i + 1, len(g)):
                dphi = abs(math.remainder(phi[i] - phi[j], 2 * math.pi))
                dr = math.hypot(eta[i] - eta[j], dphi)
                ok &= bool(dr > drmin)
                near |= rel(dr, drmin)
    return ok, near


def random_event(rng, n_f, wrap):
    """Tops (never cut) and n_f - 2 gluons spread around both sides of every
    cut; with `wrap` the two gluons straddle the azimuthal branch cut at +-pi
    with a small true gap."""
    tops = [[400.0, 10.0, -5.0, 300.0], [380.0, -10.0, 5.0, -250.0]]
    pts = rng.uniform(5.0, 60.0, n_f - 2)
    eta0 = rng.uniform(-4.0, 4.0)
    if n_f == 3:
        etas, phis = [eta0], [rng.uniform(-math.pi, math.pi)]
    elif wrap:
        a, b = rng.uniform(0.0, 0.35, 2)
        etas, phis = [eta0, eta0 + rng.uniform(-0.4, 0.4)], [math.pi - a, -math.pi + b]
    else:
        phi0 = rng.uniform(-math.pi, math.pi)
        etas = [eta0, eta0 + rng.uniform(-0.6, 0.6)]
        phis = [phi0, phi0 + rng.uniform(-0.6, 0.6)]
    if n_f == 5:      # a third gluon close to one of the first two
        j = rng.integers(0, 2)
        etas.append(etas[j] + rng.uniform(-0.6, 0.6))
        phis.append(phis[j] + rng.uniform(-0.6, 0.6))
    return np.array(tops + [gluon(p, e, f) for p, e, f in zip(pts, etas, phis)])


@pytest.mark.parametrize("n_f,cuts", [
    (3, (20.0, 2.5, 0.0)), (3, (20.0, 0.0, 0.0)), (3, (0.0, 2.5, 0.0)),
    (4, (20.0, 0.0, 0.4)), (4, (0.0, 0.0, 0.4)), (4, (20.0, 2.5, 0.4)), (4, (0.0, 2.5, 0.0)),
    (5, (20.0, 0.0, 0.4)), (5, (20.0, 2.5, 0.4)),
])
def test_cuts_against_independent_evaluation(n_f, cuts):
    ptmin, etamax, drmin = cuts
    proc = O.Process(n_g=n_f, ptmin_g=ptmin, etamax_g=etamax, drmin_gg=drmin)
    rng = np.random.default_rng(1000 * n_f + int(10 * sum(cuts)))
    n_pass = n_fail = n_wrap_fail = compared = 0
    for t in range(4000):
        wrap = n_f >= 4 and t % 2 == 1
        k = random_event(rng, n_f, wrap)
        yb = rng.uniform(-1.5, 1.5)
        ok, near = O.cuts(proc, k, yb)
        ref, ref_near = numpy_cuts(k, yb, ptmin, etamax, drmin)
        if near or ref_near:
            continue
        compared += 1
        assert ok == ref, (t, k, yb, ok, ref)
        n_pass += ok
        n_fail += not ok
        if wrap and drmin > 0 and not ok:
            n_wrap_fail += 1
    assert compared > 3900
    # both sides of the cuts are exercised
    assert n_pass > 200 and n_fail > 200, (n_pass, n_fail)
    if n_f >= 4 and drmin > 0:
        assert n_wrap_fail > 100


def test_cuts_leave_the_tops_alone():
    proc = O.Process(n_g=3, ptmin_g=20.0, etamax_g=2.5)
    k = np.array([[500.0, 0.0, 0.0, 500.0 - 1e-9], [500.0, 0.0, 0.0, -499.0],
                  gluon(30.0, 0.3, 1.0)])
    assert O.cuts(proc, k, 0.0) == (True, False)


def test_cut_edges_are_strict_and_flagged():
    proc = O.Process(n_g=3, ptmin_g=20.0)
    tops = [[400.0, 0, 0, 300.0], [400.0, 0, 0, -300.0]]
    _, near = O.cuts(proc, np.array(tops + [gluon(20.0, 0.1, 0.2)]), 0.0)
    assert near
    ok, near = O.cuts(proc, np.array(tops + [gluon(20.0 * (1 + 1e-6), 0.1, 0.2)]), 0.0)
    assert ok and not near
    ok, near = O.cuts(proc, np.array(tops + [gluon(20.0 * (1 - 1e-6), 0.1, 0.2)]), 0.0)
    assert not ok and not near
