"""Pins for the oracle's quark channels and the p p -> t tbar integrand.

The paper's pp processes (Sec. 3, Table 1) sum the g g channel and the
q qbar channels; for p p -> t tbar these are u ubar, ubar u, d dbar and
dbar d, one s-channel gluon each (7 diagrams with the 3 of g g).

* q qbar -> t tbar against the Glueck-Owens-Reya / Ellis-Stirling-Webber
  closed form (4/9)(tau1^2 + tau2^2 + rho/2) g^4, point by point; the
  partonic cross section by quadrature of the amplitude against
  8 pi alpha_s^2 beta (1 + rho/2) / (27 s); Lorentz invariance; the colour
  factor by an explicit sum over Gell-Mann generators.
* The quark tables: knot values exactly, the interpolation error against the
  analytic synthetic densities.
* The event weight: its assembly from the PDF tables and both orientations
  of the q qbar channel; the hadronic cross section against a 2-D quadrature
  of the closed forms with the analytic densities.
"""
import math

import numpy as np
import pytest
from scipy import integrate as si

import oracle as O
import workloads as W
from test_oracle_integrate import SQRT_S, gluon, sigma_hat
from test_oracle_me import M, lorentz, ttx_momenta
from test_oracle_soft_limit import T as GM_T

AS = 0.118
GS2 = 4 * math.pi * AS


@pytest.fixture(scope="module")
def pp_table():
    return W.synthetic_pdf(quarks=True)


def qqbar_closed_form(rs, c, m=M):
    rho = 4 * m * m / (rs * rs)
    b = math.sqrt(1 - rho)
    t1, t2 = (1 - b * c) / 2, (1 + b * c) / 2
    return 4 / 9 * (t1 * t1 + t2 * t2 + rho / 2)


@pytest.mark.parametrize("rs,c", [(500.0, 0.3), (400.0, -0.9), (2000.0, 0.99), (350.0, 0.0), (13000.0, -0.5),
                                  (346.1, 0.7)])
def test_qqbar_matches_closed_form(rs, c):
    p = ttx_momenta(rs, c, phi=0.4)
    assert abs(O.me2_qqbar_ttx(p, M) / 36 / qqbar_closed_form(rs, c) - 1) < 1e-13


def sigma_hat_qq(shat, m=M, alpha_s=AS):
    rho = 4 * m * m / shat
    if rho >= 1:
        return 0.0
    b = math.sqrt(1 - rho)
    return 8 * math.pi * alpha_s**2 / (27 * shat) * b * (1 + rho / 2)


def test_qqbar_sigma_hat_by_quadrature_of_the_amplitude():
    rs = 700.0
    s = rs * rs
    beta = math.sqrt(1 - 4 * M * M / s)
    xs, ws = np.polynomial.legendre.leggauss(32)
    integral = sum(w * O.me2_qqbar_ttx(ttx_momenta(rs, c), M) / 36 for c, w in zip(xs, ws)) * GS2**2
    sig = integral * 2 * math.pi * beta / (32 * math.pi**2) / (2 * s)
    assert abs(sig / sigma_hat_qq(s) - 1) < 1e-12


def test_qqbar_lorentz_invariance_and_forward_backward_symmetry():
    rng = np.random.default_rng(7)
    p = ttx_momenta(800.0, 0.37, 1.1)
    ref = O.me2_qqbar_ttx(p, M)
    for _ in range(3):
        assert abs(O.me2_qqbar_ttx(lorentz(p, rng), M) / ref - 1) < 1e-12
    # exchanging the quark and the antiquark beams: t <-> u, symmetric at tree level
    q = p[[0, 1, 3, 2]]
    assert abs(O.me2_qqbar_ttx(q, M) / ref - 1) < 1e-13


def test_qqbar_colour_factor_by_explicit_sum():
    """sum over a, i, j, k, l of |T^a_ji T^a_kl|^2 = 2 (the factor the oracle uses)."""
    amp = np.einsum("aji,akl->ijkl", GM_T, GM_T)
    assert abs(np.sum(np.abs(amp) ** 2) - 2.0) < 1e-13


def analytic_quarks(x, q2=173.0**2):
    fq = 1 + 0.1 * math.log(q2)
    ubar = 0.09 * x**-0.2 * (1 - x) ** 7
    dbar = 0.11 * x**-0.2 * (1 - x) ** 7
    return (fq * (1.6 * x**0.55 * (1 - x) ** 3.2 + ubar), fq * ubar,
            fq * (0.85 * x**0.55 * (1 - x) ** 4 + dbar), fq * dbar)


def test_quark_tables_interpolate_the_analytic_densities(pp_table):
    t = pp_table
    lx, lq = t.log_x, t.log_q2
    for f in range(4):
        for i in (3, 40, 77):
            for j in (5, 20, 44):
                assert O.pdf_xq(t, f, math.exp(lx[i]), math.exp(lq[j])) == pytest.approx(t.xq[f, j, i], rel=1e-14)
    for x in (3e-4, 0.01, 0.13, 0.4):
        ref = analytic_quarks(x)
        for f in range(4):
            assert O.pdf_xq(t, f, x, 173.0**2) == pytest.approx(ref[f], rel=2e-4)
    assert math.isnan(O.pdf_xq(W.synthetic_pdf(), 0, 0.1, 173.0**2))


def test_pp_event_weight_assembly(pp_table):
    """w = J_V W / (2 s_hat) [g g f_g f_g |M|^2_gg + (u ubar + d dbar)(x1, x2)
    |M|^2_qq + (ubar u + dbar d)(x1, x2) |M|^2_qq(beams exchanged)] in pb."""
    proc = O.Process(n_g=2, initial="pp")
    gg = O.Process(n_g=2)
    grid = np.tile(np.arange(51) / 50, (4, 1))
    q2 = 173.0**2
    checked = 0
    for e in range(60):
        w, ev = O.event_weight(proc, SQRT_S, pp_table, grid, 5, 0, e)
        wg, evg = O.event_weight(gg, SQRT_S, pp_table, grid, 5, 0, e)
        if not ev.pass_threshold:
            assert w == 0.0
            continue
        x1, x2 = ev.x[0], ev.x[1]
        rs = math.sqrt(ev.shat)
        k = ev.k
        p = np.array([k[0], k[1], [-rs / 2, 0, 0, -rs / 2], [-rs / 2, 0, 0, rs / 2]])
        mq = GS2**2 * O.me2_qqbar_ttx(p, M) / 36
        mqr = GS2**2 * O.me2_qqbar_ttx(p[[0, 1, 3, 2]], M) / 36
        u1, ub1, d1, db1 = (O.pdf_xq(pp_table, f, x1, q2) / x1 for f in range(4))
        u2, ub2, d2, db2 = (O.pdf_xq(pp_table, f, x2, q2) / x2 for f in range(4))
        lq = u1 * ub2 + d1 * db2
        lr = ub1 * u2 + db1 * d2
        quark = ev.jac * ev.ps_weight * (lq * mq + lr * mqr) / (2 * ev.shat) * 0.3893793721e9
        assert w == pytest.approx(wg + quark, rel=1e-13)
        assert ev.me2_q[0] == pytest.approx(mq, rel=1e-14) and ev.lum_q[1] == pytest.approx(lr, rel=1e-14)
        checked += 1
    assert checked > 30


def sigma_pp_quadrature(m=M):
    """sigma(p p -> t tbar) = int dx1 dx2 [g g sigma_gg + (u ubar + d dbar
    + ubar u + dbar d) sigma_qq] with the analytic synthetic densities, pb."""
    s = SQRT_S**2
    tau0 = 4 * m * m / s

    def lum(x1, x2):
        a, b = analytic_quarks(x1), analytic_quarks(x2)
        qq = (a[0] * b[1] + a[2] * b[3] + a[1] * b[0] + a[3] * b[2]) / (x1 * x2)
        return gluon(x1) * gluon(x2), qq

    def inner(l1):
        x1 = math.exp(l1)
        lo = math.log(tau0 / x1)

        def f(l2):
            x2 = math.exp(l2)
            g, q = lum(x1, x2)
            sh = x1 * x2 * s
            return x1 * x2 * (g * sigma_hat(sh, m) + q * sigma_hat_qq(sh, m))
        return si.quad(f, lo, 0.0, epsabs=0, epsrel=1e-11, limit=200)[0]

    return si.quad(inner, math.log(tau0), 0.0, epsabs=0, epsrel=1e-10, limit=200)[0] * 0.3893793721e9


def test_pp_hadronic_cross_section_matches_quadrature(pp_table):
    ref = sigma_pp_quadrature()
    gg_only = 913.4845
    assert ref > gg_only * 1.02            # the quark channels add a few percent
    r = O.integrate(O.Process(n_g=2, initial="pp"), SQRT_S, pp_table, 100_000, 5, seed=0)
    print(f"\n  p p -> t tbar: VEGAS {r.sigma:.5f} +- {r.sigma_err:.5f} pb, quadrature {ref:.5f} pb")
    assert abs(r.sigma - ref) < 4 * r.sigma_err + 5e-4 * ref
    assert r.sigma_err / r.sigma < 5e-3
