"""Pins for the oracle's q qbar -> t tbar g (the q qbar channel of the
paper's p p -> t tbar g, Sec. 3, Table 1: 5 diagrams per quark group, 36
with the 16 of g g) and the p p -> t tbar g event weight.

* Colour: the diagrams' colour-factor products summed over all 648 colour
  assignments against closed forms from SU(3) trace identities.
* Gauge invariance: the gluon polarisation replaced by its momentum gives a
  vanishing amplitude for every colour assignment (zero width); a wrong
  relative phase or sign of the three-gluon diagram fails it.
* The initial-state collinear limit, gluon along either beam:
  |M|^2 -> (1/x) (2 g^2 / (2 p.k)) C_F (1 + x^2)/(1 - x) |M_Born(x p)|^2
  with the pinned q qbar -> t tbar Born; the same limit formula with P_gg
  reproduces the pinned g g -> t tbar g (azimuthal average), which fixes its
  normalisation independently.
* Lorentz invariance and charge conjugation (quark <-> antiquark beams
  together with t <-> tbar).
* The p p -> t tbar g weight: its assembly from the tables and both beam
  orientations.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_oracle_me import lorentz

M = 173.0
AS = 0.118
GS2 = 4 * math.pi * AS
CUTS = dict(ptmin_g=20.0, etamax_g=2.5)


def ttxg_point(rs, r):
    k, w, st = O.phase_space(3, [M, M, 0.0], rs, r)
    e = rs / 2
    return np.array([k[0], k[1], [-e, 0, 0, -e], [-e, 0, 0, e], k[2]])


@pytest.fixture(scope="module")
def colour_table():
    cols = list(itertools.product(range(3), range(3), range(3), range(3), range(8)))
    return np.array([O.qqbar_ttxg_colour(c) for c in cols])


def test_colour_factors_against_trace_identities(colour_table):
    """K_dd' = sum over colours of C_d C_d'^*.  With Tr(T^a T^b) = delta/2,
    sum_a T^a T^a = C_F, T^a T^b T^a = -T^b / (2 N), Tr(T^a T^b T^c) =
    (d^abc + i f^abc)/4, sum d^2 = 40/3, sum f^2 = 24:
    K_11 = K_22 = K_33 = K_44 = C_F (N^2 - 1)/4 = 8/3, K_12 = K_34 = -1/3,
    K_13 = (40/3 + 24)/16 = 7/3, K_14 = (40/3 - 24)/16 = -2/3,
    K_15 = i sum f^2 / 8 = 3 i, K_55 = C_A (N^2 - 1)/4 = 6."""
    C = colour_table
    K = C.T @ C.conj()
    assert np.allclose(K, K.conj().T, atol=1e-14)
    for (d, e), v in {(0, 0): 8 / 3, (1, 1): 8 / 3, (2, 2): 8 / 3, (3, 3): 8 / 3, (0, 1): -1 / 3,
                      (2, 3): -1 / 3, (0, 2): 7 / 3, (1, 3): 7 / 3, (0, 3): -2 / 3, (1, 2): -2 / 3,
                      (0, 4): 3j, (4, 4): 6.0}.items():
        assert abs(K[d, e] - v) < 1e-13, (d, e, K[d, e])


@pytest.mark.parametrize("rs,seed", [(900.0, 3), (2500.0, 4), (400.0, 5)])
def test_ward_identity_every_colour_assignment(colour_table, rs, seed):
    """Relative to the largest colour-dressed term of any configuration of
    the point (helicity-violating configurations vanish to rounding)."""
    p = ttxg_point(rs, np.random.default_rng(seed).random(5))
    hels = [[h & 1, (h >> 1) & 1, (h >> 2) & 1, (h >> 3) & 1, 0] for h in range(16)]
    ward = [O.qqbar_ttxg_diagrams(p, M, 0.0, hel, ward=True) for hel in hels]
    scale = max(np.abs(colour_table * aw).sum(axis=1).max() for aw in ward)
    assert scale > 0.0
    for h, aw in enumerate(ward):
        assert np.abs(colour_table @ aw).max() <= 1e-14 * scale, h
    # the check has teeth: a sign flip of the three-gluon diagram breaks it
    hel = [1, 0, 0, 0, 0]
    aw = O.qqbar_ttxg_diagrams(p, M, 0.0, hel, ward=True)
    aw[4] = -aw[4]
    assert np.abs(colour_table @ aw).max() > 1e-3 * np.abs(aw).max()


def boost(p, b):
    b2 = b @ b
    g = 1 / math.sqrt(1 - b2)
    bp = b @ p[1:]
    return np.array([g * (p[0] + bp), *(p[1:] + ((g - 1) * bp / b2 + g * p[0]) * b)])


def pair(Q, nhat, m=M):
    """t, tbar back to back along +-nhat in the rest frame of Q, boosted to Q."""
    q2 = Q[0] ** 2 - Q[1:] @ Q[1:]
    ps = math.sqrt(q2 / 4 - m * m)
    e = math.sqrt(q2) / 2
    b = Q[1:] / Q[0]
    return boost(np.array([e, *(ps * nhat)]), b), boost(np.array([e, *(-ps * nhat)]), b)


def collinear_ratio(beam, x, delta, phi, me_born, me_real, split):
    e = 600.0
    pa, pb = np.array([e, 0, 0, e]), np.array([e, 0, 0, -e])
    nhat = np.array([math.sin(1.1) * math.cos(0.7), math.sin(1.1) * math.sin(0.7), math.cos(1.1)])
    sgn = 1.0 if beam == 0 else -1.0
    par = pa if beam == 0 else pb
    born_a, born_b = (x * pa, pb) if beam == 0 else (pa, x * pb)
    k1b, k2b = pair(born_a + born_b, nhat)
    born = me_born(np.array([k1b, k2b, -born_a, -born_b]))
    k3 = (1 - x) * e * np.array([1, math.sin(delta) * math.cos(phi), math.sin(delta) * math.sin(phi),
                                 sgn * math.cos(delta)])
    k1, k2 = pair(pa + pb - k3, nhat)
    real = me_real(np.array([k1, k2, -pa, -pb, k3]))
    pk = par[0] * k3[0] - par[1:] @ k3[1:]
    return real * pk * x / (split(x) * born)


def p_qq(x):
    return 4 / 3 * (1 + x * x) / (1 - x)


def p_gg(x):
    return 6 * (x / (1 - x) + (1 - x) / x + x * (1 - x))


def test_collinear_limit_formula_on_gg_ttxg():
    """The limit formula with P_gg against the pinned g g -> t tbar g (gluon
    spin correlations average out over the azimuths phi, phi + pi/2)."""
    for x in (0.3, 0.7):
        for delta, tol in ((1e-3, 2e-3), (1e-5, 3e-5)):
            r = [collinear_ratio(0, x, delta, phi, lambda p: O.me2_sum(2, p, M, 0.0),
                                 lambda p: O.me2_sum(3, p, M, 0.0), p_gg) for phi in (0.3, 0.3 + math.pi / 2)]
            assert abs(np.mean(r) - 1) < tol, (x, delta, r)


@pytest.mark.parametrize("beam", [0, 1])
@pytest.mark.parametrize("x", [0.2, 0.55, 0.85])
def test_collinear_limit_qqbar(beam, x):
    errs = []
    for delta in (1e-3, 1e-4, 1e-5):
        r = collinear_ratio(beam, x, delta, 0.4, lambda p: O.me2_qqbar_ttx(p, M),
                            lambda p: O.me2_qqbar_ttxg(p, M, 0.0), p_qq)
        errs.append(abs(r - 1))
    # approach linear in the angle
    assert errs[2] < 1e-4 and errs[1] < 1e-3 and errs[2] < errs[1] < errs[0], errs


def test_lorentz_invariance_and_charge_conjugation():
    rng = np.random.default_rng(21)
    p = ttxg_point(1500.0, rng.random(5))
    ref = O.me2_qqbar_ttxg(p, M, 0.0)
    for _ in range(2):
        assert abs(O.me2_qqbar_ttxg(lorentz(p, rng), M, 0.0) / ref - 1) < 1e-12
    # C: q(pa) qbar(pb) -> t(k1) tbar(k2) g  ==  q(pb) qbar(pa) -> t(k2) tbar(k1) g
    refw = O.me2_qqbar_ttxg(p, M, 1.5)
    assert abs(O.me2_qqbar_ttxg(p[[1, 0, 3, 2, 4]], M, 1.5) / refw - 1) < 1e-13
    # the beams alone exchanged differ (the charge-asymmetric interference)
    assert abs(O.me2_qqbar_ttxg(p[[0, 1, 3, 2, 4]], M, 1.5) / refw - 1) > 1e-3


def test_pp_ttxg_event_weight_assembly():
    """w = J_V W / (2 s_hat) [f_g f_g |M|^2_gg + (u ubar + d dbar) |M|^2_qq
    + (ubar u + dbar d) |M|^2_qq(beams exchanged)] with |M|^2_qq =
    g^6 sum |M|^2 / 36, in pb."""
    t = W.synthetic_pdf(quarks=True)
    proc = O.Process(n_g=3, initial="pp", **CUTS)
    gg = O.Process(n_g=3, **CUTS)
    grid = np.tile(np.arange(51) / 50, (7, 1))
    q2 = 173.0**2
    checked = 0
    for e in range(40):
        w, ev = O.event_weight(proc, 13000.0, t, grid, 5, 0, e)
        wg, _ = O.event_weight(gg, 13000.0, t, grid, 5, 0, e)
        if not ev.pass_cuts:
            assert w == 0.0
            continue
        rs = math.sqrt(ev.shat)
        k = ev.k
        p = np.array([k[0], k[1], [-rs / 2, 0, 0, -rs / 2], [-rs / 2, 0, 0, rs / 2], k[2]])
        mq = GS2**3 * O.me2_qqbar_ttxg(p, M, 1.5) / 36
        mqr = GS2**3 * O.me2_qqbar_ttxg(p[[0, 1, 3, 2, 4]], M, 1.5) / 36
        x1, x2 = ev.x[0], ev.x[1]
        u1, ub1, d1, db1 = (O.pdf_xq(t, f, x1, q2) / x1 for f in range(4))
        u2, ub2, d2, db2 = (O.pdf_xq(t, f, x2, q2) / x2 for f in range(4))
        quark = ev.jac * ev.ps_weight * ((u1 * ub2 + d1 * db2) * mq + (ub1 * u2 + db1 * d2) * mqr) \
            / (2 * ev.shat) * 0.3893793721e9
        assert w == pytest.approx(wg + quark, rel=1e-12, abs=1e-14 * (abs(wg) + abs(quark)))
        checked += 1
    assert checked > 15
    with pytest.raises(ValueError):
        O.Process(n_g=5, initial="pp").c()
