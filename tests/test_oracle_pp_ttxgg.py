"""Pins for the oracle's q qbar -> t tbar g g (the q qbar channel of the
paper's p p -> t tbar g g, Sec. 3, Table 1: 36 diagrams per quark group,
267 with the 123 of g g) and the p p -> t tbar g g event weight.

* Colour: the colour-factor products of the 38 terms (the 36 diagrams, the
  four-gluon vertex in its three colour structures) summed over all 5184
  colour assignments, against closed forms from SU(3) trace identities.
* Gauge invariance: either gluon's polarisation replaced by its momentum
  gives a vanishing amplitude for every sampled colour assignment and every
  helicity configuration (zero width); flipping the sign of one class of
  diagrams breaks it.
* The initial-state collinear limits, a gluon along either beam, onto the
  pinned q qbar -> t tbar g with C_F (1 + x^2)/(1 - x).
* Bose symmetry of the two gluons, charge conjugation, Lorentz invariance.
* The p p -> t tbar g g weight: its assembly from the tables, both beam
  orientations, g^8 and the 1/2! of the identical gluons.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_oracle_me import lorentz
from test_oracle_pp_ttxg import pair, p_qq

M = 173.0
AS = 0.118
GS2 = 4 * math.pi * AS
CUTS = dict(ptmin_g=20.0, drmin_gg=0.4)


def ttxgg_point(rs, r):
    k, w, st = O.phase_space(4, [M, M, 0.0, 0.0], rs, r)
    e = rs / 2
    return np.array([k[0], k[1], [-e, 0, 0, -e], [-e, 0, 0, e], k[2], k[3]])


@pytest.fixture(scope="module")
def colour_sample():
    rng = np.random.default_rng(17)
    cols = list(itertools.product(range(3), range(3), range(3), range(3), range(8), range(8)))
    sel = [cols[i] for i in rng.choice(len(cols), 400, replace=False)]
    return np.array([O.qqbar_ttxgg_colour(c) for c in sel])


def test_colour_matrix_against_trace_identities():
    """K_dd' = sum over colours of C_d C_d'^*.  Terms 0-5 are the orders of
    class 1 ((T^c ...)_{ji} (T^c)_{kl} with both gluons on the quark line):
    each diagonal entry is C_F^2 sum_cc' Tr(T^c T^c')^2 = 2 C_F^2 = 32/9, as
    for classes 2 and 3.  The order (g1, g2, spine) against (g2, g1, spine)
    gives C_F (C_F - C_A/2) 2 = -4/9.  The third four-gluon term,
    f^{c_q c_t e} f^{a1 a2 e}, gives C_A^2 (N^2 - 1)/4 = 18."""
    K = O.qqbar_ttxgg_colour_matrix()
    assert np.allclose(K, K.conj().T, atol=1e-13)
    w = np.linalg.eigvalsh(K)
    assert w.min() > -1e-12                        # a Gram matrix
    for d in range(20):                            # classes 1, 2, 3
        assert abs(K[d, d] - 32 / 9) < 1e-13, d
    # class 1 order 0 = (g1, g2, spine), order 2 = (g2, g1, spine) from the u end
    assert abs(K[0, 2] - (-4 / 9)) < 1e-13
    assert abs(K[32, 32] - 18.0) < 1e-12         # term 32: f^{c_q c_t e} f^{a1 a2 e}
    assert np.linalg.matrix_rank(K, tol=1e-9) < 38


@pytest.mark.parametrize("rs,seed", [(1200.0, 3), (3000.0, 4), (600.0, 5)])
def test_ward_identity_both_gluons(colour_sample, rs, seed):
    p = ttxgg_point(rs, np.random.default_rng(seed).random(8))
    hels = [[(h >> b) & 1 for b in range(6)] for h in range(64)]
    for g in (1, 2):
        ward = [O.qqbar_ttxgg_terms(p, M, 0.0, hel, ward=g) for hel in hels]
        scale = max(np.abs(colour_sample * a).sum(axis=1).max() for a in ward)
        assert scale > 0.0
        for h, a in enumerate(ward):
            assert np.abs(colour_sample @ a).max() <= 1e-14 * scale, (g, h)
    # teeth: the two-vertex spine diagrams (terms 28, 29) with the wrong sign
    a = O.qqbar_ttxgg_terms(p, M, 0.0, [1, 0, 0, 0, 0, 0], ward=1)
    a[28:30] = -a[28:30]
    assert np.abs(colour_sample @ a).max() > 1e-6 * np.abs(colour_sample * a).sum(axis=1).max()


@pytest.mark.parametrize("beam", [0, 1])
@pytest.mark.parametrize("x", [0.3, 0.7])
def test_collinear_limit_onto_ttxg(beam, x):
    """Gluon 1 along the quark (beam 0) or antiquark (beam 1) direction;
    gluon 2 and the t tbar direction fixed."""
    e = 700.0
    pa, pb = np.array([e, 0, 0, e]), np.array([e, 0, 0, -e])
    nhat = np.array([math.sin(1.1) * math.cos(0.7), math.sin(1.1) * math.sin(0.7), math.cos(1.1)])
    k4 = 150.0 * np.array([1, math.sin(1.3) * math.cos(2.0), math.sin(1.3) * math.sin(2.0), math.cos(1.3)])
    par = pa if beam == 0 else pb
    sgn = 1.0 if beam == 0 else -1.0
    ba, bb = (x * pa, pb) if beam == 0 else (pa, x * pb)
    k1b, k2b = pair(ba + bb - k4, nhat)
    born = O.me2_qqbar_ttxg(np.array([k1b, k2b, -ba, -bb, k4]), M, 0.0)
    errs = []
    for d in (1e-3, 1e-4, 1e-5):
        k3 = (1 - x) * e * np.array([1, math.sin(d) * math.cos(0.4), math.sin(d) * math.sin(0.4), sgn * math.cos(d)])
        k1, k2 = pair(pa + pb - k3 - k4, nhat)
        real = O.me2_qqbar_ttxgg(np.array([k1, k2, -pa, -pb, k3, k4]), M, 0.0)
        pk = par[0] * k3[0] - par[1:] @ k3[1:]
        errs.append(abs(real * pk * x / (p_qq(x) * born) - 1))
    assert errs[2] < 1e-5 and errs[1] < 1e-4 and errs[2] < errs[1] < errs[0], errs


def test_symmetries():
    rng = np.random.default_rng(23)
    p = ttxgg_point(1500.0, rng.random(8))
    ref = O.me2_qqbar_ttxgg(p, M, 0.0)
    assert abs(O.me2_qqbar_ttxgg(p[[0, 1, 2, 3, 5, 4]], M, 0.0) / ref - 1) < 1e-13      # Bose
    for _ in range(2):
        assert abs(O.me2_qqbar_ttxgg(lorentz(p, rng), M, 0.0) / ref - 1) < 1e-12
    refw = O.me2_qqbar_ttxgg(p, M, 1.5)
    assert abs(O.me2_qqbar_ttxgg(p[[1, 0, 3, 2, 4, 5]], M, 1.5) / refw - 1) < 1e-13     # C
    assert abs(O.me2_qqbar_ttxgg(p[[0, 1, 3, 2, 4, 5]], M, 1.5) / refw - 1) > 1e-4


def test_pp_ttxgg_event_weight_assembly():
    t = W.synthetic_pdf(quarks=True)
    proc = O.Process(n_g=4, initial="pp", **CUTS)
    gg = O.Process(n_g=4, **CUTS)
    grid = np.tile(np.arange(51) / 50, (10, 1))
    q2 = 173.0**2
    checked = 0
    for e in range(30):
        w, ev = O.event_weight(proc, 13000.0, t, grid, 5, 0, e)
        wg, _ = O.event_weight(gg, 13000.0, t, grid, 5, 0, e)
        if not ev.pass_cuts:
            assert w == 0.0
            continue
        rs = math.sqrt(ev.shat)
        k = ev.k
        p = np.array([k[0], k[1], [-rs / 2, 0, 0, -rs / 2], [-rs / 2, 0, 0, rs / 2], k[2], k[3]])
        mq = GS2**4 * O.me2_qqbar_ttxgg(p, M, 1.5) / 72
        mqr = GS2**4 * O.me2_qqbar_ttxgg(p[[0, 1, 3, 2, 4, 5]], M, 1.5) / 72
        x1, x2 = ev.x[0], ev.x[1]
        u1, ub1, d1, db1 = (O.pdf_xq(t, f, x1, q2) / x1 for f in range(4))
        u2, ub2, d2, db2 = (O.pdf_xq(t, f, x2, q2) / x2 for f in range(4))
        quark = ev.jac * ev.ps_weight * ((u1 * ub2 + d1 * db2) * mq + (ub1 * u2 + db1 * d2) * mqr) \
            / (2 * ev.shat) * 0.3893793721e9
        assert w == pytest.approx(wg + quark, rel=1e-12, abs=1e-14 * (abs(wg) + abs(quark)))
        checked += 1
    assert checked > 10
