"""Pins for the oracle's leading-colour approximation of |M|^2.

The paper (Sec. 3.2, on Fig. 4) names the leading-colour approximation as a way to
cheapen high-multiplicity matrix elements without defining it further.  The
reading taken here: in the basis (T^{a_s1} ... T^{a_sn})_{i_t j_tbar} with
T = lambda/2 the colour matrix C is replaced by c_LC times the identity,

    c_LC = (N^2 - 1) N^(n - 1) / 2^n,     N = 3,

the leading power of N in each diagonal element N C_F^n (Mangano and Parke,
Phys. Rept. 200 (1991) 301).  The approximation is then fixed by the
helicity sums of the squared colour-ordered amplitudes, sum_h |A(sigma)|^2,
which are pinned here ordering by ordering: by a closed form for g g -> t
tbar, by their colour-ordered soft limit from one multiplicity to the next
(each ordering separately, so the t tbar g and t tbar g g orderings are tied
to the closed form), by Lorentz invariance and by Bose symmetry.
"""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_me import M, lorentz, random_momenta, ttx_momenta
from test_oracle_soft_limit import hard_and_soft, lorentz_dot


def ordered_squares(n_g, p, width=0.0):
    """sum over helicities of |A(sigma)|^2 for every ordering sigma, g_s = 1."""
    S = np.zeros(math.factorial(n_g))
    for h in O.all_helicities(n_g):
        S += np.abs(O.partial_amplitudes(n_g, p, M, width, h)) ** 2
    return S


def test_lc_coefficient_is_the_leading_power_of_the_colour_diagonal():
    """N C_F^n = c_LC (1 - 1/N^2)^(n - 1): the brute-force SU(3) colour
    matrix's diagonal and c_LC agree in their leading power of N."""
    N = 3.0
    for n_g, expect in ((2, 6.0), (3, 9.0), (4, 13.5), (5, 20.25)):
        assert O.colour_lc(n_g) == expect
        diag = np.diag(O.colour_matrix(n_g))
        assert np.allclose(diag, expect * (1 - 1 / N**2) ** (n_g - 1), rtol=1e-14, atol=0)


@pytest.mark.parametrize("rs,c", [(500.0, 0.3), (400.0, -0.9), (2000.0, 0.99), (13000.0, -0.5)])
def test_ttx_colour_ordered_squares_closed_form(rs, c):
    """g g -> t tbar at zero width, with F = tau1^2 + tau2^2 + rho - rho^2/(4 tau1 tau2),
    tau1 = p_a.k_t / p_a.p_b = (1 - beta cos theta)/2 and tau2 = 1 - tau1:
        sum_h |A(t; a, b; tbar)|^2 = 8 F tau2 / tau1,
        sum_h |A(t; b, a; tbar)|^2 = 8 F tau1 / tau2,
        sum_h Re A(t; a, b; tbar) conj(A(t; b, a; tbar)) = 8 F.
    With the 2 x 2 colour matrix (16, -2; -2, 16)/3 these give the closed
    form of Glueck-Owens-Reya / Ellis-Stirling-Webber, (1/(6 tau1 tau2) - 3/8) F
    after the 1/256 average; the leading-colour value is (3/16) F (1/(tau1 tau2) - 2)."""
    p = ttx_momenta(rs, c, phi=0.4)
    shat = rs * rs
    rho = 4 * M * M / shat
    b = math.sqrt(1 - rho)
    t1, t2 = (1 - b * c) / 2, (1 + b * c) / 2
    F = t1 * t1 + t2 * t2 + rho - rho * rho / (4 * t1 * t2)
    assert [tuple(s) for s in O.orderings(2)] == [(0, 1), (1, 0)]
    S = ordered_squares(2, p)
    X = sum((A[0] * np.conj(A[1])).real
            for A in (O.partial_amplitudes(2, p, M, 0.0, h) for h in O.all_helicities(2)))
    assert S[0] == pytest.approx(8 * F * t2 / t1, rel=1e-13)
    assert S[1] == pytest.approx(8 * F * t1 / t2, rel=1e-13)
    assert X == pytest.approx(8 * F, rel=1e-12)
    # the closed forms are those of the full-colour result ...
    full = (16 / 3 * (S[0] + S[1]) - 4 / 3 * X) / 256
    assert full == pytest.approx((1 / (6 * t1 * t2) - 3 / 8) * F, rel=1e-12)
    # ... and the leading-colour sum follows from them
    lc = O.me2_sum_lc(2, p, M, 0.0) / 256
    assert lc == pytest.approx(3 / 16 * F * (1 / (t1 * t2) - 2), rel=1e-13)


@pytest.mark.parametrize("n_g", [2, 3])
def test_colour_ordered_soft_limit_per_ordering(n_g):
    """A soft gluon q between neighbours a and b of an ordering factorises:
    sum_h |A_{n+1}(..., a, q, b, ...)|^2 -> E_ab sum_h |A_n(..., a, b, ...)|^2 with
    E_ab = 2 p_a.p_b / (p_a.q p_b.q) - m_a^2 / (p_a.q)^2 - m_b^2 / (p_b.q)^2
    (minus the square of the colour-ordered eikonal current, summed over the
    soft gluon's polarisations).  Checked for every ordering of t tbar g and
    t tbar g g: the ratio tends to 1 linearly in the soft energy."""
    perms_n = [tuple(s) for s in O.orderings(n_g)]
    worst = []
    for E in (1e-2, 1e-3, 1e-4):
        p_born, p_soft = hard_and_soft(n_g, E)
        q = p_soft[-1]
        Sn, Sn1 = ordered_squares(n_g, p_born), ordered_squares(n_g + 1, p_soft)
        dev = 0.0
        for k, sg in enumerate(O.orderings(n_g + 1)):
            sg = list(sg)
            chain = [-1] + sg + [-2]              # -1 = top, -2 = antitop
            i = chain.index(n_g)                  # the soft gluon carries the last label
            slot = {-1: 0, -2: 1}
            pa = p_born[slot.get(chain[i - 1], 2 + chain[i - 1])]
            pb = p_born[slot.get(chain[i + 1], 2 + chain[i + 1])]
            Eab = (2 * lorentz_dot(pa, pb) / (lorentz_dot(pa, q) * lorentz_dot(pb, q))
                   - lorentz_dot(pa, pa) / lorentz_dot(pa, q) ** 2
                   - lorentz_dot(pb, pb) / lorentz_dot(pb, q) ** 2)
            red = tuple(g for g in sg if g != n_g)
            dev = max(dev, abs(Sn1[k] / (Eab * Sn[perms_n.index(red)]) - 1))
        worst.append(dev)
    print(f"\n  n_g = {n_g} -> {n_g + 1}: max |ratio - 1| over orderings {worst}")
    assert worst[2] < 1e-5
    assert worst[2] < 0.2 * worst[1] + 1e-9


@pytest.mark.parametrize("n_g", [3, 4])
def test_ordered_squares_lorentz_invariant(n_g):
    """Each partial amplitude is gauge invariant, so its helicity sum is
    Lorentz invariant at zero width, ordering by ordering."""
    rng = np.random.default_rng(300 + n_g)
    p = random_momenta(n_g, 1200.0, rng)
    ref = ordered_squares(n_g, p)
    # the oracle's leading-colour sum is c_LC times these pinned squares
    assert O.me2_sum_lc(n_g, p, M, 0.0) == pytest.approx(O.colour_lc(n_g) * ref.sum(), rel=1e-13)
    q = lorentz(p, rng)
    assert np.allclose(ordered_squares(n_g, q), ref, rtol=1e-11, atol=0)
    assert O.me2_sum_lc(n_g, q, M, 0.0) == pytest.approx(O.me2_sum_lc(n_g, p, M, 0.0), rel=1e-11)


def test_lc_ttgg_bose_symmetric_in_the_final_gluons():
    rng = np.random.default_rng(311)
    p = random_momenta(4, 1500.0, rng)
    q = p.copy()
    q[[4, 5]] = p[[5, 4]]
    assert O.me2_sum_lc(4, q, M, 1.5) == pytest.approx(O.me2_sum_lc(4, p, M, 1.5), rel=1e-12)


def test_lc_event_weight_differs_from_full_only_by_the_colour_sum(pdf_table):
    """The per-event weight with colour = "leading" is the full-colour weight
    with the colour sum replaced: the ratio of the two weights is the ratio of
    the two helicity sums at the event's momenta."""
    grid = np.tile(np.arange(51) / 50, (10, 1))
    full = O.Process(n_g=4, ptmin_g=20.0, drmin_gg=0.4)
    lead = O.Process(n_g=4, ptmin_g=20.0, drmin_gg=0.4, colour="leading")
    checked = 0
    for e in range(40):
        wf, ev = O.event_weight(full, 13000.0, pdf_table, grid, 0, 0, e)
        wl, _ = O.event_weight(lead, 13000.0, pdf_table, grid, 0, 0, e)
        if wf == 0.0:
            assert wl == 0.0
            continue
        k = np.asarray(ev.k)
        e_b = math.sqrt(ev.shat) / 2
        p = np.array([k[0], k[1], [-e_b, 0, 0, -e_b], [-e_b, 0, 0, e_b], k[2], k[3]])
        ratio = O.me2_sum_lc(4, p, M, 1.5) / O.me2_sum(4, p, M, 1.5)
        assert wl / wf == pytest.approx(ratio, rel=1e-12)
        checked += 1
    assert checked > 20
    with pytest.raises(ValueError):
        O.Process(n_g=4, colour="subleading").c()
