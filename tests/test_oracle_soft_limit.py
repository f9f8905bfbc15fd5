"""Absolute normalisation of the t tbar g and t tbar g g matrix elements.

When a final-state gluon of momentum q becomes soft, the squared amplitude
factorises (eikonal limit):

    sum |M_{n+1}|^2  ->  - g^2 sum_{k,l} (p_k . p_l) / ((p_k . q)(p_l . q))
                             <M_n| T_k . T_l |M_n>,

summed over colours and helicities, with all momenta and colour charges
outgoing (Catani and Seymour, Nucl. Phys. B 485 (1997) 291).  The
colour-correlated Born matrix elements are built here from the oracle's
colour-ordered partial amplitudes and explicit SU(3) colour tensors of the
basis (T^{a_s1} ... T^{a_sn})_{i_t j_tbar}, T = lambda/2.  The g g -> t tbar
matrix element is pinned by its closed form, so this fixes the normalisation
of t tbar g (couplings, colour factors, averaging conventions aside) and, one
step further, of t tbar g g.  Zero width (gauge invariance exact).
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O

M = 173.0

# Gell-Mann matrices / 2 and structure constants
_l = np.zeros((8, 3, 3), dtype=complex)
_l[0][0, 1] = _l[0][1, 0] = 1
_l[1][0, 1], _l[1][1, 0] = -1j, 1j
_l[2][0, 0], _l[2][1, 1] = 1, -1
_l[3][0, 2] = _l[3][2, 0] = 1
_l[4][0, 2], _l[4][2, 0] = -1j, 1j
_l[5][1, 2] = _l[5][2, 1] = 1
_l[6][1, 2], _l[6][2, 1] = -1j, 1j
_l[7][0, 0] = _l[7][1, 1] = 1 / math.sqrt(3)
_l[7][2, 2] = -2 / math.sqrt(3)
T = _l / 2
# f_abc = -2 i Tr([T_a, T_b] T_c)
F = np.real(-2j * (np.einsum("aij,bjk,cki->abc", T, T, T) - np.einsum("bij,ajk,cki->abc", T, T, T)))


def basis(n_g):
    """c_s[a_1 .. a_n, i, j] = (T^{a_s(1)} ... T^{a_s(n)})_{ij} for the oracle's orderings."""
    out = []
    for perm in O.orderings(n_g):
        c = None
        for g in perm:
            shape = [1] * n_g + [3, 3]
            shape[g] = 8
            t = T.reshape(8, 3, 3)
            # broadcast T^{a_g} along axis g
            tg = np.moveaxis(np.broadcast_to(t.reshape([8] + [1] * (n_g - 1) + [3, 3]),
                                             [8] + [1] * (n_g - 1) + [3, 3]), 0, g)
            tg = tg.reshape(shape)
            c = tg if c is None else np.einsum("...ij,...jk->...ik", c, tg)
        out.append(np.broadcast_to(c, [8] * n_g + [3, 3]).copy())
    return out


def charge(c, slot, a, n_g):
    """T^a of parton `slot` (0 = top, 1 = antitop, 2.. = gluons) acting on a
    colour tensor, all partons outgoing."""
    if slot == 0:      # outgoing quark: t^a on the fundamental index
        return np.einsum("ik,...kj->...ij", T[a], c)
    if slot == 1:      # outgoing antiquark: -(t^a)^T on the antifundamental index
        return -np.einsum("...ik,kj->...ij", c, T[a])
    g = slot - 2       # outgoing gluon: (T^a)_{bc} = -i f_{abc}
    m = -1j * F[a]
    return np.moveaxis(np.tensordot(m, np.moveaxis(c, g, 0), axes=(1, 0)), 0, g)


def colour_correlators(n_g):
    """C[k][l][s][t] = <c_s| T_k . T_l |c_t> for the n_g + 2 partons."""
    cs = basis(n_g)
    npart = n_g + 2
    applied = [[[charge(c, k, a, n_g) for a in range(8)] for k in range(npart)] for c in cs]
    ns = len(cs)
    C = np.zeros((npart, npart, ns, ns), dtype=complex)
    for k, l in itertools.product(range(npart), repeat=2):
        for s, t in itertools.product(range(ns), repeat=2):
            C[k, l, s, t] = sum(np.vdot(applied[s][k][a], applied[t][l][a]) for a in range(8))
    return cs, C


@pytest.fixture(scope="module", params=[2, 3])
def born(request, oracle_lib):
    return request.param, colour_correlators(request.param)


def test_colour_tensors_reproduce_the_oracle_colour_matrix(born):
    n_g, (cs, C) = born
    G = np.array([[np.vdot(a, b) for b in cs] for a in cs])
    assert np.allclose(G, O.colour_matrix(n_g), rtol=0, atol=1e-13)


def test_colour_conservation_of_the_basis(born):
    n_g, (cs, C) = born
    for c in cs:
        for a in range(8):
            tot = sum(charge(c, k, a, n_g) for k in range(n_g + 2))
            assert np.abs(tot).max() < 1e-13
    # sum_l T_k . T_l = 0 on colour singlets; T_k^2 = C_F (quarks), C_A (gluons)
    assert np.abs(C.sum(axis=1)).max() < 1e-12
    Cm = O.colour_matrix(n_g)
    for k in range(n_g + 2):
        cas = 4.0 / 3.0 if k < 2 else 3.0
        assert np.allclose(C[k, k], cas * Cm, atol=1e-12)


def lorentz_dot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def hard_and_soft(n_g, E):
    """Born momenta (n_g gluons, all outgoing) and the same configuration with a
    soft gluon of energy E added; three-momentum conserved exactly, the beams
    balance the energy."""
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    q = np.array([110.0, -40.0, 150.0])
    b = np.array([-60.0, 95.0, -30.0]) if n_g == 3 else np.zeros(3)

    def build(shift):
        kt = q - shift * n / 2
        kb = -q - b - shift * n / 2
        fin = [np.array([math.sqrt(M * M + kt @ kt), *kt]), np.array([math.sqrt(M * M + kb @ kb), *kb])]
        extra = []
        if n_g == 3:
            extra.append(np.array([np.linalg.norm(b), *b]))
        if shift > 0:
            extra.append(np.array([shift, *(shift * n)]))
        P0 = sum(v[0] for v in fin + extra)
        beams = [np.array([-P0 / 2, 0, 0, -P0 / 2]), np.array([-P0 / 2, 0, 0, P0 / 2])]
        p = np.array(fin + beams + extra)
        assert np.all(np.abs(p.sum(axis=0)) < 1e-12 * P0)
        return p
    return build(0.0), build(E)


def eikonal_born(n_g, C, p_born, qs):
    """-sum_{k,l} (p_k.p_l)/((p_k.q)(p_l.q)) <M|T_k.T_l|M>, helicity-summed."""
    hels = O.all_helicities(n_g)
    npart = n_g + 2
    G = np.zeros((npart, npart))
    for h in hels:
        A = O.partial_amplitudes(n_g, p_born, M, 0.0, h)
        for k, l in itertools.product(range(npart), repeat=2):
            G[k, l] += np.real(np.conj(A) @ C[k, l] @ A)
    tot = 0.0
    for k, l in itertools.product(range(npart), repeat=2):
        tot += -lorentz_dot(p_born[k], p_born[l]) / (lorentz_dot(p_born[k], qs) * lorentz_dot(p_born[l], qs)) * G[k, l]
    return tot


def test_soft_gluon_limit_fixes_the_normalisation(born):
    """sum |M_{n+1}|^2 / eikonal(Born) -> 1 linearly in the soft energy: from
    t tbar to t tbar g (n_g = 2 Born) and from t tbar g to t tbar g g."""
    n_g, (cs, C) = born
    ratios = []
    for E in (1e-2, 1e-3, 1e-4):
        p_born, p_soft = hard_and_soft(n_g, E)
        qs = p_soft[-1]
        full = O.me2_sum(n_g + 1, p_soft, M, 0.0)
        ratios.append(full / eikonal_born(n_g, C, p_born, qs))
    dev = [abs(r - 1) for r in ratios]
    print(f"\n  n_g = {n_g} -> {n_g + 1}: ratio - 1 = {dev}")
    assert dev[2] < 2e-5
    # approach is linear in E (the next term of the soft expansion)
    assert dev[2] < 0.2 * dev[1] + 1e-9
