"""Pins for the oracle's g g -> t tbar g g g: five gluons, 120 colour
orderings, 128 helicity configurations (the largest process of Sec. 4.2,
Fig. 4, there summed with its quark channels).

* The 120 x 120 colour matrix: every entry against the exact rational value of
  the SU(3) trace from the Fierz identities; the relabelling construction the
  oracle uses at five gluons against the full brute-force sum at two to four.
* The colour decomposition per colour assignment: the amplitude from
  colour-dressed Feynman rules (unordered currents, f^abc vertices, explicit
  SU(3) indices) equals sum_sigma (T^a_sigma1 .. T^a_sigma5)_ij A_sigma of the
  colour-ordered recursion, for random adjoint indices and helicities.
* Gauge invariance (Ward identity per partial amplitude), Lorentz invariance,
  Bose symmetry over the five gluons, C symmetry.
* The soft limit t tbar g g g -> eikonal factor x colour-correlated t tbar g g
  (Catani-Seymour), which fixes the normalisation from the pinned t tbar g g.
* The event weight: three-gluon cuts, the 1/3! symmetry factor, g^10.
"""
import itertools
import math
from itertools import permutations

import numpy as np
import pytest

import oracle as O
from test_oracle_colour import _eval
from test_oracle_me import M, lorentz, random_momenta
from test_oracle_soft_limit import T as GM_T
from test_oracle_soft_limit import basis, charge, lorentz_dot

N5 = 5


def test_colour_matrix_five_gluons_exact():
    C = O.colour_matrix(N5)
    perms = sorted(permutations(range(N5)))
    assert [tuple(r) for r in O.orderings(N5)] == perms
    for i, s in enumerate(perms):
        for j, t in enumerate(perms):
            # Tr((T^s)^dagger T^t) = Tr(T^{s_5} .. T^{s_1} T^{t_1} .. T^{t_5})
            assert C[i, j] == float(_eval([tuple(reversed(s)) + tuple(t)]))


def test_colour_matrix_five_gluons_structure():
    C = O.colour_matrix(N5)
    assert np.array_equal(C, C.T)
    assert np.all(np.diag(C) == 98304 / 7776)              # 3 (4/3)^5
    K = np.round(C * 324)
    assert np.all(np.abs(C * 324 - K) < 1e-9)               # integers over 324
    assert np.all(K.sum(axis=1) == 9300)                    # relabelling symmetry: equal row sums
    assert np.linalg.eigvalsh(C).min() > 1.9                # positive definite


@pytest.mark.parametrize("n", [2, 3, 4])
def test_relabelling_construction_equals_the_brute_force_sum(n):
    assert np.array_equal(O.colour_matrix_relabel(n), O.colour_matrix(n))


def decomposed(n, p, hel, cols, width=1.5):
    A = O.partial_amplitudes(n, p, M, width, hel)
    out = np.zeros((3, 3), dtype=complex)
    for s, perm in enumerate(O.orderings(n)):
        P = np.eye(3, dtype=complex)
        for g in perm:
            P = P @ GM_T[cols[g]]
        out += A[s] * P
    return out


@pytest.mark.parametrize("n", [3, 5])
def test_colour_dressed_feynman_rules_per_assignment(n):
    """Each colour assignment separately: a wrong f^abc sign, a missing
    four-gluon term or a transposed generator product changes single
    assignments even where a sum over all of them might hide it."""
    rng = np.random.default_rng(500 + n)
    checked = 0
    for trial in range(4):
        p = random_momenta(n, 1000.0 + 400.0 * trial, rng)
        for _ in range(25):
            hel = rng.integers(0, 2, n + 2)
            cols = rng.integers(0, 8, n)
            got = O.dressed_amplitude(n, p, M, 1.5, hel, cols)
            ref = decomposed(n, p, hel, cols)
            scale = np.abs(ref).max()
            if scale == 0.0:
                assert np.abs(got).max() == 0.0
                continue
            assert np.abs(got - ref).max() < 1e-12 * scale
            checked += 1
    assert checked > 60


@pytest.mark.parametrize("width", [0.0, 1.5])
def test_sum_over_assignments_of_one_configuration(width):
    """For one helicity configuration of t tbar g g the explicit sum over all
    8^4 assignments and 3 x 3 colours equals A^dagger C A; the same identity
    at five gluons is what the per-assignment test and the exact colour matrix
    together state."""
    rng = np.random.default_rng(77)
    p = random_momenta(4, 1300.0, rng)
    h = O.all_helicities(4)[[5, 50]]
    a = O.me2_sum_hel(4, p, M, width, h)
    b = O.me2_sum_fullcolour(4, p, M, width, h)
    assert abs(a / b - 1) < 1e-12


def test_ward_identity_five_gluons():
    rng = np.random.default_rng(65)
    for _ in range(3):
        p = random_momenta(N5, 1500.0, rng)
        hel = rng.integers(0, 2, N5 + 2)
        ref = np.abs(O.partial_amplitudes(N5, p, M, 0.0, hel)).max()
        for g in range(N5):
            A = O.partial_amplitudes(N5, p, M, 0.0, hel, ward_gluon=g)
            assert np.abs(A).max() < 1e-11 * ref * max(abs(p[2 + g][0]), 1.0)


def test_lorentz_invariance_five_gluons():
    rng = np.random.default_rng(85)
    p = random_momenta(N5, 1600.0, rng)
    ref = O.me2_sum(N5, p, M, 0.0)
    for _ in range(2):
        assert abs(O.me2_sum(N5, lorentz(p, rng), M, 0.0) / ref - 1) < 1e-11


def test_bose_and_charge_conjugation_symmetry_five_gluons():
    rng = np.random.default_rng(9)
    p = random_momenta(N5, 1400.0, rng)
    ref = O.me2_sum(N5, p, M, 1.5)
    for fin in permutations([4, 5, 6]):
        q = p[[0, 1, 2, 3, *fin]]
        assert abs(O.me2_sum(N5, q, M, 1.5) / ref - 1) < 1e-12
    # an initial gluon exchanged with a final one (crossing-symmetric amplitude)
    q = p[[0, 1, 5, 3, 4, 2, 6]]
    assert abs(O.me2_sum(N5, q, M, 1.5) / ref - 1) < 1e-12
    q = p[[1, 0, 2, 3, 4, 5, 6]]
    assert abs(O.me2_sum(N5, q, M, 1.5) / ref - 1) < 1e-11


def born_correlators(p_born, n_g=4):
    """G[k][l] = sum over helicities and a of <T_k^a M|T_l^a M> for the Born
    with explicit colour tensors M = sum_s A_s (T^a_s1 .. T^a_sn)_ij."""
    cs = np.array(basis(n_g))                           # [n!][8]*n[3][3]
    npart = n_g + 2
    G = np.zeros((npart, npart))
    for h in O.all_helicities(n_g):
        A = O.partial_amplitudes(n_g, p_born, M, 0.0, h)
        Mt = np.tensordot(A, cs, axes=(0, 0))
        X = np.array([[charge(Mt, k, a, n_g).ravel() for a in range(8)] for k in range(npart)])
        X = X.reshape(npart, -1)
        G += np.real(np.conj(X) @ X.T)
    return G


def soft_configuration(E):
    """t tbar + two hard gluons (Born) and the same with a soft gluon of
    energy E along n; three-momentum conserved exactly, beams balance the
    energy."""
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    q = np.array([110.0, -40.0, 150.0])
    b1 = np.array([-60.0, 95.0, -30.0])
    b2 = np.array([45.0, 20.0, -120.0])

    def build(shift):
        kt = q - shift * n / 2
        kb = -q - b1 - b2 - shift * n / 2
        fin = [np.array([math.sqrt(M * M + kt @ kt), *kt]), np.array([math.sqrt(M * M + kb @ kb), *kb])]
        extra = [np.array([np.linalg.norm(b), *b]) for b in (b1, b2)]
        if shift > 0:
            extra.append(np.array([shift, *(shift * n)]))
        P0 = sum(v[0] for v in fin + extra)
        beams = [np.array([-P0 / 2, 0, 0, -P0 / 2]), np.array([-P0 / 2, 0, 0, P0 / 2])]
        p = np.array(fin + beams + extra)
        assert np.all(np.abs(p.sum(axis=0)) < 1e-12 * P0)
        return p
    return build(0.0), build(E)


def test_soft_gluon_limit_from_ttgg():
    """sum |M(t tbar g g g)|^2 / [-sum_kl (p_k.p_l)/((p_k.q)(p_l.q)) <T_k.T_l>_Born]
    -> 1, linearly in the soft energy."""
    p_born, _ = soft_configuration(1.0)
    G = born_correlators(p_born)
    # colour conservation of the correlators: sum_l T_k.T_l = 0
    assert np.abs(G.sum(axis=1)).max() < 1e-10 * np.abs(G).max()
    dev = []
    for E in (1e-2, 1e-3, 1e-4):
        _, p_soft = soft_configuration(E)
        qs = p_soft[-1]
        eik = sum(-lorentz_dot(p_born[k], p_born[l]) / (lorentz_dot(p_born[k], qs) * lorentz_dot(p_born[l], qs))
                  * G[k, l] for k, l in itertools.product(range(6), repeat=2))
        dev.append(abs(O.me2_sum(N5, p_soft, M, 0.0) / eik - 1))
    print(f"\n  t tbar g g -> t tbar g g g: ratio - 1 = {dev}")
    assert dev[2] < 2e-5
    assert dev[2] < 0.2 * dev[1] + 1e-9


def test_event_weight_five_gluons(pdf_table):
    """w = J_V W f1 f2 g^10 sum|M|^2 / (4 * 64 * 3!) / (2 s_hat) in pb, with the
    gluon cuts of the event's momenta; 13 integration dimensions."""
    proc = O.Process(n_g=N5, ptmin_g=20.0, drmin_gg=0.4)
    assert O.n_dims(N5) == 13
    grid = np.tile(np.arange(51) / 50, (13, 1))
    gs2 = 4 * math.pi * proc.alpha_s
    n_pass = n_cut = 0
    for e in range(120):
        w, ev = O.event_weight(proc, 13000.0, pdf_table, grid, 3, 0, e)
        if not ev.pass_threshold:
            assert w == 0.0
            continue
        k = ev.k
        assert k.shape == (5, 4)
        rs = math.sqrt(ev.shat)
        assert np.all(np.abs(k.sum(axis=0) - [rs, 0, 0, 0]) < 1e-10 * rs)
        ok, _ = O.cuts(proc, k, 0.5 * math.log(ev.x[0] / ev.x[1]))
        assert ok == ev.pass_cuts
        if not ok:
            assert w == 0.0
            n_cut += 1
            continue
        p = np.array([k[0], k[1], [-rs / 2, 0, 0, -rs / 2], [-rs / 2, 0, 0, rs / 2], k[2], k[3], k[4]])
        me2 = gs2**5 * O.me2_sum(N5, p, M, proc.w_top) / (4 * 64 * 6)
        ref = ev.jac * ev.ps_weight * ev.f1 * ev.f2 * me2 / (2 * ev.shat) * 0.3893793721e9
        assert w == pytest.approx(ref, rel=1e-13)
        n_pass += 1
    assert n_pass > 5 and n_cut > 5, (n_pass, n_cut)
