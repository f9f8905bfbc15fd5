"""Pins for the colour matrices: an exact rational evaluation by the SU(N)
Fierz identities, independent of the oracle's explicit Gell-Mann sums."""
from fractions import Fraction
from functools import lru_cache
from itertools import permutations

import numpy as np
import pytest

import oracle as O

NC = Fraction(3)


def _eval(traces):
    """Sum over repeated adjoint indices of a product of traces of generators
    (T = lambda/2), using
        Tr(A T^a B T^a)    = 1/2 [Tr(A) Tr(B) - Tr(AB)/N]
        Tr(A T^a) Tr(B T^a) = 1/2 [Tr(AB) - Tr(A) Tr(B)/N]."""
    traces = [tuple(t) for t in traces]
    for ti, t in enumerate(traces):
        if t:
            a = t[0]
            break
    else:
        return NC ** len(traces)
    loc = [(i, j) for i, t in enumerate(traces) for j, v in enumerate(t) if v == a]
    (i1, j1), (i2, j2) = loc
    rest = [t for k, t in enumerate(traces) if k not in (i1, i2)]
    if i1 == i2:
        t = traces[i1]
        A = t[j1 + 1:j2]
        B = t[j2 + 1:] + t[:j1]
        return Fraction(1, 2) * (_eval(rest + [A, B]) - _eval(rest + [A + B]) / NC)
    t1, t2 = traces[i1], traces[i2]
    A = t1[j1 + 1:] + t1[:j1]
    B = t2[j2 + 1:] + t2[:j2]
    return Fraction(1, 2) * (_eval(rest + [A + B]) - _eval(rest + [A, B]) / NC)


def exact_colour_matrix(n):
    perms = sorted(permutations(range(n)))
    out = []
    for s in perms:
        row = []
        for t in perms:
            # Tr((T^s)^dagger T^t) = Tr(T^{s_n} .. T^{s_1} T^{t_1} .. T^{t_n})
            row.append(_eval([tuple(reversed(s)) + tuple(t)]))
        out.append(row)
    return out


@pytest.mark.parametrize("n", [2, 3, 4])
def test_colour_matrix_exact(n):
    exact = exact_colour_matrix(n)
    C = O.colour_matrix(n)
    for i, row in enumerate(exact):
        for j, v in enumerate(row):
            assert C[i, j] == float(v)          # exact rational rounded once


def test_colour_matrix_known_values():
    C2 = O.colour_matrix(2) * 3
    assert set(np.unique(C2)) == {16.0, -2.0}
    C3 = O.colour_matrix(3) * 9
    assert set(np.unique(C3)) == {64.0, -8.0, 1.0, 10.0}
    assert np.all(C3.sum(1) == 60)
    C4 = O.colour_matrix(4) * 54
    assert set(np.unique(C4)) == {512, 80, 71, 62, 8, -1, -10, -28, -64}
    assert np.all(C4.sum(1) == 705)
    for n in (2, 3, 4):
        C = O.colour_matrix(n)
        assert np.allclose(np.diag(C), 3 * (4 / 3) ** n, rtol=0, atol=1e-14)
        assert np.array_equal(C, C.T)
    eig = [np.linalg.eigvalsh(O.colour_matrix(n)).min() for n in (2, 3, 4)]
    assert abs(eig[0] - 14 / 3) < 1e-12 and abs(eig[1] - 5) < 1e-12 and abs(eig[2] - 3.8962) < 1e-4


def test_orderings_are_lexicographic():
    for n in (2, 3, 4):
        assert [tuple(r) for r in O.orderings(n)] == sorted(permutations(range(n)))
