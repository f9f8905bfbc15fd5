"""The colour tables that the kernel generators write, against the oracle
(host-side, no GPU): the generators compute their colour matrices by their
own SU(3) sums, the oracle by its own, and the kernels use only the
generated tables.

* q qbar -> t tbar g g (Sec. 3, Table 1; 36 diagrams as 38 terms): with
  K the oracle's 38 x 38 colour matrix and phi the terms' class phases (1, i,
  -1) that the kernel leaves out of its Lorentz parts, phi K phi^dagger is
  real; the kernel's basis of 11 terms (signed sums B, integer Gram matrix
  G over 36) gives B^T G B / 36 = phi K phi^dagger, and the real rank-11
  projection W of gen_qqbar.py gives W^T W = phi K phi^dagger.
* g g -> t tbar g g g (Sec. 3.2, Fig. 4): the 120 x 120 matrix of
  gen_ttggg.py (integers over a common denominator) equals the oracle's.
"""
import importlib.util
import os

import numpy as np
import pytest

import oracle as O

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_2106_10279_amd", "csrc")


def load(name):
    spec = importlib.util.spec_from_file_location(name, os.path.join(CSRC, name + ".py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def gen():
    return load("gen_amplitudes")


def test_qqbar_ttxgg_projection_against_the_oracle_colour_matrix(gen):
    Q = load("gen_qqbar")
    W, K = Q.projection(gen._helpers())
    assert W.shape == (11, 38) and np.isrealobj(W)
    Ko = O.qqbar_ttxgg_colour_matrix()
    ph = np.array(Q.PHASES, dtype=complex)
    Kp = ph[:, None] * Ko * ph.conj()[None, :]
    assert np.abs(Kp.imag).max() < 1e-12                 # real with the phases
    assert np.abs(W.T @ W - Kp.real).max() < 1e-12 * np.abs(Kp).max()
    assert np.abs(K - Kp.real).max() < 1e-12 * np.abs(Kp).max()
    # the colour sum of random Lorentz parts through the projection
    rng = np.random.default_rng(7)
    for _ in range(3):
        a = rng.normal(size=38) + 1j * rng.normal(size=38)
        direct = np.real(a @ Kp @ a.conj())
        proj = np.sum(np.abs(W @ a) ** 2)
        assert abs(proj / direct - 1) < 1e-12
    # a wrong phase on one class changes the sum: the phases matter
    bad = ph.copy()
    bad[20:28] = 1
    Kb = bad[:, None] * Ko * bad.conj()[None, :]
    assert np.abs(Kb.imag).max() > 1.0


def test_qqbar_ttxgg_sparse_basis_against_the_oracle(gen):
    """The basis the kernel uses: 11 of the terms themselves, every term's
    colour factor (with its class phase) a signed sum of theirs (B entries
    -1, 0, 1) and their Gram matrix over 36 integer: B^T G B / 36 must
    reproduce the oracle's phased colour matrix entry by entry."""
    Q = load("gen_qqbar")
    basis, B, Gi, den, K = Q.sparse_basis(gen._helpers())
    assert len(basis) == 11 and basis == sorted(basis)
    assert set(np.unique(B)) <= {-1, 0, 1}
    assert np.array_equal(B[:, basis], np.eye(11, dtype=int))
    assert np.array_equal(Gi, Gi.T) and np.all(np.linalg.eigvalsh(Gi) > 0)
    Ko = O.qqbar_ttxgg_colour_matrix()
    ph = np.array(Q.PHASES, dtype=complex)
    Kp = (ph[:, None] * Ko * ph.conj()[None, :]).real
    assert np.abs(B.T @ Gi @ B / den - Kp).max() < 1e-12 * np.abs(Kp).max()
    # the colour sum of random Lorentz parts in the basis
    rng = np.random.default_rng(8)
    for _ in range(3):
        a = rng.normal(size=38) + 1j * rng.normal(size=38)
        b = B @ a
        assert abs(np.real(b @ Gi @ b.conj()) / den / np.real(a @ Kp @ a.conj()) - 1) < 1e-12


def test_ttxggg_colour_matrix_against_the_oracle(gen):
    """The generator's integer matrix over its common denominator (from the
    Fierz contraction of one row and relabellings) against the oracle's
    brute-force sum over the 9 x 8^5 colour assignments."""
    T5 = load("gen_ttggg")
    perms, K, den = T5.colour_matrix_ng5(gen._helpers())
    assert len(perms) == 120 and perms == sorted(perms)
    Ko = O.colour_matrix(5)
    Kf = np.asarray(K, dtype=float) / den
    assert np.abs(Kf - Ko).max() < 1e-12 * np.abs(Ko).max()
    assert np.array_equal(np.asarray(K), np.asarray(K).T)
