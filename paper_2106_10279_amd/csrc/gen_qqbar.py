"""Colour tables of q qbar -> t tbar g g (the q qbar channel of p p -> t tbar
g g, Sec. 3, Table 1: 36 Feynman diagrams per quark group), written by
gen_amplitudes.py into _gen/qqbar_ttxgg.inc.

The device code evaluates the Lorentz part a_d of 38 terms per helicity
configuration (the 36 diagrams, the four-gluon vertex split into its three
colour structures), in the order of TERMS below, without the factors of i
that the Feynman rules give each class (PHASES below: 1, i or -1).  The
colour sum sum_colours |sum_d C_d phi_d a_d|^2 = sum_de a_d K_de conj(a_e),
K_de = phi_d conj(phi_e) sum_colours C_d conj(C_e), is real with the class
phases inside and of rank 11.  The kernel uses a basis of 11 of the terms
themselves (sparse_basis): every term's phased colour factor is a sum of
the basis terms' with signs, B [11][38], so K = B^T G B with G the basis
terms' Gram matrix (integers over 36), and the colour sum is
sum_rs G_rs Re(b_r conj(b_s)) with b = B a: additions per term and one
11 x 11 quadratic form.  (projection() gives the equivalent real rank-11
projection W with W^T W = K, the kernel's first form.)  The colour factors
come from an explicit sum over the 3^4 8^2 colour assignments of each
term's colour factor: products of T = lambda/2 along the quark line (v-bar
index j to u index i) and the top line (u-bar index k to v index l) and
structure constants f^{abc} = -2i Tr([T^a, T^b] T^c), internal indices
summed.

Colour slots: 0, 1 the gluons' adjoint indices; 2 + x internal index x.
A term: (quark-line slots from the u end, top-line slots from the v end,
f factors (x, y, z) -> f^{xyz}, number of internal indices).
"""
import itertools

import numpy as np


def _terms():
    t = []
    orders = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    # 1: both gluons and the spine (internal 0) on the quark line
    for o in orders:
        t.append((tuple(o), (2,), (), 1))
    # 2: both gluons and the spine on the top line
    for o in orders:
        t.append(((2,), tuple(o), (), 1))
    # 3: gluon ga on the quark line, gb on the top line, 2 x 2 orders
    for ga in (0, 1):
        gb = 1 - ga
        for oq in (0, 1):
            qs = [0, 0]
            qs[oq], qs[1 - oq] = ga, 2
            for ot in (0, 1):
                ts = [0, 0]
                ts[ot], ts[1 - ot] = gb, 2
                t.append((tuple(qs), tuple(ts), (), 1))
    # 4: ga on the spine (f^{2 ga 3}), gb on the quark line
    for ga in (0, 1):
        gb = 1 - ga
        for oq in (0, 1):
            qs = [0, 0]
            qs[oq], qs[1 - oq] = gb, 2
            t.append((tuple(qs), (3,), ((2, ga, 3),), 2))
    # 5: ga on the spine, gb on the top line
    for ga in (0, 1):
        gb = 1 - ga
        for ot in (0, 1):
            ts = [0, 0]
            ts[ot], ts[1 - ot] = gb, 3
            t.append(((2,), tuple(ts), ((2, ga, 3),), 2))
    # 6: both on the spine, ga nearer the quark line
    for ga in (0, 1):
        gb = 1 - ga
        t.append(((2,), (4,), ((2, ga, 3), (3, gb, 4)), 3))
    # the four-gluon vertex: spine in 2, spine out 3, internal 4
    t.append(((2,), (3,), ((2, 0, 4), (1, 3, 4)), 3))
    t.append(((2,), (3,), ((2, 1, 4), (0, 3, 4)), 3))
    t.append(((2,), (3,), ((2, 3, 4), (0, 1, 4)), 3))
    # 7: the composite (slot 3, f^{3 0 1}) on the quark line, the top line, the spine
    for oq in (0, 1):
        qs = [0, 0]
        qs[oq], qs[1 - oq] = 3, 2
        t.append((tuple(qs), (2,), ((3, 0, 1),), 2))
    for ot in (0, 1):
        ts = [0, 0]
        ts[ot], ts[1 - ot] = 3, 2
        t.append(((2,), tuple(ts), ((3, 0, 1),), 2))
    t.append(((2,), (3,), ((2, 4, 3), (4, 0, 1)), 3))
    return t


TERMS = _terms()

# the factor of i of each term's class: 0-19 1, 20-27 i, 28-32 -1, 33-36 i, 37 -1
PHASES = [1] * 20 + [1j] * 8 + [-1] * 5 + [1j] * 4 + [-1]


def _generators(G):
    T = np.array(G.gell_mann_half(), dtype=complex)          # [8][3][3]
    f = np.zeros((8, 8, 8))
    for a, b, c in itertools.product(range(8), repeat=3):
        comm = T[a] @ T[b] - T[b] @ T[a]
        f[a, b, c] = (-2j * np.trace(comm @ T[c])).real
    return T, f


def colour_values(G):
    """C[assignment][term] for the assignments (i, j, k, l, a1, a2) in
    lexicographic order (i slowest)."""
    T, f = _generators(G)
    n_ass = 3 ** 4 * 64
    C = np.zeros((n_ass, len(TERMS)), dtype=complex)
    for d, (qs, ts, fs, nint) in enumerate(TERMS):
        # tensor over (a1, a2, internal...) of the f product, and the line matrices
        for ints in itertools.product(range(8), repeat=nint):
            for a1 in range(8):
                for a2 in range(8):
                    slot = [a1, a2, *ints]
                    fv = 1.0
                    for x, y, z in fs:
                        fv *= f[slot[x], slot[y], slot[z]]
                    if fv == 0.0:
                        continue
                    Mq = np.eye(3, dtype=complex)
                    for s in qs:                     # from the u end: rightmost first
                        Mq = T[slot[s]] @ Mq
                    Mt = np.eye(3, dtype=complex)
                    for s in ts:
                        Mt = T[slot[s]] @ Mt
                    # assignment index of (i, j, k, l, a1, a2)
                    val = fv * np.einsum("ji,kl->ijkl", Mq, Mt).reshape(81)
                    C[np.arange(81) * 64 + a1 * 8 + a2, d] += val
    return C


def projection(G):
    """W [rank][38] real with sum_r |sum_d W_rd a_d|^2 the colour sum of the
    class-phase-free Lorentz parts a_d, and K (with the phases)."""
    C = colour_values(G)
    ph = np.array(PHASES, dtype=complex)
    K = ph[:, None] * (C.T @ C.conj()) * ph.conj()[None, :]
    assert np.abs(K.imag).max() < 1e-12 * np.abs(K).max(), "colour matrix with the class phases is not real"
    K = K.real
    # K = U diag(lam) U^T, so a^T K conj(a) = sum_r lam_r |sum_d U_dr a_d|^2
    lam, U = np.linalg.eigh(K)
    keep = lam > 1e-9 * lam.max()
    W = np.sqrt(lam[keep])[:, None] * U[:, keep].T
    return W, K


def sparse_basis(G):
    """An 11-term colour basis among the terms themselves: the first terms
    whose colour factors (with their class phases) are linearly independent.
    Every term's factor is then an integer combination of the basis factors
    (entries +-1), B [11][38], and the colour sum is
    sum_rs Gm_rs b_r conj(b_s) with b = B a and Gm the real Gram matrix of
    the basis factors (integers over den = 36).  Returns basis, B, den * Gm,
    den, and K."""
    C = colour_values(G) * np.array(PHASES, dtype=complex)[None, :]
    basis = []
    for d in range(len(TERMS)):
        if np.linalg.matrix_rank(C[:, basis + [d]], tol=1e-9) > len(basis):
            basis.append(d)
    E = C[:, basis]
    B = np.linalg.lstsq(E, C, rcond=None)[0]
    Bi = np.rint(B.real).astype(int)
    assert np.abs(B - Bi).max() < 1e-9, "basis coefficients are not integers"
    Gm = E.T @ E.conj()
    assert np.abs(Gm.imag).max() < 1e-12
    den = 36
    Gi = np.rint(Gm.real * den).astype(int)
    assert np.abs(Gm.real * den - Gi).max() < 1e-9, "Gram matrix not over 36"
    K = C.T @ C.conj()
    assert np.abs(Bi.T @ Gi @ Bi / den - K).max() < 1e-9 * np.abs(K).max()
    return basis, Bi, Gi, den, K.real


def generate(G):
    basis, B, Gi, den, _ = sparse_basis(G)
    r = B.shape[0]
    lines = ["// Generated by gen_qqbar.py: colour basis of q qbar -> t tbar g g.",
             f"constexpr int QQ4_RANK = {r};",
             f"constexpr int QQ4_TERMS = {len(TERMS)};",
             f"// basis terms {basis}; term d's colour factor (with its class phase) is",
             "// sum_r QQ4_B[r][d] times that of basis term r; the colour sum of the",
             "// class-phase-free Lorentz parts a_d is sum_rs QQ4_G[r][s] b_r conj(b_s) / QQ4_GDEN",
             "// with b_r = sum_d QQ4_B[r][d] a_d",
             f"constexpr int QQ4_GDEN = {den};",
             f"static constexpr signed char QQ4_B[{r}][{len(TERMS)}] = {{"]
    for row in B:
        lines.append("    {" + ", ".join(str(int(v)) for v in row) + "},")
    lines.append("};")
    lines.append(f"static constexpr int QQ4_G[{r}][{r}] = {{")
    for row in Gi:
        lines.append("    {" + ", ".join(str(int(v)) for v in row) + "},")
    lines.append("};")
    return "\n".join(lines) + "\n"
