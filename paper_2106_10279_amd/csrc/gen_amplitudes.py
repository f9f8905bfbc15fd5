#!/usr/bin/env python3
"""Generate the per-helicity |M|^2 device functions for g g -> t tbar + n gluons.

Sec. 2.3 of the paper builds the matrix element from external wavefunctions,
vertices and propagators and sums over helicities; MG5_aMC writes that code
per process.  This script plays the exporter's role for the three processes
here: it writes straight-line HIP code, one function per gluon count, that a
single GPU lane runs for one helicity configuration.

Physics (all particles outgoing, g_s = 1):
  * colour-flow decomposition  M = sum_sigma (T^{a_sigma1}..T^{a_sigman})_{i j} A(sigma),
    T = lambda/2 (Mangano-Parke);
  * A(sigma) from Berends-Giele recursion over ordered gluon sequences with
    the colour-ordered rules of the Lagrangian with D = d - i g T^a A^a:
        j(s)  = -(1/P^2) [ sum_{s=s1 s2} j1 ((2P1+P2).j2) - j2 ((P1+2P2).j1) + (P2-P1)(j1.j2)
                          + sum_{s=s1 s2 s3} j1 (j2.j3) - 2 j2 (j1.j3) + j3 (j1.j2) ]
        U(t)  = -[ sum_{t = a b} U(a) gamma.j(b) ] (P-slash + m) / (P^2 - m^2 + i m Gamma)
        A(s)  =  sum_{s = a b} U(a) gamma.j(b) v          (common factor i dropped)
    with U(empty) = ubar(k_t) and P = k_t + P(t) on the top line;
  * reflection j(reverse s) = (-1)^(|s|+1) j(s) halves the gluon currents;
  * colour sum  A^dagger C A  with C in exact integers over a common
    denominator, computed here by the SU(N) Fierz identities.

Representation (chosen for the GPU, unlike the CPU oracle's): chiral gamma
matrices with 2-component blocks; spinors u = (sqrt(p.sigma) xi, sqrt(p.sigma_bar) xi)
with the branch-free square root (p.sigma + m)/sqrt(2(E+m)) and xi along z;
real linear gluon polarisations, so every pure-gluon current is a real
4-vector.  Momentum sums and propagator denominators are formed in double
precision from double momenta and cast to the arithmetic type T afterwards.
"""
from __future__ import annotations

import argparse
import bisect
import functools
import itertools
import math
import os
from fractions import Fraction

# ----------------------------------------------------------------------------
# colour matrix by the Fierz identities (exact rationals)
# ----------------------------------------------------------------------------
_N = Fraction(3)


def _contract(words):
    """Sum over repeated adjoint indices of a product of traces of T = lambda/2."""
    words = [tuple(w) for w in words]
    first = next((w[0] for w in words if w), None)
    if first is None:
        return _N ** len(words)
    hits = [(i, j) for i, w in enumerate(words) for j, a in enumerate(w) if a == first]
    (i1, j1), (i2, j2) = hits
    others = [w for i, w in enumerate(words) if i not in (i1, i2)]
    half = Fraction(1, 2)
    if i1 == i2:
        w = words[i1]
        inner, outer = w[j1 + 1:j2], w[j2 + 1:] + w[:j1]
        return half * (_contract(others + [inner, outer]) - _contract(others + [inner + outer]) / _N)
    a = words[i1][j1 + 1:] + words[i1][:j1]
    b = words[i2][j2 + 1:] + words[i2][:j2]
    return half * (_contract(others + [a + b]) - _contract(others + [a, b]) / _N)


def colour_matrix(n):
    """C[s][t] = sum over colours of conj((T^s)_ij) (T^t)_ij, orderings in
    lexicographic order.  Returns (integer matrix, common denominator)."""
    perms = sorted(itertools.permutations(range(n)))
    C = [[_contract([tuple(reversed(s)) + tuple(t)]) for t in perms] for s in perms]
    den = 1
    for row in C:
        for v in row:
            den = den * v.denominator // math.gcd(den, v.denominator)
    K = [[int(v * den) for v in row] for row in C]
    return perms, K, den


def lc_numerator(n, den):
    """Leading-colour approximation: the colour matrix replaced by
    c_LC = (N^2 - 1) N^(n - 1) / 2^n times the identity (N = 3), the leading
    power of N of its diagonal N C_F^n; returned over the common denominator
    of the full matrix (an integer for n = 2, 3, 4)."""
    from fractions import Fraction
    v = Fraction(8 * 3 ** (n - 1), 2 ** n) * den
    assert v.denominator == 1
    return int(v)


def colour_count(n):
    """Colour assignments sampled by the Monte Carlo over colours: gluon
    adjoint indices (8 each), top colour and antitop anticolour (3 each)."""
    return 9 * 8 ** n


def gell_mann_half():
    """T^a = lambda^a / 2, a = 1 .. 8, as (re, im) 3 x 3 tables."""
    r3 = math.sqrt(3.0)
    lam = [[[0j] * 3 for _ in range(3)] for _ in range(8)]
    lam[0][0][1] = lam[0][1][0] = 1
    lam[1][0][1], lam[1][1][0] = -1j, 1j
    lam[2][0][0], lam[2][1][1] = 1, -1
    lam[3][0][2] = lam[3][2][0] = 1
    lam[4][0][2], lam[4][2][0] = -1j, 1j
    lam[5][1][2] = lam[5][2][1] = 1
    lam[6][1][2], lam[6][2][1] = -1j, 1j
    lam[7][0][0] = lam[7][1][1] = 1 / r3
    lam[7][2][2] = -2 / r3
    return [[[complex(v) / 2 for v in row] for row in m] for m in lam]


@functools.lru_cache(maxsize=None)
def _flow_table(n, perms):
    return flow_table_uncached(n, perms)


def flow_table(n, perms):
    return _flow_table(n, tuple(tuple(sg) for sg in perms))


def flow_table_uncached(n, perms):
    """Colour flows with a non-vanishing factor for some ordering, in
    increasing code = j + 3 i + 9 sum_g 9^g (3 a_g + b_g), packed as
    j | i << 2 | a_g << (4 + 4 g) | b_g << (6 + 4 g), each with its integer
    sampling weight 18^n sum_s c_s^2 = sum_s prod_g (3 f_g)^2 over the
    orderings s whose line reaches j, f_g the gluon's factor without the
    1/sqrt 2 (1 off the diagonal, 2/3 or -1/3 on it).  Gluon g carries colour
    a_g and anticolour b_g, state (e_ab - delta_ab / 3) / sqrt 2; each row of
    such a matrix has at most one non-zero entry, so a factor is a walk along
    the colour line from i: an off-diagonal pair (a, b) needs the current colour
    a and moves it to b, a diagonal pair keeps it.  The walk ends on j or the
    factor vanishes."""
    def weight(order, pairs, i, j):
        r, w = i, 1
        for g in order:
            a, b = pairs[g]
            if a != b:
                if r != a:
                    return 0
                r = b
                w *= 9
            else:
                w *= 4 if r == a else 1
        return w if r == j else 0

    out = []
    for code in range(9 * 9 ** n):
        j, i, rest = code % 3, (code // 3) % 3, code // 9
        pairs = [divmod((rest // 9 ** g) % 9, 3) for g in range(n)]
        wsum = sum(weight(sg, pairs, i, j) for sg in perms)
        if wsum:
            word = j | (i << 2)
            for g, (a, b) in enumerate(pairs):
                word |= (a << (4 + 4 * g)) | (b << (6 + 4 * g))
            out.append((word, wsum))
    return out


# ----------------------------------------------------------------------------
# code emission helpers
# ----------------------------------------------------------------------------
def name(seq):
    return "".join(str(g) for g in seq)


def mask(seq):
    m = 0
    for g in seq:
        m |= 1 << g
    return m


class Layout:
    """Offsets of the per-event table (doubles) shared by the helicity lanes:
    subset momenta P[m], -1/P[m]^2, top-line momenta K[m] = k_t + P[m] and
    propagator factors -1/(K^2 - m^2 + i m Gamma), ubar and v for both spins,
    polarisation vectors of the final-state gluons for both states."""

    def __init__(self, n):
        self.n = n
        off = 0
        self.P = {}
        for m in range(1, 1 << n):
            self.P[m] = off
            off += 4
        self.ninv = {}
        for m in range(1, 1 << n):
            if bin(m).count("1") >= 2:
                self.ninv[m] = off
                off += 1
        self.K = {}
        for m in range(1, (1 << n) - 1):
            self.K[m] = off          # K[0..3], fr, fi
            off += 6
        self.Kv = {}
        for m in range(1, 1 << n):
            if 1 <= bin(m).count("1") <= n - 2:
                self.Kv[m] = off     # -k_tbar - P[m] (= k_t + P[complement]), -1/(Kv^2 - m^2 + i m Gamma)
                off += 6
        self.ub = off
        off += 16
        self.v = off
        off += 16
        self.eps = {}
        for g in range(n):
            self.eps[g] = off
            off += 8
        self.size = off


class CoopTable:
    """Per-event table of the cooperative evaluation (n >= 3), in units of the
    amplitude type: subset momenta P[m] (1 <= |m| <= n-1), -1/P[m]^2
    (2 <= |m| <= n), the top-line momenta and propagator factors of single
    gluons K[g] = k_t + p_g, the antitop-line ones Kv[m] (1 <= |m| <= n-2),
    ubar and v for both spins.  The gluon polarisation vectors go straight
    into the level-1 currents of the object store."""

    def __init__(self, n):
        self.n = n
        # the spinors first: 16-byte aligned for 128-bit LDS reads
        self.ub = 0
        self.v = 16
        off = 32
        self.P = {}
        for m in range(1, 1 << n):
            if bin(m).count("1") <= n - 1:
                self.P[m] = off
                off += 4
        self.ninv = {}
        for m in range(1, 1 << n):
            if bin(m).count("1") >= 2:
                self.ninv[m] = off
                off += 1
        self.K1 = {}
        for g in range(n):
            self.K1[g] = off           # K[0..3], fr, fi
            off += 6
        self.Kv = {}
        for m in range(1, 1 << n):
            if 1 <= bin(m).count("1") <= n - 2:
                self.Kv[m] = off       # -k_tbar - P[m] (= k_t + P[complement]), -1/(Kv^2 - m^2 + i m Gamma)
                off += 6
        # a multiple of 4 elements, so that every event's table starts aligned
        self.size = (off + 3) // 4 * 4

    def mom_flops(self):
        n = self.n
        # subset sums, plus the complement sums of the antitop-line momenta
        return (sum(4 * (bin(m).count("1") - 1) for m in range(1, 1 << n)) + 8 * len(self.ninv)
                + sum(4 * (n - bin(m).count("1") - 1) for m in self.Kv)
                + 17 * (len(self.K1) + len(self.Kv)) + 4 * 24 + (n - 2) * 2 * 16 + 2)


def emit_coop_fill(n, tl, co):
    """Fill of the cooperative table by the lanes of one event: lane m
    (1 .. 2^n - 1) handles subset m, the next four the spinors, lane 0 the
    incoming polarisations, the following ones the outgoing ones (written as
    level-1 gluon currents j(g; h) = eps_g(h) into the object store)."""
    L = []
    w = L.append
    nsub = (1 << n) - 1
    w("    constexpr int CW = 16 / (int)sizeof(T);")
    w("    const double m2 = mt * mt;")
    w(f"    if (lane >= 1 && lane <= {nsub}) {{")
    w("        const int m = lane;")
    # P: the subset's momentum; C: its complement's (all momenta outgoing)
    w("        double P0 = 0.0, P1 = 0.0, P2 = 0.0, P3 = 0.0, C0 = 0.0, C1 = 0.0, C2 = 0.0, C3 = 0.0;")
    for g in range(n):
        if g == 0:
            pv = ["-eb", "0.0", "0.0", "-eb"]
        elif g == 1:
            pv = ["-eb", "0.0", "0.0", "eb"]
        else:
            pv = [f"mom[{8 + 4 * (g - 2) + mu}]" for mu in range(4)]
        w(f"        if (m & {1 << g}) {{ P0 += {pv[0]}; P1 += {pv[1]}; P2 += {pv[2]}; P3 += {pv[3]}; }}")
        w(f"        else {{ C0 += {pv[0]}; C1 += {pv[1]}; C2 += {pv[2]}; C3 += {pv[3]}; }}")
    p_off = ", ".join(str(tl.P.get(m, -1)) for m in range(1, 1 << n))
    w(f"        const short p_off[{nsub}] = {{{p_off}}};")
    w("        if (p_off[m - 1] >= 0) {")
    w("            T* o = tab + p_off[m - 1];")
    w("            o[0] = (T)P0; o[1] = (T)P1; o[2] = (T)P2; o[3] = (T)P3;")
    w("        }")
    ninv_offsets = ", ".join(str(tl.ninv.get(m, -1)) for m in range(1, 1 << n))
    w(f"        const short ninv_off[{nsub}] = {{{ninv_offsets}}};")
    w("        if (ninv_off[m - 1] >= 0)")
    w("            tab[ninv_off[m - 1]] = (T)(-1.0 / (P0 * P0 - P1 * P1 - P2 * P2 - P3 * P3));")
    k_offsets = ", ".join(str(tl.K1[(m.bit_length() - 1)]) if bin(m).count("1") == 1 else "-1"
                          for m in range(1, 1 << n))
    w(f"        const short k_off[{nsub}] = {{{k_offsets}}};")
    w("        if (k_off[m - 1] >= 0) {")
    w("            const double K0 = mom[0] + P0, K1 = mom[1] + P1, K2 = mom[2] + P2, K3 = mom[3] + P3;")
    w("            const double re = K0 * K0 - K1 * K1 - K2 * K2 - K3 * K3 - m2;")
    w("            const double inv = 1.0 / (re * re + mw * mw);")
    w("            T* k = tab + k_off[m - 1];")
    w("            k[0] = (T)K0; k[1] = (T)K1; k[2] = (T)K2; k[3] = (T)K3;")
    w("            k[4] = (T)(-re * inv);")
    w("            k[5] = (T)(mw * inv);")
    w("        }")
    kv_offsets = ", ".join(str(tl.Kv.get(m, -1)) for m in range(1, 1 << n))
    w(f"        const short kv_off[{nsub}] = {{{kv_offsets}}};")
    # the antitop-line momentum -k_tbar - P[m] is formed as k_t + P[complement]:
    # the same sum as the top-line propagator of that internal line, so that
    # both sides of a near on-shell line see the same rounding of the event's
    # momenta (their conservation holds to rounding only)
    w("        if (kv_off[m - 1] >= 0) {")
    w("            const double K0 = mom[0] + C0, K1 = mom[1] + C1, K2 = mom[2] + C2, K3 = mom[3] + C3;")
    w("            const double re = K0 * K0 - K1 * K1 - K2 * K2 - K3 * K3 - m2;")
    w("            const double inv = 1.0 / (re * re + mw * mw);")
    w("            T* k = tab + kv_off[m - 1];")
    w("            k[0] = (T)K0; k[1] = (T)K1; k[2] = (T)K2; k[3] = (T)K3;")
    w("            k[4] = (T)(-re * inv);")
    w("            k[5] = (T)(mw * inv);")
    w("        }")
    w("    }")
    w(f"    if (lane >= {nsub + 1} && lane < {nsub + 5}) {{")
    w(f"        const int t = lane - {nsub + 1};     // 0, 1: ubar spins; 2, 3: v spins")
    w("        cplx<double> sp[4];")
    w("        if (t < 2)")
    w("            spinor_ubar<double>(mom, mt, t, sp);")
    w("        else")
    w("            spinor_v<double>(mom + 4, mt, t - 2, sp);")
    w(f"        T* o = tab + (t < 2 ? {tl.ub} + 8 * t : {tl.v} + 8 * (t - 2));")
    w("        for (int i = 0; i < 4; ++i) { o[2 * i] = (T)sp[i].x; o[2 * i + 1] = (T)sp[i].y; }")
    w("    }")
    # incoming gluons along the beams: (0, 1, 0, 0) and (0, 0, 1, 0)
    w("    if (lane == 0) {")
    w(f"        st4s<NS>(obj + {co.gj}, (T)0, (T)1, (T)0, (T)0);")
    w(f"        st4s<NS>(obj + {co.gj} + CW, (T)0, (T)0, (T)1, (T)0);")
    w(f"        st4s<NS>(obj + {co.gj} + 2 * CW, (T)0, (T)1, (T)0, (T)0);")
    w(f"        st4s<NS>(obj + {co.gj} + 3 * CW, (T)0, (T)0, (T)1, (T)0);")
    w("    }")
    w(f"    if (lane >= {nsub + 5} && lane < {nsub + 5 + 2 * (n - 2)}) {{")
    w(f"        const int t = lane - {nsub + 5};")
    w("        const int g = 2 + t / 2, h = t & 1;")
    w("        double e[4];")
    w("        linear_pol<double>(mom + 8 + 4 * (g - 2), h, e);")
    w(f"        st4s<NS>(obj + {co.gj} + CW * (2 * g + h), (T)e[0], (T)e[1], (T)e[2], (T)e[3]);")
    w("    }")
    return "\n".join(L)


class Emitter:
    # Flop accounting (+, -, x = 1; fused multiply-add = 2; sqrt and divide
    # = 1 each): `hel` counts the arithmetic that depends on the helicity
    # configuration (done by every helicity lane), `mom` the arithmetic that
    # depends on the momenta only (done once per event into the table).
    def __init__(self, n, lay):
        self.n = n
        self.lay = lay
        self.lines = []
        self.done = set()
        self.hel = 0
        self.mom = 0

    def w(self, s=""):
        self.lines.append("    " + s)

    def pvec(self, m):
        return f"(tab + {self.lay.P[m]})"

    # -- gluon currents (real 4-vectors) ---------------------------------------
    def gcur(self, seq, memo=True):
        seq = tuple(seq)
        if len(seq) == 1:
            return f"eps{seq[0]}"
        key = ("j", seq)
        if key in self.done:
            return f"j{name(seq)}"
        rev = tuple(reversed(seq))
        if ("j", rev) in self.done:
            # j(reverse s) = (-1)^(|s|+1) j(s): a signed view, no copy
            sign = "" if (len(seq) + 1) % 2 == 0 else "-"
            return f"{sign}j{name(rev)}"
        L = len(seq)
        subs = []
        for a in range(1, L):
            subs.append((self.gcur(seq[:a]), self.gcur(seq[a:]), mask(seq[:a]), mask(seq[a:])))
        trip = []
        for a in range(1, L):
            for b in range(a + 1, L):
                trip.append((self.gcur(seq[:a]), self.gcur(seq[a:b]), self.gcur(seq[b:])))
        nm = f"j{name(seq)}"
        if memo:
            self.done.add(key)
        else:
            nm = f"jq{name(seq)}"
        self.w(f"T {nm}[4];")
        self.w("{")
        self.w("    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;")
        for (j1, j2, m1, m2) in subs:
            # conserved currents (P1.j1 = P2.j2 = 0): bracket
            # 2 (P1.j2) j1 - 2 (P2.j1) j2 + (j1.j2) (P2 - P1)
            self.hel += 21 + 28
            P1, P2 = self.pvec(m1), self.pvec(m2)
            self.w("    {")
            self.w(f"        const double* p1 = {P1}; const double* p2 = {P2};")
            self.w("        T q1[4], q2[4];")
            self.w("        for (int mu = 0; mu < 4; ++mu) { q1[mu] = (T)p1[mu]; q2[mu] = (T)p2[mu]; }")
            self.w(f"        const T c1 = (T)2 * (q1[0] * {j2}[0] - q1[1] * {j2}[1] - q1[2] * {j2}[2] - q1[3] * {j2}[3]);")
            self.w(f"        const T c2 = (T)2 * (q2[0] * {j1}[0] - q2[1] * {j1}[1] - q2[2] * {j1}[2] - q2[3] * {j1}[3]);")
            self.w(f"        const T c12 = {j1}[0] * {j2}[0] - {j1}[1] * {j2}[1] - {j1}[2] * {j2}[2] - {j1}[3] * {j2}[3];")
            for mu in range(4):
                self.w(f"        a{mu} += {j1}[{mu}] * c1 - {j2}[{mu}] * c2 + c12 * (q2[{mu}] - q1[{mu}]);")
            self.w("    }")
        for (j1, j2, j3) in trip:
            self.hel += 21 + 28
            self.w("    {")
            self.w(f"        const T d23 = {j2}[0] * {j3}[0] - {j2}[1] * {j3}[1] - {j2}[2] * {j3}[2] - {j2}[3] * {j3}[3];")
            self.w(f"        const T d13 = {j1}[0] * {j3}[0] - {j1}[1] * {j3}[1] - {j1}[2] * {j3}[2] - {j1}[3] * {j3}[3];")
            self.w(f"        const T d12 = {j1}[0] * {j2}[0] - {j1}[1] * {j2}[1] - {j1}[2] * {j2}[2] - {j1}[3] * {j2}[3];")
            for mu in range(4):
                self.w(f"        a{mu} += {j1}[{mu}] * d23 - (T)2 * {j2}[{mu}] * d13 + {j3}[{mu}] * d12;")
            self.w("    }")
        self.hel += 4
        self.w(f"    const T f = (T)tab[{self.lay.ninv[mask(seq)]}];")
        for mu in range(4):
            self.w(f"    {nm}[{mu}] = a{mu} * f;")
        self.w("}")
        return nm

    # -- fermion prefix currents (row spinors) --------------------------------
    def fcur(self, seq):
        seq = tuple(seq)
        if not seq:
            return "ub"
        key = ("U", seq)
        if key in self.done:
            return f"U{name(seq)}"
        terms = []
        for a in range(len(seq)):
            terms.append((self.fcur(seq[:a]), self.gcur(seq[a:])))
        m = mask(seq)
        nm = f"U{name(seq)}"
        self.done.add(key)
        self.w(f"cT {nm}[4];")
        self.w("{")
        self.w("    cT s0 = cT(0, 0), s1 = cT(0, 0), s2 = cT(0, 0), s3 = cT(0, 0);")
        self.hel += 50 * len(terms) + 80
        for (U, j) in terms:
            # row (aL, aR) x gamma.j = (aR (j.sigmabar), aL (j.sigma))
            if j.startswith("-"):
                self.w(f"    rowslash_acc<-1>({U}, {j[1:]}, s0, s1, s2, s3);")
            else:
                self.w(f"    rowslash_acc({U}, {j}, s0, s1, s2, s3);")
        o = self.lay.K[m]
        self.w(f"    const T Kc[4] = {{(T)tab[{o}], (T)tab[{o + 1}], (T)tab[{o + 2}], (T)tab[{o + 3}]}};")
        self.w(f"    rowprop(s0, s1, s2, s3, Kc, (T)mt, (T)tab[{o + 4}], (T)tab[{o + 5}], {nm});")
        self.w("}")
        return nm

    def bilinear(self, seq):
        """c^mu = U(seq) gamma^mu v (complex 4-vector)."""
        seq = tuple(seq)
        key = ("c", seq)
        nm = f"c{name(seq)}" if seq else "c_"
        if key in self.done:
            return nm
        U = self.fcur(seq)
        self.done.add(key)
        self.hel += 64
        self.w(f"cT {nm}[4];")
        self.w(f"bilinear(" + U + ", v, " + nm + ");")
        return nm


def emit_table_fill(n, lay):
    """Per-event table, filled by the lanes of one wave: lane m (1 .. 2^n - 1)
    handles subset m; lanes 2^n .. 2^n + 3 the spinors; the next ones the
    polarisation vectors."""
    L = []
    w = L.append
    nsub = (1 << n) - 1
    w("    const double m2 = mt * mt;")
    w(f"    if (lane >= 1 && lane <= {nsub}) {{")
    w("        const int m = lane;")
    w("        double P0 = 0.0, P1 = 0.0, P2 = 0.0, P3 = 0.0, C0 = 0.0, C1 = 0.0, C2 = 0.0, C3 = 0.0;")
    for g in range(n):
        if g == 0:
            pv = ["-eb", "0.0", "0.0", "-eb"]
        elif g == 1:
            pv = ["-eb", "0.0", "0.0", "eb"]
        else:
            pv = [f"mom[{8 + 4 * (g - 2) + mu}]" for mu in range(4)]
        w(f"        if (m & {1 << g}) {{ P0 += {pv[0]}; P1 += {pv[1]}; P2 += {pv[2]}; P3 += {pv[3]}; }}")
        w(f"        else {{ C0 += {pv[0]}; C1 += {pv[1]}; C2 += {pv[2]}; C3 += {pv[3]}; }}")
    w("        const int off_p = 4 * (m - 1);")
    w("        tab[off_p + 0] = P0; tab[off_p + 1] = P1; tab[off_p + 2] = P2; tab[off_p + 3] = P3;")
    # -1/P^2 for |m| >= 2
    ninv_offsets = ", ".join(str(lay.ninv.get(m, -1)) for m in range(1, 1 << n))
    w(f"        const int ninv_off[{nsub}] = {{{ninv_offsets}}};")
    w("        if (ninv_off[m - 1] >= 0)")
    w("            tab[ninv_off[m - 1]] = -1.0 / (P0 * P0 - P1 * P1 - P2 * P2 - P3 * P3);")
    k_offsets = ", ".join(str(lay.K.get(m, -1)) for m in range(1, 1 << n))
    w(f"        const int k_off[{nsub}] = {{{k_offsets}}};")
    w("        if (k_off[m - 1] >= 0) {")
    w("            const double K0 = mom[0] + P0, K1 = mom[1] + P1, K2 = mom[2] + P2, K3 = mom[3] + P3;")
    w("            const double re = K0 * K0 - K1 * K1 - K2 * K2 - K3 * K3 - m2;")
    w("            const double inv = 1.0 / (re * re + mw * mw);")
    w("            double* k = tab + k_off[m - 1];")
    w("            k[0] = K0; k[1] = K1; k[2] = K2; k[3] = K3;")
    w("            k[4] = -re * inv;")
    w("            k[5] = mw * inv;")
    w("        }")
    kv_offsets = ", ".join(str(lay.Kv.get(m, -1)) for m in range(1, 1 << n))
    w(f"        const int kv_off[{nsub}] = {{{kv_offsets}}};")
    # -k_tbar - P[m] formed as k_t + P[complement] (see the cooperative fill)
    w("        if (kv_off[m - 1] >= 0) {")
    w("            const double K0 = mom[0] + C0, K1 = mom[1] + C1, K2 = mom[2] + C2, K3 = mom[3] + C3;")
    w("            const double re = K0 * K0 - K1 * K1 - K2 * K2 - K3 * K3 - m2;")
    w("            const double inv = 1.0 / (re * re + mw * mw);")
    w("            double* k = tab + kv_off[m - 1];")
    w("            k[0] = K0; k[1] = K1; k[2] = K2; k[3] = K3;")
    w("            k[4] = -re * inv;")
    w("            k[5] = mw * inv;")
    w("        }")
    w("    }")
    w(f"    if (lane >= {nsub + 1} && lane < {nsub + 5}) {{")
    w(f"        const int t = lane - {nsub + 1};     // 0, 1: ubar spins; 2, 3: v spins")
    w("        cplx<double> sp[4];")
    w("        if (t < 2)")
    w("            spinor_ubar<double>(mom, mt, t, sp);")
    w("        else")
    w("            spinor_v<double>(mom + 4, mt, t - 2, sp);")
    w(f"        double* o = tab + (t < 2 ? {lay.ub} + 8 * t : {lay.v} + 8 * (t - 2));")
    w("        for (int i = 0; i < 4; ++i) { o[2 * i] = sp[i].x; o[2 * i + 1] = sp[i].y; }")
    w("    }")
    # incoming gluons along the beams: (0, 1, 0, 0) and (0, 0, 1, 0)
    w(f"    if (lane == 0) {{")
    w(f"        double* o = tab + {lay.eps[0]};")
    w("        for (int i = 0; i < 16; ++i) o[i] = 0.0;")
    w("        o[1] = 1.0; o[6] = 1.0; o[9] = 1.0; o[14] = 1.0;")
    w("    }")
    if n > 2:
        w(f"    if (lane >= {nsub + 5} && lane < {nsub + 5 + 2 * (n - 2)}) {{")
        w(f"        const int t = lane - {nsub + 5};")
        w("        const int g = 2 + t / 2, h = t & 1;")
        w("        double e[4];")
        w("        linear_pol<double>(mom + 8 + 4 * (g - 2), h, e);")
        w(f"        double* o = tab + {lay.eps[0]} + 8 * g + 4 * h;")
        w("        for (int mu = 0; mu < 4; ++mu) o[mu] = e[mu];")
        w("    }")
    return "\n".join(L)


def generate(n):
    perms, K, den = colour_matrix(n)
    global _LAST_COUNT
    if n >= 3:
        # cooperative evaluation only: table, object store and helicity lanes
        nperm = len(perms)
        coop_text = generate_coop(n)
        _LAST_COUNT = {"per_helicity": _COOP_COUNT["per_helicity"],
                       "momentum_only": _COOP_COUNT["momentum_only"], "n_hel": 1 << (n + 2),
                       "n_orderings": nperm, "table_doubles": _COOP_COUNT["table"]}
        kdecl = ", ".join(str(v) for row in K for v in row)
        return f"""// Generated by gen_amplitudes.py for g g -> t tbar + {n - 2} gluon(s): {nperm} colour orderings,
// {1 << (n + 2)} helicity configurations.  Do not edit.
static constexpr int NPERM_NG{n} = {nperm};
static constexpr double COLOUR_DEN_NG{n} = {den}.0;
static constexpr int COLOUR_NUM_NG{n}[{nperm * nperm}] = {{{kdecl}}};
{coop_text}"""
    lay = Layout(n)
    e = Emitter(n, lay)
    e.hel_full = 0
    lc = lc_numerator(n, den)
    nperm = len(perms)
    e.w("const int sT = hel & 1, sB = (hel >> 1) & 1;")
    for g in range(n):
        if g < 2:
            e.w(f"const T eps{g}[4] = {{(T)0, (T)(((hel >> {2 + g}) & 1) ? 0 : 1), (T)(((hel >> {2 + g}) & 1) ? 1 : 0), (T)0}};")
        else:
            e.w(f"T eps{g}[4];")
            e.w(f"{{ const double* q = tab + {lay.eps[g]} + 4 * ((hel >> {2 + g}) & 1); "
                f"for (int mu = 0; mu < 4; ++mu) eps{g}[mu] = (T)q[mu]; }}")
    e.w("cT ub[4], v[4];")
    e.w(f"{{ const double* q = tab + {lay.ub} + 8 * sT; for (int i = 0; i < 4; ++i) ub[i] = cT((T)q[2 * i], (T)q[2 * i + 1]); }}")
    e.w(f"{{ const double* q = tab + {lay.v} + 8 * sB; for (int i = 0; i < 4; ++i) v[i] = cT((T)q[2 * i], (T)q[2 * i + 1]); }}")
    e.w(f"cT A[{nperm}];")
    e.w("T me = 0;")
    for idx, sg in enumerate(perms):
        e.w(f"// ordering {name(sg)}")
        parts = []
        for k in range(n - 1):
            c = e.bilinear(sg[:k])
            # the full-length current is used by one ordering only: computed
            # here and dropped, instead of being kept for its reflection
            j = e.gcur(sg[k:], memo=(k > 0))
            parts.append((c, j))
        U = e.fcur(sg[:n - 1])
        e.hel += 42                  # W = gamma.eps v for the last gluon
        e.hel += 16 * len(parts) + 32 + 2 + 4
        e.hel_full += 4 * sum(1 for t in range(idx) if K[idx][t] != 0)
        e.w("{")
        e.w("    T ar = 0, ai = 0;")
        for (c, j) in parts:
            if j.startswith("-"):
                e.w(f"    cdotj<-1>({c}, {j[1:]}, ar, ai);")
            else:
                e.w(f"    cdotj({c}, {j}, ar, ai);")
        e.w("    cT W[4];")
        e.w(f"    slashcol(eps{sg[n - 1]}, v, W);")
        e.w(f"    rowdotcol({U}, W, ar, ai);")
        e.w(f"    A[{idx}] = cT(ar, ai);")
        # incremental colour sum: K_ss |A_s|^2 + 2 Re(conj(A_s) sum_{t<s} K_st A_t);
        # leading colour (COL = 1) keeps c_LC |A_s|^2 only
        e.w(f"    const T kss = (T)(COL == 0 ? {K[idx][idx]} : {lc});")
        e.w("    T tr = kss * ar, ti = kss * ai;")
        off = [t for t in range(idx) if K[idx][t] != 0]
        if off:
            e.w("    if constexpr (COL == 0) {")
            for t in off:
                e.w(f"        tr += (T)({2 * K[idx][t]}) * A[{t}].x; ti += (T)({2 * K[idx][t]}) * A[{t}].y;")
            e.w("    }")
        e.w("    me += ar * tr + ai * ti;")
        e.w("}")
    # momentum-only work, done once per event for the table
    nsub = (1 << n) - 1
    e.mom = sum(4 * (bin(m).count("1") - 1) for m in range(1, 1 << n)) + 8 * len(lay.ninv) \
        + (4 + 8 + 3 + 2) * len(lay.K) + 4 * 24 + (n - 2) * 2 * 16 + 2
    body = "\n".join(e.lines)
    fill = emit_table_fill(n, lay)
    _LAST_COUNT = {"per_helicity": e.hel + e.hel_full, "per_helicity_lc": e.hel, "momentum_only": e.mom,
                   "n_hel": 1 << (n + 2), "n_orderings": nperm, "table_doubles": lay.size}
    kdecl = ", ".join(str(v) for row in K for v in row)
    return f"""// Generated by gen_amplitudes.py for g g -> t tbar + {n - 2} gluon(s): {nperm} colour orderings,
// {1 << (n + 2)} helicity configurations.  Do not edit.
// Arithmetic per helicity configuration: {e.hel + e.hel_full} flops ({e.hel} in leading colour);
// per event (table): {e.mom} flops.
static constexpr int FLOPS_PER_HEL_NG{n} = {e.hel + e.hel_full};
static constexpr int FLOPS_MOMENTUM_NG{n} = {e.mom};
static constexpr int NPERM_NG{n} = {nperm};
static constexpr int TABLE_NG{n} = {lay.size};
static constexpr double COLOUR_DEN_NG{n} = {den}.0;
static constexpr int COLOUR_NUM_NG{n}[{nperm * nperm}] = {{{kdecl}}};

// Per-event table of momentum-only quantities, written by the lanes of one
// wave (lane index `lane`); the caller synchronises the wave afterwards.
// mom: t[4], tbar[4], final gluons[4 each]; eb: beam energy sqrt(s_hat)/2;
// mt: top mass; mw: m_t * Gamma_t.
__device__ __forceinline__ void fill_table_ng{n}(const double* __restrict__ mom, double eb, double mt,
                                                double mw, double* __restrict__ tab, int lane)
{{
{fill}
}}

// Sum over colours of |M|^2 for helicity configuration `hel` (bit 0: top
// spin, bit 1: antitop spin, bit 2+g: gluon g polarisation), g_s = 1,
// from the event's table.  COL = 0: full colour matrix; COL = 1: leading
// colour, {lc}/{den} times the identity.
template <typename T, int COL>
__device__ __forceinline__ double colour_summed_me2_ng{n}(const double* __restrict__ tab_in, int hel, double mt)
{{
    using cT = cplx<T>;
    const double* __restrict__ tab = tab_in;
{body}
    return (double)me / COLOUR_DEN_NG{n};
}}
"""



# ----------------------------------------------------------------------------
# Cooperative evaluation (n >= 3): helicity-recycled objects built once per
# event in LDS by the wave's lanes, then one lane per helicity configuration.
# ----------------------------------------------------------------------------
def canon(seq):
    """Canonical representative of a gluon sequence under reflection and the
    sign j(seq) = sign * j(canon)."""
    seq = tuple(seq)
    if len(seq) == 1 or seq[0] < seq[-1]:
        return seq, 1
    return tuple(reversed(seq)), (1 if (len(seq) + 1) % 2 == 0 else -1)


class CoopLayout:
    """Object store of one event, in units of T:
       gluon currents j(s; hm) for every canonical ordered sequence s of
       length 1 .. n and helicity pattern hm of its gluons (sorted labels),
       4 T each; Ubar(a; s_t, h_a) and V(d; s_tbar, h_d), V(cd; s_tbar, h_c,
       h_d), 8 T each (complex 4-spinors, re/im interleaved).  Each of the
       four regions (currents, Ubar, V, two-gluon V) is stored chunk-major in
       16-byte chunks (ld4s / ldspins): object i of a region starts CW i
       values after the region's start, CW = 16 / sizeof(T)."""

    def __init__(self, n):
        self.n = n
        self.levels = {}
        self.base = {}
        off = 0
        for L in range(1, n + 1):
            seqs = sorted(sq for sq in itertools.permutations(range(n), L) if canon(sq)[0] == sq)
            self.levels[L] = seqs
            for sq in seqs:
                self.base[sq] = off
                off += 1 << L
        self.n_gj = off
        self.gj = 0
        self.u1 = 4 * off
        self.v1 = self.u1 + 8 * 4 * n
        self.pairs = sorted(itertools.permutations(range(n), 2)) if n >= 4 else []
        self.v2 = self.v1 + 8 * 4 * n
        self.size = self.v2 + 8 * 8 * len(self.pairs)
        # objects per region: the chunk stride of the chunk-major layout
        self.n_u1 = 4 * n
        self.n_v2 = 8 * len(self.pairs)

    def obj(self, seq):
        c, sg = canon(seq)
        return self.base[c], sg, c


def pext_py(x, m):
    """Bits of x at the set positions of m, packed in order."""
    r, k = 0, 0
    for i in range(4):
        if (m >> i) & 1:
            r |= ((x >> i) & 1) << k
            k += 1
    return r


def posmask(part, whole):
    srt = sorted(whole)
    m = 0
    for g in part:
        m |= 1 << srt.index(g)
    return m


def emit_coop(n, lay, co, K, den, perms):
    # lay: CoopTable (offsets in units of T)
    L_ = []
    w = L_.append
    flops_stage = 0
    # ---- constant tables of the gluon-current levels ----
    tables = []
    for L in range(2, n + 1):
        seqs = co.levels[L]
        ni, bs = [], []
        for sq in seqs:
            ni.append(str(lay.ninv[mask(sq)]))
            bs.append(str(co.base[sq]))
        npair, ntrip = L - 1, (L - 1) * (L - 2) // 2
        # per stage item (sequence si, helicity pattern hm) and operand split:
        # the object indices of the sub-currents with their signs, and for the
        # two-current splits the table offsets of the two momenta, packed as
        #   pairs:   off1 | off2 << 9 | neg << 18 | p1 << 32 | p2 << 48
        #   triples: off1 | off2 << 9 | off3 << 18 | neg << 27
        # where neg is the sign of the product of the sub-current signs: the
        # three- and four-gluon vertices are linear in each sub-current, so
        # the split's contribution carries that product once
        px, tx = [], []
        for si, sq in enumerate(seqs):
            for hm in range(1 << L):
                for k in range(1, L):
                    p1, p2 = sq[:k], sq[k:]
                    b1, s1, _ = co.obj(p1)
                    b2, s2, _ = co.obj(p2)
                    o1 = b1 + pext_py(hm, posmask(p1, sq))
                    o2 = b2 + pext_py(hm, posmask(p2, sq))
                    P1, P2 = lay.P[mask(p1)], lay.P[mask(p2)]
                    assert o1 < 512 and o2 < 512 and P1 < 65536 and P2 < 65536
                    px.append(o1 | o2 << 9 | ((s1 * s2) < 0) << 18 | P1 << 32 | P2 << 48)
                for a in range(1, L):
                    for b in range(a + 1, L):
                        q1, q2, q3 = sq[:a], sq[a:b], sq[b:]
                        ob = [co.obj(q) for q in (q1, q2, q3)]
                        offs = [ob[i][0] + pext_py(hm, posmask(q, sq)) for i, q in enumerate((q1, q2, q3))]
                        assert max(offs) < 512
                        tx.append(offs[0] | offs[1] << 9 | offs[2] << 18
                                  | ((ob[0][1] * ob[1][1] * ob[2][1]) < 0) << 27)
        tables.append(f"static constexpr unsigned long long GJ{n}_L{L}_PAIRX[{len(px)}] = "
                      f"{{{', '.join(f'{v}ull' for v in px)}}};")
        if tx:
            tables.append(f"static constexpr unsigned int GJ{n}_L{L}_TRIPX[{len(tx)}] = "
                          f"{{{', '.join(f'{v}u' for v in tx)}}};")
        tables.append(f"static constexpr short GJ{n}_L{L}_NINV[{len(ni)}] = {{{', '.join(ni)}}};")
        tables.append(f"static constexpr int GJ{n}_L{L}_BASE[{len(bs)}] = {{{', '.join(bs)}}};")
    pairs = co.pairs
    if pairs:
        pc, pjb, pjs, pjm, pkv = [], [], [], [], []
        for (c, d) in pairs:
            b, sg, cs = co.obj((c, d))
            pc.append(f"{c}, {d}")
            pjb.append(str(b))
            pjs.append(str(sg))
            # helicity pattern of j(cd) over sorted {c, d}: bit order by label
            pjm.append("1" if c < d else "0")
            pkv.append(str(lay.Kv[(1 << c) | (1 << d)]))
        tables.append(f"static constexpr signed char V2_{n}_CD[{2 * len(pairs)}] = {{{', '.join(pc)}}};")
        tables.append(f"static constexpr int V2_{n}_JB[{len(pairs)}] = {{{', '.join(pjb)}}};")
        tables.append(f"static constexpr signed char V2_{n}_JS[{len(pairs)}] = {{{', '.join(pjs)}}};")
        tables.append(f"static constexpr signed char V2_{n}_CLOW[{len(pairs)}] = {{{', '.join(pjm)}}};")
        tables.append(f"static constexpr short V2_{n}_KV[{len(pairs)}] = {{{', '.join(pkv)}}};")
    kt_off = ", ".join(str(lay.K1[g]) for g in range(n))
    kv_off = ", ".join(str(lay.Kv[1 << g]) for g in range(n))
    tables.append(f"static constexpr short KT1_{n}[{n}] = {{{kt_off}}};")
    tables.append(f"static constexpr short KV1_{n}[{n}] = {{{kv_off}}};")

    # ---- stages ----
    w("    constexpr int CW = 16 / (int)sizeof(T);")
    w("    const double mtd = mt;")
    w("    // level 1 (the polarisation vectors j(g; h) = eps_g(h)) is written by the table fill")
    for L in range(2, n + 1):
        nseq = len(co.levels[L])
        npair, ntrip = L - 1, (L - 1) * (L - 2) // 2
        flops_stage += nseq * (1 << L) * (npair * 51 + ntrip * 49 + 4)
        w(f"    // level {L}: {nseq} canonical sequences x {1 << L} helicity patterns")
        w(f"    for (int it = lane; it < {nseq << L}; it += nl) {{")
        w(f"        const int si = it >> {L}, hm = it & {(1 << L) - 1};")
        w("        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;")
        w("#pragma unroll")
        w(f"        for (int k = 0; k < {npair}; ++k) {{")
        w(f"            const unsigned long long sp = GJ{n}_L{L}_PAIRX[it * {npair} + k];")
        w("            const unsigned lo = (unsigned)sp, hi = (unsigned)(sp >> 32);")
        w(f"            const T* q1 = al16(obj + {co.gj} + CW * (int)(lo & 511u));")
        w(f"            const T* q2 = al16(obj + {co.gj} + CW * (int)((lo >> 9) & 511u));")
        w("            const T g = (lo >> 18) & 1u ? (T)-1 : (T)1;")
        w("            T j1[4], j2[4];")
        w(f"            ld4s<COOP_NGJ_NG{n}>(q1, j1); ld4s<COOP_NGJ_NG{n}>(q2, j2);")
        w("            const T* p1 = tab + (hi & 0xffffu); const T* p2 = tab + (hi >> 16);")
        w("            const T P1[4] = {(T)p1[0], (T)p1[1], (T)p1[2], (T)p1[3]};")
        w("            const T P2[4] = {(T)p2[0], (T)p2[1], (T)p2[2], (T)p2[3]};")
        w("            const T c1 = (T)2 * (P1[0] * j2[0] - P1[1] * j2[1] - P1[2] * j2[2] - P1[3] * j2[3]);")
        w("            const T c2 = (T)2 * (P2[0] * j1[0] - P2[1] * j1[1] - P2[2] * j1[2] - P2[3] * j1[3]);")
        w("            const T c12 = j1[0] * j2[0] - j1[1] * j2[1] - j1[2] * j2[2] - j1[3] * j2[3];")
        for mu in range(4):
            w(f"            a{mu} += g * (j1[{mu}] * c1 - j2[{mu}] * c2 + c12 * (P2[{mu}] - P1[{mu}]));")
        w("        }")
        if ntrip:
            w("#pragma unroll")
            w(f"        for (int k = 0; k < {ntrip}; ++k) {{")
            w(f"            const unsigned tp = GJ{n}_L{L}_TRIPX[it * {ntrip} + k];")
            w(f"            const T* q1 = al16(obj + {co.gj} + CW * (int)(tp & 511u));")
            w(f"            const T* q2 = al16(obj + {co.gj} + CW * (int)((tp >> 9) & 511u));")
            w(f"            const T* q3 = al16(obj + {co.gj} + CW * (int)((tp >> 18) & 511u));")
            w("            const T g = (tp >> 27) & 1u ? (T)-1 : (T)1;")
            w("            T j1[4], j2[4], j3[4];")
            w(f"            ld4s<COOP_NGJ_NG{n}>(q1, j1); ld4s<COOP_NGJ_NG{n}>(q2, j2); "
              f"ld4s<COOP_NGJ_NG{n}>(q3, j3);")
            w("            const T d23 = j2[0] * j3[0] - j2[1] * j3[1] - j2[2] * j3[2] - j2[3] * j3[3];")
            w("            const T d13 = j1[0] * j3[0] - j1[1] * j3[1] - j1[2] * j3[2] - j1[3] * j3[3];")
            w("            const T d12 = j1[0] * j2[0] - j1[1] * j2[1] - j1[2] * j2[2] - j1[3] * j2[3];")
            for mu in range(4):
                w(f"            a{mu} += g * (j1[{mu}] * d23 - (T)2 * j2[{mu}] * d13 + j3[{mu}] * d12);")
            w("        }")
        w(f"        const T f = (T)tab[GJ{n}_L{L}_NINV[si]];")
        w(f"        T* o = al16(obj + {co.gj} + CW * (GJ{n}_L{L}_BASE[si] + hm));")
        w(f"        st4s<COOP_NGJ_NG{n}>(o, a0 * f, a1 * f, a2 * f, a3 * f);")
        w("    }")
        w(f"//@@END L{L}")
    # top line from the top side: Ubar(a; s_t, h_a)
    flops_stage += 4 * n * (50 + 80) + 4 * n * (42 + 80)
    w("    // Ubar(a; s_t, h) = -[ubar gamma.eps_a] (K-slash + m) / D,   V(d; s_tbar, h) = -(K'-slash + m) [gamma.eps_d v] / D'")
    w(f"    for (int it = lane; it < {8 * n}; it += nl) {{")
    w(f"        const int side = it >= {4 * n}, r = it - side * {4 * n};")
    w("        const int g = r >> 2, sp = (r >> 1) & 1, h = r & 1;")
    w(f"        T e[4];")
    w(f"        ld4s<COOP_NGJ_NG{n}>(al16(obj + {co.gj} + CW * (2 * g + h)), e);")
    w(f"        const T* q = tab + (side ? {lay.v} : {lay.ub}) + 8 * sp;")
    w("        cplx<T> x[4];")
    w("        for (int i = 0; i < 4; ++i) x[i] = cplx<T>((T)q[2 * i], (T)q[2 * i + 1]);")
    w(f"        const T* k = tab + (side ? KV1_{n}[g] : KT1_{n}[g]);")
    w("        const T Kc[4] = {(T)k[0], (T)k[1], (T)k[2], (T)k[3]};")
    w("        cplx<T> out[4];")
    w("        if (!side) {")
    w("            cplx<T> s0 = cplx<T>(0, 0), s1 = cplx<T>(0, 0), s2 = cplx<T>(0, 0), s3 = cplx<T>(0, 0);")
    w("            rowslash_acc(x, e, s0, s1, s2, s3);")
    w("            rowprop(s0, s1, s2, s3, Kc, (T)mtd, (T)k[4], (T)k[5], out);")
    w("        } else {")
    w("            cplx<T> W[4] = {cplx<T>(0, 0), cplx<T>(0, 0), cplx<T>(0, 0), cplx<T>(0, 0)};")
    w("            slashcol_acc(e, x, W);")
    w("            colprop(W, Kc, (T)mtd, (T)k[4], (T)k[5], out);")
    w("        }")
    w(f"        stspins<COOP_NU1_NG{n}>(al16(obj + (side ? {co.v1} : {co.u1}) + CW * r), out);")
    w("    }")
    w("//@@END U1V1")
    if pairs:
        flops_stage += 8 * len(pairs) * (42 + 42 + 80)
        w("    // V(cd; s_tbar, h_c, h_d) = -(K'-slash + m) [gamma.eps_c V(d) + gamma.j(cd) v] / D'")
        w(f"    for (int it = lane; it < {8 * len(pairs)}; it += nl) {{")
        w("        const int pi = it >> 3, sb = (it >> 2) & 1, hc = (it >> 1) & 1, hd = it & 1;")
        w(f"        const int c = V2_{n}_CD[2 * pi], d = V2_{n}_CD[2 * pi + 1];")
        w("        T ec[4];")
        w(f"        ld4s<COOP_NGJ_NG{n}>(al16(obj + {co.gj} + CW * (2 * c + hc)), ec);")
        w("        cplx<T> y[4];")
        w(f"        ldspins<COOP_NU1_NG{n}>(al16(obj + {co.v1} + CW * (4 * d + 2 * sb + hd)), y);")
        w("        cplx<T> W[4] = {cplx<T>(0, 0), cplx<T>(0, 0), cplx<T>(0, 0), cplx<T>(0, 0)};")
        w("        slashcol_acc(ec, y, W);")
        w(f"        const int hm = V2_{n}_CLOW[pi] ? (hc | (hd << 1)) : (hd | (hc << 1));")
        w(f"        const T gs = (T)V2_{n}_JS[pi];")
        w("        T jcd[4];")
        w(f"        ld4s<COOP_NGJ_NG{n}>(al16(obj + {co.gj} + CW * (V2_{n}_JB[pi] + hm)), jcd);")
        w("        for (int i = 0; i < 4; ++i) jcd[i] *= gs;")
        w(f"        const T* qv = tab + {lay.v} + 8 * sb;")
        w("        cplx<T> x[4];")
        w("        for (int i = 0; i < 4; ++i) x[i] = cplx<T>((T)qv[2 * i], (T)qv[2 * i + 1]);")
        w("        slashcol_acc(jcd, x, W);")
        w(f"        const T* k = tab + V2_{n}_KV[pi];")
        w("        const T Kc[4] = {(T)k[0], (T)k[1], (T)k[2], (T)k[3]};")
        w("        cplx<T> out[4];")
        w("        colprop(W, Kc, (T)mtd, (T)k[4], (T)k[5], out);")
        w(f"        stspins<COOP_NV2_NG{n}>(al16(obj + {co.v2} + CW * it), out);")
        w("    }")
        w("//@@END V2")
    # Order of the stages: level 2 and the single-gluon spinor chains depend
    # only on level 1, level 3 and the two-gluon chains only on those, each
    # further level on the one before; a wave synchronisation separates only
    # dependent groups.
    chunks, buf = {}, []
    for line in L_:
        if line.startswith("//@@END "):
            chunks[line[len("//@@END "):]] = buf
            buf = []
        else:
            buf.append(line)
    # the lines ahead of level 2 (shared declarations) open the function
    rest = chunks["L2"]
    cut = next(i for i, line in enumerate(rest) if line.startswith("    // level 2"))
    pre, chunks["L2"] = rest[:cut], rest[cut:]
    order = [["L2", "U1V1"], ["L3"] + (["V2"] if "V2" in chunks else [])] + \
        [[f"L{k}"] for k in range(4, n + 1)]
    out = list(pre)
    for grp in order:
        for name in grp:
            out.extend(chunks.pop(name))
        out.append("    wave_sync();")
    assert not chunks, chunks.keys()
    stages = "\n".join(out)

    # ---- amplitude phase: one lane per helicity configuration ----
    # A(sigma) = sum over the blocks beta of sigma that contain its second
    # gluon of  Xbar gamma.j(beta) Y,  Xbar in {ubar, Ubar(sigma_1)},
    # Y in {v, V(last), V(last two)}.  Each bilinear d^mu = Xbar gamma^mu Y is
    # formed once, contracted with the gluon currents it meets and scattered
    # (with the reflection signs) into the amplitude accumulators; only the
    # accumulators stay live.
    A = []
    a = A.append
    # an opaque copy of the helicity index: offsets derived from it are then
    # recomputed per event instead of being hoisted out of the event loop
    a('    asm volatile("" : "+v"(hel));')
    a("    constexpr int CW = 16 / (int)sizeof(T);")
    a("    const int sT = hel & 1, sB = (hel >> 1) & 1, hg = hel >> 2;")
    hel_flops = 0
    lex = {sq: i for i, sq in enumerate(perms)}
    nperm_ = len(perms)
    # Each accumulator holds sig[k] * A_k, with the sign fixed by its first
    # contribution (written, not added to zero); the colour sum absorbs the
    # signs into its coefficients.
    a(f"    T Ar[{nperm_}], Ai[{nperm_}];")
    acc_decl = len(A) - 1
    sig = {}

    def hexpr(block):
        srt = sorted(block)
        return " | ".join(f"(((hg >> {g}) & 1) << {i})" for i, g in enumerate(srt))

    def gj_ptr(block, ob):
        b, sg, cs = co.obj(block)
        return f"al16({ob} + {co.gj} + CW * ({b} + ({hexpr(cs)})))", sg

    def row_load(X, nm, ob):
        if not X:
            tb = ob.replace("ob", "tb")
            return nm, [f"    cplx<T> {nm}[4];", f"    ldspin(al16({tb} + {lay.ub} + 8 * sT), {nm});"]
        return nm, [f"    cplx<T> {nm}[4];",
                    f"    ldspins<COOP_NU1_NG{n}>(al16({ob} + {co.u1} + CW * (4 * {X[0]} + 2 * sT + "
                    f"((hg >> {X[0]}) & 1))), {nm});"]

    def col_load(Y, nm, ob):
        if not Y:
            tb = ob.replace("ob", "tb")
            return nm, [f"    cplx<T> {nm}[4];", f"    ldspin(al16({tb} + {lay.v} + 8 * sB), {nm});"]
        if len(Y) == 1:
            d = Y[0]
            idx = f"{co.v1} + CW * (4 * {d} + 2 * sB + ((hg >> {d}) & 1))"
            ns = f"COOP_NU1_NG{n}"
        else:
            c, d = Y
            pi = co.pairs.index((c, d))
            idx = f"{co.v2} + CW * ({8 * pi} + 4 * sB + 2 * ((hg >> {c}) & 1) + ((hg >> {d}) & 1))"
            ns = f"COOP_NV2_NG{n}"
        return nm, [f"    cplx<T> {nm}[4];", f"    ldspins<{ns}>(al16({ob} + {idx}), {nm});"]

    # group the terms by bilinear: key (X, Y) -> list of (beta, ordering)
    groups = {}
    for sg in perms:
        for i in (0, 1):
            for j in range(2, n + 1):
                X, beta, Y = sg[:i], sg[i:j], sg[j:]
                groups.setdefault((X, Y), []).append((beta, sg))
    # Y-major order so that a loaded V is used by all its bilinears in a row
    keys = sorted(groups, key=lambda k: (len(k[1]), k[1], k[0]))
    # Each group's LDS reads are issued one group ahead: group g + 1's reads
    # follow an opaque zero produced just before group g's arithmetic, so they
    # overlap it, while no read can be hoisted further up (each hoisted read
    # would hold registers).
    loads, computes = [], []
    for gi, (X, Y) in enumerate(keys):
        ob = f"ob{gi}"
        L = [f"    int z{gi} = 0;", f'    asm volatile("" : "+s"(z{gi}));',
             f"    const T* {ob} = (const T*)((const char*)obj + z{gi});"]
        if not X or not Y:
            L.append(f"    const T* tb{gi} = (const T*)((const char*)tab + z{gi});")
        r, lr = row_load(X, f"xr{gi}", ob)
        c, lc = col_load(Y, f"yc{gi}", ob)
        L += lr + lc
        # the currents are read at the start of the group itself (behind a
        # second opaque zero), in the shadow of the bilinear
        Cc = ["    {", "        int y = 0;", '        asm volatile("" : "+s"(y));',
              "        const T* oc = (const T*)((const char*)obj + y);"]
        cur_at = len(Cc)
        Cc += ["        cplx<T> d[4];", f"        bilinear({r}, {c}, d);"]
        hel_flops += 64
        # distinct currents (up to reflection) met by this bilinear
        byc = {}
        for (beta, sg) in groups[(X, Y)]:
            b, sgn, cs = co.obj(beta)
            byc.setdefault(cs, []).append((sgn, sg))
        touched = []
        cur_loads = []
        for ci, (cs, uses) in enumerate(byc.items()):
            ptr, _ = gj_ptr(cs, "oc")
            jn = f"j{ci}"
            Cc += [f"        T {jn}[4];", f"        ld4s<COOP_NGJ_NG{n}>({ptr}, {jn});"]
            if len(uses) == 1:
                # one ordering meets this current: multiply-add into its accumulator
                sgn, sg = uses[0]
                k = lex[sg]
                if k not in sig:
                    sig[k] = sgn
                    Cc.append(f"        cdot_set({jn}, d, Ar[{k}], Ai[{k}]);")
                    hel_flops += 14
                else:
                    Cc.append(f"        cdot_fma<{sgn * sig[k]}>({jn}, d, Ar[{k}], Ai[{k}]);")
                    hel_flops += 16
                if k not in touched:
                    touched.append(k)
                continue
            Cc.append("        {")
            Cc.append("            T sr, si;")
            Cc.append(f"            cdot_set({jn}, d, sr, si);")
            hel_flops += 14
            for (sgn, sg) in uses:
                k = lex[sg]
                if k not in sig:
                    sig[k] = sgn
                    Cc.append(f"            Ar[{k}] = sr; Ai[{k}] = si;")
                else:
                    op = "+=" if sgn * sig[k] > 0 else "-="
                    Cc.append(f"            Ar[{k}] {op} sr; Ai[{k}] {op} si;")
                    hel_flops += 2
                if k not in touched:
                    touched.append(k)
            Cc.append("        }")
        # the accumulators this group updated pass through an opaque point
        # before the next group starts, so that the group's arithmetic is not
        # deferred to the colour sum with its operands held in registers
        touched.sort()
        for c0 in range(0, len(touched), 4):
            ops = ", ".join(f'"+v"(Ar[{k}]), "+v"(Ai[{k}])' for k in touched[c0:c0 + 4])
            Cc.append(f'        asm volatile("" : {ops});')
        Cc.append("    }")
        Cc[cur_at:cur_at] = cur_loads
        loads.append(L)
        computes.append(Cc)
    # two orders of the same statements: spinor reads one group ahead, or
    # each group's reads at its own start (fewer live registers)
    head = list(A)
    A_seq = list(head)
    A.extend(loads[0])
    for gi in range(len(keys)):
        if gi + 1 < len(keys):
            A.extend(loads[gi + 1])
        A.extend(computes[gi])
    for gi in range(len(keys)):
        A_seq.extend(loads[gi])
        A_seq.extend(computes[gi])
    tail_start = len(A)
    untouched = [k for k in range(nperm_) if k not in sig]
    if untouched:
        A[acc_decl] += " " + " ".join(f"Ar[{k}] = 0; Ai[{k}] = 0;" for k in untouched)
        for k in untouched:
            sig[k] = 1
    # colour sum: sum_s K_ss |A_s|^2 + 2 sum_{t<s} K_st Re(conj(A_s) A_t), on
    # the accumulators (sig[s] A_s): K_st enters as sig[s] sig[t] K_st.
    # Leading colour (COL = 1): c_LC sum_s |A_s|^2, where the signs drop out.
    a("    T me;")
    a("    if constexpr (COL == 0) {")
    full_flops = 0
    for sidx in range(nperm_):
        a("    {")
        a(f"        T tr = {K[sidx][sidx]} * Ar[{sidx}], ti = {K[sidx][sidx]} * Ai[{sidx}];")
        full_flops += 2
        for t in range(sidx):
            if K[sidx][t]:
                kst = 2 * K[sidx][t] * sig[sidx] * sig[t]
                a(f"        tr += (T)({kst}) * Ar[{t}]; ti += (T)({kst}) * Ai[{t}];")
                full_flops += 4
        if sidx == 0:
            a(f"        me = Ar[{sidx}] * tr;")
            full_flops += 1
        else:
            a(f"        me += Ar[{sidx}] * tr;")
            full_flops += 2
        a(f"        me += Ai[{sidx}] * ti;")
        full_flops += 2
        a("    }")
    a("    } else if constexpr (COL == 1) {")
    a("        T s2 = Ar[0] * Ar[0];")
    a("        s2 += Ai[0] * Ai[0];")
    lc_flops = 3
    for sidx in range(1, nperm_):
        a(f"        s2 += Ar[{sidx}] * Ar[{sidx}];")
        a(f"        s2 += Ai[{sidx}] * Ai[{sidx}];")
        lc_flops += 4
    a(f"        me = (T){lc_numerator(n, den)} * s2;")
    lc_flops += 1
    # Monte Carlo over colours (COL = 2): the event's colour factors cf
    # (re, im per ordering) dress the amplitudes, M = sum_s c_s A_s; N_cfg |M|^2
    # over the common denominator keeps the final division of the full sum
    a("    } else if constexpr (COL == 2) {")
    a("        T mr = 0, mi = 0;")
    mc_flops = 0
    for sidx in range(nperm_):
        op = "+=" if sig[sidx] > 0 else "-="
        a(f"        {{ const T cr = cf[{2 * sidx}], ci = cf[{2 * sidx + 1}];")
        a(f"          mr {op} cr * Ar[{sidx}] - ci * Ai[{sidx}]; mi {op} cr * Ai[{sidx}] + ci * Ar[{sidx}]; }}")
        mc_flops += 8
    a(f"        me = (T){colour_count(n) * den} * (mr * mr + mi * mi);")
    mc_flops += 4
    # Monte Carlo over colour flows (COL = 3): real factors cf[s] and the
    # event's scale T / W_f in cf[n!]: (T / W_f) |M|^2
    a("    } else {")
    a("        T mr = 0, mi = 0;")
    flow_flops = 0
    for sidx in range(nperm_):
        op = "+=" if sig[sidx] > 0 else "-="
        a(f"        mr {op} cf[{sidx}] * Ar[{sidx}]; mi {op} cf[{sidx}] * Ai[{sidx}];")
        flow_flops += 4
    a(f"        me = (T){den} * cf[{nperm_}] * (mr * mr + mi * mi);")
    flow_flops += 5
    a("    }")
    A_seq[acc_decl] = A[acc_decl]
    A_seq.extend(A[tail_start:])
    amp = ("\n".join(A), "\n".join(A_seq))
    return "\n".join(tables), stages, amp, flops_stage, (hel_flops + full_flops, hel_flops + lc_flops,
                                                          hel_flops + mc_flops, hel_flops + flow_flops)


def generate_coop(n):
    perms, K, den = colour_matrix(n)
    tl = CoopTable(n)
    co = CoopLayout(n)
    tables, stages, amp, fst, (fhel, fhel_lc, fhel_mc, fhel_flow) = emit_coop(n, tl, co, K, den, perms)
    fill = emit_coop_fill(n, tl, co)
    global _COOP_COUNT
    _COOP_COUNT = {"stages": fst, "per_helicity": fhel, "per_helicity_lc": fhel_lc, "per_helicity_mc": fhel_mc,
                   "per_helicity_flow": fhel_flow,
                   "object_store": co.size, "table": tl.size, "momentum_only": tl.mom_flops()}
    gm = gell_mann_half()
    gm_re = ", ".join(repr(v.real) for m in gm for row in m for v in row)
    gm_im = ", ".join(repr(v.imag) for m in gm for row in m for v in row)
    perm_tab = ", ".join(str(g) for sg in perms for g in sg)
    flows = flow_table(n, perms)
    flow_tab = ", ".join(f"{w}u" for w, _ in flows)
    cum = [0]
    for _, wt in flows:
        cum.append(cum[-1] + wt)
    flow_cum = ", ".join(f"{c}ull" for c in cum)
    # guide table: for slice j of [0, T), the flow holding ceil(j T / G); the
    # flow holding u lies at or after GUIDE[u G / T] (Chen and Asau's method)
    n_guide = 1 << (len(flows) - 1).bit_length()
    guide = [bisect.bisect_right(cum, -(-j * cum[-1] // n_guide)) - 1 for j in range(n_guide)]
    for u in list(range(0, cum[-1], max(1, cum[-1] // 5000))) + [cum[-1] - 1] + cum[1:-1]:
        f = guide[u * n_guide // cum[-1]]
        while cum[f + 1] <= u:
            f += 1
        assert f == bisect.bisect_right(cum, u) - 1
    flow_guide = ", ".join(str(g) for g in guide)
    return f"""
// ---- cooperative evaluation (helicity-recycled objects in LDS) ----
// Table: {tl.size} T per event; object store: {co.size} T per event.  Table
// flops per event: {tl.mom_flops()}; stage flops per event: {fst}; per
// helicity lane: {fhel} ({fhel_lc} in leading colour).
static constexpr int COOP_TABLE_NG{n} = {tl.size};
static constexpr int COOP_OBJ_NG{n} = {co.size};
// objects per region of the chunk-major object store: currents, Ubar and V
// chains, two-gluon V chains
static constexpr int COOP_NGJ_NG{n} = {co.n_gj};
static constexpr int COOP_NU1_NG{n} = {co.n_u1};
static constexpr int COOP_NV2_NG{n} = {co.n_v2};
static constexpr int COOP_FLOPS_STAGES_NG{n} = {fst};
static constexpr int COOP_FLOPS_HEL_NG{n} = {fhel};
{tables}

// Per-event table of momentum-only quantities (type T) and the level-1
// gluon currents in the object store, written by the lanes of one event;
// the caller synchronises the wave afterwards.  mom: t[4], tbar[4], final
// gluons[4 each]; eb: beam energy sqrt(s_hat)/2; mt: top mass; mw: m_t Gamma_t.
// NS: objects of the current region `obj` points into (the object store's,
// or a smaller staging area that holds only the level-1 currents).
template <typename T, int NS = COOP_NGJ_NG{n}>
__device__ __forceinline__ void fill_table_coop_ng{n}(const double* __restrict__ mom, double eb, double mt, double mw,
                                                     T* __restrict__ tab, T* __restrict__ obj, int lane)
{{
{fill}
}}

// Builds the event's object store `obj` from its table: lanes 0 .. nl-1 of
// the wave serve this event; every level ends with a wave synchronisation.
template <typename T>
__device__ __forceinline__ void coop_stages_ng{n}(const T* __restrict__ tab, T* __restrict__ obj, double mt,
                                                 int lane, int nl)
{{
{stages}
}}

// Colour-summed |M|^2 (g_s = 1) of helicity configuration `hel` from the
// object store: meet-in-the-middle at the vertex that carries the second
// gluon of each colour ordering, A = sum Xbar gamma.j(block) Y.  COL = 0:
// full colour matrix; COL = 1: leading colour, {lc_numerator(n, den)}/{den} times the identity;
// COL = 2: one sampled colour assignment with factors cf (Monte Carlo over colours).
template <typename T, int COL>
__device__ __forceinline__ double coop_me2_ng{n}_ahead(const T* __restrict__ tab, const T* __restrict__ obj,
                                                      const T* __restrict__ cf, int hel)
{{
{amp[0]}
    return (double)me / COLOUR_DEN_NG{n};
}}

template <typename T, int COL>
__device__ __forceinline__ double coop_me2_ng{n}_inplace(const T* __restrict__ tab, const T* __restrict__ obj,
                                                        const T* __restrict__ cf, int hel)
{{
{amp[1]}
    return (double)me / COLOUR_DEN_NG{n};
}}

// The spinor reads go one group ahead where the registers allow it without
// spilling or losing occupancy: FP64 with four final-state partons.
template <typename T, int COL>
__device__ __forceinline__ double coop_me2_ng{n}(const T* __restrict__ tab, const T* __restrict__ obj,
                                                const T* __restrict__ cf, int hel)
{{
    if constexpr (sizeof(T) == 8 && {n} == 4)
        return coop_me2_ng{n}_ahead<T, COL>(tab, obj, cf, hel);
    else
        return coop_me2_ng{n}_inplace<T, COL>(tab, obj, cf, hel);
}}

// Monte Carlo over colours: the colour assignment of event `event` -- Philox
// block 0x80000001 of its counter, cfg = ((k >> 16) N_cfg) >> 37 with the
// 53-bit integer k of the first word pair, N_cfg = {colour_count(n)} -- and, on lanes
// 0 .. {len(perms) - 1}, the factor (T^(a_s1) .. T^(a_sn))_(i j) of ordering s into
// cf[2 s], cf[2 s + 1].  Decoding: j = cfg mod 3, i = (cfg / 3) mod 3, gluon g's
// adjoint index (cfg / 9 / 8^g) mod 8.
static constexpr int64_t COLOUR_CFG_NG{n} = {colour_count(n)};
static constexpr double GM_RE_NG{n}[72] = {{{gm_re}}};
static constexpr double GM_IM_NG{n}[72] = {{{gm_im}}};
static constexpr signed char PERM_NG{n}[{len(perms) * n}] = {{{perm_tab}}};
template <typename T>
__device__ __forceinline__ void colour_factors_ng{n}(uint64_t event, uint64_t seed, uint32_t iter,
                                                    T* __restrict__ cf, int lane)
{{
    if (lane >= {len(perms)})
        return;
    uint32_t r[4];
    philox4x32_10((uint32_t)event, (uint32_t)(event >> 32), iter, 0x80000001u, (uint32_t)seed,
                  (uint32_t)(seed >> 32), r);
    const uint64_t k = ((((uint64_t)r[0]) << 32) | (uint64_t)r[1]) >> 11;
    const uint64_t cfg = ((k >> 16) * (uint64_t)COLOUR_CFG_NG{n}) >> 37;
    const int cj = (int)(cfg % 3), ci = (int)((cfg / 3) % 3);
    const uint64_t adj = cfg / 9;
    double rr[3], ri[3];
    for (int q = 0; q < 3; ++q) {{
        rr[q] = q == ci ? 1.0 : 0.0;
        ri[q] = 0.0;
    }}
    for (int step = 0; step < {n}; ++step) {{
        const int g = PERM_NG{n}[lane * {n} + step];
        const int a = (int)((adj >> (3 * g)) & 7u);
        const double* tr = GM_RE_NG{n} + 9 * a;
        const double* ti = GM_IM_NG{n} + 9 * a;
        double nr[3], ni[3];
        for (int q = 0; q < 3; ++q) {{
            nr[q] = rr[0] * tr[q] - ri[0] * ti[q] + rr[1] * tr[3 + q] - ri[1] * ti[3 + q]
                  + rr[2] * tr[6 + q] - ri[2] * ti[6 + q];
            ni[q] = rr[0] * ti[q] + ri[0] * tr[q] + rr[1] * ti[3 + q] + ri[1] * tr[3 + q]
                  + rr[2] * ti[6 + q] + ri[2] * tr[6 + q];
        }}
        for (int q = 0; q < 3; ++q) {{
            rr[q] = nr[q];
            ri[q] = ni[q];
        }}
    }}
    const double cr = cj == 0 ? rr[0] : (cj == 1 ? rr[1] : rr[2]);
    const double cim = cj == 0 ? ri[0] : (cj == 1 ? ri[1] : ri[2]);
    cf[2 * lane] = (T)cr;
    cf[2 * lane + 1] = (T)cim;
}}

// Monte Carlo over colour flows: {len(flows)} flows with integer weights
// W_f = 18^n sum_s c_s^2, cumulative sums C_f, total T = {cum[-1]}.  The event's
// flow is the f with C_f <= u < C_(f+1), u = floor(k T / 2^53), k the 53-bit
// integer of the first word pair of Philox block 0x80000001; its word
// (j | i << 2 | a_g << (4 + 4 g) | b_g << (6 + 4 g): gluon g has colour a_g and
// anticolour b_g, state (e_ab - delta_ab / 3) / sqrt 2) gives, on lanes
// 0 .. {len(perms) - 1}, the real factor of ordering s into cf[s]: the colour
// line from i through the gluons of the ordering, where an off-diagonal pair
// needs the current colour a and moves it to b, a diagonal pair keeps it with
// factor 2/3 (same colour) or -1/3, and the line must end on j.  Lane 0 also
// stores the scale T / W_f into cf[{len(perms)}].  The search for f starts at
// FLOW_GUIDE_NG{n}[u G / T], G = {n_guide}, the flow holding ceil(j T / G) for
// slice j, and steps forward while C_(f+1) <= u; it ends because C_N = T > u.
static constexpr int64_t FLOW_COUNT_NG{n} = {len(flows)};
static constexpr uint32_t FLOW_NG{n}[{len(flows)}] = {{{flow_tab}}};
static constexpr uint64_t FLOW_CUM_NG{n}[{len(flows) + 1}] = {{{flow_cum}}};
static constexpr uint16_t FLOW_GUIDE_NG{n}[{n_guide}] = {{{flow_guide}}};
template <typename T>
__device__ __forceinline__ void flow_factors_ng{n}(uint64_t event, uint64_t seed, uint32_t iter,
                                                  T* __restrict__ cf, int lane)
{{
    if (lane >= {len(perms)})
        return;
    uint32_t r[4];
    philox4x32_10((uint32_t)event, (uint32_t)(event >> 32), iter, 0x80000001u, (uint32_t)seed,
                  (uint32_t)(seed >> 32), r);
    const uint64_t k = ((((uint64_t)r[0]) << 32) | (uint64_t)r[1]) >> 11;
    constexpr uint64_t kTotal = FLOW_CUM_NG{n}[FLOW_COUNT_NG{n}];
    const uint64_t u = __umul64hi(k << 11, kTotal);
    int lo = FLOW_GUIDE_NG{n}[u * {n_guide}ull / kTotal];
    while (FLOW_CUM_NG{n}[lo + 1] <= u)
        ++lo;
    const uint32_t f = FLOW_NG{n}[lo];
    if (lane == 0)
        cf[{len(perms)}] = (T)((double)FLOW_CUM_NG{n}[FLOW_COUNT_NG{n}]
                               / (double)(FLOW_CUM_NG{n}[lo + 1] - FLOW_CUM_NG{n}[lo]));
    uint32_t col = (f >> 2) & 3u;
    bool alive = true;
    double v = {repr(2.0 ** (-n / 2))};
    for (int step = 0; step < {n}; ++step) {{
        const int g = PERM_NG{n}[lane * {n} + step];
        const uint32_t a = (f >> (4 + 4 * g)) & 3u, b = (f >> (6 + 4 * g)) & 3u;
        if (a != b) {{
            alive = alive && col == a;
            col = b;
        }} else {{
            v *= col == a ? {repr(2.0 / 3.0)} : {repr(-1.0 / 3.0)};
        }}
    }}
    cf[lane] = (T)(alive && col == (f & 3u) ? v : 0.0);
}}
"""


_LAST_COUNT = None
_COOP_COUNT = None


def _helpers():
    import types
    return types.SimpleNamespace(_contract=_contract, CoopTable=CoopTable, emit_coop_fill=emit_coop_fill,
                                 gell_mann_half=gell_mann_half)


def _qqbar():
    """The q qbar -> t tbar g g colour tables (gen_qqbar.py next to this file)."""
    import importlib.util
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gen_qqbar.py")
    spec = importlib.util.spec_from_file_location("gen_qqbar", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _ttggg():
    """The five-gluon generator (gen_ttggg.py next to this file)."""
    import importlib.util
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gen_ttggg.py")
    spec = importlib.util.spec_from_file_location("gen_ttggg", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def flop_count(n, colour="full"):
    """Algorithmic flops per event of the |M|^2 code the kernels run for n
    gluons: the momentum table, plus either 2^(n+2) independent helicity
    evaluations (n = 2) or the shared object stages and the per-helicity
    meet-in-the-middle contractions (n >= 3).  colour = "leading" counts the
    leading-colour sum in place of the full colour matrix."""
    assert colour in ("full", "leading", "sampled", "flow")
    if n == 5:
        _, c5 = _ttggg().generate_ng5(_helpers())
        nh = 1 << (n + 2)
        c = {"algorithm": "helicity-recycled objects, amplitudes to memory, colour sum on the matrix cores",
             "n_hel": nh, "n_orderings": 120, "momentum_only": c5["momentum_only"], "stages": c5["stages"],
             "per_lane": c5["per_lane"], "lanes": 5 * nh, "colour_per_helicity": c5["colour_per_helicity"],
             "object_store": c5["object_store"], "table_doubles": c5["table"]}
        assert colour == "full", "t tbar g g g runs with the full colour sum"
        c["amplitudes"] = c["momentum_only"] + c["stages"] + c["lanes"] * c["per_lane"]
        c["colour"] = nh * c["colour_per_helicity"]
        c["per_event"] = c["amplitudes"] + c["colour"]
        return c
    generate(n)
    c = dict(_LAST_COUNT)
    lc = colour == "leading"
    if n >= 3:
        c["algorithm"] = "helicity-recycled objects"
        c["stages"] = _COOP_COUNT["stages"]
        c["per_helicity"] = _COOP_COUNT[{"full": "per_helicity", "leading": "per_helicity_lc",
                                         "sampled": "per_helicity_mc", "flow": "per_helicity_flow"}[colour]]
        c["object_store"] = _COOP_COUNT["object_store"]
        c["per_event"] = c["momentum_only"] + c["stages"] + c["n_hel"] * c["per_helicity"]
        if colour == "sampled":
            # the event's colour factors: n steps of a complex row times a 3 x 3 matrix per ordering
            c["colour_factors"] = 36 * n * c["n_orderings"]
            c["per_event"] += c["colour_factors"]
        elif colour == "flow":
            # the event's flow factors: at most n multiplications per ordering
            c["colour_factors"] = n * c["n_orderings"]
            c["per_event"] += c["colour_factors"]
    else:
        c["algorithm"] = "independent helicities"
        c["stages"] = 0
        if lc:
            c["per_helicity"] = c["per_helicity_lc"]
        assert colour not in ("sampled", "flow"), "the Monte Carlo over colours runs for n >= 3 only"
        c["per_event"] = c["momentum_only"] + c["n_hel"] * c["per_helicity"]
    return c


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    outputs = [(f"amp_ng{n}.inc", (lambda n=n: generate(n) if n <= 4 else _ttggg().generate_ng5(_helpers())[0]))
               for n in (2, 3, 4, 5)]
    outputs.append(("qqbar_ttxgg.inc", lambda: _qqbar().generate(_helpers())))
    for name, make in outputs:
        path = os.path.join(args.out, name)
        text = make()
        old = open(path).read() if os.path.exists(path) else None
        if old != text:
            with open(path, "w") as f:
                f.write(text)


if __name__ == "__main__":
    main()
