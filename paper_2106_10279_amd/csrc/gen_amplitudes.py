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


class Emitter:
    def __init__(self, n):
        self.n = n
        self.lines = []
        self.done = set()

    def w(self, s=""):
        self.lines.append("    " + s)

    # -- momenta (double) ----------------------------------------------------
    def psum(self, m):
        key = ("P", m)
        if key in self.done:
            return f"P{m}"
        self.done.add(key)
        gl = [g for g in range(self.n) if m >> g & 1]
        for mu in range(4):
            self.w(f"const double P{m}_{mu} = " + " + ".join(f"pg[{g}][{mu}]" for g in gl) + ";")
        return f"P{m}"

    def p2(self, m):
        key = ("P2", m)
        if key not in self.done:
            self.done.add(key)
            P = self.psum(m)
            self.w(f"const T ninvP2_{m} = (T)(-1.0 / ({P}_0 * {P}_0 - {P}_1 * {P}_1 - {P}_2 * {P}_2 - {P}_3 * {P}_3));")
        return f"ninvP2_{m}"

    # -- gluon currents (real 4-vectors) ---------------------------------------
    def gcur(self, seq):
        seq = tuple(seq)
        if len(seq) == 1:
            return f"eps{seq[0]}"
        key = ("j", seq)
        if key in self.done:
            return f"j{name(seq)}"
        rev = tuple(reversed(seq))
        if ("j", rev) in self.done:
            sign = "" if (len(seq) + 1) % 2 == 0 else "-"
            self.done.add(key)
            self.w(f"const T j{name(seq)}[4] = {{{', '.join(f'{sign}j{name(rev)}[{mu}]' for mu in range(4))}}};")
            return f"j{name(seq)}"
        L = len(seq)
        subs = []
        for a in range(1, L):
            subs.append((self.gcur(seq[:a]), self.gcur(seq[a:]), mask(seq[:a]), mask(seq[a:])))
        trip = []
        for a in range(1, L):
            for b in range(a + 1, L):
                trip.append((self.gcur(seq[:a]), self.gcur(seq[a:b]), self.gcur(seq[b:])))
        for (_, _, m1, m2) in subs:
            self.psum(m1)
            self.psum(m2)
        f = self.p2(mask(seq))
        nm = f"j{name(seq)}"
        self.done.add(key)
        self.w(f"T {nm}[4];")
        self.w("{")
        self.w("    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;")
        for (j1, j2, m1, m2) in subs:
            P1, P2 = f"P{m1}", f"P{m2}"
            q1 = [f"(T)(2.0 * {P1}_{mu} + {P2}_{mu})" for mu in range(4)]
            q2 = [f"(T)({P1}_{mu} + 2.0 * {P2}_{mu})" for mu in range(4)]
            d = [f"(T)({P2}_{mu} - {P1}_{mu})" for mu in range(4)]
            self.w("    {")
            self.w(f"        const T c1 = {q1[0]} * {j2}[0] - {q1[1]} * {j2}[1] - {q1[2]} * {j2}[2] - {q1[3]} * {j2}[3];")
            self.w(f"        const T c2 = {q2[0]} * {j1}[0] - {q2[1]} * {j1}[1] - {q2[2]} * {j1}[2] - {q2[3]} * {j1}[3];")
            self.w(f"        const T c12 = {j1}[0] * {j2}[0] - {j1}[1] * {j2}[1] - {j1}[2] * {j2}[2] - {j1}[3] * {j2}[3];")
            for mu in range(4):
                self.w(f"        a{mu} += {j1}[{mu}] * c1 - {j2}[{mu}] * c2 + {d[mu]} * c12;")
            self.w("    }")
        for (j1, j2, j3) in trip:
            self.w("    {")
            self.w(f"        const T d23 = {j2}[0] * {j3}[0] - {j2}[1] * {j3}[1] - {j2}[2] * {j3}[2] - {j2}[3] * {j3}[3];")
            self.w(f"        const T d13 = {j1}[0] * {j3}[0] - {j1}[1] * {j3}[1] - {j1}[2] * {j3}[2] - {j1}[3] * {j3}[3];")
            self.w(f"        const T d12 = {j1}[0] * {j2}[0] - {j1}[1] * {j2}[1] - {j1}[2] * {j2}[2] - {j1}[3] * {j2}[3];")
            for mu in range(4):
                self.w(f"        a{mu} += {j1}[{mu}] * d23 - (T)2 * {j2}[{mu}] * d13 + {j3}[{mu}] * d12;")
            self.w("    }")
        for mu in range(4):
            self.w(f"    {nm}[{mu}] = a{mu} * {f};")
        self.w("}")
        return nm

    # -- top-line propagator factor -(1/D) -----------------------------------
    def topprop(self, m):
        key = ("D", m)
        if key not in self.done:
            self.done.add(key)
            P = self.psum(m)
            self.w(f"const double K{m}_0 = kt[0] + {P}_0, K{m}_1 = kt[1] + {P}_1, "
                   f"K{m}_2 = kt[2] + {P}_2, K{m}_3 = kt[3] + {P}_3;")
            self.w(f"T fr{m}, fi{m};")
            self.w("{")
            self.w(f"    const double re = K{m}_0 * K{m}_0 - K{m}_1 * K{m}_1 - K{m}_2 * K{m}_2 - K{m}_3 * K{m}_3 - m2;")
            self.w("    const double inv = 1.0 / (re * re + mw * mw);")
            self.w(f"    fr{m} = (T)(-re * inv);")
            self.w(f"    fi{m} = (T)(mw * inv);")
            self.w("}")
        return m

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
        self.topprop(m)
        nm = f"U{name(seq)}"
        self.done.add(key)
        self.w(f"cT {nm}[4];")
        self.w("{")
        self.w("    cT s0 = cT(0, 0), s1 = cT(0, 0), s2 = cT(0, 0), s3 = cT(0, 0);")
        for (U, j) in terms:
            # row (aL, aR) x gamma.j = (aR (j.sigmabar), aL (j.sigma))
            self.w(f"    rowslash_acc({U}, {j}, s0, s1, s2, s3);")
        self.w(f"    const T Kc[4] = {{(T)K{m}_0, (T)K{m}_1, (T)K{m}_2, (T)K{m}_3}};")
        self.w(f"    rowprop(s0, s1, s2, s3, Kc, (T)mt, fr{m}, fi{m}, {nm});")
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
        self.w(f"cT {nm}[4];")
        self.w(f"bilinear(" + U + ", v, " + nm + ");")
        return nm

    def wspin(self, g):
        key = ("W", g)
        nm = f"W{g}"
        if key not in self.done:
            self.done.add(key)
            self.w(f"cT {nm}[4];")
            self.w(f"slashcol(eps{g}, v, {nm});")
        return nm


def generate(n):
    perms, K, den = colour_matrix(n)
    e = Emitter(n)
    nperm = len(perms)
    e.w("const int sT = hel & 1, sB = (hel >> 1) & 1;")
    e.w(f"double pg[{n}][4];")
    e.w("pg[0][0] = -eb; pg[0][1] = 0.0; pg[0][2] = 0.0; pg[0][3] = -eb;")
    e.w("pg[1][0] = -eb; pg[1][1] = 0.0; pg[1][2] = 0.0; pg[1][3] = eb;")
    for g in range(2, n):
        e.w(f"for (int mu = 0; mu < 4; ++mu) pg[{g}][mu] = mom[{8 + 4 * (g - 2)} + mu];")
    e.w("const double kt[4] = {mom[0], mom[1], mom[2], mom[3]};")
    e.w("const double kb[4] = {mom[4], mom[5], mom[6], mom[7]};")
    e.w("const double m2 = mt * mt;")
    for g in range(n):
        if g < 2:
            e.w(f"const T eps{g}[4] = {{(T)0, (T)(((hel >> {2 + g}) & 1) ? 0 : 1), (T)(((hel >> {2 + g}) & 1) ? 1 : 0), (T)0}};")
        else:
            e.w(f"T eps{g}[4];")
            e.w(f"linear_pol(pg[{g}], (hel >> {2 + g}) & 1, eps{g});")
    e.w("cT ub[4], v[4];")
    e.w("spinor_ubar(kt, mt, sT, ub);")
    e.w("spinor_v(kb, mt, sB, v);")
    e.w(f"cT A[{nperm}];")
    e.w("T me = 0;")
    for idx, sg in enumerate(perms):
        e.w(f"// ordering {name(sg)}")
        parts = []
        for k in range(n - 1):
            c = e.bilinear(sg[:k])
            j = e.gcur(sg[k:])
            parts.append(("cj", c, j))
        U = e.fcur(sg[:n - 1])
        W = e.wspin(sg[n - 1])
        e.w("{")
        e.w("    T ar = 0, ai = 0;")
        for (_, c, j) in parts:
            e.w(f"    cdotj({c}, {j}, ar, ai);")
        e.w(f"    rowdotcol({U}, {W}, ar, ai);")
        e.w(f"    A[{idx}] = cT(ar, ai);")
        # incremental colour sum: K_ss |A_s|^2 + 2 Re(conj(A_s) sum_{t<s} K_st A_t)
        e.w(f"    T tr = {K[idx][idx]} * ar, ti = {K[idx][idx]} * ai;")
        for t in range(idx):
            if K[idx][t] != 0:
                e.w(f"    tr += (T)({2 * K[idx][t]}) * A[{t}].x; ti += (T)({2 * K[idx][t]}) * A[{t}].y;")
        e.w("    me += ar * tr + ai * ti;")
        e.w("}")
    body = "\n".join(e.lines)
    kdecl = ", ".join(str(v) for row in K for v in row)
    return f"""// Generated by gen_amplitudes.py for g g -> t tbar + {n - 2} gluon(s): {nperm} colour orderings,
// {1 << (n + 2)} helicity configurations.  Do not edit.
static constexpr int NPERM_NG{n} = {nperm};
static constexpr double COLOUR_DEN_NG{n} = {den}.0;
static constexpr int COLOUR_NUM_NG{n}[{nperm * nperm}] = {{{kdecl}}};

// Sum over colours of |M|^2 for helicity configuration `hel` (bit 0: top
// spin, bit 1: antitop spin, bit 2+g: gluon g polarisation), g_s = 1.
// mom: t[4], tbar[4], final gluons[4 each]; eb: beam energy sqrt(s_hat)/2;
// mt: top mass; mw: m_t * Gamma_t.
template <typename T>
__device__ __forceinline__ double colour_summed_me2_ng{n}(const double* __restrict__ mom, double eb,
                                                         int hel, double mt, double mw)
{{
    using cT = cplx<T>;
{body}
    return (double)me / COLOUR_DEN_NG{n};
}}
"""


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    for n in (2, 3, 4):
        path = os.path.join(args.out, f"amp_ng{n}.inc")
        text = generate(n)
        old = open(path).read() if os.path.exists(path) else None
        if old != text:
            with open(path, "w") as f:
                f.write(text)


if __name__ == "__main__":
    main()
