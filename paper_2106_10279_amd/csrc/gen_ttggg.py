"""Device code of g g -> t tbar g g g (five gluons, 120 colour orderings,
128 helicity configurations), written by gen_amplitudes.py into
_gen/amp_ng5.inc.

Same physics and representation as the smaller processes (Sec. 2.3: external
wavefunctions, vertices and propagators; colour-ordered Berends-Giele
recursion; chiral spinors, real linear gluon polarisations), organised for a
workgroup of eight waves per event:

  * Object store in LDS, built once per event by all the workgroup's lanes: gluon
    currents j(s; h) of every ordered gluon sequence s up to reflection,
    j(reverse s) = (-1)^(|s|+1) j(s), for every helicity pattern of its
    gluons; top-line spinors Ubar(a), Ubar(ab) and antitop-line spinors
    V(d), V(cd) with one and two gluons attached.
  * Amplitudes split at the vertex of the middle (third) gluon of each
    ordering: A(sigma) = sum over blocks beta = sigma[i:j] with i <= 2 < j of
    Xbar(sigma[:i]) gamma.j(beta) Y(sigma[j:]), Xbar in {ubar, Ubar(a),
    Ubar(ab)}, Y in {v, V(d), V(cd)}.
  * One lane per (first gluon c, helicity configuration) and pass: the
    orderings that start with gluon c, in passes by their last gluon.  The
    five chunks share one code path: the cyclic
    relabelling g -> (g + c) mod 5 maps the orderings that start with gluon 0
    onto those that start with c.  Reflections of gluon sequences are
    resolved by a rule that commutes with that relabelling (the orientation
    whose last label follows the first by 1 or 2 steps mod 5), and the
    objects of a relabelling orbit sit next to each other, so an object's
    address is its orbit's base plus ((first label + c) mod 5) objects.
  * The partial amplitudes go to device memory; the colour sum A^dagger C A
    (120 x 120) runs as a matrix-core contraction in a kernel of its own.
"""
from __future__ import annotations

import itertools
import math

N = 5
NPERM = 120
CHUNK = 24
NHEL = 1 << (N + 2)
# passes over each chunk's orderings (split by the last gluon): fewer live
# accumulators and finer work items, against the antitop-side spinor products
# that every pass forms again
NPASS = 2


def shift(seq, c):
    return tuple((g + c) % N for g in seq)


def canon5(seq):
    """(canonical orientation, reflection sign, reversed?) of a gluon sequence."""
    seq = tuple(seq)
    if len(seq) == 1 or (seq[-1] - seq[0]) % N in (1, 2):
        return seq, 1, False
    return tuple(reversed(seq)), (1 if (len(seq) + 1) % 2 == 0 else -1), True


def pair_index(a, b):
    """Ordered pair (a, b): orbit (b - a) mod 5 of the relabelling, member a."""
    return (((b - a) % N) - 1) * N + a


class Store5:
    """Object store of one event, in units of T: the current region (levels
    1 .. 5, orbit-major, members by first label, 2^L helicity patterns each,
    pattern bit k = gluon at position k of the stored orientation), then
    Ubar(a; s_t, h_a) and V(d; s_tbar, h_d) (20 spinors each), then
    Ubar(ab; s_t, h_a, h_b) and V(cd; s_tbar, h_c, h_d) (160 each).  Every
    region is chunk-major in 16-byte chunks."""

    def __init__(self):
        self.reps, self.ob, self.base, self.levels = {}, {}, {}, {}
        off = 0
        for L in range(1, N + 1):
            canon = sorted(s for s in itertools.permutations(range(N), L) if canon5(s)[0] == s)
            reps = [s for s in canon if s[0] == 0]
            assert len(canon) == N * len(reps)
            self.reps[L] = reps
            self.ob[L] = off
            self.levels[L] = []
            for ri, r in enumerate(reps):
                for d in range(N):
                    cs = shift(r, d)
                    assert canon5(cs)[0] == cs
                    self.base[cs] = off + (ri * N + d) * (1 << L)
                    self.levels[L].append(cs)
            off += len(canon) * (1 << L)
        assert self.base[(0,)] == 0 and all(self.base[(g,)] == 2 * g for g in range(N))
        self.n_gj = off
        self.gj = 0
        self.u1 = 4 * off
        self.v1 = self.u1 + 8 * 4 * N
        self.u2 = self.v1 + 8 * 4 * N
        self.v2 = self.u2 + 8 * 8 * N * (N - 1)
        self.size = self.v2 + 8 * 8 * N * (N - 1)
        self.n_u1 = 4 * N
        self.n_v2 = 8 * N * (N - 1)
        self.pairs = sorted(((a, b) for a in range(N) for b in range(N) if a != b), key=lambda p: pair_index(*p))
        assert [pair_index(*p) for p in self.pairs] == list(range(N * (N - 1)))

    def rep_index(self, cs):
        return self.reps[len(cs)].index(shift(cs, -cs[0]))


def mask(seq):
    m = 0
    for g in seq:
        m |= 1 << g
    return m


def colour_matrix_ng5(G):
    """Integer colour matrix over its common denominator, orderings in
    lexicographic order: the first row by the Fierz identities, the others by
    relabelling the summed adjoint indices, C[s][t] = C[id][s^-1 t]."""
    perms = sorted(itertools.permutations(range(N)))
    index = {p: i for i, p in enumerate(perms)}
    row = [G._contract([tuple(reversed(perms[0])) + tuple(t)]) for t in perms]
    C = []
    for s in perms:
        inv = [0] * N
        for k, g in enumerate(s):
            inv[g] = k
        C.append([row[index[tuple(inv[g] for g in t)]] for t in perms])
    den = 1
    for r in C:
        for v in r:
            den = den * v.denominator // math.gcd(den, v.denominator)
    K = [[int(v * den) for v in r] for r in C]
    assert all(K[i][j] == K[j][i] for i in range(NPERM) for j in range(NPERM))
    return perms, K, den


def emit_tables(st, tl):
    """Split tables of the current levels, concatenated into one array that
    the kernel stages in LDS (STAGE_TAB_NG5, offsets STAGE_*_NG5), and the
    table offsets of -1/P^2 per sequence (STAGE_NINV_NG5)."""
    out = []
    tab, ninv, offs = [], [], {}
    for L in range(2, N + 1):
        seqs = st.levels[L]
        px, tx, ni = [], [], []
        for cs in seqs:
            ni.append(tl.ninv[mask(cs)])
            for k in range(1, L):
                parts = (cs[:k], cs[k:])
                (c1, s1, r1), (c2, s2, r2) = (canon5(p) for p in parts)
                b1, b2 = st.base[c1], st.base[c2]
                P1, P2 = tl.P[mask(parts[0])], tl.P[mask(parts[1])]
                assert b1 < 4096 and b2 < 4096 and P1 < 65536 and P2 < 65536
                lo = b1 | r1 << 12 | b2 << 13 | r2 << 25 | ((s1 * s2) < 0) << 26
                px.append(lo | (P1 | P2 << 16) << 32)
            for a in range(1, L):
                for b in range(a + 1, L):
                    parts = (cs[:a], cs[a:b], cs[b:])
                    cc = [canon5(p) for p in parts]
                    bs = [st.base[c[0]] for c in cc]
                    neg = (cc[0][1] * cc[1][1] * cc[2][1]) < 0
                    lo = bs[0] | cc[0][2] << 12 | bs[1] << 13 | cc[1][2] << 25 | neg << 26
                    tx.append(lo | (bs[2] | cc[2][2] << 12) << 32)
        offs[f"L{L}_PAIR"] = len(tab)
        tab += px
        offs[f"L{L}_TRIP"] = len(tab)
        tab += tx
        offs[f"L{L}_NINV"] = len(ninv)
        ninv += ni
    for k, v in offs.items():
        out.append(f"static constexpr int STAGE_{k}_NG5 = {v};")
    out.append(f"static constexpr int STAGE_TAB_SIZE_NG5 = {len(tab)};")
    out.append(f"static constexpr unsigned long long STAGE_TAB_NG5[{len(tab)}] = "
               f"{{{', '.join(f'{v}ull' for v in tab)}}};")
    out.append(f"static constexpr int STAGE_NINV_SIZE_NG5 = {len(ninv)};")
    out.append(f"static constexpr short STAGE_NINV_NG5[{len(ninv)}] = {{{', '.join(str(v) for v in ninv)}}};")
    # ordered pairs in object order: labels, the current j(ab) (base, sign,
    # orientation) and the momentum-table entries of the propagators
    cd, jb, js, jr, kv, ku = [], [], [], [], [], []
    for (a, b) in st.pairs:
        c, s, r = canon5((a, b))
        cd.append(f"{a}, {b}")
        jb.append(str(st.base[c]))
        js.append(str(s))
        jr.append("1" if r else "0")
        kv.append(str(tl.Kv[mask((a, b))]))
        ku.append(str(tl.Kv[((1 << N) - 1) & ~mask((a, b))]))
    out.append(f"static constexpr signed char P5_AB[{2 * len(cd)}] = {{{', '.join(cd)}}};")
    out.append(f"static constexpr short P5_JB[{len(jb)}] = {{{', '.join(jb)}}};")
    out.append(f"static constexpr signed char P5_JS[{len(js)}] = {{{', '.join(js)}}};")
    out.append(f"static constexpr signed char P5_JR[{len(jr)}] = {{{', '.join(jr)}}};")
    out.append(f"static constexpr short P5_KV[{len(kv)}] = {{{', '.join(kv)}}};")
    out.append(f"static constexpr short P5_KU[{len(ku)}] = {{{', '.join(ku)}}};")
    out.append(f"static constexpr short KT1_5[{N}] = {{{', '.join(str(tl.K1[g]) for g in range(N))}}};")
    out.append(f"static constexpr short KV1_5[{N}] = {{{', '.join(str(tl.Kv[1 << g]) for g in range(N))}}};")
    return "\n".join(out)


def emit_stages(st, tl):
    """Object stages; all lanes of the workgroup take part, and a workgroup
    barrier separates dependent groups of stages."""
    L_ = []
    w = L_.append
    flops = 0
    w("    constexpr int CW = 16 / (int)sizeof(T);")
    w("    constexpr int NG = COOP_NGJ_NG5;")
    w("    const T mtt = (T)mt;")

    nloops = [0]

    def loop(count, offset):
        # Waves take blocks of 64 items from a workgroup counter in LDS
        # (ctr[k], zero at the start of the event): a wave on a compute unit
        # SIMD shared by fewer waves runs faster and takes more blocks, so the
        # workgroup reaches the next barrier together.
        k = nloops[0]
        nloops[0] += 1
        w("    for (;;) {")
        w("        unsigned blk = 0;")
        w(f"        if ((lane & 63) == 0) blk = atomicAdd(&ctr[{k}], 64u);")
        w("        blk = __builtin_amdgcn_readfirstlane(__shfl(blk, 0));")
        w(f"        if (blk >= {count}u) break;")
        w("        const int it = (int)blk + (lane & 63);")
        w(f"        if (it >= {count}) continue;")

    def level(L, offset):
        nonlocal flops
        nseq = len(st.levels[L])
        npair, ntrip = L - 1, (L - 1) * (L - 2) // 2
        flops += nseq * (1 << L) * (npair * 51 + ntrip * 49 + 4)
        w(f"    // level {L}: {nseq} sequences x {1 << L} helicity patterns")
        loop(nseq << L, offset)
        w(f"        const int si = it >> {L};")
        w(f"        const unsigned hm = (unsigned)it & {(1 << L) - 1}u;")
        w("        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;")
        w("#pragma unroll")
        w(f"        for (int k = 1; k < {L}; ++k) {{")
        w(f"            const unsigned long long sp = stab[STAGE_L{L}_PAIR_NG5 + si * {npair} + k - 1];")
        w("            const unsigned lo = (unsigned)sp, hi = (unsigned)(sp >> 32);")
        w("            const unsigned h1 = sub_pattern(hm, 0, k, (lo >> 12) & 1u);")
        w(f"            const unsigned h2 = sub_pattern(hm, k, {L} - k, (lo >> 25) & 1u);")
        w("            const T* q1 = al16(obj + CW * (int)((lo & 4095u) + h1));")
        w("            const T* q2 = al16(obj + CW * (int)(((lo >> 13) & 4095u) + h2));")
        w("            const T g = (lo >> 26) & 1u ? (T)-1 : (T)1;")
        w("            T j1[4], j2[4];")
        w("            ld4s<NG>(q1, j1); ld4s<NG>(q2, j2);")
        w("            const T* p1 = tab + (hi & 0xffffu); const T* p2 = tab + (hi >> 16);")
        w("            const T P1[4] = {p1[0], p1[1], p1[2], p1[3]};")
        w("            const T P2[4] = {p2[0], p2[1], p2[2], p2[3]};")
        w("            const T c1 = (T)2 * (P1[0] * j2[0] - P1[1] * j2[1] - P1[2] * j2[2] - P1[3] * j2[3]);")
        w("            const T c2 = (T)2 * (P2[0] * j1[0] - P2[1] * j1[1] - P2[2] * j1[2] - P2[3] * j1[3]);")
        w("            const T c12 = j1[0] * j2[0] - j1[1] * j2[1] - j1[2] * j2[2] - j1[3] * j2[3];")
        for mu in range(4):
            w(f"            a{mu} += g * (j1[{mu}] * c1 - j2[{mu}] * c2 + c12 * (P2[{mu}] - P1[{mu}]));")
        w("        }")
        if ntrip:
            w("#pragma unroll")
            w(f"        for (int t = 0; t < {ntrip}; ++t) {{")
            w(f"            const unsigned long long tp = stab[STAGE_L{L}_TRIP_NG5 + si * {ntrip} + t];")
            w("            const unsigned lo = (unsigned)tp, hi = (unsigned)(tp >> 32);")
            # split points of triple t (a < b), in the order of the table
            spl = [(a, b) for a in range(1, L) for b in range(a + 1, L)]
            w(f"            constexpr signed char SA[{ntrip}] = {{{', '.join(str(a) for a, _ in spl)}}};")
            w(f"            constexpr signed char SB[{ntrip}] = {{{', '.join(str(b) for _, b in spl)}}};")
            w("            const int sa = SA[t], sb = SB[t];")
            w("            const unsigned h1 = sub_pattern(hm, 0, sa, (lo >> 12) & 1u);")
            w("            const unsigned h2 = sub_pattern(hm, sa, sb - sa, (lo >> 25) & 1u);")
            w(f"            const unsigned h3 = sub_pattern(hm, sb, {L} - sb, (hi >> 12) & 1u);")
            w("            const T* q1 = al16(obj + CW * (int)((lo & 4095u) + h1));")
            w("            const T* q2 = al16(obj + CW * (int)(((lo >> 13) & 4095u) + h2));")
            w("            const T* q3 = al16(obj + CW * (int)((hi & 4095u) + h3));")
            w("            const T g = (lo >> 26) & 1u ? (T)-1 : (T)1;")
            w("            T j1[4], j2[4], j3[4];")
            w("            ld4s<NG>(q1, j1); ld4s<NG>(q2, j2); ld4s<NG>(q3, j3);")
            w("            const T d23 = j2[0] * j3[0] - j2[1] * j3[1] - j2[2] * j3[2] - j2[3] * j3[3];")
            w("            const T d13 = j1[0] * j3[0] - j1[1] * j3[1] - j1[2] * j3[2] - j1[3] * j3[3];")
            w("            const T d12 = j1[0] * j2[0] - j1[1] * j2[1] - j1[2] * j2[2] - j1[3] * j2[3];")
            for mu in range(4):
                w(f"            a{mu} += g * (j1[{mu}] * d23 - (T)2 * j2[{mu}] * d13 + j3[{mu}] * d12);")
            w("        }")
        w(f"        const T f = tab[sninv[STAGE_L{L}_NINV_NG5 + si]];")
        w(f"        st4s<NG>(al16(obj + CW * ({st.ob[L]} + it)), a0 * f, a1 * f, a2 * f, a3 * f);")
        w("    }")

    def u1v1(offset):
        nonlocal flops
        flops += 4 * N * (50 + 80) + 4 * N * (42 + 80)
        w("    // Ubar(a; s_t, h) = -[ubar gamma.eps_a] (K-slash + m) / D,   V(d; s_tbar, h) = -(K'-slash + m) [gamma.eps_d v] / D'")
        loop(8 * N, offset)
        w(f"        const int side = it >= {4 * N}, r = it - side * {4 * N};")
        w("        const int g = r >> 2, sp = (r >> 1) & 1, h = r & 1;")
        w("        T e[4];")
        w("        ld4s<NG>(al16(obj + CW * (2 * g + h)), e);")
        w(f"        const T* q = tab + (side ? {tl.v} : {tl.ub}) + 8 * sp;")
        w("        cplx<T> x[4];")
        w("        for (int i = 0; i < 4; ++i) x[i] = cplx<T>(q[2 * i], q[2 * i + 1]);")
        w("        const T* k = tab + (side ? KV1_5[g] : KT1_5[g]);")
        w("        const T Kc[4] = {k[0], k[1], k[2], k[3]};")
        w("        cplx<T> out[4];")
        w("        if (!side) {")
        w("            cplx<T> s0 = cplx<T>(0, 0), s1 = cplx<T>(0, 0), s2 = cplx<T>(0, 0), s3 = cplx<T>(0, 0);")
        w("            rowslash_acc(x, e, s0, s1, s2, s3);")
        w("            rowprop(s0, s1, s2, s3, Kc, mtt, k[4], k[5], out);")
        w("        } else {")
        w("            cplx<T> W[4] = {cplx<T>(0, 0), cplx<T>(0, 0), cplx<T>(0, 0), cplx<T>(0, 0)};")
        w("            slashcol_acc(e, x, W);")
        w("            colprop(W, Kc, mtt, k[4], k[5], out);")
        w("        }")
        w(f"        stspins<COOP_NU1_NG5>(al16(obj + (side ? {st.v1} : {st.u1}) + CW * r), out);")
        w("    }")

    def pairs2(offset):
        nonlocal flops
        npair = len(st.pairs)
        flops += 2 * 8 * npair * (42 + 42 + 80)
        w("    // V(cd; s_tbar, h_c, h_d) = -(K'-slash + m) [gamma.eps_c V(d) + gamma.j(cd) v] / D'")
        w("    // Ubar(ab; s_t, h_a, h_b) = -[Ubar(a) gamma.eps_b + ubar gamma.j(ab)] (K-slash + m) / D")
        loop(16 * npair, offset)
        w(f"        const int side = it >= {8 * npair}, r = it - side * {8 * npair};")
        w("        const int pi = r >> 3, sp = (r >> 2) & 1, ha = (r >> 1) & 1, hb = r & 1;")
        w("        const int a = P5_AB[2 * pi], b = P5_AB[2 * pi + 1];")
        w("        // j(ab): pattern bit 0 belongs to the first gluon of its stored orientation")
        w("        const int hm = P5_JR[pi] ? (hb | (ha << 1)) : (ha | (hb << 1));")
        w("        const T gs = (T)P5_JS[pi];")
        w("        T jab[4];")
        w("        ld4s<NG>(al16(obj + CW * (P5_JB[pi] + hm)), jab);")
        w("        for (int i = 0; i < 4; ++i) jab[i] *= gs;")
        w("        cplx<T> out[4];")
        w("        if (side) {")
        w("            T ea[4];")
        w("            ld4s<NG>(al16(obj + CW * (2 * a + ha)), ea);")
        w("            cplx<T> y[4];")
        w(f"            ldspins<COOP_NU1_NG5>(al16(obj + {st.v1} + CW * (4 * b + 2 * sp + hb)), y);")
        w("            cplx<T> W[4] = {cplx<T>(0, 0), cplx<T>(0, 0), cplx<T>(0, 0), cplx<T>(0, 0)};")
        w("            slashcol_acc(ea, y, W);")
        w(f"            const T* qv = tab + {tl.v} + 8 * sp;")
        w("            cplx<T> x[4];")
        w("            for (int i = 0; i < 4; ++i) x[i] = cplx<T>(qv[2 * i], qv[2 * i + 1]);")
        w("            slashcol_acc(jab, x, W);")
        w("            const T* k = tab + P5_KV[pi];")
        w("            const T Kc[4] = {k[0], k[1], k[2], k[3]};")
        w("            colprop(W, Kc, mtt, k[4], k[5], out);")
        w("        } else {")
        w("            T eb[4];")
        w("            ld4s<NG>(al16(obj + CW * (2 * b + hb)), eb);")
        w("            cplx<T> x[4];")
        w(f"            ldspins<COOP_NU1_NG5>(al16(obj + {st.u1} + CW * (4 * a + 2 * sp + ha)), x);")
        w("            cplx<T> s0 = cplx<T>(0, 0), s1 = cplx<T>(0, 0), s2 = cplx<T>(0, 0), s3 = cplx<T>(0, 0);")
        w("            rowslash_acc(x, eb, s0, s1, s2, s3);")
        w(f"            const T* qu = tab + {tl.ub} + 8 * sp;")
        w("            cplx<T> u[4];")
        w("            for (int i = 0; i < 4; ++i) u[i] = cplx<T>(qu[2 * i], qu[2 * i + 1]);")
        w("            rowslash_acc(u, jab, s0, s1, s2, s3);")
        w("            const T* k = tab + P5_KU[pi];")
        w("            const T Kc[4] = {k[0], k[1], k[2], k[3]};")
        w("            rowprop(s0, s1, s2, s3, Kc, mtt, k[4], k[5], out);")
        w("        }")
        w(f"        stspins<COOP_NV2_NG5>(al16(obj + (side ? {st.v2} : {st.u2}) + CW * r), out);")
        w("    }")

    # dependent groups: level 2 and the one-gluon spinor chains read level 1;
    # level 3 and the two-gluon chains read levels 1, 2 and the one-gluon
    # chains; each further level reads the ones before
    level(2, 0)
    u1v1(40)
    w("    __syncthreads();")
    level(3, 0)
    pairs2(240)
    w("    __syncthreads();")
    level(4, 0)
    w("    __syncthreads();")
    level(5, 0)
    w("    __syncthreads();")
    assert nloops[0] <= 8
    return "\n".join(L_), flops


def emit_amplitudes(st, K, den, perms):
    """Chunk code (orderings that start with gluon 0), relabelled at run time
    to the lane's chunk c.  Returns the code, flops per lane, and the row
    order and signs of the stored amplitudes."""
    lex = {p: i for i, p in enumerate(perms)}
    chunk0 = [p for p in perms if p[0] == 0]
    assert len(chunk0) == CHUNK
    A = []
    a = A.append
    a("    constexpr int CW = 16 / (int)sizeof(T);")
    a("    constexpr int NG = COOP_NGJ_NG5;")
    a("    const int sT = hel & 1, sB = (hel >> 1) & 1;")
    a("    // gluon helicities relabelled to the chunk: bit x is that of gluon (x + c) mod 5")
    a("    const int hg0 = hel >> 2;")
    a("    const int hg = ((hg0 >> c) | (hg0 << (5 - c))) & 31;")
    for x in range(N):
        a(f"    const int m{x} = {x} + c >= 5 ? {x} + c - 5 : {x} + c;")
    flops = 0

    def hbit(g, hv="hq"):
        return f"(({hv} >> {g}) & 1)"

    def cur_ptr(cs):
        L = len(cs)
        ri = st.rep_index(cs)
        hm = " | ".join(f"({hbit(g)} << {k})" for k, g in enumerate(cs))
        return f"al16(obj + CW * ({st.ob[L] + ri * N * (1 << L)} + (m{cs[0]} << {L}) + ({hm})))"

    def x_load(X):
        if not X:
            return ["        cplx<T> xr[4];",
                    f"        {{ const T* q = tab + {st_tab.ub} + 8 * sT; "
                    "for (int i = 0; i < 4; ++i) xr[i] = cplx<T>(q[2 * i], q[2 * i + 1]); }"]
        if len(X) == 1:
            g = X[0]
            return ["        cplx<T> xr[4];",
                    f"        ldspins<COOP_NU1_NG5>(al16(obj + {st.u1} + CW * (4 * m{g} + 2 * sT + {hbit(g)})), xr);"]
        ga, gb = X
        orb = (((gb - ga) % N) - 1) * N
        return ["        cplx<T> xr[4];",
                f"        ldspins<COOP_NV2_NG5>(al16(obj + {st.u2} + CW * (8 * ({orb} + m{ga}) + 4 * sT + "
                f"2 * {hbit(ga)} + {hbit(gb)})), xr);"]

    def y_load(Y):
        if not Y:
            return ["    cplx<T> yc[4];",
                    f"    {{ const T* q = tab + {st_tab.v} + 8 * sB; "
                    "for (int i = 0; i < 4; ++i) yc[i] = cplx<T>(q[2 * i], q[2 * i + 1]); }"]
        if len(Y) == 1:
            g = Y[0]
            return ["    cplx<T> yc[4];",
                    f"    ldspins<COOP_NU1_NG5>(al16(obj + {st.v1} + CW * (4 * m{g} + 2 * sB + {hbit(g, 'hy')})), yc);"]
        gc, gd = Y
        orb = (((gd - gc) % N) - 1) * N
        return ["    cplx<T> yc[4];",
                f"    ldspins<COOP_NV2_NG5>(al16(obj + {st.v2} + CW * (8 * ({orb} + m{gc}) + 4 * sB + "
                f"2 * {hbit(gc, 'hy')} + {hbit(gd, 'hy')})), yc);"]

    # Passes over the chunk, split by the last gluon of the ordering: the
    # blocks that end before the last gluon (Y = V(d) or V(cd)) differ between
    # the passes, only the few with Y = v are formed in each pass; a fraction
    # of the accumulators is live at a time.
    rest = [g for g in range(1, N)]
    per = len(rest) // NPASS
    passes = [[k for k, sg in enumerate(chunk0) if sg[-1] in rest[q * per:(q + 1) * per]] for q in range(NPASS)]
    sig = {}
    for pi, ks in enumerate(passes):
        loc = {k: i for i, k in enumerate(ks)}
        a(f"    if (pass == {pi}) {{")
        a(f"    T Ar[{len(ks)}], Ai[{len(ks)}];")
        groups = {}
        for k in ks:
            sg = chunk0[k]
            for i in range(3):
                for j in range(3, N + 1):
                    groups.setdefault((sg[:i], sg[j:]), []).append((sg[i:j], k))
        keys = sorted(groups, key=lambda q: (len(q[1]), q[1], len(q[0]), q[0]))
        last = {}
        for gi, key in enumerate(keys):
            for (_, k) in groups[key]:
                last[k] = gi
        # Each group forms its addresses from an opaque copy of the helicity
        # bits (hp0 / hp1 alternately), defined at the start of the group
        # before it: the addresses and LDS reads of a group can move up into
        # the arithmetic of the one before, not further (each further group
        # ahead would hold its operands in registers).
        a("    int hp0 = hg, hp1 = hg;")
        a('    asm volatile("" : "+v"(hp0));')
        for gi, (X, Y) in enumerate(keys):
            cur, nxt = f"hp{gi % 2}", f"hp{(gi + 1) % 2}"
            if gi == 0 or keys[gi - 1][1] != Y:
                # a run of groups with the same antitop-side spinor Y: read
                # once for the run
                a("    {")
                a(f"    const int hy = {cur};")
                A.extend(y_load(Y))
            a("    {")
            a(f"        const int hq = {cur};")
            a(f"        {nxt} = hg;")
            a(f'        asm volatile("" : "+v"({nxt}));')
            A.extend(x_load(X))
            a("        cplx<T> d[4];")
            a("        bilinear(xr, yc, d);")
            flops += 64
            byc = {}
            for (beta, k) in groups[(X, Y)]:
                cs, sgn, _ = canon5(beta)
                byc.setdefault(cs, []).append((sgn, k))
            touched = []
            for ci, (cs, uses) in enumerate(byc.items()):
                jn = f"j{ci}"
                a(f"        T {jn}[4];")
                a(f"        ld4s<NG>({cur_ptr(cs)}, {jn});")
                if len(uses) == 1:
                    sgn, k = uses[0]
                    i = loc[k]
                    touched.append(i)
                    if k not in sig:
                        sig[k] = sgn
                        a(f"        cdot_set({jn}, d, Ar[{i}], Ai[{i}]);")
                        flops += 14
                    else:
                        a(f"        cdot_fma<{sgn * sig[k]}>({jn}, d, Ar[{i}], Ai[{i}]);")
                        flops += 16
                    continue
                a("        {")
                a("            T sr, si;")
                a(f"            cdot_set({jn}, d, sr, si);")
                flops += 14
                for (sgn, k) in uses:
                    i = loc[k]
                    touched.append(i)
                    if k not in sig:
                        sig[k] = sgn
                        a(f"            Ar[{i}] = sr; Ai[{i}] = si;")
                    else:
                        op = "+=" if sgn * sig[k] > 0 else "-="
                        a(f"            Ar[{i}] {op} sr; Ai[{i}] {op} si;")
                        flops += 2
                a("        }")
            # the group's arithmetic completes here (not deferred, with its
            # operands held, to the stores)
            touched = sorted(set(touched))
            for c0 in range(0, len(touched), 4):
                ops = ", ".join(f'"+v"(Ar[{i}]), "+v"(Ai[{i}])' for i in touched[c0:c0 + 4])
                a(f'        asm volatile("" : {ops});')
            a("    }")
            # orderings complete after this group go to memory at once
            for k in sorted(k for k, g in last.items() if g == gi):
                i = loc[k]
                a(f"    if constexpr (LC) lc += (double)Ar[{i}] * (double)Ar[{i}] + (double)Ai[{i}] * (double)Ai[{i}];")
                a(f"    else stj(J + (size_t)(c * {CHUNK} + {k}) * {2 * NHEL} + 2 * hel, Ar[{i}], Ai[{i}]);")
            if gi + 1 == len(keys) or keys[gi + 1][1] != Y:
                a("    }")
        a("    }")
    assert len(sig) == CHUNK
    # row R = c * 24 + k holds sig[k] A(shift(chunk0[k], c))
    rows = [lex[shift(chunk0[k], c)] for c in range(N) for k in range(CHUNK)]
    signs = [sig[k] for c in range(N) for k in range(CHUNK)]
    return "\n".join(A), flops, rows, signs


st_tab = None


def colour_fragments(K, rows, signs, rowoff):
    """Matrix-core fragments of the colour sum in the row order of the stored
    amplitudes: K'[R][R'] = sign_R sign_R' K[row R][row R'], lower block
    triangle of 16 x 16 tiles with the blocks below the diagonal doubled.
    Fragment (tile pair p, step s, lane l) = K'[16 a + l % 16][16 b + rowoff(l / 16, s)]
    for p = a (a + 1) / 2 + b, b <= a; zero beyond row or column 119.
    rowoff(k, s) is the row of tile b that lane group k contracts in step s:
    chosen so that a lane's operands over the four steps are the rows of the
    result that the lane holds (the result layouts of the FP64 and FP32
    steps differ)."""
    def kp(r, q):
        if r >= NPERM or q >= NPERM:
            return 0
        return signs[r] * signs[q] * K[rows[r]][rows[q]]
    out = []
    for ta in range(8):
        for tb in range(ta + 1):
            f = 2 if tb < ta else 1
            for s in range(4):
                for lane in range(64):
                    out.append(f * kp(16 * ta + lane % 16, 16 * tb + rowoff(lane // 16, s)))
    assert max(abs(v) for v in out) < 32768
    return out


def generate_ng5(G):
    """G: the helpers of gen_amplitudes (_contract, CoopTable, emit_coop_fill).
    Returns the text of amp_ng5.inc and the flop counts."""
    global st_tab
    perms, K, den = colour_matrix_ng5(G)
    tl = G.CoopTable(N)
    st_tab = tl
    st = Store5()
    tables = emit_tables(st, tl)
    stages, fst = emit_stages(st, tl)
    amp, fhel, rows, signs = emit_amplitudes(st, K, den, perms)
    fill = G.emit_coop_fill(N, tl, st)
    # FP64 steps: lane group k holds result rows k + 4 r; FP32 steps: 4 k + r
    frag64 = colour_fragments(K, rows, signs, lambda k, s: k + 4 * s)
    frag32 = colour_fragments(K, rows, signs, lambda k, s: 4 * k + s)
    # algorithmic colour-sum flops per helicity: the symmetric form
    # sum_s K_ss |A_s|^2 + 2 sum_{t<s} K_st Re(conj A_s A_t), 4 per (s, t<s) and 4 per s
    colour = 4 * NPERM * (NPERM - 1) // 2 + 4 * NPERM
    counts = {"stages": fst, "per_lane": fhel, "colour_per_helicity": colour, "object_store": st.size,
                      "table": tl.size, "momentum_only": tl.mom_flops()}
    rows_s = ", ".join(str(r) for r in rows)
    signs_s = ", ".join(str(s) for s in signs)
    frag64_s = ", ".join(str(v) for v in frag64)
    frag32_s = ", ".join(str(v) for v in frag32)
    text = f"""// Generated by gen_amplitudes.py for g g -> t tbar g g g: {NPERM} colour orderings,
// {NHEL} helicity configurations.  Do not edit.
static constexpr int NPERM_NG5 = {NPERM};
static constexpr double COLOUR_DEN_NG5 = {den}.0;
static constexpr short COLOUR_NUM_NG5[{NPERM * NPERM}] = {{{", ".join(str(v) for row in K for v in row)}}};
// Table: {tl.size} T per event; object store: {st.size} T per event.  Flops per
// event: table {tl.mom_flops()}, stages {fst}; per (chunk, helicity) lane {fhel};
// colour sum {colour} per helicity configuration.
static constexpr int COOP_TABLE_NG5 = {tl.size};
static constexpr int COOP_OBJ_NG5 = {st.size};
static constexpr int COOP_NGJ_NG5 = {st.n_gj};
static constexpr int COOP_NU1_NG5 = {st.n_u1};
static constexpr int COOP_NV2_NG5 = {st.n_v2};
static constexpr int COOP_FLOPS_STAGES_NG5 = {fst};
static constexpr int COOP_FLOPS_LANE_NG5 = {fhel};
static constexpr int COLOUR_FLOPS_HEL_NG5 = {colour};
// stored amplitude rows: row R = 24 c + k holds ROW_SIGN_NG5[R] A(ROW_ORDERING_NG5[R])
// (lexicographic ordering index)
static constexpr short ROW_ORDERING_NG5[{NPERM}] = {{{rows_s}}};
static constexpr signed char ROW_SIGN_NG5[{NPERM}] = {{{signs_s}}};
// colour-sum fragments of the matrix cores over the common denominator, for
// the FP64 and the FP32 16 x 16 x 4 steps (step s of tile b contracts rows
// 16 b + k + 4 s, resp. 16 b + 4 k + s, in lane group k)
static constexpr short CFRAG64_NG5[{len(frag64)}] = {{{frag64_s}}};
static constexpr short CFRAG32_NG5[{len(frag32)}] = {{{frag32_s}}};
{tables}

// Items of the amplitude phase per event: chunk (first gluon) x pass (a
// subset of the last gluon's labels after relabelling) x half of the
// helicity configurations, one wave each; item = c + 5 (half + 2 pass).
static constexpr int AMP_PASSES_NG5 = {NPASS};
static constexpr int AMP_ITEMS_NG5 = {5 * 2 * NPASS};

// Per-event table and level-1 currents, written by lanes 0 .. 63.
template <typename T, int NS = COOP_NGJ_NG5>
__device__ __forceinline__ void fill_table_coop_ng5(const double* __restrict__ mom, double eb, double mt, double mw,
                                                   T* __restrict__ tab, T* __restrict__ obj, int lane)
{{
{fill}
}}

// The event's object store from its table; every lane of the workgroup
// calls it (it contains workgroup barriers, the last at its end).  ctr: eight
// work counters in LDS, zero on entry; stab, sninv: copies of STAGE_TAB_NG5
// and STAGE_NINV_NG5 in LDS.
template <typename T>
__device__ __forceinline__ void coop_stages_ng5(const T* __restrict__ tab, T* __restrict__ obj, double mt,
                                               int lane, unsigned* ctr,
                                               const unsigned long long* __restrict__ stab,
                                               const short* __restrict__ sninv)
{{
{stages}
}}

// The partial amplitudes of pass `pass` of chunk c (orderings whose
// first gluon is c) for helicity configuration hel, into their rows of the
// event's amplitude block J ([row][hel][re, im], rows 24 c .. 24 c + 23);
// with LC (the leading-colour sum) their squared moduli are added to lc
// instead and nothing is stored.  c and pass are uniform over the wave.
template <typename T, bool LC = false>
__device__ __forceinline__ void coop_amp_ng5(const T* __restrict__ tab, const T* __restrict__ obj, int hel, int c,
                                            int pass, T* __restrict__ J, double& lc)
{{
{amp}
}}
"""
    return text, counts
