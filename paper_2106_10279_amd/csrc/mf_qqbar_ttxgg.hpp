// q qbar -> t tbar g g: the q qbar channel of p p -> t tbar g g (Sec. 3,
// Table 1: 36 Feynman diagrams per quark group), FP64, chiral basis as in
// mf_qqbar_ttxg.hpp; one wave per event, helicity-recycled (below).
//
// The quark line vbar(pb) ... u(pa) and the top line ubar(k1) ... v(k2) are
// joined by one gluon, the spine.  Each line is a chain of vertices from its
// column end; an attachment emits momentum q (a gluon: its momentum; the
// spine seen from the quark line: the momentum it carries to the top side,
// seen from the top line: minus that; the pair g1 g2 joined at a
// three-gluon vertex, "composite": K = k3 + k4).  The 38 terms, in the
// order of gen_qqbar.py's TERMS (their colour basis QQ4_B, QQ4_G is
// generated there):
//    0- 5  both gluons and the spine on the quark line (3! orders)
//    6-11  both on the top line
//   12-19  gluon ga on the quark line, gb on the top line (2 x 2 orders)
//   20-23  ga on the spine (three-gluon vertex), gb on the quark line
//   24-27  ga on the spine, gb on the top line
//   28-29  both on the spine, two three-gluon vertices, ga first
//   30-32  the four-gluon vertex, one term per colour structure
//   33-37  the composite on the quark line (2), the top line (2), the spine
// Feynman gauge, vertex and propagator factors of i counted per class: terms
// 0-19 carry 1, 20-27 and 33-36 i, 28-32 and 37 -1 (a common factor
// dropped); these phases sit in the colour basis (gen_qqbar.py), in which
// every term's colour factor is a sum of basis factors with signs.  Three-gluon vertex with the spine current J (momentum P into
// the vertex), a gluon or the composite e (momentum k out of it):
// (J.e)(P + k) + e J.(P - 2k) + J e.(k - 2P), the spine continuing with
// P - k.  The composite: [e1 e2.(K + k3) + e1.e2 (k4 - k3) - e2 e1.(K + k4)]
// / K^2.  Four-gluon vertex: Xq.e2 e1.Xt - Xq.Xt e1.e2,
// Xq.e1 e2.Xt - Xq.Xt e1.e2, Xq.e1 e2.Xt - Xq.e2 e1.Xt.
#pragma once

namespace mf {

#include "_gen/qqbar_ttxgg.inc"

// (P-slash + m) in / (P^2 - m^2 + i m Gamma), column and row forms.
__host__ __device__ __forceinline__ void q4_prop_col(const double* P, double m, double mw, const cplx<double>* in,
                                                     cplx<double>* out)
{
    cplx<double> Pc[4], t[4];
    qq_real(P, Pc);
    qq_slash_col(Pc, in, t);
    const cplx<double> r = qq_div(cplx<double>(1.0, 0.0), cplx<double>(qq_m2(P) - m * m, mw));
    for (int i = 0; i < 4; ++i)
        out[i] = cmul(cplx<double>(t[i].x + m * in[i].x, t[i].y + m * in[i].y), r);
}

__host__ __device__ __forceinline__ void q4_prop_row(const double* P, double m, double mw, const cplx<double>* in,
                                                     cplx<double>* out)
{
    cplx<double> Pc[4], t[4];
    qq_real(P, Pc);
    qq_row_slash(in, Pc, t);
    const cplx<double> r = qq_div(cplx<double>(1.0, 0.0), cplx<double>(qq_m2(P) - m * m, mw));
    for (int i = 0; i < 4; ++i)
        out[i] = cmul(cplx<double>(t[i].x + m * in[i].x, t[i].y + m * in[i].y), r);
}

// Three-gluon vertex: J (momentum P in), e (momentum k out) -> continuing current.
__host__ __device__ __forceinline__ void q4_v3(const cplx<double>* J, const double* P, const cplx<double>* e,
                                               const double* k, cplx<double>* out)
{
    double Pk[4], P2k[4], k2P[4];
    for (int mu = 0; mu < 4; ++mu) {
        Pk[mu] = P[mu] + k[mu];
        P2k[mu] = P[mu] - 2.0 * k[mu];
        k2P[mu] = k[mu] - 2.0 * P[mu];
    }
    const cplx<double> je = qq_dot(J, e), jp = qq_dotr(J, P2k), ek = qq_dotr(e, k2P);
    for (int mu = 0; mu < 4; ++mu) {
        const cplx<double> a = cmul(e[mu], jp), b = cmul(J[mu], ek);
        out[mu] = cplx<double>(je.x * Pk[mu] + a.x + b.x, je.y * Pk[mu] + a.y + b.y);
    }
}

// Adds term d's Lorentz part A (without its class phase) to the colour-basis
// sums b_r = sum_d QQ4_B[r][d] a_d; the entries are +-1 or 0 and known at
// compile time once the caller's loops over the terms are unrolled, so only
// the additions remain.
__device__ __forceinline__ void q4_basis_add(int d, cplx<double> A, cplx<double>* b)
{
#pragma unroll
    for (int r = 0; r < QQ4_RANK; ++r) {
        const int c = QQ4_B[r][d];
        if (c > 0)
            b[r] = cplx<double>(b[r].x + A.x, b[r].y + A.y);
        else if (c < 0)
            b[r] = cplx<double>(b[r].x - A.x, b[r].y - A.y);
    }
    // the additions happen here: without the pin the compiler defers them
    // to the colour sum and keeps every term's A live (spilling)
#pragma unroll
    for (int r = 0; r < QQ4_RANK; ++r)
        asm volatile("" : "+v"(b[r].x), "+v"(b[r].y));
}

// The colour sum sum_rs QQ4_G[r][s] Re(b_r conj(b_s)) / QQ4_GDEN (the Gram
// matrix of the basis terms' colour factors, real and symmetric).
__device__ __forceinline__ double q4_colour_sum(const cplx<double>* b)
{
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < QQ4_RANK; ++r) {
        double t = (double)QQ4_G[r][r] * (b[r].x * b[r].x + b[r].y * b[r].y);
#pragma unroll
        for (int q = 0; q < r; ++q)
            t += (double)(2 * QQ4_G[r][q]) * (b[r].x * b[q].x + b[r].y * b[q].y);
        s += t;
    }
    return s / (double)QQ4_GDEN;
}

// ---------------------------------------------------------------------------
// Helicity recycling.  The terms depend on the helicity configuration only
// through a few objects, each a function of a subset of the helicity bits:
// the currents J (orientation, quark spin) and K (top spins); the quark-line
// chains with both gluons (6 orders x orientation, quark spin, two
// polarisations), with one gluon (gluon, order x orientation, quark spin,
// its polarisation), with the composite (order x orientation, quark spin,
// polarisations); the top-line chains likewise (top spins in place of
// orientation and quark spin); J after a three-gluon vertex with one gluon.
// One wave per event builds these 344 objects into LDS, then each lane
// contracts them for one configuration.
//
// The chains share their ends.  From the column end, R[x] = S(p0 - q_x)
// e_x-slash col and R[x, y] = S(p0 - q_x - q_y) e_y-slash R[x]; from the row
// end, L[z] = row e_z-slash S(p_end + q_z) and L[z, y] = L[z] e_y-slash
// S(p_end + q_z + q_y), with p_end the momentum that leaves at the row end
// (-p_b on the quark line, k1 on the top line).  A chain with the open
// (spine) slot between them is bilinear(L..., R...): spine last
// bilinear(row, R[x, y]), in the middle bilinear(L[z], R[x]), first
// bilinear(L[z, y], col); likewise with one gluon or the composite.
// ---------------------------------------------------------------------------
constexpr int kQ4J = 0, kQ4K = 4, kQ4Q1 = 8, kQ4T2 = 104, kQ4Q3 = 200, kQ4T3 = 232, kQ4Q7 = 264, kQ4T7 = 296,
              kQ4V5 = 328, kQ4Objects = 344;

struct Q4Kin {
    const double* k1;
    const double* k2;
    const double* kg[2];
    double eb, mt, mw;
    double P0[4], Q[4], K[4], mk2[4];
};

// kin.kg[g] by address arithmetic (the momenta are contiguous: t, tbar,
// g1, g2, as q4_kinematics sets them): indexing kin.kg by a run-time value,
// or selecting between its two members, would place kin in scratch memory
__host__ __device__ __forceinline__ const double* q4_kg(const Q4Kin& kin, int g)
{
    return kin.k1 + 8 + 4 * g;
}

__host__ __device__ __forceinline__ void q4_pol(const Q4Kin& kin, int g, int h, cplx<double>* e)
{
    double ep[4];
    qq_linear_pol(q4_kg(kin, g), h, ep);
    qq_real(ep, e);
}

// The composite current of polarisations (h1, h2).
__host__ __device__ __forceinline__ void q4_composite(const Q4Kin& kin, int h1, int h2, cplx<double>* J12)
{
    cplx<double> e1[4], e2[4];
    q4_pol(kin, 0, h1, e1);
    q4_pol(kin, 1, h2, e2);
    double Kk3[4], k43[4], Kk4[4];
    for (int mu = 0; mu < 4; ++mu) {
        Kk3[mu] = kin.K[mu] + kin.kg[0][mu];
        k43[mu] = kin.kg[1][mu] - kin.kg[0][mu];
        Kk4[mu] = kin.K[mu] + kin.kg[1][mu];
    }
    const cplx<double> x = qq_dotr(e2, Kk3), y = qq_dot(e1, e2), z = qq_dotr(e1, Kk4);
    const double rK = 1.0 / qq_m2(kin.K);
    for (int mu = 0; mu < 4; ++mu) {
        const cplx<double> p1 = cmul(e1[mu], x), p3 = cmul(e2[mu], z);
        J12[mu] = cplx<double>((p1.x + y.x * k43[mu] - p3.x) * rK, (p1.y + y.y * k43[mu] - p3.y) * rK);
    }
}

// One line's ends: line 0 the quark line vbar(p_b) ... u(p_a) with
// s = orientation << 1 | quark spin, line 1 the top line ubar(k1) ... v(k2)
// with s = top spin << 1 | antitop spin.
struct Q4Line {
    cplx<double> row[4], col[4];
    double p0[4], pend[4];
    double m, mw;
};

__device__ __forceinline__ void q4_line(const Q4Kin& kin, int line, int s, Q4Line& L)
{
    const bool top = line != 0;
    const int hi = s >> 1, lo = s & 1;
    double pA[4], pB[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const double z = mu == 3 ? (hi ? -kin.eb : kin.eb) : (mu == 0 ? kin.eb : 0.0);   // the quark's p_a
        pA[mu] = top ? kin.k1[mu] : z;
        pB[mu] = top ? kin.k2[mu] : (mu == 3 ? -z : z);
    }
    const double m = top ? kin.mt : 0.0;
    // the quark line's u and vbar are the conjugate-swapped ubar(p_a) and v(p_b)
    cplx<double> a[4], b[4];
    spinor_ubar<double>(pA, m, top ? hi : lo, a);
    spinor_v<double>(pB, m, top ? lo : (lo ^ 1), b);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const cplx<double> ca(a[(i + 2) & 3].x, -a[(i + 2) & 3].y), cb(b[(i + 2) & 3].x, -b[(i + 2) & 3].y);
        L.row[i] = top ? a[i] : cb;
        L.col[i] = top ? b[i] : ca;
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        L.p0[mu] = top ? -kin.k2[mu] : pA[mu];
        L.pend[mu] = top ? kin.k1[mu] : -pB[mu];
    }
    L.m = m;
    L.mw = top ? kin.mw : 0.0;
}

// One vertex and propagator from the column end (in -> S(P) e-slash in) and
// from the row end (in -> in e-slash S(P)).
__device__ __forceinline__ void q4_step_col(const double* P, double m, double mw, const cplx<double>* e,
                                            const cplx<double>* in, cplx<double>* out)
{
    cplx<double> t[4];
    qq_slash_col(e, in, t);
    q4_prop_col(P, m, mw, t, out);
}

__device__ __forceinline__ void q4_step_row(const double* P, double m, double mw, const cplx<double>* e,
                                            const cplx<double>* in, cplx<double>* out)
{
    cplx<double> t[4];
    qq_row_slash(in, e, t);
    q4_prop_row(P, m, mw, t, out);
}

__device__ __forceinline__ void q4_store(cplx<double>* dst, const cplx<double>* v)
{
#pragma unroll
    for (int i = 0; i < 4; ++i)
        dst[i] = v[i];
}

__device__ __forceinline__ void q4_load(const cplx<double>* src, cplx<double>* v)
{
#pragma unroll
    for (int i = 0; i < 4; ++i)
        v[i] = src[i];
}

// First pass of a wave over the event, lane = line << 5 | s << 3 | k: k < 4
// the gluon k >> 1 with polarisation k & 1, k >= 4 the composite of
// polarisations (k >> 1 & 1, k & 1).  Each lane forms R and L of its
// attachment and the two chains with it and the spine (one-gluon and
// composite objects); the one-gluon R and L go to the slots of the
// both-gluon chains of orders 1 and 3, which the second pass fills last.
// Also J or K (k == 0), J after a three-gluon vertex (quark line, k < 4),
// the polarisations and composites (line 0, s == 0) into eps and j12.
__device__ __forceinline__ void q4_objects_pass1(const Q4Kin& kin, int lane, cplx<double> (*ob)[4], double (*eps)[4],
                                                 cplx<double> (*j12)[4])
{
    const int line = lane >> 5, s = (lane >> 3) & 3, k = lane & 7;
    const bool comp = k >= 4;
    const int g = (k >> 1) & 1, lam = k & 1;
    Q4Line L;
    q4_line(kin, line, s, L);
    cplx<double> e[4];
    if (comp)
        q4_composite(kin, g, lam, e);
    else
        q4_pol(kin, g, lam, e);
    double Pr[4], Pl[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const double q = comp ? kin.kg[0][mu] + kin.kg[1][mu] : q4_kg(kin, g)[mu];   // K or k_g
        Pr[mu] = L.p0[mu] - q;
        Pl[mu] = L.pend[mu] + q;
    }
    cplx<double> R[4], Lp[4], X[4];
    q4_step_col(Pr, L.m, L.mw, e, L.col, R);
    q4_step_row(Pl, L.m, L.mw, e, L.row, Lp);
    const int b1 = line ? kQ4T2 : kQ4Q1, b3 = line ? kQ4T3 : kQ4Q3, b7 = line ? kQ4T7 : kQ4Q7;
    // attachment first from the column end, then the spine; and the reverse
    bilinear(L.row, R, X);
    q4_store(ob[comp ? b7 + (s << 2) + (k & 3) : b3 + 16 * g + ((s << 1) | lam)], X);
    bilinear(Lp, L.col, X);
    q4_store(ob[comp ? b7 + 16 + (s << 2) + (k & 3) : b3 + 16 * g + 8 + ((s << 1) | lam)], X);
    if (!comp) {
        q4_store(ob[b1 + 16 + ((s << 2) | k)], R);
        q4_store(ob[b1 + 48 + ((s << 2) | k)], Lp);
    }
    bilinear(L.row, L.col, X);                      // J (line 0) or K (line 1)
    if (k == 0)
        q4_store(ob[(line ? kQ4K : kQ4J) + s], X);
    if (line == 0 && !comp) {
        cplx<double> V[4];
        q4_v3(X, kin.P0, e, q4_kg(kin, g), V);
        q4_store(ob[kQ4V5 + 8 * g + ((s << 1) | lam)], V);
    }
    if (line == 0 && s == 0) {
        if (comp) {
            q4_store(j12[k & 3], e);
        } else {
#pragma unroll
            for (int mu = 0; mu < 4; ++mu)
                eps[k][mu] = e[mu].x;
        }
    }
}

// Second pass, lane = line << 5 | s << 3 | a << 2 | l1 << 1 | l2: with gluon
// a first from the column end R[a, 1 - a] (orders 0, 2: spine last), with a
// first from the row end L[a, 1 - a] (orders 5, 4: spine first), and
// bilinear(L[1 - a], R[a]) (orders 1, 3: spine in the middle), whose slots
// held the one-gluon R and L: every lane reads before any writes.
__device__ __forceinline__ void q4_objects_pass2(const Q4Kin& kin, int lane, cplx<double> (*ob)[4])
{
    const int line = lane >> 5, s = (lane >> 3) & 3, a = (lane >> 2) & 1, ll = lane & 3;
    const int la = a ? (ll & 1) : (ll >> 1), lb = a ? (ll >> 1) : (ll & 1);   // polarisations of a, 1 - a
    const int b1 = line ? kQ4T2 : kQ4Q1;
    cplx<double> Ra[4], La[4], Lb[4];
    q4_load(ob[b1 + 16 + ((s << 2) | (a << 1) | la)], Ra);
    q4_load(ob[b1 + 48 + ((s << 2) | (a << 1) | la)], La);
    q4_load(ob[b1 + 48 + ((s << 2) | ((1 - a) << 1) | lb)], Lb);
    __syncthreads();
    Q4Line L;
    q4_line(kin, line, s, L);
    cplx<double> e[4];
    q4_pol(kin, 1 - a, lb, e);
    const double* ka = q4_kg(kin, a);
    const double* kb = q4_kg(kin, 1 - a);
    double Pr[4], Pl[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        Pr[mu] = (L.p0[mu] - ka[mu]) - kb[mu];
        Pl[mu] = (L.pend[mu] + ka[mu]) + kb[mu];
    }
    cplx<double> Y[4], X[4];
    q4_step_col(Pr, L.m, L.mw, e, Ra, Y);
    bilinear(L.row, Y, X);
    q4_store(ob[b1 + 16 * (a ? 2 : 0) + ((s << 2) | ll)], X);
    q4_step_row(Pl, L.m, L.mw, e, La, Y);
    bilinear(Y, L.col, X);
    q4_store(ob[b1 + 16 * (a ? 4 : 5) + ((s << 2) | ll)], X);
    bilinear(Lb, Ra, X);
    q4_store(ob[b1 + 16 * (a ? 3 : 1) + ((s << 2) | ll)], X);
}

// The amplitude of three-gluon vertex v3(X, P, e, k) (see q4_v3) contracted
// with the current Y, by linearity without forming the vertex's output:
// (X.e)((P + k).Y) + (e.Y)(X.(P - 2k)) + (X.Y)(e.(k - 2P)), e real.
__device__ __forceinline__ cplx<double> q4_v3_dot(const cplx<double>* X, const double* P, const double* e,
                                                  const double* k, const cplx<double>* Y, cplx<double> eY,
                                                  cplx<double> XY)
{
    double Pk[4], P2k[4], k2P[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        Pk[mu] = P[mu] + k[mu];
        P2k[mu] = P[mu] - 2.0 * k[mu];
        k2P[mu] = k[mu] - 2.0 * P[mu];
    }
    const cplx<double> Xe = qq_dotr(X, e), PkY = qq_dotr(Y, Pk), XP = qq_dotr(X, P2k);
    const double ek = e[0] * k2P[0] - e[1] * k2P[1] - e[2] * k2P[2] - e[3] * k2P[3];
    const cplx<double> t1 = cmul(Xe, PkY), t2 = cmul(eY, XP);
    return cplx<double>(t1.x + t2.x + XY.x * ek, t1.y + t2.y + XY.y * ek);
}

__device__ __forceinline__ cplx<double> q4_scale(cplx<double> a, double r)
{
    return cplx<double>(a.x * r, a.y * r);
}

// |M|^2 of configuration c (bit 0 gluon 1 and bit 1 gluon 2 linear
// polarisation, bit 2 antitop spin, bit 3 top spin, bit 4 quark spin, the
// antiquark's opposite), orientation rev (0: the quark along +z),
// from the event's objects, polarisations eps[g << 1 | h] and composites
// j12[h1 << 1 | h2] in LDS.  Scheduling barriers between the term groups
// keep the compiler from hoisting every group's LDS loads to the top (which
// spills registers).
__device__ __forceinline__ double q4_config_from_objects(const Q4Kin& kin, const cplx<double> (*ob)[4],
                                                         const double (*eps)[4], const cplx<double> (*j12)[4], int c,
                                                         int rev)
{
    const int l1 = c & 1, l2 = (c >> 1) & 1, stb = (c >> 2) & 1, st = (c >> 3) & 1, sq = (c >> 4) & 1;
    const int bq = (rev << 3) | (sq << 2) | (l1 << 1) | l2;
    const int bt = (st << 3) | (stb << 2) | (l1 << 1) | l2;
    const cplx<double>* J = ob[kQ4J + ((rev << 1) | sq)];
    const cplx<double>* K = ob[kQ4K + ((st << 1) | stb)];
    const double* e1 = eps[l1];
    const double* e2 = eps[2 + l2];
    const double rP02 = 1.0 / qq_m2(kin.P0), rQ2 = 1.0 / qq_m2(kin.Q);
    double Pg[2][4], rPg[2];                            // P0 - k_g and 1 / its square
#pragma unroll
    for (int g = 0; g < 2; ++g) {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
            Pg[g][mu] = kin.P0[mu] - q4_kg(kin, g)[mu];
        rPg[g] = 1.0 / qq_m2(Pg[g]);
    }
    // currents dotted with the polarisations and with each other
    const cplx<double> qt = qq_dot(J, K);
    const cplx<double> eK[2] = {qq_dotr(K, e1), qq_dotr(K, e2)};
    const cplx<double> q1 = qq_dotr(J, e1), q2 = qq_dotr(J, e2);
    cplx<double> bsum[QQ4_RANK];                      // the colour-basis sums
#pragma unroll
    for (int r = 0; r < QQ4_RANK; ++r)
        bsum[r] = cplx<double>(0.0, 0.0);
    int d = 0;
#pragma unroll
    for (int o = 0; o < 6; ++o)                         // terms 0-5
        q4_basis_add(d++, q4_scale(qq_dot(ob[kQ4Q1 + 16 * o + bq], K), rQ2), bsum);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int o = 0; o < 6; ++o)                         // terms 6-11
        q4_basis_add(d++, q4_scale(qq_dot(J, ob[kQ4T2 + 16 * o + bt]), rP02), bsum);
    __builtin_amdgcn_sched_barrier(0);
    // the one-gluon chains: quark (g, oq; rev, sq, lam_g), top (g, ot; st, stb, lam_g)
    auto qidx = [&](int g, int oq) { return kQ4Q3 + 16 * g + 8 * oq + ((rev << 2) | (sq << 1) | (g ? l2 : l1)); };
    auto tidx = [&](int g, int ot) { return kQ4T3 + 16 * g + 8 * ot + ((st << 2) | (stb << 1) | (g ? l2 : l1)); };
#pragma unroll
    for (int ga = 0; ga < 2; ++ga)                      // terms 12-19
#pragma unroll
        for (int oq = 0; oq < 2; ++oq)
#pragma unroll
            for (int ot = 0; ot < 2; ++ot)
                q4_basis_add(d++, q4_scale(qq_dot(ob[qidx(ga, oq)], ob[tidx(1 - ga, ot)]), rPg[ga]), bsum);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ga = 0; ga < 2; ++ga) {                    // terms 20-23
        const int gb = 1 - ga;
#pragma unroll
        for (int oq = 0; oq < 2; ++oq) {
            const cplx<double>* X = ob[qidx(gb, oq)];
            const cplx<double> A = q4_v3_dot(X, Pg[gb], ga ? e2 : e1, q4_kg(kin, ga), K, eK[ga], qq_dot(X, K));
            q4_basis_add(d++, q4_scale(A, rPg[gb] * rQ2), bsum);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    auto vidx = [&](int g) { return kQ4V5 + 8 * g + ((rev << 2) | (sq << 1) | (g ? l2 : l1)); };
#pragma unroll
    for (int ga = 0; ga < 2; ++ga)                      // terms 24-27
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
            q4_basis_add(d++, q4_scale(qq_dot(ob[vidx(ga)], ob[tidx(1 - ga, ot)]), rP02 * rPg[ga]), bsum);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ga = 0; ga < 2; ++ga) {                    // terms 28-29
        const int gb = 1 - ga;
        const cplx<double>* V = ob[vidx(ga)];
        const cplx<double> A = q4_v3_dot(V, Pg[ga], gb ? e2 : e1, q4_kg(kin, gb), K, eK[gb], qq_dot(V, K));
        q4_basis_add(d++, q4_scale(A, rP02 * rPg[ga] * rQ2), bsum);
    }
    __builtin_amdgcn_sched_barrier(0);
    {                                                   // terms 30-32
        const double e12 = e1[0] * e2[0] - e1[1] * e2[1] - e1[2] * e2[2] - e1[3] * e2[3];
        const double r = rP02 * rQ2;
        const cplx<double> a1 = cmul(q2, eK[0]), a2(qt.x * e12, qt.y * e12), a3 = cmul(q1, eK[1]);
        q4_basis_add(d++, q4_scale(cplx<double>(a1.x - a2.x, a1.y - a2.y), r), bsum);
        q4_basis_add(d++, q4_scale(cplx<double>(a3.x - a2.x, a3.y - a2.y), r), bsum);
        q4_basis_add(d++, q4_scale(cplx<double>(a3.x - a1.x, a3.y - a1.y), r), bsum);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int oq = 0; oq < 2; ++oq)                      // terms 33-34
        q4_basis_add(d++, q4_scale(qq_dot(ob[kQ4Q7 + 16 * oq + bq], K), rQ2), bsum);
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)                      // terms 35-36
        q4_basis_add(d++, q4_scale(qq_dot(J, ob[kQ4T7 + 16 * ot + bt]), rP02), bsum);
    __builtin_amdgcn_sched_barrier(0);
    {                                                   // term 37: v3(J, P0, J12, K) . K
        const cplx<double>* J12 = j12[(l1 << 1) | l2];
        double Pk[4], P2k[4], k2P[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            Pk[mu] = kin.P0[mu] + kin.K[mu];
            P2k[mu] = kin.P0[mu] - 2.0 * kin.K[mu];
            k2P[mu] = kin.K[mu] - 2.0 * kin.P0[mu];
        }
        const cplx<double> t1 = cmul(qq_dot(J, J12), qq_dotr(K, Pk)), t2 = cmul(qq_dot(J12, K), qq_dotr(J, P2k));
        const cplx<double> t3 = cmul(qt, qq_dotr(J12, k2P));
        q4_basis_add(d++, q4_scale(cplx<double>(t1.x + t2.x + t3.x, t1.y + t2.y + t3.y), rP02 * rQ2), bsum);
    }
    return q4_colour_sum(bsum);
}

__host__ __device__ __forceinline__ Q4Kin q4_kinematics(const double* mom, double eb, double mt, double mw)
{
    Q4Kin k;
    k.k1 = mom;
    k.k2 = mom + 4;
    k.kg[0] = mom + 8;
    k.kg[1] = mom + 12;
    k.eb = eb;
    k.mt = mt;
    k.mw = mw;
    for (int mu = 0; mu < 4; ++mu) {
        k.P0[mu] = mu == 0 ? 2.0 * eb : 0.0;
        k.Q[mu] = mom[mu] + mom[4 + mu];
        k.K[mu] = mom[8 + mu] + mom[12 + mu];
        k.mk2[mu] = -mom[4 + mu];
    }
    return k;
}

}  // namespace mf
