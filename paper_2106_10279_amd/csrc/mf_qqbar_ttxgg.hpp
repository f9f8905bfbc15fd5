// q qbar -> t tbar g g: the q qbar channel of p p -> t tbar g g (Sec. 3,
// Table 1: 36 Feynman diagrams per quark group).  One helicity
// configuration per lane, FP64, chiral basis as in mf_qqbar_ttxg.hpp.
//
// The quark line vbar(pb) ... u(pa) and the top line ubar(k1) ... v(k2) are
// joined by one gluon, the spine.  Each line is a chain of vertices from its
// column end; an attachment emits momentum q (a gluon: its momentum; the
// spine seen from the quark line: the momentum it carries to the top side,
// seen from the top line: minus that; the pair g1 g2 joined at a
// three-gluon vertex, "composite": K = k3 + k4).  The 38 terms, in the
// order of gen_qqbar.py's TERMS (their colour projection QQ4_W is generated
// there):
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
// dropped).  Three-gluon vertex with the spine current J (momentum P into
// the vertex), a gluon or the composite e (momentum k out of it):
// (J.e)(P + k) + e J.(P - 2k) + J e.(k - 2P), the spine continuing with
// P - k.  The composite: [e1 e2.(K + k3) + e1.e2 (k4 - k3) - e2 e1.(K + k4)]
// / K^2.  Four-gluon vertex: Xq.e2 e1.Xt - Xq.Xt e1.e2,
// Xq.e1 e2.Xt - Xq.Xt e1.e2, Xq.e1 e2.Xt - Xq.e2 e1.Xt.
#pragma once

namespace mf {

#include "_gen/qqbar_ttxgg.inc"

struct Q4Att {
    cplx<double> e[4];   // polarisation or off-shell current (unused at the open slot)
    double q[4];         // outgoing momentum
};

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

// X^mu = row V_{N-1} S(P_{N-1}) ... S(P_1) V_0 col with V_a = e_a-slash,
// except at the open slot S, which carries gamma^mu; P_a = p0 - q_0 - ... -
// q_{a-1}.  N and S are compile-time so that every array stays in registers.
template <int N, int S>
__host__ __device__ __forceinline__ void q4_chain(const cplx<double>* row, const cplx<double>* col, const double* p0,
                                                  double m, double mw, const Q4Att* att, cplx<double>* X)
{
    static_assert(N >= 1 && N <= 3 && S >= 0 && S < N, "chain shape");
    double P[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
        P[mu] = p0[mu];
    cplx<double> R[4], L[4], t[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        R[i] = col[i];
#pragma unroll
    for (int a = 0; a < S; ++a) {
        qq_slash_col(att[a].e, R, t);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
            P[mu] -= att[a].q[mu];
        q4_prop_col(P, m, mw, t, R);
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
        P[mu] -= att[S].q[mu];
    double Pt[N][4];
#pragma unroll
    for (int a = S + 1; a < N; ++a)
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            Pt[a][mu] = P[mu];
            P[mu] -= att[a].q[mu];
        }
#pragma unroll
    for (int i = 0; i < 4; ++i)
        L[i] = row[i];
#pragma unroll
    for (int a = N - 1; a > S; --a) {
        qq_row_slash(L, att[a].e, t);
        q4_prop_row(Pt[a], m, mw, t, L);
    }
    bilinear(L, R, X);
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

__host__ __device__ __forceinline__ void q4_set(Q4Att& a, const cplx<double>* e, const double* q)
{
    for (int mu = 0; mu < 4; ++mu) {
        a.e[mu] = e[mu];
        a.q[mu] = q[mu];
    }
}

__host__ __device__ __forceinline__ void q4_set_open(Q4Att& a, const double* q)
{
    for (int mu = 0; mu < 4; ++mu) {
        a.e[mu] = cplx<double>(0.0, 0.0);
        a.q[mu] = q[mu];
    }
}

// Adds factor * A to the colour projections.
__host__ __device__ __forceinline__ void q4_project(int d, cplx<double> A, cplx<double>* proj)
{
#pragma unroll
    for (int r = 0; r < QQ4_RANK; ++r) {
        const cplx<double> w(QQ4_W[r][d][0], QQ4_W[r][d][1]);
        const cplx<double> p = cmul(w, A);
        proj[r] = cplx<double>(proj[r].x + p.x, proj[r].y + p.y);
    }
}

__host__ __device__ __forceinline__ cplx<double> q4_times(cplx<double> a, int f)
{
    // f = 0: 1, 1: i, 2: -1
    return f == 0 ? a : (f == 1 ? cplx<double>(-a.y, a.x) : cplx<double>(-a.x, -a.y));
}

// |M|^2 (g = 1, colour-summed) of configuration c of q qbar -> t tbar g g:
// bit 0 gluon 1 and bit 1 gluon 2 linear polarisation, bit 2 antitop spin,
// bit 3 top spin, bit 4 quark spin (antiquark opposite); rev = 0: the quark
// along +z, 1: along -z.  mom: t[4], tbar[4], g1[4], g2[4]; eb = sqrt(s)/2.
__host__ __device__ __forceinline__ double qqbar_ttxgg_config(const double* __restrict__ mom, double eb, double mt,
                                                              double mw, int c, int rev)
{
    const double* k1 = mom;
    const double* k2 = mom + 4;
    const double* kg[2] = {mom + 8, mom + 12};
    const double pz[4] = {eb, 0.0, 0.0, eb}, mz[4] = {eb, 0.0, 0.0, -eb};
    const double* pa = rev ? mz : pz;
    const double* pb = rev ? pz : mz;
    const int sq = (c >> 4) & 1;
    cplx<double> a[4], b[4], u[4], vb[4], ub[4], v[4];
    spinor_ubar<double>(pa, 0.0, sq, a);
    spinor_v<double>(pb, 0.0, sq ^ 1, b);
    for (int i = 0; i < 4; ++i) {
        u[i] = cplx<double>(a[(i + 2) & 3].x, -a[(i + 2) & 3].y);
        vb[i] = cplx<double>(b[(i + 2) & 3].x, -b[(i + 2) & 3].y);
    }
    spinor_ubar<double>(k1, mt, (c >> 3) & 1, ub);
    spinor_v<double>(k2, mt, (c >> 2) & 1, v);
    cplx<double> eps[2][4];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        double e[4];
        qq_linear_pol(kg[g], (c >> g) & 1, e);
        qq_real(e, eps[g]);
    }
    double P0[4], Q[4], K[4], mk2[4], mQ[4], mP0[4];
    for (int mu = 0; mu < 4; ++mu) {
        P0[mu] = pa[mu] + pb[mu];
        Q[mu] = k1[mu] + k2[mu];
        K[mu] = kg[0][mu] + kg[1][mu];
        mk2[mu] = -k2[mu];
        mQ[mu] = -Q[mu];
        mP0[mu] = -P0[mu];
    }
    const double P02 = qq_m2(P0), Q2 = qq_m2(Q);
    // the composite
    cplx<double> J12[4];
    {
        double Kk3[4], k43[4], Kk4[4];
        for (int mu = 0; mu < 4; ++mu) {
            Kk3[mu] = K[mu] + kg[0][mu];
            k43[mu] = kg[1][mu] - kg[0][mu];
            Kk4[mu] = K[mu] + kg[1][mu];
        }
        const cplx<double> x = qq_dotr(eps[1], Kk3), y = qq_dot(eps[0], eps[1]), z = qq_dotr(eps[0], Kk4);
        const double rK = 1.0 / qq_m2(K);
        for (int mu = 0; mu < 4; ++mu) {
            const cplx<double> p1 = cmul(eps[0][mu], x), p3 = cmul(eps[1][mu], z);
            J12[mu] = cplx<double>((p1.x + y.x * k43[mu] - p3.x) * rK, (p1.y + y.y * k43[mu] - p3.y) * rK);
        }
    }
    cplx<double> proj[QQ4_RANK];
    for (int r = 0; r < QQ4_RANK; ++r)
        proj[r] = cplx<double>(0.0, 0.0);
    Q4Att qa[3], ta[3];
    cplx<double> Xq[4], Xt[4], J1[4], J2[4];
    int d = 0;
    constexpr int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    // terms 0-5: both gluons and the spine on the quark line; the top line is K
    q4_set_open(ta[0], mQ);
    q4_chain<1, 0>(ub, v, mk2, mt, mw, ta, Xt);
#pragma unroll
    for (int o = 0; o < 6; ++o) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int x = perm3[o][t];
            if (x < 2)
                q4_set(qa[t], eps[x], kg[x]);
            else
                q4_set_open(qa[t], Q);
        }
        // the open slot: where 2 sits in perm3[o]
        if (o == 4 || o == 5)
            q4_chain<3, 0>(vb, u, pa, 0.0, 0.0, qa, Xq);
        else if (o == 1 || o == 3)
            q4_chain<3, 1>(vb, u, pa, 0.0, 0.0, qa, Xq);
        else
            q4_chain<3, 2>(vb, u, pa, 0.0, 0.0, qa, Xq);
        const cplx<double> A = qq_dot(Xq, Xt);
        q4_project(d++, cplx<double>(A.x / Q2, A.y / Q2), proj);
    }
    // terms 6-11: both on the top line; the quark line is J
    q4_set_open(qa[0], P0);
    q4_chain<1, 0>(vb, u, pa, 0.0, 0.0, qa, Xq);
#pragma unroll
    for (int o = 0; o < 6; ++o) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int x = perm3[o][t];
            if (x < 2)
                q4_set(ta[t], eps[x], kg[x]);
            else
                q4_set_open(ta[t], mP0);
        }
        if (o == 4 || o == 5)
            q4_chain<3, 0>(ub, v, mk2, mt, mw, ta, Xt);
        else if (o == 1 || o == 3)
            q4_chain<3, 1>(ub, v, mk2, mt, mw, ta, Xt);
        else
            q4_chain<3, 2>(ub, v, mk2, mt, mw, ta, Xt);
        const cplx<double> A = qq_dot(Xq, Xt);
        q4_project(d++, cplx<double>(A.x / P02, A.y / P02), proj);
    }
    // terms 12-19: ga on the quark line, gb on the top line
#pragma unroll
    for (int ga = 0; ga < 2; ++ga) {
        const int gb = 1 - ga;
        double Pq[4], mPq[4];
        for (int mu = 0; mu < 4; ++mu) {
            Pq[mu] = P0[mu] - kg[ga][mu];
            mPq[mu] = -Pq[mu];
        }
        const double Pq2 = qq_m2(Pq);
#pragma unroll
        for (int oq = 0; oq < 2; ++oq) {
            q4_set(qa[oq], eps[ga], kg[ga]);
            q4_set_open(qa[1 - oq], Pq);
            if (oq == 0)
                q4_chain<2, 1>(vb, u, pa, 0.0, 0.0, qa, Xq);
            else
                q4_chain<2, 0>(vb, u, pa, 0.0, 0.0, qa, Xq);
#pragma unroll
            for (int ot = 0; ot < 2; ++ot) {
                q4_set(ta[ot], eps[gb], kg[gb]);
                q4_set_open(ta[1 - ot], mPq);
                if (ot == 0)
                    q4_chain<2, 1>(ub, v, mk2, mt, mw, ta, Xt);
                else
                    q4_chain<2, 0>(ub, v, mk2, mt, mw, ta, Xt);
                const cplx<double> A = qq_dot(Xq, Xt);
                q4_project(d++, cplx<double>(A.x / Pq2, A.y / Pq2), proj);
            }
        }
    }
    // terms 20-23: ga on the spine, gb on the quark line; the top line is K
    q4_set_open(ta[0], mQ);
    q4_chain<1, 0>(ub, v, mk2, mt, mw, ta, Xt);
#pragma unroll
    for (int ga = 0; ga < 2; ++ga) {
        const int gb = 1 - ga;
        double Pq[4];
        for (int mu = 0; mu < 4; ++mu)
            Pq[mu] = P0[mu] - kg[gb][mu];
        const double den = qq_m2(Pq) * Q2;
#pragma unroll
        for (int oq = 0; oq < 2; ++oq) {
            q4_set(qa[oq], eps[gb], kg[gb]);
            q4_set_open(qa[1 - oq], Pq);
            if (oq == 0)
                q4_chain<2, 1>(vb, u, pa, 0.0, 0.0, qa, Xq);
            else
                q4_chain<2, 0>(vb, u, pa, 0.0, 0.0, qa, Xq);
            q4_v3(Xq, Pq, eps[ga], kg[ga], J1);
            const cplx<double> A = qq_dot(J1, Xt);
            q4_project(d++, q4_times(cplx<double>(A.x / den, A.y / den), 1), proj);
        }
    }
    // terms 24-27: ga on the spine, gb on the top line; the quark line is J
    q4_set_open(qa[0], P0);
    q4_chain<1, 0>(vb, u, pa, 0.0, 0.0, qa, Xq);
#pragma unroll
    for (int ga = 0; ga < 2; ++ga) {
        const int gb = 1 - ga;
        double Pt[4], mPt[4];
        for (int mu = 0; mu < 4; ++mu) {
            Pt[mu] = P0[mu] - kg[ga][mu];
            mPt[mu] = -Pt[mu];
        }
        const double den = P02 * qq_m2(Pt);
        q4_v3(Xq, P0, eps[ga], kg[ga], J1);
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) {
            q4_set(ta[ot], eps[gb], kg[gb]);
            q4_set_open(ta[1 - ot], mPt);
            if (ot == 0)
                q4_chain<2, 1>(ub, v, mk2, mt, mw, ta, Xt);
            else
                q4_chain<2, 0>(ub, v, mk2, mt, mw, ta, Xt);
            const cplx<double> A = qq_dot(J1, Xt);
            q4_project(d++, q4_times(cplx<double>(A.x / den, A.y / den), 1), proj);
        }
    }
    // terms 28-32: both on the spine (Xq = J with P0, Xt = K with Q)
    q4_set_open(ta[0], mQ);
    q4_chain<1, 0>(ub, v, mk2, mt, mw, ta, Xt);
#pragma unroll
    for (int ga = 0; ga < 2; ++ga) {
        const int gb = 1 - ga;
        double P1[4];
        for (int mu = 0; mu < 4; ++mu)
            P1[mu] = P0[mu] - kg[ga][mu];
        q4_v3(Xq, P0, eps[ga], kg[ga], J1);
        q4_v3(J1, P1, eps[gb], kg[gb], J2);
        const double den = P02 * qq_m2(P1) * Q2;
        const cplx<double> A = qq_dot(J2, Xt);
        q4_project(d++, q4_times(cplx<double>(A.x / den, A.y / den), 2), proj);
    }
    {
        const cplx<double> q2 = qq_dot(Xq, eps[1]), q1 = qq_dot(Xq, eps[0]), qt = qq_dot(Xq, Xt);
        const cplx<double> t1 = qq_dot(eps[0], Xt), t2 = qq_dot(eps[1], Xt), e12 = qq_dot(eps[0], eps[1]);
        const double den = P02 * Q2;
        const cplx<double> a1 = cmul(q2, t1), a2 = cmul(qt, e12), a3 = cmul(q1, t2);
        q4_project(d++, q4_times(cplx<double>((a1.x - a2.x) / den, (a1.y - a2.y) / den), 2), proj);
        q4_project(d++, q4_times(cplx<double>((a3.x - a2.x) / den, (a3.y - a2.y) / den), 2), proj);
        q4_project(d++, q4_times(cplx<double>((a3.x - a1.x) / den, (a3.y - a1.y) / den), 2), proj);
    }
    // terms 33-37: the composite
#pragma unroll
    for (int oq = 0; oq < 2; ++oq) {        // on the quark line; the top line is K (Xt)
        q4_set(qa[oq], J12, K);
        q4_set_open(qa[1 - oq], Q);
        if (oq == 0)
            q4_chain<2, 1>(vb, u, pa, 0.0, 0.0, qa, J1);
        else
            q4_chain<2, 0>(vb, u, pa, 0.0, 0.0, qa, J1);
        const cplx<double> A = qq_dot(J1, Xt);
        q4_project(d++, q4_times(cplx<double>(A.x / Q2, A.y / Q2), 1), proj);
    }
#pragma unroll
    for (int ot = 0; ot < 2; ++ot) {        // on the top line; the quark line is J (Xq)
        q4_set(ta[ot], J12, K);
        q4_set_open(ta[1 - ot], mP0);
        if (ot == 0)
            q4_chain<2, 1>(ub, v, mk2, mt, mw, ta, J1);
        else
            q4_chain<2, 0>(ub, v, mk2, mt, mw, ta, J1);
        const cplx<double> A = qq_dot(Xq, J1);
        q4_project(d++, q4_times(cplx<double>(A.x / P02, A.y / P02), 1), proj);
    }
    {                                       // on the spine
        q4_v3(Xq, P0, J12, K, J1);
        const double den = P02 * Q2;
        const cplx<double> A = qq_dot(J1, Xt);
        q4_project(d++, q4_times(cplx<double>(A.x / den, A.y / den), 2), proj);
    }
    double sum = 0.0;
    for (int r = 0; r < QQ4_RANK; ++r)
        sum += proj[r].x * proj[r].x + proj[r].y * proj[r].y;
    return sum;
}

}  // namespace mf
