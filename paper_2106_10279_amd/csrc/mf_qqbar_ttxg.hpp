// q qbar -> t tbar g: the q qbar channel of p p -> t tbar g (Sec. 3, Table 1:
// five diagrams per quark group).  One helicity configuration per lane, FP64.
//
// Chiral (Weyl) basis, gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]] with
// sigma = (1, sigma_k), sigmabar = (1, -sigma_k), as `bilinear` uses it.  The
// incoming quark's column spinor is u = gamma^0 ubar^dagger and the incoming
// antiquark's row spinor vbar = v^dagger gamma^0 (gamma^0 swaps the halves).
//
// With quark q(pa), antiquark qbar(pb), top t(k1), antitop tbar(k2), gluon
// g(k3) of polarisation eps, J = vbar(pb) gamma u(pa), K = ubar(k1) gamma
// v(k2), s = (pa + pb)^2, s12 = (k1 + k2)^2 and the propagator numerators
// p-slash + m over p^2 - m^2 + i m Gamma, the Feynman-gauge diagrams are
//   A1 = [vbar g^nu (pa - k3)-slash eps-slash u] K_nu / ((pa - k3)^2 s12)   gluon off the quark
//   A2 = [vbar eps-slash (k3 - pb)-slash g^nu u] K_nu / ((k3 - pb)^2 s12)   off the antiquark
//   A3 = [ubar eps-slash S(k1 + k3) g^nu v] J_nu / s                        off the top
//   A4 = [ubar g^nu S(-k2 - k3) eps-slash v] J_nu / s                       off the antitop
//   N5 = [J.K (P + Q).eps + K.eps J.(k3 - Q) - J.eps K.(k3 + P)] / (s s12)  three-gluon vertex
// (P = pa + pb, Q = k1 + k2), and the colour-summed |M|^2 of the
// configuration (g = 1) is sum_de K'_de Re(B_d conj(B_e)) for B = (A1 .. A4,
// N5).  K' follows from the colour factors (T^b T^a)_ji (T^b)_kl,
// (T^a T^b)_ji (T^b)_kl, (T^b)_ji (T^a T^b)_kl, (T^b)_ji (T^b T^a)_kl and
// f^{bca} (T^b)_ji (T^c)_kl (the last with the relative factor i of the
// vertex rules) with Tr(T^a T^b) = delta/2, T^a T^a = C_F,
// T^a T^b T^a = -T^b/6 and Tr(T^a T^b T^c) = (d^abc + i f^abc)/4:
//   3 K' = [[8, -1, 7, -2, 9], [-1, 8, -2, 7, -9], [7, -2, 8, -1, 9],
//           [-2, 7, -1, 8, -9], [9, -9, 9, -9, 18]].
// Massless quarks conserve helicity along the beam line: with spins
// quantised along z the configurations with equal quark and antiquark spin
// vanish, so a lane takes the antiquark spin opposite to the quark's.
#pragma once

namespace mf {

// out = a-slash psi for a complex vector a (contravariant components).
__host__ __device__ __forceinline__ void qq_slash_col(const cplx<double>* a, const cplx<double>* psi,
                                                      cplx<double>* out)
{
    // upper-right block a0 - a.sigma, lower-left a0 + a.sigma
    const cplx<double> ap(a[1].x - a[2].y, a[1].y + a[2].x);   // a1 + i a2
    const cplx<double> am(a[1].x + a[2].y, a[1].y - a[2].x);   // a1 - i a2
    const cplx<double> d0(a[0].x - a[3].x, a[0].y - a[3].y);   // a0 - a3
    const cplx<double> d1(a[0].x + a[3].x, a[0].y + a[3].y);   // a0 + a3
    const cplx<double> o0 = cmul(d0, psi[2]), o1 = cmul(am, psi[3]);
    const cplx<double> o2 = cmul(ap, psi[2]), o3 = cmul(d1, psi[3]);
    const cplx<double> o4 = cmul(d1, psi[0]), o5 = cmul(am, psi[1]);
    const cplx<double> o6 = cmul(ap, psi[0]), o7 = cmul(d0, psi[1]);
    out[0] = cplx<double>(o0.x - o1.x, o0.y - o1.y);
    out[1] = cplx<double>(o3.x - o2.x, o3.y - o2.y);
    out[2] = cplx<double>(o4.x + o5.x, o4.y + o5.y);
    out[3] = cplx<double>(o6.x + o7.x, o6.y + o7.y);
}

// out = row a-slash.
__host__ __device__ __forceinline__ void qq_row_slash(const cplx<double>* row, const cplx<double>* a,
                                                      cplx<double>* out)
{
    const cplx<double> ap(a[1].x - a[2].y, a[1].y + a[2].x);
    const cplx<double> am(a[1].x + a[2].y, a[1].y - a[2].x);
    const cplx<double> d0(a[0].x - a[3].x, a[0].y - a[3].y);
    const cplx<double> d1(a[0].x + a[3].x, a[0].y + a[3].y);
    // columns 0, 1 come from the lower-left block (rows 2, 3), columns 2, 3
    // from the upper-right block (rows 0, 1)
    const cplx<double> o0 = cmul(row[2], d1), o1 = cmul(row[3], ap);
    const cplx<double> o2 = cmul(row[2], am), o3 = cmul(row[3], d0);
    const cplx<double> o4 = cmul(row[0], d0), o5 = cmul(row[1], ap);
    const cplx<double> o6 = cmul(row[0], am), o7 = cmul(row[1], d1);
    out[0] = cplx<double>(o0.x + o1.x, o0.y + o1.y);
    out[1] = cplx<double>(o2.x + o3.x, o2.y + o3.y);
    out[2] = cplx<double>(o4.x - o5.x, o4.y - o5.y);
    out[3] = cplx<double>(o7.x - o6.x, o7.y - o6.y);
}

__host__ __device__ __forceinline__ void qq_real(const double* p, cplx<double>* a)
{
    for (int i = 0; i < 4; ++i)
        a[i] = cplx<double>(p[i], 0.0);
}

__host__ __device__ __forceinline__ cplx<double> qq_dot(const cplx<double>* a, const cplx<double>* b)
{
    const cplx<double> t0 = cmul(a[0], b[0]), t1 = cmul(a[1], b[1]), t2 = cmul(a[2], b[2]), t3 = cmul(a[3], b[3]);
    return cplx<double>(t0.x - t1.x - t2.x - t3.x, t0.y - t1.y - t2.y - t3.y);
}

__host__ __device__ __forceinline__ cplx<double> qq_dotr(const cplx<double>* a, const double* b)
{
    return cplx<double>(a[0].x * b[0] - a[1].x * b[1] - a[2].x * b[2] - a[3].x * b[3],
                        a[0].y * b[0] - a[1].y * b[1] - a[2].y * b[2] - a[3].y * b[3]);
}

__host__ __device__ __forceinline__ double qq_m2(const double* p)
{
    return p[0] * p[0] - p[1] * p[1] - p[2] * p[2] - p[3] * p[3];
}

__host__ __device__ __forceinline__ cplx<double> qq_div(cplx<double> a, cplx<double> d)
{
    const double r = 1.0 / (d.x * d.x + d.y * d.y);
    return cplx<double>((a.x * d.x + a.y * d.y) * r, (a.y * d.x - a.x * d.y) * r);
}

// Real linear polarisation transverse to the 3-momentum of k (h = 0: in the
// plane of k and z, h = 1: normal to it), as in the gluon amplitude kernels.
__host__ __device__ __forceinline__ void qq_linear_pol(const double* k, int h, double* e)
{
    const double pt2 = k[1] * k[1] + k[2] * k[2];
    const double pt = sqrt(pt2);
    const double kk = sqrt(pt2 + k[3] * k[3]);
    const bool has_pt = pt > 0.0;
    const double cph = has_pt ? k[1] / pt : 1.0, sph = has_pt ? k[2] / pt : 0.0;
    const double cth = k[3] / kk, sth = pt / kk;
    e[0] = 0.0;
    e[1] = h ? -sph : cth * cph;
    e[2] = h ? cph : cth * sph;
    e[3] = h ? 0.0 : -sth;
}

// |M|^2 (g = 1, colour-summed) of configuration c of q qbar -> t tbar g:
// bit 0 gluon polarisation, bit 1 antitop spin, bit 2 top spin, bit 3 quark
// spin (antiquark opposite); rev = 0: the quark along +z, 1: along -z.
// mom: t[4], tbar[4], g[4]; eb = sqrt(s)/2; mw = m_top Gamma_top.
__host__ __device__ __forceinline__ double qqbar_ttxg_config(const double* __restrict__ mom, double eb, double mt,
                                                             double mw, int c, int rev)
{
    const double* k1 = mom;
    const double* k2 = mom + 4;
    const double* k3 = mom + 8;
    const double pz[4] = {eb, 0.0, 0.0, eb}, mz[4] = {eb, 0.0, 0.0, -eb};
    const double* pa = rev ? mz : pz;
    const double* pb = rev ? pz : mz;
    const int sq = (c >> 3) & 1;
    cplx<double> a[4], b[4], u[4], vb[4], ub[4], v[4];
    spinor_ubar<double>(pa, 0.0, sq, a);
    spinor_v<double>(pb, 0.0, sq ^ 1, b);
    for (int i = 0; i < 4; ++i) {
        u[i] = cplx<double>(a[(i + 2) & 3].x, -a[(i + 2) & 3].y);
        vb[i] = cplx<double>(b[(i + 2) & 3].x, -b[(i + 2) & 3].y);
    }
    spinor_ubar<double>(k1, mt, (c >> 2) & 1, ub);
    spinor_v<double>(k2, mt, (c >> 1) & 1, v);
    double ep[4];
    qq_linear_pol(k3, c & 1, ep);
    cplx<double> E[4];
    qq_real(ep, E);
    cplx<double> J[4], K[4];
    bilinear(vb, u, J);
    bilinear(ub, v, K);
    const double s = 4.0 * eb * eb;
    double Q[4], P[4];
    for (int mu = 0; mu < 4; ++mu) {
        Q[mu] = k1[mu] + k2[mu];
        P[mu] = pa[mu] + pb[mu];
    }
    const double s12 = qq_m2(Q);
    cplx<double> B[5];
    cplx<double> t[4], w[4], X[4], q[4];
    // A1: vbar g^nu (pa - k3)-slash eps-slash u
    {
        double d[4];
        for (int mu = 0; mu < 4; ++mu)
            d[mu] = pa[mu] - k3[mu];
        qq_slash_col(E, u, t);
        qq_real(d, q);
        qq_slash_col(q, t, w);
        bilinear(vb, w, X);
        const cplx<double> xk = qq_dot(X, K);
        const double den = qq_m2(d) * s12;
        B[0] = cplx<double>(xk.x / den, xk.y / den);
    }
    // A2: vbar eps-slash (k3 - pb)-slash g^nu u
    {
        double d[4];
        for (int mu = 0; mu < 4; ++mu)
            d[mu] = k3[mu] - pb[mu];
        qq_row_slash(vb, E, t);
        qq_real(d, q);
        qq_row_slash(t, q, w);
        bilinear(w, u, X);
        const cplx<double> xk = qq_dot(X, K);
        const double den = qq_m2(d) * s12;
        B[1] = cplx<double>(xk.x / den, xk.y / den);
    }
    // A3: ubar eps-slash (k1 + k3 + m) g^nu v / D
    {
        double d[4];
        for (int mu = 0; mu < 4; ++mu)
            d[mu] = k1[mu] + k3[mu];
        qq_row_slash(ub, E, t);
        qq_real(d, q);
        qq_row_slash(t, q, w);
        for (int i = 0; i < 4; ++i)
            w[i] = cplx<double>(w[i].x + mt * t[i].x, w[i].y + mt * t[i].y);
        bilinear(w, v, X);
        const cplx<double> xj = qq_dot(X, J);
        B[2] = qq_div(xj, cplx<double>((qq_m2(d) - mt * mt) * s, mw * s));
    }
    // A4: ubar g^nu (-k2 - k3 + m) eps-slash v / D
    {
        double d[4];
        for (int mu = 0; mu < 4; ++mu)
            d[mu] = -k2[mu] - k3[mu];
        qq_slash_col(E, v, t);
        qq_real(d, q);
        qq_slash_col(q, t, w);
        for (int i = 0; i < 4; ++i)
            w[i] = cplx<double>(w[i].x + mt * t[i].x, w[i].y + mt * t[i].y);
        bilinear(ub, w, X);
        const cplx<double> xj = qq_dot(X, J);
        B[3] = qq_div(xj, cplx<double>((qq_m2(d) - mt * mt) * s, mw * s));
    }
    // N5: three-gluon vertex
    {
        double pq[4], kq[4], kp[4];
        for (int mu = 0; mu < 4; ++mu) {
            pq[mu] = P[mu] + Q[mu];
            kq[mu] = k3[mu] - Q[mu];
            kp[mu] = k3[mu] + P[mu];
        }
        const cplx<double> jk = qq_dot(J, K), ke = qq_dotr(K, ep), je = qq_dotr(J, ep);
        const cplx<double> jq = qq_dotr(J, kq), kpv = qq_dotr(K, kp);
        const double pe = pq[0] * ep[0] - pq[1] * ep[1] - pq[2] * ep[2] - pq[3] * ep[3];
        const cplx<double> t1 = cmul(ke, jq), t2 = cmul(je, kpv);
        const double den = s * s12;
        B[4] = cplx<double>((jk.x * pe + t1.x - t2.x) / den, (jk.y * pe + t1.y - t2.y) / den);
    }
    constexpr double k3d[5][5] = {{8.0, -1.0, 7.0, -2.0, 9.0},
                                  {-1.0, 8.0, -2.0, 7.0, -9.0},
                                  {7.0, -2.0, 8.0, -1.0, 9.0},
                                  {-2.0, 7.0, -1.0, 8.0, -9.0},
                                  {9.0, -9.0, 9.0, -9.0, 18.0}};
    double sum = 0.0;
    for (int d = 0; d < 5; ++d) {
        sum += k3d[d][d] * (B[d].x * B[d].x + B[d].y * B[d].y);
        for (int e = d + 1; e < 5; ++e)
            sum += 2.0 * k3d[d][e] * (B[d].x * B[e].x + B[d].y * B[e].y);
    }
    return sum / 3.0;
}

// ---------------------------------------------------------------------------
// Helicity recycling.  A1, A2 depend on the helicities only through the
// quark-line chains X1 = vbar g^nu (pa - k3)-slash eps-slash u and
// X2 = vbar eps-slash (k3 - pb)-slash g^nu u (beam orientation, quark spin,
// gluon polarisation: 8 combinations) contracted with K (top and antitop
// spins: 4); A3, A4 through the top-line chains Y3 = ubar eps-slash
// S(k1 + k3) g^nu v and Y4 = ubar g^nu S(-k2 - k3) eps-slash v (top spins,
// gluon polarisation: 8, the same for both orientations) contracted with J
// (orientation, quark spin: 4).  The chains carry their denominators.
// ---------------------------------------------------------------------------

// Beam combination b = (orientation << 2) | (quark spin << 1) | gluon
// polarisation: X1, X2 and, for the current J of (orientation, quark spin),
// want_j; mom: t, tbar, g; eb = sqrt(s)/2.
__host__ __device__ __forceinline__ void qq_beam_chains(const double* __restrict__ mom, double eb, int b,
                                                        bool want_j, cplx<double>* X1, cplx<double>* X2,
                                                        cplx<double>* J)
{
    const double* k1 = mom;
    const double* k2 = mom + 4;
    const double* k3 = mom + 8;
    const int rev = b >> 2, sq = (b >> 1) & 1;
    const double pz[4] = {eb, 0.0, 0.0, eb}, mz[4] = {eb, 0.0, 0.0, -eb};
    const double* pa = rev ? mz : pz;
    const double* pb = rev ? pz : mz;
    cplx<double> a[4], bb[4], u[4], vb[4];
    spinor_ubar<double>(pa, 0.0, sq, a);
    spinor_v<double>(pb, 0.0, sq ^ 1, bb);
    for (int i = 0; i < 4; ++i) {
        u[i] = cplx<double>(a[(i + 2) & 3].x, -a[(i + 2) & 3].y);
        vb[i] = cplx<double>(bb[(i + 2) & 3].x, -bb[(i + 2) & 3].y);
    }
    if (want_j)
        bilinear(vb, u, J);
    double ep[4];
    qq_linear_pol(k3, b & 1, ep);
    cplx<double> E[4], q[4], t[4], w[4];
    qq_real(ep, E);
    double Q[4];
    for (int mu = 0; mu < 4; ++mu)
        Q[mu] = k1[mu] + k2[mu];
    const double s12 = qq_m2(Q);
    double d[4];
    for (int mu = 0; mu < 4; ++mu)
        d[mu] = pa[mu] - k3[mu];
    qq_slash_col(E, u, t);
    qq_real(d, q);
    qq_slash_col(q, t, w);
    bilinear(vb, w, X1);
    const double r1 = 1.0 / (qq_m2(d) * s12);
    for (int mu = 0; mu < 4; ++mu)
        d[mu] = k3[mu] - pb[mu];
    qq_row_slash(vb, E, t);
    qq_real(d, q);
    qq_row_slash(t, q, w);
    bilinear(w, u, X2);
    const double r2 = 1.0 / (qq_m2(d) * s12);
    for (int mu = 0; mu < 4; ++mu) {
        X1[mu] = cplx<double>(X1[mu].x * r1, X1[mu].y * r1);
        X2[mu] = cplx<double>(X2[mu].x * r2, X2[mu].y * r2);
    }
}

// Top combination c = (top spin << 2) | (antitop spin << 1) | gluon
// polarisation: Y3, Y4 (over s times the Breit-Wigner denominator) and, for
// the current K of the two spins, want_k.
__host__ __device__ __forceinline__ void qq_top_chains(const double* __restrict__ mom, double eb, double mt,
                                                       double mw, int c, bool want_k, cplx<double>* Y3,
                                                       cplx<double>* Y4, cplx<double>* K)
{
    const double* k1 = mom;
    const double* k2 = mom + 4;
    const double* k3 = mom + 8;
    cplx<double> ub[4], v[4];
    spinor_ubar<double>(k1, mt, (c >> 2) & 1, ub);
    spinor_v<double>(k2, mt, (c >> 1) & 1, v);
    if (want_k)
        bilinear(ub, v, K);
    double ep[4];
    qq_linear_pol(k3, c & 1, ep);
    cplx<double> E[4], q[4], t[4], w[4];
    qq_real(ep, E);
    const double s = 4.0 * eb * eb;
    double d[4];
    for (int mu = 0; mu < 4; ++mu)
        d[mu] = k1[mu] + k3[mu];
    qq_row_slash(ub, E, t);
    qq_real(d, q);
    qq_row_slash(t, q, w);
    for (int i = 0; i < 4; ++i)
        w[i] = cplx<double>(w[i].x + mt * t[i].x, w[i].y + mt * t[i].y);
    bilinear(w, v, Y3);
    cplx<double> r3 = qq_div(cplx<double>(1.0, 0.0), cplx<double>((qq_m2(d) - mt * mt) * s, mw * s));
    for (int mu = 0; mu < 4; ++mu)
        d[mu] = -k2[mu] - k3[mu];
    qq_slash_col(E, v, t);
    qq_real(d, q);
    qq_slash_col(q, t, w);
    for (int i = 0; i < 4; ++i)
        w[i] = cplx<double>(w[i].x + mt * t[i].x, w[i].y + mt * t[i].y);
    bilinear(ub, w, Y4);
    cplx<double> r4 = qq_div(cplx<double>(1.0, 0.0), cplx<double>((qq_m2(d) - mt * mt) * s, mw * s));
    for (int mu = 0; mu < 4; ++mu) {
        Y3[mu] = cmul(Y3[mu], r3);
        Y4[mu] = cmul(Y4[mu], r4);
    }
}

// Colour-summed |M|^2 of one configuration from its chains: X1, X2, J of the
// beam side, Y3, Y4, K of the top side, ep the gluon polarisation, pe =
// (P + Q).eps, kq = k3 - Q, kp = k3 + P, inv = 1 / (s s12).
__host__ __device__ __forceinline__ double qq_config_from_chains(const cplx<double>* X1, const cplx<double>* X2,
                                                                 const cplx<double>* J, const cplx<double>* Y3,
                                                                 const cplx<double>* Y4, const cplx<double>* K,
                                                                 const double* ep, double pe, const double* kq,
                                                                 const double* kp, double inv)
{
    cplx<double> B[5];
    B[0] = qq_dot(X1, K);
    B[1] = qq_dot(X2, K);
    B[2] = qq_dot(Y3, J);
    B[3] = qq_dot(Y4, J);
    const cplx<double> jk = qq_dot(J, K), ke = qq_dotr(K, ep), je = qq_dotr(J, ep);
    const cplx<double> jq = qq_dotr(J, kq), kpv = qq_dotr(K, kp);
    const cplx<double> t1 = cmul(ke, jq), t2 = cmul(je, kpv);
    B[4] = cplx<double>((jk.x * pe + t1.x - t2.x) * inv, (jk.y * pe + t1.y - t2.y) * inv);
    constexpr double k3d[5][5] = {{8.0, -1.0, 7.0, -2.0, 9.0},
                                  {-1.0, 8.0, -2.0, 7.0, -9.0},
                                  {7.0, -2.0, 8.0, -1.0, 9.0},
                                  {-2.0, 7.0, -1.0, 8.0, -9.0},
                                  {9.0, -9.0, 9.0, -9.0, 18.0}};
    double sum = 0.0;
    for (int d = 0; d < 5; ++d) {
        sum += k3d[d][d] * (B[d].x * B[d].x + B[d].y * B[d].y);
        for (int e = d + 1; e < 5; ++e)
            sum += 2.0 * k3d[d][e] * (B[d].x * B[e].x + B[d].y * B[e].y);
    }
    return sum / 3.0;
}

}  // namespace mf
