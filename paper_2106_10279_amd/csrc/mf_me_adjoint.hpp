// mf_me_adjoint.hpp -- reverse-mode derivative of the colour- and
// helicity-summed |M|^2 of g g -> t tbar (Sec. 2.3: tree-level helicity
// amplitudes summed over helicities, colour sum with the process colour
// matrix).
//
// The forward pass is the same computation as the generated amplitude code
// for two gluons: colour-ordered amplitudes A(12), A(21) from the s-channel
// gluon current and the top-exchange diagram, with the top propagator
// -1/(K^2 - m^2 + i m Gamma) and real linear gluon polarisations.  Each
// amplitude is a bilinear form A = ubar(k_t) M v(k_tbar), so its adjoints
// are products that the forward primitives already compute:
//   dA/d ubar = M v,   dA/d v = ubar M,
//   dA/d K^mu = g_mu mu (ubar eps0-slash) gamma^mu (eps1-slash v) x prop,
// and the complex adjoint of a holomorphic product z = a b is
// a_bar = z_bar conj(b) (with z_bar = dL/dRe z + i dL/dIm z).  The helicity
// loop recomputes each amplitude and immediately runs its reverse step, so
// no amplitude is stored; the momentum-only quantities (propagators,
// spinors, the gluon current normalisation) collect adjoints over the loop
// and are reversed once at the end.
#pragma once

#include "mf_device.hpp"

namespace mf {

__host__ __device__ __forceinline__ double metric(int mu) { return mu == 0 ? 1.0 : -1.0; }

// a x conj(b)
__host__ __device__ __forceinline__ cplx<double> cmulc(cplx<double> a, cplx<double> b)
{
    return cplx<double>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// Real-parameter adjoint: Re(conj(zbar) dz) for a complex derivative dz.
__host__ __device__ __forceinline__ double radj(cplx<double> zbar, cplx<double> dz)
{
    return zbar.x * dz.x + zbar.y * dz.y;
}

// Reverse of the spinor blocks sqrt_blocks(p, m, s): every entry is
// L(p, m) n with n = (2 (p0 + m))^(-1/2); Abar, Bbar are the adjoints of the
// (re, im) entries.  Accumulates into pbar[4] and mbar.
__host__ __device__ __forceinline__ void sqrt_blocks_adjoint(const double* p, double m, int s, const double* Abar,
                                                             const double* Bbar, double* pbar, double& mbar)
{
    const double n = 1.0 / sqrt(2.0 * (p[0] + m));
    double nbar = 0.0;
    // Each entry: value = L n;  Lbar = vbar n;  nbar += vbar L.
    auto entry = [&](double vbar, double L, double d0, double d1, double d2, double d3, double dm) {
        nbar += vbar * L;
        const double Lbar = vbar * n;
        pbar[0] += Lbar * d0;
        pbar[1] += Lbar * d1;
        pbar[2] += Lbar * d2;
        pbar[3] += Lbar * d3;
        mbar += Lbar * dm;
    };
    if (s == 0) {
        entry(Abar[0], p[0] - p[3] + m, 1.0, 0.0, 0.0, -1.0, 1.0);
        entry(Abar[2], -p[1], 0.0, -1.0, 0.0, 0.0, 0.0);
        entry(Abar[3], -p[2], 0.0, 0.0, -1.0, 0.0, 0.0);
        entry(Bbar[0], p[0] + p[3] + m, 1.0, 0.0, 0.0, 1.0, 1.0);
        entry(Bbar[2], p[1], 0.0, 1.0, 0.0, 0.0, 0.0);
        entry(Bbar[3], p[2], 0.0, 0.0, 1.0, 0.0, 0.0);
    } else {
        entry(Abar[0], -p[1], 0.0, -1.0, 0.0, 0.0, 0.0);
        entry(Abar[1], p[2], 0.0, 0.0, 1.0, 0.0, 0.0);
        entry(Abar[2], p[0] + p[3] + m, 1.0, 0.0, 0.0, 1.0, 1.0);
        entry(Bbar[0], p[1], 0.0, 1.0, 0.0, 0.0, 0.0);
        entry(Bbar[1], -p[2], 0.0, 0.0, -1.0, 0.0, 0.0);
        entry(Bbar[2], p[0] - p[3] + m, 1.0, 0.0, 0.0, -1.0, 1.0);
    }
    // dn/dp0 = dn/dm = -n^3
    const double dn = -n * n * n * nbar;
    pbar[0] += dn;
    mbar += dn;
}

// |M|^2 summed over colours and helicities, g_s = 1, divided by the colour
// denominator (the value the forward amplitude code returns), for outgoing
// top kt, antitop kb, incoming gluons of energy eb along +z and -z, top
// mass m and width gam.  me_bar is dL/d(|M|^2); the adjoints of kt, kb, eb
// and m are accumulated (+=) into kt_bar, kb_bar, eb_bar and m_bar.
__host__ __device__ inline double ttx_me2_adjoint(const double* kt, const double* kb, double eb, double m, double gam,
                                                  double me_bar, double* kt_bar, double* kb_bar, double& eb_bar,
                                                  double& m_bar)
{
    using C = cplx<double>;
    // ---- momentum-only quantities -------------------------------------
    // crossed incoming gluons (all momenta outgoing): q1 = -p_a, q2 = -p_b
    const double q1[4] = {-eb, 0.0, 0.0, -eb};
    const double q2[4] = {-eb, 0.0, 0.0, eb};
    double P3[4];
    for (int mu = 0; mu < 4; ++mu)
        P3[mu] = q1[mu] + q2[mu];
    const double P3sq = P3[0] * P3[0] - P3[1] * P3[1] - P3[2] * P3[2] - P3[3] * P3[3];
    const double f = -1.0 / P3sq;  // gluon propagator times the metric sign of the current
    double K1[4], K2[4];
    for (int mu = 0; mu < 4; ++mu) {
        K1[mu] = kt[mu] + q1[mu];
        K2[mu] = kt[mu] + q2[mu];
    }
    const double mw = m * gam;
    const double re1 = K1[0] * K1[0] - K1[1] * K1[1] - K1[2] * K1[2] - K1[3] * K1[3] - m * m;
    const double re2 = K2[0] * K2[0] - K2[1] * K2[1] - K2[2] * K2[2] - K2[3] * K2[3] - m * m;
    const double inv1 = 1.0 / (re1 * re1 + mw * mw), inv2 = 1.0 / (re2 * re2 + mw * mw);
    const C pr1(-re1 * inv1, mw * inv1), pr2(-re2 * inv2, mw * inv2);  // -1 / (re + i mw)
    C ub[2][4], v[2][4];
    for (int s = 0; s < 2; ++s) {
        spinor_ubar<double>(kt, m, s, ub[s]);
        spinor_v<double>(kb, m, s, v[s]);
    }

    // ---- adjoint accumulators of the momentum-only quantities ----------
    C ub_bar[2][4], v_bar[2][4];
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < 4; ++i) {
            ub_bar[s][i] = C(0.0, 0.0);
            v_bar[s][i] = C(0.0, 0.0);
        }
    double K1_bar[4] = {0, 0, 0, 0}, K2_bar[4] = {0, 0, 0, 0}, q1_bar[4] = {0, 0, 0, 0}, q2_bar[4] = {0, 0, 0, 0};
    C pr1_bar(0.0, 0.0), pr2_bar(0.0, 0.0);
    double f_bar = 0.0;

    const double sc = me_bar / 3.0;  // colour denominator of the 2 x 2 colour matrix {16, -2} / 3
    double me = 0.0;
    // spins unrolled (constant indices into the spinor arrays), polarisations looped
#pragma unroll
    for (int sT = 0; sT < 2; ++sT)
#pragma unroll
    for (int sB = 0; sB < 2; ++sB)
#pragma unroll 1
    for (int hl = 0; hl < 4; ++hl) {
        const int l0 = hl & 1, l1 = (hl >> 1) & 1;
        const double e0[4] = {0.0, l0 ? 0.0 : 1.0, l0 ? 1.0 : 0.0, 0.0};
        const double e1[4] = {0.0, l1 ? 0.0 : 1.0, l1 ? 1.0 : 0.0, 0.0};
        const C* u = ub[sT];
        const C* w = v[sB];
        // ---- forward ----
        const double e0q1 = e0[0] * q1[0] - e0[1] * q1[1] - e0[2] * q1[2] - e0[3] * q1[3];
        const double e0q2 = e0[0] * q2[0] - e0[1] * q2[1] - e0[2] * q2[2] - e0[3] * q2[3];
        const double e1q1 = e1[0] * q1[0] - e1[1] * q1[1] - e1[2] * q1[2] - e1[3] * q1[3];
        const double e1q2 = e1[0] * q2[0] - e1[1] * q2[1] - e1[2] * q2[2] - e1[3] * q2[3];
        const double e01 = e0[0] * e1[0] - e0[1] * e1[1] - e0[2] * e1[2] - e0[3] * e1[3];
        // three-gluon vertex currents for the orderings (12) and (21)
        double V01[4], V10[4], j01[4], j10[4];
        for (int mu = 0; mu < 4; ++mu) {
            V01[mu] = e0[mu] * (2.0 * e1q1) - e1[mu] * (2.0 * e0q2) + e01 * (q2[mu] - q1[mu]);
            V10[mu] = e1[mu] * (2.0 * e0q2) - e0[mu] * (2.0 * e1q1) + e01 * (q1[mu] - q2[mu]);
            j01[mu] = f * V01[mu];
            j10[mu] = f * V10[mu];
        }
        C c[4];
        bilinear(u, w, c);
        C s0[4] = {C(0, 0), C(0, 0), C(0, 0), C(0, 0)}, s1[4] = {C(0, 0), C(0, 0), C(0, 0), C(0, 0)};
        rowslash_acc(u, e0, s0[0], s0[1], s0[2], s0[3]);
        rowslash_acc(u, e1, s1[0], s1[1], s1[2], s1[3]);
        C W0[4], W1[4];
        slashcol(e0, w, W0);
        slashcol(e1, w, W1);
        C t0[4], t1[4];
        rowprop(s0[0], s0[1], s0[2], s0[3], K1, m, 1.0, 0.0, t0);
        rowprop(s1[0], s1[1], s1[2], s1[3], K2, m, 1.0, 0.0, t1);
        double y0r = 0.0, y0i = 0.0, y1r = 0.0, y1i = 0.0;
        rowdotcol(t0, W1, y0r, y0i);
        rowdotcol(t1, W0, y1r, y1i);
        const C Y0(y0r, y0i), Y1(y1r, y1i);
        double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
        cdotj(c, j01, a0r, a0i);
        cdotj(c, j10, a1r, a1i);
        const C P0 = cmul(pr1, Y0), P1 = cmul(pr2, Y1);
        const C A0(a0r + P0.x, a0i + P0.y), A1(a1r + P1.x, a1i + P1.y);
        me += 16.0 * (A0.x * A0.x + A0.y * A0.y) + 16.0 * (A1.x * A1.x + A1.y * A1.y)
              - 4.0 * (A0.x * A1.x + A0.y * A1.y);

        // ---- reverse ----
        const C A0b(sc * (32.0 * A0.x - 4.0 * A1.x), sc * (32.0 * A0.y - 4.0 * A1.y));
        const C A1b(sc * (32.0 * A1.x - 4.0 * A0.x), sc * (32.0 * A1.y - 4.0 * A0.y));
        // s-channel terms ubar (j-slash) v with real j
        {
            C jv0[4], jv1[4];
            slashcol(j01, w, jv0);
            slashcol(j10, w, jv1);
            C uj0[4] = {C(0, 0), C(0, 0), C(0, 0), C(0, 0)}, uj1[4] = {C(0, 0), C(0, 0), C(0, 0), C(0, 0)};
            rowslash_acc(u, j01, uj0[0], uj0[1], uj0[2], uj0[3]);
            rowslash_acc(u, j10, uj1[0], uj1[1], uj1[2], uj1[3]);
            for (int i = 0; i < 4; ++i) {
                const C a = cmulc(A0b, jv0[i]), b = cmulc(A1b, jv1[i]);
                ub_bar[sT][i].x += a.x + b.x;
                ub_bar[sT][i].y += a.y + b.y;
                const C d = cmulc(A0b, uj0[i]), e = cmulc(A1b, uj1[i]);
                v_bar[sB][i].x += d.x + e.x;
                v_bar[sB][i].y += d.y + e.y;
            }
            double j01_bar[4], j10_bar[4];
            for (int mu = 0; mu < 4; ++mu) {
                j01_bar[mu] = metric(mu) * radj(A0b, c[mu]);
                j10_bar[mu] = metric(mu) * radj(A1b, c[mu]);
            }
            // j = f V, V linear in q1, q2
            double a01 = 0.0, b01 = 0.0, a10 = 0.0, b10 = 0.0;
            for (int mu = 0; mu < 4; ++mu) {
                f_bar += j01_bar[mu] * V01[mu] + j10_bar[mu] * V10[mu];
                const double v01 = f * j01_bar[mu], v10 = f * j10_bar[mu];
                a01 += e0[mu] * v01;
                b01 += e1[mu] * v01;
                a10 += e1[mu] * v10;
                b10 += e0[mu] * v10;
                q1_bar[mu] += -e01 * v01 + e01 * v10;
                q2_bar[mu] += e01 * v01 - e01 * v10;
            }
            for (int mu = 0; mu < 4; ++mu) {
                const double g = metric(mu);
                q1_bar[mu] += 2.0 * g * e1[mu] * a01 - 2.0 * g * e1[mu] * b10;
                q2_bar[mu] += -2.0 * g * e0[mu] * b01 + 2.0 * g * e0[mu] * a10;
            }
        }
        // top-exchange terms prop x Y with Y = ubar eps-slash (K-slash + m) eps'-slash v
        {
            pr1_bar.x += cmulc(A0b, Y0).x;
            pr1_bar.y += cmulc(A0b, Y0).y;
            pr2_bar.x += cmulc(A1b, Y1).x;
            pr2_bar.y += cmulc(A1b, Y1).y;
            const C Y0b = cmulc(A0b, pr1), Y1b = cmulc(A1b, pr2);
            // dY/d ubar = eps-slash (K-slash + m) W,  dY/d v = t eps'-slash
            C nw0[4], nw1[4], r0[4], r1[4];
            colprop(W1, K1, m, 1.0, 0.0, nw0);
            colprop(W0, K2, m, 1.0, 0.0, nw1);
            slashcol(e0, nw0, r0);
            slashcol(e1, nw1, r1);
            C l0v[4] = {C(0, 0), C(0, 0), C(0, 0), C(0, 0)}, l1v[4] = {C(0, 0), C(0, 0), C(0, 0), C(0, 0)};
            rowslash_acc(t0, e1, l0v[0], l0v[1], l0v[2], l0v[3]);
            rowslash_acc(t1, e0, l1v[0], l1v[1], l1v[2], l1v[3]);
            for (int i = 0; i < 4; ++i) {
                const C a = cmulc(Y0b, r0[i]), b = cmulc(Y1b, r1[i]);
                ub_bar[sT][i].x += a.x + b.x;
                ub_bar[sT][i].y += a.y + b.y;
                const C d = cmulc(Y0b, l0v[i]), e = cmulc(Y1b, l1v[i]);
                v_bar[sB][i].x += d.x + e.x;
                v_bar[sB][i].y += d.y + e.y;
            }
            // dY/dK^mu = g_mu (s gamma^mu W),  dY/dm = s W
            C b0[4], b1[4];
            bilinear(s0, W1, b0);
            bilinear(s1, W0, b1);
            for (int mu = 0; mu < 4; ++mu) {
                K1_bar[mu] += metric(mu) * radj(Y0b, b0[mu]);
                K2_bar[mu] += metric(mu) * radj(Y1b, b1[mu]);
            }
            double sw0r = 0.0, sw0i = 0.0, sw1r = 0.0, sw1i = 0.0;
            rowdotcol(s0, W1, sw0r, sw0i);
            rowdotcol(s1, W0, sw1r, sw1i);
            m_bar += radj(Y0b, C(sw0r, sw0i)) + radj(Y1b, C(sw1r, sw1i));
        }
    }

    // ---- reverse of the momentum-only quantities -------------------------
    // propagators pr = -1/z, z = re + i mw:  dpr/dz = pr^2
    {
        const C d1 = cmul(pr1, pr1), d2 = cmul(pr2, pr2);
        const C z1b = cmulc(pr1_bar, d1), z2b = cmulc(pr2_bar, d2);
        const double mw_bar = z1b.y + z2b.y;
        for (int mu = 0; mu < 4; ++mu) {
            K1_bar[mu] += 2.0 * metric(mu) * K1[mu] * z1b.x;
            K2_bar[mu] += 2.0 * metric(mu) * K2[mu] * z2b.x;
        }
        m_bar += -2.0 * m * (z1b.x + z2b.x) + gam * mw_bar;
    }
    for (int mu = 0; mu < 4; ++mu) {
        kt_bar[mu] += K1_bar[mu] + K2_bar[mu];
        q1_bar[mu] += K1_bar[mu];
        q2_bar[mu] += K2_bar[mu];
    }
    // f = -1/P3^2, P3 = q1 + q2
    for (int mu = 0; mu < 4; ++mu) {
        const double P3_bar = f_bar * 2.0 * metric(mu) * P3[mu] / (P3sq * P3sq);
        q1_bar[mu] += P3_bar;
        q2_bar[mu] += P3_bar;
    }
    eb_bar += -q1_bar[0] - q1_bar[3] - q2_bar[0] + q2_bar[3];
    // spinors: ubar = (conj B, conj A), v = (A, -B) from sqrt_blocks
    for (int s = 0; s < 2; ++s) {
        double Ab[4], Bb[4];
        Bb[0] = ub_bar[s][0].x; Bb[1] = -ub_bar[s][0].y; Bb[2] = ub_bar[s][1].x; Bb[3] = -ub_bar[s][1].y;
        Ab[0] = ub_bar[s][2].x; Ab[1] = -ub_bar[s][2].y; Ab[2] = ub_bar[s][3].x; Ab[3] = -ub_bar[s][3].y;
        sqrt_blocks_adjoint(kt, m, s, Ab, Bb, kt_bar, m_bar);
        Ab[0] = v_bar[s][0].x; Ab[1] = v_bar[s][0].y; Ab[2] = v_bar[s][1].x; Ab[3] = v_bar[s][1].y;
        Bb[0] = -v_bar[s][2].x; Bb[1] = -v_bar[s][2].y; Bb[2] = -v_bar[s][3].x; Bb[3] = -v_bar[s][3].y;
        sqrt_blocks_adjoint(kb, m, s, Ab, Bb, kb_bar, m_bar);
    }
    return me / 3.0;
}

}  // namespace mf
