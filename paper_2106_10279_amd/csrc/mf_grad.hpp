// mf_grad.hpp -- adjoint of the g g -> t tbar event weight: d w / d m_t,
// d w / d alpha_s and d w / d y (the random inputs), one event per lane.
//
// The weight is the integrand L(x1, x2) x sigma_hat of Fig. 1 sampled by
// VEGAS: w = J_V W f(x1) f(x2) |M|^2 / (2 s_hat) in pb.  The kernel
// recomputes each event (the same Philox words, bins, VEGAS map, phase
// space and PDF interpolation as the event kernel), then sweeps backwards:
//   weight -> PDFs (derivative of the Hermite interpolant in ln x),
//          -> |M|^2 (mf_me_adjoint.hpp: spinors, propagators, currents),
//          -> momenta -> the mass-rescaling root xi (implicit function
//             theorem on F(xi) = sum_i sqrt(m_i^2 + xi^2 E_i^2) - sqrt(s_hat)),
//          -> the flat two-body momenta -> s_hat, cos theta, phi -> x -> y.
// Inside a VEGAS bin dx_d/dy_d = J_d, and J_V is constant.  d w / d alpha_s
// is n_g w / alpha_s because |M|^2 carries g_s^(2 n_g).  The factorisation
// scale is held fixed when m_t varies.
#pragma once

#include "mf_kernels.hpp"
#include "mf_me_adjoint.hpp"

namespace mf {

struct GradParams {
    EventParams P;          // forward parameters (process must be g g -> t tbar)
    double alpha_s, w_top;
    double* dw_dy;          // [n][4] or null
    double* dw_dmt;         // [n] or null
    double* w_out;          // [n] or null
    double* partials;       // entry-major [4][n_waves]: (sum, comp) of dw/dm_t, then of dw/dalpha_s
};

// d/dv of the cubic Hermite interpolant of `hermite` on interval i.
__device__ __forceinline__ double hermite_dv(const double* t, const double* f, int i, int last, double v)
{
#pragma clang fp contract(off)
    const double h = t[i + 1] - t[i];
    const double u = (v - t[i]) / h;
    const double u2 = u * u;
    const double d00 = 6.0 * u2 - 6.0 * u;
    const double d10 = 3.0 * u2 - 4.0 * u + 1.0;
    const double d01 = -6.0 * u2 + 6.0 * u;
    const double d11 = 3.0 * u2 - 2.0 * u;
    return (d00 * f[i] + d10 * h * knot_slope(t, f, i, last) + d01 * f[i + 1] +
            d11 * h * knot_slope(t, f, i + 1, last)) / h;
}

// x g(x) at mu_F and its derivative in ln x, from the row staged at mu_F^2
// (stage_pdf_row): the derivative of the same cubic.
__device__ __forceinline__ void pdf_xg_dlnx(const EventParams& P, const double* row, const double* lx_knots,
                                            double x, double& G, double& dG)
{
    const double lx = log(x);
    const int k = find_interval(lx_knots, P.n_x, lx);
    G = hermite(lx_knots, row, k, P.n_x - 1, lx);
    dG = hermite_dv(lx_knots, row, k, P.n_x - 1, lx);
}

__global__ void __launch_bounds__(kBlock) grad_kernel_ttx(GradParams G)
{
    constexpr int D = 4;
    const EventParams& P = G.P;
    __shared__ double s_lx[kMaxPdfX];
    __shared__ double s_row[kMaxPdfX];
    const int tid = threadIdx.x;
    const int lane = tid % kWave;
    const int wave_id = blockIdx.x * kWavesPerBlock + tid / kWave;
    const int nb = P.n_bins;
    for (int i = tid; i < P.n_x; i += kBlock)
        s_lx[i] = P.log_x[i];
    stage_pdf_row(P, P.xf, s_row, tid, kBlock);
    __syncthreads();

    Neumaier sm{0.0, 0.0}, sa{0.0, 0.0};
    const uint64_t n_chunks = (P.n_events + kWave - 1) / kWave;
    const uint32_t key0 = (uint32_t)P.seed, key1 = (uint32_t)(P.seed >> 32);
    const double m = P.m_top;

    for (uint64_t chunk = wave_id; chunk < n_chunks; chunk += P.n_waves) {
        const uint64_t ev = chunk * kWave + lane;
        if (ev >= P.n_events)
            continue;
        double x[D], jd[D];
        double jac = 1.0;
        if (P.y_in) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const double t = P.y_in[ev * D + d] * (double)nb;
                int b = (int)floor(t);
                b = b > nb - 1 ? nb - 1 : (b < 0 ? 0 : b);
                x[d] = vegas_map_dim(P.grid + d * (nb + 1), b, t - (double)b, jd[d], nb);
                jac = jac * jd[d];
            }
        } else {
            const uint64_t eid = P.event_ids ? P.event_ids[ev] : ev;
#pragma unroll
            for (int blk = 0; blk < D / 2; ++blk) {
                uint32_t r[4];
                philox4x32_10((uint32_t)eid, (uint32_t)(eid >> 32), P.iter, (uint32_t)blk, key0, key1, r);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int d = 2 * blk + h;
                    const uint64_t kk = ((((uint64_t)r[2 * h]) << 32) | (uint64_t)r[2 * h + 1]) >> 11;
                    const uint64_t prod = kk * (uint64_t)nb;
                    const int b = (int)(prod >> 53);
                    const double delta = (double)(prod & ((1ull << 53) - 1)) * 0x1p-53;
                    x[d] = vegas_map_dim(P.grid + d * (nb + 1), b, delta, jd[d], nb);
                    jac = jac * jd[d];
                }
            }
        }
        double w = 0.0, dm = 0.0, dy[D] = {0.0, 0.0, 0.0, 0.0};
        const double x1 = x[0], x2 = x[1];
        const double shat = x1 * x2 * P.s_had;
        const double thr = 2.0 * m;
        double k[2][4], W = 0.0;
        if (shat > thr * thr && phase_space<2>(x + 2, sqrt(shat), m, P.max_newton, P.ps_const, k, W)) {
            const double rs = sqrt(shat);
            double G1, dG1, G2, dG2;
            pdf_xg_dlnx(P, s_row, s_lx, x1, G1, dG1);
            pdf_xg_dlnx(P, s_row, s_lx, x2, G2, dG2);
            const double f1 = G1 / x1, f2 = G2 / x2;
            const double pref = jac * W * f1 * f2 / (2.0 * shat);
            // ---- forward |M|^2 with its reverse sweep (seed d w / d|M|^2) ----
            double kt_bar[4] = {0, 0, 0, 0}, kb_bar[4] = {0, 0, 0, 0}, eb_bar = 0.0, m_bar = 0.0;
            const double me = ttx_me2_adjoint(k[0], k[1], 0.5 * rs, m, G.w_top, pref * P.me_norm, kt_bar, kb_bar,
                                              eb_bar, m_bar);
            w = pref * (me * P.me_norm);
            // ---- weight: w = jac W f1 f2 me me_norm / (2 shat) ----
            const double cme = me * P.me_norm;
            const double W_bar = jac * f1 * f2 / (2.0 * shat) * cme;
            const double f1_bar = jac * W * f2 / (2.0 * shat) * cme;
            const double f2_bar = jac * W * f1 / (2.0 * shat) * cme;
            double shat_bar = -w / shat;
            // ---- two-body phase space: k_t = (e, rho n), k_tbar = (e, -rho n) ----
            const double cth = 2.0 * x[2] - 1.0;
            const double sth = sqrt(1.0 - cth * cth);
            const double phi = 2.0 * kPi * x[3];
            double sp, cp;
            sincos(phi, &sp, &cp);
            const double nv[3] = {sth * cp, sth * sp, cth};
            const double q = 0.5 * rs;                    // massless energies E_1 = E_2 = q
            const double e = k[0][0];
            const double rho = sqrt(k[0][1] * k[0][1] + k[0][2] * k[0][2] + k[0][3] * k[0][3]);
            const double xi = rho / q;
            double e_bar = kt_bar[0] + kb_bar[0];
            double rho_bar = 0.0, n_bar[3];
            for (int i = 0; i < 3; ++i) {
                const double dd = kt_bar[i + 1] - kb_bar[i + 1];
                rho_bar += dd * nv[i];
                n_bar[i] = rho * dd;
            }
            // W = ps_const rho / e for two bodies
            rho_bar += W_bar * P.ps_const / e;
            e_bar += -W_bar * P.ps_const * rho / (e * e);
            // e = sqrt(m^2 + rho^2)
            rho_bar += e_bar * rho / e;
            m_bar += e_bar * m / e;
            // rho = xi q, xi(m, q, rs) from F = 2 sqrt(m^2 + xi^2 q^2) - rs = 0
            const double xi_bar = rho_bar * q;
            double q_bar = rho_bar * xi;
            const double F_xi = 2.0 * xi * q * q / e, F_m = 2.0 * m / e, F_q = 2.0 * xi * xi * q / e;
            m_bar += -xi_bar * F_m / F_xi;
            q_bar += -xi_bar * F_q / F_xi;
            double rs_bar = xi_bar / F_xi;                // F_rs = -1
            rs_bar += 0.5 * q_bar + 0.5 * eb_bar;          // q = rs/2, incoming energies rs/2
            // direction n(cos theta, phi)
            // (at sin theta = 0 the direction is not differentiable in cos theta; only the
            // z component contributes there)
            const double cth_bar = n_bar[2] + (sth > 0.0 ? (n_bar[0] * cp + n_bar[1] * sp) * (-cth / sth) : 0.0);
            const double phi_bar = sth * (-n_bar[0] * sp + n_bar[1] * cp);
            shat_bar += rs_bar / (2.0 * rs);
            // PDFs f = G(ln x)/x:  df/dx = (G' - G)/x^2
            double x1_bar = shat_bar * x2 * P.s_had + f1_bar * (dG1 - G1) / (x1 * x1);
            double x2_bar = shat_bar * x1 * P.s_had + f2_bar * (dG2 - G2) / (x2 * x2);
            dy[0] = x1_bar * jd[0];
            dy[1] = x2_bar * jd[1];
            dy[2] = 2.0 * cth_bar * jd[2];
            dy[3] = 2.0 * kPi * phi_bar * jd[3];
            dm = m_bar;
        }
        const double da = (double)P.n_g * w / G.alpha_s;
        nm_add(sm, dm);
        nm_add(sa, da);
        if (G.dw_dmt)
            G.dw_dmt[ev] = dm;
        if (G.w_out)
            G.w_out[ev] = w;
        if (G.dw_dy) {
#pragma unroll
            for (int d = 0; d < D; ++d)
                G.dw_dy[ev * D + d] = dy[d];
        }
    }
    if (G.partials) {
        for (int off = kWave >> 1; off > 0; off >>= 1) {
            Neumaier o1{__shfl_down(sm.s, off), __shfl_down(sm.c, off)};
            Neumaier o2{__shfl_down(sa.s, off), __shfl_down(sa.c, off)};
            sm = nm_merge(sm, o1);
            sa = nm_merge(sa, o2);
        }
        if (lane == 0) {
            const size_t nw = (size_t)P.n_waves;
            G.partials[0 * nw + wave_id] = sm.s;
            G.partials[1 * nw + wave_id] = sm.c;
            G.partials[2 * nw + wave_id] = sa.s;
            G.partials[3 * nw + wave_id] = sa.c;
        }
    }
}

}  // namespace mf
