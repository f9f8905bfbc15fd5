/*
 * phase_space_pdf.c -- oracle: flat phase space, fiducial cuts, PDF.
 * Test infrastructure only (see mfo.h).
 *
 * Phase space (Sec. 2.4): the paper uses RAMBO (Kleiss, Stirling, Ellis,
 * CPC 40 (1986) 359), a flat n-body generator.  The integration dimensions
 * of the workloads here are 3 n_f - 4 per event (4, 7, 10 including x1 and
 * x2), so the massless momenta come from the minimal-dimension flat
 * generator of Plaetzer ("RAMBO on diet", arXiv:1308.2922), which samples
 * exactly RAMBO's flat massless phase space, followed by RAMBO's massive
 * rescaling step.
 *
 * PDFs (Sec. 1 ingredient (ii), PDFFlow): x g(x, Q^2) tabulated on a grid
 * in (ln x, ln Q^2), interpolated by cubic Hermite splines in ln x on the
 * bracketing Q^2 rows, then in ln Q^2.
 */
#include <math.h>
#include "mfo.h"

static const double PI = 3.14159265358979323846;

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i)
        f *= (double)i;
    return f;
}

/* Volume of massless n-body phase space (2 pi)^4 delta^4 prod d^3p/((2pi)^3 2E):
 * (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!). */
double mfo_massless_volume(int n_f, double shat)
{
    return pow(2.0 * PI, 4 - 3 * n_f) * pow(PI / 2.0, n_f - 1) * pow(shat, n_f - 2)
           / (factorial(n_f - 1) * factorial(n_f - 2));
}

/* Invert the cumulative distribution of the squared-mass ratio u of the
 * (n_f + 1 - i)-particle remainder: (n_f+1-i) u^(n_f-i) - (n_f-i) u^(n_f+1-i) = r. */
static double solve_mass_ratio(int power, double r)
{
    if (power == 1)                  /* 2u - u^2 = r */
        return 1.0 - sqrt(1.0 - r);
    if (power == 2)                  /* 3u^2 - 2u^3 = r; u = 1/2 - sin(asin(1 - 2r)/3) */
        return 0.5 - sin(asin(1.0 - 2.0 * r) / 3.0);
    /* power 3: 4u^3 - 3u^4 = r, increasing on [0, 1]: bisection until the
     * bracket cannot shrink (the root to the last bit) */
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi)
            break;
        double f = 4.0 * mid * mid * mid - 3.0 * mid * mid * mid * mid - r;
        if (f < 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Boost v, given in the rest frame of Q (mass M), to the frame where Q has
 * the stated components. */
static void boost_from_rest(const double Q[4], double M, const double v[4], double out[4])
{
    double qv = Q[1] * v[1] + Q[2] * v[2] + Q[3] * v[3];
    double e = (Q[0] * v[0] + qv) / M;
    double c = (v[0] + e) / (Q[0] + M);
    out[0] = e;
    out[1] = v[1] + c * Q[1];
    out[2] = v[2] + c * Q[2];
    out[3] = v[3] + c * Q[3];
}

/* r layout (3 n_f - 4 values): mass variables for i = 2 .. n_f-1, then the
 * pairs (cos theta_i variable, phi_i variable) for i = 1 .. n_f-1.
 * k: [n_f][4] massive momenta in the partonic CM frame. */
int mfo_phase_space(int n_f, const double *mass, double sqrt_shat,
                    const double *r, int max_newton, double *k, double *weight)
{
    double shat = sqrt_shat * sqrt_shat;
    double M[MFO_MAX_F + 1];
    double p[MFO_MAX_F][4];

    /* Intermediate invariant masses M_1 = sqrt(s) > M_2 > ... > M_n = 0. */
    M[1] = sqrt_shat;
    for (int i = 2; i <= n_f - 1; ++i) {
        double u = solve_mass_ratio(n_f - i, r[i - 2]);
        M[i] = sqrt(u) * M[i - 1];
    }
    M[n_f] = 0.0;

    /* Chain of two-body decays Q_i -> p_i + Q_{i+1}, each isotropic in the
     * Q_i rest frame, then boosted to the CM frame. */
    double Q[4] = { sqrt_shat, 0.0, 0.0, 0.0 };
    for (int i = 1; i <= n_f - 1; ++i) {
        double cth = 2.0 * r[(n_f - 2) + 2 * (i - 1)] - 1.0;
        double phi = 2.0 * PI * r[(n_f - 2) + 2 * (i - 1) + 1];
        double sth = sqrt(1.0 - cth * cth);
        double q = (M[i] * M[i] - M[i + 1] * M[i + 1]) / (2.0 * M[i]);
        double prest[4] = { q, q * sth * cos(phi), q * sth * sin(phi), q * cth };
        double qrest[4] = { sqrt(q * q + M[i + 1] * M[i + 1]), -prest[1], -prest[2], -prest[3] };
        double Qn[4];
        boost_from_rest(Q, M[i], prest, p[i - 1]);
        boost_from_rest(Q, M[i], qrest, Qn);
        for (int mu = 0; mu < 4; ++mu)
            Q[mu] = Qn[mu];
    }
    for (int mu = 0; mu < 4; ++mu)
        p[n_f - 1][mu] = Q[mu];

    double w0 = mfo_massless_volume(n_f, shat);

    double msum = 0.0;
    int massive = 0;
    for (int i = 0; i < n_f; ++i) {
        msum += mass[i];
        if (mass[i] != 0.0)
            massive = 1;
    }
    if (!massive) {
        for (int i = 0; i < n_f; ++i)
            for (int mu = 0; mu < 4; ++mu)
                k[4 * i + mu] = p[i][mu];
        *weight = w0;
        return 0;
    }

    /* RAMBO massive step: scale 3-momenta by xi so that the energies
     * sqrt(m_i^2 + xi^2 E_i^2) add up to sqrt(s); Newton on xi.  The
     * iteration stops when the step is below 1e-15 xi, or when the residual
     * is already at the rounding level of the energy sum (2 n_f eps sqrt(s)),
     * which is all that can be reached close to threshold. */
    double xi = sqrt(1.0 - (msum / sqrt_shat) * (msum / sqrt_shat));
    double floor_res = 2.0 * n_f * 0x1p-52 * sqrt_shat;
    int converged = 0;
    for (int it = 0; it < max_newton; ++it) {
        double f = -sqrt_shat, fp = 0.0;
        for (int i = 0; i < n_f; ++i) {
            double e = sqrt(mass[i] * mass[i] + xi * xi * p[i][0] * p[i][0]);
            f += e;
            fp += xi * p[i][0] * p[i][0] / e;
        }
        if (fabs(f) <= floor_res) {
            converged = 1;
            break;
        }
        double step = f / fp;
        xi = xi - step;
        if (fabs(step) <= 1e-15 * xi) {
            converged = 1;
            break;
        }
    }
    if (!converged) {
        *weight = 0.0;
        return 1;
    }

    double sum_abs = 0.0, prod_ratio = 1.0, sum_sq_over_e = 0.0;
    for (int i = 0; i < n_f; ++i) {
        double e = sqrt(mass[i] * mass[i] + xi * xi * p[i][0] * p[i][0]);
        k[4 * i + 0] = e;
        k[4 * i + 1] = xi * p[i][1];
        k[4 * i + 2] = xi * p[i][2];
        k[4 * i + 3] = xi * p[i][3];
        double a = sqrt(k[4 * i + 1] * k[4 * i + 1] + k[4 * i + 2] * k[4 * i + 2]
                        + k[4 * i + 3] * k[4 * i + 3]);
        sum_abs += a;
        prod_ratio *= a / e;
        sum_sq_over_e += a * a / e;
    }
    *weight = w0 * pow(sum_abs / sqrt_shat, 2 * n_f - 3) * prod_ratio * sqrt_shat / sum_sq_over_e;
    return 0;
}

static double pseudorapidity(const double *k)
{
    double a = sqrt(k[1] * k[1] + k[2] * k[2] + k[3] * k[3]);
    return 0.5 * log((a + k[3]) / (a - k[3]));
}

static int near(double v, double cut)
{
    return fabs(v - cut) < 1e-9 * fabs(cut);
}

/* Fiducial cuts on the final-state gluons (slots 2 .. n_f-1): pT and
 * |eta| in the laboratory frame (rapidities shift by y_boost), Delta R
 * between every pair.  All inequalities are strict.  Returns 1 if passed. */
int mfo_cuts(const mfo_process *proc, int n_f, const double *k, double y_boost, int *near_edge)
{
    int pass = 1;
    *near_edge = 0;
    for (int i = 2; i < n_f; ++i) {
        const double *ki = k + 4 * i;
        if (proc->ptmin_g > 0.0) {
            double pt = sqrt(ki[1] * ki[1] + ki[2] * ki[2]);
            if (near(pt, proc->ptmin_g)) *near_edge = 1;
            if (!(pt > proc->ptmin_g)) pass = 0;
        }
        if (proc->etamax_g > 0.0) {
            double eta = fabs(pseudorapidity(ki) + y_boost);
            if (near(eta, proc->etamax_g)) *near_edge = 1;
            if (!(eta < proc->etamax_g)) pass = 0;
        }
    }
    if (proc->drmin_gg > 0.0) {
        for (int i = 2; i < n_f; ++i)
            for (int j = i + 1; j < n_f; ++j) {
                const double *ki = k + 4 * i, *kj = k + 4 * j;
                double deta = pseudorapidity(ki) - pseudorapidity(kj);
                double dphi = fabs(atan2(ki[2], ki[1]) - atan2(kj[2], kj[1]));
                if (dphi > PI)
                    dphi = 2.0 * PI - dphi;
                double dr = sqrt(deta * deta + dphi * dphi);
                if (near(dr, proc->drmin_gg)) *near_edge = 1;
                if (!(dr > proc->drmin_gg)) pass = 0;
            }
    }
    return pass;
}

/* Index of the interval [knot_i, knot_{i+1}) holding v, clamped to [0, n-2]. */
static int find_interval(const double *knots, int n, double v)
{
    int lo = 0, hi = n - 1;
    if (v < knots[0]) return 0;
    if (v >= knots[n - 1]) return n - 2;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (knots[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

/* Slope at knot i of data f over knots t: mean of the two adjacent secant
 * slopes inside, the one available secant at either end.  Only knots in
 * [first, last] count as existing. */
static double knot_slope(const double *t, const double *f, int i, int first, int last)
{
    if (i == first)
        return (f[i + 1] - f[i]) / (t[i + 1] - t[i]);
    if (i == last)
        return (f[i] - f[i - 1]) / (t[i] - t[i - 1]);
    return 0.5 * ((f[i] - f[i - 1]) / (t[i] - t[i - 1]) + (f[i + 1] - f[i]) / (t[i + 1] - t[i]));
}

/* Cubic Hermite on [t_i, t_{i+1}] with the slopes above. */
static double hermite(const double *t, const double *f, int i, int first, int last, double v)
{
    double h = t[i + 1] - t[i];
    double u = (v - t[i]) / h;
    double u2 = u * u, u3 = u2 * u;
    double h00 = 2.0 * u3 - 3.0 * u2 + 1.0;
    double h10 = u3 - 2.0 * u2 + u;
    double h01 = -2.0 * u3 + 3.0 * u2;
    double h11 = u3 - u2;
    double s0 = knot_slope(t, f, i, first, last);
    double s1 = knot_slope(t, f, i + 1, first, last);
    return h00 * f[i] + h10 * h * s0 + h01 * f[i + 1] + h11 * h * s1;
}

static double pdf_table_value(const mfo_pdf_grid *g, const double *table, double x, double q2)
{
    double lx = log(x), lq = log(q2);
    int kx = find_interval(g->log_x, g->n_x, lx);
    int mq = find_interval(g->log_q2, g->n_q2, lq);

    /* Rows m-1 .. m+2 of the Q^2 stencil that exist in the grid. */
    int first = mq - 1 < 0 ? 0 : mq - 1;
    int last = mq + 2 > g->n_q2 - 1 ? g->n_q2 - 1 : mq + 2;
    double rowval[64];
    for (int r = first; r <= last; ++r) {
        const double *row = table + (size_t)r * g->n_x;
        rowval[r - first] = hermite(g->log_x, row, kx, 0, g->n_x - 1, lx);
    }
    return hermite(g->log_q2 + first, rowval, mq - first, 0, last - first, lq);
}

double mfo_pdf_xf(const mfo_pdf_grid *g, double x, double q2)
{
    return pdf_table_value(g, g->xf, x, q2);
}

double mfo_pdf_xq(const mfo_pdf_grid *g, int flavour, double x, double q2)
{
    if (!g->xq || flavour < 0 || flavour > 3)
        return NAN;
    return pdf_table_value(g, g->xq + (size_t)flavour * g->n_q2 * g->n_x, x, q2);
}
