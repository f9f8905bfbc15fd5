/*
 * unweight.c -- oracle: hit-or-miss unweighting of weighted events and their
 * lab-frame records.  Test infrastructure only (see mfo.h).
 *
 * Sec. 2.5 turns the weighted events of the integration into unweighted
 * ones for the LHE output: an event of weight w is kept with probability
 * |w| / w_max, after which it carries a unit weight with the sign of w.
 * The uniform u_e deciding event e is the first 53-bit uniform of the Philox
 * block b = 0x80000000 of that event's counter (e mod 2^32, e >> 32, iter,
 * b); the integrand itself draws only from blocks 0 .. ceil(D/2) - 1.
 *
 * The record of a kept event lists the momenta in the hadronic (lab) frame:
 * the two incoming gluons x1 sqrt(s)/2 (1, 0, 0, +1) and x2 sqrt(s)/2
 * (1, 0, 0, -1), then t, tbar and the final gluons, obtained from the
 * partonic CM momenta by the longitudinal boost of rapidity
 * y = ln(x1 / x2) / 2 (Fig. 1: the partonic system moves along the beam).
 */
#include <math.h>
#include <string.h>
#include "mfo.h"

double mfo_unweight_uniform(uint64_t seed, uint32_t iter, uint64_t event)
{
    uint32_t ctr[4] = { (uint32_t)event, (uint32_t)(event >> 32), iter, 0x80000000u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t r[4];
    mfo_philox4x32_10(ctr, key, r);
    uint64_t k = ((((uint64_t)r[0]) << 32) | (uint64_t)r[1]) >> 11;
    return (double)k * 0x1p-53;
}

uint64_t mfo_unweight(uint64_t n, const double *w, double w_max, uint64_t seed, uint32_t iter,
                      signed char *keep, uint64_t *n_over)
{
    uint64_t kept = 0, over = 0;
    for (uint64_t e = 0; e < n; ++e) {
        double a = fabs(w[e]);
        double u = mfo_unweight_uniform(seed, iter, e);
        int k = u * w_max < a;
        keep[e] = (signed char)(k ? (w[e] > 0.0 ? 1 : -1) : 0);
        kept += (uint64_t)k;
        over += (uint64_t)(a > w_max);
    }
    if (n_over)
        *n_over = over;
    return kept;
}

int mfo_lab_event(const mfo_process *proc, double sqrt_s, int n_bins, const double *grid,
                  uint64_t seed, int iter, uint64_t event, double *p)
{
    int n_f = proc->n_g;
    int D = mfo_n_dims(proc->n_g);
    uint64_t k53[MFO_MAX_DIM];
    int bin[MFO_MAX_DIM];
    double delta[MFO_MAX_DIM], x[MFO_MAX_DIM];
    mfo_event_k53(seed, (uint32_t)iter, event, D, k53);
    for (int d = 0; d < D; ++d)
        mfo_bin_from_k53(k53[d], n_bins, &bin[d], &delta[d]);
    mfo_vegas_map(D, n_bins, grid, bin, delta, x);
    double x1 = x[0], x2 = x[1];
    double shat = x1 * x2 * sqrt_s * sqrt_s;
    double m = proc->m_top;
    memset(p, 0, sizeof(double) * 4 * (n_f + 2));
    if (!(shat > (2.0 * m) * (2.0 * m)))
        return 1;
    double mass[MFO_MAX_F] = { m, m, 0.0, 0.0 };
    double k[MFO_MAX_F][4], W;
    if (mfo_phase_space(n_f, mass, sqrt(shat), x + 2, 50, &k[0][0], &W) != 0)
        return 2;
    double eb = 0.5 * sqrt_s;
    double pa[4] = { x1 * eb, 0.0, 0.0, x1 * eb };
    double pb[4] = { x2 * eb, 0.0, 0.0, -x2 * eb };
    memcpy(p, pa, sizeof(pa));
    memcpy(p + 4, pb, sizeof(pb));
    double y = 0.5 * log(x1 / x2);
    double ch = cosh(y), sh = sinh(y);
    for (int i = 0; i < n_f; ++i) {
        double *q = p + 4 * (2 + i);
        q[0] = k[i][0] * ch + k[i][3] * sh;
        q[1] = k[i][1];
        q[2] = k[i][2];
        q[3] = k[i][3] * ch + k[i][0] * sh;
    }
    return 0;
}
