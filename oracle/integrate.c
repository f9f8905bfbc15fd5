/*
 * integrate.c -- oracle: per-event weight, VEGAS iterations, combination,
 * and the closed-form gradient check for g g -> t tbar.
 * Test infrastructure only (see mfo.h).
 *
 * Each event follows the paper's pipeline (Sec. 2.2): random numbers ->
 * VEGAS map -> partonic kinematics -> phase space (Sec. 2.4) -> cuts ->
 * PDFs -> matrix element (Sec. 2.3) -> weight; the hadronic cross section is
 * the convolution L(x1, x2) (x) sigma_hat of Fig. 1.  Iterations accumulate
 * sum w, sum w^2 and the per-bin sum of w^2 used to refine the grid.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include "mfo.h"

static const double PI = 3.14159265358979323846;
static const double GEV2_TO_PB = 0.3893793721e9;   /* (hbar c)^2 in GeV^2 pb */

int mfo_n_dims(int n_g)
{
    return 2 + 3 * n_g - 4;
}

/* Neumaier's compensated summation, left to right. */
double mfo_neumaier_sum(int n, const double *v)
{
    double s = 0.0, c = 0.0;
    for (int i = 0; i < n; ++i) {
        double t = s + v[i];
        if (fabs(s) >= fabs(v[i]))
            c += (s - t) + v[i];
        else
            c += (v[i] - t) + s;
        s = t;
    }
    return s + c;
}

typedef struct { double s, c; } neumaier;

static void nm_add(neumaier *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double nm_value(const neumaier *a)
{
    return a->s + a->c;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i)
        f *= (double)i;
    return f;
}

/* Where the interpolated x g(x) passes close to zero (the cubic overshoots
 * below zero in the last interval towards x = 1) its relative value is
 * ill-conditioned: |d ln(x g)/d ln x| above 1e3 means that a one-ulp change
 * of ln x moves the result by more than ~1e-13.  Estimated by a central
 * difference of the interpolant itself with relative step 1e-7 in x. */
static double pdf_value(const mfo_pdf_grid *pdf, int table, double x, double q2)
{
    return table < 0 ? mfo_pdf_xf(pdf, x, q2) : mfo_pdf_xq(pdf, table, x, q2);
}

static int table_ill_conditioned(const mfo_pdf_grid *pdf, int table, double x, double q2)
{
    double h = 1e-7;
    double up = pdf_value(pdf, table, x * (1.0 + h), q2);
    double dn = pdf_value(pdf, table, x * (1.0 - h), q2);
    if (up == 0.0 || dn == 0.0 || (up > 0.0) != (dn > 0.0))
        return 1;
    double kappa = fabs(log(fabs(up)) - log(fabs(dn))) / (2.0 * h);
    return kappa > 1e3;
}

/* The gluon table (table -1) and, for p p, the four quark tables. */
static int pdf_ill_conditioned(const mfo_pdf_grid *pdf, double x, double q2, int quarks)
{
    for (int t = -1; t < (quarks ? 4 : 0); ++t)
        if (table_ill_conditioned(pdf, t, x, q2))
            return 1;
    return 0;
}

/* Everything after the VEGAS map: x = mapped variables, jac = J_V. */
static double weight_from_x(const mfo_process *proc, double sqrt_s,
                            const mfo_pdf_grid *pdf, double jac, mfo_event *ev)
{
    int n_g = proc->n_g;
    int n_f = n_g;                         /* t, tbar and n_g - 2 gluons */
    double m = proc->m_top;
    ev->jac = jac;
    ev->x1 = ev->x[0];
    ev->x2 = ev->x[1];
    ev->shat = ev->x1 * ev->x2 * sqrt_s * sqrt_s;
    ev->pass_threshold = 0;
    ev->pass_cuts = 0;
    ev->newton_fail = 0;
    ev->near_edge = 0;
    ev->ill_conditioned = 0;
    ev->colour_kappa = 0.0;
    ev->newton_kappa = 0.0;
    ev->ps_weight = ev->f1 = ev->f2 = ev->me2 = 0.0;
    ev->me2_q[0] = ev->me2_q[1] = ev->lum_q[0] = ev->lum_q[1] = 0.0;
    ev->w = 0.0;
    memset(ev->k, 0, sizeof(ev->k));

    /* Partonic threshold: below (2 m_t)^2 the event has zero weight. */
    if (!(ev->shat > (2.0 * m) * (2.0 * m)))
        return 0.0;
    ev->pass_threshold = 1;

    double sqrt_shat = sqrt(ev->shat);
    double mass[MFO_MAX_F] = { m, m, 0.0, 0.0 };
    double W;
    if (mfo_phase_space(n_f, mass, sqrt_shat, ev->x + 2, 50, &ev->k[0][0], &W) != 0) {
        ev->newton_fail = 1;
        return 0.0;
    }
    ev->ps_weight = W;
    /* Condition number of the rescaling root xi (Sec. 2.4 massive step):
     * F(xi) = sum_i sqrt(m_i^2 + xi^2 E_i^2) - sqrt(s_hat) is known only to
     * its rounding (the residual floor of the Newton stop), so xi is fixed
     * only to that over xi F'(xi) = sum_i |k_i|^2 / k_i^0, relative to
     * sqrt(s_hat).  Close to threshold this becomes large (1 / beta^2 for
     * t tbar). */
    {
        double den = 0.0;
        for (int i = 0; i < n_f; ++i) {
            double a2 = ev->k[i][1] * ev->k[i][1] + ev->k[i][2] * ev->k[i][2] + ev->k[i][3] * ev->k[i][3];
            den += a2 / ev->k[i][0];
        }
        ev->newton_kappa = sqrt_shat / den;
    }

    double y_boost = 0.5 * log(ev->x1 / ev->x2);
    int near_edge = 0;
    int pass = mfo_cuts(proc, n_f, &ev->k[0][0], y_boost, &near_edge);
    ev->near_edge = near_edge;
    if (!pass)
        return 0.0;
    ev->pass_cuts = 1;

    double q2 = proc->mu_f * proc->mu_f;
    ev->f1 = mfo_pdf_xf(pdf, ev->x1, q2) / ev->x1;
    ev->f2 = mfo_pdf_xf(pdf, ev->x2, q2) / ev->x2;
    const int pp = proc->initial == 1;
    ev->ill_conditioned = pdf_ill_conditioned(pdf, ev->x1, q2, pp) || pdf_ill_conditioned(pdf, ev->x2, q2, pp);

    /* All-outgoing momenta for the amplitude: t, tbar, -p_a, -p_b, gluons. */
    double p[(MFO_MAX_G + 2) * 4];
    double e = 0.5 * sqrt_shat;
    memcpy(p, ev->k[0], sizeof(double) * 4);
    memcpy(p + 4, ev->k[1], sizeof(double) * 4);
    double pa[4] = { -e, 0.0, 0.0, -e };
    double pb[4] = { -e, 0.0, 0.0, e };
    memcpy(p + 8, pa, sizeof(pa));
    memcpy(p + 12, pb, sizeof(pb));
    for (int i = 2; i < n_f; ++i)
        memcpy(p + 4 * (2 + i), ev->k[i], sizeof(double) * 4);

    double gs2 = 4.0 * PI * proc->alpha_s;
    double sum;
    if (proc->helicity == 1) {
        int cfg_ok = (proc->colour != 2 && proc->colour != 3) || ev->colour_cfg >= 0;
        sum = ev->hel_cfg >= 0 && cfg_ok
                  ? (double)mfo_hel_count(n_g) * mfo_me2_hel(n_g, p, m, proc->w_top, proc->colour,
                                                             ev->colour_cfg, ev->hel_cfg, &ev->colour_kappa)
                  : NAN;
    } else if (proc->colour == 2 || proc->colour == 3)
        sum = ev->colour_cfg >= 0 ? mfo_me2_sum_sampled(n_g, p, m, proc->w_top, proc->colour, ev->colour_cfg,
                                                        &ev->colour_kappa)
                                  : NAN;
    else if (proc->colour == 1)
        sum = mfo_me2_sum_lc(n_g, p, m, proc->w_top);
    else
        sum = mfo_me2_sum(n_g, p, m, proc->w_top);
    /* average over 2 x 2 initial helicities and 8 x 8 initial colours,
     * symmetry factor 1/(n_g - 2)! for identical final-state gluons */
    ev->me2 = pow(gs2, n_g) * sum / (4.0 * 64.0 * factorial(n_g - 2));
    ev->me2_q[0] = ev->me2_q[1] = 0.0;
    ev->lum_q[0] = ev->lum_q[1] = 0.0;
    if (pp) {
        /* q qbar channels: the quark from beam 1 (u ubar, d dbar) or from beam 2
         * (ubar u, dbar d); average over 2 x 2 helicities and 3 x 3 colours;
         * t tbar (n_g = 2), t tbar g (n_g = 3) or t tbar g g (n_g = 4) */
        double pr[(MFO_MAX_G + 2) * 4];
        memcpy(pr, p, sizeof(double) * 4 * (n_g + 2));
        memcpy(pr + 8, pb, sizeof(pb));
        memcpy(pr + 12, pa, sizeof(pa));
        if (n_g == 2) {
            ev->me2_q[0] = gs2 * gs2 * mfo_me2_qqbar_ttx(p, m) / 36.0;
            ev->me2_q[1] = gs2 * gs2 * mfo_me2_qqbar_ttx(pr, m) / 36.0;
        } else if (n_g == 3) {
            ev->me2_q[0] = gs2 * gs2 * gs2 * mfo_me2_qqbar_ttxg(p, m, proc->w_top) / 36.0;
            ev->me2_q[1] = gs2 * gs2 * gs2 * mfo_me2_qqbar_ttxg(pr, m, proc->w_top) / 36.0;
        } else if (n_g == 4) {
            /* and 1/2! for the two identical gluons */
            const double g8 = gs2 * gs2 * gs2 * gs2;
            ev->me2_q[0] = g8 * mfo_me2_qqbar_ttxgg(p, m, proc->w_top) / (36.0 * 2.0);
            ev->me2_q[1] = g8 * mfo_me2_qqbar_ttxgg(pr, m, proc->w_top) / (36.0 * 2.0);
        } else {
            ev->me2_q[0] = ev->me2_q[1] = NAN;   /* q qbar channels with more gluons: not in the oracle */
        }
        double x1 = ev->x1, x2 = ev->x2;
        double u1 = mfo_pdf_xq(pdf, 0, x1, q2) / x1, ub1 = mfo_pdf_xq(pdf, 1, x1, q2) / x1;
        double d1 = mfo_pdf_xq(pdf, 2, x1, q2) / x1, db1 = mfo_pdf_xq(pdf, 3, x1, q2) / x1;
        double u2 = mfo_pdf_xq(pdf, 0, x2, q2) / x2, ub2 = mfo_pdf_xq(pdf, 1, x2, q2) / x2;
        double d2 = mfo_pdf_xq(pdf, 2, x2, q2) / x2, db2 = mfo_pdf_xq(pdf, 3, x2, q2) / x2;
        ev->lum_q[0] = u1 * ub2 + d1 * db2;
        ev->lum_q[1] = ub1 * u2 + db1 * d2;
    }

    ev->w = jac * W * ev->f1 * ev->f2 * ev->me2 / (2.0 * ev->shat) * GEV2_TO_PB;
    if (pp)
        ev->w += jac * W * (ev->lum_q[0] * ev->me2_q[0] + ev->lum_q[1] * ev->me2_q[1]) / (2.0 * ev->shat) * GEV2_TO_PB;
    return ev->w;
}

double mfo_event_weight(const mfo_process *proc, double sqrt_s,
                        const mfo_pdf_grid *pdf, int n_bins, const double *grid,
                        uint64_t seed, int iter, uint64_t event, mfo_event *ev)
{
    int D = mfo_n_dims(proc->n_g);
    uint64_t k53[MFO_MAX_DIM];
    double delta[MFO_MAX_DIM];
    mfo_event_k53(seed, (uint32_t)iter, event, D, k53);
    for (int d = 0; d < D; ++d) {
        ev->y[d] = (double)k53[d] * 0x1p-53;
        mfo_bin_from_k53(k53[d], n_bins, &ev->bin[d], &delta[d]);
    }
    double jac = mfo_vegas_map(D, n_bins, grid, ev->bin, delta, ev->x);
    ev->colour_cfg = proc->colour == 2 ? mfo_colour_config(proc->n_g, seed, (uint32_t)iter, event)
                   : proc->colour == 3 ? mfo_flow_config(proc->n_g, seed, (uint32_t)iter, event) : -1;
    ev->hel_cfg = proc->helicity == 1 ? mfo_hel_config(proc->n_g, seed, (uint32_t)iter, event) : -1;
    return weight_from_x(proc, sqrt_s, pdf, jac, ev);
}

/* Caller uniforms carry no event counter: with colour = 2 the weight is NaN. */
double mfo_event_weight_y(const mfo_process *proc, double sqrt_s,
                          const mfo_pdf_grid *pdf, int n_bins, const double *grid,
                          const double *y, mfo_event *ev)
{
    int D = mfo_n_dims(proc->n_g);
    double delta[MFO_MAX_DIM];
    for (int d = 0; d < D; ++d) {
        ev->y[d] = y[d];
        double t = y[d] * (double)n_bins;
        int b = (int)floor(t);
        if (b > n_bins - 1) b = n_bins - 1;
        if (b < 0) b = 0;
        ev->bin[d] = b;
        delta[d] = t - (double)b;
    }
    double jac = mfo_vegas_map(D, n_bins, grid, ev->bin, delta, ev->x);
    ev->colour_cfg = -1;
    ev->hel_cfg = -1;
    return weight_from_x(proc, sqrt_s, pdf, jac, ev);
}

/* Inverse-variance weighted mean of the iteration estimates: iterations
 * with V_j > 0 enter with weight 1/V_j; sigma_I = (sum 1/V_j)^(-1/2);
 * chi^2/dof = sum (I_j - I)^2 / V_j / (n_used - 1).  Any n_iter. */
void mfo_combine(int n_iter, const double *I, const double *V,
                 double *sigma, double *err, double *chi2_dof)
{
    int cap = n_iter > 0 ? n_iter : 1;
    double *num = malloc(sizeof(double) * (size_t)cap);
    double *den = malloc(sizeof(double) * (size_t)cap);
    double *chi = malloc(sizeof(double) * (size_t)cap);
    int n = 0;
    for (int j = 0; j < n_iter; ++j) {
        if (V[j] > 0.0) {
            num[n] = I[j] / V[j];
            den[n] = 1.0 / V[j];
            ++n;
        }
    }
    if (n == 0) {
        *sigma = n_iter > 0 ? I[n_iter - 1] : 0.0;
        *err = 0.0;
        *chi2_dof = 0.0;
    } else {
        double snum = mfo_neumaier_sum(n, num), sden = mfo_neumaier_sum(n, den);
        double mean = snum / sden;
        *sigma = mean;
        *err = 1.0 / sqrt(sden);
        int k = 0;
        for (int j = 0; j < n_iter; ++j)
            if (V[j] > 0.0)
                chi[k++] = (I[j] - mean) * (I[j] - mean) / V[j];
        *chi2_dof = n > 1 ? mfo_neumaier_sum(k, chi) / (double)(n - 1) : 0.0;
    }
    free(num);
    free(den);
    free(chi);
}

typedef struct {
    const mfo_process *proc;
    double sqrt_s;
    const mfo_pdf_grid *pdf;
    int n_bins, D, iter;
    uint64_t seed, e0, e1;
    const double *grid;
    double *weights;              /* may be NULL */
    neumaier sw, sw2;
    double *hist;                 /* [D][n_bins] */
    double w_max;
    int64_t n_pass, n_fail, n_near;
} worker;

static void *run_worker(void *arg)
{
    worker *wk = (worker *)arg;
    mfo_event ev;
    for (uint64_t e = wk->e0; e < wk->e1; ++e) {
        double w = mfo_event_weight(wk->proc, wk->sqrt_s, wk->pdf, wk->n_bins, wk->grid,
                                    wk->seed, wk->iter, e, &ev);
        nm_add(&wk->sw, w);
        nm_add(&wk->sw2, w * w);
        for (int d = 0; d < wk->D; ++d)
            wk->hist[d * wk->n_bins + ev.bin[d]] += w * w;
        if (w > wk->w_max) wk->w_max = w;
        if (ev.pass_cuts) wk->n_pass++;
        if (ev.newton_fail) wk->n_fail++;
        if (ev.near_edge) wk->n_near++;
        if (wk->weights) wk->weights[e] = w;
    }
    return NULL;
}

int mfo_integrate(const mfo_process *proc, double sqrt_s, const mfo_pdf_grid *pdf,
                  uint64_t n_events, int n_iter, uint64_t seed, int start_iter,
                  int n_bins, double alpha, int n_threads,
                  double *grid, double *iter_sigma, double *iter_var,
                  double *hist_last, double *weights_last, mfo_result *res)
{
    if (n_events < 2 || n_iter < 1 || n_iter > 256 || n_bins < 2 || n_bins > 1024 || n_threads < 1)
        return -1;
    int D = mfo_n_dims(proc->n_g);
    double *I = calloc((size_t)n_iter, sizeof(double));
    double *V = calloc((size_t)n_iter, sizeof(double));
    double *hist = calloc((size_t)D * n_bins, sizeof(double));
    double *grid_new = calloc((size_t)D * (n_bins + 1), sizeof(double));
    worker *wk = calloc((size_t)n_threads, sizeof(worker));
    pthread_t *th = calloc((size_t)n_threads, sizeof(pthread_t));
    double w_max = 0.0;
    int64_t n_pass = 0, n_fail = 0, n_near = 0;

    for (int j = 0; j < n_iter; ++j) {
        int iter = start_iter + j;
        int is_last = (j == n_iter - 1);
        for (int t = 0; t < n_threads; ++t) {
            worker *w = &wk[t];
            memset(w, 0, sizeof(*w));
            w->proc = proc;
            w->sqrt_s = sqrt_s;
            w->pdf = pdf;
            w->n_bins = n_bins;
            w->D = D;
            w->iter = iter;
            w->seed = seed;
            w->e0 = n_events * (uint64_t)t / (uint64_t)n_threads;
            w->e1 = n_events * (uint64_t)(t + 1) / (uint64_t)n_threads;
            w->grid = grid;
            w->weights = is_last ? weights_last : NULL;
            w->hist = calloc((size_t)D * n_bins, sizeof(double));
            pthread_create(&th[t], NULL, run_worker, w);
        }
        neumaier sw = { 0, 0 }, sw2 = { 0, 0 };
        memset(hist, 0, sizeof(double) * (size_t)D * n_bins);
        for (int t = 0; t < n_threads; ++t) {
            pthread_join(th[t], NULL);
            nm_add(&sw, nm_value(&wk[t].sw));
            nm_add(&sw2, nm_value(&wk[t].sw2));
            for (int b = 0; b < D * n_bins; ++b)
                hist[b] += wk[t].hist[b];
            if (is_last) {
                if (wk[t].w_max > w_max) w_max = wk[t].w_max;
                n_pass += wk[t].n_pass;
                n_fail += wk[t].n_fail;
                n_near += wk[t].n_near;
            }
            free(wk[t].hist);
        }
        double N = (double)n_events;
        I[j] = nm_value(&sw) / N;
        V[j] = (nm_value(&sw2) / N - I[j] * I[j]) / (N - 1.0);
        if (iter_sigma) iter_sigma[j] = I[j];
        if (iter_var) iter_var[j] = V[j];
        if (is_last && hist_last)
            memcpy(hist_last, hist, sizeof(double) * (size_t)D * n_bins);
        mfo_vegas_refine(D, n_bins, alpha, hist, grid, grid_new);
        memcpy(grid, grid_new, sizeof(double) * (size_t)D * (n_bins + 1));
    }
    mfo_combine(n_iter, I, V, &res->sigma, &res->sigma_err, &res->chi2_dof);
    res->w_max = w_max;
    res->n_pass = n_pass;
    res->n_newton_fail = n_fail;
    res->n_near_edge = n_near;
    free(I); free(V); free(hist); free(grid_new); free(wk); free(th);
    return 0;
}

/* Weights of a list of events, split over threads (each event is
 * independent; the results do not depend on the split). */
typedef struct {
    const mfo_process *proc;
    double sqrt_s;
    const mfo_pdf_grid *pdf;
    int n_bins, iter;
    uint64_t seed, i0, i1;
    const double *grid;
    const uint64_t *ids;
    double *w;
    int *flags;
    double *kappa;
} list_worker;

static void *run_list(void *arg)
{
    list_worker *lw = (list_worker *)arg;
    mfo_event ev;
    for (uint64_t i = lw->i0; i < lw->i1; ++i) {
        lw->w[i] = mfo_event_weight(lw->proc, lw->sqrt_s, lw->pdf, lw->n_bins, lw->grid, lw->seed,
                                    lw->iter, lw->ids[i], &ev);
        lw->flags[i] = ev.pass_threshold | ev.newton_fail << 1 | ev.pass_cuts << 2 | ev.near_edge << 3
                       | ev.ill_conditioned << 4 | (ev.colour_kappa > 50.0) << 5
                       | (ev.newton_kappa > 1e3) << 6;
        if (lw->kappa)
            lw->kappa[i] = ev.newton_kappa;
    }
    return NULL;
}

int mfo_event_weights(const mfo_process *proc, double sqrt_s, const mfo_pdf_grid *pdf, int n_bins,
                      const double *grid, uint64_t seed, int iter, uint64_t n, const uint64_t *ids,
                      int n_threads, double *w, int *flags, double *newton_kappa)
{
    if (n_threads < 1)
        return -1;
    list_worker *lw = calloc((size_t)n_threads, sizeof(list_worker));
    pthread_t *th = calloc((size_t)n_threads, sizeof(pthread_t));
    for (int t = 0; t < n_threads; ++t) {
        list_worker *x = &lw[t];
        x->proc = proc;
        x->sqrt_s = sqrt_s;
        x->pdf = pdf;
        x->n_bins = n_bins;
        x->iter = iter;
        x->seed = seed;
        x->i0 = n * (uint64_t)t / (uint64_t)n_threads;
        x->i1 = n * (uint64_t)(t + 1) / (uint64_t)n_threads;
        x->grid = grid;
        x->ids = ids;
        x->w = w;
        x->flags = flags;
        x->kappa = newton_kappa;
        pthread_create(&th[t], NULL, run_list, x);
    }
    for (int t = 0; t < n_threads; ++t)
        pthread_join(th[t], NULL);
    free(lw);
    free(th);
    return 0;
}

/* Closed-form LO g g -> t tbar (zero width), averaged |M|^2 / g^4 in terms of
 * tau_{1,2} = (1 -/+ beta cos theta)/2 and rho = 4 m^2 / s:
 *   (1/(6 tau1 tau2) - 3/8) (tau1^2 + tau2^2 + rho - rho^2/(4 tau1 tau2))
 * (Glueck, Owens, Reya 1978; Ellis, Stirling, Webber, QCD and Collider
 * Physics).  With the uniforms held fixed the top direction does not move
 * when m_t changes, so d w / d m_t follows by differentiating beta, rho,
 * tau_{1,2} and the two-body weight beta/(8 pi). */
double mfo_ttx_dweight_dmt_analytic(const mfo_process *proc, double sqrt_s,
                                    const mfo_pdf_grid *pdf, int n_bins,
                                    const double *grid, const double *y,
                                    double *w_out)
{
    mfo_event ev;
    int D = 4;
    double delta[4];
    for (int d = 0; d < D; ++d) {
        double t = y[d] * (double)n_bins;
        int b = (int)floor(t);
        if (b > n_bins - 1) b = n_bins - 1;
        if (b < 0) b = 0;
        ev.bin[d] = b;
        delta[d] = t - (double)b;
    }
    double jac = mfo_vegas_map(D, n_bins, grid, ev.bin, delta, ev.x);
    double x1 = ev.x[0], x2 = ev.x[1];
    double s = x1 * x2 * sqrt_s * sqrt_s;
    double m = proc->m_top;
    double rho = 4.0 * m * m / s;
    if (!(rho < 1.0)) {
        *w_out = 0.0;
        return 0.0;
    }
    double beta = sqrt(1.0 - rho);
    double c = 2.0 * ev.x[2] - 1.0;
    double t1 = 0.5 * (1.0 - beta * c), t2 = 0.5 * (1.0 + beta * c);
    double P = t1 * t2;
    double A = 1.0 / (6.0 * P) - 3.0 / 8.0;
    double B = t1 * t1 + t2 * t2 + rho - rho * rho / (4.0 * P);
    double F = A * B;
    double q2 = proc->mu_f * proc->mu_f;
    double f1 = mfo_pdf_xf(pdf, x1, q2) / x1, f2 = mfo_pdf_xf(pdf, x2, q2) / x2;
    double gs2 = 4.0 * PI * proc->alpha_s;
    double w = jac * (beta / (8.0 * PI)) * f1 * f2 * gs2 * gs2 * F / (2.0 * s) * GEV2_TO_PB;

    double drho = 8.0 * m / s;
    double dbeta = -drho / (2.0 * beta);
    double dt1 = -0.5 * c * dbeta, dt2 = 0.5 * c * dbeta;
    double dP = dt1 * t2 + t1 * dt2;
    double dA = -dP / (6.0 * P * P);
    double dB = 2.0 * t1 * dt1 + 2.0 * t2 * dt2 + drho - 2.0 * rho * drho / (4.0 * P)
                + rho * rho * dP / (4.0 * P * P);
    double dF = dA * B + A * dB;
    *w_out = w;
    return w * (dbeta / beta + dF / F);
}
