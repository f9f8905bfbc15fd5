/*
 * mfo.h -- plain FP64 CPU oracle for the per-event MadFlow integrand
 * (Carrazza, Cruz-Martinez, Rossi, Zaro, arXiv:2106.10279).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or constant
 * with the GPU path.
 *
 * The oracle follows the event-generation pipeline of Sec. 2.2 (random
 * numbers -> phase space -> PDFs -> matrix element -> accumulation), with
 * VEGAS importance sampling for the integrator (Sec. 1, ingredient (i)), a
 * flat phase-space generator of the RAMBO family (Sec. 2.4), log-bicubic
 * PDF interpolation (PDFFlow's role, Sec. 1 ingredient (ii)) and tree-level
 * helicity amplitudes summed over helicities (Sec. 2.3).  Every function is
 * written one event at a time, in double precision, for clarity rather than
 * speed; the library is compiled with -O2 -ffp-contract=off.
 *
 * Particle slots (all momenta are 4-vectors (E, px, py, pz), metric +---):
 *   final state in the partonic centre-of-mass frame: 0 = t, 1 = tbar,
 *   2.. = final-state gluons.  Amplitude routines take all momenta as
 *   outgoing: [t, tbar, g_1, ..., g_n] where g_1, g_2 are the crossed
 *   incoming gluons (momentum -p_a, -p_b).
 */
#ifndef MFO_H
#define MFO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFO_MAX_G   5          /* gluons in the process (2 .. 5)             */
#define MFO_MAX_F   5          /* final-state particles                      */
#define MFO_MAX_DIM 13         /* integration dimensions 2 + 3 n_f - 4       */

typedef struct {
    int    n_g;                /* total gluons: 2 (tt), 3 (ttg), 4 (ttgg)     */
    double m_top, w_top;       /* GeV                                          */
    double alpha_s;            /* fixed strong coupling                        */
    double mu_f;               /* factorisation scale, GeV                     */
    double ptmin_g;            /* gluon pT cut (GeV); <= 0 disables            */
    double etamax_g;           /* gluon |eta| cut; <= 0 disables               */
    double drmin_gg;           /* Delta R between final gluons; <= 0 disables  */
    int    colour;             /* 0: full colour sum; 1: leading colour;
                                  2: colour Monte Carlo (one sampled assignment);
                                  3: Monte Carlo over colour flows          */
    int    helicity;           /* 0: sum over helicity configurations;
                                  1: Monte Carlo over them (one sampled
                                  configuration of the linear basis)         */
    int    initial;            /* 0: g g initial state; 1: p p, the g g channel
                                  plus q qbar from the quark tables (u, ubar,
                                  d, dbar; n_g = 2 only)                     */
} mfo_process;

typedef struct {
    int n_x, n_q2;
    const double *log_x;       /* [n_x]  ascending ln x knots                  */
    const double *log_q2;      /* [n_q2] ascending ln Q^2 knots                */
    const double *xf;          /* [n_q2][n_x] row-major values of x g(x, Q^2)  */
    const double *xq;          /* [4][n_q2][n_x] x q(x, Q^2) for u, ubar, d,
                                  dbar, or NULL (gluons only)                 */
} mfo_pdf_grid;

typedef struct {
    double y[MFO_MAX_DIM];     /* uniforms in [0,1)                            */
    int    bin[MFO_MAX_DIM];   /* VEGAS bin per dimension                      */
    double x[MFO_MAX_DIM];     /* mapped variables                             */
    double jac;                /* VEGAS Jacobian J_V                           */
    double x1, x2, shat;
    double ps_weight;          /* phase-space weight W (massive)               */
    double f1, f2;             /* g(x1), g(x2) number densities                */
    double me2;                /* averaged |M|^2 (with g_s powers)             */
    double w;                  /* event weight in pb                           */
    double k[MFO_MAX_F][4];    /* final-state momenta, partonic CM frame       */
    int    pass_threshold;
    int    pass_cuts;
    int    newton_fail;
    int    near_edge;          /* a cut variable lies within 1e-9 of its cut   */
    int    ill_conditioned;    /* |d ln(x g) / d ln x| > 1e3 at x1 or x2      */
    int64_t colour_cfg;        /* colour = 2, 3: the event's assignment, flow   */
    double colour_kappa;       /* colour = 2, 3: condition number of the sum   */
    int    hel_cfg;            /* helicity = 1: the event's configuration      */
    double me2_q[2];           /* p p: averaged q qbar |M|^2 (with g_s powers),
                                  quark from beam 1 / from beam 2             */
    double lum_q[2];           /* p p: sum over u, d of q(x1) qbar(x2) and of
                                  qbar(x1) q(x2) number densities            */
    double newton_kappa;       /* condition number of the mass-rescaling root:
                                  sqrt(s_hat) / (xi F'(xi)) = sqrt(s_hat) /
                                  sum_i |k_i|^2 / E_i (1 for massless momenta,
                                  1 / beta^2 for t tbar); 0 below threshold */
} mfo_event;

typedef struct {
    double sigma, sigma_err, chi2_dof, w_max;
    int64_t n_pass, n_newton_fail, n_near_edge;
} mfo_result;

/* ---- random numbers (Philox4x32-10, Salmon et al. SC'11) ---------------- */
void mfo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* 53-bit integers k_d (uniform y_d = k_d 2^-53) for event e of iteration it. */
void mfo_event_k53(uint64_t seed, uint32_t iter, uint64_t event, int n_dim, uint64_t *k53);
void mfo_bin_from_k53(uint64_t k53, int n_bins, int *bin, double *delta);

/* ---- VEGAS ------------------------------------------------------------- */
double mfo_vegas_map(int n_dim, int n_bins, const double *grid,
                     const int *bin, const double *delta, double *x);
void mfo_vegas_refine(int n_dim, int n_bins, double alpha, const double *hist,
                      const double *grid_in, double *grid_out);

/* ---- phase space -------------------------------------------------------- */
double mfo_massless_volume(int n_f, double shat);
/* Returns 0 on success, 1 if the mass-rescaling Newton iteration failed.   */
int mfo_phase_space(int n_f, const double *mass, double sqrt_shat,
                    const double *r, int max_newton, double *k, double *weight);
int mfo_cuts(const mfo_process *proc, int n_f, const double *k, double y_boost,
             int *near_edge);

/* ---- PDF ---------------------------------------------------------------- */
double mfo_pdf_xf(const mfo_pdf_grid *g, double x, double q2);
/* x q(x, Q^2) of quark table `flavour` (0 u, 1 ubar, 2 d, 3 dbar). */
double mfo_pdf_xq(const mfo_pdf_grid *g, int flavour, double x, double q2);

/* ---- colour and matrix element ----------------------------------------- */
int  mfo_n_orderings(int n_g);
void mfo_orderings(int n_g, int *perm);           /* [n_g!][n_g], 0-based     */
void mfo_colour_matrix(int n_g, double *C);       /* [n_g!][n_g!]            */
/* The same matrix from its brute-force first row and the relabelling
 * symmetry C_{sigma tau} = C_{id, sigma^-1 tau} (used for five gluons). */
void mfo_colour_matrix_relabel(int n_g, double *C);
/* q(pa) qbar(pb) -> t tbar: |M|^2 summed over helicities and colours, g = 1.
 * p: [4][4] all outgoing: t, tbar, -pa, -pb. */
double mfo_me2_qqbar_ttx(const double *p, double m);
/* q(pa) qbar(pb) -> t tbar g from its five Feynman diagrams (amplitudes.c):
 * the colour-stripped diagram amplitudes of helicity configuration hel[5]
 * (quark, antiquark, top, antitop spin; gluon helicity), amp[2 d] = Re,
 * [2 d + 1] = Im; ward != 0 replaces the gluon polarisation by its momentum.
 * p: [5][4] all outgoing: t, tbar, -pa, -pb, g. */
void mfo_qqbar_ttxg_diagrams(const double *p, double m, double width, const int *hel, int ward, double *amp);
/* The diagrams' colour factors for cols[5] = (quark colour, antiquark
 * anticolour, top colour, antitop anticolour, gluon adjoint index). */
void mfo_qqbar_ttxg_colour(const int *cols, double *c);
/* Sum over helicities and colour assignments of |sum_d C_d A_d|^2, g = 1. */
double mfo_me2_qqbar_ttxg(const double *p, double m, double width);
/* q(pa) qbar(pb) -> t tbar g g from its 36 Feynman diagrams (amplitudes.c),
 * 38 terms (the four-gluon vertex in its three colour structures):
 * the Lorentz parts of helicity configuration hel[6] (quark, antiquark, top,
 * antitop spin; gluon 1, gluon 2 helicity), amp[2 d], [2 d + 1]; ward = 1 or
 * 2 replaces that gluon's polarisation by its momentum.  p: [6][4] all
 * outgoing: t, tbar, -pa, -pb, g1, g2. */
void mfo_qqbar_ttxgg_terms(const double *p, double m, double width, const int *hel, int ward, double *amp);
/* The terms' colour factors for cols[6] = (quark colour, antiquark
 * anticolour, top colour, antitop anticolour, a1, a2). */
void mfo_qqbar_ttxgg_colour(const int *cols, double *c);
/* K_de = sum over colours of C_d conj(C_e), [38][38][re, im]. */
void mfo_qqbar_ttxgg_colour_matrix(double *K);
/* Sum over helicities and colours of |M|^2, g = 1. */
double mfo_me2_qqbar_ttxgg(const double *p, double m, double width);
/* Colour-dressed amplitude M_ij from Feynman rules with explicit SU(3)
 * indices for one assignment of gluon adjoint indices cols[n_g] (0 .. 7) and
 * helicity configuration hel: out[2 (3 i + j)] = Re M_ij, [+1] = Im, i the
 * top colour, j the antitop anticolour. */
void mfo_dressed_amplitude(int n_g, const double *p, double m, double width, const int *hel,
                           const int *cols, double *out);
/* Colour-ordered partial amplitudes for one helicity configuration.
 * p: [n_g+2][4] all-outgoing momenta; hel: [n_g+2] (0/1 for each slot);
 * ward_gluon >= 0 replaces that gluon's polarisation by its momentum.
 * A: [n_g!][2] (re, im), g_s = 1.                                           */
void mfo_partial_amplitudes(int n_g, const double *p, double m, double width,
                            const int *hel, int ward_gluon, double *A);
/* Sum over helicities and colours of |M|^2 with g_s = 1.                   */
double mfo_me2_sum(int n_g, const double *p, double m, double width);
/* Same sum for the listed helicity configurations, computed with fully
 * colour-dressed Feynman rules and an explicit loop over every external
 * colour assignment.  Used only to pin the colour decomposition.          */
double mfo_me2_sum_fullcolour(int n_g, const double *p, double m, double width,
                              int n_hel, const int *hel_list);
double mfo_me2_sum_hel(int n_g, const double *p, double m, double width,
                       int n_hel, const int *hel_list);
/* Leading-colour approximation (the paper names it, Sec. 3.2 on Fig. 4, as a way to
 * cheapen high-multiplicity matrix elements): the colour matrix replaced by
 * c_LC times the identity, c_LC = (N^2 - 1) N^(n_g - 1) / 2^n_g with N = 3,
 * the leading power of N in every diagonal element N C_F^n_g (T = lambda/2;
 * Mangano-Parke, Phys. Rept. 200 (1991) 301).  mfo_colour_lc returns c_LC;
 * mfo_me2_sum_lc the helicity sum of c_LC sum_sigma |A(sigma)|^2, g_s = 1. */
double mfo_colour_lc(int n_g);
double mfo_me2_sum_lc(int n_g, const double *p, double m, double width);
/* Monte Carlo over colours (also named in Sec. 3.2 on Fig. 4): each event carries one
 * colour assignment -- adjoint indices a_1 .. a_n of the gluons (labels as
 * in the amplitudes), colour i of the top and anticolour j of the antitop --
 * drawn uniformly from the N_cfg = 9 * 8^n_g assignments.  The word pair
 * (r0, r1) of Philox block 0x80000001 of the event's counter gives
 * k = ((r0 << 32) | r1) >> 11 and cfg = ((k >> 16) * N_cfg) >> 37, decoded
 * as j = cfg mod 3, i = (cfg / 3) mod 3, a_g = (cfg / 9 / 8^g) mod 8.  The
 * colour-dressed amplitude is M = sum_sigma (T^{a_sigma1} .. T^{a_sigman})_{ij}
 * A(sigma), and N_cfg |M|^2 summed over helicities is an unbiased estimate of
 * the colour sum: its sum over all assignments is A^dagger C A.            */
int64_t mfo_colour_config(int n_g, uint64_t seed, uint32_t iter, uint64_t event);
int64_t mfo_colour_count(int n_g);
/* c: [n_g!][2] (re, im) colour factors of the orderings for assignment cfg. */
void mfo_colour_factors(int n_g, int64_t cfg, double *c);
/* N_cfg * sum_h |M(cfg)|^2, g_s = 1.                                        */
double mfo_me2_sum_colour_config(int n_g, const double *p, double m, double width, int64_t cfg);
/* Monte Carlo over colour flows (colour = 3): gluon g carries a colour a_g
 * and an anticolour b_g ('t Hooft double line; Maltoni, Paul, Stelzer and
 * Willenbrock, Phys. Rev. D67 (2003) 014026), state matrix
 * G_ab = (e_ab - delta_ab 1/N) / sqrt 2, whose 9 pairs resolve
 * sum_a T^a (x) conj(T^a).  Flows are coded as
 * code = j + 3 i + 9 sum_g 9^g (3 a_g + b_g); those whose factors vanish
 * for every ordering are dropped and the remaining N_flow are numbered in
 * increasing code.  Flow f has the integer weight
 * W_f = 2^n 9^n sum_sigma c_sigma(f)^2 (every factor is (1/sqrt 2)^n times a
 * product of 1, 2/3 and -1/3), total T = sum_f W_f, cumulative
 * C_f = sum_{f' < f} W_f'.  An event draws its flow with probability W_f / T:
 * with k the 53-bit integer of the first word pair of Philox block
 * 0x80000001, u = floor(k T / 2^53) and the flow is the f with
 * C_f <= u < C_{f+1}.  M = sum_sigma (G_{sigma1} .. G_{sigman})_{ij} A(sigma),
 * and (T / W_f) |M|^2 summed over helicities estimates the colour sum
 * without bias.  n_g = 2..4; mfo_flow_count and mfo_flow_total return -1
 * otherwise, mfo_flow_code and mfo_flow_weight -1 for an index out of
 * range.                                                                   */
int64_t mfo_flow_count(int n_g);
int64_t mfo_flow_code(int n_g, int64_t idx);
int64_t mfo_flow_weight(int n_g, int64_t idx);
int64_t mfo_flow_total(int n_g);
int64_t mfo_flow_config(int n_g, uint64_t seed, uint32_t iter, uint64_t event);
/* c: [n_g!] real colour factors of the orderings for flow index idx.       */
void mfo_flow_factors(int n_g, int64_t idx, double *c);
/* (T / W_idx) * sum_h |M(flow idx)|^2, g_s = 1.                             */
double mfo_me2_sum_colour_flow(int n_g, const double *p, double m, double width, int64_t idx);
/* Monte Carlo over helicities (Sec. 3.2 on Fig. 4 names it with the one over
 * colours): each event carries one configuration h of the gluon
 * polarisations and top spins, uniform over N_h = 2^(n_g + 2), from Philox
 * block 0x80000002 of its counter (k the 53-bit integer of the first word
 * pair, h = (k N_h) >> 53).  Configurations are those of the kernels: top and
 * antitop spin along z in their rest frames (bits 0, 1), and for gluon g
 * (bit 2 + g) the real linear polarisation e1 = (0, cos th cos ph,
 * cos th sin ph, -sin th) or e2 = (0, -sin ph, cos ph, 0) of its momentum's
 * angles.  N_h |M_h|^2 estimates the helicity sum without bias.            */
int mfo_hel_count(int n_g);
int mfo_hel_config(int n_g, uint64_t seed, uint32_t iter, uint64_t event);
/* Colour sum (mode 0 full, 1 leading colour, 2 assignment cfg, 3 flow cfg)
 * of |M|^2 with g_s = 1 for the single configuration h of the linear basis. */
double mfo_me2_hel(int n_g, const double *p, double m, double width, int mode, int64_t cfg, int h,
                   double *kappa);

/* Either sampled sum (mode 2: adjoint assignment cfg; mode 3: flow index
 * cfg) and, if kappa is not NULL, its condition number
 * kappa = sum_h |M_h| sum_sigma |c_sigma A_sigma,h| / sum_h |M_h|^2 (>= 1;
 * 0 if the sum vanishes): cancellations between orderings magnify relative
 * rounding errors of the partial amplitudes by up to 2 kappa.  NaN (and
 * kappa NaN) for a mode other than 2 and 3, n_g outside 2..4 or cfg out of
 * range; mfo_flow_config returns -1 and mfo_flow_factors sets c[0] = NaN for
 * an n_g or index out of range.                                            */
double mfo_me2_sum_sampled(int n_g, const double *p, double m, double width, int mode, int64_t cfg,
                           double *kappa);

/* ---- per-event weight and integration ---------------------------------- */
int mfo_n_dims(int n_g);
double mfo_event_weight(const mfo_process *proc, double sqrt_s,
                        const mfo_pdf_grid *pdf, int n_bins, const double *grid,
                        uint64_t seed, int iter, uint64_t event, mfo_event *ev);
/* Same with the uniforms given directly (bin = floor(y n_bins)).           */
double mfo_event_weight_y(const mfo_process *proc, double sqrt_s,
                          const mfo_pdf_grid *pdf, int n_bins, const double *grid,
                          const double *y, mfo_event *ev);

/* ---- hit-or-miss unweighting (Sec. 2.5) --------------------------------- */
/* u_e: first 53-bit uniform of Philox block 0x80000000 of event e.         */
double mfo_unweight_uniform(uint64_t seed, uint32_t iter, uint64_t event);
/* keep[e] = sign(w_e) if u_e w_max < |w_e|, else 0; returns the number kept;
 * *n_over (may be NULL) counts |w_e| > w_max.                               */
uint64_t mfo_unweight(uint64_t n, const double *w, double w_max, uint64_t seed, uint32_t iter,
                      signed char *keep, uint64_t *n_over);
/* p: [n_f + 2][4] lab-frame (E, px, py, pz) of gluon a (+z), gluon b (-z),
 * t, tbar, final gluons.  Returns 0, or 1 below threshold, 2 if the
 * mass-rescaling Newton iteration failed (p is then zero).                 */
int mfo_lab_event(const mfo_process *proc, double sqrt_s, int n_bins, const double *grid,
                  uint64_t seed, int iter, uint64_t event, double *p);

/* Weights w[i] of events ids[i] of iteration iter on n_threads threads;
 * flags[i]: bit 0 above threshold, bit 1 Newton failed, bit 2 passed the
 * cuts, bit 3 near a cut edge, bit 4 ill-conditioned PDF value, bit 5
 * sampled colour sum with condition number colour_kappa > 50, bit 6
 * mass-rescaling root with condition number newton_kappa > 1e3 (written to
 * newton_kappa[i] unless it is NULL).                                      */
int mfo_event_weights(const mfo_process *proc, double sqrt_s, const mfo_pdf_grid *pdf, int n_bins,
                      const double *grid, uint64_t seed, int iter, uint64_t n, const uint64_t *ids,
                      int n_threads, double *w, int *flags, double *newton_kappa);

int mfo_integrate(const mfo_process *proc, double sqrt_s, const mfo_pdf_grid *pdf,
                  uint64_t n_events, int n_iter, uint64_t seed, int start_iter,
                  int n_bins, double alpha, int n_threads,
                  double *grid,            /* in/out [n_dim][n_bins+1]           */
                  double *iter_sigma,      /* [n_iter] or NULL                   */
                  double *iter_var,        /* [n_iter] or NULL                   */
                  double *hist_last,       /* [n_dim][n_bins] or NULL            */
                  double *weights_last,    /* [n_events] or NULL                 */
                  mfo_result *res);

/* Per-iteration estimates and their inverse-variance combination.         */
void mfo_combine(int n_iter, const double *est, const double *var,
                 double *sigma, double *err, double *chi2_dof);
double mfo_neumaier_sum(int n, const double *v);

/* ---- gradients (g g -> t tbar only) ------------------------------------ */
/* Analytic d w / d m_t of one event from the closed-form LO |M|^2 at zero
 * top width, holding the uniforms, the VEGAS grid and mu_F fixed.          */
double mfo_ttx_dweight_dmt_analytic(const mfo_process *proc, double sqrt_s,
                                    const mfo_pdf_grid *pdf, int n_bins,
                                    const double *grid, const double *y,
                                    double *w_out);

#ifdef __cplusplus
}
#endif
#endif
