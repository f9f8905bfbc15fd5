/*
 * mf.h -- C ABI of libmadflow_mi355x: the per-event VEGAS / phase-space /
 * PDF / |M|^2 integrand of MadFlow (Carrazza, Cruz-Martinez, Rossi, Zaro,
 * arXiv:2106.10279) for g g -> t tbar + 0, 1, 2 gluons on one AMD MI355X.
 *
 * The paper's user-level operation (abstract; Fig. 1 of Sec. 2.2) is: take a
 * process at a hadronic sqrt(s) with PDFs, integrate it with VEGAS and return
 * the cross section and the events.  Each event runs the pipeline of
 * Sec. 2.2: random numbers -> phase space (RAMBO family, Sec. 2.4) -> PDFs
 * -> matrix element summed over helicities (Sec. 2.3) -> weight and
 * histogram accumulation; the VEGAS grid is refined after every iteration.
 *
 * Conventions for every entry point:
 *   - All functions are extern "C", never throw, and return mf_status.
 *     On a non-OK status mf_last_error() returns a message (thread-local);
 *     scalar outputs are then untouched and array contents are unspecified.
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory on the current device.  The caller owns every buffer;
 *     the library keeps no pointer after returning.
 *   - Work is enqueued on options->stream (a hipStream_t; NULL = the null
 *     stream).  Calls that return host results synchronise that stream.
 *   - Validation happens on the host before any device call, so argument
 *     errors are reported without touching the GPU.
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MF_OK = 0,
    MF_EINVAL = -1,          /* invalid argument                                   */
    MF_ENOMEM = -2,          /* device allocation failed or size overflow          */
    MF_EDEVICE = -3,         /* HIP runtime error / no device                      */
    MF_ENOCONV = -4,         /* strict mode: mass-rescaling Newton did not converge */
    MF_EUNSUPPORTED = -5     /* valid request the library does not implement       */
} mf_status;

/* Processes: g g -> t tbar + (n_g - 2) gluons.  MF_GG_TTXGGG (five gluons,
 * the gluon channel of the paper's largest process, Sec. 3.2 and Fig. 4)
 * runs with the full helicity sum (MF_HELICITY_SUM) and the full or the
 * leading-colour sum (MF_COLOUR_FULL, MF_COLOUR_LEADING with c_LC = 20.25),
 * not in mf_integrate_static, and with at most 2^15 events per batch: for
 * the full sum each event's 120 x 128 complex partial amplitudes (240 KB in
 * FP64, 120 KB in FP32) pass through device memory between the amplitude
 * kernel and the matrix-core colour sum; for the leading-colour sum only 20
 * partial sums per event do.  mf_matrix_element gives the full sum. */
/* MF_PP_TTX, MF_PP_TTXG and MF_PP_TTXGG are p p -> t tbar (g (g)) as in
 * Sec. 3 and Table 1: the g g channel plus the q qbar channels u ubar,
 * ubar u, d dbar, dbar d (1, 5 and 36 diagrams per quark group; 7, 36 and
 * 267 with g g), weighted by the quark tables of mf_pdf_grid (xq, required); full
 * colour and helicity sums, FP64 or FP32 amplitudes for the g g channel
 * (the q qbar channel is FP64), no gradients, not in mf_integrate_static.
 * The cuts of mf_process apply to the final gluons as for MF_GG_TTXG(G). */
typedef enum {
    MF_GG_TTX = 0, MF_GG_TTXG = 1, MF_GG_TTXGG = 2, MF_GG_TTXGGG = 3, MF_PP_TTX = 4, MF_PP_TTXG = 5,
    MF_PP_TTXGG = 6
} mf_process_id;

/* Arithmetic of the helicity amplitudes and colour sum.  Everything else
 * (VEGAS, phase space, PDF, accumulation, refinement) is FP64 in both. */
typedef enum { MF_FP64 = 0, MF_FP32_KAHAN = 1 } mf_precision;

/* Colour sum of |M|^2.  MF_COLOUR_LEADING is the leading-colour
 * approximation that Sec. 3.2 names for high multiplicities (on Fig. 4): in the colour
 * basis (T^{a_s1} ... T^{a_sn})_{i_t j_tbar}, T = lambda/2, the colour matrix
 * is replaced by c_LC = (N^2 - 1) N^(n_g - 1) / 2^n_g (N = 3: 6, 9, 13.5, 20.25)
 * times the identity, the leading power of N of its diagonal; it changes the
 * integrand (by O(1/N^2)), not only its variance. */
/* MF_COLOUR_SAMPLED is the Monte Carlo over colours that Sec. 3.2 names as
 * well: every event carries one colour assignment (gluon adjoint indices,
 * top colour, antitop anticolour), drawn uniformly from the N_cfg = 9 8^n_g
 * assignments with Philox block 0x80000001 of its counter (the integrand
 * uses blocks 0 .. ceil(D/2) - 1, unweighting block 0x80000000): with k the
 * 53-bit integer of the block's first word pair, cfg = ((k >> 16) N_cfg) >> 37,
 * j = cfg mod 3, i = (cfg / 3) mod 3, gluon g's index (cfg / 9 / 8^g) mod 8.
 * The event's |M|^2 is N_cfg |sum_sigma (T^{a_sigma1} .. T^{a_sigman})_{ij}
 * A(sigma)|^2 summed over helicities: an unbiased estimate of the colour sum
 * with a larger variance.  mf_integrate only, for MF_GG_TTXG and MF_GG_TTXGG;
 * other calls return MF_EUNSUPPORTED. */
/* MF_COLOUR_FLOW samples colour flows instead: gluon g carries a colour a_g
 * and an anticolour b_g with state (e_ab - delta_ab / 3) / sqrt 2, whose 9
 * pairs resolve sum_a T^a (x) conj(T^a) ('t Hooft double line with the U(1)
 * part removed; Maltoni, Paul, Stelzer and Willenbrock, Phys. Rev. D67 (2003)
 * 014026).  Flows are ordered by code = j + 3 i + 9 sum_g 9^g (3 a_g + b_g);
 * those whose factor vanishes for every ordering are dropped, leaving 585
 * (MF_GG_TTXG) and 4311 (MF_GG_TTXGG).  Flow f has the integer weight
 * W_f = 18^n sum_sigma c_sigma(f)^2, T = sum_f W_f (248832 and 23887872), and
 * the event draws flow f with probability W_f / T: u = floor(k T / 2^53) with
 * k from the same Philox block, f the flow with C_f <= u < C_(f+1) for the
 * cumulative weights C in flow order.  |M|^2 is
 * (T / W_f) |sum_sigma (G_{sigma1} .. G_{sigman})_{ij} A(sigma)|^2 summed over
 * helicities: unbiased, with a per-event variance several times smaller than
 * that of MF_COLOUR_SAMPLED.  Same entry points as SAMPLED. */
typedef enum {
    MF_COLOUR_FULL = 0, MF_COLOUR_LEADING = 1, MF_COLOUR_SAMPLED = 2, MF_COLOUR_FLOW = 3
} mf_colour;

/* Helicity treatment of |M|^2.  MF_HELICITY_SAMPLED is the Monte Carlo over
 * helicity configurations that Sec. 3.2 names (on Fig. 4) with the one over
 * colours: every event carries one configuration h of the N_h = 2^(n_g + 2)
 * (bit 0 top spin, bit 1 antitop spin along z in their rest frames; bit 2 + g
 * gluon g's real linear polarisation, e1 = (0, cos th cos ph, cos th sin ph,
 * -sin th) for 0 and e2 = (0, -sin ph, cos ph, 0) for 1, th and ph the angles
 * of its momentum), uniform, from Philox block 0x80000002 of its counter:
 * k the 53-bit integer of the first word pair, h = (k N_h) >> 53.  |M|^2 is
 * N_h times the colour sum (of any mf_colour mode) for that configuration: an
 * unbiased estimate of the helicity sum.  Needs the events' Philox counters:
 * mf_integrate, or mf_evaluate with y = NULL (MF_EINVAL otherwise). */
typedef enum { MF_HELICITY_SUM = 0, MF_HELICITY_SAMPLED = 1 } mf_helicity;

typedef struct {
    mf_process_id id;
    double m_top;            /* GeV, > 0                                       */
    double w_top;            /* GeV, >= 0; width in internal top propagators   */
    double alpha_s;          /* fixed strong coupling, > 0                     */
    double mu_f;             /* factorisation scale in GeV (mu_F^2 in the grid) */
    double ptmin_g;          /* final-gluon pT cut in GeV; <= 0 disables       */
    double etamax_g;         /* final-gluon |eta| (lab) cut; <= 0 disables     */
    double drmin_gg;         /* Delta R between final gluons; <= 0 disables    */
} mf_process;

/* PDF table x g(x, Q^2) on knots ascending in ln x and ln Q^2 (host memory,
 * copied to the device by every call that takes it). */
typedef struct {
    int n_x, n_q2;           /* 4 <= n_x <= 256, 4 <= n_q2 <= 4096            */
    const double *log_x;     /* host [n_x]                                     */
    const double *log_q2;    /* host [n_q2]                                    */
    const double *xf;        /* host [n_q2][n_x], row-major                    */
    const double *xq;        /* host [4][n_q2][n_x] x q(x, Q^2) for u, ubar, d, dbar
                                (the MF_PP_ processes), NULL for the g g
                                processes                                      */
} mf_pdf_grid;

typedef struct {
    int n_bins;              /* VEGAS bins per dimension, 2 .. 1024 (50)        */
    double alpha;            /* grid damping exponent, > 0 (1.5)                */
    int start_iter;          /* first iteration index in the Philox counter (0) */
    mf_precision precision;  /* MF_FP64 or MF_FP32_KAHAN                        */
    int strict;              /* 1: any Newton failure returns MF_ENOCONV        */
    int max_newton;          /* Newton step cap for the mass rescaling (50)     */
    const double *grid_in;   /* host [D][n_bins+1] start grid, NULL = uniform   */
    void *stream;            /* hipStream_t or NULL                             */
    int profile;             /* 1: time every kernel with HIP events (0)        */
    uint64_t max_batch;      /* mf_integrate: events per batch of the per-event device
                                buffers (about 170 B per event), 0 = 2^27 (0)   */
    mf_colour colour;        /* MF_COLOUR_FULL, _LEADING, _SAMPLED or _FLOW (FULL);
                                the gradient entry points take FULL only       */
    mf_helicity helicity;    /* MF_HELICITY_SUM or _SAMPLED (SUM); the gradient
                                entry points take SUM only                     */
} mf_options;

typedef struct {
    double sigma, sigma_err, chi2_dof;   /* combined estimate, pb               */
    double w_max;                        /* largest weight, last iteration      */
    double *iter_sigma;      /* host [n_iter] per-iteration I_j, may be NULL    */
    double *iter_var;        /* host [n_iter] per-iteration V_j, may be NULL    */
    double *grid;            /* host [D][n_bins+1] refined grid out, may be NULL */
    double *hist;            /* host [D][n_bins] last-iteration sum w^2 per bin, may be NULL */
    double *weights;         /* device [n_events] last-iteration weights, may be NULL */
    int64_t n_pass;          /* events passing threshold and cuts, last iteration */
    int64_t n_newton_fail;   /* Newton failures summed over all iterations      */
    double event_kernel_ms;  /* profile = 1: summed event-kernel time, ms       */
    double reduce_kernel_ms; /* profile = 1: summed reduce/refine time, ms      */
    double *iter_pass;       /* host [n_iter] events passing threshold and cuts per iteration, may be NULL */
    double *iter_event_ms;   /* host [n_iter] profile = 1: time of the per-event kernels per iteration, ms, may be NULL */
    double *iter_amp_ms;     /* host [n_iter] profile = 1: of which the helicity-amplitude code, ms, may be NULL
                                (mf_integrate runs it as a kernel of its own between phase space and accumulation) */
    uint64_t n_batches;      /* event batches per iteration (up to 2^27 events each, or max_batch) */
    double *grid_last;       /* host [D][n_bins+1] the grid the last iteration ran on (the one
                                its weights belong to), may be NULL */
    double *iter_colour_ms;  /* host [n_iter] profile = 1, MF_GG_TTXGGG: of the per-event kernels,
                                the matrix-core colour sum (a kernel of its own after the
                                amplitudes), ms, may be NULL */
} mf_result;

/* Fills *opt with the defaults shown above. */
void mf_default_options(mf_options *opt);

/* Number of integration dimensions D = 2 + 3 n_f - 4 (4, 7, 10, 13), or -1. */
int mf_n_dims(int process_id);

/*
 * mf_integrate -- VEGAS integration of the hadronic cross section.
 *   proc, pdf:  process and PDF table (host).
 *   sqrt_s:     hadronic centre-of-mass energy in GeV, > 2 m_top.
 *   n_events:   events per iteration, 2 .. 2^40.
 *   n_iter:     iterations, 1 .. 256.  The grid is refined after each one.
 *   seed:       Philox key.  Event e of iteration j uses the counter
 *               (e mod 2^32, e >> 32, start_iter + j, block).
 * Per iteration: I_j = mean weight, V_j = (mean w^2 - I_j^2)/(N - 1);
 * combined: inverse-variance weighted mean, its error, chi^2/dof.
 */
mf_status mf_integrate(const mf_process *proc, double sqrt_s, const mf_pdf_grid *pdf,
                       uint64_t n_events, int n_iter, uint64_t seed,
                       const mf_options *opt, mf_result *res);

/*
 * mf_integrate_static -- mf_integrate for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, validation, kernels and results
 * as mf_integrate; it calls no hipMalloc, hipFree or other allocating
 * routine.  Its device working memory is one static 96 MiB array per device
 * (held from the library's load until the process ends), shared by every
 * call on that device: calls that overlap on one device race, so the caller
 * serialises them (the library's per-device lock does so within one process).
 * The array holds the PDF table, both grids, the per-iteration results, the
 * per-wave partial sums and the per-event hand-over of one
 * batch of events, which takes the room the rest leaves.  The partial sums
 * take 256 (8 + n_dims n_bins) bytes per compute unit (33 MB for
 * g g -> t tbar g g on 256 compute units, leaving a batch of about 3.8e5
 * events); larger n_events run as several batches, with the same per-event
 * weights and sums that agree to rounding.
 * Limits (MF_EINVAL beyond them): n_dims * n_bins <= 512 and n_x * n_q2 <=
 * 65536.  options->profile must be 0 (MF_EUNSUPPORTED otherwise).  A device
 * whose partial sums and a batch of 256 events do not fit returns MF_ENOMEM.
 * Weights are written to res->weights as in mf_integrate (caller-owned
 * device memory).
 */
mf_status mf_integrate_static(const mf_process *proc, double sqrt_s, const mf_pdf_grid *pdf,
                              uint64_t n_events, int n_iter, uint64_t seed,
                              const mf_options *opt, mf_result *res);

/*
 * mf_evaluate -- per-event weights for a fixed grid (no accumulation).
 *   grid:      host [D][n_bins+1], NULL = uniform.
 *   y:         device [n][D] uniforms in [0,1), or NULL to draw them from
 *              Philox(seed, iter, event); with explicit y the bin is
 *              floor(y n_bins) and the position inside it y n_bins - bin.
 *   event_ids: device [n] event indices for the Philox counter, or NULL
 *              for 0 .. n-1 (ignored when y is given).
 *   w_out:     device [n] weights in pb.
 *   k53_out:   device [n][D] 53-bit integers behind the uniforms, or NULL.
 *   bins_out:  device [n][D] VEGAS bin indices, or NULL.
 *   record_out: device [n][8 + 4 n_f] per-stage record, or NULL:
 *              x1, x2, J_V, phase-space weight W, g(x1), g(x2),
 *              sum over helicities and colours of |M|^2 at g_s = 1,
 *              flags (bit 0: above threshold, bit 1: Newton failed,
 *              bit 2: passed the cuts), then the final-state momenta
 *              t, tbar, gluons in the partonic CM frame (zero when not
 *              generated).
 */
mf_status mf_evaluate(const mf_process *proc, double sqrt_s, const mf_pdf_grid *pdf,
                      const double *grid, const double *y, const uint64_t *event_ids,
                      uint64_t n, uint64_t seed, int iter, const mf_options *opt,
                      double *w_out, uint64_t *k53_out, int32_t *bins_out,
                      double *record_out);

/*
 * mf_refine_grid -- one VEGAS refinement step on the device.
 *   hist: device [D][n_bins] sum of w^2 per bin; grid_in, grid_out: device
 *   [D][n_bins+1].  Smoothing with the neighbours, damping
 *   ((1 - rho)/(-ln rho))^alpha, equal-share rebinning.
 */
mf_status mf_refine_grid(int n_dims, int n_bins, double alpha, const double *hist,
                         const double *grid_in, double *grid_out, void *stream);

/* Colour matrix C[s][t] (host out, [n!][n!]) of the process, orderings of the
 * gluons in lexicographic order, generators T = lambda/2. */
mf_status mf_colour_matrix(int process_id, double *C);

/* Colour- and helicity-summed |M|^2 with g_s = 1 for explicit momenta
 * (the MF_PP_ processes: the q qbar channel, the quark along +z, FP64):
 *   mom: device [n][4 (t) + 4 (tbar) + 4 (n_g-2) (final gluons)] in the
 *        partonic CM frame with the beams along +z/-z; eb: device [n] beam
 *        energies sqrt(s_hat)/2.  out: device [n].
 * MF_EINVAL for an unknown process or precision, a null pointer, n outside
 * [1, 2^40] (outside [1, 2^31 - 1] for MF_PP_TTXGG: one workgroup per event)
 * or m_top, w_top out of range. */
mf_status mf_matrix_element(int process_id, mf_precision precision, const double *mom,
                            const double *eb, uint64_t n, double m_top, double w_top,
                            double *out, void *stream);

/*
 * Gradients of the g g -> t tbar cross section (MF_GG_TTX only, FP64 only;
 * other processes or MF_FP32_KAHAN return MF_EUNSUPPORTED).  Not part of the
 * paper: an adjoint of the integrand of Fig. 1 (the weight of Sec. 2.2 with
 * the phase space of Sec. 2.4 and the amplitudes of Sec. 2.3).  For every
 * event the kernel recomputes the forward pass and runs a hand-written
 * reverse sweep; no helicity amplitude is stored.  d/dm_t differentiates the
 * phase space (through the mass-rescaling root), the spinors and the top
 * propagators; mu_F and the grid are held fixed.  d/dalpha_s = n_g w/alpha_s.
 */
typedef struct {
    double dsigma_dmt;       /* combined d sigma / d m_t, pb/GeV                */
    double dsigma_dalphas;   /* combined d sigma / d alpha_s, pb                */
    double *iter_dmt;        /* host [n_iter] per-iteration mean dw/dm_t, may be NULL     */
    double *iter_dalphas;    /* host [n_iter] per-iteration mean dw/dalpha_s, may be NULL */
    double *dw_dy;           /* device [n_events][D] last iteration dw/dy, may be NULL    */
    double *dw_dmt;          /* device [n_events] last iteration dw/dm_t, may be NULL     */
    double *iter_grad_ms;    /* host [n_iter] options->profile = 1: duration of the adjoint
                                kernel per iteration in ms (HIP events on the stream), may be NULL */
} mf_grad_result;

/*
 * mf_integrate_grad -- mf_integrate plus the gradient.  The integration
 * (grids, I_j, V_j, res) is exactly that of mf_integrate with the same
 * arguments.  Iteration j's gradient g_j is the mean of dw/dtheta over its
 * events on its own (frozen) grid; the combined gradient is
 * sum_j (g_j / V_j) / sum_j (1 / V_j) with the estimate's V_j held fixed.
 */
mf_status mf_integrate_grad(const mf_process *proc, double sqrt_s, const mf_pdf_grid *pdf,
                            uint64_t n_events, int n_iter, uint64_t seed,
                            const mf_options *opt, mf_result *res, mf_grad_result *grad);

/*
 * mf_evaluate_grad -- per-event weight and its gradient for a fixed grid;
 * arguments as mf_evaluate.  Outputs (device, may be NULL except w_out):
 *   w_out [n] weights in pb, dw_dy [n][D] derivative in the uniforms y (inside
 *   the event's VEGAS bins, dx_d/dy_d = J_d), dw_dmt [n] derivative in m_t.
 */
mf_status mf_evaluate_grad(const mf_process *proc, double sqrt_s, const mf_pdf_grid *pdf,
                           const double *grid, const double *y, const uint64_t *event_ids,
                           uint64_t n, uint64_t seed, int iter, const mf_options *opt,
                           double *w_out, double *dw_dy, double *dw_dmt);

/*
 * Hit-or-miss unweighting (Sec. 2.5: the weighted events of an iteration
 * become unit-weight events for the LHE output).  Not a step of the
 * integration itself: it runs on the weights one iteration left behind.
 *
 * Event e (0 <= e < n) of weight w[e] is kept when u_e * w_max < |w[e]|
 * (FP64 product, then comparison), with u_e = k 2^-53 and k the top 53 bits
 * of the first two words of the Philox4x32-10 block with counter
 * (e mod 2^32, e >> 32, iter, 0x80000000) and key seed; the integrand uses
 * blocks 0 .. ceil(D/2) - 1 of the same counters only.  A kept event
 * carries the sign of w[e] (unit weight in units of w_max).  Zero and NaN
 * weights are never kept; |w[e]| >= w_max is always kept.  Kept events are
 * written in increasing e.
 */
typedef struct {
    uint64_t capacity;       /* records the arrays below can hold (0: count only)       */
    uint64_t *event;         /* device [capacity] event indices; required if capacity > 0 */
    double *p;               /* device [capacity][n_f + 2][4] (E, px, py, pz) in GeV in the
                                hadronic frame: gluon a (+z, x1 sqrt(s)/2), gluon b (-z,
                                x2 sqrt(s)/2), t, tbar, final gluons; may be NULL        */
    int8_t *sign;            /* device [capacity] sign of the kept weight, may be NULL  */
    uint64_t n_kept;         /* out: events kept (only the first `capacity` are written) */
    uint64_t n_over;         /* out: events with |w| > w_max                             */
    double kernel_ms[3];     /* out, options->profile = 1: durations of the count, write
                                and record kernels in ms (0 when not run)                */
} mf_events;

/*
 * mf_unweight -- keep events of one iteration by hit-or-miss.
 *   proc, sqrt_s: as in mf_integrate (the cuts are not re-applied: an event
 *                 with w = 0 is never kept).
 *   grid:   host [D][n_bins+1], the grid the weights were computed on
 *           (mf_result.grid_last after mf_integrate), NULL = uniform.
 *   w:      device [n] weights in pb (mf_result.weights); n <= 2^40, n = 0
 *           returns no events.
 *   seed, iter: the Philox key and the iteration index the weights were
 *           drawn with (mf_integrate: start_iter + n_iter - 1 for its last
 *           iteration).
 *   w_max:  finite, > 0 (mf_result.w_max).
 *   opt:    n_bins and max_newton as for the integration; stream.
 * The kinematics of each kept event are regenerated from its counter with
 * the same draw, VEGAS map and phase space as the integration.  Synchronises
 * the stream.
 */
mf_status mf_unweight(const mf_process *proc, double sqrt_s, const double *grid, const double *w,
                      uint64_t n, uint64_t seed, int iter, double w_max, const mf_options *opt,
                      mf_events *out);

/* Message for the last non-OK status on this thread. */
const char *mf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
