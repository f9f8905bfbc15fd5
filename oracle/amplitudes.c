/*
 * amplitudes.c -- oracle: tree-level |M|^2 for g g -> t tbar + (n_g - 2) g.
 * Test infrastructure only (see mfo.h).
 *
 * Sec. 2.3 of the paper: the matrix element loops over the helicities of
 * all external particles and adds up their contributions; external
 * wavefunctions (spinors, polarisation vectors), vertices and propagators
 * are the building blocks.  Here the amplitude of each helicity
 * configuration is written in the colour-flow decomposition
 *     M = g^n sum_sigma (T^{a_sigma1} ... T^{a_sigman})_{i_t j_tbar} A(sigma)
 * (Mangano-Parke, Phys. Rept. 200 (1991) 301; T = lambda/2), the partial
 * amplitudes A(sigma) are built by Berends-Giele recursion (Nucl. Phys.
 * B306 (1988) 759) over ordered gluon subsets with colour-ordered rules
 * derived from the QCD Lagrangian with D = d - i g T^a A^a, and the colour
 * sum is  sum_col |M|^2 = g^(2n) A^dagger C A  with C computed by explicit
 * summation over the Gell-Mann generators.
 *
 * Representation: Dirac gamma matrices, spinors quantised along z, gluon
 * helicity eigenstates.  All particles are outgoing; a crossed incoming
 * gluon carries momentum -p and the polarisation of the physical gluon.
 */
#include <complex.h>
#include <math.h>
#include <string.h>
#include <stdlib.h>
#include <pthread.h>
#include "mfo.h"

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Gell-Mann generators and the colour matrix                                */
/* ------------------------------------------------------------------------ */

static void gell_mann_T(cplx T[8][3][3])
{
    memset(T, 0, sizeof(cplx) * 8 * 9);
    const double s3 = 1.0 / sqrt(3.0);
    /* lambda_1 .. lambda_8, then T = lambda / 2 */
    T[0][0][1] = 1; T[0][1][0] = 1;
    T[1][0][1] = -I; T[1][1][0] = I;
    T[2][0][0] = 1; T[2][1][1] = -1;
    T[3][0][2] = 1; T[3][2][0] = 1;
    T[4][0][2] = -I; T[4][2][0] = I;
    T[5][1][2] = 1; T[5][2][1] = 1;
    T[6][1][2] = -I; T[6][2][1] = I;
    T[7][0][0] = s3; T[7][1][1] = s3; T[7][2][2] = -2.0 * s3;
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                T[a][i][j] *= 0.5;
}

static void mat3_mul(cplx A[3][3], cplx B[3][3], cplx C[3][3])
{
    cplx tmp[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int l = 0; l < 3; ++l)
                s += A[i][l] * B[l][j];
            tmp[i][j] = s;
        }
    memcpy(C, tmp, sizeof(tmp));
}

int mfo_n_orderings(int n_g)
{
    int f = 1;
    for (int i = 2; i <= n_g; ++i)
        f *= i;
    return f;
}

/* All permutations of 0..n-1 in lexicographic order. */
void mfo_orderings(int n_g, int *perm)
{
    int a[MFO_MAX_G + 1];
    for (int i = 0; i < n_g; ++i)
        a[i] = i;
    int count = mfo_n_orderings(n_g);
    for (int c = 0; c < count; ++c) {
        memcpy(perm + c * n_g, a, sizeof(int) * n_g);
        /* next permutation */
        int i = n_g - 2;
        while (i >= 0 && a[i] > a[i + 1]) --i;
        if (i < 0) break;
        int j = n_g - 1;
        while (a[j] < a[i]) --j;
        int t = a[i]; a[i] = a[j]; a[j] = t;
        for (int l = i + 1, r = n_g - 1; l < r; ++l, --r) {
            t = a[l]; a[l] = a[r]; a[r] = t;
        }
    }
}

/* Lexicographic index of a permutation of 0..n-1. */
static int perm_index(int n, const int *p)
{
    int idx = 0;
    for (int i = 0; i < n; ++i) {
        int smaller = 0;
        for (int j = i + 1; j < n; ++j)
            if (p[j] < p[i]) ++smaller;
        idx = idx * (n - i) + smaller;
    }
    return idx;
}

/* The same matrix from its first row: the sum over all adjoint indices is
 * unchanged by relabelling the gluons, so C_{sigma tau} = C_{id, sigma^-1 tau}
 * with (sigma^-1 tau)_k = sigma^-1(tau_k); the first row is summed by brute
 * force over the 8^n assignments. */
void mfo_colour_matrix_relabel(int n_g, double *C)
{
    cplx T[8][3][3];
    gell_mann_T(T);
    int nperm = mfo_n_orderings(n_g);
    int *perm = malloc(sizeof(int) * nperm * n_g);
    mfo_orderings(n_g, perm);
    double *row = calloc((size_t)nperm, sizeof(double));
    int total = 1;
    for (int i = 0; i < n_g; ++i)
        total *= 8;
    int a[MFO_MAX_G];
    for (int code = 0; code < total; ++code) {
        int c = code;
        for (int i = 0; i < n_g; ++i) {
            a[i] = c % 8;
            c /= 8;
        }
        cplx P0[3][3], P[3][3];
        memcpy(P0, T[a[0]], sizeof(cplx) * 9);
        for (int l = 1; l < n_g; ++l)
            mat3_mul(P0, T[a[l]], P0);
        for (int t = 0; t < nperm; ++t) {
            const int *tg = perm + t * n_g;
            memcpy(P, T[a[tg[0]]], sizeof(cplx) * 9);
            for (int l = 1; l < n_g; ++l)
                mat3_mul(P, T[a[tg[l]]], P);
            cplx tr = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    tr += conj(P0[i][j]) * P[i][j];
            row[t] += creal(tr);
        }
    }
    double den = pow(6.0, n_g);
    for (int s = 0; s < nperm; ++s) {
        const int *sg = perm + s * n_g;
        int inv[MFO_MAX_G], q[MFO_MAX_G];
        for (int k = 0; k < n_g; ++k)
            inv[sg[k]] = k;
        for (int t = 0; t < nperm; ++t) {
            const int *tg = perm + t * n_g;
            for (int k = 0; k < n_g; ++k)
                q[k] = inv[tg[k]];
            C[s * nperm + t] = nearbyint(row[perm_index(n_g, q)] * den) / den;
        }
    }
    free(row);
    free(perm);
}

/* C_{sigma sigma'} = sum over all adjoint indices and i, j of
 * conj((T^sigma)_{ij}) (T^sigma')_{ij}, by brute force over the 8^n
 * assignments of Gell-Mann generators.  The exact value is a rational
 * number with denominator dividing 6^n; the sum is rounded to it once.
 * For five gluons (120 orderings) the matrix is built from its first row
 * (mfo_colour_matrix_relabel), which the tests check against this full
 * sum for two to four gluons. */
void mfo_colour_matrix(int n_g, double *C)
{
    if (n_g >= 5) {
        mfo_colour_matrix_relabel(n_g, C);
        return;
    }
    cplx T[8][3][3];
    gell_mann_T(T);
    int nperm = mfo_n_orderings(n_g);
    int *perm = malloc(sizeof(int) * nperm * n_g);
    mfo_orderings(n_g, perm);
    double *acc = calloc((size_t)nperm * nperm, sizeof(double));
    cplx (*P)[3][3] = malloc(sizeof(cplx) * 9 * nperm);
    int total = 1;
    for (int i = 0; i < n_g; ++i)
        total *= 8;
    int a[MFO_MAX_G];
    for (int code = 0; code < total; ++code) {
        int c = code;
        for (int i = 0; i < n_g; ++i) {
            a[i] = c % 8;
            c /= 8;
        }
        for (int s = 0; s < nperm; ++s) {
            const int *sg = perm + s * n_g;
            memcpy(P[s], T[a[sg[0]]], sizeof(cplx) * 9);
            for (int l = 1; l < n_g; ++l)
                mat3_mul(P[s], T[a[sg[l]]], P[s]);
        }
        for (int s = 0; s < nperm; ++s)
            for (int t = 0; t < nperm; ++t) {
                cplx tr = 0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        tr += conj(P[s][i][j]) * P[t][i][j];
                acc[s * nperm + t] += creal(tr);
            }
    }
    double den = pow(6.0, n_g);
    for (int s = 0; s < nperm * nperm; ++s)
        C[s] = nearbyint(acc[s] * den) / den;
    free(P);
    free(acc);
    free(perm);
}

/* ------------------------------------------------------------------------ */
/* Dirac algebra                                                             */
/* ------------------------------------------------------------------------ */

static cplx G[4][4][4];          /* gamma^mu in the Dirac representation */
static pthread_once_t gamma_once = PTHREAD_ONCE_INIT;

static void fill_gamma(void)
{
    memset(G, 0, sizeof(G));
    G[0][0][0] = 1; G[0][1][1] = 1; G[0][2][2] = -1; G[0][3][3] = -1;
    /* gamma^k = [[0, sigma_k], [-sigma_k, 0]] */
    cplx sig[3][2][2] = {
        { { 0, 1 }, { 1, 0 } },
        { { 0, -I }, { I, 0 } },
        { { 1, 0 }, { 0, -1 } },
    };
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                G[k + 1][i][j + 2] = sig[k][i][j];
                G[k + 1][i + 2][j] = -sig[k][i][j];
            }
}

static void init_gamma(void)
{
    pthread_once(&gamma_once, fill_gamma);
}

static cplx mdot(const cplx *a, const cplx *b)
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* slash(a) = gamma^mu a_mu */
static void slash(const cplx *a, cplx S[4][4])
{
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            S[i][j] = a[0] * G[0][i][j] - a[1] * G[1][i][j] - a[2] * G[2][i][j] - a[3] * G[3][i][j];
}

static void row_times(const cplx *row, cplx M[4][4], cplx *out)
{
    cplx t[4];
    for (int j = 0; j < 4; ++j) {
        cplx s = 0;
        for (int i = 0; i < 4; ++i)
            s += row[i] * M[i][j];
        t[j] = s;
    }
    memcpy(out, t, sizeof(t));
}

static cplx row_dot_col(const cplx *row, const cplx *col)
{
    cplx s = 0;
    for (int i = 0; i < 4; ++i)
        s += row[i] * col[i];
    return s;
}

/* sigma . p as a 2x2 matrix */
static void sigma_dot(const double *p, cplx m[2][2])
{
    m[0][0] = p[3];
    m[0][1] = p[1] - I * p[2];
    m[1][0] = p[1] + I * p[2];
    m[1][1] = -p[3];
}

/* ubar(p, s) for an outgoing fermion: u = (sqrt(E+m) chi, (sigma.p) chi / sqrt(E+m)),
 * ubar = u^dagger gamma^0, chi_0 = (1, 0), chi_1 = (0, 1). */
static void spinor_ubar(const double *p, double m, int s, cplx *ub)
{
    double n = sqrt(p[0] + m);
    cplx sp[2][2];
    sigma_dot(p, sp);
    cplx chi[2] = { s == 0 ? 1 : 0, s == 0 ? 0 : 1 };
    cplx u[4];
    u[0] = n * chi[0];
    u[1] = n * chi[1];
    u[2] = (sp[0][0] * chi[0] + sp[0][1] * chi[1]) / n;
    u[3] = (sp[1][0] * chi[0] + sp[1][1] * chi[1]) / n;
    ub[0] = conj(u[0]);
    ub[1] = conj(u[1]);
    ub[2] = -conj(u[2]);
    ub[3] = -conj(u[3]);
}

/* v(p, s) for an outgoing antifermion: v = ((sigma.p) eta / sqrt(E+m), sqrt(E+m) eta). */
static void spinor_v(const double *p, double m, int s, cplx *v)
{
    double n = sqrt(p[0] + m);
    cplx sp[2][2];
    sigma_dot(p, sp);
    cplx eta[2] = { s == 0 ? 1 : 0, s == 0 ? 0 : 1 };
    v[0] = (sp[0][0] * eta[0] + sp[0][1] * eta[1]) / n;
    v[1] = (sp[1][0] * eta[0] + sp[1][1] * eta[1]) / n;
    v[2] = n * eta[0];
    v[3] = n * eta[1];
}

/* u(p, s) for an incoming fermion (the column spinor whose Dirac adjoint is
 * spinor_ubar), and vbar(p, s) = v^dagger gamma^0 for an incoming antifermion. */
static void spinor_u(const double *p, double m, int s, cplx *u)
{
    cplx ub[4];
    spinor_ubar(p, m, s, ub);
    u[0] = conj(ub[0]);
    u[1] = conj(ub[1]);
    u[2] = -conj(ub[2]);
    u[3] = -conj(ub[3]);
}

static void spinor_vbar(const double *p, double m, int s, cplx *vb)
{
    cplx v[4];
    spinor_v(p, m, s, v);
    vb[0] = conj(v[0]);
    vb[1] = conj(v[1]);
    vb[2] = -conj(v[2]);
    vb[3] = -conj(v[3]);
}

/* Helicity polarisation vectors transverse to the 3-momentum of p:
 * eps_pm = (-/+ e1 - i e2)/sqrt(2) with e1 = (0, cos th cos ph, cos th sin ph, -sin th),
 * e2 = (0, -sin ph, cos ph, 0).  hel 0 -> +, 1 -> -. */
static void polarisation(const double *p, int hel, cplx *eps)
{
    double pt = sqrt(p[1] * p[1] + p[2] * p[2]);
    double th = atan2(pt, p[3]);
    double ph = pt > 0.0 ? atan2(p[2], p[1]) : 0.0;
    double e1[4] = { 0.0, cos(th) * cos(ph), cos(th) * sin(ph), -sin(th) };
    double e2[4] = { 0.0, -sin(ph), cos(ph), 0.0 };
    double sgn = hel == 0 ? -1.0 : 1.0;
    for (int mu = 0; mu < 4; ++mu)
        eps[mu] = (sgn * e1[mu] - I * e2[mu]) / sqrt(2.0);
}

/* Real linear polarisations of the same frame: hel 0 -> e1, 1 -> e2.  The
 * helicity vectors above are (-/+ e1 - i e2)/sqrt(2) of these, so both pairs
 * span the same transverse plane and the polarisation sum is the same. */
static void polarisation_linear(const double *p, int hel, cplx *eps)
{
    double pt = sqrt(p[1] * p[1] + p[2] * p[2]);
    double th = atan2(pt, p[3]);
    double ph = pt > 0.0 ? atan2(p[2], p[1]) : 0.0;
    double e1[4] = { 0.0, cos(th) * cos(ph), cos(th) * sin(ph), -sin(th) };
    double e2[4] = { 0.0, -sin(ph), cos(ph), 0.0 };
    for (int mu = 0; mu < 4; ++mu)
        eps[mu] = hel == 0 ? e1[mu] : e2[mu];
}

/* Gluon polarisation basis of the partial amplitudes on this thread: 0 the
 * helicity vectors, 1 the linear ones (the Monte Carlo over helicities
 * samples configurations of the linear basis). */
static __thread int pol_linear;

/* ------------------------------------------------------------------------ */
/* Colour-ordered Berends-Giele recursion                                    */
/* ------------------------------------------------------------------------ */

#define MAXCODE 7776   /* codes of ordered gluon sequences, base n+1 <= 6 */

typedef struct {
    int n;
    const double *p;           /* [n+2][4] all outgoing: t, tbar, g_1 .. g_n */
    double m, width;
    cplx eps[MFO_MAX_G][4];
    cplx gcur[MAXCODE][4];
    char gdone[MAXCODE];
    cplx fcur[MAXCODE][4];
    char fdone[MAXCODE];
} bg_state;

static int seq_code(const int *seq, int len, int n)
{
    int code = 0, base = 1;
    for (int t = 0; t < len; ++t) {
        code += (seq[t] + 1) * base;
        base *= (n + 1);
    }
    return code;
}

static void seq_momentum(const bg_state *st, const int *seq, int len, double *P)
{
    P[0] = P[1] = P[2] = P[3] = 0.0;
    for (int t = 0; t < len; ++t)
        for (int mu = 0; mu < 4; ++mu)
            P[mu] += st->p[4 * (2 + seq[t]) + mu];
}

static double rdot(const double *a, const double *b)
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* Colour-ordered gluon current j(seq), off-shell leg propagator included:
 *   j = -(1/P^2) { sum over splits seq = s1 s2 of
 *                    j1 ((2P1 + P2).j2) - j2 ((P1 + 2P2).j1) + (P2 - P1)(j1.j2)
 *                  + sum over splits seq = s1 s2 s3 of
 *                    j1 (j2.j3) - 2 j2 (j1.j3) + j3 (j1.j2) }            */
static const cplx *gluon_current(bg_state *st, const int *seq, int len)
{
    int code = seq_code(seq, len, st->n);
    if (st->gdone[code])
        return st->gcur[code];
    cplx *out = st->gcur[code];
    if (len == 1) {
        memcpy(out, st->eps[seq[0]], sizeof(cplx) * 4);
        st->gdone[code] = 1;
        return out;
    }
    cplx acc[4] = { 0, 0, 0, 0 };
    for (int a = 1; a < len; ++a) {
        const cplx *j1 = gluon_current(st, seq, a);
        const cplx *j2 = gluon_current(st, seq + a, len - a);
        double P1[4], P2[4];
        seq_momentum(st, seq, a, P1);
        seq_momentum(st, seq + a, len - a, P2);
        cplx q1[4], q2[4];
        for (int mu = 0; mu < 4; ++mu) {
            q1[mu] = 2.0 * P1[mu] + P2[mu];
            q2[mu] = P1[mu] + 2.0 * P2[mu];
        }
        cplx c1 = mdot(q1, j2), c2 = mdot(q2, j1), c12 = mdot(j1, j2);
        for (int mu = 0; mu < 4; ++mu)
            acc[mu] += j1[mu] * c1 - j2[mu] * c2 + (P2[mu] - P1[mu]) * c12;
    }
    for (int a = 1; a < len; ++a)
        for (int b = a + 1; b < len; ++b) {
            const cplx *j1 = gluon_current(st, seq, a);
            const cplx *j2 = gluon_current(st, seq + a, b - a);
            const cplx *j3 = gluon_current(st, seq + b, len - b);
            cplx d23 = mdot(j2, j3), d13 = mdot(j1, j3), d12 = mdot(j1, j2);
            for (int mu = 0; mu < 4; ++mu)
                acc[mu] += j1[mu] * d23 - 2.0 * j2[mu] * d13 + j3[mu] * d12;
        }
    double P[4];
    seq_momentum(st, seq, len, P);
    double P2 = rdot(P, P);
    for (int mu = 0; mu < 4; ++mu)
        out[mu] = -acc[mu] / P2;
    st->gdone[code] = 1;
    return out;
}

/* i (P-slash + m) / (P^2 - m^2 + i m Gamma) applied from the right to a row spinor. */
static void fermion_propagate(const bg_state *st, const double *P, const cplx *row, cplx *out)
{
    cplx Pc[4] = { P[0], P[1], P[2], P[3] };
    cplx S[4][4];
    slash(Pc, S);
    for (int i = 0; i < 4; ++i)
        S[i][i] += st->m;
    cplx den = rdot(P, P) - st->m * st->m + I * st->m * st->width;
    cplx t[4];
    row_times(row, S, t);
    for (int i = 0; i < 4; ++i)
        out[i] = I * t[i] / den;
}

/* Row spinor ubar(k_t) with the ordered gluons seq attached (vertex i gamma.j),
 * including the propagator of the top line after the last attachment.      */
static const cplx *fermion_current(bg_state *st, const cplx *ubar, const int *seq, int len)
{
    if (len == 0)
        return ubar;
    int code = seq_code(seq, len, st->n);
    if (st->fdone[code])
        return st->fcur[code];
    cplx acc[4] = { 0, 0, 0, 0 };
    for (int a = 0; a < len; ++a) {
        const cplx *left = fermion_current(st, ubar, seq, a);
        const cplx *j = gluon_current(st, seq + a, len - a);
        cplx S[4][4], t[4];
        slash(j, S);
        row_times(left, S, t);
        for (int i = 0; i < 4; ++i)
            acc[i] += I * t[i];
    }
    double P[4];
    seq_momentum(st, seq, len, P);
    for (int mu = 0; mu < 4; ++mu)
        P[mu] += st->p[mu];                 /* + k_t */
    fermion_propagate(st, P, acc, st->fcur[code]);
    st->fdone[code] = 1;
    return st->fcur[code];
}

static void partial_amplitudes_core(int n, const double *p, double m, double width,
                                    const int *hel, int ward_gluon, cplx *A)
{
    init_gamma();
    static __thread bg_state st_tls;
    bg_state *st = &st_tls;
    st->n = n;
    st->p = p;
    st->m = m;
    st->width = width;
    memset(st->gdone, 0, sizeof(st->gdone));
    memset(st->fdone, 0, sizeof(st->fdone));
    for (int g = 0; g < n; ++g) {
        if (g == ward_gluon) {
            for (int mu = 0; mu < 4; ++mu)
                st->eps[g][mu] = p[4 * (2 + g) + mu];
        } else if (pol_linear) {
            polarisation_linear(p + 4 * (2 + g), hel[2 + g], st->eps[g]);
        } else {
            polarisation(p + 4 * (2 + g), hel[2 + g], st->eps[g]);
        }
    }
    cplx ubar[4], v[4];
    spinor_ubar(p, m, hel[0], ubar);
    spinor_v(p + 4, m, hel[1], v);

    int nperm = mfo_n_orderings(n);
    int perm[120 * MFO_MAX_G];
    mfo_orderings(n, perm);
    for (int s = 0; s < nperm; ++s) {
        const int *sg = perm + s * n;
        cplx amp = 0;
        for (int a = 0; a < n; ++a) {
            const cplx *left = fermion_current(st, ubar, sg, a);
            const cplx *j = gluon_current(st, sg + a, n - a);
            cplx S[4][4], t[4];
            slash(j, S);
            row_times(left, S, t);
            amp += I * row_dot_col(t, v);
        }
        A[s] = amp;
    }
}

void mfo_partial_amplitudes(int n_g, const double *p, double m, double width,
                            const int *hel, int ward_gluon, double *A)
{
    cplx amp[120];
    partial_amplitudes_core(n_g, p, m, width, hel, ward_gluon, amp);
    for (int s = 0; s < mfo_n_orderings(n_g); ++s) {
        A[2 * s] = creal(amp[s]);
        A[2 * s + 1] = cimag(amp[s]);
    }
}

static pthread_mutex_t colour_lock = PTHREAD_MUTEX_INITIALIZER;
static double colour_cache[MFO_MAX_G + 1][120 * 120];
static int colour_ready[MFO_MAX_G + 1];

static const double *colour_matrix_cached(int n_g)
{
    pthread_mutex_lock(&colour_lock);
    if (!colour_ready[n_g]) {
        mfo_colour_matrix(n_g, colour_cache[n_g]);
        colour_ready[n_g] = 1;
    }
    pthread_mutex_unlock(&colour_lock);
    return colour_cache[n_g];
}

static void hel_from_index(int n_g, int h, int *hel)
{
    for (int i = 0; i < n_g + 2; ++i)
        hel[i] = (h >> i) & 1;
}

double mfo_me2_sum_hel(int n_g, const double *p, double m, double width,
                       int n_hel, const int *hel_list)
{
    int nperm = mfo_n_orderings(n_g);
    const double *C = colour_matrix_cached(n_g);
    double total = 0.0;
    for (int h = 0; h < n_hel; ++h) {
        cplx A[120];
        partial_amplitudes_core(n_g, p, m, width, hel_list + h * (n_g + 2), -1, A);
        double s = 0.0;
        for (int a = 0; a < nperm; ++a)
            for (int b = 0; b < nperm; ++b)
                s += creal(conj(A[a]) * C[a * nperm + b] * A[b]);
        total += s;
    }
    return total;
}

double mfo_colour_lc(int n_g)
{
    const double N = 3.0;
    return (N * N - 1.0) * pow(N, n_g - 1) / pow(2.0, n_g);
}

double mfo_me2_sum_lc(int n_g, const double *p, double m, double width)
{
    int nperm = mfo_n_orderings(n_g);
    int nh = 1 << (n_g + 2);
    double total = 0.0;
    for (int h = 0; h < nh; ++h) {
        int hel[MFO_MAX_G + 2];
        hel_from_index(n_g, h, hel);
        cplx A[120];
        partial_amplitudes_core(n_g, p, m, width, hel, -1, A);
        for (int a = 0; a < nperm; ++a)
            total += creal(A[a]) * creal(A[a]) + cimag(A[a]) * cimag(A[a]);
    }
    return mfo_colour_lc(n_g) * total;
}

int64_t mfo_colour_count(int n_g)
{
    int64_t n = 9;
    for (int g = 0; g < n_g; ++g)
        n *= 8;
    return n;
}

int64_t mfo_colour_config(int n_g, uint64_t seed, uint32_t iter, uint64_t event)
{
    uint32_t ctr[4] = { (uint32_t)event, (uint32_t)(event >> 32), iter, 0x80000001u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t r[4];
    mfo_philox4x32_10(ctr, key, r);
    uint64_t k = ((((uint64_t)r[0]) << 32) | (uint64_t)r[1]) >> 11;
    return (int64_t)(((k >> 16) * (uint64_t)mfo_colour_count(n_g)) >> 37);
}

static cplx gm_T[8][3][3];
static pthread_once_t gm_once = PTHREAD_ONCE_INIT;

static void gm_init(void)
{
    gell_mann_T(gm_T);
}

void mfo_colour_factors(int n_g, int64_t cfg, double *c)
{
    pthread_once(&gm_once, gm_init);
    cplx (*T)[3][3] = gm_T;
    int jj = (int)(cfg % 3);
    int ii = (int)((cfg / 3) % 3);
    int a[MFO_MAX_G];
    int64_t rest = cfg / 9;
    for (int g = 0; g < n_g; ++g) {
        a[g] = (int)(rest % 8);
        rest /= 8;
    }
    int nperm = mfo_n_orderings(n_g);
    int perm[120 * MFO_MAX_G];
    mfo_orderings(n_g, perm);
    for (int s = 0; s < nperm; ++s) {
        /* row i of the product T^{a_sigma1} ... T^{a_sigman}, then entry j */
        cplx row[3] = { 0, 0, 0 };
        row[ii] = 1;
        for (int k = 0; k < n_g; ++k) {
            cplx (*M)[3] = T[a[perm[s * n_g + k]]];
            cplx nr[3];
            for (int q = 0; q < 3; ++q)
                nr[q] = row[0] * M[0][q] + row[1] * M[1][q] + row[2] * M[2][q];
            memcpy(row, nr, sizeof(nr));
        }
        c[2 * s] = creal(row[jj]);
        c[2 * s + 1] = cimag(row[jj]);
    }
}

/* sum_h |sum_sigma c_sigma A_sigma,h|^2 for factors c (re, im per ordering)
 * and, in *kappa, sum_h |M_h| sum_sigma |c_sigma A_sigma,h| / sum_h |M_h|^2:
 * the factor by which the sum magnifies relative errors of the amplitudes
 * (0 if the sum vanishes). */
static double dressed_sum(int n_g, const double *p, double m, double width, const double *c, double *kappa)
{
    int nperm = mfo_n_orderings(n_g);
    int nh = 1 << (n_g + 2);
    double total = 0.0, bound = 0.0;
    for (int h = 0; h < nh; ++h) {
        int hel[MFO_MAX_G + 2];
        hel_from_index(n_g, h, hel);
        cplx A[120];
        partial_amplitudes_core(n_g, p, m, width, hel, -1, A);
        cplx M = 0;
        double mag = 0.0;
        for (int s = 0; s < nperm; ++s) {
            cplx t = (c[2 * s] + I * c[2 * s + 1]) * A[s];
            M += t;
            mag += cabs(t);
        }
        total += creal(M) * creal(M) + cimag(M) * cimag(M);
        bound += cabs(M) * mag;
    }
    if (kappa)
        *kappa = total > 0.0 ? bound / total : 0.0;
    return total;
}

double mfo_me2_sum_sampled(int n_g, const double *p, double m, double width, int mode, int64_t cfg,
                           double *kappa)
{
    double c[2 * 120];
    int64_t count;
    if (kappa)
        *kappa = NAN;
    if ((mode != 2 && mode != 3) || n_g < 2 || n_g > MFO_MAX_G || cfg < 0 ||
        cfg >= (mode == 2 ? mfo_colour_count(n_g) : mfo_flow_count(n_g)))
        return NAN;
    if (mode == 2) {
        mfo_colour_factors(n_g, cfg, c);
        count = mfo_colour_count(n_g);
    } else {
        int nperm = mfo_n_orderings(n_g);
        double r[120];
        mfo_flow_factors(n_g, cfg, r);
        for (int s = 0; s < nperm; ++s) {
            c[2 * s] = r[s];
            c[2 * s + 1] = 0.0;
        }
        return (double)mfo_flow_total(n_g) / (double)mfo_flow_weight(n_g, cfg) * dressed_sum(n_g, p, m, width, c, kappa);
    }
    return (double)count * dressed_sum(n_g, p, m, width, c, kappa);
}

/* ---- Monte Carlo over helicities -------------------------------------- */

int mfo_hel_count(int n_g)
{
    return 1 << (n_g + 2);
}

/* Configuration h of event `event`: Philox block 0x80000002 of its counter,
 * k the 53-bit integer of the first word pair, h = (k N_h) >> 53, uniform over
 * the N_h = 2^(n_g + 2) configurations (bit 0 top spin, bit 1 antitop spin,
 * bit 2 + g polarisation of gluon g). */
int mfo_hel_config(int n_g, uint64_t seed, uint32_t iter, uint64_t event)
{
    uint32_t ctr[4] = { (uint32_t)event, (uint32_t)(event >> 32), iter, 0x80000002u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t r[4];
    mfo_philox4x32_10(ctr, key, r);
    uint64_t k = ((((uint64_t)r[0]) << 32) | (uint64_t)r[1]) >> 11;
    return (int)((k * (uint64_t)mfo_hel_count(n_g)) >> 53);
}

/* Colour sum of |M|^2 for the one configuration h of the linear basis, with
 * the colour treatment of mode (0 full, 1 leading colour, 2 assignment cfg,
 * 3 flow cfg; for 2 and 3 including their N_cfg or T / W_f scale).  *kappa
 * (may be NULL): for modes 2 and 3 the condition number of the dressed sum,
 * as in mfo_me2_sum_sampled. */
double mfo_me2_hel(int n_g, const double *p, double m, double width, int mode, int64_t cfg, int h,
                   double *kappa)
{
    if (kappa)
        *kappa = 0.0;
    if (n_g < 2 || n_g > MFO_MAX_G || h < 0 || h >= mfo_hel_count(n_g) || mode < 0 || mode > 3)
        return NAN;
    if ((mode == 2 && (cfg < 0 || cfg >= mfo_colour_count(n_g))) ||
        (mode == 3 && (cfg < 0 || cfg >= mfo_flow_count(n_g))))
        return NAN;
    int nperm = mfo_n_orderings(n_g);
    int hel[MFO_MAX_G + 2];
    hel_from_index(n_g, h, hel);
    cplx A[120];
    pol_linear = 1;
    partial_amplitudes_core(n_g, p, m, width, hel, -1, A);
    pol_linear = 0;
    if (mode == 0) {
        const double *C = colour_matrix_cached(n_g);
        double s = 0.0;
        for (int a = 0; a < nperm; ++a)
            for (int b = 0; b < nperm; ++b)
                s += creal(conj(A[a]) * C[a * nperm + b] * A[b]);
        return s;
    }
    if (mode == 1) {
        double s = 0.0;
        for (int a = 0; a < nperm; ++a)
            s += creal(A[a]) * creal(A[a]) + cimag(A[a]) * cimag(A[a]);
        return mfo_colour_lc(n_g) * s;
    }
    double c[2 * 120], scale;
    if (mode == 2) {
        mfo_colour_factors(n_g, cfg, c);
        scale = (double)mfo_colour_count(n_g);
    } else {
        double r[120];
        mfo_flow_factors(n_g, cfg, r);
        for (int s = 0; s < nperm; ++s) {
            c[2 * s] = r[s];
            c[2 * s + 1] = 0.0;
        }
        scale = (double)mfo_flow_total(n_g) / (double)mfo_flow_weight(n_g, cfg);
    }
    cplx M = 0;
    double mag = 0.0;
    for (int s = 0; s < nperm; ++s) {
        cplx t = (c[2 * s] + I * c[2 * s + 1]) * A[s];
        M += t;
        mag += cabs(t);
    }
    double v = creal(M) * creal(M) + cimag(M) * cimag(M);
    if (kappa)
        *kappa = v > 0.0 ? cabs(M) * mag / v : 0.0;
    return scale * v;
}

double mfo_me2_sum_colour_config(int n_g, const double *p, double m, double width, int64_t cfg)
{
    return mfo_me2_sum_sampled(n_g, p, m, width, 2, cfg, NULL);
}

/* Colour flows: gluon g carries a colour a_g and an anticolour b_g, state
 * G_ab = (e_ab - delta_ab 1/N) / sqrt 2 with (e_ab)_{rs} = delta_ra delta_sb.
 * Summed over the 9 pairs, G_ab (x) conj(G_ab) equals sum_a T^a (x) conj(T^a),
 * so flows replace adjoint indices without changing the colour sum.  The
 * flows are enumerated by code = j + 3 i + 9 sum_g 9^g (3 a_g + b_g); a flow
 * whose factors vanish for every ordering contributes nothing and is dropped,
 * the rest are numbered in increasing code and drawn with probability
 * proportional to W_f = 18^n sum_sigma c_sigma^2, an integer.               */
static int64_t *flow_codes[MFO_MAX_G + 1];
static int64_t *flow_cum[MFO_MAX_G + 1];      /* [n + 1] cumulative weights          */
static int64_t flow_n[MFO_MAX_G + 1];
static pthread_once_t flow_once = PTHREAD_ONCE_INIT;

static void flow_matrix(int a, int b, double G[3][3])
{
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s)
            G[r][s] = ((r == a && s == b ? 1.0 : 0.0) - (a == b && r == s ? 1.0 / 3.0 : 0.0)) / sqrt(2.0);
}

/* c[sigma] = (G_{sigma1} ... G_{sigman})_{ij} for the flow with this code. */
static void flow_factors_of_code(int n_g, int64_t code, const int *perm, int nperm, double *c)
{
    int jj = (int)(code % 3), ii = (int)((code / 3) % 3);
    double G[MFO_MAX_G][3][3];
    int64_t rest = code / 9;
    for (int g = 0; g < n_g; ++g) {
        int pr = (int)(rest % 9);
        rest /= 9;
        flow_matrix(pr / 3, pr % 3, G[g]);
    }
    for (int s = 0; s < nperm; ++s) {
        double P[3][3] = { { 1, 0, 0 }, { 0, 1, 0 }, { 0, 0, 1 } };
        for (int k = 0; k < n_g; ++k) {
            double (*Gk)[3] = G[perm[s * n_g + k]];
            double Q[3][3];
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q)
                    Q[r][q] = P[r][0] * Gk[0][q] + P[r][1] * Gk[1][q] + P[r][2] * Gk[2][q];
            memcpy(P, Q, sizeof(Q));
        }
        c[s] = P[ii][jj];
    }
}

static void flow_init(void)
{
    /* flows are tabulated for up to four gluons (9^(n+1) codes each) */
    for (int n_g = 2; n_g <= 4; ++n_g) {
        int64_t total = 9;
        for (int g = 0; g < n_g; ++g)
            total *= 9;
        int nperm = mfo_n_orderings(n_g);
        int perm[120 * MFO_MAX_G];
        mfo_orderings(n_g, perm);
        flow_codes[n_g] = malloc(sizeof(int64_t) * (size_t)total);
        flow_cum[n_g] = malloc(sizeof(int64_t) * (size_t)(total + 1));
        double scale = pow(18.0, n_g);         /* 2^n 9^n: c_sigma^2 times it is an integer */
        int64_t k = 0;
        flow_cum[n_g][0] = 0;
        for (int64_t code = 0; code < total; ++code) {
            double c[120];
            flow_factors_of_code(n_g, code, perm, nperm, c);
            double w = 0.0;
            for (int s = 0; s < nperm; ++s)
                w += c[s] * c[s] * scale;
            if (w > 0.5) {
                flow_codes[n_g][k] = code;
                flow_cum[n_g][k + 1] = flow_cum[n_g][k] + llround(w);
                ++k;
            }
        }
        flow_n[n_g] = k;
    }
}

int64_t mfo_flow_count(int n_g)
{
    if (n_g < 2 || n_g > 4)
        return -1;
    pthread_once(&flow_once, flow_init);
    return flow_n[n_g];
}

int64_t mfo_flow_code(int n_g, int64_t idx)
{
    int64_t n = mfo_flow_count(n_g);
    if (n < 0 || idx < 0 || idx >= n)
        return -1;
    return flow_codes[n_g][idx];
}

int64_t mfo_flow_weight(int n_g, int64_t idx)
{
    int64_t n = mfo_flow_count(n_g);
    if (n < 0 || idx < 0 || idx >= n)
        return -1;
    return flow_cum[n_g][idx + 1] - flow_cum[n_g][idx];
}

int64_t mfo_flow_total(int n_g)
{
    int64_t n = mfo_flow_count(n_g);
    return n < 0 ? -1 : flow_cum[n_g][n];
}

int64_t mfo_flow_config(int n_g, uint64_t seed, uint32_t iter, uint64_t event)
{
    uint32_t ctr[4] = { (uint32_t)event, (uint32_t)(event >> 32), iter, 0x80000001u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t r[4];
    mfo_philox4x32_10(ctr, key, r);
    uint64_t k = ((((uint64_t)r[0]) << 32) | (uint64_t)r[1]) >> 11;
    if (mfo_flow_count(n_g) < 0)
        return -1;
    uint64_t u = (uint64_t)(((unsigned __int128)k * (uint64_t)mfo_flow_total(n_g)) >> 53);
    /* the flow whose weight interval [C_idx, C_idx+1) holds u */
    int64_t lo = 0, hi = mfo_flow_count(n_g);
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if ((uint64_t)flow_cum[n_g][mid] <= u)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

void mfo_flow_factors(int n_g, int64_t idx, double *c)
{
    int64_t code = mfo_flow_code(n_g, idx);
    if (code < 0) {
        c[0] = NAN;                            /* n_g or idx out of range */
        return;
    }
    int nperm = mfo_n_orderings(n_g);
    int perm[120 * MFO_MAX_G];
    mfo_orderings(n_g, perm);
    flow_factors_of_code(n_g, code, perm, nperm, c);
}

double mfo_me2_sum_colour_flow(int n_g, const double *p, double m, double width, int64_t idx)
{
    return mfo_me2_sum_sampled(n_g, p, m, width, 3, idx, NULL);
}

double mfo_me2_sum(int n_g, const double *p, double m, double width)
{
    int nh = 1 << (n_g + 2);
    int hel[(4 << MFO_MAX_G) * (MFO_MAX_G + 2)];
    for (int h = 0; h < nh; ++h)
        hel_from_index(n_g, h, hel + h * (n_g + 2));
    return mfo_me2_sum_hel(n_g, p, m, width, nh, hel);
}

/* ------------------------------------------------------------------------ */
/* q qbar -> t tbar                                                          */
/* ------------------------------------------------------------------------ */
/* One s-channel gluon (Peskin-Schroeder rules as below, g = 1):
 *   M = T^a_{i_qbar i_q} T^a_{i_t i_tbar} [vbar(pb) gamma^mu u(pa)]
 *       [ubar(k1) gamma_mu v(k2)] / s      (overall phase dropped);
 * the colour sum of |T^a_{ji} T^a_{kl}|^2 over all indices is
 * Tr(T^a T^b) Tr(T^a T^b) = delta^ab delta^ab / 4 = 2.  Massless quarks. */
double mfo_me2_qqbar_ttx(const double *p, double m)
{
    init_gamma();
    double pa[4], pb[4];
    for (int mu = 0; mu < 4; ++mu) {
        pa[mu] = -p[8 + mu];
        pb[mu] = -p[12 + mu];
    }
    double P[4] = { pa[0] + pb[0], pa[1] + pb[1], pa[2] + pb[2], pa[3] + pb[3] };
    double s = P[0] * P[0] - P[1] * P[1] - P[2] * P[2] - P[3] * P[3];
    double total = 0.0;
    for (int h = 0; h < 16; ++h) {
        cplx u[4], vb[4], ub[4], v[4];
        spinor_u(pa, 0.0, h & 1, u);
        spinor_vbar(pb, 0.0, (h >> 1) & 1, vb);
        spinor_ubar(p, m, (h >> 2) & 1, ub);
        spinor_v(p + 4, m, (h >> 3) & 1, v);
        cplx J[4], K[4];
        for (int mu = 0; mu < 4; ++mu) {
            cplx t[4];
            row_times(vb, G[mu], t);
            J[mu] = row_dot_col(t, u);
            row_times(ub, G[mu], t);
            K[mu] = row_dot_col(t, v);
        }
        cplx amp = (J[0] * K[0] - J[1] * K[1] - J[2] * K[2] - J[3] * K[3]) / s;
        total += creal(amp * conj(amp));
    }
    return 2.0 * total;
}

/* ------------------------------------------------------------------------ */
/* Fully colour-dressed Feynman rules (pin for the colour decomposition)     */
/* ------------------------------------------------------------------------ */
/* Rules (Peskin-Schroeder conventions, D = d - i g A^a T^a, g = 1):
 *   quark-gluon vertex      i gamma^mu T^a
 *   quark propagator        i (p-slash + m) / (p^2 - m^2 + i m Gamma)
 *   gluon propagator        -i g_{mu nu} delta^{ab} / p^2       (Feynman gauge)
 *   3-gluon vertex          f^{abc} [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
 *                           (all momenta incoming)
 *   4-gluon vertex          -i [f^{abe} f^{cde} (g^{mu rho} g^{nu sigma} - g^{mu sigma} g^{nu rho})
 *                               + f^{ace} f^{bde} (g^{mu nu} g^{rho sigma} - g^{mu sigma} g^{nu rho})
 *                               + f^{ade} f^{bce} (g^{mu nu} g^{rho sigma} - g^{mu rho} g^{nu sigma})]
 * Currents are over unordered gluon subsets, every external colour
 * assignment is summed explicitly.                                          */

typedef struct {
    int n;
    const double *p;
    double m, width;
    cplx T[8][3][3];
    double f[8][8][8];
    double ff[8][8][8][8];      /* sum_e f^{abe} f^{cde} */
    cplx eps[MFO_MAX_G][4];
    int col[MFO_MAX_G];
    cplx J[1 << MFO_MAX_G][8][4];
    char Jdone[1 << MFO_MAX_G];
} fc_state;

static void subset_momentum(const fc_state *st, int S, double *P)
{
    P[0] = P[1] = P[2] = P[3] = 0.0;
    for (int g = 0; g < st->n; ++g)
        if (S & (1 << g))
            for (int mu = 0; mu < 4; ++mu)
                P[mu] += st->p[4 * (2 + g) + mu];
}

static int is_zero4(const cplx *v)
{
    return v[0] == 0 && v[1] == 0 && v[2] == 0 && v[3] == 0;
}

static void fc_current(fc_state *st, int S)
{
    if (st->Jdone[S]) return;
    cplx (*out)[4] = st->J[S];
    memset(out, 0, sizeof(cplx) * 32);
    if ((S & (S - 1)) == 0) {              /* single gluon */
        int g = __builtin_ctz(S);
        memcpy(out[st->col[g]], st->eps[g], sizeof(cplx) * 4);
        st->Jdone[S] = 1;
        return;
    }
    double P[4];
    subset_momentum(st, S, P);
    cplx acc[8][4];
    memset(acc, 0, sizeof(acc));
    /* 3-gluon vertex: ordered pairs (S1, S2), factor 1/2 */
    for (int S1 = (S - 1) & S; S1 > 0; S1 = (S1 - 1) & S) {
        int S2 = S & ~S1;
        fc_current(st, S1);
        fc_current(st, S2);
        double P1[4], P2[4];
        subset_momentum(st, S1, P1);
        subset_momentum(st, S2, P2);
        /* incoming momenta at the vertex: k = P, p = -P1, q = -P2 */
        cplx kmp[4], qmk[4];
        double pmq[4];
        for (int mu = 0; mu < 4; ++mu) {
            kmp[mu] = P[mu] + P1[mu];
            pmq[mu] = -P1[mu] + P2[mu];
            qmk[mu] = -P2[mu] - P[mu];
        }
        for (int b = 0; b < 8; ++b) {
            const cplx *X = st->J[S1][b];
            if (is_zero4(X)) continue;
            for (int c = 0; c < 8; ++c) {
                const cplx *Y = st->J[S2][c];
                if (is_zero4(Y)) continue;
                cplx ky = mdot(kmp, Y), xy = mdot(X, Y), qx = mdot(qmk, X);
                for (int a = 0; a < 8; ++a) {
                    double fabc = st->f[a][b][c];
                    if (fabc == 0.0) continue;
                    for (int mu = 0; mu < 4; ++mu)
                        acc[a][mu] += 0.5 * fabc * (X[mu] * ky + xy * pmq[mu] + Y[mu] * qx);
                }
            }
        }
    }
    /* 4-gluon vertex: ordered triples (S1, S2, S3), factor 1/6 */
    for (int S1 = (S - 1) & S; S1 > 0; S1 = (S1 - 1) & S) {
        int R = S & ~S1;
        for (int S2 = (R - 1) & R; S2 > 0; S2 = (S2 - 1) & R) {
            int S3 = R & ~S2;
            fc_current(st, S1);
            fc_current(st, S2);
            fc_current(st, S3);
            for (int b = 0; b < 8; ++b) {
                const cplx *X = st->J[S1][b];
                if (is_zero4(X)) continue;
                for (int c = 0; c < 8; ++c) {
                    const cplx *Y = st->J[S2][c];
                    if (is_zero4(Y)) continue;
                    for (int d = 0; d < 8; ++d) {
                        const cplx *Z = st->J[S3][d];
                        if (is_zero4(Z)) continue;
                        cplx xz = mdot(X, Z), xy = mdot(X, Y), yz = mdot(Y, Z);
                        for (int a = 0; a < 8; ++a) {
                            double F1 = st->ff[a][b][c][d];
                            double F2 = st->ff[a][c][b][d];
                            double F3 = st->ff[a][d][b][c];
                            if (F1 == 0.0 && F2 == 0.0 && F3 == 0.0) continue;
                            for (int mu = 0; mu < 4; ++mu) {
                                cplx v = F1 * (Y[mu] * xz - Z[mu] * xy)
                                       + F2 * (X[mu] * yz - Z[mu] * xy)
                                       + F3 * (X[mu] * yz - Y[mu] * xz);
                                acc[a][mu] += -I * v / 6.0;
                            }
                        }
                    }
                }
            }
        }
    }
    double P2 = rdot(P, P);
    for (int a = 0; a < 8; ++a)
        for (int mu = 0; mu < 4; ++mu)
            out[a][mu] = -I * acc[a][mu] / P2;
    st->Jdone[S] = 1;
}

/* K_{c'c}(S) = sum_a (T^a)_{c'c} J^a(S) */
static void colour_contract(const fc_state *st, int S, cplx K[3][3][4])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int mu = 0; mu < 4; ++mu) {
                cplx s = 0;
                for (int a = 0; a < 8; ++a)
                    if (st->T[a][i][j] != 0)
                        s += st->T[a][i][j] * st->J[S][a][mu];
                K[i][j][mu] = s;
            }
}

/* Colour constants of the Feynman-rule evaluation: generators, f^abc and
 * sum_e f^abe f^cde. */
static void fc_init(fc_state *st, int n_g, const double *p, double m, double width)
{
    st->n = n_g;
    st->p = p;
    st->m = m;
    st->width = width;
    gell_mann_T(st->T);
    /* f^{abc} = -2 i Tr([T^a, T^b] T^c) */
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            for (int c = 0; c < 8; ++c) {
                cplx AB[3][3], BA[3][3], X[3][3];
                mat3_mul(st->T[a], st->T[b], AB);
                mat3_mul(st->T[b], st->T[a], BA);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        X[i][j] = AB[i][j] - BA[i][j];
                mat3_mul(X, st->T[c], X);
                cplx tr = X[0][0] + X[1][1] + X[2][2];
                double v = creal(-2.0 * I * tr);
                st->f[a][b][c] = fabs(v) < 1e-14 ? 0.0 : v;
            }
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            for (int c = 0; c < 8; ++c)
                for (int d = 0; d < 8; ++d) {
                    double s = 0.0;
                    for (int e = 0; e < 8; ++e)
                        s += st->f[a][b][e] * st->f[c][d][e];
                    st->ff[a][b][c][d] = s;
                }
}

/* M_ij for the external colours st->col and polarisations st->eps: the
 * colour-dressed amplitude with top colour i and antitop anticolour j. */
static void fc_Mij(fc_state *st, const double *p, double m, double width, const cplx *ubar, const cplx *v,
                   cplx Mij[3][3])
{
    int n_g = st->n;
    int full = (1 << n_g) - 1;
    memset(st->Jdone, 0, sizeof(st->Jdone));
    /* colour-dressed fermion currents U[S][top colour][line colour][4] */
    cplx U[1 << MFO_MAX_G][3][3][4];
    memset(U, 0, sizeof(U));
    for (int it = 0; it < 3; ++it)
        memcpy(U[0][it][it], ubar, sizeof(cplx) * 4);
    /* subsets in increasing order: every proper subset of S precedes S */
    for (int S = 1; S < full; ++S) {
        double P[4];
        subset_momentum(st, S, P);
        for (int mu = 0; mu < 4; ++mu)
            P[mu] += p[mu];
        cplx acc[3][3][4];
        memset(acc, 0, sizeof(acc));
        for (int S2 = S; S2 > 0; S2 = (S2 - 1) & S) {
            int S1 = S & ~S2;
            fc_current(st, S2);
            cplx K[3][3][4];
            colour_contract(st, S2, K);
            for (int cp = 0; cp < 3; ++cp)
                for (int cc = 0; cc < 3; ++cc) {
                    if (is_zero4(K[cp][cc])) continue;
                    cplx Sl[4][4];
                    slash(K[cp][cc], Sl);
                    for (int it = 0; it < 3; ++it) {
                        cplx t[4];
                        row_times(U[S1][it][cp], Sl, t);
                        for (int i = 0; i < 4; ++i)
                            acc[it][cc][i] += I * t[i];
                    }
                }
        }
        bg_state tmp;          /* only m, width used by the propagator */
        tmp.m = m;
        tmp.width = width;
        for (int it = 0; it < 3; ++it)
            for (int cc = 0; cc < 3; ++cc)
                fermion_propagate(&tmp, P, acc[it][cc], U[S][it][cc]);
    }
    /* close the line on v(k_tbar) with antitop colour j */
    memset(Mij, 0, sizeof(cplx) * 9);
    for (int S2 = full; S2 > 0; S2 = (S2 - 1) & full) {
        int S1 = full & ~S2;
        fc_current(st, S2);
        cplx K[3][3][4];
        colour_contract(st, S2, K);
        for (int cp = 0; cp < 3; ++cp)
            for (int jj = 0; jj < 3; ++jj) {
                if (is_zero4(K[cp][jj])) continue;
                cplx Sl[4][4];
                slash(K[cp][jj], Sl);
                for (int it = 0; it < 3; ++it) {
                    cplx t[4];
                    row_times(U[S1][it][cp], Sl, t);
                    Mij[it][jj] += I * row_dot_col(t, v);
                }
            }
    }
}

double mfo_me2_sum_fullcolour(int n_g, const double *p, double m, double width,
                              int n_hel, const int *hel_list)
{
    init_gamma();
    fc_state *st = malloc(sizeof(fc_state));
    fc_init(st, n_g, p, m, width);
    int total_col = 1;
    for (int i = 0; i < n_g; ++i)
        total_col *= 8;
    double total = 0.0;
    for (int h = 0; h < n_hel; ++h) {
        const int *hel = hel_list + h * (n_g + 2);
        for (int g = 0; g < n_g; ++g)
            polarisation(p + 4 * (2 + g), hel[2 + g], st->eps[g]);
        cplx ubar[4], v[4];
        spinor_ubar(p, m, hel[0], ubar);
        spinor_v(p + 4, m, hel[1], v);
        for (int code = 0; code < total_col; ++code) {
            int c = code;
            for (int g = 0; g < n_g; ++g) {
                st->col[g] = c % 8;
                c /= 8;
            }
            cplx Mij[3][3];
            fc_Mij(st, p, m, width, ubar, v, Mij);
            for (int it = 0; it < 3; ++it)
                for (int jj = 0; jj < 3; ++jj)
                    total += creal(Mij[it][jj] * conj(Mij[it][jj]));
        }
    }
    free(st);
    return total;
}

/* The colour-dressed amplitude M_ij (Feynman rules with explicit SU(3)
 * indices, helicity polarisations) for gluon adjoint indices cols[0 .. n-1],
 * top colour i, antitop anticolour j: out[2 (3 i + j)] re, [+1] im. */
void mfo_dressed_amplitude(int n_g, const double *p, double m, double width, const int *hel, const int *cols,
                           double *out)
{
    init_gamma();
    fc_state *st = malloc(sizeof(fc_state));
    fc_init(st, n_g, p, m, width);
    for (int g = 0; g < n_g; ++g) {
        polarisation(p + 4 * (2 + g), hel[2 + g], st->eps[g]);
        st->col[g] = cols[g];
    }
    cplx ubar[4], v[4];
    spinor_ubar(p, m, hel[0], ubar);
    spinor_v(p + 4, m, hel[1], v);
    cplx Mij[3][3];
    fc_Mij(st, p, m, width, ubar, v, Mij);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            out[2 * (3 * i + j)] = creal(Mij[i][j]);
            out[2 * (3 * i + j) + 1] = cimag(Mij[i][j]);
        }
    free(st);
}

/* ------------------------------------------------------------------------ */
/* q qbar -> t tbar g (the q qbar channel of p p -> t tbar g, Sec. 3)        */
/* ------------------------------------------------------------------------ */
/* Feynman rules as listed above the colour-dressed engine (g = 1).  Legs:
 * quark q(pa) with colour i, antiquark qbar(pb) with anticolour j, top t(k1)
 * colour k, antitop tbar(k2) anticolour l, gluon g(k3) adjoint a; s = (pa +
 * pb)^2, s12 = (k1 + k2)^2.  The five diagrams:
 *   D1  g emitted by the quark:     vbar(pb) g^nu S(pa - k3) eps u(pa) . ubar(k1) g_nu v(k2) / s12
 *                                   colour (T^b T^a)_ji (T^b)_kl
 *   D2  g emitted by the antiquark: vbar(pb) eps S(k3 - pb) g^nu u(pa) . ubar g_nu v / s12
 *                                   colour (T^a T^b)_ji (T^b)_kl
 *   D3  g emitted by the top:       ubar(k1) eps S(k1 + k3) g^nu v(k2) . vbar g_nu u / s
 *                                   colour (T^b)_ji (T^a T^b)_kl
 *   D4  g emitted by the antitop:   ubar(k1) g^nu S(-k2 - k3) eps v(k2) . vbar g_nu u / s
 *                                   colour (T^b)_ji (T^b T^a)_kl
 *   D5  three-gluon vertex: J = vbar g u (gluon b, momentum P = pa + pb into
 *       the vertex), K = ubar g v (gluon c, momentum -Q = -(k1 + k2) into the
 *       vertex), the external gluon (a, momentum -k3 into the vertex):
 *       [J.K (P + Q).eps + K.eps J.(k3 - Q) - J.eps K.(k3 + P)] / (s s12)
 *                                   colour f^{bca} (T^b)_ji (T^c)_kl
 * with S(p) = (p-slash + m) / (p^2 - m^2 + i m Gamma) (m = 0 on the quark
 * line).  Counting the factors i of the rules, D1 .. D4 carry -i and D5
 * carries +1, so M = -i [A1 C1 + A2 C2 + A3 C3 + A4 C4 + i A5 C5]; the
 * common factor -i is dropped.                                              */

static void qq_vec_current(const cplx *row, const cplx *col, cplx *J)
{
    for (int mu = 0; mu < 4; ++mu) {
        cplx t[4];
        row_times(row, G[mu], t);
        J[mu] = row_dot_col(t, col);
    }
}

static void qq_mat_col(cplx M[4][4], const cplx *col, cplx *out)
{
    cplx t[4];
    for (int i = 0; i < 4; ++i) {
        cplx s = 0;
        for (int j = 0; j < 4; ++j)
            s += M[i][j] * col[j];
        t[i] = s;
    }
    memcpy(out, t, sizeof(t));
}

/* (p-slash + m) / (p^2 - m^2 + i m Gamma) as a matrix */
static void qq_propagator(const double *p, double m, double width, cplx S[4][4])
{
    cplx pc[4] = { p[0], p[1], p[2], p[3] };
    slash(pc, S);
    cplx den = rdot(p, p) - m * m + I * m * width;
    for (int i = 0; i < 4; ++i) {
        S[i][i] += m;
        for (int j = 0; j < 4; ++j)
            S[i][j] /= den;
    }
}

static cplx qq_cdot(const cplx *a, const double *b)
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

void mfo_qqbar_ttxg_diagrams(const double *p, double m, double width, const int *hel, int ward, double *amp)
{
    init_gamma();
    double pa[4], pb[4], k1[4], k2[4], k3[4];
    for (int mu = 0; mu < 4; ++mu) {
        k1[mu] = p[mu];
        k2[mu] = p[4 + mu];
        pa[mu] = -p[8 + mu];
        pb[mu] = -p[12 + mu];
        k3[mu] = p[16 + mu];
    }
    cplx u[4], vb[4], ub[4], v[4], eps[4];
    spinor_u(pa, 0.0, hel[0], u);
    spinor_vbar(pb, 0.0, hel[1], vb);
    spinor_ubar(k1, m, hel[2], ub);
    spinor_v(k2, m, hel[3], v);
    if (ward) {
        for (int mu = 0; mu < 4; ++mu)
            eps[mu] = k3[mu];
    } else {
        polarisation(k3, hel[4], eps);
    }
    double P[4], Q[4];
    for (int mu = 0; mu < 4; ++mu) {
        P[mu] = pa[mu] + pb[mu];
        Q[mu] = k1[mu] + k2[mu];
    }
    double s = rdot(P, P), s12 = rdot(Q, Q);
    cplx E[4][4], S[4][4], t[4], w[4];
    slash(eps, E);
    cplx J[4], K[4], X[4];
    qq_vec_current(vb, u, J);
    qq_vec_current(ub, v, K);
    cplx A[5];
    /* D1 */
    double q1[4];
    for (int mu = 0; mu < 4; ++mu)
        q1[mu] = pa[mu] - k3[mu];
    qq_propagator(q1, 0.0, 0.0, S);
    qq_mat_col(E, u, t);
    qq_mat_col(S, t, w);
    qq_vec_current(vb, w, X);
    A[0] = mdot(X, K) / s12;
    /* D2 */
    double q2[4];
    for (int mu = 0; mu < 4; ++mu)
        q2[mu] = k3[mu] - pb[mu];
    qq_propagator(q2, 0.0, 0.0, S);
    row_times(vb, E, t);
    row_times(t, S, w);
    qq_vec_current(w, u, X);
    A[1] = mdot(X, K) / s12;
    /* D3 */
    double q3[4];
    for (int mu = 0; mu < 4; ++mu)
        q3[mu] = k1[mu] + k3[mu];
    qq_propagator(q3, m, width, S);
    row_times(ub, E, t);
    row_times(t, S, w);
    qq_vec_current(w, v, X);
    A[2] = mdot(X, J) / s;
    /* D4 */
    double q4[4];
    for (int mu = 0; mu < 4; ++mu)
        q4[mu] = -k2[mu] - k3[mu];
    qq_propagator(q4, m, width, S);
    qq_mat_col(E, v, t);
    qq_mat_col(S, t, w);
    qq_vec_current(ub, w, X);
    A[3] = mdot(X, J) / s;
    /* D5 */
    double PQ[4], kQ[4], kP[4];
    for (int mu = 0; mu < 4; ++mu) {
        PQ[mu] = P[mu] + Q[mu];
        kQ[mu] = k3[mu] - Q[mu];
        kP[mu] = k3[mu] + P[mu];
    }
    cplx v5 = mdot(J, K) * qq_cdot(eps, PQ) + mdot(K, eps) * qq_cdot(J, kQ) - mdot(J, eps) * qq_cdot(K, kP);
    A[4] = I * v5 / (s * s12);
    for (int d = 0; d < 5; ++d) {
        amp[2 * d] = creal(A[d]);
        amp[2 * d + 1] = cimag(A[d]);
    }
}

static cplx qq_T[8][3][3];
static double qq_f[8][8][8];
static pthread_once_t qq_once = PTHREAD_ONCE_INIT;

static void qq_colour_init(void)
{
    gell_mann_T(qq_T);
    /* f^{abc} = -2 i Tr([T^a, T^b] T^c) */
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            for (int c = 0; c < 8; ++c) {
                cplx tr = 0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k)
                            tr += (qq_T[a][i][j] * qq_T[b][j][k] - qq_T[b][i][j] * qq_T[a][j][k]) * qq_T[c][k][i];
                qq_f[a][b][c] = creal(-2.0 * I * tr);
            }
}

void mfo_qqbar_ttxg_colour(const int *cols, double *c)
{
    pthread_once(&qq_once, qq_colour_init);
    const int i = cols[0], j = cols[1], k = cols[2], l = cols[3], a = cols[4];
    cplx C[5] = { 0, 0, 0, 0, 0 };
    for (int b = 0; b < 8; ++b) {
        cplx ba_ji = 0, ab_ji = 0, ab_kl = 0, ba_kl = 0;
        for (int x = 0; x < 3; ++x) {
            ba_ji += qq_T[b][j][x] * qq_T[a][x][i];
            ab_ji += qq_T[a][j][x] * qq_T[b][x][i];
            ab_kl += qq_T[a][k][x] * qq_T[b][x][l];
            ba_kl += qq_T[b][k][x] * qq_T[a][x][l];
        }
        C[0] += ba_ji * qq_T[b][k][l];
        C[1] += ab_ji * qq_T[b][k][l];
        C[2] += qq_T[b][j][i] * ab_kl;
        C[3] += qq_T[b][j][i] * ba_kl;
        for (int cc = 0; cc < 8; ++cc)
            C[4] += qq_f[b][cc][a] * qq_T[b][j][i] * qq_T[cc][k][l];
    }
    for (int d = 0; d < 5; ++d) {
        c[2 * d] = creal(C[d]);
        c[2 * d + 1] = cimag(C[d]);
    }
}

/* Sum over the 32 helicity configurations and the 3^4 x 8 colour
 * assignments of |sum_d C_d A_d|^2 (g = 1, no averaging).                  */
double mfo_me2_qqbar_ttxg(const double *p, double m, double width)
{
    double C[648][10];
    for (int ci = 0; ci < 648; ++ci) {
        int cols[5] = { ci % 3, (ci / 3) % 3, (ci / 9) % 3, (ci / 27) % 3, ci / 81 };
        mfo_qqbar_ttxg_colour(cols, C[ci]);
    }
    double total = 0.0;
    for (int h = 0; h < 32; ++h) {
        int hel[5] = { h & 1, (h >> 1) & 1, (h >> 2) & 1, (h >> 3) & 1, (h >> 4) & 1 };
        double A[10];
        mfo_qqbar_ttxg_diagrams(p, m, width, hel, 0, A);
        for (int ci = 0; ci < 648; ++ci) {
            const double *c = C[ci];
            double re = 0.0, im = 0.0;
            for (int d = 0; d < 5; ++d) {
                re += c[2 * d] * A[2 * d] - c[2 * d + 1] * A[2 * d + 1];
                im += c[2 * d] * A[2 * d + 1] + c[2 * d + 1] * A[2 * d];
            }
            total += re * re + im * im;
        }
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* q qbar -> t tbar g g (the q qbar channel of p p -> t tbar g g, Sec. 3)    */
/* ------------------------------------------------------------------------ */
/* The 36 Feynman diagrams, written out by where the two gluons attach, with
 * the rules above (g = 1).  The quark line vbar(pb) ... u(pa) and the top
 * line ubar(k1) ... v(k2) are joined by one gluon, the spine.  Each line is
 * a chain of vertices from its column end; an attachment emits momentum q
 * (external gluon: k; spine, seen from the quark line: the momentum it
 * carries to the top side; seen from the top line: minus that; the pair
 * g1 g2 joined by a three-gluon vertex, "composite": K = k3 + k4).
 *   1  both gluons on the quark line, 3! orders              (6)
 *   2  both on the top line                                   (6)
 *   3  one on each line, 2 x 2 orders, 2 assignments          (8)
 *   4  one on the spine (three-gluon vertex), one on the quark line (4)
 *   5  one on the spine, one on the top line                  (4)
 *   6  both on the spine: two three-gluon vertices in either order (2),
 *      or the four-gluon vertex (its three colour structures counted as
 *      three terms)
 *   7  the composite on the quark line (2), the top line (2), the spine (1)
 * Counting the factors i of vertices and propagators, classes 1-3 carry i,
 * classes 4, 5 and 7 (on a line) -1, class 6 and 7 (on the spine) -i; the
 * common factor i is dropped, so the relative factors are 1, i and -1.
 * Three-gluon vertex with the spine current J (colour c, momentum P into
 * the vertex), a gluon (colour a, polarisation e, momentum k out of it) and
 * the continuing spine (colour c', momentum P - k): colour f^{c a c'},
 * current (J.e)(P + k) + e J.(P - 2k) + J e.(k - 2P).  The composite:
 * colour f^{e a1 a2}, current [eps1 eps2.(K + k3) + eps1.eps2 (k4 - k3)
 * - eps2 eps1.(K + k4)] / K^2.  Four-gluon vertex (spine in: colour c_q,
 * gluons a1, a2, spine out: c_t, internal e): f^{c_q a1 e} f^{a2 c_t e}
 * [Xq.eps2 eps1.Xt - Xq.Xt eps1.eps2] + f^{c_q a2 e} f^{a1 c_t e}
 * [Xq.eps1 eps2.Xt - Xq.Xt eps1.eps2] + f^{c_q c_t e} f^{a1 a2 e}
 * [Xq.eps1 eps2.Xt - Xq.eps2 eps1.Xt], times -i.                           */

#define Q4_TERMS 38

typedef struct {
    double q[4];      /* outgoing momentum */
    cplx e[4];        /* polarisation or off-shell current (unused if open) */
    int open;         /* the line's free index (the spine) */
} q4_att;

/* colour slots: 0, 1 the gluons' adjoint indices a1, a2; 2 + x internal index x */
typedef struct {
    int nq, qs[3];    /* quark line, from the u end */
    int nt, ts[3];    /* top line, from the v end */
    int nf, f[3][3];  /* structure constants f^{xyz} */
    int nint;
} q4_colour;

/* X^mu = row V_{n-1} S(P_{n-1}) ... S(P_1) V_0 col, V_t = e_t-slash except
 * the open attachment, which carries gamma^mu; P_t = p0 - q_0 - ... - q_{t-1}. */
static void q4_line(const cplx *row, const cplx *col, const double *p0, double m, double width, int n,
                    const q4_att *att, cplx *X)
{
    int s = 0;
    while (!att[s].open)
        ++s;
    double P[4];
    memcpy(P, p0, sizeof(P));
    cplx R[4], t[4], S[4][4], E[4][4];
    memcpy(R, col, sizeof(R));
    for (int a = 0; a < s; ++a) {
        slash(att[a].e, E);
        qq_mat_col(E, R, t);
        for (int mu = 0; mu < 4; ++mu)
            P[mu] -= att[a].q[mu];
        qq_propagator(P, m, width, S);
        qq_mat_col(S, t, R);
    }
    /* momentum after the open attachment, then the left part */
    for (int mu = 0; mu < 4; ++mu)
        P[mu] -= att[s].q[mu];
    double Pt[3][4];
    for (int a = s + 1; a < n; ++a) {
        memcpy(Pt[a - s - 1], P, sizeof(P));   /* the segment between a - 1 and a */
        for (int mu = 0; mu < 4; ++mu)
            P[mu] -= att[a].q[mu];
    }
    cplx L[4];
    memcpy(L, row, sizeof(L));
    for (int a = n - 1; a > s; --a) {
        slash(att[a].e, E);
        row_times(L, E, t);
        qq_propagator(Pt[a - s - 1], m, width, S);
        row_times(t, S, L);
    }
    qq_vec_current(L, R, X);
}

static cplx q4_dot(const cplx *a, const cplx *b)
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* three-gluon vertex: J (momentum P in), e (momentum k out) -> continuing current */
static void q4_v3(const cplx *J, const double *P, const cplx *e, const double *k, cplx *out)
{
    cplx Pk[4], P2k[4], k2P[4];
    for (int mu = 0; mu < 4; ++mu) {
        Pk[mu] = P[mu] + k[mu];
        P2k[mu] = P[mu] - 2.0 * k[mu];
        k2P[mu] = k[mu] - 2.0 * P[mu];
    }
    cplx je = q4_dot(J, e), jp = q4_dot(J, P2k), ek = q4_dot(e, k2P);
    for (int mu = 0; mu < 4; ++mu)
        out[mu] = je * Pk[mu] + e[mu] * jp + J[mu] * ek;
}

static void q4_set_colour(q4_colour *c, int nq, const int *qs, int nt, const int *ts, int nf, const int (*f)[3],
                          int nint)
{
    memset(c, 0, sizeof(*c));
    c->nq = nq;
    for (int i = 0; i < nq; ++i)
        c->qs[i] = qs[i];
    c->nt = nt;
    for (int i = 0; i < nt; ++i)
        c->ts[i] = ts[i];
    c->nf = nf;
    for (int i = 0; i < nf; ++i)
        for (int j = 0; j < 3; ++j)
            c->f[i][j] = f[i][j];
    c->nint = nint;
}

static double q4_m2(const double *p)
{
    return p[0] * p[0] - p[1] * p[1] - p[2] * p[2] - p[3] * p[3];
}

/* The 38 terms (Lorentz part with its relative factor, colour structure) of
 * helicity configuration hel[6] = (quark, antiquark, top, antitop spin,
 * gluon 1, gluon 2 helicity); ward = 1 or 2 replaces that gluon's
 * polarisation by its momentum.  p: [6][4] all outgoing: t, tbar, -pa,
 * -pb, g1, g2.  Returns the number of terms. */
static int q4_terms(const double *p, double m, double width, const int *hel, int ward, cplx *A, q4_colour *C)
{
    init_gamma();
    double k1[4], k2[4], pa[4], pb[4], kg[2][4];
    for (int mu = 0; mu < 4; ++mu) {
        k1[mu] = p[mu];
        k2[mu] = p[4 + mu];
        pa[mu] = -p[8 + mu];
        pb[mu] = -p[12 + mu];
        kg[0][mu] = p[16 + mu];
        kg[1][mu] = p[20 + mu];
    }
    cplx u[4], vb[4], ub[4], v[4], eps[2][4];
    spinor_u(pa, 0.0, hel[0], u);
    spinor_vbar(pb, 0.0, hel[1], vb);
    spinor_ubar(k1, m, hel[2], ub);
    spinor_v(k2, m, hel[3], v);
    for (int g = 0; g < 2; ++g) {
        if (ward == g + 1)
            for (int mu = 0; mu < 4; ++mu)
                eps[g][mu] = kg[g][mu];
        else
            polarisation(kg[g], hel[4 + g], eps[g]);
    }
    double P0[4], Q[4], K[4], mk2[4];
    for (int mu = 0; mu < 4; ++mu) {
        P0[mu] = pa[mu] + pb[mu];
        Q[mu] = k1[mu] + k2[mu];
        K[mu] = kg[0][mu] + kg[1][mu];
        mk2[mu] = -k2[mu];
    }
    /* the composite g1 g2 current (colour f^{e a1 a2}) */
    cplx J12[4];
    {
        double Kk3[4], k43[4], Kk4[4];
        for (int mu = 0; mu < 4; ++mu) {
            Kk3[mu] = K[mu] + kg[0][mu];
            k43[mu] = kg[1][mu] - kg[0][mu];
            Kk4[mu] = K[mu] + kg[1][mu];
        }
        cplx a = q4_dot(eps[1], (cplx[4]){ Kk3[0], Kk3[1], Kk3[2], Kk3[3] });
        cplx b = q4_dot(eps[0], eps[1]);
        cplx c = q4_dot(eps[0], (cplx[4]){ Kk4[0], Kk4[1], Kk4[2], Kk4[3] });
        double K2 = q4_m2(K);
        for (int mu = 0; mu < 4; ++mu)
            J12[mu] = (eps[0][mu] * a + b * k43[mu] - eps[1][mu] * c) / K2;
    }
    int n = 0;
    q4_att qa[3], ta[3];
    cplx Xq[4], Xt[4], J1[4], J2[4];
    const cplx I1 = I;
    static const int perm3[6][3] = { { 0, 1, 2 }, { 0, 2, 1 }, { 1, 0, 2 }, { 1, 2, 0 }, { 2, 0, 1 }, { 2, 1, 0 } };
    /* attachment builders */
#define Q4_GLUON(att, g) do { memcpy((att).q, kg[g], sizeof(double) * 4); memcpy((att).e, eps[g], sizeof(cplx) * 4); (att).open = 0; } while (0)
#define Q4_COMP(att) do { memcpy((att).q, K, sizeof(double) * 4); memcpy((att).e, J12, sizeof(cplx) * 4); (att).open = 0; } while (0)
#define Q4_SPINE(att, qq) do { for (int mu_ = 0; mu_ < 4; ++mu_) (att).q[mu_] = (qq)[mu_]; (att).open = 1; } while (0)
    double mQ[4], mP0[4];
    for (int mu = 0; mu < 4; ++mu) {
        mQ[mu] = -Q[mu];
        mP0[mu] = -P0[mu];
    }
    /* class 1: both gluons and the spine on the quark line */
    Q4_SPINE(ta[0], mQ);
    q4_line(ub, v, mk2, m, width, 1, ta, Xt);
    for (int o = 0; o < 6; ++o) {
        int slots[3];
        for (int t = 0; t < 3; ++t) {
            int x = perm3[o][t];
            if (x < 2) {
                Q4_GLUON(qa[t], x);
                slots[t] = x;
            } else {
                Q4_SPINE(qa[t], Q);
                slots[t] = 2;
            }
        }
        q4_line(vb, u, pa, 0.0, 0.0, 3, qa, Xq);
        A[n] = q4_dot(Xq, Xt) / q4_m2(Q);
        int ts[1] = { 2 };
        q4_set_colour(&C[n], 3, slots, 1, ts, 0, NULL, 1);
        ++n;
    }
    /* class 2: both gluons and the spine on the top line */
    Q4_SPINE(qa[0], P0);
    q4_line(vb, u, pa, 0.0, 0.0, 1, qa, Xq);
    for (int o = 0; o < 6; ++o) {
        int slots[3];
        for (int t = 0; t < 3; ++t) {
            int x = perm3[o][t];
            if (x < 2) {
                Q4_GLUON(ta[t], x);
                slots[t] = x;
            } else {
                Q4_SPINE(ta[t], mP0);
                slots[t] = 2;
            }
        }
        q4_line(ub, v, mk2, m, width, 3, ta, Xt);
        A[n] = q4_dot(Xq, Xt) / q4_m2(P0);
        int qs[1] = { 2 };
        q4_set_colour(&C[n], 1, qs, 3, slots, 0, NULL, 1);
        ++n;
    }
    /* class 3: gluon ga on the quark line, gb on the top line */
    for (int ga = 0; ga < 2; ++ga) {
        int gb = 1 - ga;
        double Pq[4], mPq[4];
        for (int mu = 0; mu < 4; ++mu) {
            Pq[mu] = P0[mu] - kg[ga][mu];
            mPq[mu] = -Pq[mu];
        }
        for (int oq = 0; oq < 2; ++oq) {
            int qs[2];
            Q4_GLUON(qa[oq], ga);
            qs[oq] = ga;
            Q4_SPINE(qa[1 - oq], Pq);
            qs[1 - oq] = 2;
            q4_line(vb, u, pa, 0.0, 0.0, 2, qa, Xq);
            for (int ot = 0; ot < 2; ++ot) {
                int ts[2];
                Q4_GLUON(ta[ot], gb);
                ts[ot] = gb;
                Q4_SPINE(ta[1 - ot], mPq);
                ts[1 - ot] = 2;
                q4_line(ub, v, mk2, m, width, 2, ta, Xt);
                A[n] = q4_dot(Xq, Xt) / q4_m2(Pq);
                q4_set_colour(&C[n], 2, qs, 2, ts, 0, NULL, 1);
                ++n;
            }
        }
    }
    /* class 4: ga on the spine, gb on the quark line */
    Q4_SPINE(ta[0], mQ);
    q4_line(ub, v, mk2, m, width, 1, ta, Xt);   /* the spine reaches the top line with Q */
    for (int ga = 0; ga < 2; ++ga) {
        int gb = 1 - ga;
        double Pq[4];
        for (int mu = 0; mu < 4; ++mu)
            Pq[mu] = P0[mu] - kg[gb][mu];
        for (int oq = 0; oq < 2; ++oq) {
            int qs[2];
            Q4_GLUON(qa[oq], gb);
            qs[oq] = gb;
            Q4_SPINE(qa[1 - oq], Pq);
            qs[1 - oq] = 2;
            q4_line(vb, u, pa, 0.0, 0.0, 2, qa, Xq);
            q4_v3(Xq, Pq, eps[ga], kg[ga], J1);
            A[n] = I1 * q4_dot(J1, Xt) / (q4_m2(Pq) * q4_m2(Q));
            int ts[1] = { 3 };
            int f[1][3] = { { 2, ga, 3 } };
            q4_set_colour(&C[n], 2, qs, 1, ts, 1, (const int (*)[3])f, 2);
            ++n;
        }
    }
    /* class 5: ga on the spine, gb on the top line */
    Q4_SPINE(qa[0], P0);
    q4_line(vb, u, pa, 0.0, 0.0, 1, qa, Xq);
    for (int ga = 0; ga < 2; ++ga) {
        int gb = 1 - ga;
        double Pt[4], mPt[4];
        for (int mu = 0; mu < 4; ++mu) {
            Pt[mu] = P0[mu] - kg[ga][mu];
            mPt[mu] = -Pt[mu];
        }
        q4_v3(Xq, P0, eps[ga], kg[ga], J1);
        for (int ot = 0; ot < 2; ++ot) {
            int ts[2];
            Q4_GLUON(ta[ot], gb);
            ts[ot] = gb;
            Q4_SPINE(ta[1 - ot], mPt);
            ts[1 - ot] = 3;
            q4_line(ub, v, mk2, m, width, 2, ta, Xt);
            A[n] = I1 * q4_dot(J1, Xt) / (q4_m2(P0) * q4_m2(Pt));
            int qs[1] = { 2 };
            int f[1][3] = { { 2, ga, 3 } };
            q4_set_colour(&C[n], 1, qs, 2, ts, 1, (const int (*)[3])f, 2);
            ++n;
        }
    }
    /* class 6: both gluons on the spine (Xq with P0, Xt with Q) */
    Q4_SPINE(ta[0], mQ);
    q4_line(ub, v, mk2, m, width, 1, ta, Xt);
    for (int ga = 0; ga < 2; ++ga) {
        int gb = 1 - ga;
        double P1[4];
        for (int mu = 0; mu < 4; ++mu)
            P1[mu] = P0[mu] - kg[ga][mu];
        q4_v3(Xq, P0, eps[ga], kg[ga], J1);
        q4_v3(J1, P1, eps[gb], kg[gb], J2);
        A[n] = -q4_dot(J2, Xt) / (q4_m2(P0) * q4_m2(P1) * q4_m2(Q));
        int qs[1] = { 2 }, ts[1] = { 4 };
        int f[2][3] = { { 2, ga, 3 }, { 3, gb, 4 } };
        q4_set_colour(&C[n], 1, qs, 1, ts, 2, (const int (*)[3])f, 3);
        ++n;
    }
    {
        cplx q2 = q4_dot(Xq, eps[1]), q1 = q4_dot(Xq, eps[0]), qt = q4_dot(Xq, Xt);
        cplx t1 = q4_dot(eps[0], Xt), t2 = q4_dot(eps[1], Xt), e12 = q4_dot(eps[0], eps[1]);
        double den = q4_m2(P0) * q4_m2(Q);
        int qs[1] = { 2 }, ts[1] = { 3 };
        int f1[2][3] = { { 2, 0, 4 }, { 1, 3, 4 } };
        A[n] = -(q2 * t1 - qt * e12) / den;
        q4_set_colour(&C[n], 1, qs, 1, ts, 2, (const int (*)[3])f1, 3);
        ++n;
        int f2[2][3] = { { 2, 1, 4 }, { 0, 3, 4 } };
        A[n] = -(q1 * t2 - qt * e12) / den;
        q4_set_colour(&C[n], 1, qs, 1, ts, 2, (const int (*)[3])f2, 3);
        ++n;
        int f3[2][3] = { { 2, 3, 4 }, { 0, 1, 4 } };
        A[n] = -(q1 * t2 - q2 * t1) / den;
        q4_set_colour(&C[n], 1, qs, 1, ts, 2, (const int (*)[3])f3, 3);
        ++n;
    }
    /* class 7: the composite (colour slot 3, f^{3 0 1}) */
    {
        /* on the quark line (spine slot 2, carrying Q to the top line) */
        Q4_SPINE(ta[0], mQ);
        q4_line(ub, v, mk2, m, width, 1, ta, Xt);
        for (int oq = 0; oq < 2; ++oq) {
            int qs[2];
            Q4_COMP(qa[oq]);
            qs[oq] = 3;
            Q4_SPINE(qa[1 - oq], Q);
            qs[1 - oq] = 2;
            q4_line(vb, u, pa, 0.0, 0.0, 2, qa, Xq);
            A[n] = I1 * q4_dot(Xq, Xt) / q4_m2(Q);
            int ts[1] = { 2 };
            int f[1][3] = { { 3, 0, 1 } };
            q4_set_colour(&C[n], 2, qs, 1, ts, 1, (const int (*)[3])f, 2);
            ++n;
        }
        /* on the top line */
        Q4_SPINE(qa[0], P0);
        q4_line(vb, u, pa, 0.0, 0.0, 1, qa, Xq);
        for (int ot = 0; ot < 2; ++ot) {
            int ts[2];
            Q4_COMP(ta[ot]);
            ts[ot] = 3;
            Q4_SPINE(ta[1 - ot], mP0);
            ts[1 - ot] = 2;
            q4_line(ub, v, mk2, m, width, 2, ta, Xt);
            A[n] = I1 * q4_dot(Xq, Xt) / q4_m2(P0);
            int qs[1] = { 2 };
            int f[1][3] = { { 3, 0, 1 } };
            q4_set_colour(&C[n], 1, qs, 2, ts, 1, (const int (*)[3])f, 2);
            ++n;
        }
        /* on the spine: spine in slot 2, composite 4, spine out 3 */
        Q4_SPINE(ta[0], mQ);
        q4_line(ub, v, mk2, m, width, 1, ta, Xt);
        q4_v3(Xq, P0, J12, K, J1);
        A[n] = -q4_dot(J1, Xt) / (q4_m2(P0) * q4_m2(Q));
        int qs[1] = { 2 }, ts[1] = { 3 };
        int f[2][3] = { { 2, 4, 3 }, { 4, 0, 1 } };
        q4_set_colour(&C[n], 1, qs, 1, ts, 2, (const int (*)[3])f, 3);
        ++n;
    }
#undef Q4_GLUON
#undef Q4_COMP
#undef Q4_SPINE
    return n;
}

/* Value of a colour structure for the external colours ext[6] = (quark
 * colour i, antiquark anticolour j, top colour k, antitop anticolour l,
 * gluon adjoint indices a1, a2), the internal indices summed. */
static cplx q4_colour_value(const q4_colour *c, const int *ext)
{
    pthread_once(&qq_once, qq_colour_init);
    int slot[5];
    slot[0] = ext[4];
    slot[1] = ext[5];
    int nint = c->nint, total = 1;
    for (int x = 0; x < nint; ++x)
        total *= 8;
    cplx sum = 0;
    for (int code = 0; code < total; ++code) {
        int cc = code;
        for (int x = 0; x < nint; ++x) {
            slot[2 + x] = cc % 8;
            cc /= 8;
        }
        double fv = 1.0;
        for (int t = 0; t < c->nf; ++t)
            fv *= qq_f[slot[c->f[t][0]]][slot[c->f[t][1]]][slot[c->f[t][2]]];
        if (fv == 0.0)
            continue;
        /* quark line (T^{s_{n-1}} ... T^{s_0})_{j i}: a row vector from j */
        cplx rq[3] = { 0, 0, 0 };
        rq[ext[1]] = 1;
        for (int t = c->nq - 1; t >= 0; --t) {
            cplx nr[3] = { 0, 0, 0 };
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    nr[b] += rq[a] * qq_T[slot[c->qs[t]]][a][b];
            memcpy(rq, nr, sizeof(nr));
        }
        cplx rt[3] = { 0, 0, 0 };
        rt[ext[2]] = 1;
        for (int t = c->nt - 1; t >= 0; --t) {
            cplx nr[3] = { 0, 0, 0 };
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    nr[b] += rt[a] * qq_T[slot[c->ts[t]]][a][b];
            memcpy(rt, nr, sizeof(nr));
        }
        sum += fv * rq[ext[0]] * rt[ext[3]];
    }
    return sum;
}

static double complex q4_K[Q4_TERMS][Q4_TERMS];
static pthread_once_t q4_once = PTHREAD_ONCE_INIT;

/* K_de = sum over the 3^4 8^2 colour assignments of C_d conj(C_e). */
static void q4_K_init(void)
{
    static const double p[24] = { 0 };
    int hel[6] = { 0, 0, 0, 0, 0, 0 };
    cplx A[Q4_TERMS];
    q4_colour C[Q4_TERMS];
    (void)p;
    double pp[24] = { 300, 0, 0, 100, 300, 0, 0, -100, -400, 0, 0, -400, -400, 0, 0, 400,
                      100, 100, 0, 0, 100, -100, 0, 0 };
    int n = q4_terms(pp, 173.0, 0.0, hel, 0, A, C);
    static cplx val[5184][Q4_TERMS];
    for (int ci = 0; ci < 5184; ++ci) {
        int ext[6] = { ci % 3, (ci / 3) % 3, (ci / 9) % 3, (ci / 27) % 3, (ci / 81) % 8, ci / 648 };
        for (int d = 0; d < n; ++d)
            val[ci][d] = q4_colour_value(&C[d], ext);
    }
    for (int d = 0; d < n; ++d)
        for (int e = 0; e < n; ++e) {
            cplx s = 0;
            for (int ci = 0; ci < 5184; ++ci)
                s += val[ci][d] * conj(val[ci][e]);
            q4_K[d][e] = s;
        }
}

void mfo_qqbar_ttxgg_terms(const double *p, double m, double width, const int *hel, int ward, double *amp)
{
    cplx A[Q4_TERMS];
    q4_colour C[Q4_TERMS];
    q4_terms(p, m, width, hel, ward, A, C);
    for (int d = 0; d < Q4_TERMS; ++d) {
        amp[2 * d] = creal(A[d]);
        amp[2 * d + 1] = cimag(A[d]);
    }
}

void mfo_qqbar_ttxgg_colour(const int *cols, double *c)
{
    cplx A[Q4_TERMS];
    q4_colour C[Q4_TERMS];
    double pp[24] = { 300, 0, 0, 100, 300, 0, 0, -100, -400, 0, 0, -400, -400, 0, 0, 400,
                      100, 100, 0, 0, 100, -100, 0, 0 };
    int hel[6] = { 0, 0, 0, 0, 0, 0 };
    q4_terms(pp, 173.0, 0.0, hel, 0, A, C);
    for (int d = 0; d < Q4_TERMS; ++d) {
        cplx v = q4_colour_value(&C[d], cols);
        c[2 * d] = creal(v);
        c[2 * d + 1] = cimag(v);
    }
}

void mfo_qqbar_ttxgg_colour_matrix(double *K)
{
    pthread_once(&q4_once, q4_K_init);
    for (int d = 0; d < Q4_TERMS; ++d)
        for (int e = 0; e < Q4_TERMS; ++e) {
            K[2 * (d * Q4_TERMS + e)] = creal(q4_K[d][e]);
            K[2 * (d * Q4_TERMS + e) + 1] = cimag(q4_K[d][e]);
        }
}

/* Sum over the 64 helicity configurations of A^dagger K A, g = 1. */
double mfo_me2_qqbar_ttxgg(const double *p, double m, double width)
{
    pthread_once(&q4_once, q4_K_init);
    double total = 0.0;
    for (int h = 0; h < 64; ++h) {
        int hel[6] = { h & 1, (h >> 1) & 1, (h >> 2) & 1, (h >> 3) & 1, (h >> 4) & 1, (h >> 5) & 1 };
        cplx A[Q4_TERMS];
        q4_colour C[Q4_TERMS];
        int n = q4_terms(p, m, width, hel, 0, A, C);
        double s = 0.0;
        for (int d = 0; d < n; ++d) {
            cplx row = 0;
            for (int e = 0; e < n; ++e)
                row += q4_K[d][e] * conj(A[e]);
            s += creal(A[d] * row);
        }
        total += s;
    }
    return total;
}
