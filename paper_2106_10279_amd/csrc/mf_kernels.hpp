// mf_kernels.hpp -- gfx950 kernels of the per-event MadFlow integrand.
//
// One fused kernel evaluates chunks of 64 events per wavefront:
//   phase 1 (one event per lane): Philox uniforms -> VEGAS map -> partonic
//           kinematics -> flat phase space with massive rescaling -> cuts ->
//           PDFs; momenta and the event prefactor go to the wave's LDS slot;
//   phase 2 (one helicity configuration per lane): colour-summed |M_h|^2 of
//           the chunk's events from LDS, reduced over the helicity lanes;
//   phase 3 (one event per lane): weight, compensated sum w / w^2, per-bin
//           w^2 histogram owned lane-per-bin (deterministic), weight store.
// Each wave walks its chunks in a fixed order and writes one row of partial
// sums; a single-workgroup kernel reduces the rows in a fixed order and
// refines the VEGAS grid.  Sec. 2.2 (pipeline), 2.3 (matrix element), 2.4
// (phase space).
#pragma once

#include <type_traits>

#include "mf_device.hpp"
#include "mf_qqbar_ttxg.hpp"
#include "mf_qqbar_ttxgg.hpp"

namespace mf {

#include "_gen/amp_ng2.inc"
#include "_gen/amp_ng3.inc"
#include "_gen/amp_ng4.inc"
#include "_gen/amp_ng5.inc"

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kMaxDims = 13;
constexpr int kPartialHead = 8;         // sw.s, sw.c, sw2.s, sw2.c, w_max, n_pass, n_fail, spare
constexpr int kMaxPdfX = 256;
constexpr double kGeV2ToPb = 0.3893793721e9;
constexpr double kPi = 3.14159265358979323846;

struct EventParams {
    int n_g, n_dims, n_bins, max_newton;
    uint64_t n_events;
    uint64_t seed;
    uint32_t iter;
    const double* grid;              // [D][n_bins+1]
    const double* y_in;              // [n][D] or null
    const uint64_t* event_ids;       // [n] or null
    // PDF table (device) and the Q^2 stencil rows staged in LDS
    int n_x, n_q2, q2_first, q2_rows, q2_interval;
    const double* log_x;
    const double* log_q2;
    const double* xf;
    double log_muf2;
    // physics
    double sqrt_s, s_had, m_top, mw, ptmin, etamax, drmin;
    double me_norm;                  // g^(2n) / (4 64 (n-2)!) x (hbar c)^2 in pb
    double ps_const;                 // (2pi)^(4-3n) (pi/2)^(n-1) / ((n-1)! (n-2)!)
    // outputs
    double* weights;                 // [n] or null
    uint64_t* k53_out;               // [n][D] or null
    int32_t* bins_out;               // [n][D] or null
    double* partials;                // [n_waves][stride] or null
    double* record;                  // [n][8 + 4 NF] per-stage record or null
    int stride;
    int n_waves;
    int hel_mc;                      // 1: Monte Carlo over helicity configurations
    // p p initial state (g g -> t tbar plus the q qbar channels)
    int pp;                          // 1: add the q qbar channels
    const double* xq;                // [4][n_q2][n_x] x q for u, ubar, d, dbar (device)
    double me_norm_q;                // g^4 / (4 9) x (hbar c)^2 in pb
};

// Monte Carlo over helicities: lane `h` of an event holds the colour sum of
// |M_h|^2 for configuration h; with sampling only the event's drawn
// configuration counts, scaled by the number of configurations, so that the
// group sum over the event's lanes is N_h |M_h*|^2 (an unbiased estimate of
// the helicity sum).
template <int NHEL>
__device__ __forceinline__ double hel_sampled(double v, int h, uint64_t event, uint64_t seed, uint32_t iter)
{
    return h == hel_config(event, seed, iter, NHEL) ? (double)NHEL * v : 0.0;
}

// ---------------------------------------------------------------------------
// VEGAS map.  The bin index and the position in the bin come from the exact
// integer product k n_bins; the map itself is evaluated without contraction
// so that x, the bin index and J_V are reproducible operation by operation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double vegas_map_dim(const double* __restrict__ e, int i, double delta, double& jd,
                                                int n_bins)
{
#pragma clang fp contract(off)
    const double lo = e[i], hi = e[i + 1];
    const double width = hi - lo;
    const double shift = delta * width;
    jd = (double)n_bins * width;
    return lo + shift;
}

// ---------------------------------------------------------------------------
// Phase space, cuts and PDF are evaluated without FMA contraction: they cost
// little next to |M|^2, and a fixed operation order keeps ill-conditioned
// spots (sqrt(1 - cos^2), boosts, Hermite sums) reproducible.
//
// Flat n-body phase space with 3n-4 uniforms, then massive rescaling.
// Slots: 0 = t, 1 = tbar (mass m), 2.. = gluons (massless).  Returns false
// when the Newton iteration on xi does not converge within max_newton steps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void boost_from_rest(const double* Q, double M, const double* v, double* out)
{
#pragma clang fp contract(off)
    const double qv = Q[1] * v[1] + Q[2] * v[2] + Q[3] * v[3];
    const double e = (Q[0] * v[0] + qv) / M;
    const double c = (v[0] + e) / (Q[0] + M);
    out[0] = e;
    out[1] = v[1] + c * Q[1];
    out[2] = v[2] + c * Q[2];
    out[3] = v[3] + c * Q[3];
}

// The mass-ratio equation of degree 3, 4u^3 - 3u^4 = r (increasing on
// [0, 1]): Newton steps kept inside a bisection bracket, until a step falls
// below the spacing of doubles at the iterate.
__device__ __forceinline__ double mass_ratio3(double r)
{
#pragma clang fp contract(off)
    if (!(r > 0.0))
        return 0.0;
    if (!(r < 1.0))
        return 1.0;
    double lo = 0.0, hi = 1.0, u = 0.5;
    for (int it = 0; it < 200; ++it) {
        const double u2 = u * u;
        const double f = 4.0 * u2 * u - 3.0 * u2 * u2 - r;
        if (f == 0.0)
            return u;
        if (f < 0.0)
            lo = u;
        else
            hi = u;
        const double fp = 12.0 * u2 * (1.0 - u);
        double un = u - f / fp;
        if (!(un > lo && un < hi))
            un = 0.5 * (lo + hi);
        if (fabs(un - u) <= 0x1p-52 * un)
            return un;
        u = un;
    }
    return u;
}

template <int NF>
__device__ bool phase_space(const double* __restrict__ r, double rs, double m, int max_newton, double ps_const,
                            double (&k)[NF][4], double& W)
{
#pragma clang fp contract(off)
    double M[NF + 1];
    double p[NF][4];
    M[1] = rs;
#pragma unroll
    for (int i = 2; i <= NF - 1; ++i) {
        const int power = NF - i;
        const double ri = r[i - 2];
        const double u = (power == 1) ? 1.0 - sqrt(1.0 - ri)
                         : (power == 2 ? 0.5 - sin(asin(1.0 - 2.0 * ri) / 3.0) : mass_ratio3(ri));
        M[i] = sqrt(u) * M[i - 1];
    }
    M[NF] = 0.0;
    double Q[4] = {rs, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 1; i <= NF - 1; ++i) {
        const double cth = 2.0 * r[(NF - 2) + 2 * (i - 1)] - 1.0;
        const double phi = 2.0 * kPi * r[(NF - 2) + 2 * (i - 1) + 1];
        const double sth = sqrt(1.0 - cth * cth);
        const double q = (M[i] * M[i] - M[i + 1] * M[i + 1]) / (2.0 * M[i]);
        double sp, cp;
        sincos(phi, &sp, &cp);
        const double prest[4] = {q, q * sth * cp, q * sth * sp, q * cth};
        const double qrest[4] = {sqrt(q * q + M[i + 1] * M[i + 1]), -prest[1], -prest[2], -prest[3]};
        double Qn[4];
        boost_from_rest(Q, M[i], prest, p[i - 1]);
        boost_from_rest(Q, M[i], qrest, Qn);
        Q[0] = Qn[0]; Q[1] = Qn[1]; Q[2] = Qn[2]; Q[3] = Qn[3];
    }
    p[NF - 1][0] = Q[0]; p[NF - 1][1] = Q[1]; p[NF - 1][2] = Q[2]; p[NF - 1][3] = Q[3];

    double w0 = ps_const;
#pragma unroll
    for (int i = 0; i < NF - 2; ++i)
        w0 *= rs * rs;

    // xi such that sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt(s)
    const double msum = 2.0 * m;
    double xi = sqrt(1.0 - (msum / rs) * (msum / rs));
    const double floor_res = 2.0 * NF * 0x1p-52 * rs;
    bool converged = false;
    for (int it = 0; it < max_newton; ++it) {
        double f = -rs, fp = 0.0;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const double mi = i < 2 ? m : 0.0;
            const double e = sqrt(mi * mi + xi * xi * p[i][0] * p[i][0]);
            f += e;
            fp += xi * p[i][0] * p[i][0] / e;
        }
        if (fabs(f) <= floor_res) {
            converged = true;
            break;
        }
        const double step = f / fp;
        xi = xi - step;
        if (fabs(step) <= 1e-15 * xi) {
            converged = true;
            break;
        }
    }
    if (!converged) {
        W = 0.0;
        return false;
    }
    double sum_abs = 0.0, prod_ratio = 1.0, sum_sq_over_e = 0.0;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const double mi = i < 2 ? m : 0.0;
        const double e = sqrt(mi * mi + xi * xi * p[i][0] * p[i][0]);
        k[i][0] = e;
        k[i][1] = xi * p[i][1];
        k[i][2] = xi * p[i][2];
        k[i][3] = xi * p[i][3];
        const double a = sqrt(k[i][1] * k[i][1] + k[i][2] * k[i][2] + k[i][3] * k[i][3]);
        sum_abs += a;
        prod_ratio *= a / e;
        sum_sq_over_e += a * a / e;
    }
    double pw = 1.0;
    const double ratio = sum_abs / rs;
#pragma unroll
    for (int i = 0; i < 2 * NF - 3; ++i)
        pw *= ratio;
    W = w0 * pw * prod_ratio * rs / sum_sq_over_e;
    return true;
}

__device__ __forceinline__ double pseudorapidity(const double* k)
{
#pragma clang fp contract(off)
    const double a = sqrt(k[1] * k[1] + k[2] * k[2] + k[3] * k[3]);
    return 0.5 * log((a + k[3]) / (a - k[3]));
}

// Strict inequalities on the final-state gluons: pT, |eta_lab|, Delta R.
template <int NF>
__device__ __forceinline__ bool pass_cuts(const double (&k)[NF][4], double y_boost, double ptmin, double etamax,
                                          double drmin)
{
#pragma clang fp contract(off)
    bool pass = true;
#pragma unroll
    for (int i = 2; i < NF; ++i) {
        if (ptmin > 0.0) {
            const double pt = sqrt(k[i][1] * k[i][1] + k[i][2] * k[i][2]);
            pass = pass && (pt > ptmin);
        }
        if (etamax > 0.0) {
            const double eta = fabs(pseudorapidity(k[i]) + y_boost);
            pass = pass && (eta < etamax);
        }
    }
    if (drmin > 0.0) {
#pragma unroll
        for (int i = 2; i < NF; ++i)
#pragma unroll
            for (int j = i + 1; j < NF; ++j) {
                const double deta = pseudorapidity(k[i]) - pseudorapidity(k[j]);
                double dphi = fabs(atan2(k[i][2], k[i][1]) - atan2(k[j][2], k[j][1]));
                if (dphi > kPi)
                    dphi = 2.0 * kPi - dphi;
                pass = pass && (sqrt(deta * deta + dphi * dphi) > drmin);
            }
    }
    return pass;
}

// ---------------------------------------------------------------------------
// PDF: cubic Hermite in ln x on each staged Q^2 row, then in ln Q^2.  Knot
// slopes: mean of the adjacent secants inside, one-sided at the ends.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double knot_slope(const double* t, const double* f, int i, int last)
{
#pragma clang fp contract(off)
    if (i == 0)
        return (f[1] - f[0]) / (t[1] - t[0]);
    if (i == last)
        return (f[i] - f[i - 1]) / (t[i] - t[i - 1]);
    return 0.5 * ((f[i] - f[i - 1]) / (t[i] - t[i - 1]) + (f[i + 1] - f[i]) / (t[i + 1] - t[i]));
}

__device__ __forceinline__ double hermite(const double* t, const double* f, int i, int last, double v)
{
#pragma clang fp contract(off)
    const double h = t[i + 1] - t[i];
    const double u = (v - t[i]) / h;
    const double u2 = u * u, u3 = u2 * u;
    const double h00 = 2.0 * u3 - 3.0 * u2 + 1.0;
    const double h10 = u3 - 2.0 * u2 + u;
    const double h01 = -2.0 * u3 + 3.0 * u2;
    const double h11 = u3 - u2;
    return h00 * f[i] + h10 * h * knot_slope(t, f, i, last) + h01 * f[i + 1] + h11 * h * knot_slope(t, f, i + 1, last);
}

__device__ __forceinline__ int find_interval(const double* knots, int n, double v)
{
    if (v < knots[0])
        return 0;
    if (v >= knots[n - 1])
        return n - 2;
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (knots[mid] <= v)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// The table's values at mu_F^2 on every x knot, staged once per workgroup:
// the cubic Hermite interpolation in ln Q^2 over the four bracketing Q^2 rows
// is done per knot, so an event interpolates in ln x only.  Both steps are
// linear in the table values along their own axis (the knot slopes too), so
// taking ln Q^2 first gives the same interpolant as taking ln x first.
// xf: [n_q2][n_x] in device memory, row: [n_x] in LDS.
__device__ __forceinline__ void stage_pdf_row(const EventParams& P, const double* __restrict__ xf, double* row,
                                              int tid, int nthreads)
{
    double lq[4], rv[4];
    for (int r = 0; r < P.q2_rows; ++r)
        lq[r] = P.log_q2[P.q2_first + r];
    for (int i = tid; i < P.n_x; i += nthreads) {
        for (int r = 0; r < P.q2_rows; ++r)
            rv[r] = xf[(size_t)(P.q2_first + r) * P.n_x + i];
        row[i] = hermite(lq, rv, P.q2_interval - P.q2_first, P.q2_rows - 1, P.log_muf2);
    }
}

// x g(x, mu_F^2) from the staged row; lx_knots: LDS [n_x].
__device__ __forceinline__ double pdf_xg(const EventParams& P, const double* row, const double* lx_knots, double x)
{
    const double lx = log(x);
    const int k = find_interval(lx_knots, P.n_x, lx);
    return hermite(lx_knots, row, k, P.n_x - 1, lx);
}

// The four quark tables (u, ubar, d, dbar; staged rows at f * n_x) at one x:
// one logarithm and one interval search for all of them, divided by x.
__device__ __forceinline__ void pdf_xq4(const EventParams& P, const double* rows, const double* lx_knots, double x,
                                        double* q)
{
    const double lx = log(x);
    const int k = find_interval(lx_knots, P.n_x, lx);
#pragma unroll
    for (int f = 0; f < 4; ++f)
        q[f] = hermite(lx_knots, rows + f * P.n_x, k, P.n_x - 1, lx) / x;
}

// Reduce v over groups of `width` consecutive lanes; lane 0 of each group
// receives the sum in a fixed association order.
__device__ __forceinline__ double group_sum(double v, int width)
{
    for (int off = width >> 1; off > 0; off >>= 1)
        v += __shfl_down(v, off, width);
    return v;
}

// Table element type: double for the per-lane evaluation (n_g = 2), the
// amplitude type for the cooperative one (its table entries are only ever
// read converted to that type).
template <int NG, typename T>
using TabT = std::conditional_t<(NG >= 3), T, double>;

// Per-event table (and, for n_g >= 3, the level-1 currents of the object
// store) from the momenta, written by the lanes of one event.
template <int NG, typename T>
__device__ __forceinline__ void fill_table(const double* mom, double eb, double mt, double mw, TabT<NG, T>* tab,
                                           T* obj, int lane)
{
    if constexpr (NG == 2)
        fill_table_ng2(mom, eb, mt, mw, tab, lane);
    else if constexpr (NG == 3)
        fill_table_coop_ng3<T>(mom, eb, mt, mw, tab, obj, lane);
    else
        fill_table_coop_ng4<T>(mom, eb, mt, mw, tab, obj, lane);
}

// Momenta stored per event: t[4], tbar[4], final gluons[4 each], beam energy.
template <int NG>
struct Layout {
    static constexpr int kMom = 8 + 4 * (NG - 2) + 1;
    static constexpr int kHel = 1 << (NG + 2);
    static constexpr int kEventsPerPass = kHel <= kWave ? kWave / kHel : 1;   // 4, 2, 1 (t tbar g g g: a workgroup)
    static constexpr int kTable = NG == 2 ? TABLE_NG2
                                  : (NG == 3 ? COOP_TABLE_NG3 : (NG == 4 ? COOP_TABLE_NG4 : COOP_TABLE_NG5));
    // helicity-recycled object store per event (units of the amplitude type)
    static constexpr bool kCoop = NG >= 3;
    static constexpr int kObj = NG == 2 ? 1 : (NG == 3 ? COOP_OBJ_NG3 : (NG == 4 ? COOP_OBJ_NG4 : COOP_OBJ_NG5));
    // objects sit at multiples of 4 elements: 16-byte aligned in every event's store
    static_assert(!kCoop || kObj % 4 == 0, "object store rows must keep 16-byte alignment");
};

// Colour-summed |M|^2 of helicity `h` for the event whose table is `tab`:
// lanes of the event (h = 0 .. 2^(NG+2) - 1) build the object store first
// (n_g >= 3).  `any_live` must be uniform over the wave.  COL = 0: full
// colour matrix; COL = 1: leading-colour approximation; COL = 2: one sampled
// colour assignment whose complex factors are cf; COL = 3: one sampled colour
// flow whose real factors are cf (n_g >= 3; Sec. 3.2, discussing Fig. 4, names leading colour and
// colour sampling).
template <int NG, typename T, int COL = 0>
__device__ __forceinline__ double event_me2(const TabT<NG, T>* tab, T* obj, int h, double mt, bool live, bool any_live,
                                            const T* cf = nullptr)
{
    using L = Layout<NG>;
    if constexpr (L::kCoop) {
        if (any_live) {
            if constexpr (NG == 3)
                coop_stages_ng3<T>(tab, obj, mt, h, L::kHel);
            else
                coop_stages_ng4<T>(tab, obj, mt, h, L::kHel);
        }
        if (!live)
            return 0.0;
        if constexpr (NG == 3)
            return coop_me2_ng3<T, COL>(tab, obj, cf, h);
        else
            return coop_me2_ng4<T, COL>(tab, obj, cf, h);
    } else {
        static_assert(COL < 2, "the Monte Carlo over colours runs for n_g >= 3 only");
        return live ? colour_summed_me2_ng2<T, COL>(tab, h, mt) : 0.0;
    }
}

// The point of one event in the unit hypercube and its VEGAS map: Philox
// words (or the caller's uniforms), integer bins, x and J_V (returned).
// bins[d * bin_stride] receives the bin of dimension d; k53_out and bins_out
// of P are written if set.
template <int D>
__device__ __forceinline__ double draw_point(const EventParams& P, uint64_t ev, double (&x)[D],
                                             unsigned short* bins, size_t bin_stride)
{
    const int nb = P.n_bins;
    const uint32_t key0 = (uint32_t)P.seed, key1 = (uint32_t)(P.seed >> 32);
    double jac = 1.0;
    if (P.y_in) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double y = P.y_in[ev * D + d];
            const double t = y * (double)nb;
            int b = (int)floor(t);
            b = b > nb - 1 ? nb - 1 : (b < 0 ? 0 : b);
            double jd;
            x[d] = vegas_map_dim(P.grid + d * (nb + 1), b, t - (double)b, jd, nb);
            jac = jac * jd;
            bins[d * bin_stride] = (unsigned short)b;
            if (P.bins_out)
                P.bins_out[ev * D + d] = b;
        }
    } else {
        const uint64_t eid = P.event_ids ? P.event_ids[ev] : ev;
#pragma unroll
        for (int blk = 0; blk < (D + 1) / 2; ++blk) {
            uint32_t r[4];
            philox4x32_10((uint32_t)eid, (uint32_t)(eid >> 32), P.iter, (uint32_t)blk, key0, key1, r);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int d = 2 * blk + h;
                if (d < D) {
                    const uint64_t kk = ((((uint64_t)r[2 * h]) << 32) | (uint64_t)r[2 * h + 1]) >> 11;
                    const uint64_t prod = kk * (uint64_t)nb;
                    const int b = (int)(prod >> 53);
                    const double delta = (double)(prod & ((1ull << 53) - 1)) * 0x1p-53;
                    double jd;
                    x[d] = vegas_map_dim(P.grid + d * (nb + 1), b, delta, jd, nb);
                    jac = jac * jd;
                    bins[d * bin_stride] = (unsigned short)b;
                    if (P.k53_out)
                        P.k53_out[ev * D + d] = kk;
                    if (P.bins_out)
                        P.bins_out[ev * D + d] = b;
                }
            }
        }
    }
    return jac;
}

// Phase 1 of one event (one lane): the point and its VEGAS map, threshold,
// phase space with the massive rescaling, cuts and the two PDFs.  Returns
// the flags (bit 0 above threshold, bit 1 Newton failed, bit 2 passed the
// cuts).  For a passing event the momenta and the beam energy go to
// mom[0 .. 4 NF] and pref = J_V W f1 f2 / (2 s_hat); otherwise pref = 0 and
// mom is untouched.  bins[d * bin_stride] receives the bin of dimension d;
// k53_out, bins_out and record of P are written if set.
template <int NF>
__device__ __forceinline__ int event_kinematics(const EventParams& P, uint64_t ev, const double* s_row,
                                                const double* s_lx, unsigned short* bins,
                                                size_t bin_stride, double* mom, double& pref,
                                                const double* s_qrows = nullptr, double* pref_q = nullptr)
{
    constexpr int D = 2 + 3 * NF - 4;
    pref = 0.0;
    double x[D];
    const double jac = draw_point<D>(P, ev, x, bins, bin_stride);
    const double x1 = x[0], x2 = x[1];
    const double shat = x1 * x2 * P.sqrt_s * P.sqrt_s;
    const double thr = 2.0 * P.m_top;
    double* rec = P.record ? P.record + ev * (8 + 4 * NF) : nullptr;
    double W = 0.0, f1 = 0.0, f2 = 0.0;
    int flags = 0;
    double k[NF][4];
    if (shat > thr * thr) {
        flags |= 1;
        const double rs = sqrt(shat);
        if (phase_space<NF>(x + 2, rs, P.m_top, P.max_newton, P.ps_const, k, W)) {
            const double y_boost = 0.5 * log(x1 / x2);
            if (pass_cuts<NF>(k, y_boost, P.ptmin, P.etamax, P.drmin)) {
                flags |= 4;
                f1 = pdf_xg(P, s_row, s_lx, x1) / x1;
                f2 = pdf_xg(P, s_row, s_lx, x2) / x2;
                pref = jac * W * f1 * f2 / (2.0 * shat);
                if (s_qrows && pref != 0.0) {
                    // q qbar luminosities, number densities: the quark from beam 1
                    // (u ubar, d dbar) and from beam 2 (ubar u, dbar d).  For t tbar
                    // the summed q qbar |M|^2 is the same for both orientations
                    // (symmetric under t <-> u at tree level) and one prefactor
                    // carries both; for t tbar g they differ.
                    double q1[4], q2[4];
                    pdf_xq4(P, s_qrows, s_lx, x1, q1);
                    pdf_xq4(P, s_qrows, s_lx, x2, q2);
                    const double lf = q1[0] * q2[1] + q1[2] * q2[3];
                    const double lr = q1[1] * q2[0] + q1[3] * q2[2];
                    if constexpr (NF == 2) {
                        pref_q[0] = jac * W * (lf + lr) / (2.0 * shat);
                    } else {
                        pref_q[0] = jac * W * lf / (2.0 * shat);
                        pref_q[1] = jac * W * lr / (2.0 * shat);
                    }
                }
#pragma unroll
                for (int i = 0; i < NF; ++i)
#pragma unroll
                    for (int mu = 0; mu < 4; ++mu)
                        mom[4 * i + mu] = k[i][mu];
                mom[4 * NF] = 0.5 * rs;
            }
        } else {
            flags |= 2;
        }
    }
    if (rec) {
        rec[0] = x1;
        rec[1] = x2;
        rec[2] = jac;
        rec[3] = W;
        rec[4] = f1;
        rec[5] = f2;
        rec[7] = (double)flags;
#pragma unroll
        for (int i = 0; i < NF; ++i)
#pragma unroll
            for (int mu = 0; mu < 4; ++mu)
                rec[8 + 4 * i + mu] = (flags & 1) && !(flags & 2) ? k[i][mu] : 0.0;
    }
    return flags;
}

// g g -> t tbar is bound by latency more than by issue: three resident waves
// per SIMD (at most 168 registers, a few loop invariants spilled) run it
// faster than two without spills.  The heavier processes keep their registers.
template <int NG, typename T, int COL = 0>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NG == 2 ? 3 : 1)))
event_kernel(EventParams P)
{
    constexpr int NF = NG;
    constexpr int D = 2 + 3 * NF - 4;
    using L = Layout<NG>;
    __shared__ double s_mom[kWavesPerBlock][kWave][L::kMom];
    __shared__ double s_pref[kWavesPerBlock][kWave];
    __shared__ double s_me[kWavesPerBlock][kWave];
    __shared__ unsigned short s_bin[kWavesPerBlock][D][kWave];
    __shared__ double s_lx[kMaxPdfX];
    __shared__ double s_row[kMaxPdfX];
    __shared__ __align__(16) TabT<NG, T> s_tab[kWavesPerBlock][L::kEventsPerPass][L::kTable];
    __shared__ __align__(16) T s_obj[kWavesPerBlock][L::kEventsPerPass][L::kObj];
    extern __shared__ double s_hist[];     // [kWavesPerBlock][D][n_bins]

    const int tid = threadIdx.x;
    const int wv = tid / kWave;
    const int lane = tid % kWave;
    const int wave_id = blockIdx.x * kWavesPerBlock + wv;
    const int nb = P.n_bins;

    // Stage ln x knots and the PDF table at mu_F^2 in LDS.
    for (int i = tid; i < P.n_x; i += kBlock)
        s_lx[i] = P.log_x[i];
    stage_pdf_row(P, P.xf, s_row, tid, kBlock);
    double* hist = s_hist + (size_t)wv * D * nb;
    if (P.partials)
        for (int i = lane; i < D * nb; i += kWave)
            hist[i] = 0.0;
    __syncthreads();

    Neumaier sw{0.0, 0.0}, sw2{0.0, 0.0};
    double wmax = 0.0, npass = 0.0, nfail = 0.0;
    const uint64_t n_chunks = (P.n_events + kWave - 1) / kWave;
    const uint32_t key0 = (uint32_t)P.seed, key1 = (uint32_t)(P.seed >> 32);

    for (uint64_t chunk = wave_id; chunk < n_chunks; chunk += P.n_waves) {
        // ---------------- phase 1: one event per lane ----------------------
        const uint64_t ev = chunk * kWave + lane;
        const bool active = ev < P.n_events;
        double pref = 0.0;
        double* mom = s_mom[wv][lane];
        if (active) {
            const int flags = event_kinematics<NF>(P, ev, s_row, s_lx, &s_bin[wv][0][lane], kWave, mom, pref);
            if (flags & 4)
                npass += 1.0;
            if (flags & 2)
                nfail += 1.0;
        }
        s_pref[wv][lane] = pref;
        wave_sync();

        // ---------------- phase 2: one helicity configuration per lane -----
        // The lanes of each event first fill its table of momentum-only
        // quantities, then every lane evaluates one helicity configuration.
        {
            const int h0 = lane % L::kHel;
            const int sub = lane / L::kHel;
            TabT<NG, T>* tab = s_tab[wv][sub];
            T* obj = s_obj[wv][sub];
            for (int g = 0; g < kWave / L::kEventsPerPass; ++g) {
                // opaque per iteration, so that lane-dependent addresses of the
                // table and object store are not hoisted out of this loop
                int h = h0;
                asm volatile("" : "+v"(h));
                const int e = g * L::kEventsPerPass + sub;
                const double* m_e = s_mom[wv][e];
                const bool live = s_pref[wv][e] != 0.0;
                const bool any_live = __any(live);
                if (live)
                    fill_table<NG, T>(m_e, m_e[L::kMom - 1], P.m_top, P.mw, tab, obj, h);
                wave_sync();
                double v = event_me2<NG, T, COL>(tab, obj, h, P.m_top, live, any_live);
                if (P.hel_mc && live) {
                    const uint64_t ev_e = chunk * kWave + e;
                    v = hel_sampled<L::kHel>(v, h, P.event_ids ? P.event_ids[ev_e] : ev_e, P.seed, P.iter);
                }
                v = group_sum(v, L::kHel);
                if (h == 0)
                    s_me[wv][e] = v;
                wave_sync();
            }
        }
        wave_sync();

        // ---------------- phase 3: one event per lane ----------------------
        const double w = pref * (s_me[wv][lane] * P.me_norm);
        if (active) {
            if (P.record)
                P.record[ev * (8 + 4 * NF) + 6] = pref != 0.0 ? s_me[wv][lane] : 0.0;
            if (P.weights)
                P.weights[ev] = w;
            nm_add(sw, w);
            nm_add(sw2, w * w);
            wmax = fmax(wmax, w);
        }
        if (P.partials) {
            s_me[wv][lane] = active ? w * w : 0.0;
            wave_sync();
            for (int b = lane; b < nb; b += kWave) {
                for (int d = 0; d < D; ++d) {
                    double acc = hist[d * nb + b];
                    for (int e = 0; e < kWave; ++e)
                        if (s_bin[wv][d][e] == b)
                            acc += s_me[wv][e];
                    hist[d * nb + b] = acc;
                }
            }
        }
        wave_sync();
    }

    if (P.partials) {
        // Fixed-order wave reduction of the lane partials.
        for (int off = kWave >> 1; off > 0; off >>= 1) {
            Neumaier o1{__shfl_down(sw.s, off), __shfl_down(sw.c, off)};
            Neumaier o2{__shfl_down(sw2.s, off), __shfl_down(sw2.c, off)};
            const double om = __shfl_down(wmax, off);
            const double op = __shfl_down(npass, off);
            const double of = __shfl_down(nfail, off);
            sw = nm_merge(sw, o1);
            sw2 = nm_merge(sw2, o2);
            wmax = fmax(wmax, om);
            npass += op;
            nfail += of;
        }
        // entry-major rows: entry k of wave w at partials[k * n_waves + w]
        double* out = P.partials + wave_id;
        const size_t nw = (size_t)P.n_waves;
        if (lane == 0) {
            out[0 * nw] = sw.s;
            out[1 * nw] = sw.c;
            out[2 * nw] = sw2.s;
            out[3 * nw] = sw2.c;
            out[4 * nw] = wmax;
            out[5 * nw] = npass;
            out[6 * nw] = nfail;
            out[7 * nw] = 0.0;
        }
        for (int i = lane; i < D * nb; i += kWave)
            out[(kPartialHead + i) * nw] = hist[i];
    }
}

// ---------------------------------------------------------------------------
// Three-kernel form for the amplitude-heavy processes (g g -> t tbar g and
// t tbar g g).  The fused event kernel needs phase 1's registers and LDS
// (momenta of 64 events, PDF rows, histogram) next to the amplitude stages,
// which leaves one wave per SIMD.  Here phase 1 and phase 3 run as their own
// kernels and hand over per-event data through HBM (about 170 B per event),
// and the amplitude kernel runs one wave per workgroup with only the table
// and the object store in LDS, so several waves share each SIMD.  Per-event
// values are those of the fused kernel, operation for operation.
// ---------------------------------------------------------------------------
struct StageParams {
    EventParams P;           // forward parameters; P.n_waves = waves of kin/acc
    uint64_t first, count;   // global index of the batch's first event, events in the batch
    double* mom;             // [count][4 NF + 1] momenta and beam energy (passing events)
    double* pref;            // [count] J_V W f1 f2 / (2 s_hat), 0 for rejected events
    double* me;              // [count] sum over helicities and colours of |M|^2 (passing events)
    unsigned short* bins;    // [D][count]
    unsigned char* flags;    // [count] event_kinematics flags
    int first_batch;         // acc: 1 = start the per-wave partials from zero
    unsigned long long* next_group;  // amp: work counter, cleared by kin_kernel
    void* amps;              // t tbar g g g: [count][120][128][re, im] partial amplitudes (type T)
    double* pref_q;          // p p: J_V W L_qqbar / (2 s_hat); t tbar: [count], both beam orientations,
                             // t tbar g: [2][count], the quark from beam 1 / beam 2
    double* me_q;            // p p: q qbar |M|^2 summed over helicities and colours; [count] / [2][count]
    // Optional list of the batch's events with a non-zero prefactor, in no
    // particular order (kin_kernel appends, n_live cleared before it); the
    // amplitude kernels of n_g <= 4 then take only these.  nullptr: all
    // events in order.
    unsigned* live = nullptr;
    unsigned long long* n_live = nullptr;
};

template <int NF, bool PP = false>
__global__ void __launch_bounds__(kBlock) kin_kernel(StageParams S)
{
    const EventParams& P = S.P;
    __shared__ double s_lx[kMaxPdfX];
    __shared__ double s_row[kMaxPdfX];
    __shared__ double s_qrows[PP ? 4 * kMaxPdfX : 1];   // p p: the quark tables at mu_F^2
    const int tid = threadIdx.x;
    const int lane = tid % kWave;
    const int wave_id = blockIdx.x * kWavesPerBlock + tid / kWave;
    if (blockIdx.x == 0 && tid == 0)
        *S.next_group = 0ull;
    for (int i = tid; i < P.n_x; i += kBlock)
        s_lx[i] = P.log_x[i];
    stage_pdf_row(P, P.xf, s_row, tid, kBlock);
    if constexpr (PP) {
        for (int f = 0; f < 4; ++f)
            stage_pdf_row(P, P.xq + (size_t)f * P.n_q2 * P.n_x, s_qrows + f * P.n_x, tid, kBlock);
    }
    __syncthreads();
    const uint64_t n_chunks = (S.count + kWave - 1) / kWave;
    // a wave takes the chunks wave_id + k n_waves; kLiveBatch of them at a
    // time, so that the live events of all of them are appended with one
    // atomic (one counter for the whole batch)
    constexpr int kLiveBatch = 8;
    for (uint64_t c0 = wave_id; c0 < n_chunks; c0 += (uint64_t)kLiveBatch * P.n_waves) {
        unsigned live = 0u;                       // bit t: the event of chunk t is live
#pragma unroll 1
        for (int t = 0; t < kLiveBatch; ++t) {
            const uint64_t e = (c0 + (uint64_t)t * P.n_waves) * kWave + lane;
            if (e < S.count) {
                double pref, pq[2] = {0.0, 0.0};
                const int flags = event_kinematics<NF>(P, S.first + e, s_row, s_lx, S.bins + e, S.count,
                                                       S.mom + e * (4 * NF + 1), pref, PP ? s_qrows : nullptr, pq);
                S.pref[e] = pref;
                S.flags[e] = (unsigned char)flags;
                if constexpr (PP) {
                    S.pref_q[e] = pq[0];
                    if constexpr (NF >= 3)
                        S.pref_q[S.count + e] = pq[1];
                }
                live |= (pref != 0.0 ? 1u : 0u) << t;
            }
        }
        if (S.live) {
            unsigned long long mask[kLiveBatch];
            unsigned long long total = 0;
#pragma unroll
            for (int t = 0; t < kLiveBatch; ++t) {
                mask[t] = __ballot((live >> t) & 1u);
                total += (unsigned long long)__popcll(mask[t]);
            }
            if (total) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(S.n_live, total);
                base = __shfl(base, 0);
                const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
                for (int t = 0; t < kLiveBatch; ++t) {
                    if ((live >> t) & 1u)
                        S.live[base + __popcll(mask[t] & below)] =
                            (unsigned)((c0 + (uint64_t)t * P.n_waves) * kWave + lane);
                    base += (unsigned long long)__popcll(mask[t]);
                }
            }
        }
    }
}

// One wave per workgroup; a persistent loop over groups of events (one event
// per pass for t tbar g g, two for t tbar g).  The waves take chunks of
// kAmpChunk groups from a device counter (cleared by kin_kernel), so that
// they all finish within about one chunk of each other; each event's |M|^2
// is written by whichever wave evaluates it, so the results do not depend on
// the order.  The chunk after the current one is claimed one chunk ahead,
// and the prefactor and momenta of the next group are loaded while the
// current one is evaluated (lane h < kMom of each event holds one stored
// momentum component).  Groups without a passing event are skipped whole.
constexpr int kAmpChunk = 16;

// t tbar g: the table fill (divisions, square roots, lane groups on different
// paths) costs about as much per pass whether it serves one event or more,
// and next to the short 32-helicity amplitudes of this process it is a large
// share of the work.  A wave therefore fills the tables of four events at
// once (16 lanes each), then builds the objects and evaluates the helicities
// of two pairs of them in turn (32 helicity lanes per event).  The level-1
// currents that the fill writes go to an extension of each event's table and
// are copied into the pair's object store before its stages.  The chunks of
// the work counter stay in units of pairs (kAmpChunk pairs = kAmpChunk / 2
// quads), and the results do not depend on the grouping.
template <typename T, int COL>
__device__ __forceinline__ void amp_quads_ng3(const StageParams& S)
{
    using L = Layout<3>;
    constexpr int kQ = 4;                    // events per fill pass
    constexpr int kL1 = 4 * 2 * 3;           // level-1 currents of an event, in T
    static_assert(kQ * L::kMom <= kWave && kQ * 16 == kWave && 2 * L::kHel == kWave, "quad layout");
    static_assert(L::kTable % 4 == 0, "16-byte aligned table rows");
    __shared__ __align__(16) T s_tab[kQ][L::kTable + kL1];
    __shared__ __align__(16) T s_obj[2][L::kObj];
    __shared__ double s_mom[kQ][L::kMom];
    constexpr int kCf = COL >= 2 ? 2 * 6 : 2;
    __shared__ __align__(16) T s_cf[2][kCf];
    const int lane = threadIdx.x;
    const int h0 = lane % L::kHel, sub = lane / L::kHel;      // helicity phase: 2 events x 32 lanes
    const int fq = lane / 16, fl0 = lane % 16;                // fill: 4 events x 16 lanes
    const int mq = lane / L::kMom, mk = lane % L::kMom;       // momenta: 4 events x 13 values
    // the events to evaluate: the live list, or all events in order
    const uint64_t n_ev = S.live ? (uint64_t)*S.n_live : S.count;
    const uint64_t n_quads = (n_ev + kQ - 1) / kQ;
    auto claim = [&]() -> uint64_t {
        unsigned long long c = 0;
        if (lane == 0)
            c = atomicAdd(S.next_group, (unsigned long long)kAmpChunk);
        return (uint64_t)__shfl(c, 0) / 2;   // pairs -> quads
    };
    auto event_of = [&](uint64_t i) -> uint64_t { return S.live ? (uint64_t)S.live[i] : i; };
    // the fill lanes' event (S.count if none) and prefactor, the momenta lanes' value
    auto load = [&](uint64_t qd, double& pref, double& mc, uint64_t& ef) {
        const uint64_t i = qd * kQ + fq, im = qd * kQ + mq;
        pref = 0.0;
        mc = 0.0;
        ef = S.count;
        if (qd < n_quads) {
            if (i < n_ev) {
                ef = event_of(i);
                pref = S.pref[ef];
            }
            if (mq < kQ && im < n_ev)
                mc = S.mom[event_of(im) * L::kMom + mk];
        }
    };
    uint64_t cur = claim();
    uint64_t nxt = claim();
    double pref_next, mc_next;
    uint64_t ef_next;
    load(cur, pref_next, mc_next, ef_next);
    int j = 0;
    while (cur < n_quads) {
        const uint64_t qd = cur + j;
        const double pref = pref_next, mc = mc_next;
        const uint64_t ef = ef_next;
        const bool last_in_chunk = j + 1 == kAmpChunk / 2 || qd + 1 >= n_quads;
        load(last_in_chunk ? nxt : qd + 1, pref_next, mc_next, ef_next);
        int h = h0, fl = fl0;
        asm volatile("" : "+v"(h), "+v"(fl));
        const bool live_f = ef < S.count && pref != 0.0;
        if (__any(live_f)) {
            if (mq < kQ)
                s_mom[mq][mk] = mc;
            wave_sync();
            // the fill stages each event's level-1 currents (6 objects,
            // chunk-major over those 6) in the extension of its table
            if (live_f)
                fill_table_coop_ng3<T, 6>(s_mom[fq], s_mom[fq][L::kMom - 1], S.P.m_top, S.P.mw, s_tab[fq],
                                          s_tab[fq] + L::kTable, fl);
            wave_sync();
            for (int pr = 0; pr < 2; ++pr) {
                const int k = 2 * pr + sub;
                const uint64_t e = __shfl(ef, 16 * k);
                const double pe = __shfl(pref, 16 * k);
                const bool live = e < S.count && pe != 0.0;
                const bool any_live = __any(live);
                if (!any_live)
                    continue;
                const T* tab = s_tab[k];
                T* obj = s_obj[sub];
                if (live && h < kL1) {
                    // value h of the staging area: chunk h / (6 CW), place h mod (6 CW);
                    // in the store the chunks of the current region are COOP_NGJ_NG3 apart
                    constexpr int CW = 16 / (int)sizeof(T);
                    obj[(h / (6 * CW)) * CW * COOP_NGJ_NG3 + h % (6 * CW)] = tab[L::kTable + h];
                }
                if constexpr (COL == 2) {
                    if (live)
                        colour_factors_ng3<T>(S.first + e, S.P.seed, S.P.iter, s_cf[sub], h);
                } else if constexpr (COL == 3) {
                    if (live)
                        flow_factors_ng3<T>(S.first + e, S.P.seed, S.P.iter, s_cf[sub], h);
                }
                wave_sync();
                double v = event_me2<3, T, COL>(tab, obj, h, S.P.m_top, live, any_live, s_cf[sub]);
                if (S.P.hel_mc && live)
                    v = hel_sampled<L::kHel>(v, h, S.first + e, S.P.seed, S.P.iter);
                v = group_sum(v, L::kHel);
                if (h == 0 && live)
                    S.me[e] = v;
                wave_sync();
            }
        }
        if (last_in_chunk) {
            cur = nxt;
            nxt = claim();
            j = 0;
        } else {
            ++j;
        }
    }
}

// q qbar -> t tbar for the p p processes (Sec. 3, Table 1): one s-channel
// gluon, |M_h|^2 = 2 |J . K|^2 / s^2 for helicity configuration h, summed over
// colours (the factor 2), g = 1, with K^mu = ubar(k1) gamma^mu v(k2) the top
// current and J^mu = vbar(pb) gamma^mu u(pa) the beam current.  Massless beams
// along +-z in the partonic frame conserve helicity: J vanishes for two of
// the four beam configurations and is sqrt(s) (0, 1, +-i, 0) up to a phase for
// the other two, for either orientation of the beams (so the summed |M|^2 is
// the same for the quark along +z and along -z).  h: bits 0-1 beam
// configuration (bit 1 set: the vanishing ones), bit 2 top and bit 3 antitop
// spin.
__device__ __forceinline__ double qqbar_me2_config(const double* __restrict__ mom, double eb, double mt, int h)
{
    if (h & 2)
        return 0.0;
    cplx<double> ub[4], v[4], K[4];
    spinor_ubar<double>(mom, mt, (h >> 2) & 1, ub);
    spinor_v<double>(mom + 4, mt, (h >> 3) & 1, v);
    bilinear(ub, v, K);
    // J . K = -sqrt(s) (K^1 +- i K^2) up to a phase
    const double sg = (h & 1) ? -1.0 : 1.0;
    const double re = K[1].x - sg * K[2].y, im = K[1].y + sg * K[2].x;
    return 2.0 * (re * re + im * im) / (4.0 * eb * eb);
}

template <int NG, typename T, int COL, bool PP = false>
__device__ __forceinline__ void amp_groups(const StageParams& S)
{
    using L = Layout<NG>;
    // lanes per event: t tbar evaluates two helicity configurations per lane
    // (h and h + 8: the second gluon's polarisation), eight events per pass;
    // the pair sum then the 8-lane tree is the 16-lane tree of one per lane
    constexpr int kLanes = NG == 2 ? L::kHel / 2 : L::kHel;
    constexpr int kPass = kLanes <= kWave ? kWave / kLanes : 1;
    __shared__ __align__(16) TabT<NG, T> s_tab[kPass][L::kTable];
    __shared__ __align__(16) T s_obj[kPass][L::kObj];
    __shared__ double s_mom[kPass][L::kMom];
    // colour factors of the sampled assignment (COL = 2: re and im per
    // ordering) or flow (COL = 3: one real value per ordering)
    constexpr int kCf = COL >= 2 ? 2 * (NG == 3 ? 6 : 24) : 2;
    __shared__ __align__(16) T s_cf[kPass][kCf];
    const int lane = threadIdx.x;
    const int h0 = lane % kLanes;
    const int sub = lane / kLanes;
    TabT<NG, T>* tab = s_tab[sub];
    T* obj = s_obj[sub];
    double* mom = s_mom[sub];
    T* cf = s_cf[sub];
    // the events to evaluate: the live list, or all events in order
    const uint64_t n_ev = S.live ? (uint64_t)*S.n_live : S.count;
    const uint64_t n_groups = (n_ev + kPass - 1) / kPass;
    // one lane claims a chunk with a vector atomic; the wave reads its value
    auto claim = [&]() -> uint64_t {
        unsigned long long c = 0;
        if (lane == 0)
            c = atomicAdd(S.next_group, (unsigned long long)kAmpChunk);
        return (uint64_t)__shfl(c, 0);
    };
    // slot `sub` of group g: its event (S.count if none), prefactor, momenta
    // (values h0 and h0 + kLanes of the kMom stored per event)
    auto load = [&](uint64_t g, double& pref, double& mc, double& mc2, uint64_t& ev) {
        const uint64_t i = g * kPass + sub;
        pref = 0.0;
        mc = 0.0;
        mc2 = 0.0;
        ev = S.count;
        if (g < n_groups && i < n_ev) {
            ev = S.live ? (uint64_t)S.live[i] : i;
            pref = S.pref[ev];
            if (h0 < L::kMom)
                mc = S.mom[ev * L::kMom + h0];
            if (h0 + kLanes < L::kMom)
                mc2 = S.mom[ev * L::kMom + h0 + kLanes];
        }
    };
    uint64_t cur = claim();
    uint64_t nxt = claim();
    double pref_next, mc_next, mc2_next;
    uint64_t ev_next;
    load(cur, pref_next, mc_next, mc2_next, ev_next);
    int j = 0;
    while (cur < n_groups) {
        const uint64_t g = cur + j;
        const double pref = pref_next, mc = mc_next, mc2 = mc2_next;
        const uint64_t e = ev_next;
        // the group after this one: in this chunk, or the first of the next
        const bool last_in_chunk = j + 1 == kAmpChunk || g + 1 >= n_groups;
        load(last_in_chunk ? nxt : g + 1, pref_next, mc_next, mc2_next, ev_next);
        int h = h0;
        asm volatile("" : "+v"(h));
        const bool live = e < S.count && pref != 0.0;
        const bool any_live = __any(live);
        if (any_live) {
            if (h0 < L::kMom)
                mom[h0] = mc;
            if (h0 + kLanes < L::kMom)
                mom[h0 + kLanes] = mc2;
            wave_sync();
            if (live) {
                fill_table<NG, T>(mom, mom[L::kMom - 1], S.P.m_top, S.P.mw, tab, obj, h);
                if constexpr (COL == 2) {
                    if constexpr (NG == 3)
                        colour_factors_ng3<T>(S.first + e, S.P.seed, S.P.iter, cf, h);
                    else
                        colour_factors_ng4<T>(S.first + e, S.P.seed, S.P.iter, cf, h);
                } else if constexpr (COL == 3) {
                    if constexpr (NG == 3)
                        flow_factors_ng3<T>(S.first + e, S.P.seed, S.P.iter, cf, h);
                    else
                        flow_factors_ng4<T>(S.first + e, S.P.seed, S.P.iter, cf, h);
                }
            }
            wave_sync();
            double v = event_me2<NG, T, COL>(tab, obj, h, S.P.m_top, live, any_live, cf);
            if (S.P.hel_mc && live)
                v = hel_sampled<L::kHel>(v, h, S.first + e, S.P.seed, S.P.iter);
            if constexpr (NG == 2) {
                // one configuration after the other: interleaving the two
                // chains only adds register pressure
                __builtin_amdgcn_sched_barrier(0);
                double v2 = event_me2<NG, T, COL>(tab, obj, h + kLanes, S.P.m_top, live, any_live, cf);
                if (S.P.hel_mc && live)
                    v2 = hel_sampled<L::kHel>(v2, h + kLanes, S.first + e, S.P.seed, S.P.iter);
                v += v2;
            }
            v = group_sum(v, kLanes);
            if (h == 0 && live)
                S.me[e] = v;
            if constexpr (PP) {
                // p p: the q qbar channel of the same event, configurations h
                // and h + 8 of the lane (16 of them, like g g)
                double q = live ? qqbar_me2_config(mom, mom[L::kMom - 1], S.P.m_top, h) +
                                      qqbar_me2_config(mom, mom[L::kMom - 1], S.P.m_top, h + kLanes)
                                : 0.0;
                q = group_sum(q, kLanes);
                if (h == 0 && live)
                    S.me_q[e] = q;
            }
            wave_sync();
        }
        if (last_in_chunk) {
            cur = nxt;
            nxt = claim();
            j = 0;
        } else {
            ++j;
        }
    }
}

// The amplitude kernel: quads of events for t tbar g, single events for t tbar g g.
// PP (n_g = 2 only): p p, the q qbar channel evaluated alongside g g.
template <int NG, typename T, int COL = 0, bool PP = false>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 || NG == 3 ? 4 : (NG == 2 ? 3 : 2)))) amp_kernel(StageParams S)
{
    static_assert(!PP || NG == 2, "the q qbar channel runs with n_g = 2");
    if constexpr (NG == 3)
        amp_quads_ng3<T, COL>(S);
    else
        amp_groups<NG, T, COL, PP>(S);
}

// Phase 3 over a batch: weights, compensated sums, w_max, counts and the
// deterministic lane-per-bin histogram, continuing each wave's partials
// across the batches of an iteration.
template <int NF>
__global__ void __launch_bounds__(kBlock) acc_kernel(StageParams S)
{
    constexpr int D = 2 + 3 * NF - 4;
    const EventParams& P = S.P;
    __shared__ double s_w2[kWavesPerBlock][kWave];
    __shared__ unsigned short s_bin[kWavesPerBlock][D][kWave];
    extern __shared__ double s_hist[];     // [kWavesPerBlock][D][n_bins]
    const int tid = threadIdx.x;
    const int wv = tid / kWave;
    const int lane = tid % kWave;
    const int wave_id = blockIdx.x * kWavesPerBlock + wv;
    const int nb = P.n_bins;
    double* hist = s_hist + (size_t)wv * D * nb;
    double* out = P.partials + wave_id;
    const size_t nw = (size_t)P.n_waves;
    Neumaier sw{0.0, 0.0}, sw2{0.0, 0.0};
    double wmax = 0.0, npass = 0.0, nfail = 0.0;
    if (S.first_batch) {
        for (int i = lane; i < D * nb; i += kWave)
            hist[i] = 0.0;
    } else {
        for (int i = lane; i < D * nb; i += kWave)
            hist[i] = out[(kPartialHead + i) * nw];
        if (lane == 0) {
            sw = Neumaier{out[0 * nw], out[1 * nw]};
            sw2 = Neumaier{out[2 * nw], out[3 * nw]};
            wmax = out[4 * nw];
            npass = out[5 * nw];
            nfail = out[6 * nw];
        }
    }
    wave_sync();
    const uint64_t n_chunks = (S.count + kWave - 1) / kWave;
    for (uint64_t chunk = wave_id; chunk < n_chunks; chunk += P.n_waves) {
        const uint64_t e = chunk * kWave + lane;
        const bool active = e < S.count;
        double w = 0.0;
        if (active) {
            const double pref = S.pref[e];
            const int flags = S.flags[e];
            if (pref != 0.0) {
                w = pref * (S.me[e] * P.me_norm);
                if (P.pp) {
                    w += S.pref_q[e] * (S.me_q[e] * P.me_norm_q);
                    if constexpr (NF >= 3)
                        w += S.pref_q[S.count + e] * (S.me_q[S.count + e] * P.me_norm_q);
                }
            }
            if (P.weights)
                P.weights[S.first + e] = w;
            nm_add(sw, w);
            nm_add(sw2, w * w);
            wmax = fmax(wmax, w);
            npass += (flags & 4) ? 1.0 : 0.0;
            nfail += (flags & 2) ? 1.0 : 0.0;
        }
        s_w2[wv][lane] = active ? w * w : 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d)
            s_bin[wv][d][lane] = active ? S.bins[(size_t)d * S.count + e] : (unsigned short)0;
        wave_sync();
        for (int b = lane; b < nb; b += kWave) {
            for (int d = 0; d < D; ++d) {
                double acc = hist[d * nb + b];
                for (int q = 0; q < kWave; ++q)
                    if (s_bin[wv][d][q] == b)
                        acc += s_w2[wv][q];
                hist[d * nb + b] = acc;
            }
        }
        wave_sync();
    }
    for (int off = kWave >> 1; off > 0; off >>= 1) {
        Neumaier o1{__shfl_down(sw.s, off), __shfl_down(sw.c, off)};
        Neumaier o2{__shfl_down(sw2.s, off), __shfl_down(sw2.c, off)};
        const double om = __shfl_down(wmax, off);
        const double op = __shfl_down(npass, off);
        const double of = __shfl_down(nfail, off);
        sw = nm_merge(sw, o1);
        sw2 = nm_merge(sw2, o2);
        wmax = fmax(wmax, om);
        npass += op;
        nfail += of;
    }
    if (lane == 0) {
        out[0 * nw] = sw.s;
        out[1 * nw] = sw.c;
        out[2 * nw] = sw2.s;
        out[3 * nw] = sw2.c;
        out[4 * nw] = wmax;
        out[5 * nw] = npass;
        out[6 * nw] = nfail;
        out[7 * nw] = 0.0;
    }
    for (int i = lane; i < D * nb; i += kWave)
        out[(kPartialHead + i) * nw] = hist[i];
}

// ---------------------------------------------------------------------------
// g g -> t tbar g g g (Sec. 3.2, Fig. 4: the paper's largest process).  The
// object store of one event (15560 values: 124 KB in FP64, 62 KB in FP32)
// takes most of a compute unit's LDS, so one workgroup of eight waves (two
// per SIMD) serves one event at a time -- in FP32 two workgroups share a
// compute unit.  All 512 lanes build the objects, then the waves take the
// event's 20 amplitude items -- (first gluon c, pass, half of the 128
// helicity configurations), 12 orderings for 64 configurations each -- and
// store the partial amplitudes to the event's block in device memory.  Work
// is handed out per wave from LDS counters, so that waves that run faster
// (a SIMD shared with fewer waves) take more of it and the workgroup meets
// at its barriers together.  The colour sum over 120 x 120 orderings
// is a dense contraction and runs on the matrix cores in colour_kernel_ng5.
// Events are claimed one at a time from a device counter (cleared by
// kin_kernel); rejected events (prefactor 0) are skipped.
// ---------------------------------------------------------------------------
constexpr int kBlockNg5 = 512;
constexpr int kAmpRowNg5 = 2 * 128;                        // T per row: 128 helicities x (re, im)
constexpr size_t kAmpEventNg5 = (size_t)NPERM_NG5 * kAmpRowNg5;  // T per event

// LC: the leading-colour sum instead (the colour matrix replaced by
// kColourLcNg5 times the identity): each amplitude item adds its squared
// moduli over the wave and stores that one value, slot `item` of the event's
// AMP_ITEMS_NG5 doubles at the start of S.amps; lc_kernel_ng5 adds them in
// item order, so the result does not depend on which wave took which item.
template <typename T, bool LC = false>
__global__ void __launch_bounds__(kBlockNg5) amp_kernel_ng5(StageParams S)
{
    using L = Layout<5>;
    __shared__ __align__(16) T s_tab[COOP_TABLE_NG5];
    __shared__ __align__(16) T s_obj[COOP_OBJ_NG5];
    __shared__ double s_mom[L::kMom];
    __shared__ unsigned long long s_ev;
    __shared__ unsigned s_ctr[9];          // work counters: eight for the stages, one for the amplitude items
    __shared__ unsigned long long s_stab[STAGE_TAB_SIZE_NG5];   // split tables of the current levels
    __shared__ short s_ninv[STAGE_NINV_SIZE_NG5];
    const int tid = threadIdx.x;
    T* J = static_cast<T*>(S.amps);
    for (int i = tid; i < STAGE_TAB_SIZE_NG5; i += kBlockNg5)
        s_stab[i] = STAGE_TAB_NG5[i];
    for (int i = tid; i < STAGE_NINV_SIZE_NG5; i += kBlockNg5)
        s_ninv[i] = STAGE_NINV_NG5[i];
    if (tid == 0)
        s_ev = atomicAdd(S.next_group, 1ull);
    __syncthreads();
    uint64_t e = s_ev;
    __syncthreads();
    while (e < S.count) {
        // the next event is claimed now; its index is read after this one
        if (tid == 0)
            s_ev = atomicAdd(S.next_group, 1ull);
        if (S.pref[e] != 0.0) {
            if (tid < L::kMom)
                s_mom[tid] = S.mom[e * L::kMom + tid];
            if (tid < 9)
                s_ctr[tid] = 0u;
            __syncthreads();
            if (tid < kWave)
                fill_table_coop_ng5<T>(s_mom, s_mom[L::kMom - 1], S.P.m_top, S.P.mw, s_tab, s_obj, tid);
            __syncthreads();
            coop_stages_ng5<T>(s_tab, s_obj, S.P.m_top, tid, s_ctr, s_stab, s_ninv);
            // amplitude items (chunk, pass, helicity half), one wave each, taken
            // from a counter so that waves on less crowded SIMDs take more
            for (;;) {
                unsigned item = 0;
                if ((tid & 63) == 0)
                    item = atomicAdd(&s_ctr[8], 1u);
                item = __builtin_amdgcn_readfirstlane(__shfl(item, 0));
                if (item >= (unsigned)AMP_ITEMS_NG5)
                    break;
                const int c = (int)(item % 5u), rest = (int)(item / 5u);
                double lc = 0.0;
                coop_amp_ng5<T, LC>(s_tab, s_obj, 64 * (rest & 1) + (tid & 63), c, rest >> 1,
                                    J + e * kAmpEventNg5, lc);
                if constexpr (LC) {
                    // every lane stores the wave's sum (one address, one
                    // value): a store by lane 0 alone, branching on the same
                    // condition as the claim above, lets the compiler fold
                    // the two into a loop that lanes leave one by one, whose
                    // other lanes then read an item from an inactive lane 0
                    lc = __shfl(group_sum(lc, kWave), 0);
                    static_cast<double*>(S.amps)[e * AMP_ITEMS_NG5 + item] = lc;
                }
            }
        }
        __syncthreads();
        e = s_ev;
        // every lane has read the index before lane 0 claims the next one
        __syncthreads();
    }
}

typedef double mf_d4v __attribute__((ext_vector_type(4)));
typedef float mf_f4v __attribute__((ext_vector_type(4)));
template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
    using type = mf_d4v;
};
template <>
struct MfmaAcc<float> {
    using type = mf_f4v;
};

// D += A B for one 16 x 16 x 4 matrix-core step (wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; in component r it holds
// D[l / 16 + 4 r][l % 16] (FP64 step) or D[4 (l / 16) + r][l % 16] (FP32 step).
__device__ __forceinline__ mf_d4v mfma_16x16x4(double a, double b, mf_d4v d)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
}
__device__ __forceinline__ mf_f4v mfma_16x16x4(float a, float b, mf_f4v d)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0);
}

// Colour sum of t tbar g g g on the matrix cores.  Per event the stored
// amplitudes form X[120 rows][256 columns] (column = 2 h + re/im), and
// sum_h A_h^dagger C A_h = sum over columns of x^T K' x / den with K' the
// integer colour matrix in the stored row order and signs.  Rows are cut in
// tiles of 16 (the last padded with zeros); with K' symmetric only the block
// lower triangle is needed, the blocks below the diagonal doubled (36 tile
// pairs, CFRAG_NG5).  For column block cb (16 columns) a wave forms
// D_a = sum_(b <= a) K'_ab X_b with four 16 x 16 x 4 steps per tile pair and
// contracts D_a with X_a.  Step s of tile b contracts, in lane group
// k = l / 16, the tile row that the lane holds in component s of D (row
// k + 4 s for the FP64 step, 4 k + s for the FP32 step), so one set of 32
// loaded values per lane serves both the products and the final
// contraction.  The fragments of K' sit in LDS; one wave per event.
template <typename T>
__global__ void __launch_bounds__(kBlock) colour_kernel_ng5(StageParams S)
{
    constexpr int kFrag = 36 * 4 * kWave;
    __shared__ T s_frag[kFrag];
    const int tid = threadIdx.x;
    for (int i = tid; i < kFrag; i += kBlock)
        s_frag[i] = (T)(sizeof(T) == 8 ? CFRAG64_NG5[i] : CFRAG32_NG5[i]);
    __syncthreads();
    const int lane = tid % kWave, q = lane >> 4, col0 = lane & 15;
    const T* J = static_cast<const T*>(S.amps);
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock;
    for (uint64_t e = (uint64_t)blockIdx.x * kWavesPerBlock + tid / kWave; e < S.count; e += stride) {
        if (S.pref[e] == 0.0)
            continue;
        const T* X = J + e * kAmpEventNg5;
        double acc = 0.0;
        // the lane's 32 values of column block cb (rows of the tiles it holds)
        auto load = [&](int cb, T (&v)[8][4]) {
            const int col = 16 * cb + col0;
#pragma unroll
            for (int b = 0; b < 8; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * b + (sizeof(T) == 8 ? q + 4 * r : 4 * q + r);
                    v[b][r] = row < NPERM_NG5 ? X[(size_t)row * kAmpRowNg5 + col] : (T)0;
                }
        };
        T x[8][4], xn[8][4];
        load(0, x);
        for (int cb = 0; cb < kAmpRowNg5 / 16; ++cb) {
            // the next column block is read while this one is contracted
            if (cb + 1 < kAmpRowNg5 / 16)
                load(cb + 1, xn);
            // tile pairs in order (a, b <= a); the four fragments of the next
            // pair are read from LDS while the current pair's steps run
            constexpr int PA[36] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 4, 5, 5, 5,
                                    5, 5, 5, 6, 6, 6, 6, 6, 6, 6, 7, 7, 7, 7, 7, 7, 7, 7};
            constexpr int PB[36] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4, 0, 1, 2,
                                    3, 4, 5, 0, 1, 2, 3, 4, 5, 6, 0, 1, 2, 3, 4, 5, 6, 7};
            const T* fr = s_frag + lane;
            T f[4] = {fr[0], fr[kWave], fr[2 * kWave], fr[3 * kWave]};
            typename MfmaAcc<T>::type d = {0, 0, 0, 0};
#pragma unroll
            for (int p = 0; p < 36; ++p) {
                const int a = PA[p], b = PB[p];
                T g[4] = {0, 0, 0, 0};
                if (p + 1 < 36) {
                    const T* fn = fr + (p + 1) * 4 * kWave;
                    g[0] = fn[0];
                    g[1] = fn[kWave];
                    g[2] = fn[2 * kWave];
                    g[3] = fn[3 * kWave];
                }
                if (b == 0)
                    d = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    d = mfma_16x16x4(f[s], x[b][s], d);
                if (b == a)
                    acc += (double)x[a][0] * (double)d[0] + (double)x[a][1] * (double)d[1] +
                           (double)x[a][2] * (double)d[2] + (double)x[a][3] * (double)d[3];
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    f[s] = g[s];
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int b = 0; b < 8; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    x[b][r] = xn[b][r];
        }
        for (int off = kWave >> 1; off > 0; off >>= 1)
            acc += __shfl_xor(acc, off);
        if (lane == 0)
            S.me[e] = acc / COLOUR_DEN_NG5;
    }
}

// Leading colour of t tbar g g g: c_LC = (N^2 - 1) N^4 / 2^5 with N = 3,
// the leading power of N of the colour matrix's diagonal N C_F^5.
constexpr double kColourLcNg5 = 8.0 * 81.0 / 32.0;

// The leading-colour |M|^2 of the batch's events from the amplitude kernel's
// per-item sums (added in item order), one thread per event.
__global__ void __launch_bounds__(kBlock) lc_kernel_ng5(StageParams S)
{
    const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= S.count || S.pref[e] == 0.0)
        return;
    const double* q = static_cast<const double*>(S.amps) + e * AMP_ITEMS_NG5;
    double s = 0.0;
    for (int i = 0; i < AMP_ITEMS_NG5; ++i)
        s += q[i];
    S.me[e] = kColourLcNg5 * s;
}

// mf_matrix_element for t tbar g g g: the caller's momenta [n][20] and beam
// energies into the amplitude kernel's per-event layout [n][21], prefactor 1
// (every event evaluated); thread 0 clears the amplitude kernel's counter.
__global__ void __launch_bounds__(kBlock) me_prep_kernel_ng5(const double* __restrict__ mom,
                                                             const double* __restrict__ eb, uint64_t n,
                                                             StageParams S)
{
    const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e == 0)
        *S.next_group = 0ull;
    if (e >= n)
        return;
    constexpr int K = Layout<5>::kMom;
    for (int i = 0; i < K - 1; ++i)
        S.mom[e * K + i] = mom[e * (K - 1) + i];
    S.mom[e * K + K - 1] = eb[e];
    S.pref[e] = 1.0;
}

// mf_matrix_element for the q qbar channel of p p -> t tbar: quark along +z.
__global__ void __launch_bounds__(kBlock) qqbar_me_kernel(const double* __restrict__ mom, const double* __restrict__ eb,
                                                          uint64_t n, double mt, double* __restrict__ out)
{
    const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n)
        return;
    double sum = 0.0;
    for (int h = 0; h < 16; ++h)
        sum += qqbar_me2_config(mom + 8 * e, eb[e], mt, h);
    out[e] = sum;
}

// p p -> t tbar g: the q qbar amplitudes of the batch's passing events,
// with helicity recycling.  Eight events per one-wave workgroup, eight lanes
// per event.  Lane c first builds the beam chains X1, X2 of beam combination
// c and the top chains Y3, Y4 of top combination c (and, for even c, the
// currents J and K they belong with) into LDS; then it evaluates the four
// configurations with top combination c (both orientations, both quark
// spins).  The sums go to me_q[e] (quark along +z) and me_q[count + e].
constexpr int kQqEvents = kWave / 8;
__global__ void __launch_bounds__(kWave) qqbar_ttxg_kernel(StageParams S)
{
    // per event: X1[8], X2[8], Y3[8], Y4[8], J[4], K[4] (complex 4-vectors)
    __shared__ __align__(16) cplx<double> s_ch[kQqEvents][40][4];
    const int lane = threadIdx.x;
    const int ev = lane >> 3, c = lane & 7;
    const uint64_t i = (uint64_t)blockIdx.x * kQqEvents + ev;
    const uint64_t n_ev = S.live ? (uint64_t)*S.n_live : S.count;
    const uint64_t e = i < n_ev ? (S.live ? (uint64_t)S.live[i] : i) : S.count;
    const bool live = e < S.count && S.pref[e] != 0.0;
    double mom[13];
    if (live)
        for (int i = 0; i < 13; ++i)
            mom[i] = S.mom[e * 13 + i];
    cplx<double>(*ch)[4] = s_ch[ev];
    if (live) {
        const bool cur = (c & 1) == 0;
        qq_beam_chains(mom, mom[12], c, cur, ch[c], ch[8 + c], ch[32 + (c >> 1)]);
        qq_top_chains(mom, mom[12], S.P.m_top, S.P.mw, c, cur, ch[16 + c], ch[24 + c], ch[36 + (c >> 1)]);
    }
    __syncthreads();
    double acc[2] = {0.0, 0.0};
    if (live) {
        const double eb = mom[12];
        double ep[4], Q[4], kq[4], kp[4];
        qq_linear_pol(mom + 8, c & 1, ep);
        for (int mu = 0; mu < 4; ++mu) {
            Q[mu] = mom[mu] + mom[4 + mu];
            kq[mu] = mom[8 + mu] - Q[mu];
            kp[mu] = mom[8 + mu];
        }
        kp[0] += 2.0 * eb;                        // k3 + P, P = (2 eb, 0, 0, 0)
        const double pe = (2.0 * eb + Q[0]) * ep[0] - Q[1] * ep[1] - Q[2] * ep[2] - Q[3] * ep[3];
        const double inv = 1.0 / (4.0 * eb * eb * qq_m2(Q));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = (j << 1) | (c & 1);     // orientation j >> 1, quark spin j & 1
            acc[j >> 1] += qq_config_from_chains(ch[b], ch[8 + b], ch[32 + (b >> 1)], ch[16 + c], ch[24 + c],
                                                 ch[36 + (c >> 1)], ep, pe, kq, kp, inv);
        }
    }
    const double f = group_sum(acc[0], 8);
    const double r = group_sum(acc[1], 8);
    if (live && c == 0) {
        S.me_q[e] = f;
        S.me_q[S.count + e] = r;
    }
}

// q qbar -> t tbar g |M|^2 (g = 1) for explicit momenta [n][12] (t, tbar, g),
// the quark along +z; 16 lanes per event.
__global__ void __launch_bounds__(kBlock) qqbar_ttxg_me_kernel(const double* __restrict__ mom,
                                                               const double* __restrict__ eb, uint64_t n,
                                                               double mt, double mw, double* __restrict__ out)
{
    const uint64_t e = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 4;
    const int c = threadIdx.x & 15;
    double v = 0.0;
    if (e < n)
        v = qqbar_ttxg_config(mom + 12 * e, eb[e], mt, mw, c, 0);
    v = group_sum(v, 16);
    if (e < n && c == 0)
        out[e] = v;
}

// The q qbar -> t tbar g g |M|^2 (g = 1) of one event by one wave: the 344
// helicity-recycled objects (currents and line chains, mf_qqbar_ttxgg.hpp)
// built into LDS in two passes of all 64 lanes, then lane = orientation x 32
// + configuration (the 32 with the antiquark spin opposite the quark's)
// contracting them.  Returns the sum over the lane's 32-lane half (quark
// along +z for lanes 0-31, along -z for 32-63).  mom: LDS [t, tbar, g1, g2,
// sqrt(s)/2].
__device__ __forceinline__ double qqbar_ttxgg_event(const double* mom, double mt, double mw, int lane)
{
    __shared__ __align__(16) cplx<double> s_ob[kQ4Objects][4];
    __shared__ __align__(16) cplx<double> s_j12[4][4];
    __shared__ double s_eps[4][4];
    const Q4Kin kin = q4_kinematics(mom, mom[16], mt, mw);
    q4_objects_pass1(kin, lane, s_ob, s_eps, s_j12);
    __syncthreads();
    q4_objects_pass2(kin, lane, s_ob);           // synchronises between its reads and writes
    __syncthreads();
    const double v = q4_config_from_objects(kin, s_ob, s_eps, s_j12, lane & 31, lane >> 5);
    return group_sum(v, 32);
}

// p p -> t tbar g g: the q qbar amplitudes of the batch's live events, one
// one-wave workgroup per event; the sums go to me_q[e] (quark along +z) and
// me_q[count + e].
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) qqbar_ttxgg_kernel(StageParams S)
{
    __shared__ double s_mom[17];
    const int lane = threadIdx.x;
    const uint64_t i = blockIdx.x;
    const uint64_t n_ev = S.live ? (uint64_t)*S.n_live : S.count;
    const uint64_t e = i < n_ev ? (S.live ? (uint64_t)S.live[i] : i) : S.count;
    if (e >= S.count || S.pref[e] == 0.0)
        return;                                  // uniform over the workgroup
    if (lane < 17)
        s_mom[lane] = S.mom[e * 17 + lane];
    __syncthreads();
    const double v = qqbar_ttxgg_event(s_mom, S.P.m_top, S.P.mw, lane);
    if ((lane & 31) == 0)
        S.me_q[(uint64_t)(lane >> 5) * S.count + e] = v;
}

// q qbar -> t tbar g g |M|^2 (g = 1) for explicit momenta [n][16] (t, tbar,
// g1, g2), the quark along +z: the integrand's evaluation, one one-wave
// workgroup per event.
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) qqbar_ttxgg_me_kernel(
    const double* __restrict__ mom, const double* __restrict__ eb, uint64_t n, double mt, double mw,
    double* __restrict__ out)
{
    __shared__ double s_mom[17];
    const int lane = threadIdx.x;
    const uint64_t e = blockIdx.x;
    if (e >= n)
        return;                                  // uniform over the workgroup
    if (lane < 16)
        s_mom[lane] = mom[16 * e + lane];
    else if (lane == 16)
        s_mom[16] = eb[e];
    __syncthreads();
    const double v = qqbar_ttxgg_event(s_mom, mt, mw, lane);
    if (lane == 0)
        out[e] = v;
}

// mf_evaluate for the staged processes: weight (and the record's |M|^2 entry)
// of every event of the batch.
__global__ void __launch_bounds__(kBlock) weight_kernel(StageParams S, int nf)
{
    const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= S.count)
        return;
    const double pref = S.pref[e];
    const double me = pref != 0.0 ? S.me[e] : 0.0;
    double w = pref != 0.0 ? pref * (me * S.P.me_norm) : 0.0;
    if (S.P.pp && pref != 0.0) {
        w += S.pref_q[e] * (S.me_q[e] * S.P.me_norm_q);
        if (nf >= 3)
            w += S.pref_q[S.count + e] * (S.me_q[S.count + e] * S.P.me_norm_q);
    }
    S.P.weights[S.first + e] = w;
    if (S.P.record)
        S.P.record[(S.first + e) * (8 + 4 * (uint64_t)nf) + 6] = me;
}

// ---------------------------------------------------------------------------
// Reduce the per-wave partials: one workgroup per entry (entry-major layout,
// coalesced), each thread a fixed strided subset of waves with compensated
// sums, then a fixed-shape tree in LDS -- the result does not depend on
// scheduling.  Then one workgroup estimates I_j, V_j and refines the grid.
// ---------------------------------------------------------------------------
struct ReduceParams {
    const double* partials;  // [stride][n_waves]
    int n_waves, stride, n_dims, n_bins;
    double n_events, alpha;
    const double* grid_in;
    double* grid_out;
    double* entries;         // [stride] reduced entries
    const double* hist;      // [D][n_bins] reduced histogram (read by refine)
    double* iter_I;          // [n_iter]
    double* iter_V;
    double* iter_pass;       // [n_iter] events passing threshold and cuts, or null
    double* stats;           // [4]: w_max (this iteration), n_pass, n_fail (cumulative)
    int j;
};

constexpr int kReduceBlock = 256;

__global__ void __launch_bounds__(kReduceBlock) reduce_entries_kernel(ReduceParams R)
{
    __shared__ double s_s[kReduceBlock], s_c[kReduceBlock];
    const int k = blockIdx.x;            // entry
    const int tid = threadIdx.x;
    const double* row = R.partials + (size_t)k * R.n_waves;
    Neumaier a{0.0, 0.0};
    double mx = 0.0;
    if (k == 0 || k == 2) {
        // compensated pairs (s, c) of sum w and sum w^2
        const double* crow = row + R.n_waves;
        for (int w = tid; w < R.n_waves; w += kReduceBlock)
            a = nm_merge(a, Neumaier{row[w], crow[w]});
    } else if (k == 4) {
        for (int w = tid; w < R.n_waves; w += kReduceBlock)
            mx = fmax(mx, row[w]);
        a.s = mx;
    } else {
        for (int w = tid; w < R.n_waves; w += kReduceBlock)
            nm_add(a, row[w]);
    }
    s_s[tid] = a.s;
    s_c[tid] = a.c;
    __syncthreads();
    for (int off = kReduceBlock / 2; off > 0; off >>= 1) {
        if (tid < off) {
            if (k == 4) {
                s_s[tid] = fmax(s_s[tid], s_s[tid + off]);
            } else {
                const Neumaier m = nm_merge(Neumaier{s_s[tid], s_c[tid]}, Neumaier{s_s[tid + off], s_c[tid + off]});
                s_s[tid] = m.s;
                s_c[tid] = m.c;
            }
        }
        __syncthreads();
    }
    if (tid == 0)
        R.entries[k] = (k == 4) ? s_s[0] : s_s[0] + s_c[0];
}

__global__ void __launch_bounds__(256) refine_kernel(ReduceParams R)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        const double N = R.n_events;
        const double I = R.entries[0] / N;
        const double V = (R.entries[2] / N - I * I) / (N - 1.0);
        R.iter_I[R.j] = I;
        R.iter_V[R.j] = V;
        if (R.iter_pass)
            R.iter_pass[R.j] = R.entries[5];
        R.stats[0] = R.entries[4];
        R.stats[1] = R.entries[5];
        R.stats[2] += R.entries[6];
    }
    // One thread per dimension: smoothing, damping, equal-share rebinning.
    for (int d = tid; d < R.n_dims; d += blockDim.x) {
        const int n = R.n_bins;
        const double* h = R.hist + d * n;
        const double* e = R.grid_in + d * (n + 1);
        double* en = R.grid_out + d * (n + 1);
        auto smoothed = [&](int i) -> double {
            if (i == 0)
                return (h[0] + h[1]) / 2.0;
            if (i == n - 1)
                return (h[n - 2] + h[n - 1]) / 2.0;
            return (h[i - 1] + h[i] + h[i + 1]) / 3.0;
        };
        double total = 0.0;
        for (int i = 0; i < n; ++i)
            total += smoothed(i);
        if (total == 0.0) {
            for (int i = 0; i <= n; ++i)
                en[i] = e[i];
            continue;
        }
        auto importance = [&](int i) -> double {
            const double rho = smoothed(i) / total;
            if (rho <= 0.0)
                return 0.0;
            if (rho >= 1.0)
                return 1.0;
            return pow((1.0 - rho) / (-log(rho)), R.alpha);
        };
        double rsum = 0.0;
        for (int i = 0; i < n; ++i)
            rsum += importance(i);
        const double share = rsum / (double)n;
        // grid_out never aliases grid_in, so the old edges stay readable.
        en[0] = 0.0;
        int i = 0;
        double cum = 0.0;
        double ri = importance(0);
        for (int kk = 1; kk < n; ++kk) {
            const double target = (double)kk * share;
            while (i < n - 1 && (cum + ri < target || ri == 0.0)) {
                cum += ri;
                ++i;
                ri = importance(i);
            }
            double frac = ri > 0.0 ? (target - cum) / ri : 1.0;
            if (frac > 1.0)
                frac = 1.0;
            en[kk] = e[i] + frac * (e[i + 1] - e[i]);
        }
        en[n] = 1.0;
    }
}

// Stand-alone |M|^2: one helicity per lane, events of the launch in groups.
template <int NG, typename T>
__global__ void __launch_bounds__(kBlock) me_kernel(const double* __restrict__ mom, const double* __restrict__ eb,
                                                     uint64_t n, double mt, double mw, double* __restrict__ out)
{
    using L = Layout<NG>;
    __shared__ __align__(16) TabT<NG, T> s_tab[kWavesPerBlock][L::kEventsPerPass][L::kTable];
    __shared__ __align__(16) T s_obj[kWavesPerBlock][L::kEventsPerPass][L::kObj];
    const int lane = threadIdx.x % kWave;
    const int wv = threadIdx.x / kWave;
    const uint64_t wave = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    const uint64_t e = wave * L::kEventsPerPass + lane / L::kHel;
    const int h = lane % L::kHel;
    TabT<NG, T>* tab = s_tab[wv][lane / L::kHel];
    T* obj = s_obj[wv][lane / L::kHel];
    const bool live = e < n;
    if (live)
        fill_table<NG, T>(mom + e * (L::kMom - 1), eb[e], mt, mw, tab, obj, h);
    wave_sync();
    double v = event_me2<NG, T>(tab, obj, h, mt, live, __any(live));
    v = group_sum(v, L::kHel);
    if (h == 0 && e < n)
        out[e] = v;
}

}  // namespace mf
