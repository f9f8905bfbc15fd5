/*
 * rng_vegas.c -- oracle: random numbers, VEGAS map and grid refinement.
 * Test infrastructure only (see mfo.h).
 *
 * The paper's integrator (VegasFlow, Sec. 1 ingredient (i) and Sec. 2.2)
 * starts each event from uniform random numbers and maps them through an
 * adaptive VEGAS grid; after each iteration the grid is refined from the
 * accumulated histogram.  The random numbers come from the counter-based
 * Philox4x32-10 generator (Salmon, Moraes, Dror, Shaw, SC'11) so that any
 * event of any iteration can be regenerated independently.
 */
#include <math.h>
#include <string.h>
#include "mfo.h"

/* One Philox4x32-10 block: ten rounds of the S-box
 *   (c0,c1,c2,c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
 * with M0 = 0xD2511F53, M1 = 0xCD9E8D57 and the key bumped by the Weyl
 * constants (0x9E3779B9, 0xBB67AE85) between rounds (SC'11, Sec. 3). */
void mfo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream layout: key = (seed mod 2^32, seed >> 32); block b of event e in
 * iteration it has counter (e mod 2^32, e >> 32, it, b).  Each block gives
 * two 53-bit integers, k = ((r_hi << 32) | r_lo) >> 11, from the word pairs
 * (r0, r1) and (r2, r3).  Dimension 2b takes the first, 2b+1 the second. */
void mfo_event_k53(uint64_t seed, uint32_t iter, uint64_t event, int n_dim, uint64_t *k53)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (int b = 0; 2 * b < n_dim; ++b) {
        uint32_t ctr[4] = { (uint32_t)event, (uint32_t)(event >> 32), iter, (uint32_t)b };
        uint32_t r[4];
        mfo_philox4x32_10(ctr, key, r);
        uint64_t ka = ((((uint64_t)r[0]) << 32) | (uint64_t)r[1]) >> 11;
        uint64_t kb = ((((uint64_t)r[2]) << 32) | (uint64_t)r[3]) >> 11;
        k53[2 * b] = ka;
        if (2 * b + 1 < n_dim)
            k53[2 * b + 1] = kb;
    }
}

/* y = k 2^-53.  The VEGAS bin of y is floor(y N_b) and the position inside
 * the bin delta = y N_b - bin; both are taken from the exact integer product
 * k N_b so that the bin index involves no floating-point rounding. */
void mfo_bin_from_k53(uint64_t k53, int n_bins, int *bin, double *delta)
{
    uint64_t prod = k53 * (uint64_t)n_bins;          /* < 2^63 for n_bins <= 1024 */
    *bin = (int)(prod >> 53);
    *delta = (double)(prod & ((UINT64_C(1) << 53) - 1)) * 0x1p-53;
}

/* VEGAS map (Lepage 1978): inside bin i of dimension d the variable is
 * linear, x = e_i + delta (e_{i+1} - e_i), with Jacobian N_b (e_{i+1} - e_i).
 * The total Jacobian is the product over dimensions, taken in order. */
double mfo_vegas_map(int n_dim, int n_bins, const double *grid,
                     const int *bin, const double *delta, double *x)
{
    double jac = 1.0;
    for (int d = 0; d < n_dim; ++d) {
        const double *e = grid + (size_t)d * (n_bins + 1);
        int i = bin[d];
        double width = e[i + 1] - e[i];
        double shift = delta[d] * width;
        x[d] = e[i] + shift;
        double jd = (double)n_bins * width;
        jac = jac * jd;
    }
    return jac;
}

/* Grid refinement (Lepage 1978, with the usual smoothing and damping):
 * d_i = sum of w^2 over the events in bin i; smooth with the neighbours;
 * rho_i = normalised smoothed d_i; importance r_i = ((1 - rho)/(-ln rho))^alpha;
 * then place the new edges so that every new bin holds the same share of
 * sum r, interpolating linearly inside the old bins. */
void mfo_vegas_refine(int n_dim, int n_bins, double alpha, const double *hist,
                      const double *grid_in, double *grid_out)
{
    double ds[1024], r[1024];
    for (int d = 0; d < n_dim; ++d) {
        const double *h = hist + (size_t)d * n_bins;
        const double *e = grid_in + (size_t)d * (n_bins + 1);
        double *en = grid_out + (size_t)d * (n_bins + 1);

        ds[0] = (h[0] + h[1]) / 2.0;
        ds[n_bins - 1] = (h[n_bins - 2] + h[n_bins - 1]) / 2.0;
        for (int i = 1; i < n_bins - 1; ++i)
            ds[i] = (h[i - 1] + h[i] + h[i + 1]) / 3.0;

        double total = 0.0;
        for (int i = 0; i < n_bins; ++i)
            total += ds[i];
        if (total == 0.0) {
            memmove(en, e, sizeof(double) * (size_t)(n_bins + 1));
            continue;
        }

        double rsum = 0.0;
        for (int i = 0; i < n_bins; ++i) {
            double rho = ds[i] / total;
            if (rho <= 0.0)
                r[i] = 0.0;
            else if (rho >= 1.0)
                r[i] = 1.0;
            else
                r[i] = pow((1.0 - rho) / (-log(rho)), alpha);
            rsum += r[i];
        }
        double share = rsum / (double)n_bins;

        double old[1025];
        memcpy(old, e, sizeof(double) * (size_t)(n_bins + 1));
        en[0] = 0.0;
        en[n_bins] = 1.0;
        int i = 0;
        double cum = 0.0;            /* sum of r_l for l < i */
        for (int k = 1; k < n_bins; ++k) {
            double target = (double)k * share;
            while (i < n_bins - 1 && (cum + r[i] < target || r[i] == 0.0)) {
                cum += r[i];
                ++i;
            }
            /* Rounding in the running sum can leave the last bin a hair
             * short of the target: the fraction is capped at 1 (and a
             * zero-importance last bin maps to its upper edge). */
            double frac = (r[i] > 0.0) ? (target - cum) / r[i] : 1.0;
            if (frac > 1.0)
                frac = 1.0;
            en[k] = old[i] + frac * (old[i + 1] - old[i]);
        }
    }
}
