// mf_unweight.hpp -- hit-or-miss unweighting of weighted events on the GPU
// (Sec. 2.5: the weighted events of the integration are turned into
// unit-weight events for the LHE output).
//
// Event e of weight w_e is kept when u_e w_max < |w_e|, u_e being the first
// 53-bit uniform of the Philox block 0x80000000 of the event's counter
// (e mod 2^32, e >> 32, iter, 0x80000000); the integrand draws only from
// blocks 0 .. ceil(D/2) - 1.  A kept event carries the sign of w_e.
//
// Two passes over contiguous event ranges, one range per workgroup: a count
// pass (kept and above-w_max events per workgroup), a host-side exclusive
// scan, and a write pass that ranks the kept events of each 256-event chunk
// with wave ballots, so that records come out in increasing event index.
// For each kept event the write pass regenerates the phase-space point from
// its counter (the same draw and map as the integration) and stores the
// lab-frame momenta.
#pragma once

#include "mf_kernels.hpp"

namespace mf {

struct UnweightParams {
    EventParams P;           // grid, seed, iter, sqrt_s, m_top, max_newton, ps_const, n_bins
    const double* w;         // [n] weights of the iteration
    uint64_t n;
    double w_max;
    uint64_t per_block;      // events per workgroup, a multiple of kBlock
    uint64_t* counts;        // [n_blocks][2]: kept, above w_max (count pass)
    const uint64_t* offsets; // [n_blocks] first record of each workgroup (write pass)
    uint64_t capacity;
    uint64_t* ev_out;        // [capacity]
    double* p_out;           // [capacity][NF + 2][4] or null
    signed char* sign_out;   // [capacity] or null
};

__device__ __forceinline__ bool keep_event(const UnweightParams& U, uint64_t e, bool& over, signed char& sign)
{
#pragma clang fp contract(off)
    const double w = U.w[e];
    const double a = fabs(w);
    const uint32_t key0 = (uint32_t)U.P.seed, key1 = (uint32_t)(U.P.seed >> 32);
    uint32_t r[4];
    philox4x32_10((uint32_t)e, (uint32_t)(e >> 32), U.P.iter, 0x80000000u, key0, key1, r);
    const uint64_t k = ((((uint64_t)r[0]) << 32) | (uint64_t)r[1]) >> 11;
    const double u = (double)k * 0x1p-53;
    over = a > U.w_max;
    sign = w > 0.0 ? 1 : -1;
    return u * U.w_max < a;
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* s_red)
{
    for (int off = kWave / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0)
        s_red[wv] = v;
    __syncthreads();
    uint64_t t = 0;
    for (int i = 0; i < kWavesPerBlock; ++i)
        t += s_red[i];
    __syncthreads();
    return t;
}

__global__ void __launch_bounds__(kBlock) unweight_count_kernel(UnweightParams U)
{
    __shared__ uint64_t s_red[kWavesPerBlock];
    const uint64_t start = (uint64_t)blockIdx.x * U.per_block;
    const uint64_t end = start + U.per_block < U.n ? start + U.per_block : U.n;
    uint64_t kept = 0, over = 0;
    for (uint64_t e = start + threadIdx.x; e < end; e += kBlock) {
        bool ov;
        signed char sg;
        kept += keep_event(U, e, ov, sg) ? 1 : 0;
        over += ov ? 1 : 0;
    }
    kept = block_sum_u64(kept, s_red);
    over = block_sum_u64(over, s_red);
    if (threadIdx.x == 0) {
        U.counts[2 * blockIdx.x] = kept;
        U.counts[2 * blockIdx.x + 1] = over;
    }
}

// Lab-frame momenta of event e: gluon a (+z), gluon b (-z), t, tbar, final
// gluons.  The partonic CM momenta are boosted along z with
// gamma = (x1 + x2) / (2 sqrt(x1 x2)), gamma beta = (x1 - x2) / (2 sqrt(x1 x2)).
// Returns false if the event has no phase-space point.
template <int NF>
__device__ bool lab_momenta(const EventParams& P, uint64_t e, double* out)
{
#pragma clang fp contract(off)
    constexpr int D = 2 + 3 * NF - 4;
    double x[D];
    unsigned short bins[D];
    draw_point<D>(P, e, x, bins, 1);
    const double x1 = x[0], x2 = x[1];
    const double shat = x1 * x2 * P.sqrt_s * P.sqrt_s;
    const double thr = 2.0 * P.m_top;
    if (!(shat > thr * thr))
        return false;
    double k[NF][4], W;
    if (!phase_space<NF>(x + 2, sqrt(shat), P.m_top, P.max_newton, P.ps_const, k, W))
        return false;
    const double eb = 0.5 * P.sqrt_s;
    out[0] = x1 * eb; out[1] = 0.0; out[2] = 0.0; out[3] = x1 * eb;
    out[4] = x2 * eb; out[5] = 0.0; out[6] = 0.0; out[7] = -(x2 * eb);
    const double r2 = 2.0 * sqrt(x1 * x2);
    const double g = (x1 + x2) / r2, gb = (x1 - x2) / r2;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        double* q = out + 4 * (2 + i);
        q[0] = g * k[i][0] + gb * k[i][3];
        q[1] = k[i][1];
        q[2] = k[i][2];
        q[3] = g * k[i][3] + gb * k[i][0];
    }
    return true;
}

template <int NF>
__global__ void __launch_bounds__(kBlock) unweight_write_kernel(UnweightParams U)
{
    __shared__ uint64_t s_cnt[kWavesPerBlock];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint64_t start = (uint64_t)blockIdx.x * U.per_block;
    const uint64_t end = start + U.per_block < U.n ? start + U.per_block : U.n;
    uint64_t base = U.offsets[blockIdx.x];
    for (uint64_t c0 = start; c0 < end; c0 += kBlock) {
        const uint64_t e = c0 + threadIdx.x;
        bool over = false;
        signed char sign = 0;
        const bool keep = e < end && keep_event(U, e, over, sign);
        const uint64_t mask = __ballot(keep);
        if (lane == 0)
            s_cnt[wv] = (uint64_t)__popcll(mask);
        __syncthreads();
        uint64_t before = 0, total = 0;
        for (int i = 0; i < kWavesPerBlock; ++i) {
            before += i < wv ? s_cnt[i] : 0;
            total += s_cnt[i];
        }
        const uint64_t below = mask & ((1ull << lane) - 1ull);
        const uint64_t slot = base + before + (uint64_t)__popcll(below);
        if (keep && slot < U.capacity) {
            U.ev_out[slot] = e;
            if (U.sign_out)
                U.sign_out[slot] = sign;
            if (U.p_out) {
                double q[4 * (NF + 2)];
                if (!lab_momenta<NF>(U.P, e, q))
                    for (int i = 0; i < 4 * (NF + 2); ++i)
                        q[i] = 0.0;
                for (int i = 0; i < 4 * (NF + 2); ++i)
                    U.p_out[slot * (4 * (NF + 2)) + i] = q[i];
            }
        }
        base += total;
        __syncthreads();
    }
}

}  // namespace mf
