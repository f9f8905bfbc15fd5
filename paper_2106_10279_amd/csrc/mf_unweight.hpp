// mf_unweight.hpp -- hit-or-miss unweighting of weighted events on the GPU
// (Sec. 2.5: the weighted events of the integration are turned into
// unit-weight events for the LHE output).
//
// Event e of weight w_e is kept when u_e w_max < |w_e|, u_e being the first
// 53-bit uniform of the Philox block 0x80000000 of the event's counter
// (e mod 2^32, e >> 32, iter, 0x80000000); the integrand draws only from
// blocks 0 .. ceil(D/2) - 1.  A kept event carries the sign of w_e.
//
// Kernels over contiguous event ranges, one range per workgroup: a count
// pass that forms the keep flag (the sign, or 0) of every event and counts
// kept and above-w_max events per workgroup, and a write pass in which every
// thread reads 16 consecutive flags and places its kept events after a
// workgroup scan, so that records come out in increasing event index.  A
// last kernel, one thread per written record, adds the lab-frame momenta.
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
    signed char* flags;      // [n] sign of each kept event, 0 for the others (count pass)
    uint64_t* totals;        // [2]: kept, above w_max over all events (write pass)
    uint64_t n_blocks;
    uint64_t capacity;
    uint64_t* ev_out;        // [capacity]
    double* p_out;           // [capacity][NF + 2][4] or null
    signed char* sign_out;   // [capacity] or null
};

__device__ __forceinline__ bool keep_w(const UnweightParams& U, uint64_t e, double w, bool& over, signed char& sign)
{
#pragma clang fp contract(off)
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

constexpr int kUnweightTile = 16 * kBlock;   // events per tile of a workgroup's range
constexpr int kUnweightSeg = kUnweightTile / kBlock;

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
    for (uint64_t t0 = start; t0 < end; t0 += kUnweightTile) {
        double wv[kUnweightSeg];
#pragma unroll
        for (int i = 0; i < kUnweightSeg; ++i) {
            const uint64_t e = t0 + (uint64_t)(i * kBlock) + threadIdx.x;
            wv[i] = e < end ? U.w[e] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kUnweightSeg; ++i) {
            const uint64_t e = t0 + (uint64_t)(i * kBlock) + threadIdx.x;
            if (e < end) {
                bool ov;
                signed char sg;
                const bool k = keep_w(U, e, wv[i], ov, sg);
                U.flags[e] = k ? sg : 0;
                kept += k ? 1 : 0;
                over += ov ? 1 : 0;
            }
        }
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

// Exclusive prefix sum over the threads of a workgroup (wave scans, then the
// wave totals through LDS); *total receives the workgroup's sum.
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* s_wave, uint64_t* total)
{
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    uint64_t incl = v;
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t o = __shfl_up(incl, off, kWave);
        if (lane >= off)
            incl += o;
    }
    if (lane == kWave - 1)
        s_wave[wv] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
        before += i < wv ? s_wave[i] : 0;
        all += s_wave[i];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// The workgroup's range in tiles of 4096 events; each thread reads the
// flags of 16 consecutive events (one 16-byte load), and after a workgroup
// scan writes the index and sign of its kept events in event order.  The
// workgroup's first record follows the kept events of all workgroups before
// it (summed here from the count pass); workgroup 0 also writes the totals.
__global__ void __launch_bounds__(kBlock) unweight_write_kernel(UnweightParams U)
{
    __shared__ uint64_t s_wave[kWavesPerBlock];
    const uint64_t b = blockIdx.x;
    uint64_t pre = 0;
    for (uint64_t i = threadIdx.x; i < b; i += kBlock)
        pre += U.counts[2 * i];
    uint64_t base = block_sum_u64(pre, s_wave);
    if (b == 0) {
        uint64_t k = 0, o = 0;
        for (uint64_t i = threadIdx.x; i < U.n_blocks; i += kBlock) {
            k += U.counts[2 * i];
            o += U.counts[2 * i + 1];
        }
        k = block_sum_u64(k, s_wave);
        o = block_sum_u64(o, s_wave);
        if (threadIdx.x == 0) {
            U.totals[0] = k;
            U.totals[1] = o;
        }
    }
    const uint64_t start = b * U.per_block;
    const uint64_t end = start + U.per_block < U.n ? start + U.per_block : U.n;
    for (uint64_t t0 = start; t0 < end; t0 += kUnweightTile) {
        const uint64_t e0 = t0 + (uint64_t)kUnweightSeg * threadIdx.x;
        signed char f[kUnweightSeg];
        if (e0 + kUnweightSeg <= end) {
            const int4 v = *reinterpret_cast<const int4*>(U.flags + e0);
            const int words[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < kUnweightSeg; ++j)
                f[j] = (signed char)((unsigned)words[j / 4] >> (8 * (j % 4)));
        } else {
#pragma unroll
            for (int j = 0; j < kUnweightSeg; ++j)
                f[j] = e0 + j < end ? U.flags[e0 + j] : 0;
        }
        uint64_t cnt = 0;
#pragma unroll
        for (int j = 0; j < kUnweightSeg; ++j)
            cnt += f[j] != 0 ? 1 : 0;
        uint64_t total;
        uint64_t slot = base + block_exclusive_scan(cnt, s_wave, &total);
#pragma unroll
        for (int j = 0; j < kUnweightSeg; ++j) {
            if (f[j] == 0)
                continue;
            if (slot < U.capacity) {
                U.ev_out[slot] = e0 + j;
                if (U.sign_out)
                    U.sign_out[slot] = f[j];
            }
            ++slot;
        }
        base += total;
    }
}

// Lab-frame record of every written event (slots below min(capacity, kept)).
template <int NF>
__global__ void __launch_bounds__(kBlock) unweight_record_kernel(UnweightParams U, const uint64_t* totals)
{
    const uint64_t kept = totals[0] < U.capacity ? totals[0] : U.capacity;
    for (uint64_t slot = (uint64_t)blockIdx.x * kBlock + threadIdx.x; slot < kept;
         slot += (uint64_t)gridDim.x * kBlock) {
        double q[4 * (NF + 2)];
        if (!lab_momenta<NF>(U.P, U.ev_out[slot], q))
            for (int i = 0; i < 4 * (NF + 2); ++i)
                q[i] = 0.0;
        for (int i = 0; i < 4 * (NF + 2); ++i)
            U.p_out[slot * (4 * (NF + 2)) + i] = q[i];
    }
}

}  // namespace mf
