// mf_lib.hip -- host runtime and C ABI of libmadflow_mi355x (see include/mf.h).
//
// The iteration loop of the VEGAS integration (Sec. 2.2) is enqueued on one
// HIP stream without host round trips: per iteration one fused event kernel
// and one reduce-and-refine kernel; the per-iteration estimates stay on the
// device until the loop ends.  Argument checks run on the host before any
// HIP call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mf.h"
#include "mf_grad.hpp"
#include "mf_kernels.hpp"
#include "mf_unweight.hpp"

// Static device scratch of mf_integrate_static, for callers that cannot
// allocate device memory.  Every device the library runs on holds its own
// copy from module load until the process ends.  Host code never passes this
// name to a kernel or a copy: it uses the address hipGetSymbolAddress returns
// on that device (Workspace::scratch).
constexpr size_t kScratchBytes = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxIter = 256;            // iterations per call
constexpr int kScratchMaxCells = 512;    // n_dims * n_bins in the static scratch
constexpr long kScratchMaxPdf = 65536;   // PDF table values in the static scratch

thread_local std::string g_error;

// Clears n doubles (a kernel rather than a memset node, so that a captured
// stream replays it faithfully).
__global__ void zero_kernel(double* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0.0;
}

// Clears the live-event count of a batch before kin_kernel appends to it.
__global__ void clear_count_kernel(unsigned long long* n)
{
    *n = 0ull;
}

mf_status fail(mf_status st, const std::string& msg)
{
    g_error = msg;
    return st;
}

#define MF_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(MF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

int n_gluons(int id)
{
    switch (id) {
    case MF_GG_TTX: return 2;
    case MF_GG_TTXG: return 3;
    case MF_GG_TTXGG: return 4;
    case MF_GG_TTXGGG: return 5;
    case MF_PP_TTX: return 2;
    case MF_PP_TTXG: return 3;
    case MF_PP_TTXGG: return 4;
    default: return -1;
    }
}

// p p processes: the g g channel plus the q qbar channels from the quark tables.
bool is_pp(int id)
{
    return id == MF_PP_TTX || id == MF_PP_TTXG || id == MF_PP_TTXGG;
}

double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i)
        f *= i;
    return f;
}

// Device buffers reused across calls on one device (grow-only).
struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Events per batch of the three-kernel form (per-event buffers of about
// 170 B for t tbar g g: 23 GB at the cap, sized for a 288 GB device).
constexpr uint64_t kStageBatch = 1ull << 27;
// t tbar g g g: the partial amplitudes of a batch pass through device memory
// (120 x 128 complex values per event: 8 GB per batch in FP64).
constexpr uint64_t kStageBatchNg5 = 1ull << 15;

struct Workspace {
    std::mutex lock;
    Buffer grid[2], log_x, log_q2, xf, partials, entries, iter_I, iter_V, iter_pass, stats, gpartials, gsum;
    Buffer st_mom, st_pref, st_me, st_bins, st_flags;   // per-event hand-over of the three-kernel form
    Buffer amp_counter;                                  // work counter of amp_kernel (8 bytes)
    Buffer live_list, live_count;                        // live events of a batch (n_g <= 4) and their count
    Buffer st_amp;                                       // t tbar g g g: partial amplitudes of a batch
    Buffer xq, st_prefq, st_meq;                         // p p: quark tables; per-event q qbar prefactors, |M|^2
    Buffer uw_counts, uw_flags, uw_totals;               // unweighting: per-workgroup counts, keep flags, totals
    int n_cu = 0;
    void* scratch = nullptr;  // this device's address of the static scratch array (mf_integrate_static)
};

Workspace g_ws[64];

mf_status ensure(Buffer& b, size_t bytes)
{
    if (b.bytes >= bytes)
        return MF_OK;
    if (b.ptr) {
        hipError_t e = hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
        if (e != hipSuccess)
            return fail(MF_EDEVICE, std::string("hipFree: ") + hipGetErrorString(e));
    }
    size_t want = bytes < 256 ? 256 : bytes;
    hipError_t e = hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        return fail(MF_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    b.bytes = want;
    return MF_OK;
}

// Device memory of one integration: pointers into the grow-only workspace
// (mf_integrate) or into the static scratch array (mf_integrate_static).
struct Mem {
    double* grid[2] = {nullptr, nullptr};
    double *log_x = nullptr, *log_q2 = nullptr, *xf = nullptr;
    double *partials = nullptr, *entries = nullptr, *iter_I = nullptr, *iter_V = nullptr, *iter_pass = nullptr;
    double *stats = nullptr, *gpartials = nullptr, *gsum = nullptr;
    double *st_mom = nullptr, *st_pref = nullptr, *st_me = nullptr;
    unsigned short* st_bins = nullptr;
    unsigned char* st_flags = nullptr;
    unsigned long long* amp_counter = nullptr;
    unsigned* live_list = nullptr;
    unsigned long long* live_count = nullptr;
    void* st_amp = nullptr;
    double *xq = nullptr, *st_prefq = nullptr, *st_meq = nullptr;
};

// Consecutive 256-byte aligned pieces of a fixed device region.
struct Carve {
    unsigned char* base;
    size_t used, cap;
    template <typename T>
    T* take(size_t count)
    {
        const size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        if (bytes > cap - used)
            return nullptr;
        T* p = (T*)(base + used);
        used += bytes;
        return p;
    }
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

bool ascending(const double* v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i]))
            return false;
    for (int i = 1; i < n; ++i)
        if (!(v[i] > v[i - 1]))
            return false;
    return true;
}

int host_interval(const double* knots, int n, double v)
{
    if (v < knots[0]) return 0;
    if (v >= knots[n - 1]) return n - 2;
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (knots[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

mf_status validate_process(const mf_process* proc, double sqrt_s, int* ng)
{
    if (!proc)
        return fail(MF_EINVAL, "process is NULL");
    *ng = n_gluons(proc->id);
    if (*ng < 0)
        return fail(MF_EINVAL, "unknown process id");
    if (!finite_pos(proc->m_top))
        return fail(MF_EINVAL, "m_top must be finite and > 0");
    if (!std::isfinite(proc->w_top) || proc->w_top < 0.0)
        return fail(MF_EINVAL, "w_top must be finite and >= 0");
    if (!finite_pos(proc->alpha_s))
        return fail(MF_EINVAL, "alpha_s must be finite and > 0");
    if (!finite_pos(proc->mu_f))
        return fail(MF_EINVAL, "mu_f must be finite and > 0");
    if (!std::isfinite(proc->ptmin_g) || !std::isfinite(proc->etamax_g) || !std::isfinite(proc->drmin_gg))
        return fail(MF_EINVAL, "cut values must be finite");
    if (!std::isfinite(sqrt_s) || !(sqrt_s > 2.0 * proc->m_top))
        return fail(MF_EINVAL, "sqrt_s must exceed 2 m_top");
    return MF_OK;
}

mf_status validate_pdf(const mf_pdf_grid* pdf, double mu_f)
{
    if (!pdf || !pdf->log_x || !pdf->log_q2 || !pdf->xf)
        return fail(MF_EINVAL, "PDF grid or one of its arrays is NULL");
    if (pdf->n_x < 4 || pdf->n_x > mf::kMaxPdfX)
        return fail(MF_EINVAL, "n_x must be in [4, 256]");
    if (pdf->n_q2 < 4 || pdf->n_q2 > 4096)
        return fail(MF_EINVAL, "n_q2 must be in [4, 4096]");
    if (!ascending(pdf->log_x, pdf->n_x) || !ascending(pdf->log_q2, pdf->n_q2))
        return fail(MF_EINVAL, "PDF knots must be finite and strictly ascending");
    const double lq = std::log(mu_f * mu_f);
    if (lq < pdf->log_q2[0] || lq > pdf->log_q2[pdf->n_q2 - 1])
        return fail(MF_EINVAL, "mu_f^2 lies outside the PDF Q^2 grid");
    for (long i = 0; i < (long)pdf->n_x * pdf->n_q2; ++i)
        if (!std::isfinite(pdf->xf[i]))
            return fail(MF_EINVAL, "PDF values must be finite");
    return MF_OK;
}

// p p processes: the quark tables must be there and finite.
mf_status validate_quarks(const mf_process* proc, const mf_pdf_grid* pdf)
{
    if (!is_pp(proc->id))
        return MF_OK;
    if (!pdf->xq)
        return fail(MF_EINVAL, "p p processes need the quark tables (pdf->xq)");
    for (long i = 0; i < 4L * pdf->n_x * pdf->n_q2; ++i)
        if (!std::isfinite(pdf->xq[i]))
            return fail(MF_EINVAL, "quark PDF values must be finite");
    return MF_OK;
}

mf_status validate_options(const mf_options* opt, int D)
{
    if (!opt)
        return fail(MF_EINVAL, "options are NULL");
    if (opt->n_bins < 2 || opt->n_bins > 1024)
        return fail(MF_EINVAL, "n_bins must be in [2, 1024]");
    if ((long)D * opt->n_bins > 2048)
        return fail(MF_EUNSUPPORTED, "n_dims * n_bins above 2048 does not fit the LDS histogram");
    if (!finite_pos(opt->alpha))
        return fail(MF_EINVAL, "alpha must be finite and > 0");
    if (opt->precision != MF_FP64 && opt->precision != MF_FP32_KAHAN)
        return fail(MF_EINVAL, "unknown precision");
    if (opt->colour != MF_COLOUR_FULL && opt->colour != MF_COLOUR_LEADING && opt->colour != MF_COLOUR_SAMPLED &&
        opt->colour != MF_COLOUR_FLOW)
        return fail(MF_EINVAL, "unknown colour mode");
    if (opt->helicity != MF_HELICITY_SUM && opt->helicity != MF_HELICITY_SAMPLED)
        return fail(MF_EINVAL, "unknown helicity mode");
    if (opt->max_batch > kStageBatch)
        return fail(MF_EINVAL, "max_batch must be at most 2^27");
    if (opt->max_newton < 0 || opt->max_newton > 1000)
        return fail(MF_EINVAL, "max_newton must be in [0, 1000]");
    if (opt->start_iter < 0)
        return fail(MF_EINVAL, "start_iter must be >= 0");
    if (opt->grid_in) {
        const int nb = opt->n_bins;
        for (int d = 0; d < D; ++d) {
            const double* e = opt->grid_in + (size_t)d * (nb + 1);
            if (e[0] != 0.0 || e[nb] != 1.0 || !ascending(e, nb + 1))
                return fail(MF_EINVAL, "grid rows must rise strictly from 0 to 1");
        }
    }
    return MF_OK;
}

struct Setup {
    int ng, D;
    mf::EventParams P;
    hipStream_t stream;
    Workspace* ws;
};

// PDF buffers of the grow-only workspace.
mf_status workspace_pdf(const mf_pdf_grid* pdf, Workspace& ws, Mem& m)
{
    const int nx = pdf->n_x, nq = pdf->n_q2;
    mf_status st;
    if ((st = ensure(ws.log_x, sizeof(double) * nx)) != MF_OK) return st;
    if ((st = ensure(ws.log_q2, sizeof(double) * nq)) != MF_OK) return st;
    if ((st = ensure(ws.xf, sizeof(double) * nx * (size_t)nq)) != MF_OK) return st;
    m.log_x = (double*)ws.log_x.ptr;
    m.log_q2 = (double*)ws.log_q2.ptr;
    m.xf = (double*)ws.xf.ptr;
    if (pdf->xq) {
        if ((st = ensure(ws.xq, sizeof(double) * 4 * nx * (size_t)nq)) != MF_OK) return st;
        m.xq = (double*)ws.xq.ptr;
    }
    return MF_OK;
}

// Upload the PDF table into m's PDF buffers and fill the launch parameters
// shared by all modes.
mf_status prepare(const mf_process* proc, double sqrt_s, const mf_pdf_grid* pdf, const mf_options* opt,
                  const Mem& m, Setup& S)
{
    const int nx = pdf->n_x, nq = pdf->n_q2;
    MF_HIP(hipMemcpyAsync(m.log_x, pdf->log_x, sizeof(double) * nx, hipMemcpyHostToDevice, S.stream));
    MF_HIP(hipMemcpyAsync(m.log_q2, pdf->log_q2, sizeof(double) * nq, hipMemcpyHostToDevice, S.stream));
    MF_HIP(hipMemcpyAsync(m.xf, pdf->xf, sizeof(double) * nx * (size_t)nq, hipMemcpyHostToDevice, S.stream));
    const bool pp = is_pp(proc->id);
    if (pp) {
        if (!m.xq)
            return fail(MF_EUNSUPPORTED, "no device room for the quark tables");
        MF_HIP(hipMemcpyAsync(m.xq, pdf->xq, sizeof(double) * 4 * nx * (size_t)nq, hipMemcpyHostToDevice, S.stream));
    }

    mf::EventParams& P = S.P;
    std::memset(&P, 0, sizeof(P));
    P.n_g = S.ng;
    P.n_dims = S.D;
    P.n_bins = opt->n_bins;
    P.max_newton = opt->max_newton;
    P.n_x = nx;
    P.n_q2 = nq;
    P.log_muf2 = std::log(proc->mu_f * proc->mu_f);
    const int mq = host_interval(pdf->log_q2, nq, P.log_muf2);
    const int first = mq - 1 < 0 ? 0 : mq - 1;
    const int last = mq + 2 > nq - 1 ? nq - 1 : mq + 2;
    P.q2_first = first;
    P.q2_rows = last - first + 1;
    P.q2_interval = mq;
    P.log_x = m.log_x;
    P.log_q2 = m.log_q2;
    P.xf = m.xf;
    P.sqrt_s = sqrt_s;
    P.s_had = sqrt_s * sqrt_s;
    P.m_top = proc->m_top;
    P.mw = proc->m_top * proc->w_top;
    P.ptmin = proc->ptmin_g;
    P.etamax = proc->etamax_g;
    P.drmin = proc->drmin_gg;
    const int n = S.ng;
    const double gs2 = 4.0 * mf::kPi * proc->alpha_s;
    P.me_norm = std::pow(gs2, n) / (4.0 * 64.0 * factorial(n - 2)) * mf::kGeV2ToPb;
    P.ps_const = std::pow(2.0 * mf::kPi, 4 - 3 * n) * std::pow(mf::kPi / 2.0, n - 1) /
                 (factorial(n - 1) * factorial(n - 2));
    P.hel_mc = opt->helicity == MF_HELICITY_SAMPLED;
    P.pp = pp ? 1 : 0;
    P.xq = pp ? m.xq : nullptr;
    // q qbar: average over 2 x 2 helicities and 3 x 3 colours, g_s^(2 n_g),
    // 1/(n_g - 2)! for identical final-state gluons
    P.me_norm_q = std::pow(gs2, n) / (36.0 * factorial(n - 2)) * mf::kGeV2ToPb;
    return MF_OK;
}

template <int NG, typename T, int COL>
mf_status launch_event(const mf::EventParams& P, int blocks, hipStream_t stream)
{
    constexpr int D = 2 + 3 * NG - 4;
    const size_t dyn = P.partials ? sizeof(double) * mf::kWavesPerBlock * D * P.n_bins : 0;
    hipLaunchKernelGGL((mf::event_kernel<NG, T, COL>), dim3(blocks), dim3(mf::kBlock), dyn, stream, P);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <int NG, int COL>
mf_status launch_event_prec(mf_precision prec, const mf::EventParams& P, int blocks, hipStream_t s)
{
    return prec == MF_FP32_KAHAN ? launch_event<NG, float, COL>(P, blocks, s)
                                 : launch_event<NG, double, COL>(P, blocks, s);
}

mf_status dispatch_event(int ng, mf_precision prec, mf_colour col, const mf::EventParams& P, int blocks,
                         hipStream_t s)
{
    if (col == MF_COLOUR_SAMPLED || col == MF_COLOUR_FLOW)
        return fail(MF_EUNSUPPORTED, "the Monte Carlo over colours runs in mf_integrate for g g -> t tbar g (g) only");
    const bool lc = col == MF_COLOUR_LEADING;
    switch (ng) {
    case 2: return lc ? launch_event_prec<2, 1>(prec, P, blocks, s) : launch_event_prec<2, 0>(prec, P, blocks, s);
    case 3: return lc ? launch_event_prec<3, 1>(prec, P, blocks, s) : launch_event_prec<3, 0>(prec, P, blocks, s);
    default: return lc ? launch_event_prec<4, 1>(prec, P, blocks, s) : launch_event_prec<4, 0>(prec, P, blocks, s);
    }
}

// Amplitude-kernel workgroups (one wave each) for the persistent loop: as
// many as can be resident at once, so that every workgroup runs from start to
// end alongside all the others (the groups of events are assigned statically).
template <int NG, typename T, int COL, bool PP = false>
mf_status amp_grid_for(uint64_t n_groups, int n_cu, int* grid)
{
    int per_cu = 0;
    MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mf::amp_kernel<NG, T, COL, PP>, mf::kWave, 0));
    if (per_cu < 1)
        per_cu = 1;
    const uint64_t cap = (uint64_t)n_cu * per_cu;
    *grid = (int)(n_groups < cap ? (n_groups < 1 ? 1 : n_groups) : cap);
    return MF_OK;
}

template <int NG, typename T, int COL>
mf_status launch_stages(const mf::StageParams& S, int kin_blocks, int n_cu, hipStream_t stream,
                        hipEvent_t amp_begin, hipEvent_t amp_end, bool accumulate = true)
{
    constexpr int D = 2 + 3 * NG - 4;
    constexpr bool kCanPP = NG == 2 && COL == 0;
    const bool pp = kCanPP && S.P.pp;
    const uint64_t n_groups = (S.count + mf::Layout<NG>::kEventsPerPass - 1) / mf::Layout<NG>::kEventsPerPass;
    int amp_grid = 1;
    mf_status st = pp ? amp_grid_for<NG, T, COL, kCanPP>(n_groups, n_cu, &amp_grid)
                      : amp_grid_for<NG, T, COL>(n_groups, n_cu, &amp_grid);
    if (st != MF_OK)
        return st;
    if (S.live) {
        hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(1), 0, stream, S.n_live);
        MF_HIP(hipGetLastError());
    }
    if constexpr (NG == 2 || NG == 3 || NG == 4) {
        if (S.P.pp)
            hipLaunchKernelGGL((mf::kin_kernel<NG, true>), dim3(kin_blocks), dim3(mf::kBlock), 0, stream, S);
        else
            hipLaunchKernelGGL((mf::kin_kernel<NG>), dim3(kin_blocks), dim3(mf::kBlock), 0, stream, S);
    } else {
        hipLaunchKernelGGL((mf::kin_kernel<NG>), dim3(kin_blocks), dim3(mf::kBlock), 0, stream, S);
    }
    MF_HIP(hipGetLastError());
    if (amp_begin)
        MF_HIP(hipEventRecord(amp_begin, stream));
    if (pp)
        hipLaunchKernelGGL((mf::amp_kernel<NG, T, COL, kCanPP>), dim3(amp_grid), dim3(mf::kWave), 0, stream, S);
    else
        hipLaunchKernelGGL((mf::amp_kernel<NG, T, COL>), dim3(amp_grid), dim3(mf::kWave), 0, stream, S);
    MF_HIP(hipGetLastError());
    if (NG == 3 && S.P.pp) {
        // the q qbar channel of t tbar g (FP64): eight events per one-wave workgroup
        const uint64_t qb = (S.count + mf::kQqEvents - 1) / mf::kQqEvents;
        if (qb > 0x7FFFFFFFull)
            return fail(MF_EINVAL, "too many events for one launch");
        hipLaunchKernelGGL(mf::qqbar_ttxg_kernel, dim3((unsigned)qb), dim3(mf::kWave), 0, stream, S);
        MF_HIP(hipGetLastError());
    }
    if (NG == 4 && S.P.pp) {
        // the q qbar channel of t tbar g g (FP64): one one-wave workgroup per event
        if (S.count > 0x7FFFFFFFull)
            return fail(MF_EINVAL, "too many events for one launch");
        hipLaunchKernelGGL(mf::qqbar_ttxgg_kernel, dim3((unsigned)S.count), dim3(mf::kWave), 0, stream, S);
        MF_HIP(hipGetLastError());
    }
    if (amp_end)
        MF_HIP(hipEventRecord(amp_end, stream));
    if (accumulate) {
        const size_t dyn = sizeof(double) * mf::kWavesPerBlock * D * S.P.n_bins;
        hipLaunchKernelGGL((mf::acc_kernel<NG>), dim3(kin_blocks), dim3(mf::kBlock), dyn, stream, S);
    } else {
        const unsigned wb = (unsigned)((S.count + mf::kBlock - 1) / mf::kBlock);
        hipLaunchKernelGGL(mf::weight_kernel, dim3(wb), dim3(mf::kBlock), 0, stream, S, NG);
    }
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <int NG, int COL>
mf_status launch_stages_prec(mf_precision prec, const mf::StageParams& S, int kin_blocks, int n_cu, hipStream_t s,
                             hipEvent_t a, hipEvent_t b)
{
    return prec == MF_FP32_KAHAN ? launch_stages<NG, float, COL>(S, kin_blocks, n_cu, s, a, b)
                                 : launch_stages<NG, double, COL>(S, kin_blocks, n_cu, s, a, b);
}

// t tbar g g g: phase space, amplitudes (one ten-wave workgroup per event,
// as many as fit at once), colour sum on the matrix cores, accumulation.
// LC: the leading-colour sum (lc_kernel_ng5 in place of the colour kernel).
template <typename T, bool LC = false>
mf_status launch_stages_ng5(const mf::StageParams& S, int kin_blocks, int n_cu, hipStream_t stream,
                            hipEvent_t amp_begin, hipEvent_t amp_end, bool accumulate, hipEvent_t col_begin = nullptr,
                            hipEvent_t col_end = nullptr)
{
    constexpr int D = 2 + 3 * 5 - 4;
    int per_cu = 0, col_per_cu = 0;
    MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mf::amp_kernel_ng5<T, LC>, mf::kBlockNg5, 0));
    MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&col_per_cu, mf::colour_kernel_ng5<T>, mf::kBlock, 0));
    if (per_cu < 1)
        return fail(MF_EDEVICE, "the t tbar g g g amplitude kernel does not fit a compute unit");
    if (col_per_cu < 1)
        col_per_cu = 1;
    const uint64_t amp_cap = (uint64_t)n_cu * per_cu;
    const int amp_grid = (int)(S.count < amp_cap ? S.count : amp_cap);
    const uint64_t col_need = (S.count + mf::kWavesPerBlock - 1) / mf::kWavesPerBlock;
    const uint64_t col_cap = (uint64_t)n_cu * col_per_cu;
    const int col_grid = (int)(col_need < col_cap ? col_need : col_cap);
    hipLaunchKernelGGL((mf::kin_kernel<5>), dim3(kin_blocks), dim3(mf::kBlock), 0, stream, S);
    MF_HIP(hipGetLastError());
    if (amp_begin)
        MF_HIP(hipEventRecord(amp_begin, stream));
    hipLaunchKernelGGL((mf::amp_kernel_ng5<T, LC>), dim3(amp_grid), dim3(mf::kBlockNg5), 0, stream, S);
    MF_HIP(hipGetLastError());
    if (amp_end)
        MF_HIP(hipEventRecord(amp_end, stream));
    if (col_begin)
        MF_HIP(hipEventRecord(col_begin, stream));
    if constexpr (LC) {
        const unsigned lb = (unsigned)((S.count + mf::kBlock - 1) / mf::kBlock);
        hipLaunchKernelGGL(mf::lc_kernel_ng5, dim3(lb), dim3(mf::kBlock), 0, stream, S);
    } else {
        hipLaunchKernelGGL((mf::colour_kernel_ng5<T>), dim3(col_grid), dim3(mf::kBlock), 0, stream, S);
    }
    MF_HIP(hipGetLastError());
    if (col_end)
        MF_HIP(hipEventRecord(col_end, stream));
    if (accumulate) {
        const size_t dyn = sizeof(double) * mf::kWavesPerBlock * D * S.P.n_bins;
        hipLaunchKernelGGL((mf::acc_kernel<5>), dim3(kin_blocks), dim3(mf::kBlock), dyn, stream, S);
    } else {
        const unsigned wb = (unsigned)((S.count + mf::kBlock - 1) / mf::kBlock);
        hipLaunchKernelGGL(mf::weight_kernel, dim3(wb), dim3(mf::kBlock), 0, stream, S, 5);
    }
    MF_HIP(hipGetLastError());
    return MF_OK;
}

mf_status dispatch_stages(int ng, mf_precision prec, mf_colour col, const mf::StageParams& S, int kin_blocks,
                          int n_cu, hipStream_t s, hipEvent_t a, hipEvent_t b, hipEvent_t c = nullptr,
                          hipEvent_t d = nullptr)
{
    if (ng == 5) {
        if (col == MF_COLOUR_LEADING)
            return prec == MF_FP32_KAHAN ? launch_stages_ng5<float, true>(S, kin_blocks, n_cu, s, a, b, true, c, d)
                                         : launch_stages_ng5<double, true>(S, kin_blocks, n_cu, s, a, b, true, c, d);
        if (col != MF_COLOUR_FULL)
            return fail(MF_EUNSUPPORTED, "g g -> t tbar g g g runs with the full or the leading-colour sum");
        return prec == MF_FP32_KAHAN ? launch_stages_ng5<float>(S, kin_blocks, n_cu, s, a, b, true, c, d)
                                     : launch_stages_ng5<double>(S, kin_blocks, n_cu, s, a, b, true, c, d);
    }
    if (ng == 2)
        return col == MF_COLOUR_LEADING ? launch_stages_prec<2, 1>(prec, S, kin_blocks, n_cu, s, a, b)
                                        : launch_stages_prec<2, 0>(prec, S, kin_blocks, n_cu, s, a, b);
    if (ng == 3) {
        if (col == MF_COLOUR_SAMPLED)
            return launch_stages_prec<3, 2>(prec, S, kin_blocks, n_cu, s, a, b);
        if (col == MF_COLOUR_FLOW)
            return launch_stages_prec<3, 3>(prec, S, kin_blocks, n_cu, s, a, b);
        return col == MF_COLOUR_LEADING ? launch_stages_prec<3, 1>(prec, S, kin_blocks, n_cu, s, a, b)
                                        : launch_stages_prec<3, 0>(prec, S, kin_blocks, n_cu, s, a, b);
    }
    if (col == MF_COLOUR_SAMPLED)
        return launch_stages_prec<4, 2>(prec, S, kin_blocks, n_cu, s, a, b);
    if (col == MF_COLOUR_FLOW)
        return launch_stages_prec<4, 3>(prec, S, kin_blocks, n_cu, s, a, b);
    return col == MF_COLOUR_LEADING ? launch_stages_prec<4, 1>(prec, S, kin_blocks, n_cu, s, a, b)
                                    : launch_stages_prec<4, 0>(prec, S, kin_blocks, n_cu, s, a, b);
}

mf_status device_workspace(Workspace** out)
{
    int dev = 0;
    MF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64)
        return fail(MF_EDEVICE, "device index out of range");
    Workspace& ws = g_ws[dev];
    if (ws.n_cu == 0) {
        hipDeviceProp_t prop;
        MF_HIP(hipGetDeviceProperties(&prop, dev));
        ws.n_cu = prop.multiProcessorCount;
    }
    *out = &ws;
    return MF_OK;
}

// Waves launched for n_chunks chunks of 64 events: enough to cover every CU
// several times over, fixed for a given device so the reduction order (and
// hence the result) is reproducible.
int waves_for(uint64_t n_chunks, int n_cu)
{
    uint64_t cap = (uint64_t)n_cu * 32;
    uint64_t w = n_chunks < cap ? n_chunks : cap;
    w = (w + mf::kWavesPerBlock - 1) / mf::kWavesPerBlock * mf::kWavesPerBlock;
    return (int)(w < mf::kWavesPerBlock ? mf::kWavesPerBlock : w);
}

// Neumaier's compensated summation, one term at a time.
void neumaier_add(double& s, double& c, double x)
{
    const double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
}

void combine(int n, const double* I, const double* V, double* sigma, double* err, double* chi2)
{
    // inverse-variance weighted mean with compensated sums over the
    // iterations with V_j > 0, in iteration order
    double ns = 0.0, nc = 0.0, ds = 0.0, dc = 0.0;
    int used = 0;
    for (int j = 0; j < n; ++j)
        if (V[j] > 0.0) {
            neumaier_add(ns, nc, I[j] / V[j]);
            neumaier_add(ds, dc, 1.0 / V[j]);
            ++used;
        }
    if (used == 0) {
        *sigma = n > 0 ? I[n - 1] : 0.0;
        *err = 0.0;
        *chi2 = 0.0;
        return;
    }
    const double sden = ds + dc;
    const double mean = (ns + nc) / sden;
    double cs = 0.0, cc = 0.0;
    for (int j = 0; j < n; ++j)
        if (V[j] > 0.0)
            neumaier_add(cs, cc, (I[j] - mean) * (I[j] - mean) / V[j]);
    *sigma = mean;
    *err = 1.0 / std::sqrt(sden);
    *chi2 = used > 1 ? (cs + cc) / (double)(used - 1) : 0.0;
}

// sum_j (g_j / V_j) / sum_j (1 / V_j) over iterations with V_j > 0 (the
// same weights as the estimate), compensated.
void combine_fixed(int n, const double* g, const double* V, double* out)
{
    double ns = 0.0, nc = 0.0, ds = 0.0, dc = 0.0;
    int used = 0;
    for (int j = 0; j < n; ++j)
        if (V[j] > 0.0) {
            neumaier_add(ns, nc, g[j] / V[j]);
            neumaier_add(ds, dc, 1.0 / V[j]);
            ++used;
        }
    *out = used ? (ns + nc) / (ds + dc) : (n > 0 ? g[n - 1] : 0.0);
}

}  // namespace

extern "C" {

void mf_default_options(mf_options* opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->n_bins = 50;
    opt->alpha = 1.5;
    opt->start_iter = 0;
    opt->precision = MF_FP64;
    opt->strict = 0;
    opt->max_newton = 50;
    opt->grid_in = nullptr;
    opt->stream = nullptr;
    opt->profile = 0;
    opt->max_batch = 0;
    opt->colour = MF_COLOUR_FULL;
    opt->helicity = MF_HELICITY_SUM;
}

int mf_n_dims(int process_id)
{
    const int n = n_gluons(process_id);
    return n < 0 ? -1 : 2 + 3 * n - 4;
}

const char* mf_last_error(void) { return g_error.c_str(); }

}  // extern "C"

namespace {

// The iteration loop of mf_integrate; with `grad`, every iteration also runs
// the adjoint kernel on the grid that iteration used.
mf_status integrate_impl(const mf_process* proc, double sqrt_s, const mf_pdf_grid* pdf, uint64_t n_events,
                         int n_iter, uint64_t seed, const mf_options* opt, mf_result* res, mf_grad_result* grad,
                         bool fixed_scratch)
{
    int ng = 0;
    mf_status st;
    if ((st = validate_process(proc, sqrt_s, &ng)) != MF_OK) return st;
    if ((st = validate_pdf(pdf, proc->mu_f)) != MF_OK) return st;
    if ((st = validate_quarks(proc, pdf)) != MF_OK) return st;
    const int D = 2 + 3 * ng - 4;
    if ((st = validate_options(opt, D)) != MF_OK) return st;
    if (!res)
        return fail(MF_EINVAL, "result is NULL");
    if (n_events < 2 || n_events > (1ull << 40))
        return fail(MF_EINVAL, "n_events must be in [2, 2^40]");
    if (n_iter < 1 || n_iter > kMaxIter)
        return fail(MF_EINVAL, "n_iter must be in [1, 256]");
    if ((uint64_t)opt->start_iter + (uint64_t)n_iter > 0xFFFFFFFFull)
        return fail(MF_EINVAL, "iteration index exceeds the 32-bit Philox counter word");
    if ((opt->colour == MF_COLOUR_SAMPLED || opt->colour == MF_COLOUR_FLOW) && ng == 2)
        return fail(MF_EUNSUPPORTED, "the Monte Carlo over colours runs for g g -> t tbar g (g) only");
    if (ng == 5) {
        if (opt->colour != MF_COLOUR_FULL && opt->colour != MF_COLOUR_LEADING)
            return fail(MF_EUNSUPPORTED, "g g -> t tbar g g g runs with the full or the leading-colour sum");
        if (opt->helicity != MF_HELICITY_SUM)
            return fail(MF_EUNSUPPORTED, "g g -> t tbar g g g runs with the full helicity sum only");
        if (fixed_scratch)
            return fail(MF_EUNSUPPORTED, "mf_integrate_static does not run g g -> t tbar g g g");
    }
    const bool pp = is_pp(proc->id);
    if (pp) {
        if (opt->colour != MF_COLOUR_FULL || opt->helicity != MF_HELICITY_SUM)
            return fail(MF_EUNSUPPORTED, "p p processes run with the full colour and helicity sums only");
        if (fixed_scratch)
            return fail(MF_EUNSUPPORTED, "mf_integrate_static does not run p p processes");
        if (grad)
            return fail(MF_EUNSUPPORTED, "gradients are implemented for g g -> t tbar only");
    }
    if (grad) {
        if (ng != 2)
            return fail(MF_EUNSUPPORTED, "gradients are implemented for g g -> t tbar only");
        if (opt->precision != MF_FP64)
            return fail(MF_EUNSUPPORTED, "gradients are computed in FP64 only");
        if (opt->colour != MF_COLOUR_FULL)
            return fail(MF_EUNSUPPORTED, "gradients are computed with the full colour sum only");
        if (opt->helicity != MF_HELICITY_SUM)
            return fail(MF_EUNSUPPORTED, "gradients are computed with the full helicity sum only");
    }
    const int nb = opt->n_bins;
    if (fixed_scratch) {
        if (grad)
            return fail(MF_EUNSUPPORTED, "mf_integrate_static computes no gradients");
        if (opt->profile)
            return fail(MF_EUNSUPPORTED, "mf_integrate_static does not time kernels (profile must be 0)");
        if (D * nb > kScratchMaxCells)
            return fail(MF_EINVAL, "mf_integrate_static: n_dims * n_bins must be at most 512");
        if ((long)pdf->n_x * pdf->n_q2 > kScratchMaxPdf)
            return fail(MF_EINVAL, "mf_integrate_static: the PDF table must hold at most 65536 values");
    }

    Workspace* wsp = nullptr;
    if ((st = device_workspace(&wsp)) != MF_OK) return st;
    Workspace& ws = *wsp;
    std::lock_guard<std::mutex> guard(ws.lock);

    const uint64_t n_chunks = (n_events + mf::kWave - 1) / mf::kWave;
    const int n_waves = waves_for(n_chunks, ws.n_cu);
    const int stride = mf::kPartialHead + D * nb;
    const size_t grid_bytes = sizeof(double) * D * (size_t)(nb + 1);
    // every process runs as three kernels per batch: phase space, amplitudes,
    // accumulation (mf_evaluate keeps the fused kernel)
    const bool staged = true;
    const int nf = ng;
    uint64_t cap = opt->max_batch ? opt->max_batch : kStageBatch;
    if (ng == 5 && cap > kStageBatchNg5)
        cap = kStageBatchNg5;
    const size_t amp_bytes = ng == 5 ? (opt->precision == MF_FP32_KAHAN ? sizeof(float) : sizeof(double)) *
                                           mf::kAmpEventNg5 : 0;
    Mem m;
    if (fixed_scratch) {
        if (!ws.scratch) {
            // this device's copy of the array; host code uses only this address
            void* addr = nullptr;
            MF_HIP(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)));
            ws.scratch = addr;
        }
        Carve c{(unsigned char*)ws.scratch, 0, kScratchBytes};
        m.grid[0] = c.take<double>((size_t)D * (nb + 1));
        m.grid[1] = c.take<double>((size_t)D * (nb + 1));
        m.log_x = c.take<double>(pdf->n_x);
        m.log_q2 = c.take<double>(pdf->n_q2);
        m.xf = c.take<double>((size_t)pdf->n_x * pdf->n_q2);
        m.entries = c.take<double>(stride);
        m.iter_I = c.take<double>(n_iter);
        m.iter_V = c.take<double>(n_iter);
        m.iter_pass = c.take<double>(n_iter);
        m.stats = c.take<double>(4);
        m.amp_counter = c.take<unsigned long long>(1);
        m.partials = c.take<double>((size_t)n_waves * stride);
        if (!m.partials)
            return fail(MF_ENOMEM, "mf_integrate_static: the per-wave partial sums do not fit the static scratch");
        if (staged) {
            // the per-event hand-over takes what is left, in whole 256-event steps
            const size_t per_event = sizeof(double) * (4 * nf + 1) + 2 * sizeof(double) +
                                     sizeof(unsigned short) * D + 1;
            const size_t left = c.cap - c.used;
            uint64_t fit = left > 5 * 256 ? (left - 5 * 256) / per_event / 256 * 256 : 0;
            if (fit < 256)
                return fail(MF_ENOMEM, "mf_integrate_static: no room left in the static scratch for an event batch");
            if (cap > fit)
                cap = fit;
        }
        const uint64_t b0 = n_events < cap ? n_events : cap;
        if (staged) {
            m.st_mom = c.take<double>((size_t)(4 * nf + 1) * b0);
            m.st_pref = c.take<double>(b0);
            m.st_me = c.take<double>(b0);
            m.st_bins = c.take<unsigned short>((size_t)D * b0);
            m.st_flags = c.take<unsigned char>(b0);
            if (!m.st_flags)
                return fail(MF_ENOMEM, "mf_integrate_static: event batch does not fit the static scratch");
        }
    } else {
        if ((st = workspace_pdf(pdf, ws, m)) != MF_OK) return st;
        if ((st = ensure(ws.grid[0], grid_bytes)) != MF_OK) return st;
        if ((st = ensure(ws.grid[1], grid_bytes)) != MF_OK) return st;
        if ((st = ensure(ws.partials, sizeof(double) * (size_t)n_waves * stride)) != MF_OK) return st;
        if ((st = ensure(ws.entries, sizeof(double) * (size_t)stride)) != MF_OK) return st;
        if ((st = ensure(ws.iter_I, sizeof(double) * n_iter)) != MF_OK) return st;
        if ((st = ensure(ws.iter_V, sizeof(double) * n_iter)) != MF_OK) return st;
        if ((st = ensure(ws.iter_pass, sizeof(double) * n_iter)) != MF_OK) return st;
        if ((st = ensure(ws.stats, sizeof(double) * 4)) != MF_OK) return st;
        const uint64_t b0 = n_events < cap ? n_events : cap;
        if (staged) {
            if ((st = ensure(ws.st_mom, sizeof(double) * (4 * nf + 1) * b0)) != MF_OK) return st;
            if ((st = ensure(ws.st_pref, sizeof(double) * b0)) != MF_OK) return st;
            if ((st = ensure(ws.st_me, sizeof(double) * b0)) != MF_OK) return st;
            if ((st = ensure(ws.st_bins, sizeof(unsigned short) * D * b0)) != MF_OK) return st;
            if ((st = ensure(ws.st_flags, b0)) != MF_OK) return st;
            if ((st = ensure(ws.amp_counter, sizeof(unsigned long long))) != MF_OK) return st;
            if (amp_bytes && (st = ensure(ws.st_amp, amp_bytes * b0)) != MF_OK) return st;
            if (ng <= 4) {
                if ((st = ensure(ws.live_list, sizeof(unsigned) * b0)) != MF_OK) return st;
                if ((st = ensure(ws.live_count, sizeof(unsigned long long))) != MF_OK) return st;
            }
            if (pp) {
                const size_t orient = ng >= 3 ? 2 : 1;   // t tbar g (g): both beam orientations
                if ((st = ensure(ws.st_prefq, sizeof(double) * orient * b0)) != MF_OK) return st;
                if ((st = ensure(ws.st_meq, sizeof(double) * orient * b0)) != MF_OK) return st;
            }
        }
        if (grad) {
            if ((st = ensure(ws.gpartials, sizeof(double) * 4 * (size_t)n_waves)) != MF_OK) return st;
            if ((st = ensure(ws.gsum, sizeof(double) * 4 * (size_t)n_iter)) != MF_OK) return st;
        }
        m.grid[0] = (double*)ws.grid[0].ptr;
        m.grid[1] = (double*)ws.grid[1].ptr;
        m.partials = (double*)ws.partials.ptr;
        m.entries = (double*)ws.entries.ptr;
        m.iter_I = (double*)ws.iter_I.ptr;
        m.iter_V = (double*)ws.iter_V.ptr;
        m.iter_pass = (double*)ws.iter_pass.ptr;
        m.stats = (double*)ws.stats.ptr;
        m.gpartials = (double*)ws.gpartials.ptr;
        m.gsum = (double*)ws.gsum.ptr;
        m.st_mom = (double*)ws.st_mom.ptr;
        m.st_pref = (double*)ws.st_pref.ptr;
        m.st_me = (double*)ws.st_me.ptr;
        m.st_bins = (unsigned short*)ws.st_bins.ptr;
        m.st_flags = (unsigned char*)ws.st_flags.ptr;
        m.amp_counter = (unsigned long long*)ws.amp_counter.ptr;
        m.st_amp = amp_bytes ? ws.st_amp.ptr : nullptr;
        m.live_list = staged && ng <= 4 ? (unsigned*)ws.live_list.ptr : nullptr;
        m.live_count = staged && ng <= 4 ? (unsigned long long*)ws.live_count.ptr : nullptr;
        m.st_prefq = pp ? (double*)ws.st_prefq.ptr : nullptr;
        m.st_meq = pp ? (double*)ws.st_meq.ptr : nullptr;
    }
    const uint64_t batch = n_events < cap ? n_events : cap;
    const uint64_t n_batches = (n_events + batch - 1) / batch;

    Setup S;
    S.ng = ng;
    S.D = D;
    S.stream = (hipStream_t)opt->stream;
    if ((st = prepare(proc, sqrt_s, pdf, opt, m, S)) != MF_OK) return st;
    mf::EventParams& P = S.P;

    // host copy of the start grid (n_dims * n_bins <= 2048)
    double grid0[2048 + mf::kMaxDims];
    if (opt->grid_in)
        std::memcpy(grid0, opt->grid_in, grid_bytes);
    else
        for (int d = 0; d < D; ++d)
            for (int i = 0; i <= nb; ++i)
                grid0[(size_t)d * (nb + 1) + i] = (double)i / (double)nb;
    MF_HIP(hipMemcpyAsync(m.grid[0], grid0, grid_bytes, hipMemcpyHostToDevice, S.stream));
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, S.stream, m.stats, 4);
    MF_HIP(hipGetLastError());

    P.n_events = n_events;
    P.seed = seed;
    P.partials = m.partials;
    P.stride = stride;
    P.n_waves = n_waves;
    mf::ReduceParams R;
    R.partials = P.partials;
    R.n_waves = n_waves;
    R.stride = stride;
    R.n_dims = D;
    R.n_bins = nb;
    R.n_events = (double)n_events;
    R.alpha = opt->alpha;
    R.entries = m.entries;
    R.hist = R.entries + mf::kPartialHead;
    R.iter_I = m.iter_I;
    R.iter_V = m.iter_V;
    R.iter_pass = m.iter_pass;
    R.stats = m.stats;

    // Optional per-kernel timing: events recorded on the stream around every
    // launch (marks[3j] .. marks[3j+2]).
    std::vector<hipEvent_t> marks, amp_marks, grad_marks;
    // per batch: amplitude kernel begin / end, and for t tbar g g g the colour kernel's
    const size_t kMarks = ng == 5 ? 4 : 2;
    if (opt->profile) {
        marks.resize(3 * (size_t)n_iter);
        for (auto& ev : marks)
            MF_HIP(hipEventCreate(&ev));
        if (grad) {
            grad_marks.resize(2 * (size_t)n_iter);
            for (auto& ev : grad_marks)
                MF_HIP(hipEventCreate(&ev));
        }
        if (staged) {
            amp_marks.resize(kMarks * (size_t)n_iter * n_batches);
            for (auto& ev : amp_marks)
                MF_HIP(hipEventCreate(&ev));
        }
    }
    int cur = 0;
    for (int j = 0; j < n_iter; ++j) {
        P.iter = (uint32_t)(opt->start_iter + j);
        P.grid = m.grid[cur];
        P.weights = (j == n_iter - 1) ? res->weights : nullptr;
        if (opt->profile)
            MF_HIP(hipEventRecord(marks[3 * j], S.stream));
        if (staged) {
            for (uint64_t bi = 0; bi < n_batches; ++bi) {
                mf::StageParams SP;
                SP.P = P;
                SP.first = bi * batch;
                SP.count = (bi + 1 == n_batches) ? n_events - SP.first : batch;
                SP.mom = m.st_mom;
                SP.pref = m.st_pref;
                SP.me = m.st_me;
                SP.bins = m.st_bins;
                SP.flags = m.st_flags;
                SP.first_batch = bi == 0;
                SP.next_group = m.amp_counter;
                SP.amps = m.st_amp;
                SP.pref_q = m.st_prefq;
                SP.me_q = m.st_meq;
                SP.live = m.live_list;
                SP.n_live = m.live_count;
                hipEvent_t a = nullptr, b = nullptr, c = nullptr, d = nullptr;
                if (opt->profile) {
                    const size_t at = kMarks * ((size_t)j * n_batches + bi);
                    a = amp_marks[at];
                    b = amp_marks[at + 1];
                    if (kMarks == 4) {
                        c = amp_marks[at + 2];
                        d = amp_marks[at + 3];
                    }
                }
                if ((st = dispatch_stages(ng, opt->precision, opt->colour, SP, n_waves / mf::kWavesPerBlock,
                                          ws.n_cu, S.stream, a, b, c, d)) != MF_OK)
                    return st;
            }
        } else if ((st = dispatch_event(ng, opt->precision, opt->colour, P, n_waves / mf::kWavesPerBlock,
                                        S.stream)) != MF_OK) {
            return st;
        }
        if (grad) {
            mf::GradParams G;
            G.P = P;
            G.P.weights = nullptr;
            G.P.partials = nullptr;
            G.alpha_s = proc->alpha_s;
            G.w_top = proc->w_top;
            G.dw_dy = (j == n_iter - 1) ? grad->dw_dy : nullptr;
            G.dw_dmt = (j == n_iter - 1) ? grad->dw_dmt : nullptr;
            G.w_out = nullptr;
            G.partials = m.gpartials;
            if (opt->profile)
                MF_HIP(hipEventRecord(grad_marks[2 * j], S.stream));
            hipLaunchKernelGGL(mf::grad_kernel_ttx, dim3(n_waves / mf::kWavesPerBlock), dim3(mf::kBlock), 0, S.stream,
                               G);
            MF_HIP(hipGetLastError());
            if (opt->profile)
                MF_HIP(hipEventRecord(grad_marks[2 * j + 1], S.stream));
            mf::ReduceParams RG = R;
            RG.partials = G.partials;
            RG.stride = 4;
            RG.entries = m.gsum + 4 * (size_t)j;
            hipLaunchKernelGGL(mf::reduce_entries_kernel, dim3(4), dim3(mf::kReduceBlock), 0, S.stream, RG);
            MF_HIP(hipGetLastError());
        }
        if (opt->profile)
            MF_HIP(hipEventRecord(marks[3 * j + 1], S.stream));
        R.grid_in = m.grid[cur];
        R.grid_out = m.grid[1 - cur];
        R.j = j;
        hipLaunchKernelGGL(mf::reduce_entries_kernel, dim3(stride), dim3(mf::kReduceBlock), 0, S.stream, R);
        MF_HIP(hipGetLastError());
        hipLaunchKernelGGL(mf::refine_kernel, dim3(1), dim3(256), 0, S.stream, R);
        MF_HIP(hipGetLastError());
        if (opt->profile)
            MF_HIP(hipEventRecord(marks[3 * j + 2], S.stream));
        cur = 1 - cur;
    }

    double I[kMaxIter], V[kMaxIter], npass[kMaxIter], stats[4], gs[4 * kMaxIter];
    MF_HIP(hipMemcpyAsync(npass, m.iter_pass, sizeof(double) * n_iter, hipMemcpyDeviceToHost, S.stream));
    if (grad)
        MF_HIP(hipMemcpyAsync(gs, m.gsum, sizeof(double) * 4 * n_iter, hipMemcpyDeviceToHost, S.stream));
    MF_HIP(hipMemcpyAsync(I, m.iter_I, sizeof(double) * n_iter, hipMemcpyDeviceToHost, S.stream));
    MF_HIP(hipMemcpyAsync(V, m.iter_V, sizeof(double) * n_iter, hipMemcpyDeviceToHost, S.stream));
    MF_HIP(hipMemcpyAsync(stats, m.stats, sizeof(double) * 4, hipMemcpyDeviceToHost, S.stream));
    if (res->grid)
        MF_HIP(hipMemcpyAsync(res->grid, m.grid[cur], grid_bytes, hipMemcpyDeviceToHost, S.stream));
    if (res->grid_last)
        MF_HIP(hipMemcpyAsync(res->grid_last, m.grid[1 - cur], grid_bytes, hipMemcpyDeviceToHost, S.stream));
    if (res->hist)
        MF_HIP(hipMemcpyAsync(res->hist, m.entries + mf::kPartialHead, sizeof(double) * D * (size_t)nb,
                              hipMemcpyDeviceToHost, S.stream));
    MF_HIP(hipStreamSynchronize(S.stream));
    res->event_kernel_ms = 0.0;
    res->reduce_kernel_ms = 0.0;
    if (opt->profile) {
        for (int j = 0; j < n_iter; ++j) {
            float a = 0.f, b = 0.f;
            MF_HIP(hipEventElapsedTime(&a, marks[3 * j], marks[3 * j + 1]));
            MF_HIP(hipEventElapsedTime(&b, marks[3 * j + 1], marks[3 * j + 2]));
            res->event_kernel_ms += a;
            res->reduce_kernel_ms += b;
            if (res->iter_event_ms)
                res->iter_event_ms[j] = a;
            double amp = a, colour = 0.0;
            if (staged) {
                amp = 0.0;
                for (uint64_t bi = 0; bi < n_batches; ++bi) {
                    const size_t at = kMarks * ((size_t)j * n_batches + bi);
                    float c = 0.f;
                    MF_HIP(hipEventElapsedTime(&c, amp_marks[at], amp_marks[at + 1]));
                    amp += c;
                    if (kMarks == 4) {
                        MF_HIP(hipEventElapsedTime(&c, amp_marks[at + 2], amp_marks[at + 3]));
                        colour += c;
                    }
                }
            }
            if (res->iter_amp_ms)
                res->iter_amp_ms[j] = amp;
            if (res->iter_colour_ms)
                res->iter_colour_ms[j] = colour;
        }
        if (grad && grad->iter_grad_ms)
            for (int j = 0; j < n_iter; ++j) {
                float c = 0.f;
                MF_HIP(hipEventElapsedTime(&c, grad_marks[2 * j], grad_marks[2 * j + 1]));
                grad->iter_grad_ms[j] = c;
            }
        for (auto& ev : marks)
            (void)hipEventDestroy(ev);
        for (auto& ev : amp_marks)
            (void)hipEventDestroy(ev);
        for (auto& ev : grad_marks)
            (void)hipEventDestroy(ev);
    }

    if (opt->strict && stats[2] > 0.0)
        return fail(MF_ENOCONV, "mass-rescaling Newton iteration failed for " +
                                    std::to_string((long long)stats[2]) + " events");
    combine(n_iter, I, V, &res->sigma, &res->sigma_err, &res->chi2_dof);
    res->w_max = stats[0];
    res->n_batches = staged ? n_batches : 1;
    res->n_pass = (int64_t)stats[1];
    res->n_newton_fail = (int64_t)stats[2];
    if (res->iter_sigma)
        std::memcpy(res->iter_sigma, I, sizeof(double) * n_iter);
    if (res->iter_var)
        std::memcpy(res->iter_var, V, sizeof(double) * n_iter);
    if (res->iter_pass)
        std::memcpy(res->iter_pass, npass, sizeof(double) * n_iter);
    if (grad) {
        // Per-iteration means of dw/dtheta on frozen grids, combined with the
        // inverse-variance weights of the estimate (V_j held fixed).
        double gm[kMaxIter], ga[kMaxIter];
        for (int j = 0; j < n_iter; ++j) {
            gm[j] = gs[4 * (size_t)j + 0] / (double)n_events;
            ga[j] = gs[4 * (size_t)j + 2] / (double)n_events;
        }
        combine_fixed(n_iter, gm, V, &grad->dsigma_dmt);
        combine_fixed(n_iter, ga, V, &grad->dsigma_dalphas);
        if (grad->iter_dmt)
            std::memcpy(grad->iter_dmt, gm, sizeof(double) * n_iter);
        if (grad->iter_dalphas)
            std::memcpy(grad->iter_dalphas, ga, sizeof(double) * n_iter);
    }
    return MF_OK;
}

}  // namespace

extern "C" {

mf_status mf_integrate(const mf_process* proc, double sqrt_s, const mf_pdf_grid* pdf, uint64_t n_events,
                       int n_iter, uint64_t seed, const mf_options* opt, mf_result* res)
{
    return integrate_impl(proc, sqrt_s, pdf, n_events, n_iter, seed, opt, res, nullptr, false);
}

mf_status mf_integrate_static(const mf_process* proc, double sqrt_s, const mf_pdf_grid* pdf, uint64_t n_events,
                              int n_iter, uint64_t seed, const mf_options* opt, mf_result* res)
{
    return integrate_impl(proc, sqrt_s, pdf, n_events, n_iter, seed, opt, res, nullptr, true);
}

mf_status mf_integrate_grad(const mf_process* proc, double sqrt_s, const mf_pdf_grid* pdf, uint64_t n_events,
                            int n_iter, uint64_t seed, const mf_options* opt, mf_result* res, mf_grad_result* grad)
{
    if (!grad)
        return fail(MF_EINVAL, "grad is NULL");
    return integrate_impl(proc, sqrt_s, pdf, n_events, n_iter, seed, opt, res, grad, false);
}

}  // extern "C"

namespace {

// Validation, PDF and grid upload for the fixed-grid entry points; the
// workspace stays locked through `lock` until the caller's launch is done.
mf_status fixed_grid_setup(const mf_process* proc, double sqrt_s, const mf_pdf_grid* pdf, const double* grid,
                           uint64_t n, uint64_t seed, int iter, const mf_options* opt, const double* y,
                           const uint64_t* event_ids, std::unique_lock<std::mutex>& lock, Setup& S)
{
    int ng = 0;
    mf_status st;
    if ((st = validate_process(proc, sqrt_s, &ng)) != MF_OK) return st;
    if ((st = validate_pdf(pdf, proc->mu_f)) != MF_OK) return st;
    if ((st = validate_quarks(proc, pdf)) != MF_OK) return st;
    const int D = 2 + 3 * ng - 4;
    if ((st = validate_options(opt, D)) != MF_OK) return st;
    if (n < 1 || n > (1ull << 40))
        return fail(MF_EINVAL, "n must be in [1, 2^40]");
    if (iter < 0)
        return fail(MF_EINVAL, "iter must be >= 0");
    const int nb = opt->n_bins;
    if (grid)
        for (int d = 0; d < D; ++d) {
            const double* e = grid + (size_t)d * (nb + 1);
            if (e[0] != 0.0 || e[nb] != 1.0 || !ascending(e, nb + 1))
                return fail(MF_EINVAL, "grid rows must rise strictly from 0 to 1");
        }
    Workspace* wsp = nullptr;
    if ((st = device_workspace(&wsp)) != MF_OK) return st;
    Workspace& ws = *wsp;
    lock = std::unique_lock<std::mutex>(ws.lock);
    S.ng = ng;
    S.D = D;
    S.ws = wsp;
    S.stream = (hipStream_t)opt->stream;
    Mem m;
    if ((st = workspace_pdf(pdf, ws, m)) != MF_OK) return st;
    if ((st = prepare(proc, sqrt_s, pdf, opt, m, S)) != MF_OK) return st;
    mf::EventParams& P = S.P;
    const size_t grid_bytes = sizeof(double) * D * (size_t)(nb + 1);
    if ((st = ensure(ws.grid[0], grid_bytes)) != MF_OK) return st;
    std::vector<double> g((size_t)D * (nb + 1));
    if (grid)
        std::memcpy(g.data(), grid, grid_bytes);
    else
        for (int d = 0; d < D; ++d)
            for (int i = 0; i <= nb; ++i)
                g[(size_t)d * (nb + 1) + i] = (double)i / (double)nb;
    MF_HIP(hipMemcpyAsync(ws.grid[0].ptr, g.data(), grid_bytes, hipMemcpyHostToDevice, S.stream));
    // the staged host vector must outlive the copy
    MF_HIP(hipStreamSynchronize(S.stream));
    const uint64_t n_chunks = (n + mf::kWave - 1) / mf::kWave;
    P.n_events = n;
    P.seed = seed;
    P.iter = (uint32_t)iter;
    P.grid = (const double*)ws.grid[0].ptr;
    P.y_in = y;
    P.event_ids = event_ids;
    P.partials = nullptr;
    P.n_waves = waves_for(n_chunks, ws.n_cu);
    return MF_OK;
}

// Per-event buffers of a t tbar g g g batch in the grow-only workspace.
mf_status stage_buffers_ng5(Workspace& ws, uint64_t b0, mf_precision prec, mf::StageParams& SP)
{
    constexpr int D = 2 + 3 * 5 - 4;
    constexpr int K = mf::Layout<5>::kMom;
    const size_t amp_bytes = (prec == MF_FP32_KAHAN ? sizeof(float) : sizeof(double)) * mf::kAmpEventNg5;
    mf_status st;
    if ((st = ensure(ws.st_mom, sizeof(double) * K * b0)) != MF_OK) return st;
    if ((st = ensure(ws.st_pref, sizeof(double) * b0)) != MF_OK) return st;
    if ((st = ensure(ws.st_me, sizeof(double) * b0)) != MF_OK) return st;
    if ((st = ensure(ws.st_bins, sizeof(unsigned short) * D * b0)) != MF_OK) return st;
    if ((st = ensure(ws.st_flags, b0)) != MF_OK) return st;
    if ((st = ensure(ws.amp_counter, sizeof(unsigned long long))) != MF_OK) return st;
    if ((st = ensure(ws.st_amp, amp_bytes * b0)) != MF_OK) return st;
    SP.mom = (double*)ws.st_mom.ptr;
    SP.pref = (double*)ws.st_pref.ptr;
    SP.me = (double*)ws.st_me.ptr;
    SP.bins = (unsigned short*)ws.st_bins.ptr;
    SP.flags = (unsigned char*)ws.st_flags.ptr;
    SP.next_group = (unsigned long long*)ws.amp_counter.ptr;
    SP.amps = ws.st_amp.ptr;
    SP.first_batch = 1;
    return MF_OK;
}

// mf_evaluate for the processes that only the staged kernels run (t tbar g g g,
// p p -> t tbar): batches of phase space, amplitudes and weight_kernel,
// which writes the weights (and the records' |M|^2).
mf_status evaluate_staged(Setup& S, const mf_options* opt, uint64_t n)
{
    const bool lc = S.ng == 5 && opt->colour == MF_COLOUR_LEADING;
    if (opt->colour != MF_COLOUR_FULL && !lc)
        return fail(MF_EUNSUPPORTED, "this process runs with the full colour sum only");
    if (opt->helicity != MF_HELICITY_SUM)
        return fail(MF_EUNSUPPORTED, "this process runs with the full helicity sum only");
    const uint64_t big = S.ng == 5 ? kStageBatchNg5 : kStageBatch;
    const uint64_t cap = opt->max_batch && opt->max_batch < big ? opt->max_batch : big;
    const uint64_t batch = n < cap ? n : cap;
    mf::StageParams SP;
    SP.P = S.P;
    mf_status st;
    if (S.ng == 5) {
        if ((st = stage_buffers_ng5(*S.ws, batch, opt->precision, SP)) != MF_OK) return st;
    } else {
        Workspace& ws = *S.ws;
        const int K = 4 * S.ng + 1;           // momenta and beam energy
        if ((st = ensure(ws.st_mom, sizeof(double) * K * batch)) != MF_OK) return st;
        if ((st = ensure(ws.st_pref, sizeof(double) * batch)) != MF_OK) return st;
        if ((st = ensure(ws.st_me, sizeof(double) * batch)) != MF_OK) return st;
        if ((st = ensure(ws.st_bins, sizeof(unsigned short) * S.D * batch)) != MF_OK) return st;
        if ((st = ensure(ws.st_flags, batch)) != MF_OK) return st;
        if ((st = ensure(ws.amp_counter, sizeof(unsigned long long))) != MF_OK) return st;
        const size_t orient = S.ng >= 3 ? 2 : 1;
        if ((st = ensure(ws.st_prefq, sizeof(double) * orient * batch)) != MF_OK) return st;
        if ((st = ensure(ws.st_meq, sizeof(double) * orient * batch)) != MF_OK) return st;
        SP.mom = (double*)ws.st_mom.ptr;
        SP.pref = (double*)ws.st_pref.ptr;
        SP.me = (double*)ws.st_me.ptr;
        SP.bins = (unsigned short*)ws.st_bins.ptr;
        SP.flags = (unsigned char*)ws.st_flags.ptr;
        SP.next_group = (unsigned long long*)ws.amp_counter.ptr;
        SP.amps = nullptr;
        SP.pref_q = (double*)ws.st_prefq.ptr;
        SP.me_q = (double*)ws.st_meq.ptr;
        if ((st = ensure(ws.live_list, sizeof(unsigned) * batch)) != MF_OK) return st;
        if ((st = ensure(ws.live_count, sizeof(unsigned long long))) != MF_OK) return st;
        SP.live = (unsigned*)ws.live_list.ptr;
        SP.n_live = (unsigned long long*)ws.live_count.ptr;
        SP.first_batch = 1;
    }
    for (uint64_t first = 0; first < n; first += batch) {
        SP.first = first;
        SP.count = n - first < batch ? n - first : batch;
        SP.P.n_waves = waves_for((SP.count + mf::kWave - 1) / mf::kWave, S.ws->n_cu);
        const int kin_blocks = SP.P.n_waves / mf::kWavesPerBlock;
        if (S.ng == 5 && lc)
            st = opt->precision == MF_FP32_KAHAN
                     ? launch_stages_ng5<float, true>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false)
                     : launch_stages_ng5<double, true>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false);
        else if (S.ng == 5)
            st = opt->precision == MF_FP32_KAHAN
                     ? launch_stages_ng5<float>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false)
                     : launch_stages_ng5<double>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false);
        else if (S.ng == 3)
            st = opt->precision == MF_FP32_KAHAN
                     ? launch_stages<3, float, 0>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false)
                     : launch_stages<3, double, 0>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false);
        else if (S.ng == 4)
            st = opt->precision == MF_FP32_KAHAN
                     ? launch_stages<4, float, 0>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false)
                     : launch_stages<4, double, 0>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false);
        else
            st = opt->precision == MF_FP32_KAHAN
                     ? launch_stages<2, float, 0>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false)
                     : launch_stages<2, double, 0>(SP, kin_blocks, S.ws->n_cu, S.stream, nullptr, nullptr, false);
        if (st != MF_OK)
            return st;
    }
    return MF_OK;
}

}  // namespace

extern "C" {

mf_status mf_evaluate(const mf_process* proc, double sqrt_s, const mf_pdf_grid* pdf, const double* grid,
                      const double* y, const uint64_t* event_ids, uint64_t n, uint64_t seed, int iter,
                      const mf_options* opt, double* w_out, uint64_t* k53_out, int32_t* bins_out,
                      double* record_out)
{
    if (!w_out)
        return fail(MF_EINVAL, "w_out is NULL");
    if (opt && (opt->colour == MF_COLOUR_SAMPLED || opt->colour == MF_COLOUR_FLOW))
        return fail(MF_EUNSUPPORTED, "the Monte Carlo over colours runs in mf_integrate only");
    if (opt && opt->helicity == MF_HELICITY_SAMPLED && y)
        return fail(MF_EINVAL, "the Monte Carlo over helicities needs the events' Philox counters (y must be NULL)");
    std::unique_lock<std::mutex> lock;
    Setup S;
    mf_status st;
    if ((st = fixed_grid_setup(proc, sqrt_s, pdf, grid, n, seed, iter, opt, y, event_ids, lock, S)) != MF_OK)
        return st;
    mf::EventParams& P = S.P;
    P.weights = w_out;
    P.k53_out = k53_out;
    P.bins_out = bins_out;
    P.record = record_out;
    if (S.ng == 5 || is_pp(proc->id)) {
        if ((st = evaluate_staged(S, opt, n)) != MF_OK)
            return st;
        MF_HIP(hipStreamSynchronize(S.stream));
        return MF_OK;
    }
    if ((st = dispatch_event(S.ng, opt->precision, opt->colour, P, P.n_waves / mf::kWavesPerBlock, S.stream)) != MF_OK)
        return st;
    MF_HIP(hipStreamSynchronize(S.stream));
    return MF_OK;
}

mf_status mf_evaluate_grad(const mf_process* proc, double sqrt_s, const mf_pdf_grid* pdf, const double* grid,
                           const double* y, const uint64_t* event_ids, uint64_t n, uint64_t seed, int iter,
                           const mf_options* opt, double* w_out, double* dw_dy, double* dw_dmt)
{
    if (!w_out)
        return fail(MF_EINVAL, "w_out is NULL");
    if (proc && proc->id != MF_GG_TTX)
        return fail(MF_EUNSUPPORTED, "gradients are implemented for g g -> t tbar only");
    if (opt && opt->precision != MF_FP64)
        return fail(MF_EUNSUPPORTED, "gradients are computed in FP64 only");
    if (opt && opt->colour != MF_COLOUR_FULL)
        return fail(MF_EUNSUPPORTED, "gradients are computed with the full colour sum only");
    if (opt && opt->helicity != MF_HELICITY_SUM)
        return fail(MF_EUNSUPPORTED, "gradients are computed with the full helicity sum only");
    std::unique_lock<std::mutex> lock;
    Setup S;
    mf_status st;
    if ((st = fixed_grid_setup(proc, sqrt_s, pdf, grid, n, seed, iter, opt, y, event_ids, lock, S)) != MF_OK)
        return st;
    mf::GradParams G;
    G.P = S.P;
    G.alpha_s = proc->alpha_s;
    G.w_top = proc->w_top;
    G.dw_dy = dw_dy;
    G.dw_dmt = dw_dmt;
    G.w_out = w_out;
    G.partials = nullptr;
    hipLaunchKernelGGL(mf::grad_kernel_ttx, dim3(G.P.n_waves / mf::kWavesPerBlock), dim3(mf::kBlock), 0, S.stream, G);
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(S.stream));
    return MF_OK;
}

mf_status mf_refine_grid(int n_dims, int n_bins, double alpha, const double* hist, const double* grid_in,
                         double* grid_out, void* stream)
{
    if (n_dims < 1 || n_dims > mf::kMaxDims)
        return fail(MF_EINVAL, "n_dims must be in [1, 10]");
    if (n_bins < 2 || n_bins > 1024)
        return fail(MF_EINVAL, "n_bins must be in [2, 1024]");
    if (!finite_pos(alpha))
        return fail(MF_EINVAL, "alpha must be finite and > 0");
    if (!hist || !grid_in || !grid_out || grid_in == grid_out)
        return fail(MF_EINVAL, "hist, grid_in, grid_out must be distinct non-NULL device pointers");
    Workspace* wsp = nullptr;
    mf_status st;
    if ((st = device_workspace(&wsp)) != MF_OK) return st;
    Workspace& ws = *wsp;
    std::lock_guard<std::mutex> guard(ws.lock);
    if ((st = ensure(ws.entries, sizeof(double) * mf::kPartialHead)) != MF_OK) return st;
    if ((st = ensure(ws.iter_I, sizeof(double))) != MF_OK) return st;
    if ((st = ensure(ws.iter_V, sizeof(double))) != MF_OK) return st;
    if ((st = ensure(ws.stats, sizeof(double) * 4)) != MF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    MF_HIP(hipMemsetAsync(ws.entries.ptr, 0, sizeof(double) * mf::kPartialHead, s));
    mf::ReduceParams R;
    std::memset(&R, 0, sizeof(R));
    R.n_dims = n_dims;
    R.n_bins = n_bins;
    R.n_events = 2.0;
    R.alpha = alpha;
    R.grid_in = grid_in;
    R.grid_out = grid_out;
    R.entries = (double*)ws.entries.ptr;
    R.hist = hist;
    R.iter_I = (double*)ws.iter_I.ptr;
    R.iter_V = (double*)ws.iter_V.ptr;
    R.stats = (double*)ws.stats.ptr;
    R.j = 0;
    hipLaunchKernelGGL(mf::refine_kernel, dim3(1), dim3(256), 0, s, R);
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(s));
    return MF_OK;
}

mf_status mf_unweight(const mf_process* proc, double sqrt_s, const double* grid, const double* w, uint64_t n,
                      uint64_t seed, int iter, double w_max, const mf_options* opt, mf_events* out)
{
    int ng = 0;
    mf_status st;
    if (!out)
        return fail(MF_EINVAL, "out is NULL");
    if ((st = validate_process(proc, sqrt_s, &ng)) != MF_OK) return st;
    const int D = 2 + 3 * ng - 4;
    if ((st = validate_options(opt, D)) != MF_OK) return st;
    if (n > (1ull << 40))
        return fail(MF_EINVAL, "n must be at most 2^40");
    if (n > 0 && !w)
        return fail(MF_EINVAL, "w is NULL");
    if (iter < 0)
        return fail(MF_EINVAL, "iter must be >= 0");
    if (!finite_pos(w_max))
        return fail(MF_EINVAL, "w_max must be finite and > 0");
    if (out->capacity > 0 && !out->event)
        return fail(MF_EINVAL, "event is NULL while capacity > 0");
    const int nb = opt->n_bins;
    if (grid)
        for (int d = 0; d < D; ++d) {
            const double* e = grid + (size_t)d * (nb + 1);
            if (e[0] != 0.0 || e[nb] != 1.0 || !ascending(e, nb + 1))
                return fail(MF_EINVAL, "grid rows must rise strictly from 0 to 1");
        }
    if (n == 0) {
        out->n_kept = 0;
        out->n_over = 0;
        return MF_OK;
    }
    Workspace* wsp = nullptr;
    if ((st = device_workspace(&wsp)) != MF_OK) return st;
    Workspace& ws = *wsp;
    std::lock_guard<std::mutex> lock(ws.lock);
    hipStream_t stream = (hipStream_t)opt->stream;

    mf::UnweightParams U;
    std::memset(&U, 0, sizeof(U));
    mf::EventParams& P = U.P;
    P.n_g = ng;
    P.n_dims = D;
    P.n_bins = nb;
    P.max_newton = opt->max_newton;
    P.n_events = n;
    P.seed = seed;
    P.iter = (uint32_t)iter;
    P.sqrt_s = sqrt_s;
    P.s_had = sqrt_s * sqrt_s;
    P.m_top = proc->m_top;
    P.ps_const = std::pow(2.0 * mf::kPi, 4 - 3 * ng) * std::pow(mf::kPi / 2.0, ng - 1) /
                 (factorial(ng - 1) * factorial(ng - 2));
    const size_t grid_bytes = sizeof(double) * D * (size_t)(nb + 1);
    if ((st = ensure(ws.grid[0], grid_bytes)) != MF_OK) return st;
    std::vector<double> g((size_t)D * (nb + 1));
    if (grid)
        std::memcpy(g.data(), grid, grid_bytes);
    else
        for (int d = 0; d < D; ++d)
            for (int i = 0; i <= nb; ++i)
                g[(size_t)d * (nb + 1) + i] = (double)i / (double)nb;
    MF_HIP(hipMemcpyAsync(ws.grid[0].ptr, g.data(), grid_bytes, hipMemcpyHostToDevice, stream));
    P.grid = (const double*)ws.grid[0].ptr;

    // contiguous event ranges of whole write tiles, at most 2048 workgroups
    // (each write workgroup sums the counts of those before it)
    const uint64_t tile = mf::kUnweightTile;
    uint64_t per = (n + 2047) / 2048;
    per = (per + tile - 1) / tile * tile;
    const uint64_t n_blocks = (n + per - 1) / per;
    U.w = w;
    U.n = n;
    U.w_max = w_max;
    U.per_block = per;
    if ((st = ensure(ws.uw_counts, sizeof(uint64_t) * 2 * n_blocks)) != MF_OK) return st;
    if ((st = ensure(ws.uw_flags, (n + 15) / 16 * 16)) != MF_OK) return st;
    if ((st = ensure(ws.uw_totals, sizeof(uint64_t) * 2)) != MF_OK) return st;
    U.counts = (uint64_t*)ws.uw_counts.ptr;
    U.flags = (signed char*)ws.uw_flags.ptr;
    U.totals = (uint64_t*)ws.uw_totals.ptr;
    U.n_blocks = n_blocks;
    // profile: events around the count, write and record kernels
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    struct EventGuard {
        hipEvent_t* e;
        ~EventGuard() { for (int i = 0; i < 4; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    if (opt->profile)
        for (int i = 0; i < 4; ++i)
            MF_HIP(hipEventCreate(&ev[i]));
    for (int i = 0; i < 3; ++i)
        out->kernel_ms[i] = 0.0;
    if (opt->profile)
        MF_HIP(hipEventRecord(ev[0], stream));
    hipLaunchKernelGGL(mf::unweight_count_kernel, dim3((unsigned)n_blocks), dim3(mf::kBlock), 0, stream, U);
    MF_HIP(hipGetLastError());
    if (opt->profile)
        MF_HIP(hipEventRecord(ev[1], stream));
    U.capacity = out->capacity;
    U.ev_out = out->event;
    U.p_out = out->p;
    U.sign_out = out->sign;
    hipLaunchKernelGGL(mf::unweight_write_kernel, dim3((unsigned)n_blocks), dim3(mf::kBlock), 0, stream, U);
    MF_HIP(hipGetLastError());
    if (opt->profile)
        MF_HIP(hipEventRecord(ev[2], stream));
    const bool records = out->p && out->capacity > 0;
    if (records) {
        const uint64_t recs = out->capacity < n ? out->capacity : n;
        const uint64_t rb = (recs + mf::kBlock - 1) / mf::kBlock;
        const dim3 grid((unsigned)(rb < 65536 ? rb : 65536));
        const uint64_t* tot = (const uint64_t*)ws.uw_totals.ptr;
        switch (ng) {
        case 2: hipLaunchKernelGGL(mf::unweight_record_kernel<2>, grid, dim3(mf::kBlock), 0, stream, U, tot); break;
        case 3: hipLaunchKernelGGL(mf::unweight_record_kernel<3>, grid, dim3(mf::kBlock), 0, stream, U, tot); break;
        case 4: hipLaunchKernelGGL(mf::unweight_record_kernel<4>, grid, dim3(mf::kBlock), 0, stream, U, tot); break;
        default: hipLaunchKernelGGL(mf::unweight_record_kernel<5>, grid, dim3(mf::kBlock), 0, stream, U, tot); break;
        }
        MF_HIP(hipGetLastError());
    }
    if (opt->profile)
        MF_HIP(hipEventRecord(ev[3], stream));
    uint64_t totals[2] = {0, 0};
    MF_HIP(hipMemcpyAsync(totals, ws.uw_totals.ptr, sizeof(totals), hipMemcpyDeviceToHost, stream));
    MF_HIP(hipStreamSynchronize(stream));
    if (opt->profile) {
        float t = 0.f;
        MF_HIP(hipEventElapsedTime(&t, ev[0], ev[1]));
        out->kernel_ms[0] = t;
        MF_HIP(hipEventElapsedTime(&t, ev[1], ev[2]));
        out->kernel_ms[1] = t;
        if (records) {
            MF_HIP(hipEventElapsedTime(&t, ev[2], ev[3]));
            out->kernel_ms[2] = t;
        }
    }
    const uint64_t kept = totals[0], over = totals[1];
    out->n_kept = kept;
    out->n_over = over;
    return MF_OK;
}

mf_status mf_colour_matrix(int process_id, double* C)
{
    const int n = n_gluons(process_id);
    if (n < 0)
        return fail(MF_EINVAL, "unknown process id");
    if (!C)
        return fail(MF_EINVAL, "C is NULL");
    if (n == 5) {
        for (int i = 0; i < 120 * 120; ++i)
            C[i] = (double)mf::COLOUR_NUM_NG5[i] / mf::COLOUR_DEN_NG5;
        return MF_OK;
    }
    const int* num = n == 2 ? mf::COLOUR_NUM_NG2 : (n == 3 ? mf::COLOUR_NUM_NG3 : mf::COLOUR_NUM_NG4);
    const double den = n == 2 ? mf::COLOUR_DEN_NG2 : (n == 3 ? mf::COLOUR_DEN_NG3 : mf::COLOUR_DEN_NG4);
    const int np = n == 2 ? 2 : (n == 3 ? 6 : 24);
    for (int i = 0; i < np * np; ++i)
        C[i] = (double)num[i] / den;
    return MF_OK;
}

}  // extern "C"

namespace {

// mf_matrix_element for t tbar g g g: the amplitude and colour kernels of
// the staged path in batches, on the caller's momenta.
mf_status matrix_element_ng5(mf_precision precision, const double* mom, const double* eb, uint64_t n, double m_top,
                             double w_top, double* out, hipStream_t s)
{
    Workspace* wsp = nullptr;
    mf_status st;
    if ((st = device_workspace(&wsp)) != MF_OK) return st;
    Workspace& ws = *wsp;
    std::lock_guard<std::mutex> guard(ws.lock);
    const uint64_t batch = n < kStageBatchNg5 ? n : kStageBatchNg5;
    mf::StageParams SP;
    std::memset(&SP.P, 0, sizeof(SP.P));
    SP.P.m_top = m_top;
    SP.P.mw = m_top * w_top;
    if ((st = stage_buffers_ng5(ws, batch, precision, SP)) != MF_OK) return st;
    constexpr int K = mf::Layout<5>::kMom;
    for (uint64_t first = 0; first < n; first += batch) {
        SP.first = first;
        SP.count = n - first < batch ? n - first : batch;
        SP.me = out + first;
        const unsigned pb = (unsigned)((SP.count + mf::kBlock - 1) / mf::kBlock);
        hipLaunchKernelGGL(mf::me_prep_kernel_ng5, dim3(pb), dim3(mf::kBlock), 0, s, mom + first * (K - 1),
                           eb + first, SP.count, SP);
        MF_HIP(hipGetLastError());
        int per_cu = 0, col_per_cu = 0;
        const bool f32 = precision == MF_FP32_KAHAN;
        MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, f32 ? (const void*)mf::amp_kernel_ng5<float> : (const void*)mf::amp_kernel_ng5<double>,
            mf::kBlockNg5, 0));
        MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &col_per_cu, f32 ? (const void*)mf::colour_kernel_ng5<float> : (const void*)mf::colour_kernel_ng5<double>,
            mf::kBlock, 0));
        if (per_cu < 1)
            return fail(MF_EDEVICE, "the t tbar g g g amplitude kernel does not fit a compute unit");
        const uint64_t acap = (uint64_t)ws.n_cu * per_cu;
        const int agrid = (int)(SP.count < acap ? SP.count : acap);
        const uint64_t cneed = (SP.count + mf::kWavesPerBlock - 1) / mf::kWavesPerBlock;
        const uint64_t ccap = (uint64_t)ws.n_cu * (col_per_cu < 1 ? 1 : col_per_cu);
        const int cgrid = (int)(cneed < ccap ? cneed : ccap);
        if (f32) {
            hipLaunchKernelGGL((mf::amp_kernel_ng5<float>), dim3(agrid), dim3(mf::kBlockNg5), 0, s, SP);
            MF_HIP(hipGetLastError());
            hipLaunchKernelGGL((mf::colour_kernel_ng5<float>), dim3(cgrid), dim3(mf::kBlock), 0, s, SP);
        } else {
            hipLaunchKernelGGL((mf::amp_kernel_ng5<double>), dim3(agrid), dim3(mf::kBlockNg5), 0, s, SP);
            MF_HIP(hipGetLastError());
            hipLaunchKernelGGL((mf::colour_kernel_ng5<double>), dim3(cgrid), dim3(mf::kBlock), 0, s, SP);
        }
        MF_HIP(hipGetLastError());
    }
    MF_HIP(hipStreamSynchronize(s));
    return MF_OK;
}

}  // namespace

extern "C" {

mf_status mf_matrix_element(int process_id, mf_precision precision, const double* mom, const double* eb,
                            uint64_t n, double m_top, double w_top, double* out, void* stream)
{
    const int ng = n_gluons(process_id);
    if (ng < 0)
        return fail(MF_EINVAL, "unknown process id");
    if (precision != MF_FP64 && precision != MF_FP32_KAHAN)
        return fail(MF_EINVAL, "unknown precision");
    if (!mom || !eb || !out)
        return fail(MF_EINVAL, "mom, eb and out must be device pointers");
    if (n < 1 || n > (1ull << 40))
        return fail(MF_EINVAL, "n must be in [1, 2^40]");
    if (!finite_pos(m_top) || !std::isfinite(w_top) || w_top < 0.0)
        return fail(MF_EINVAL, "m_top must be > 0 and w_top >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (ng == 5)
        return matrix_element_ng5(precision, mom, eb, n, m_top, w_top, out, s);
    if (process_id == MF_PP_TTXGG) {
        // the q qbar channel (quark along +z), FP64, one wave per event
        if (n > 0x7FFFFFFFull)
            return fail(MF_EINVAL, "too many events for one launch");
        hipLaunchKernelGGL(mf::qqbar_ttxgg_me_kernel, dim3((unsigned)n), dim3(mf::kWave), 0, s, mom, eb, n, m_top,
                           m_top * w_top, out);
        MF_HIP(hipGetLastError());
        MF_HIP(hipStreamSynchronize(s));
        return MF_OK;
    }
    if (process_id == MF_PP_TTXG) {
        // the q qbar channel (quark along +z), FP64
        const uint64_t qb = (n * 16 + mf::kBlock - 1) / mf::kBlock;
        if (n > (1ull << 36) || qb > 0x7FFFFFFFull)
            return fail(MF_EINVAL, "too many events for one launch");
        hipLaunchKernelGGL(mf::qqbar_ttxg_me_kernel, dim3((unsigned)qb), dim3(mf::kBlock), 0, s, mom, eb, n, m_top,
                           m_top * w_top, out);
        MF_HIP(hipGetLastError());
        MF_HIP(hipStreamSynchronize(s));
        return MF_OK;
    }
    if (process_id == MF_PP_TTX) {
        // the q qbar channel (quark along +z), FP64
        const uint64_t qb = (n + mf::kBlock - 1) / mf::kBlock;
        if (qb > 0x7FFFFFFFull)
            return fail(MF_EINVAL, "too many events for one launch");
        hipLaunchKernelGGL(mf::qqbar_me_kernel, dim3((unsigned)qb), dim3(mf::kBlock), 0, s, mom, eb, n, m_top, out);
        MF_HIP(hipGetLastError());
        MF_HIP(hipStreamSynchronize(s));
        return MF_OK;
    }
    const int epp = mf::kWave >> (ng + 2);              // events per wave
    const uint64_t per_block = (uint64_t)epp * mf::kWavesPerBlock;
    const uint64_t blocks = (n + per_block - 1) / per_block;
    if (blocks > 0x7FFFFFFFull)
        return fail(MF_EINVAL, "too many events for one launch");
    const double mw = m_top * w_top;
    const bool f32 = precision == MF_FP32_KAHAN;
#define MF_ME_LAUNCH(NG)                                                                                   \
    if (f32)                                                                                               \
        hipLaunchKernelGGL((mf::me_kernel<NG, float>), dim3((unsigned)blocks), dim3(mf::kBlock), 0, s, mom, \
                           eb, n, m_top, mw, out);                                                         \
    else                                                                                                   \
        hipLaunchKernelGGL((mf::me_kernel<NG, double>), dim3((unsigned)blocks), dim3(mf::kBlock), 0, s,    \
                           mom, eb, n, m_top, mw, out);
    if (ng == 2) { MF_ME_LAUNCH(2) } else if (ng == 3) { MF_ME_LAUNCH(3) } else { MF_ME_LAUNCH(4) }
#undef MF_ME_LAUNCH
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(s));
    return MF_OK;
}

}  // extern "C"
