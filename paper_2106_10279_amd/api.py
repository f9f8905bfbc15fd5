"""Python API over the C ABI: torch tensors for device memory and streams.

    integrate(...)          VEGAS integration (mf_integrate)
    evaluate_weights(...)   per-event weights for a fixed grid (mf_evaluate)
    matrix_element(...)     colour/helicity-summed |M|^2 for given momenta
    refine_grid(...)        one VEGAS refinement step (mf_refine_grid)
    colour_matrix(...)      the process colour matrix
    integrate_grad(...)     integration plus d sigma/d m_t, d sigma/d alpha_s (mf_integrate_grad)
    evaluate_weights_grad(...)  per-event weights with dw/dy and dw/dm_t (mf_evaluate_grad)
    CrossSection            torch.autograd.Function: sigma(m_t, alpha_s)
    EventWeights            torch.autograd.Function: w(y, m_t) per event
    unweight(...)           hit-or-miss unweighting of an iteration's weights (mf_unweight)
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, replace

import numpy as np
import torch

from . import _lib
from ._lib import MF_FP32_KAHAN, MF_FP64, MFError, check, lib  # noqa: F401

PROCESS_IDS = {"gg_ttx": _lib.MF_GG_TTX, "gg_ttxg": _lib.MF_GG_TTXG, "gg_ttxgg": _lib.MF_GG_TTXGG,
               "gg_ttxggg": _lib.MF_GG_TTXGGG, "pp_ttx": _lib.MF_PP_TTX, "pp_ttxg": _lib.MF_PP_TTXG,
               "pp_ttxgg": _lib.MF_PP_TTXGG,
               2: _lib.MF_GG_TTX, 3: _lib.MF_GG_TTXG, 4: _lib.MF_GG_TTXGG, 5: _lib.MF_GG_TTXGGG}
PRECISIONS = {"fp64": MF_FP64, "fp32_kahan": MF_FP32_KAHAN}
# colour sum: the full colour matrix, the leading-colour approximation, or a
# Monte Carlo over colour assignments or colour flows (mf_integrate, n_g >= 3)
COLOURS = {"full": 0, "leading": 1, "sampled": 2, "flow": 3}
HELICITIES = {"sum": 0, "sampled": 1}

_dp = C.POINTER(C.c_double)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


@dataclass
class Process:
    process: str | int = "gg_ttx"
    m_top: float = 173.0
    w_top: float = 1.5
    alpha_s: float = 0.118
    mu_f: float = 173.0
    ptmin_g: float = 0.0
    etamax_g: float = 0.0
    drmin_gg: float = 0.0

    @property
    def id(self) -> int:
        return PROCESS_IDS[self.process]

    def c(self):
        return _lib.mf_process(self.id, self.m_top, self.w_top, self.alpha_s, self.mu_f,
                               self.ptmin_g, self.etamax_g, self.drmin_gg)


class _Pdf:
    def __init__(self, table):
        self.log_x = np.ascontiguousarray(table.log_x, dtype=np.float64)
        self.log_q2 = np.ascontiguousarray(table.log_q2, dtype=np.float64)
        self.xf = np.ascontiguousarray(table.xf, dtype=np.float64)
        xq = getattr(table, "xq", None)
        self.xq = None if xq is None else np.ascontiguousarray(xq, dtype=np.float64)
        self.c = _lib.mf_pdf_grid(len(self.log_x), len(self.log_q2), _ptr(self.log_x),
                                  _ptr(self.log_q2), _ptr(self.xf),
                                  _ptr(self.xq) if self.xq is not None else None)


def n_dims(process) -> int:
    return lib.mf_n_dims(PROCESS_IDS[process])


def _options(n_bins, alpha, start_iter, precision, strict, max_newton, grid_in, stream, profile=False,
             max_batch=0, colour="full", helicity="sum"):
    o = _lib.mf_options()
    lib.mf_default_options(C.byref(o))
    o.n_bins = n_bins
    o.alpha = alpha
    o.start_iter = start_iter
    o.precision = PRECISIONS.get(precision, precision)
    o.strict = int(strict)
    o.max_newton = max_newton
    o.grid_in = _ptr(grid_in) if grid_in is not None else None
    o.stream = _stream(stream)
    o.profile = int(profile)
    o.max_batch = int(max_batch)
    o.colour = COLOURS.get(colour, colour)
    o.helicity = HELICITIES.get(helicity, helicity)
    return o


@dataclass
class IntegrationResult:
    sigma: float
    sigma_err: float
    chi2_dof: float
    w_max: float
    n_pass: int
    n_newton_fail: int
    iter_sigma: np.ndarray
    iter_var: np.ndarray
    grid: np.ndarray
    hist: np.ndarray
    weights: torch.Tensor | None
    event_kernel_ms: float = 0.0
    reduce_kernel_ms: float = 0.0
    iter_pass: np.ndarray | None = None
    iter_event_ms: np.ndarray | None = None
    iter_amp_ms: np.ndarray | None = None
    n_batches: int = 1
    grid_last: np.ndarray | None = None
    iter_colour_ms: np.ndarray | None = None


def integrate(proc: Process, sqrt_s: float, pdf_table, n_events: int, n_iter: int, seed: int,
              n_bins: int = 50, alpha: float = 1.5, precision="fp64", start_iter: int = 0,
              grid_in=None, keep_weights: bool = True, strict: bool = False,
              max_newton: int = 50, stream=None, weights_out: torch.Tensor | None = None,
              profile: bool = False, max_batch: int = 0, colour="full", static_scratch: bool = False,
              helicity="sum"):
    """VEGAS integration (mf_integrate); static_scratch=True calls
    mf_integrate_static, which allocates no device memory."""
    D = n_dims(proc.process)
    pdf = _Pdf(pdf_table)
    gin = None if grid_in is None else np.ascontiguousarray(grid_in, dtype=np.float64)
    opt = _options(n_bins, alpha, start_iter, precision, strict, max_newton, gin, stream, profile,
                   max_batch, colour, helicity)
    I = np.zeros(n_iter)
    V = np.zeros(n_iter)
    grid = np.zeros((D, n_bins + 1))
    hist = np.zeros((D, n_bins))
    w = weights_out
    if w is None and keep_weights:
        w = torch.empty(n_events, dtype=torch.float64, device="cuda")
    res = _lib.mf_result()
    res.iter_sigma = _ptr(I)
    res.iter_var = _ptr(V)
    res.grid = _ptr(grid)
    res.hist = _ptr(hist)
    res.weights = C.cast(C.c_void_p(w.data_ptr()), _dp) if w is not None else None
    npass = np.zeros(n_iter)
    tms = np.zeros(n_iter)
    ams = np.zeros(n_iter)
    cms = np.zeros(n_iter)
    res.iter_pass = _ptr(npass)
    res.iter_event_ms = _ptr(tms)
    res.iter_amp_ms = _ptr(ams)
    res.iter_colour_ms = _ptr(cms)
    grid_last = np.zeros((D, n_bins + 1))
    res.grid_last = _ptr(grid_last)
    pc = proc.c()
    fn = lib.mf_integrate_static if static_scratch else lib.mf_integrate
    check(fn(C.byref(pc), sqrt_s, C.byref(pdf.c), n_events, n_iter, seed, C.byref(opt), C.byref(res)))
    return IntegrationResult(res.sigma, res.sigma_err, res.chi2_dof, res.w_max, res.n_pass,
                             res.n_newton_fail, I, V, grid, hist, w, res.event_kernel_ms,
                             res.reduce_kernel_ms, npass, tms if profile else None,
                             ams if profile else None, res.n_batches, grid_last,
                             cms if profile else None)


def evaluate_weights(proc: Process, sqrt_s: float, pdf_table, n: int, seed: int = 0, it: int = 0,
                     grid=None, y: torch.Tensor | None = None,
                     event_ids: torch.Tensor | None = None, n_bins: int = 50,
                     precision="fp64", max_newton: int = 50, return_k53: bool = False,
                     return_bins: bool = False, return_record: bool = False, stream=None,
                     colour="full", helicity="sum"):
    """Per-event weights (pb) for a fixed grid; optionally the Philox integers,
    the bin indices and the per-stage record (see mf_evaluate in include/mf.h)."""
    D = n_dims(proc.process)
    pdf = _Pdf(pdf_table)
    g = None if grid is None else np.ascontiguousarray(grid, dtype=np.float64)
    opt = _options(n_bins, 1.5, 0, precision, False, max_newton, None, stream, colour=colour,
                   helicity=helicity)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    k53 = torch.empty((n, D), dtype=torch.int64, device="cuda") if return_k53 else None
    bins = torch.empty((n, D), dtype=torch.int32, device="cuda") if return_bins else None
    n_f = {4: 2, 7: 3, 10: 4, 13: 5}[D]
    rec = torch.empty((n, 8 + 4 * n_f), dtype=torch.float64, device="cuda") if return_record else None
    if y is not None:
        assert y.dtype == torch.float64 and y.is_cuda and y.is_contiguous() and y.shape == (n, D)
    if event_ids is not None:
        assert event_ids.dtype == torch.int64 and event_ids.is_cuda and event_ids.shape == (n,)
    pc = proc.c()
    check(lib.mf_evaluate(C.byref(pc), sqrt_s, C.byref(pdf.c), _ptr(g) if g is not None else None,
                          C.c_void_p(y.data_ptr()) if y is not None else None,
                          C.c_void_p(event_ids.data_ptr()) if event_ids is not None else None,
                          n, seed, it, C.byref(opt), C.c_void_p(w.data_ptr()),
                          C.c_void_p(k53.data_ptr()) if k53 is not None else None,
                          C.c_void_p(bins.data_ptr()) if bins is not None else None,
                          C.c_void_p(rec.data_ptr()) if rec is not None else None))
    out = [w]
    if return_k53:
        out.append(k53)
    if return_bins:
        out.append(bins)
    if return_record:
        out.append(rec)
    return out[0] if len(out) == 1 else tuple(out)


def matrix_element(process, mom: torch.Tensor, eb: torch.Tensor, m_top=173.0, w_top=1.5,
                   precision="fp64", stream=None):
    """mom: [n, 4 n_f] (t, tbar, final gluons), eb: [n] beam energies; both float64 CUDA."""
    pid = PROCESS_IDS[process]
    assert mom.dtype == torch.float64 and mom.is_cuda and mom.is_contiguous()
    assert eb.dtype == torch.float64 and eb.is_cuda and eb.is_contiguous()
    n = eb.shape[0]
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    check(lib.mf_matrix_element(pid, PRECISIONS.get(precision, precision),
                                C.c_void_p(mom.data_ptr()), C.c_void_p(eb.data_ptr()), n, m_top,
                                w_top, C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def refine_grid(hist: torch.Tensor, grid: torch.Tensor, alpha: float = 1.5, stream=None):
    D, nb = hist.shape
    out = torch.empty_like(grid)
    check(lib.mf_refine_grid(D, nb, alpha, C.c_void_p(hist.data_ptr()),
                             C.c_void_p(grid.data_ptr()), C.c_void_p(out.data_ptr()),
                             _stream(stream)))
    return out


def colour_matrix(process) -> np.ndarray:
    pid = PROCESS_IDS[process]
    n = {0: 2, 1: 6, 2: 24, 3: 120, 4: 2, 5: 6, 6: 24}[pid]
    C_ = np.zeros((n, n))
    check(lib.mf_colour_matrix(pid, _ptr(C_)))
    return C_


@dataclass
class GradResult:
    dsigma_dmt: float
    dsigma_dalphas: float
    iter_dmt: np.ndarray
    iter_dalphas: np.ndarray
    dw_dy: torch.Tensor | None
    dw_dmt: torch.Tensor | None
    iter_grad_ms: np.ndarray | None = None


def integrate_grad(proc: Process, sqrt_s: float, pdf_table, n_events: int, n_iter: int, seed: int,
                   n_bins: int = 50, alpha: float = 1.5, start_iter: int = 0, grid_in=None,
                   keep_weights: bool = False, keep_event_grads: bool = False, max_newton: int = 50,
                   stream=None, profile: bool = False):
    """mf_integrate_grad: the integration of `integrate` (same grids and
    estimates) plus the gradient; g g -> t tbar, FP64 only."""
    D = n_dims(proc.process)
    pdf = _Pdf(pdf_table)
    gin = None if grid_in is None else np.ascontiguousarray(grid_in, dtype=np.float64)
    opt = _options(n_bins, alpha, start_iter, "fp64", False, max_newton, gin, stream, profile)
    I = np.zeros(n_iter)
    V = np.zeros(n_iter)
    grid = np.zeros((D, n_bins + 1))
    hist = np.zeros((D, n_bins))
    w = torch.empty(n_events, dtype=torch.float64, device="cuda") if keep_weights else None
    res = _lib.mf_result()
    res.iter_sigma = _ptr(I)
    res.iter_var = _ptr(V)
    res.grid = _ptr(grid)
    res.hist = _ptr(hist)
    res.weights = C.cast(C.c_void_p(w.data_ptr()), _dp) if w is not None else None
    gm = np.zeros(n_iter)
    ga = np.zeros(n_iter)
    dy = torch.empty((n_events, D), dtype=torch.float64, device="cuda") if keep_event_grads else None
    dm = torch.empty(n_events, dtype=torch.float64, device="cuda") if keep_event_grads else None
    g = _lib.mf_grad_result()
    g.iter_dmt = _ptr(gm)
    g.iter_dalphas = _ptr(ga)
    g.dw_dy = C.cast(C.c_void_p(dy.data_ptr()), _dp) if dy is not None else None
    g.dw_dmt = C.cast(C.c_void_p(dm.data_ptr()), _dp) if dm is not None else None
    gms = np.zeros(n_iter)
    g.iter_grad_ms = _ptr(gms)
    tms = np.zeros(n_iter)
    res.iter_event_ms = _ptr(tms)
    npass = np.zeros(n_iter)
    res.iter_pass = _ptr(npass)
    pc = proc.c()
    check(lib.mf_integrate_grad(C.byref(pc), sqrt_s, C.byref(pdf.c), n_events, n_iter, seed,
                                C.byref(opt), C.byref(res), C.byref(g)))
    r = IntegrationResult(res.sigma, res.sigma_err, res.chi2_dof, res.w_max, res.n_pass,
                          res.n_newton_fail, I, V, grid, hist, w, res.event_kernel_ms, res.reduce_kernel_ms,
                          npass, tms if profile else None)
    return r, GradResult(g.dsigma_dmt, g.dsigma_dalphas, gm, ga, dy, dm, gms if profile else None)


def evaluate_weights_grad(proc: Process, sqrt_s: float, pdf_table, n: int, seed: int = 0, it: int = 0,
                          grid=None, y: torch.Tensor | None = None,
                          event_ids: torch.Tensor | None = None, n_bins: int = 50,
                          max_newton: int = 50, stream=None):
    """mf_evaluate_grad: (w, dw/dy [n, D], dw/dm_t [n]) for a fixed grid."""
    D = n_dims(proc.process)
    pdf = _Pdf(pdf_table)
    g = None if grid is None else np.ascontiguousarray(grid, dtype=np.float64)
    opt = _options(n_bins, 1.5, 0, "fp64", False, max_newton, None, stream)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    dy = torch.empty((n, D), dtype=torch.float64, device="cuda")
    dm = torch.empty(n, dtype=torch.float64, device="cuda")
    if y is not None:
        assert y.dtype == torch.float64 and y.is_cuda and y.is_contiguous() and y.shape == (n, D)
    if event_ids is not None:
        assert event_ids.dtype == torch.int64 and event_ids.is_cuda and event_ids.shape == (n,)
    pc = proc.c()
    check(lib.mf_evaluate_grad(C.byref(pc), sqrt_s, C.byref(pdf.c), _ptr(g) if g is not None else None,
                               C.c_void_p(y.data_ptr()) if y is not None else None,
                               C.c_void_p(event_ids.data_ptr()) if event_ids is not None else None,
                               n, seed, it, C.byref(opt), C.c_void_p(w.data_ptr()),
                               C.c_void_p(dy.data_ptr()), C.c_void_p(dm.data_ptr())))
    return w, dy, dm


class CrossSection(torch.autograd.Function):
    """sigma(m_t, alpha_s) in pb for g g -> t tbar.  Forward runs mf_integrate;
    backward runs mf_integrate_grad with the same arguments, which replays the
    same iterations (and so the same grids) and returns the adjoint gradient."""

    @staticmethod
    def forward(ctx, m_t, alpha_s, proc, sqrt_s, pdf_table, n_events, n_iter, seed):
        p = replace(proc, m_top=float(m_t), alpha_s=float(alpha_s))
        r = integrate(p, sqrt_s, pdf_table, n_events, n_iter, seed, keep_weights=False)
        ctx.args = (p, sqrt_s, pdf_table, n_events, n_iter, seed)
        return torch.tensor(r.sigma, dtype=torch.float64, device=m_t.device)

    @staticmethod
    def backward(ctx, grad_out):
        p, sqrt_s, pdf_table, n_events, n_iter, seed = ctx.args
        _, g = integrate_grad(p, sqrt_s, pdf_table, n_events, n_iter, seed)
        go = grad_out.detach().to(torch.float64)
        return go * g.dsigma_dmt, go * g.dsigma_dalphas, None, None, None, None, None, None


class EventWeights(torch.autograd.Function):
    """Per-event weights w(y, m_t) of g g -> t tbar for uniforms y [n, 4]
    (float64, CUDA) on a fixed grid; backward gives dL/dy and dL/dm_t from
    mf_evaluate_grad."""

    @staticmethod
    def forward(ctx, y, m_t, proc, sqrt_s, pdf_table, grid):
        p = replace(proc, m_top=float(m_t))
        yc = y.detach().contiguous()
        w = evaluate_weights(p, sqrt_s, pdf_table, yc.shape[0], grid=grid, y=yc)
        ctx.args = (p, sqrt_s, pdf_table, grid)
        ctx.mt_device = m_t.device
        ctx.save_for_backward(yc)
        return w

    @staticmethod
    def backward(ctx, grad_w):
        (yc,) = ctx.saved_tensors
        p, sqrt_s, pdf_table, grid = ctx.args
        _, dy, dm = evaluate_weights_grad(p, sqrt_s, pdf_table, yc.shape[0], grid=grid, y=yc)
        g = grad_w.detach().to(torch.float64)
        return g[:, None] * dy, (g * dm).sum().to(ctx.mt_device), None, None, None, None


@dataclass
class UnweightedEvents:
    event: torch.Tensor        # int64 [n_kept] event indices, ascending
    p: torch.Tensor | None     # float64 [n_kept, n_f + 2, 4] lab-frame (E, px, py, pz): beams, t, tbar, gluons
    sign: torch.Tensor         # int8 [n_kept] sign of the kept weight
    n_kept: int
    n_over: int                # events with |w| > w_max
    kernel_ms: tuple | None = None   # profile=True: count, write, record kernel durations


def unweight(proc: Process, sqrt_s: float, weights: torch.Tensor, w_max: float, seed: int, it: int,
             grid=None, n_bins: int = 50, max_newton: int = 50, stream=None,
             momenta: bool = True, capacity: int | None = None, profile: bool = False) -> UnweightedEvents:
    """Hit-or-miss unweighting (mf_unweight): event e is kept when
    u_e w_max < |w_e| with u_e from Philox block 0x80000000 of its counter.
    `grid` is the grid the weights were computed on (IntegrationResult.grid_last)
    and `it` their Philox iteration index.  With capacity=None a counting
    call sizes the output first."""
    assert weights.is_cuda and weights.dtype == torch.float64 and weights.is_contiguous()
    n = weights.numel()
    n_f = n_dims(proc.process)
    n_f = {4: 2, 7: 3, 10: 4, 13: 5}[n_f]
    g = None if grid is None else np.ascontiguousarray(grid, dtype=np.float64)
    opt = _options(n_bins, 1.5, 0, "fp64", False, max_newton, None, stream, profile)
    pc = proc.c()
    wp = C.c_void_p(weights.data_ptr())
    if capacity is None:
        ev = _lib.mf_events()
        check(lib.mf_unweight(C.byref(pc), sqrt_s, _ptr(g) if g is not None else None, wp, n, seed, it,
                              w_max, C.byref(opt), C.byref(ev)))
        capacity = int(ev.n_kept)
    dev = weights.device
    event = torch.empty(capacity, dtype=torch.int64, device=dev)
    sign = torch.empty(capacity, dtype=torch.int8, device=dev)
    p = torch.empty((capacity, n_f + 2, 4), dtype=torch.float64, device=dev) if momenta else None
    ev = _lib.mf_events()
    ev.capacity = capacity
    ev.event = C.c_void_p(event.data_ptr()) if capacity else None
    ev.sign = C.c_void_p(sign.data_ptr()) if capacity else None
    ev.p = C.c_void_p(p.data_ptr()) if (p is not None and capacity) else None
    check(lib.mf_unweight(C.byref(pc), sqrt_s, _ptr(g) if g is not None else None, wp, n, seed, it,
                          w_max, C.byref(opt), C.byref(ev)))
    k = min(capacity, int(ev.n_kept))
    return UnweightedEvents(event[:k], p[:k] if p is not None else None, sign[:k], int(ev.n_kept),
                            int(ev.n_over), tuple(ev.kernel_ms) if profile else None)
