"""ctypes binding of oracle/libmfo.so (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MFO_LIB names another build of the same sources (the reference writer's
# contracted build, libmfo_fma.so); it is loaded as it is, without building.
_LIB_PATH = os.environ.get("MFO_LIB") or os.path.join(_HERE, "libmfo.so")
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_u32p = C.POINTER(C.c_uint32)
_u64p = C.POINTER(C.c_uint64)


class _Process(C.Structure):
    _fields_ = [("n_g", C.c_int), ("m_top", C.c_double), ("w_top", C.c_double),
                ("alpha_s", C.c_double), ("mu_f", C.c_double), ("ptmin_g", C.c_double),
                ("etamax_g", C.c_double), ("drmin_gg", C.c_double), ("colour", C.c_int),
                ("helicity", C.c_int), ("initial", C.c_int)]


class _Pdf(C.Structure):
    _fields_ = [("n_x", C.c_int), ("n_q2", C.c_int), ("log_x", _dp), ("log_q2", _dp),
                ("xf", _dp), ("xq", _dp)]


class _Event(C.Structure):
    _fields_ = [("y", C.c_double * 13), ("bin", C.c_int * 13), ("x", C.c_double * 13),
                ("jac", C.c_double), ("x1", C.c_double), ("x2", C.c_double),
                ("shat", C.c_double), ("ps_weight", C.c_double), ("f1", C.c_double),
                ("f2", C.c_double), ("me2", C.c_double), ("w", C.c_double),
                ("k", C.c_double * 20), ("pass_threshold", C.c_int), ("pass_cuts", C.c_int),
                ("newton_fail", C.c_int), ("near_edge", C.c_int), ("ill_conditioned", C.c_int),
                ("colour_cfg", C.c_int64), ("colour_kappa", C.c_double), ("hel_cfg", C.c_int),
                ("me2_q", C.c_double * 2), ("lum_q", C.c_double * 2), ("newton_kappa", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("sigma", C.c_double), ("sigma_err", C.c_double), ("chi2_dof", C.c_double),
                ("w_max", C.c_double), ("n_pass", C.c_int64), ("n_newton_fail", C.c_int64),
                ("n_near_edge", C.c_int64)]


def build(force: bool = False) -> str:
    """Compile libmfo.so with the oracle's Makefile (plain gcc).  An exclusive
    lock on a file beside it keeps concurrent test processes from building
    (and loading a half-written library) at the same time."""
    import fcntl
    if os.environ.get("MFO_LIB"):
        return _LIB_PATH
    with open(os.path.join(_HERE, ".build.lock"), "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        if force or not os.path.exists(_LIB_PATH) or _stale():
            subprocess.run(["make", "-C", _HERE, "-B" if force else "-s", "libmfo.so"],
                           check=True, capture_output=True)
    return _LIB_PATH


def _stale() -> bool:
    t = os.path.getmtime(_LIB_PATH)
    for f in os.listdir(_HERE):
        if f.endswith((".c", ".h")) and os.path.getmtime(os.path.join(_HERE, f)) > t:
            return True
    return False


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        L.mfo_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.mfo_event_k53.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, _u64p]
        L.mfo_bin_from_k53.argtypes = [C.c_uint64, C.c_int, _ip, _dp]
        L.mfo_vegas_map.argtypes = [C.c_int, C.c_int, _dp, _ip, _dp, _dp]
        L.mfo_vegas_map.restype = C.c_double
        L.mfo_vegas_refine.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp, _dp]
        L.mfo_massless_volume.argtypes = [C.c_int, C.c_double]
        L.mfo_massless_volume.restype = C.c_double
        L.mfo_phase_space.argtypes = [C.c_int, _dp, C.c_double, _dp, C.c_int, _dp, _dp]
        L.mfo_phase_space.restype = C.c_int
        L.mfo_cuts.argtypes = [C.POINTER(_Process), C.c_int, _dp, C.c_double, _ip]
        L.mfo_cuts.restype = C.c_int
        L.mfo_pdf_xf.argtypes = [C.POINTER(_Pdf), C.c_double, C.c_double]
        L.mfo_pdf_xq.argtypes = [C.POINTER(_Pdf), C.c_int, C.c_double, C.c_double]
        L.mfo_pdf_xq.restype = C.c_double
        L.mfo_me2_qqbar_ttx.argtypes = [_dp, C.c_double]
        L.mfo_me2_qqbar_ttx.restype = C.c_double
        L.mfo_qqbar_ttxg_diagrams.argtypes = [_dp, C.c_double, C.c_double, _ip, C.c_int, _dp]
        L.mfo_qqbar_ttxg_diagrams.restype = None
        L.mfo_qqbar_ttxg_colour.argtypes = [_ip, _dp]
        L.mfo_qqbar_ttxg_colour.restype = None
        L.mfo_me2_qqbar_ttxg.argtypes = [_dp, C.c_double, C.c_double]
        L.mfo_me2_qqbar_ttxg.restype = C.c_double
        L.mfo_qqbar_ttxgg_terms.argtypes = [_dp, C.c_double, C.c_double, _ip, C.c_int, _dp]
        L.mfo_qqbar_ttxgg_terms.restype = None
        L.mfo_qqbar_ttxgg_colour.argtypes = [_ip, _dp]
        L.mfo_qqbar_ttxgg_colour.restype = None
        L.mfo_qqbar_ttxgg_colour_matrix.argtypes = [_dp]
        L.mfo_qqbar_ttxgg_colour_matrix.restype = None
        L.mfo_me2_qqbar_ttxgg.argtypes = [_dp, C.c_double, C.c_double]
        L.mfo_me2_qqbar_ttxgg.restype = C.c_double
        L.mfo_pdf_xf.restype = C.c_double
        L.mfo_n_orderings.argtypes = [C.c_int]
        L.mfo_n_orderings.restype = C.c_int
        L.mfo_orderings.argtypes = [C.c_int, _ip]
        L.mfo_colour_matrix.argtypes = [C.c_int, _dp]
        L.mfo_colour_matrix_relabel.argtypes = [C.c_int, _dp]
        L.mfo_partial_amplitudes.argtypes = [C.c_int, _dp, C.c_double, C.c_double, _ip,
                                             C.c_int, _dp]
        L.mfo_me2_sum.argtypes = [C.c_int, _dp, C.c_double, C.c_double]
        L.mfo_me2_sum.restype = C.c_double
        L.mfo_me2_sum_hel.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int, _ip]
        L.mfo_me2_sum_hel.restype = C.c_double
        L.mfo_colour_lc.argtypes = [C.c_int]
        L.mfo_colour_lc.restype = C.c_double
        L.mfo_me2_sum_lc.argtypes = [C.c_int, _dp, C.c_double, C.c_double]
        L.mfo_me2_sum_lc.restype = C.c_double
        L.mfo_colour_count.argtypes = [C.c_int]
        L.mfo_colour_count.restype = C.c_int64
        L.mfo_colour_config.argtypes = [C.c_int, C.c_uint64, C.c_uint32, C.c_uint64]
        L.mfo_colour_config.restype = C.c_int64
        L.mfo_colour_factors.argtypes = [C.c_int, C.c_int64, _dp]
        L.mfo_me2_sum_colour_config.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int64]
        L.mfo_me2_sum_colour_config.restype = C.c_double
        L.mfo_flow_count.argtypes = [C.c_int]
        L.mfo_flow_count.restype = C.c_int64
        L.mfo_flow_code.argtypes = [C.c_int, C.c_int64]
        L.mfo_flow_code.restype = C.c_int64
        L.mfo_flow_weight.argtypes = [C.c_int, C.c_int64]
        L.mfo_flow_weight.restype = C.c_int64
        L.mfo_flow_total.argtypes = [C.c_int]
        L.mfo_flow_total.restype = C.c_int64
        L.mfo_flow_config.argtypes = [C.c_int, C.c_uint64, C.c_uint32, C.c_uint64]
        L.mfo_flow_config.restype = C.c_int64
        L.mfo_flow_factors.argtypes = [C.c_int, C.c_int64, _dp]
        L.mfo_me2_sum_colour_flow.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int64]
        L.mfo_me2_sum_colour_flow.restype = C.c_double
        L.mfo_me2_sum_sampled.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int, C.c_int64,
                                          C.POINTER(C.c_double)]
        L.mfo_me2_sum_sampled.restype = C.c_double
        L.mfo_me2_sum_fullcolour.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int, _ip]
        L.mfo_me2_sum_fullcolour.restype = C.c_double
        L.mfo_dressed_amplitude.argtypes = [C.c_int, _dp, C.c_double, C.c_double, _ip, _ip, _dp]
        L.mfo_n_dims.argtypes = [C.c_int]
        L.mfo_n_dims.restype = C.c_int
        L.mfo_event_weight.argtypes = [C.POINTER(_Process), C.c_double, C.POINTER(_Pdf),
                                       C.c_int, _dp, C.c_uint64, C.c_int, C.c_uint64,
                                       C.POINTER(_Event)]
        L.mfo_event_weight.restype = C.c_double
        L.mfo_event_weight_y.argtypes = [C.POINTER(_Process), C.c_double, C.POINTER(_Pdf),
                                         C.c_int, _dp, _dp, C.POINTER(_Event)]
        L.mfo_event_weight_y.restype = C.c_double
        L.mfo_integrate.argtypes = [C.POINTER(_Process), C.c_double, C.POINTER(_Pdf),
                                    C.c_uint64, C.c_int, C.c_uint64, C.c_int, C.c_int,
                                    C.c_double, C.c_int, _dp, _dp, _dp, _dp, _dp,
                                    C.POINTER(_Result)]
        L.mfo_integrate.restype = C.c_int
        L.mfo_combine.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.mfo_neumaier_sum.argtypes = [C.c_int, _dp]
        L.mfo_neumaier_sum.restype = C.c_double
        L.mfo_ttx_dweight_dmt_analytic.argtypes = [C.POINTER(_Process), C.c_double,
                                                   C.POINTER(_Pdf), C.c_int, _dp, _dp, _dp]
        L.mfo_ttx_dweight_dmt_analytic.restype = C.c_double
        L.mfo_unweight_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
        L.mfo_unweight_uniform.restype = C.c_double
        L.mfo_unweight.argtypes = [C.c_uint64, _dp, C.c_double, C.c_uint64, C.c_uint32,
                                   C.POINTER(C.c_byte), _u64p]
        L.mfo_unweight.restype = C.c_uint64
        L.mfo_lab_event.argtypes = [C.POINTER(_Process), C.c_double, C.c_int, _dp, C.c_uint64,
                                    C.c_int, C.c_uint64, _dp]
        L.mfo_lab_event.restype = C.c_int
        L.mfo_hel_count.argtypes = [C.c_int]
        L.mfo_hel_count.restype = C.c_int
        L.mfo_hel_config.argtypes = [C.c_int, C.c_uint64, C.c_uint32, C.c_uint64]
        L.mfo_hel_config.restype = C.c_int
        L.mfo_me2_hel.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int, C.c_int64, C.c_int, _dp]
        L.mfo_me2_hel.restype = C.c_double
        L.mfo_event_weights.argtypes = [C.POINTER(_Process), C.c_double, C.POINTER(_Pdf), C.c_int, _dp,
                                        C.c_uint64, C.c_int, C.c_uint64, _u64p, C.c_int, _dp, _ip,
                                        _dp]
        L.mfo_event_weights.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Process:
    n_g: int
    m_top: float = 173.0
    w_top: float = 1.5
    alpha_s: float = 0.118
    mu_f: float = 173.0
    ptmin_g: float = 0.0
    etamax_g: float = 0.0
    drmin_gg: float = 0.0
    colour: str = "full"        # "full", "leading" (leading colour), "sampled" (colour Monte Carlo
                                # over adjoint indices) or "flow" (Monte Carlo over colour flows)
    helicity: str = "sum"       # "sum" or "sampled" (Monte Carlo over helicity configurations)
    initial: str = "gg"         # "gg" or "pp" (g g plus the q qbar channels from the quark tables)

    def c(self):
        modes = {"full": 0, "leading": 1, "sampled": 2, "flow": 3}
        if self.colour not in modes:
            raise ValueError(f"colour must be one of {sorted(modes)}, not {self.colour!r}")
        hmodes = {"sum": 0, "sampled": 1}
        if self.helicity not in hmodes:
            raise ValueError(f"helicity must be one of {sorted(hmodes)}, not {self.helicity!r}")
        imodes = {"gg": 0, "pp": 1}
        if self.initial not in imodes:
            raise ValueError(f"initial must be one of {sorted(imodes)}, not {self.initial!r}")
        if self.initial == "pp" and self.n_g not in (2, 3, 4):
            raise ValueError("the q qbar channels are in the oracle for p p -> t tbar, t tbar g, t tbar g g only")
        return _Process(self.n_g, self.m_top, self.w_top, self.alpha_s, self.mu_f,
                        self.ptmin_g, self.etamax_g, self.drmin_gg, modes[self.colour],
                        hmodes[self.helicity], imodes[self.initial])


class _PdfHandle:
    """Keeps the numpy buffers alive while the C struct points into them."""

    def __init__(self, table):
        self.log_x = _f64(table.log_x)
        self.log_q2 = _f64(table.log_q2)
        self.xf = _f64(table.xf)
        xq = getattr(table, "xq", None)
        self.xq = None if xq is None else _f64(xq)
        self.c = _Pdf(len(self.log_x), len(self.log_q2), _d(self.log_x), _d(self.log_q2),
                      _d(self.xf), _d(self.xq) if self.xq is not None else None)


@dataclass
class EventInfo:
    y: np.ndarray
    bins: np.ndarray
    x: np.ndarray
    jac: float
    shat: float
    ps_weight: float
    f1: float
    f2: float
    me2: float
    w: float
    k: np.ndarray
    pass_threshold: bool
    pass_cuts: bool
    newton_fail: bool
    near_edge: bool
    ill_conditioned: bool
    colour_kappa: float = 0.0
    newton_kappa: float = 0.0
    me2_q: tuple = (0.0, 0.0)
    lum_q: tuple = (0.0, 0.0)


def _event_info(ev, D):
    return EventInfo(np.array(ev.y[:D]), np.array(ev.bin[:D]), np.array(ev.x[:D]), ev.jac,
                     ev.shat, ev.ps_weight, ev.f1, ev.f2, ev.me2, ev.w,
                     np.array(ev.k[:]).reshape(5, 4)[:(D + 2) // 3], bool(ev.pass_threshold),
                     bool(ev.pass_cuts), bool(ev.newton_fail), bool(ev.near_edge),
                     bool(ev.ill_conditioned), ev.colour_kappa, ev.newton_kappa,
                     (ev.me2_q[0], ev.me2_q[1]), (ev.lum_q[0], ev.lum_q[1]))


def n_dims(n_g: int) -> int:
    return lib().mfo_n_dims(n_g)


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().mfo_philox4x32_10(c, k, o)
    return list(o)


def event_k53(seed: int, it: int, event: int, D: int) -> np.ndarray:
    out = (C.c_uint64 * D)()
    lib().mfo_event_k53(seed, it, event, D, out)
    return np.array(out[:], dtype=np.uint64)


def bin_from_k53(k: int, n_bins: int):
    b = C.c_int()
    dl = C.c_double()
    lib().mfo_bin_from_k53(int(k), n_bins, C.byref(b), C.byref(dl))
    return b.value, dl.value


def vegas_map(grid, bins, deltas):
    grid = _f64(grid)
    D, nb1 = grid.shape
    b = np.ascontiguousarray(bins, dtype=np.int32)
    dl = _f64(deltas)
    x = np.zeros(D)
    jac = lib().mfo_vegas_map(D, nb1 - 1, _d(grid), b.ctypes.data_as(_ip), _d(dl), _d(x))
    return x, jac


def vegas_refine(hist, grid, alpha=1.5):
    grid = _f64(grid)
    hist = _f64(hist)
    D, nb1 = grid.shape
    out = np.zeros_like(grid)
    lib().mfo_vegas_refine(D, nb1 - 1, alpha, _d(hist), _d(grid), _d(out))
    return out


def massless_volume(n_f: int, shat: float) -> float:
    return lib().mfo_massless_volume(n_f, shat)


def phase_space(n_f, masses, sqrt_shat, r, max_newton=50):
    m = _f64(masses)
    r = _f64(r)
    k = np.zeros((n_f, 4))
    w = C.c_double()
    st = lib().mfo_phase_space(n_f, _d(m), sqrt_shat, _d(r), max_newton, _d(k), C.byref(w))
    return k, w.value, st


def cuts(proc: Process, k, y_boost):
    """Fiducial cuts on the final-state gluons of momenta k [n_f][4] (partonic CM
    frame, slots t, tbar, gluons); returns (passed, near_edge)."""
    k = _f64(k)
    near = C.c_int()
    pc = proc.c()
    ok = lib().mfo_cuts(C.byref(pc), k.shape[0], _d(k), y_boost, C.byref(near))
    return bool(ok), bool(near.value)


def pdf_xf(table, x, q2):
    h = _PdfHandle(table)
    return lib().mfo_pdf_xf(C.byref(h.c), x, q2)


def pdf_xq(table, flavour, x, q2):
    """x q(x, Q^2) of quark table `flavour` (0 u, 1 ubar, 2 d, 3 dbar)."""
    h = _PdfHandle(table)
    return lib().mfo_pdf_xq(C.byref(h.c), flavour, x, q2)


def me2_qqbar_ttx(p, m):
    """q qbar -> t tbar |M|^2 summed over helicities and colours (g = 1);
    p: [4][4] all outgoing: t, tbar, -p_q, -p_qbar."""
    return lib().mfo_me2_qqbar_ttx(_d(_f64(p)), m)


def qqbar_ttxg_diagrams(p, m, width, hel, ward=False):
    """The five colour-stripped diagram amplitudes of q qbar -> t tbar g
    (complex [5]); p: [5][4] all outgoing: t, tbar, -p_q, -p_qbar, g;
    hel: (quark, antiquark, top, antitop spin, gluon helicity)."""
    out = np.zeros(10)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    lib().mfo_qqbar_ttxg_diagrams(_d(_f64(p)), m, width, h.ctypes.data_as(_ip), int(bool(ward)), _d(out))
    return out[0::2] + 1j * out[1::2]


def qqbar_ttxg_colour(cols):
    """Colour factors (complex [5]) of the diagrams for cols = (i_q, j_qbar,
    k_t, l_tbar, a_g)."""
    out = np.zeros(10)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    lib().mfo_qqbar_ttxg_colour(c.ctypes.data_as(_ip), _d(out))
    return out[0::2] + 1j * out[1::2]


def me2_qqbar_ttxg(p, m, width):
    """q qbar -> t tbar g |M|^2 summed over helicities and colours (g = 1)."""
    return lib().mfo_me2_qqbar_ttxg(_d(_f64(p)), m, width)


def qqbar_ttxgg_terms(p, m, width, hel, ward=0):
    """The 38 Lorentz terms (complex) of q qbar -> t tbar g g for helicities
    hel = (quark, antiquark, top, antitop spin, gluon 1, gluon 2); ward = 1
    or 2 replaces that gluon's polarisation by its momentum.  p: [6][4] all
    outgoing: t, tbar, -p_q, -p_qbar, g1, g2."""
    out = np.zeros(76)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    lib().mfo_qqbar_ttxgg_terms(_d(_f64(p)), m, width, h.ctypes.data_as(_ip), int(ward), _d(out))
    return out[0::2] + 1j * out[1::2]


def qqbar_ttxgg_colour(cols):
    """Colour factors (complex [38]) for cols = (i_q, j_qbar, k_t, l_tbar, a1, a2)."""
    out = np.zeros(76)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    lib().mfo_qqbar_ttxgg_colour(c.ctypes.data_as(_ip), _d(out))
    return out[0::2] + 1j * out[1::2]


def qqbar_ttxgg_colour_matrix():
    out = np.zeros(38 * 38 * 2)
    lib().mfo_qqbar_ttxgg_colour_matrix(_d(out))
    return (out[0::2] + 1j * out[1::2]).reshape(38, 38)


def me2_qqbar_ttxgg(p, m, width):
    """q qbar -> t tbar g g |M|^2 summed over helicities and colours (g = 1)."""
    return lib().mfo_me2_qqbar_ttxgg(_d(_f64(p)), m, width)


def colour_matrix(n_g):
    n = lib().mfo_n_orderings(n_g)
    out = np.zeros((n, n))
    lib().mfo_colour_matrix(n_g, _d(out))
    return out


def orderings(n_g):
    n = lib().mfo_n_orderings(n_g)
    out = np.zeros((n, n_g), dtype=np.int32)
    lib().mfo_orderings(n_g, out.ctypes.data_as(_ip))
    return out


def partial_amplitudes(n_g, p, m, width, hel, ward_gluon=-1):
    p = _f64(p)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    n = lib().mfo_n_orderings(n_g)
    out = np.zeros(2 * n)
    lib().mfo_partial_amplitudes(n_g, _d(p), m, width, h.ctypes.data_as(_ip), ward_gluon,
                                 _d(out))
    return out[0::2] + 1j * out[1::2]


def me2_sum(n_g, p, m, width):
    p = _f64(p)
    return lib().mfo_me2_sum(n_g, _d(p), m, width)


def colour_lc(n_g):
    """Leading-colour coefficient (N^2 - 1) N^(n_g - 1) / 2^n_g, N = 3."""
    return lib().mfo_colour_lc(n_g)


def me2_sum_lc(n_g, p, m, width):
    """Helicity sum of c_LC sum_sigma |A(sigma)|^2 (leading colour), g_s = 1."""
    p = _f64(p)
    return lib().mfo_me2_sum_lc(n_g, _d(p), m, width)


def colour_count(n_g):
    """Number of colour assignments 9 * 8^n_g sampled by the colour Monte Carlo."""
    return lib().mfo_colour_count(n_g)


def colour_config(n_g, seed, it, event):
    """The colour assignment of an event (Philox block 0x80000001)."""
    return lib().mfo_colour_config(n_g, seed, it, event)


def colour_factors(n_g, cfg):
    """(T^{a_sigma1} ... T^{a_sigman})_{ij} for every ordering, assignment cfg."""
    n = lib().mfo_n_orderings(n_g)
    out = np.zeros(2 * n)
    lib().mfo_colour_factors(n_g, cfg, _d(out))
    return out[0::2] + 1j * out[1::2]


def me2_sum_colour_config(n_g, p, m, width, cfg):
    """N_cfg times the helicity sum of |M|^2 for colour assignment cfg, g_s = 1."""
    p = _f64(p)
    return lib().mfo_me2_sum_colour_config(n_g, _d(p), m, width, cfg)


def flow_count(n_g):
    """Number of colour flows with a non-vanishing factor for some ordering."""
    return lib().mfo_flow_count(n_g)


def flow_code(n_g, idx):
    """code = j + 3 i + 9 sum_g 9^g (3 a_g + b_g) of flow idx (-1 out of range)."""
    return lib().mfo_flow_code(n_g, idx)


def flow_weight(n_g, idx):
    """Integer sampling weight W = 2^n 9^n sum_sigma c_sigma^2 of flow idx."""
    return lib().mfo_flow_weight(n_g, idx)


def flow_total(n_g):
    """T = sum of the flow weights."""
    return lib().mfo_flow_total(n_g)


def flow_config(n_g, seed, it, event):
    """The colour-flow index of an event (Philox block 0x80000001)."""
    return lib().mfo_flow_config(n_g, seed, it, event)


def flow_factors(n_g, idx):
    """(G_{sigma1} ... G_{sigman})_{ij} for every ordering, flow idx (real)."""
    out = np.zeros(lib().mfo_n_orderings(n_g))
    lib().mfo_flow_factors(n_g, idx, _d(out))
    return out


def me2_sum_sampled(n_g, p, m, width, mode, cfg):
    """(sampled colour sum, condition number) for mode 2 (adjoint assignment
    cfg) or 3 (flow index cfg), g_s = 1."""
    p = _f64(p)
    k = C.c_double()
    v = lib().mfo_me2_sum_sampled(n_g, _d(p), m, width, mode, cfg, C.byref(k))
    return v, k.value


def me2_sum_colour_flow(n_g, p, m, width, idx):
    """T / W_idx times the helicity sum of |M|^2 for colour flow idx, g_s = 1."""
    p = _f64(p)
    return lib().mfo_me2_sum_colour_flow(n_g, _d(p), m, width, idx)


def all_helicities(n_g):
    nh = 1 << (n_g + 2)
    return np.array([[(h >> i) & 1 for i in range(n_g + 2)] for h in range(nh)], dtype=np.int32)


def me2_sum_hel(n_g, p, m, width, hels):
    p = _f64(p)
    h = np.ascontiguousarray(hels, dtype=np.int32)
    return lib().mfo_me2_sum_hel(n_g, _d(p), m, width, len(h), h.ctypes.data_as(_ip))


def colour_matrix_relabel(n_g):
    """The colour matrix from its first row (brute force over the 8^n_g
    assignments) and the relabelling symmetry of the sum over adjoint indices."""
    n = lib().mfo_n_orderings(n_g)
    out = np.zeros((n, n))
    lib().mfo_colour_matrix_relabel(n_g, _d(out))
    return out


def dressed_amplitude(n_g, p, m, width, hel, cols):
    """[3][3] colour-dressed amplitude M_ij (Feynman rules, explicit SU(3)
    indices) for gluon adjoint indices cols and helicity configuration hel."""
    p = _f64(p)
    h = np.ascontiguousarray(hel, dtype=np.int32)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    out = np.zeros(18)
    lib().mfo_dressed_amplitude(n_g, _d(p), m, width, h.ctypes.data_as(_ip), c.ctypes.data_as(_ip), _d(out))
    return (out[0::2] + 1j * out[1::2]).reshape(3, 3)


def me2_sum_fullcolour(n_g, p, m, width, hels):
    p = _f64(p)
    h = np.ascontiguousarray(hels, dtype=np.int32)
    return lib().mfo_me2_sum_fullcolour(n_g, _d(p), m, width, len(h), h.ctypes.data_as(_ip))


def event_weight(proc: Process, sqrt_s, table, grid, seed, it, event):
    h = _PdfHandle(table)
    grid = _f64(grid)
    ev = _Event()
    pc = proc.c()
    w = lib().mfo_event_weight(C.byref(pc), sqrt_s, C.byref(h.c), grid.shape[1] - 1,
                               _d(grid), seed, it, event, C.byref(ev))
    return w, _event_info(ev, grid.shape[0])


def event_weight_y(proc: Process, sqrt_s, table, grid, y):
    h = _PdfHandle(table)
    grid = _f64(grid)
    y = _f64(y)
    ev = _Event()
    pc = proc.c()
    w = lib().mfo_event_weight_y(C.byref(pc), sqrt_s, C.byref(h.c), grid.shape[1] - 1,
                                 _d(grid), _d(y), C.byref(ev))
    return w, _event_info(ev, grid.shape[0])


@dataclass
class IntegrationResult:
    sigma: float
    sigma_err: float
    chi2_dof: float
    w_max: float
    n_pass: int
    n_newton_fail: int
    n_near_edge: int
    iter_sigma: np.ndarray
    iter_var: np.ndarray
    grid: np.ndarray
    hist_last: np.ndarray
    weights_last: np.ndarray | None


def integrate(proc: Process, sqrt_s, table, n_events, n_iter, seed, n_bins=50, alpha=1.5,
              n_threads=None, grid=None, start_iter=0, keep_weights=True):
    D = n_dims(proc.n_g)
    if grid is None:
        grid = np.tile(np.arange(n_bins + 1) / n_bins, (D, 1))
    grid = np.array(grid, dtype=np.float64, copy=True, order="C")
    if n_threads is None:
        n_threads = max(1, min(os.cpu_count() or 1, 16))
    h = _PdfHandle(table)
    I = np.zeros(n_iter)
    V = np.zeros(n_iter)
    hist = np.zeros((D, n_bins))
    w = np.zeros(n_events) if keep_weights else None
    res = _Result()
    pc = proc.c()
    st = lib().mfo_integrate(C.byref(pc), sqrt_s, C.byref(h.c), n_events, n_iter, seed,
                             start_iter, n_bins, alpha, n_threads, _d(grid), _d(I), _d(V),
                             _d(hist), _d(w) if w is not None else None, C.byref(res))
    if st != 0:
        raise ValueError("oracle rejected the arguments")
    return IntegrationResult(res.sigma, res.sigma_err, res.chi2_dof, res.w_max, res.n_pass,
                             res.n_newton_fail, res.n_near_edge, I, V, grid, hist, w)


def combine(I, V):
    I = _f64(I)
    V = _f64(V)
    s, e, c = C.c_double(), C.c_double(), C.c_double()
    lib().mfo_combine(len(I), _d(I), _d(V), C.byref(s), C.byref(e), C.byref(c))
    return s.value, e.value, c.value


def neumaier_sum(v):
    v = _f64(v)
    return lib().mfo_neumaier_sum(len(v), _d(v))


def ttx_dweight_dmt_analytic(proc: Process, sqrt_s, table, grid, y):
    h = _PdfHandle(table)
    grid = _f64(grid)
    y = _f64(y)
    w = C.c_double()
    pc = proc.c()
    g = lib().mfo_ttx_dweight_dmt_analytic(C.byref(pc), sqrt_s, C.byref(h.c),
                                           grid.shape[1] - 1, _d(grid), _d(y), C.byref(w))
    return g, w.value


def unweight_uniform(seed: int, it: int, event: int) -> float:
    """u_e of the hit-or-miss step: Philox block 0x80000000 of event e."""
    return lib().mfo_unweight_uniform(seed, it, event)


def unweight(w, w_max, seed, it):
    """keep[e] = sign(w_e) if u_e w_max < |w_e| else 0; returns (keep, n_kept, n_over)."""
    w = _f64(w)
    keep = np.zeros(len(w), dtype=np.int8)
    over = C.c_uint64()
    n = lib().mfo_unweight(len(w), _d(w), w_max, seed, it,
                           keep.ctypes.data_as(C.POINTER(C.c_byte)), C.byref(over))
    return keep, int(n), int(over.value)


def lab_event(proc: Process, sqrt_s, grid, seed, it, event):
    """Lab-frame momenta [n_f + 2][4] of event e (beams, t, tbar, gluons) and a
    status: 0, 1 below threshold, 2 Newton failure."""
    grid = _f64(grid)
    p = np.zeros((proc.n_g + 2, 4))
    pc = proc.c()
    st = lib().mfo_lab_event(C.byref(pc), sqrt_s, grid.shape[1] - 1, _d(grid), seed, it, event, _d(p))
    return p, st


def event_weights(proc: Process, sqrt_s, table, grid, seed, it, ids, n_threads=None,
                  return_kappa=False):
    """Weights of the events `ids` of iteration `it`, threaded; returns (w, flags)
    with flags bit 0 above threshold, 1 Newton failed, 2 passed the cuts,
    3 near a cut edge, 4 ill-conditioned PDF value, 5 sampled colour sum
    with condition number above 50 (EventInfo.colour_kappa gives it), 6
    mass-rescaling root with condition number above 1e3.  With
    return_kappa=True also returns that condition number per event."""
    h = _PdfHandle(table)
    grid = _f64(grid)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    if n_threads is None:
        n_threads = max(1, min(os.cpu_count() or 1, 16))
    w = np.zeros(len(ids))
    flags = np.zeros(len(ids), dtype=np.int32)
    pc = proc.c()
    kappa = np.zeros(len(ids))
    lib().mfo_event_weights(C.byref(pc), sqrt_s, C.byref(h.c), grid.shape[1] - 1, _d(grid), seed, it,
                            len(ids), ids.ctypes.data_as(_u64p), n_threads, _d(w),
                            flags.ctypes.data_as(_ip), _d(kappa))
    return (w, flags, kappa) if return_kappa else (w, flags)


def hel_count(n_g: int) -> int:
    return lib().mfo_hel_count(n_g)


def hel_config(n_g: int, seed: int, it: int, event: int) -> int:
    """Helicity configuration of event e (Monte Carlo over helicities): Philox
    block 0x80000002, h = (k N_h) >> 53."""
    return lib().mfo_hel_config(n_g, seed, it, event)


def me2_hel(n_g: int, p, m=173.0, width=1.5, colour="full", cfg=-1, h=0, return_kappa=False):
    """Colour sum of |M|^2 (g_s = 1) for the single configuration h of the linear
    polarisation basis; colour "full", "leading", "sampled" (assignment cfg) or
    "flow" (flow cfg)."""
    p = _f64(p)
    modes = {"full": 0, "leading": 1, "sampled": 2, "flow": 3}
    k = C.c_double()
    v = lib().mfo_me2_hel(n_g, _d(p), m, width, modes[colour], cfg, h, C.byref(k))
    return (v, k.value) if return_kappa else v
