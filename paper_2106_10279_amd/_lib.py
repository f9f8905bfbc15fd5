"""ctypes binding of libmadflow_mi355x.so (declarations in include/mf.h).

Argument marshalling only: every step of the integrand runs in the HIP
library.  If the library is missing this module raises at import time;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libmadflow_mi355x.so")

MF_OK, MF_EINVAL, MF_ENOMEM, MF_EDEVICE, MF_ENOCONV, MF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MF_GG_TTX, MF_GG_TTXG, MF_GG_TTXGG, MF_GG_TTXGGG, MF_PP_TTX, MF_PP_TTXG, MF_PP_TTXGG = 0, 1, 2, 3, 4, 5, 6
MF_FP64, MF_FP32_KAHAN = 0, 1

_dp = C.POINTER(C.c_double)


class mf_process(C.Structure):
    _fields_ = [("id", C.c_int), ("m_top", C.c_double), ("w_top", C.c_double),
                ("alpha_s", C.c_double), ("mu_f", C.c_double), ("ptmin_g", C.c_double),
                ("etamax_g", C.c_double), ("drmin_gg", C.c_double)]


class mf_pdf_grid(C.Structure):
    _fields_ = [("n_x", C.c_int), ("n_q2", C.c_int), ("log_x", _dp), ("log_q2", _dp),
                ("xf", _dp), ("xq", _dp)]


class mf_options(C.Structure):
    _fields_ = [("n_bins", C.c_int), ("alpha", C.c_double), ("start_iter", C.c_int),
                ("precision", C.c_int), ("strict", C.c_int), ("max_newton", C.c_int),
                ("grid_in", _dp), ("stream", C.c_void_p), ("profile", C.c_int),
                ("max_batch", C.c_uint64), ("colour", C.c_int), ("helicity", C.c_int)]


class mf_result(C.Structure):
    _fields_ = [("sigma", C.c_double), ("sigma_err", C.c_double), ("chi2_dof", C.c_double),
                ("w_max", C.c_double), ("iter_sigma", _dp), ("iter_var", _dp), ("grid", _dp),
                ("hist", _dp), ("weights", _dp), ("n_pass", C.c_int64),
                ("n_newton_fail", C.c_int64), ("event_kernel_ms", C.c_double),
                ("reduce_kernel_ms", C.c_double), ("iter_pass", _dp), ("iter_event_ms", _dp),
                ("iter_amp_ms", _dp), ("n_batches", C.c_uint64), ("grid_last", _dp),
                ("iter_colour_ms", _dp)]


class mf_grad_result(C.Structure):
    _fields_ = [("dsigma_dmt", C.c_double), ("dsigma_dalphas", C.c_double), ("iter_dmt", _dp),
                ("iter_dalphas", _dp), ("dw_dy", _dp), ("dw_dmt", _dp), ("iter_grad_ms", _dp)]


class mf_events(C.Structure):
    _fields_ = [("capacity", C.c_uint64), ("event", C.c_void_p), ("p", C.c_void_p),
                ("sign", C.c_void_p), ("n_kept", C.c_uint64), ("n_over", C.c_uint64),
                ("kernel_ms", C.c_double * 3)]


EXPORTS = ("mf_default_options", "mf_n_dims", "mf_integrate", "mf_integrate_static", "mf_evaluate",
           "mf_refine_grid", "mf_colour_matrix", "mf_matrix_element", "mf_integrate_grad",
           "mf_evaluate_grad", "mf_unweight", "mf_last_error")


class MFError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2106_10279_amd/build.py "
                          "(hipcc, gfx950); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    L.mf_default_options.argtypes = [C.POINTER(mf_options)]
    L.mf_default_options.restype = None
    L.mf_n_dims.argtypes = [C.c_int]
    L.mf_n_dims.restype = C.c_int
    L.mf_integrate.argtypes = [C.POINTER(mf_process), C.c_double, C.POINTER(mf_pdf_grid),
                               C.c_uint64, C.c_int, C.c_uint64, C.POINTER(mf_options),
                               C.POINTER(mf_result)]
    L.mf_integrate.restype = C.c_int
    L.mf_integrate_static.argtypes = L.mf_integrate.argtypes
    L.mf_integrate_static.restype = C.c_int
    L.mf_evaluate.argtypes = [C.POINTER(mf_process), C.c_double, C.POINTER(mf_pdf_grid), _dp,
                              C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint64, C.c_int,
                              C.POINTER(mf_options), C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p]
    L.mf_evaluate.restype = C.c_int
    L.mf_integrate_grad.argtypes = [C.POINTER(mf_process), C.c_double, C.POINTER(mf_pdf_grid),
                                    C.c_uint64, C.c_int, C.c_uint64, C.POINTER(mf_options),
                                    C.POINTER(mf_result), C.POINTER(mf_grad_result)]
    L.mf_integrate_grad.restype = C.c_int
    L.mf_evaluate_grad.argtypes = [C.POINTER(mf_process), C.c_double, C.POINTER(mf_pdf_grid), _dp,
                                   C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint64, C.c_int,
                                   C.POINTER(mf_options), C.c_void_p, C.c_void_p, C.c_void_p]
    L.mf_evaluate_grad.restype = C.c_int
    L.mf_refine_grid.argtypes = [C.c_int, C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]
    L.mf_refine_grid.restype = C.c_int
    L.mf_colour_matrix.argtypes = [C.c_int, _dp]
    L.mf_colour_matrix.restype = C.c_int
    L.mf_matrix_element.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_uint64,
                                    C.c_double, C.c_double, C.c_void_p, C.c_void_p]
    L.mf_matrix_element.restype = C.c_int
    L.mf_unweight.argtypes = [C.POINTER(mf_process), C.c_double, _dp, C.c_void_p, C.c_uint64,
                              C.c_uint64, C.c_int, C.c_double, C.POINTER(mf_options),
                              C.POINTER(mf_events)]
    L.mf_unweight.restype = C.c_int
    L.mf_last_error.argtypes = []
    L.mf_last_error.restype = C.c_char_p
    return L


lib = load()


def check(status):
    if status != MF_OK:
        raise MFError(status, lib.mf_last_error().decode())
