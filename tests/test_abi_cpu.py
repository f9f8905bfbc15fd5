"""C-ABI checks that need no GPU: every declared symbol is exported and
argument validation answers before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2106_10279_amd import _lib
    return _lib


def test_header_declares_the_expected_entry_points():
    names = declared_functions()
    for n in ("mf_integrate", "mf_evaluate", "mf_refine_grid", "mf_colour_matrix",
              "mf_matrix_element", "mf_last_error", "mf_n_dims", "mf_default_options",
              "mf_integrate_grad", "mf_evaluate_grad", "mf_unweight"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    lib = C.CDLL(L.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_n_dims(L):
    assert [L.lib.mf_n_dims(i) for i in (0, 1, 2)] == [4, 7, 10]
    assert L.lib.mf_n_dims(7) == -1


def _args(L, pdf_table, **kw):
    from paper_2106_10279_amd import api
    proc = api.Process(kw.pop("process", "gg_ttx"), **{k: kw.pop(k) for k in list(kw)
                                                        if k in ("m_top", "w_top", "alpha_s", "mu_f")})
    return api, proc


@pytest.mark.parametrize("bad", [
    dict(n_events=1), dict(n_iter=0), dict(n_iter=300), dict(sqrt_s=300.0), dict(n_bins=1),
    dict(mu_f=1.0), dict(m_top=-1.0), dict(alpha_s=0.0), dict(n_bins=300),
])
def test_validation_errors_without_device(L, pdf_table, bad):
    from paper_2106_10279_amd import api
    pk = {k: bad[k] for k in ("m_top", "alpha_s", "mu_f") if k in bad}
    proc = api.Process("gg_ttxgg", **pk)
    with pytest.raises(L.MFError) as e:
        api.integrate(proc, bad.get("sqrt_s", 13000.0), pdf_table, bad.get("n_events", 1000),
                      bad.get("n_iter", 2), 0, n_bins=bad.get("n_bins", 50), keep_weights=False,
                      stream=0)
    assert e.value.status in (L.MF_EINVAL, L.MF_EUNSUPPORTED)


def test_bad_pdf_grid_rejected(L, pdf_table):
    from paper_2106_10279_amd import api
    import workloads
    t = pdf_table
    bad = workloads.PdfTable(t.log_x[::-1].copy(), t.log_q2, t.xf)
    with pytest.raises(L.MFError):
        api.integrate(api.Process(), 13000.0, bad, 1000, 1, 0, keep_weights=False, stream=0)
    grid = np.tile(np.arange(51) / 50, (4, 1))
    grid[1, 10] = grid[1, 11]
    with pytest.raises(L.MFError):
        api.integrate(api.Process(), 13000.0, pdf_table, 1000, 1, 0, grid_in=grid,
                      keep_weights=False, stream=0)


def test_colour_matrix_matches_oracle_bitwise(L):
    from paper_2106_10279_amd import api
    import oracle as O
    for proc, n in (("gg_ttx", 2), ("gg_ttxg", 3), ("gg_ttxgg", 4)):
        assert np.array_equal(api.colour_matrix(proc), O.colour_matrix(n))


@pytest.mark.parametrize("process", ["gg_ttxg", "gg_ttxgg"])
def test_gradients_reject_processes_other_than_ttx_without_device(L, pdf_table, process):
    from paper_2106_10279_amd import api
    proc = api.Process(process)
    with pytest.raises(L.MFError) as e:
        api.integrate_grad(proc, 13000.0, pdf_table, 1000, 1, 0, stream=0)
    assert e.value.status == L.MF_EUNSUPPORTED


def test_gradient_rejects_fp32_without_device(L, pdf_table):
    from paper_2106_10279_amd import api
    o = L.mf_options()
    L.lib.mf_default_options(C.byref(o))
    o.precision = L.MF_FP32_KAHAN
    proc = api.Process("gg_ttx").c()
    pdf = api._Pdf(pdf_table)
    res = L.mf_result()
    g = L.mf_grad_result()
    st = L.lib.mf_integrate_grad(C.byref(proc), 13000.0, C.byref(pdf.c), 1000, 1, 0, C.byref(o),
                                 C.byref(res), C.byref(g))
    assert st == L.MF_EUNSUPPORTED
    assert b"FP64" in L.lib.mf_last_error()


def test_max_batch_above_the_cap_rejected_without_device(L, pdf_table):
    from paper_2106_10279_amd import api
    with pytest.raises(L.MFError) as e:
        api.integrate(api.Process("gg_ttxgg"), 13000.0, pdf_table, 1000, 1, 0, keep_weights=False,
                      stream=0, max_batch=(1 << 27) + 1)
    assert e.value.status == L.MF_EINVAL
    assert b"max_batch" in L.lib.mf_last_error()


def _unweight_call(L, process="gg_ttxgg", sqrt_s=13000.0, grid=None, w=None, n=10, it=0, w_max=1.0,
                   capacity=0, event=None):
    from paper_2106_10279_amd import api
    o = L.mf_options()
    L.lib.mf_default_options(C.byref(o))
    proc = api.Process(process).c()
    ev = L.mf_events()
    ev.capacity = capacity
    ev.event = event
    g = None if grid is None else np.ascontiguousarray(grid, dtype=np.float64)
    st = L.lib.mf_unweight(C.byref(proc), sqrt_s, g.ctypes.data_as(C.POINTER(C.c_double)) if g is not None
                           else None, w, n, 0, it, w_max, C.byref(o), C.byref(ev))
    return st, ev


@pytest.mark.parametrize("bad", [dict(w_max=0.0), dict(w_max=float("inf")), dict(w_max=float("nan")),
                                 dict(it=-1), dict(sqrt_s=300.0), dict(n=(1 << 40) + 1),
                                 dict(w=None), dict(capacity=5)])
def test_unweight_validation_without_device(L, bad):
    kw = dict(w=C.c_void_p(16))   # never dereferenced: every case fails validation first
    kw.update(bad)
    st, _ = _unweight_call(L, **kw)
    assert st == L.MF_EINVAL, L.lib.mf_last_error()


def test_unweight_rejects_bad_grid_without_device(L):
    grid = np.tile(np.arange(51) / 50, (10, 1))
    grid[3, 7] = grid[3, 6]
    st, _ = _unweight_call(L, w=C.c_void_p(16), grid=grid)
    assert st == L.MF_EINVAL
    assert b"grid" in L.lib.mf_last_error()


def test_unweight_of_no_events_returns_nothing_without_device(L):
    st, ev = _unweight_call(L, w=None, n=0)
    assert st == L.MF_OK
    assert ev.n_kept == 0 and ev.n_over == 0


def test_colour_mode_default_and_validation_without_device(L, pdf_table):
    from paper_2106_10279_amd import api
    o = L.mf_options()
    L.lib.mf_default_options(C.byref(o))
    assert o.colour == 0                      # MF_COLOUR_FULL
    with pytest.raises(L.MFError) as e:
        api.integrate(api.Process("gg_ttxgg"), 13000.0, pdf_table, 1000, 1, 0, keep_weights=False,
                      stream=0, colour=4)
    assert e.value.status == L.MF_EINVAL
    assert b"colour" in L.lib.mf_last_error()
    # the Monte Carlo over colours (adjoint indices or flows): mf_integrate for
    # n_g >= 3 only, rejected before any device call
    for mode, code in (("sampled", 2), ("flow", 3)):
        with pytest.raises(L.MFError) as e:
            api.integrate(api.Process("gg_ttx"), 13000.0, pdf_table, 1000, 1, 0, keep_weights=False,
                          stream=0, colour=mode)
        assert e.value.status == L.MF_EUNSUPPORTED
        o.colour = code
        proc = api.Process("gg_ttxgg").c()
        pdf = api._Pdf(pdf_table)
        st = L.lib.mf_evaluate(C.byref(proc), 13000.0, C.byref(pdf.c), None, None, None, 10, 0, 0, C.byref(o),
                               C.c_void_p(16), None, None, None)
        assert st == L.MF_EUNSUPPORTED
        assert b"colours" in L.lib.mf_last_error()


def test_gradient_rejects_leading_colour_without_device(L, pdf_table):
    from paper_2106_10279_amd import api
    o = L.mf_options()
    L.lib.mf_default_options(C.byref(o))
    o.colour = 1                              # MF_COLOUR_LEADING
    proc = api.Process("gg_ttx").c()
    pdf = api._Pdf(pdf_table)
    res = L.mf_result()
    g = L.mf_grad_result()
    st = L.lib.mf_integrate_grad(C.byref(proc), 13000.0, C.byref(pdf.c), 1000, 1, 0, C.byref(o),
                                 C.byref(res), C.byref(g))
    assert st == L.MF_EUNSUPPORTED
    assert b"colour" in L.lib.mf_last_error()
    w = C.c_void_p(16)                         # never dereferenced: rejected before any device call
    st = L.lib.mf_evaluate_grad(C.byref(proc), 13000.0, C.byref(pdf.c), None, None, None, 10, 0, 0,
                                C.byref(o), w, None, None)
    assert st == L.MF_EUNSUPPORTED
