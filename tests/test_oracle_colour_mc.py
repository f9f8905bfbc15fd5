"""Pins for the oracle's Monte Carlo over colours (colour = "sampled").

Sec. 3.2 (on Fig. 4) names a Monte Carlo over colour configurations as a remedy for
high-multiplicity matrix elements.  Here each event carries one colour
assignment (gluon adjoint indices, top colour, antitop anticolour), drawn
uniformly from the 9 * 8^n assignments with Philox block 0x80000001, and
9 * 8^n times the helicity-summed |M|^2 of the colour-dressed amplitude
sum_sigma (T^{a_sigma1} ... T^{a_sigman})_{ij} A(sigma) estimates the colour
sum.  The colour factors come from explicit products of Gell-Mann matrices;
their sum over all assignments must rebuild the colour matrix, which is
pinned separately (exact values, Fierz identities, colour-dressed Feynman
rules), and the estimator must then be unbiased.
"""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_me import M, random_momenta


def all_factors(n_g):
    n = O.colour_count(n_g)
    return np.array([O.colour_factors(n_g, c) for c in range(n)])


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_colour_factors_rebuild_the_colour_matrix(n_g):
    """sum over assignments of conj(c_s) c_t = C_st, and the factor of the
    first assignment (all gluons lambda_1 / 2, i = j = 0) by hand."""
    F = all_factors(n_g)
    C = np.einsum("ks,kt->st", F.conj(), F)
    assert np.allclose(C.imag, 0.0, atol=1e-14)
    assert np.allclose(C.real, O.colour_matrix(n_g), rtol=0, atol=1e-12)   # 36864 terms for n_g = 4
    # (T^1)^n: T^1 = sigma_x / 2 on the first two colours, so (T^1)^n_00 = 2^-n (n even), 0 (odd)
    assert np.allclose(F[0], (0.5 ** n_g) * (n_g % 2 == 0), atol=0)


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_sum_over_assignments_is_the_colour_sum(n_g):
    """sum_cfg sum_h |M(cfg)|^2 = sum_h A^dagger C A at a random point:
    the estimator is unbiased by construction of the sampling."""
    rng = np.random.default_rng(700 + n_g)
    p = random_momenta(n_g, 1100.0, rng)
    A = np.array([O.partial_amplitudes(n_g, p, M, 1.5, h) for h in O.all_helicities(n_g)])
    F = all_factors(n_g)
    total = float(np.sum(np.abs(F @ A.T) ** 2))
    assert total == pytest.approx(O.me2_sum(n_g, p, M, 1.5), rel=1e-12)
    # the per-assignment oracle function agrees with the same products
    for cfg in (0, 5, O.colour_count(n_g) - 1, O.colour_count(n_g) // 3):
        ref = O.colour_count(n_g) * float(np.sum(np.abs(A @ F[cfg]) ** 2))
        assert O.me2_sum_colour_config(n_g, p, M, 1.5, cfg) == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_assignment_is_philox_block_0x80000001(torch_philox):
    cases = [(0, 0, 0), (0, 9, 4), (3, 123456789, 0), (2**40 + 1, 2**33 + 5, 7)]
    triples = [(seed, e, it | (0x80000001 << 32)) for seed, e, it in cases]
    for n_g in (3, 4):
        for (seed, e, it), r in zip(cases, torch_philox(triples)):
            k = ((r[0] << 32) | r[1]) >> 11
            assert O.colour_config(n_g, seed, it, e) == ((k >> 16) * O.colour_count(n_g)) >> 37


def test_assignments_uniform_and_estimate_unbiased():
    """Over 20000 events the assignments cover [0, N) uniformly, and the
    sampled estimate of the t tbar colour sum at a fixed point agrees with
    the exact sum within its Monte Carlo error."""
    n_g, n = 2, 20000
    N = O.colour_count(n_g)
    cfg = np.array([O.colour_config(n_g, 0, 0, e) for e in range(n)])
    assert cfg.min() >= 0 and cfg.max() < N
    counts = np.bincount(cfg, minlength=N)
    chi2 = float(np.sum((counts - n / N) ** 2 / (n / N)))
    assert abs(chi2 - (N - 1)) < 6 * math.sqrt(2 * (N - 1))
    rng = np.random.default_rng(9)
    p = random_momenta(n_g, 900.0, rng)
    A = np.array([O.partial_amplitudes(n_g, p, M, 1.5, h) for h in O.all_helicities(n_g)])
    F = all_factors(n_g)
    est = N * np.sum(np.abs(F[cfg] @ A.T) ** 2, axis=1)
    exact = O.me2_sum(n_g, p, M, 1.5)
    err = est.std() / math.sqrt(n)
    print(f"\n  sampled {est.mean():.6g} +- {err:.2g}, exact {exact:.6g}; relative variance per event "
          f"{est.var() / exact**2:.3g}")
    assert abs(est.mean() - exact) < 5 * err


def test_sampled_event_weight_uses_the_events_assignment(pdf_table):
    grid = np.tile(np.arange(51) / 50, (10, 1))
    full = O.Process(n_g=4, ptmin_g=20.0, drmin_gg=0.4)
    samp = O.Process(n_g=4, ptmin_g=20.0, drmin_gg=0.4, colour="sampled")
    checked = 0
    for e in range(30):
        wf, ev = O.event_weight(full, 13000.0, pdf_table, grid, 0, 0, e)
        ws, _ = O.event_weight(samp, 13000.0, pdf_table, grid, 0, 0, e)
        if wf == 0.0:
            assert ws == 0.0
            continue
        k = np.asarray(ev.k)
        e_b = math.sqrt(ev.shat) / 2
        p = np.array([k[0], k[1], [-e_b, 0, 0, -e_b], [-e_b, 0, 0, e_b], k[2], k[3]])
        cfg = O.colour_config(4, 0, 0, e)
        ratio = O.me2_sum_colour_config(4, p, M, 1.5, cfg) / O.me2_sum(4, p, M, 1.5)
        assert ws == pytest.approx(wf * ratio, rel=1e-12, abs=1e-300)
        checked += 1
    assert checked > 15
    # caller uniforms carry no event counter: no colour assignment
    y = np.full(10, 0.37)
    w, _ = O.event_weight_y(samp, 13000.0, pdf_table, grid, y)
    assert math.isnan(w)
