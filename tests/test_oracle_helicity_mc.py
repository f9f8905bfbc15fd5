"""Pins for the oracle's Monte Carlo over helicities (helicity="sampled").

Sec. 3.2 (on Fig. 4) names a Monte Carlo over helicity (and colour)
configurations as a remedy for high-multiplicity matrix elements.  Here each
event carries one configuration h of the 2^(n_g + 2): top and antitop spin
along z in their rest frames, and for every gluon one of the real linear
polarisations e1, e2 of its momentum's frame (the basis the kernels compute
in).  N_h times the colour-summed |M_h|^2 estimates the helicity sum.

The linear-basis amplitudes are pinned against the helicity-basis ones, which
the closed forms, Ward identities and soft limits pin: with eps_+- =
(-/+ e1 - i e2)/sqrt 2, linearity in each polarisation gives
A(e1) = (A(-) - A(+))/sqrt 2 and A(e2) = i (A(+) + A(-))/sqrt 2 gluon by
gluon.
"""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_me import M, random_momenta

R2 = math.sqrt(2.0)


def linear_from_helicity(n_g, p):
    """[N_h][n_g!] partial amplitudes in the linear basis, built from the
    helicity-basis amplitudes by the change of basis above."""
    nh = 1 << (n_g + 2)
    hel = np.array([O.partial_amplitudes(n_g, p, M, 1.5, [(h >> i) & 1 for i in range(n_g + 2)])
                    for h in range(nh)])
    A = hel.reshape([2] * n_g + [4, -1])          # gluon bits (most significant first), spins, orderings
    for g in range(n_g):
        ax = n_g - 1 - g                          # bit 2 + g of h
        plus = np.take(A, 0, axis=ax)
        minus = np.take(A, 1, axis=ax)
        A = np.stack([(minus - plus) / R2, 1j * (plus + minus) / R2], axis=ax)
    return A.reshape(nh, -1)


@pytest.mark.parametrize("n_g", [2, 3, 4, 5])
def test_linear_basis_configurations_against_the_helicity_basis(n_g):
    rng = np.random.default_rng(1300 + n_g)
    C = O.colour_matrix(n_g)
    for trial in range(2):
        p = random_momenta(n_g, 1100.0 + 300.0 * trial, rng)
        A = linear_from_helicity(n_g, p)
        ref = np.real(np.einsum("hs,st,ht->h", A.conj(), C, A))
        got = np.array([O.me2_hel(n_g, p, M, 1.5, "full", -1, h) for h in range(O.hel_count(n_g))])
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-14 * ref.max())
        # summed over configurations: the helicity sum of the other basis
        assert got.sum() == pytest.approx(O.me2_sum(n_g, p, M, 1.5), rel=1e-12)
        # leading colour per configuration
        lc = np.array([O.me2_hel(n_g, p, M, 1.5, "leading", -1, h) for h in range(O.hel_count(n_g))])
        assert np.allclose(lc, O.colour_lc(n_g) * np.sum(np.abs(A) ** 2, axis=1), rtol=1e-11)
        # colour assignment and colour flow per configuration sum to the oracle's sampled sums
        if 3 <= n_g <= 4:
            for mode, cfg in (("sampled", 12345 % O.colour_count(n_g)), ("flow", 17)):
                per = [O.me2_hel(n_g, p, M, 1.5, mode, cfg, h) for h in range(O.hel_count(n_g))]
                whole, _ = O.me2_sum_sampled(n_g, p, M, 1.5, {"sampled": 2, "flow": 3}[mode], cfg)
                assert math.fsum(per) == pytest.approx(whole, rel=1e-11, abs=1e-300)


def test_rejected_arguments():
    p = random_momenta(2, 900.0, np.random.default_rng(3))
    assert math.isnan(O.me2_hel(2, p, M, 1.5, "full", -1, 16))
    assert math.isnan(O.me2_hel(2, p, M, 1.5, "full", -1, -1))
    assert math.isnan(O.me2_hel(3, random_momenta(3, 900.0, np.random.default_rng(4)), M, 1.5,
                                "sampled", -1, 0))


def test_configuration_is_philox_block_0x80000002(torch_philox):
    cases = [(0, 0, 0), (0, 9, 4), (3, 123456789, 0), (2**40 + 1, 2**33 + 5, 7)]
    triples = [(seed, e, it | (0x80000002 << 32)) for seed, e, it in cases]
    for n_g in (2, 3, 4):
        for (seed, e, it), r in zip(cases, torch_philox(triples)):
            k = ((r[0] << 32) | r[1]) >> 11
            assert O.hel_config(n_g, seed, it, e) == (k * (1 << (n_g + 2))) >> 53


def test_configurations_uniform_estimate_unbiased_with_exact_variance():
    """Over 40000 events the configurations cover the 64 of t tbar g g
    uniformly; at a fixed point the mean of N_h |M_h|^2 agrees with the exact
    helicity sum within its error, and the sample variance with the exact one,
    N_h sum_h |M_h|^4 - (sum_h |M_h|^2)^2."""
    n_g, n = 4, 40000
    N = O.hel_count(n_g)
    h = np.array([O.hel_config(n_g, 0, 0, e) for e in range(n)])
    counts = np.bincount(h, minlength=N)
    assert h.min() >= 0 and h.max() < N
    chi2 = float(np.sum((counts - n / N) ** 2 / (n / N)))
    assert abs(chi2 - (N - 1)) < 6 * math.sqrt(2 * (N - 1))
    p = random_momenta(n_g, 1200.0, np.random.default_rng(21))
    per = np.array([O.me2_hel(n_g, p, M, 1.5, "full", -1, c) for c in range(N)])
    exact = O.me2_sum(n_g, p, M, 1.5)
    var = N * float(np.sum(per**2)) - exact**2
    est = N * per[h]
    err = math.sqrt(var / n)
    print(f"\n  sampled {est.mean():.6g} +- {err:.2g}, exact {exact:.6g}; relative variance per event "
          f"{var / exact**2:.3g} (sample {est.var() / exact**2:.3g})")
    assert abs(est.mean() - exact) < 5 * err
    # the sample variance of n draws has relative spread sqrt((kurtosis - 1) / n)
    k4 = N * float(np.sum((N * per - exact) ** 4)) / N**2
    assert abs(est.var() / var - 1) < 5 * math.sqrt((k4 / var**2 - 1) / n)


@pytest.mark.parametrize("colour", ["full", "flow"])
def test_sampled_event_weight_uses_the_events_configuration(pdf_table, colour):
    grid = np.tile(np.arange(51) / 50, (10, 1))
    full = O.Process(n_g=4, ptmin_g=20.0, drmin_gg=0.4)
    samp = O.Process(n_g=4, ptmin_g=20.0, drmin_gg=0.4, colour=colour, helicity="sampled")
    checked = 0
    for e in range(30):
        wf, ev = O.event_weight(full, 13000.0, pdf_table, grid, 0, 0, e)
        ws, evs = O.event_weight(samp, 13000.0, pdf_table, grid, 0, 0, e)
        if wf == 0.0:
            assert ws == 0.0
            continue
        k = np.asarray(ev.k)
        e_b = math.sqrt(ev.shat) / 2
        p = np.array([k[0], k[1], [-e_b, 0, 0, -e_b], [-e_b, 0, 0, e_b], k[2], k[3]])
        h = O.hel_config(4, 0, 0, e)
        cfg = O.flow_config(4, 0, 0, e) if colour == "flow" else -1
        ratio = O.hel_count(4) * O.me2_hel(4, p, M, 1.5, colour, cfg, h) / O.me2_sum(4, p, M, 1.5)
        assert ws == pytest.approx(wf * ratio, rel=1e-12, abs=1e-300)
        checked += 1
    assert checked > 15
    # caller uniforms carry no event counter: no configuration
    w, _ = O.event_weight_y(samp, 13000.0, pdf_table, grid, np.full(10, 0.37))
    assert math.isnan(w)
