"""Pins for the oracle's Monte Carlo over colour flows (colour = "flow").

Sec. 3.2 (on Fig. 4) names a Monte Carlo over colours as a remedy for high-multiplicity
matrix elements.  Besides adjoint indices, the colour of a gluon can be
sampled as a colour-anticolour pair (a, b) with state matrix
G_ab = (e_ab - delta_ab / N) / sqrt 2 (the 't Hooft double line with the
U(1) part projected out), whose nine pairs resolve
sum_a T^a (x) conj(T^a) exactly.  Flows whose factors vanish for every
ordering carry no weight and are dropped; drawing uniformly among the rest
gives an unbiased estimate of the colour sum with a smaller variance than
adjoint sampling, because each surviving flow selects few orderings; drawing
flow f with probability proportional to its integer weight
W_f = 18^n sum_sigma c_sigma(f)^2 and scaling by T / W_f lowers it further.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_me import M, random_momenta


def all_flow_factors(n_g):
    return np.array([O.flow_factors(n_g, k) for k in range(O.flow_count(n_g))])


def walk_factor(order, pairs, i, j):
    """(G_{order1} ... G_{ordern})_{ij} by following the colour line: an
    off-diagonal pair (a, b) moves colour a to b (factor 1/sqrt 2), a
    diagonal pair (a, a) keeps the colour with factor ([r == a] - 1/3)/sqrt 2.
    A second algorithm, independent of the oracle's matrix products."""
    r, v = i, 1.0
    for g in order:
        a, b = pairs[g]
        if a != b:
            if r != a:
                return 0.0
            r = b
            v /= math.sqrt(2.0)
        else:
            v *= ((1.0 if r == a else 0.0) - 1.0 / 3.0) / math.sqrt(2.0)
    return v if r == j else 0.0


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_kept_flows_are_exactly_those_with_a_nonzero_factor(n_g):
    """Enumerate every code by the colour-line walk: the oracle's list is the
    set of codes with some non-vanishing factor, in increasing order, and its
    factors agree with the walk."""
    orders = [tuple(s) for s in O.orderings(n_g)]
    kept = []
    for code in range(9 * 9 ** n_g):
        j, i, rest = code % 3, (code // 3) % 3, code // 9
        pairs = [divmod((rest // 9 ** g) % 9, 3) for g in range(n_g)]
        f = [walk_factor(s, pairs, i, j) for s in orders]
        if any(x != 0.0 for x in f):
            kept.append((code, f))
    assert O.flow_count(n_g) == len(kept)
    assert [O.flow_code(n_g, k) for k in range(len(kept))] == [c for c, _ in kept]
    assert O.flow_code(n_g, len(kept)) == -1 and O.flow_code(n_g, -1) == -1
    for k in range(0, len(kept), max(1, len(kept) // 50)):
        assert np.allclose(O.flow_factors(n_g, k), kept[k][1], rtol=1e-14, atol=0)
        assert O.flow_weight(n_g, k) == round(18 ** n_g * sum(x * x for x in kept[k][1]))
    assert O.flow_weight(n_g, len(kept)) == -1


def test_flow_counts_and_factors_by_hand():
    assert [O.flow_count(n) for n in (2, 3, 4)] == [87, 585, 4311]
    assert O.flow_count(1) == -1 and O.flow_count(5) == -1 and O.flow_total(5) == -1
    for n in (2, 3, 4):
        # T = 18^n sum_f sum_s c_s^2 = 18^n tr C (the colour matrix is pinned on its own)
        assert O.flow_total(n) == round(18 ** n * np.trace(O.colour_matrix(n)))
        assert O.flow_total(n) == sum(O.flow_weight(n, k) for k in range(O.flow_count(n)))
        # code 0: every ordering's factor is (2/3)^n / 2^(n/2): weight n! 4^n
        assert O.flow_weight(n, 0) == math.factorial(n) * 4 ** n
    assert [O.flow_total(n) for n in (2, 3, 4)] == [3456, 248832, 23887872]
    # code 0: every pair (0, 0), i = j = 0: (2/3)^n / 2^(n/2) for each ordering
    for n in (2, 3, 4):
        assert np.allclose(O.flow_factors(n, 0), (2 / 3) ** n / 2 ** (n / 2), rtol=1e-15, atol=0)
    # i = 0, gluon 0 = (0 -> 1), gluon 1 = (1 -> 2), j = 2: only the ordering (0, 1) connects
    code = 2 + 3 * 0 + 9 * ((3 * 0 + 1) + 9 * (3 * 1 + 2))
    k = [O.flow_code(2, q) for q in range(O.flow_count(2))].index(code)
    assert [tuple(s) for s in O.orderings(2)] == [(0, 1), (1, 0)]
    assert np.allclose(O.flow_factors(2, k), [0.5, 0.0], rtol=1e-15, atol=0)
    assert O.flow_weight(2, k) == 81


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_flow_factors_rebuild_the_colour_matrix(n_g):
    """sum over kept flows of c_s c_t = C_st (the dropped flows add zero)."""
    F = all_flow_factors(n_g)
    assert np.allclose(F.T @ F, O.colour_matrix(n_g), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_flow_estimator_unbiased_and_tighter_than_adjoint_sampling(n_g):
    """At a random point: the sum over flows of |M|^2 is the colour sum, the
    oracle's per-flow function is T / W_f times the same products, and the
    exact variance per event of the weighted flow draw (probability W_f / T)
    is below that of the uniform flow draw and of adjoint sampling."""
    rng = np.random.default_rng(800 + n_g)
    p = random_momenta(n_g, 1300.0, rng)
    A = np.array([O.partial_amplitudes(n_g, p, M, 1.5, h) for h in O.all_helicities(n_g)])
    exact = O.me2_sum(n_g, p, M, 1.5)
    F = all_flow_factors(n_g)
    per_flow = np.sum(np.abs(F @ A.T) ** 2, axis=1)
    assert per_flow.sum() == pytest.approx(exact, rel=1e-12)
    n = len(F)
    T = O.flow_total(n_g)
    W = np.array([O.flow_weight(n_g, k) for k in range(n)], dtype=float)
    for k in (0, 7, n // 2, n - 1):
        ref = T / W[k] * per_flow[k]
        assert O.me2_sum_colour_flow(n_g, p, M, 1.5, k) == pytest.approx(ref, rel=1e-12, abs=1e-300)
    relvar_uniform = n * np.sum(per_flow ** 2) / exact ** 2 - 1
    relvar_flow = np.sum(per_flow ** 2 * T / W) / exact ** 2 - 1
    Fa = np.array([O.colour_factors(n_g, c) for c in range(O.colour_count(n_g))])
    per_adj = np.sum(np.abs(Fa @ A.T) ** 2, axis=1)
    relvar_adj = len(Fa) * np.sum(per_adj ** 2) / exact ** 2 - 1
    print(f"\n  n_g = {n_g}: relative variance per event, weighted flows {relvar_flow:.3g}, uniform flows "
          f"{relvar_uniform:.3g}, adjoint indices {relvar_adj:.3g}")
    assert relvar_flow < relvar_uniform < relvar_adj


def test_flow_draw_is_philox_block_0x80000001(torch_philox):
    cases = [(0, 0, 0), (0, 9, 4), (3, 123456789, 0), (2**40 + 1, 2**33 + 5, 7)]
    triples = [(seed, e, it | (0x80000001 << 32)) for seed, e, it in cases]
    for n_g in (3, 4):
        for (seed, e, it), r in zip(cases, torch_philox(triples)):
            k = ((r[0] << 32) | r[1]) >> 11
            u = (k * O.flow_total(n_g)) >> 53
            cum = np.cumsum([0] + [O.flow_weight(n_g, f) for f in range(O.flow_count(n_g))])
            assert O.flow_config(n_g, seed, it, e) == int(np.searchsorted(cum, u, side="right")) - 1


def test_flow_draw_frequencies_follow_the_weights():
    n_g, n = 3, 60000
    N = O.flow_count(n_g)
    idx = np.array([O.flow_config(n_g, 1, 2, e) for e in range(n)])
    assert idx.min() >= 0 and idx.max() < N
    counts = np.bincount(idx, minlength=N)
    expect = n * np.array([O.flow_weight(n_g, f) for f in range(N)]) / O.flow_total(n_g)
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert abs(chi2 - (N - 1)) < 6 * math.sqrt(2 * (N - 1))


def test_flow_event_weight_uses_the_events_flow(pdf_table):
    grid = np.tile(np.arange(51) / 50, (10, 1))
    full = O.Process(n_g=4, ptmin_g=20.0, drmin_gg=0.4)
    flow = O.Process(n_g=4, ptmin_g=20.0, drmin_gg=0.4, colour="flow")
    checked = 0
    for e in range(30):
        wf, ev = O.event_weight(full, 13000.0, pdf_table, grid, 0, 0, e)
        ws, evs = O.event_weight(flow, 13000.0, pdf_table, grid, 0, 0, e)
        if wf == 0.0:
            assert ws == 0.0
            continue
        k = np.asarray(ev.k)
        e_b = math.sqrt(ev.shat) / 2
        p = np.array([k[0], k[1], [-e_b, 0, 0, -e_b], [-e_b, 0, 0, e_b], k[2], k[3]])
        idx = O.flow_config(4, 0, 0, e)
        ratio = O.me2_sum_colour_flow(4, p, M, 1.5, idx) / O.me2_sum(4, p, M, 1.5)
        assert ws == pytest.approx(wf * ratio, rel=1e-12, abs=1e-300)
        checked += 1
    assert checked > 15
    y = np.full(10, 0.37)
    w, _ = O.event_weight_y(flow, 13000.0, pdf_table, grid, y)
    assert math.isnan(w)


def test_condition_number_of_the_sampled_sums():
    """kappa = sum_h |M_h| sum_s |c_s A_s,h| / sum_h |M_h|^2 against its
    definition; kappa = 1 exactly when a single ordering contributes, and
    kappa >= 1 always (triangle inequality)."""
    rng = np.random.default_rng(900)
    p = random_momenta(4, 1400.0, rng)
    A = np.array([O.partial_amplitudes(4, p, M, 1.5, h) for h in O.all_helicities(4)])
    for k in range(0, O.flow_count(4), 97):
        c = O.flow_factors(4, k)
        v, kappa = O.me2_sum_sampled(4, p, M, 1.5, 3, k)
        Mh = A @ c
        S = np.sum(np.abs(Mh) ** 2)
        assert v == pytest.approx(O.flow_total(4) / O.flow_weight(4, k) * S, rel=1e-12)
        assert kappa == pytest.approx(np.sum(np.abs(Mh) * (np.abs(A) @ np.abs(c))) / S, rel=1e-12)
        assert kappa >= 1.0 - 1e-14
    # a single contributing ordering: i = 0, gluon 0 = (0 -> 1), gluon 1 = (1 -> 2), j = 2
    code = 2 + 9 * ((3 * 0 + 1) + 9 * (3 * 1 + 2))
    k = [O.flow_code(2, q) for q in range(O.flow_count(2))].index(code)
    p2 = random_momenta(2, 900.0, rng)
    assert O.me2_sum_sampled(2, p2, M, 1.5, 3, k)[1] == pytest.approx(1.0, rel=1e-14)
    v, kappa = O.me2_sum_sampled(4, p, M, 1.5, 2, 12345)
    assert v == pytest.approx(O.me2_sum_colour_config(4, p, M, 1.5, 12345), rel=1e-15, abs=1e-300)
    assert kappa == 0.0 or kappa >= 1.0 - 1e-14


def test_out_of_range_arguments_are_rejected():
    p = random_momenta(3, 1000.0, np.random.default_rng(4))
    assert O.flow_config(5, 0, 0, 1) == -1
    assert math.isnan(O.flow_factors(3, O.flow_count(3))[0])
    assert math.isnan(O.flow_factors(3, -1)[0])
    for mode, cfg in ((4, 0), (3, O.flow_count(3)), (2, O.colour_count(3)), (3, -1)):
        v, kappa = O.me2_sum_sampled(3, p, M, 1.5, mode, cfg)
        assert math.isnan(v) and math.isnan(kappa)
