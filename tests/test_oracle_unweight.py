"""Pins for the oracle's hit-or-miss unweighting and lab-frame event records
(Sec. 2.5: weighted events become unit-weight events for the LHE output).

* The deciding uniform u_e is the Philox block 0x80000000 of event e's
  counter: checked word by word against PyTorch's independent Philox engine.
* Event e is kept with probability min(1, |w_e| / w_max): checked on
  synthetic weights and on the oracle's own g g -> t tbar weights, where the
  unweighted estimate w_max (N_+ - N_-) / N must agree with the weighted mean
  within its binomial error.
* The lab record conserves four-momentum, keeps the masses and transverse
  momenta, shifts every rapidity by ln(x1/x2)/2, and satisfies the lab-frame
  cuts that selected the event.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

SQRT_S = 13000.0


def _uniform_grid(D, nb=50):
    return np.tile(np.arange(nb + 1) / nb, (D, 1))


def test_unweighting_uniform_is_philox_block_0x80000000(torch_philox):
    cases = [(0, 0, 0), (0, 9, 4), (3, 123456789, 0), (2**40 + 1, 2**33 + 5, 7)]
    triples = [(seed, e, it | (0x80000000 << 32)) for seed, e, it in cases]
    for (seed, e, it), r in zip(cases, torch_philox(triples)):
        k = ((r[0] << 32) | r[1]) >> 11
        assert O.unweight_uniform(seed, it, e) == k * 2.0**-53


def test_unweighting_uniform_is_independent_of_the_event_uniforms():
    n = 20000
    u = np.array([O.unweight_uniform(0, 0, e) for e in range(n)])
    y0 = np.array([O.event_k53(0, 0, e, 4)[0] for e in range(n)], dtype=np.float64) * 2.0**-53
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5 / math.sqrt(12 * n)
    assert abs(np.corrcoef(u, y0)[0, 1]) < 5 / math.sqrt(n)
    assert not np.any(u == y0)


def test_keep_probability_is_abs_weight_over_wmax():
    n = 100000
    rng = np.random.default_rng(11)
    r = 0.3
    w = np.where(rng.random(n) < 0.5, r, -r)
    keep, n_kept, n_over = O.unweight(w, 1.0, 5, 2)
    assert n_over == 0
    assert n_kept == int(np.count_nonzero(keep))
    p = n_kept / n
    assert abs(p - r) < 5 * math.sqrt(r * (1 - r) / n)
    kept = keep != 0
    assert np.all(keep[kept] == np.sign(w[kept]))


def test_edge_weights():
    w = np.array([0.0, 1.0, -1.0, 2.5, -3.0, 0.0, 1e-300])
    keep, n_kept, n_over = O.unweight(w, 1.0, 0, 0)
    assert keep[0] == 0 and keep[5] == 0              # zero weight: never kept
    assert keep[1] == 1 and keep[2] == -1             # |w| = w_max: always kept (u < 1)
    assert keep[3] == 1 and keep[4] == -1 and n_over == 2
    assert n_kept == int(np.count_nonzero(keep))


def test_unweighted_estimate_matches_the_weighted_mean(pdf_table):
    n = 20000
    res = O.integrate(O.Process(n_g=2), SQRT_S, pdf_table, n, 1, 0)
    w = res.weights_last
    assert res.w_max == w.max()
    keep, n_kept, n_over = O.unweight(w, res.w_max, 0, 0)
    assert n_over == 0
    prob = np.minimum(1.0, np.abs(w) / res.w_max)
    assert abs(n_kept - prob.sum()) < 5 * math.sqrt((prob * (1 - prob)).sum()) + 1
    est = res.w_max * keep.astype(np.float64).sum() / n
    # per event the unweighted contribution w_max s_e k_e has mean w_e and
    # variance w_max |w_e| - w_e^2
    err = math.sqrt((res.w_max * np.abs(w) - w * w).sum()) / n
    assert abs(est - w.mean()) < 5 * err


@pytest.mark.parametrize("n_g,cuts", [(2, {}), (3, dict(ptmin_g=20.0, etamax_g=2.5)),
                                      (4, dict(ptmin_g=20.0, drmin_gg=0.4))])
def test_lab_record_kinematics(pdf_table, n_g, cuts):
    proc = O.Process(n_g=n_g, **cuts)
    D = O.n_dims(n_g)
    grid = _uniform_grid(D)
    m = proc.m_top
    checked = 0
    for e in range(200):
        w, info = O.event_weight(proc, SQRT_S, pdf_table, grid, 0, 1, e)
        p, st = O.lab_event(proc, SQRT_S, grid, 0, 1, e)
        if not info.pass_threshold:
            assert st == 1 and not p.any()
            continue
        if info.newton_fail:
            assert st == 2
            continue
        assert st == 0
        x1, x2 = info.x[0], info.x[1]
        scale = SQRT_S
        # incoming gluons along +z and -z with x1 sqrt(s)/2 and x2 sqrt(s)/2
        assert np.allclose(p[0], [x1 * SQRT_S / 2, 0, 0, x1 * SQRT_S / 2], rtol=0, atol=1e-12 * scale)
        assert np.allclose(p[1], [x2 * SQRT_S / 2, 0, 0, -x2 * SQRT_S / 2], rtol=0, atol=1e-12 * scale)
        # four-momentum conservation in the lab
        assert np.abs(p[0] + p[1] - p[2:].sum(axis=0)).max() < 1e-11 * scale
        for i in range(n_g):
            q, k = p[2 + i], info.k[i]
            mass2 = q[0] ** 2 - q[1] ** 2 - q[2] ** 2 - q[3] ** 2
            assert abs(mass2 - (m * m if i < 2 else 0.0)) < 1e-9 * q[0] ** 2
            assert q[1] == k[1] and q[2] == k[2]          # transverse: untouched
            # rapidities add along the beam
            y_lab = 0.5 * math.log((q[0] + q[3]) / (q[0] - q[3]))
            y_cm = 0.5 * math.log((k[0] + k[3]) / (k[0] - k[3]))
            assert abs(y_lab - y_cm - 0.5 * math.log(x1 / x2)) < 1e-10
        if info.pass_cuts:
            for i in range(2, n_g):
                q = p[2 + i]
                pt = math.hypot(q[1], q[2])
                if proc.ptmin_g > 0:
                    assert pt > proc.ptmin_g
                if proc.etamax_g > 0:
                    pabs = math.sqrt(q[1] ** 2 + q[2] ** 2 + q[3] ** 2)
                    eta = 0.5 * math.log((pabs + q[3]) / (pabs - q[3]))
                    assert abs(eta) < proc.etamax_g + 1e-9
        checked += 1
    assert checked > 100


def test_threaded_event_weights_equal_single_evaluations(pdf_table):
    """The threaded batch form used by the full-size checks returns what the
    single-event evaluation returns, flags included."""
    proc = O.Process(n_g=4, ptmin_g=20.0, drmin_gg=0.4)
    grid = _uniform_grid(10)
    ids = np.array([0, 3, 77, 5000, 123457, 2**33 + 1], dtype=np.uint64)
    w, flags = O.event_weights(proc, SQRT_S, pdf_table, grid, 0, 2, ids, n_threads=3)
    for i, e in enumerate(ids):
        w1, info = O.event_weight(proc, SQRT_S, pdf_table, grid, 0, 2, int(e))
        assert w[i] == w1
        assert bool(flags[i] & 1) == info.pass_threshold and bool(flags[i] & 2) == info.newton_fail
        assert bool(flags[i] & 4) == info.pass_cuts and bool(flags[i] & 8) == info.near_edge
        assert bool(flags[i] & 16) == info.ill_conditioned
