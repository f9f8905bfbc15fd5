"""Pins for the oracle's VEGAS map and grid refinement (Lepage 1978)."""
import math

import mpmath as mp
import numpy as np

import oracle as O


def uniform_grid(D, nb):
    return np.tile(np.arange(nb + 1) / nb, (D, 1))


def test_uniform_grid_is_identity_map():
    D, nb = 10, 50
    g = uniform_grid(D, nb)
    rng = np.random.default_rng(0)
    for _ in range(200):
        k = rng.integers(0, 2**53, D)
        bins, deltas = zip(*(O.bin_from_k53(int(v), nb) for v in k))
        x, jac = O.vegas_map(g, bins, deltas)
        y = k * 2.0**-53
        np.testing.assert_allclose(x, y, rtol=0, atol=4e-16)
        # each width e_{i+1} - e_i of the edges i/N_b is off by <= 1 ulp of 1,
        # so each factor N_b (e_{i+1} - e_i) is within N_b 2^-52 of one
        assert abs(jac - 1.0) < D * nb * 2.0**-52


def test_constant_histogram_is_fixed_point():
    D, nb = 3, 50
    g = uniform_grid(D, nb)
    h = np.full((D, nb), 2.5)
    out = O.vegas_refine(h, g, 1.5)
    np.testing.assert_allclose(out, g, rtol=0, atol=4 * 2.0**-52)


def hand_refine(h, e, alpha):
    """The refinement rule worked out in 50-digit arithmetic for one dimension."""
    mp.mp.dps = 50
    n = len(h)
    h = [mp.mpf(v) for v in h]
    e = [mp.mpf(v) for v in e]
    ds = [(h[0] + h[1]) / 2] + [(h[i - 1] + h[i] + h[i + 1]) / 3 for i in range(1, n - 1)] \
        + [(h[n - 2] + h[n - 1]) / 2]
    S = sum(ds)
    r = []
    for d in ds:
        rho = d / S
        r.append(mp.mpf(0) if rho == 0 else ((1 - rho) / (-mp.log(rho))) ** alpha)
    share = sum(r) / n
    new = [mp.mpf(0)]
    cum = [mp.mpf(0)]
    for v in r:
        cum.append(cum[-1] + v)
    for k in range(1, n):
        T = k * share
        i = next(i for i in range(n) if cum[i + 1] >= T and r[i] > 0)
        new.append(e[i] + (T - cum[i]) / r[i] * (e[i + 1] - e[i]))
    new.append(mp.mpf(1))
    return [float(v) for v in new]


def test_refinement_hand_worked_example():
    e = [0.0, 0.25, 0.5, 0.75, 1.0]
    for h in ([1.0, 0.0, 0.0, 0.0], [4.0, 1.0, 0.5, 2.0], [0.0, 3.0, 0.0, 0.0]):
        out = O.vegas_refine(np.array([h]), np.array([e]), 1.5)[0]
        np.testing.assert_allclose(out, hand_refine(h, e, 1.5), rtol=1e-14, atol=1e-15)
    # first example by hand: smoothed (1/2, 1/3, 0, 0), rho = (3/5, 2/5, 0, 0)
    r0 = (0.4 / -math.log(0.6)) ** 1.5
    r1 = (0.6 / -math.log(0.4)) ** 1.5
    share = (r0 + r1) / 4
    out = O.vegas_refine(np.array([[1.0, 0, 0, 0]]), np.array([e]), 1.5)[0]
    assert abs(out[1] - share / r0 * 0.25) < 1e-15
    assert abs(out[2] - (0.25 + (2 * share - r0) / r1 * 0.25)) < 1e-15 \
        if 2 * share > r0 else abs(out[2] - 2 * share / r0 * 0.25) < 1e-15


def test_refined_edges_strictly_increase():
    rng = np.random.default_rng(5)
    for _ in range(50):
        D, nb = 4, 50
        g = uniform_grid(D, nb)
        h = rng.exponential(size=(D, nb)) ** 3
        h[:, rng.integers(0, nb, 10)] = 0.0
        out = O.vegas_refine(h, g, 1.5)
        assert np.all(np.diff(out, axis=1) > 0)
        assert np.all(out[:, 0] == 0.0) and np.all(out[:, -1] == 1.0)


def test_vegas_adapts_and_integrates_product_of_powers():
    """VEGAS on prod_d 3 x_d^2 over the unit cube (exact integral 1): the
    estimate agrees within its error and the grid adaptation cuts the variance."""
    D, nb, N = 3, 50, 20000
    g = uniform_grid(D, nb)
    rng = np.random.default_rng(11)
    variances, estimates = [], []
    for it in range(6):
        k = rng.integers(0, 2**53, (N, D))
        w = np.empty(N)
        hist = np.zeros((D, nb))
        for e in range(N):
            bins, deltas = zip(*(O.bin_from_k53(int(v), nb) for v in k[e]))
            x, jac = O.vegas_map(g, bins, deltas)
            w[e] = jac * np.prod(3 * x**2)
            for d in range(D):
                hist[d, bins[d]] += w[e] ** 2
        I = w.mean()
        V = (np.mean(w**2) - I * I) / (N - 1)
        estimates.append(I)
        variances.append(V)
        g = O.vegas_refine(hist, g, 1.5)
    sigma, err, chi2 = O.combine(estimates, variances)
    assert abs(sigma - 1.0) < 4 * err
    assert variances[-1] < 0.2 * variances[0]
