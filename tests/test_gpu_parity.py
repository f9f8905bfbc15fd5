"""GPU parity: the HIP path through the C ABI against the CPU oracle."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_checks import assert_integration_parity

pytestmark = pytest.mark.gpu

SQRT_S = 13000.0
CONF = {
    2: dict(process="gg_ttx"),
    3: dict(process="gg_ttxg", ptmin_g=20.0, etamax_g=2.5),
    4: dict(process="gg_ttxgg", ptmin_g=20.0, drmin_gg=0.4),
}


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10279_amd import api
    return api


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gproc(api, n_g, **kw):
    c = dict(CONF[n_g])
    c.update(kw)
    return api.Process(**c)


def oproc(n_g, **kw):
    c = {k: v for k, v in CONF[n_g].items() if k != "process"}
    c.update(kw)
    return O.Process(n_g=n_g, **c)


def uniform_grid(D, nb=50):
    return np.tile(np.arange(nb + 1) / nb, (D, 1))


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_philox_words_and_bins_bit_exact(api, pdf_table, n_g):
    say(f"philox/bins n_g={n_g}")
    D = 2 + 3 * n_g - 4
    n = 4100
    for seed, it in ((0, 0), (3, 7), (2**40 + 5, 2)):
        w, k53, bins = api.evaluate_weights(gproc(api, n_g), SQRT_S, pdf_table, n, seed=seed,
                                            it=it, return_k53=True, return_bins=True)
        k53 = k53.cpu().numpy().astype(np.uint64)
        bins = bins.cpu().numpy()
        for e in list(range(0, n, 37)) + [n - 1]:
            ref = O.event_k53(seed, it, e, D)
            assert np.array_equal(k53[e], ref), (seed, it, e)
            assert list(bins[e]) == [O.bin_from_k53(int(k), 50)[0] for k in ref]


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_matrix_element_fp64(api, n_g):
    import torch
    say(f"matrix element n_g={n_g}")
    rng = np.random.default_rng(100 + n_g)
    M = 173.0
    moms, ebs, refs = [], [], []
    for _ in range({2: 200, 3: 100, 4: 40}[n_g]):
        rs = 2 * M + 60.0 + rng.exponential(600.0)
        k, w, st = O.phase_space(n_g, [M, M] + [0.0] * (n_g - 2), rs, rng.random(3 * n_g - 4))
        E = rs / 2
        p = np.array([k[0], k[1], [-E, 0, 0, -E], [-E, 0, 0, E]] + [k[i] for i in range(2, n_g)])
        refs.append(O.me2_sum(n_g, p, M, 1.5))
        moms.append(k.reshape(-1))
        ebs.append(E)
    mom = torch.tensor(np.array(moms), dtype=torch.float64, device="cuda").contiguous()
    eb = torch.tensor(np.array(ebs), dtype=torch.float64, device="cuda")
    got = api.matrix_element(CONF[n_g]["process"], mom, eb, 173.0, 1.5).cpu().numpy()
    rel = np.abs(got / np.array(refs) - 1)
    say("  max rel", rel.max())
    assert rel.max() < 1e-12
    got32 = api.matrix_element(CONF[n_g]["process"], mom, eb, 173.0, 1.5,
                               precision="fp32_kahan").cpu().numpy()
    rel32 = np.abs(got32 / np.array(refs) - 1)
    say("  fp32 max rel", rel32.max(), "median", np.median(rel32))
    assert np.median(rel32) < 1e-4


def compare_weights(got, ref, near, tol=1e-12):
    ok = ~near
    denom = np.maximum(np.abs(ref), 1e-300)
    rel = np.where(ok, np.abs(got - ref) / denom, 0.0)
    zero = ref == 0.0
    assert np.all(got[zero & ok] == 0.0)
    return rel.max()


@pytest.mark.parametrize("n_g,n", [(2, 3000), (3, 1500), (4, 300)])
def test_event_weights_match_oracle(api, pdf_table, n_g, n):
    """Per-event weights and every stage of the per-event record."""
    say(f"weights n_g={n_g} n={n}")
    D = 2 + 3 * n_g - 4
    rng = np.random.default_rng(n_g)
    grids = [uniform_grid(D)]
    # a non-trivial grid: one oracle refinement from a random histogram
    grids.append(O.vegas_refine(rng.exponential(size=(D, 50)) ** 2, uniform_grid(D)))
    gs2n = (4 * math.pi * 0.118) ** n_g / (256 * math.factorial(n_g - 2))
    for gi, grid in enumerate(grids):
        w, rec = api.evaluate_weights(gproc(api, n_g), SQRT_S, pdf_table, n, seed=1, it=2,
                                      grid=grid, return_record=True)
        w = w.cpu().numpy()
        rec = rec.cpu().numpy()
        ref = np.zeros(n)
        near = np.zeros(n, dtype=bool)
        stage = {k: np.zeros(n) for k in ("x", "jac", "W", "f", "me", "k")}
        for e in range(n):
            ref[e], ev = O.event_weight(oproc(n_g), SQRT_S, pdf_table, grid, 1, 2, e)
            near[e] = ev.near_edge or ev.ill_conditioned
            r = rec[e]
            stage["x"][e] = max(abs(r[0] - ev.x[0]), abs(r[1] - ev.x[1]))
            stage["jac"][e] = abs(r[2] / ev.jac - 1)
            if ev.pass_threshold and not ev.newton_fail:
                stage["W"][e] = abs(r[3] / ev.ps_weight - 1)
                kk = r[8:8 + 4 * n_g].reshape(n_g, 4)
                stage["k"][e] = np.abs(kk - ev.k[:n_g]).max() / math.sqrt(ev.shat)
            if ev.pass_cuts:
                stage["f"][e] = max(abs(r[4] / ev.f1 - 1), abs(r[5] / ev.f2 - 1))
                stage["me"][e] = abs(r[6] * gs2n / ev.me2 - 1)
        rel = compare_weights(w, ref, near)
        worst = int(np.argmax(np.where(near, 0.0, np.abs(w - ref) / np.maximum(np.abs(ref), 1e-300))))
        say(f"  grid {gi}: weight max rel {rel:.3e} (event {worst}); nonzero {int((ref != 0).sum())},"
            f" excluded (cut edge or ill-conditioned PDF) {int(near.sum())}")
        say("   stages: " + ", ".join(f"{k} {v.max():.2e}@{int(np.argmax(v))}" for k, v in stage.items()))
        say(f"   worst event stages: " + ", ".join(f"{k} {v[worst]:.2e}" for k, v in stage.items()))
        assert stage["x"].max() == 0.0 and stage["jac"].max() == 0.0
        assert rel < 1e-12


def test_explicit_uniforms_path(api, pdf_table):
    import torch
    n_g, n = 3, 700
    D = 7
    y = W.random_uniforms(n, D, 5)
    w = api.evaluate_weights(gproc(api, n_g), SQRT_S, pdf_table, n,
                             y=torch.tensor(y, device="cuda")).cpu().numpy()
    grid = uniform_grid(D)
    for e in range(n):
        ref, ev = O.event_weight_y(oproc(n_g), SQRT_S, pdf_table, grid, y[e])
        if not (ev.near_edge or ev.ill_conditioned):
            assert abs(w[e] - ref) <= 1e-12 * abs(ref), e


@pytest.mark.parametrize("n_g,n,iters", [(2, 20_000, 3), (3, 3_000, 2), (4, 700, 2)])
def test_integration_matches_oracle(api, pdf_table, n_g, n, iters):
    say(f"integrate n_g={n_g} n={n} iters={iters}")
    g = api.integrate(gproc(api, n_g), SQRT_S, pdf_table, n, iters, seed=0)
    o = O.integrate(oproc(n_g), SQRT_S, pdf_table, n, iters, seed=0)
    say("  gpu", g.sigma, g.sigma_err, g.chi2_dof, "oracle", o.sigma, o.sigma_err, o.chi2_dof)
    assert_integration_parity(g, o, n, say=say)
    w = g.weights.cpu().numpy()
    np.testing.assert_allclose(w, o.weights_last, rtol=1e-11, atol=0)
    assert g.n_pass == o.n_pass and g.n_newton_fail == o.n_newton_fail


@pytest.mark.parametrize("n_g", [2, 4])
def test_stage_isolated_refinement(api, pdf_table, n_g):
    """The oracle's refinement of the GPU's own histogram reproduces the GPU grid,
    and the GPU histogram matches the oracle's."""
    D = 2 + 3 * n_g - 4
    n = 5000 if n_g == 2 else 500
    g = api.integrate(gproc(api, n_g), SQRT_S, pdf_table, n, 1, seed=7)
    o = O.integrate(oproc(n_g), SQRT_S, pdf_table, n, 1, seed=7)
    np.testing.assert_allclose(O.vegas_refine(g.hist, uniform_grid(D)), g.grid, rtol=0, atol=1e-14)
    np.testing.assert_allclose(g.hist, o.hist_last, rtol=1e-11, atol=0)


def test_refine_kernel_matches_oracle(api):
    import torch
    rng = np.random.default_rng(9)
    for D, nb in ((4, 50), (10, 50), (3, 7), (1, 200)):
        hist = rng.exponential(size=(D, nb)) ** 3
        hist[:, rng.integers(0, nb, max(1, nb // 5))] = 0.0
        grid = O.vegas_refine(rng.exponential(size=(D, nb)), uniform_grid(D, nb))
        out = api.refine_grid(torch.tensor(hist, device="cuda"), torch.tensor(grid, device="cuda"))
        np.testing.assert_allclose(out.cpu().numpy(), O.vegas_refine(hist, grid), rtol=0, atol=1e-14)


def test_run_to_run_bit_identical(api, pdf_table):
    a = api.integrate(gproc(api, 3), SQRT_S, pdf_table, 50_000, 2, seed=4)
    b = api.integrate(gproc(api, 3), SQRT_S, pdf_table, 50_000, 2, seed=4)
    assert a.sigma == b.sigma and np.array_equal(a.grid, b.grid)
    assert np.array_equal(a.weights.cpu().numpy(), b.weights.cpu().numpy())


@pytest.mark.parametrize("n", [2, 63, 65, 129])
def test_ragged_and_tiny_sizes(api, pdf_table, n):
    g = api.integrate(gproc(api, 2), SQRT_S, pdf_table, n, 1, seed=0)
    o = O.integrate(oproc(2), SQRT_S, pdf_table, n, 1, seed=0)
    np.testing.assert_allclose(g.weights.cpu().numpy(), o.weights_last, rtol=1e-12, atol=0)
    assert abs(g.iter_sigma[0] - o.iter_sigma[0]) <= 1e-12 * abs(o.iter_sigma[0])


def test_newton_failure_counted_and_strict(api, pdf_table):
    from paper_2106_10279_amd import _lib
    g = api.integrate(gproc(api, 3), SQRT_S, pdf_table, 1000, 1, seed=0, max_newton=0)
    o = O.integrate(oproc(3), SQRT_S, pdf_table, 1000, 1, seed=0)
    assert g.n_newton_fail > 0 and g.sigma == 0.0
    with pytest.raises(_lib.MFError) as e:
        api.integrate(gproc(api, 3), SQRT_S, pdf_table, 1000, 1, seed=0, max_newton=0, strict=True)
    assert e.value.status == _lib.MF_ENOCONV


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_three_kernel_integration_weights_equal_the_fused_kernel(api, pdf_table, n_g):
    """The integration runs phase space, amplitudes and accumulation as three
    kernels; its per-event weights are bit for bit those of the fused event
    kernel (mf_evaluate) on the same events and grid, also when the iteration
    is split into many batches."""
    import torch
    if n_g == 2:
        proc = api.Process("gg_ttx")
    else:
        proc = api.Process({3: "gg_ttxg", 4: "gg_ttxgg"}[n_g], ptmin_g=20.0,
                           etamax_g=2.5 if n_g == 3 else 0.0, drmin_gg=0.4 if n_g == 4 else 0.0)
    N = 5000
    g1 = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, keep_weights=False).grid
    r = api.integrate(proc, SQRT_S, pdf_table, N, 2, 0, keep_weights=True)
    assert r.n_batches == 1
    w_fused = api.evaluate_weights(proc, SQRT_S, pdf_table, N, seed=0, it=1, grid=g1)
    assert torch.equal(r.weights, w_fused)
    # many batches: same events, sums continued across batches in another order
    r1 = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, keep_weights=True)
    rb = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, keep_weights=True, max_batch=777)
    assert rb.n_batches == (N + 776) // 777
    assert torch.equal(rb.weights, r1.weights)
    assert rb.iter_sigma[0] == pytest.approx(r1.iter_sigma[0], rel=1e-13)
    assert rb.iter_var[0] == pytest.approx(r1.iter_var[0], rel=1e-11)
    assert np.allclose(rb.hist, r1.hist, rtol=1e-13, atol=0)
    assert np.allclose(rb.grid, r1.grid, rtol=0, atol=1e-13)
    assert rb.n_pass == r1.n_pass
