"""Pins of the oracle's estimates against what the paper and the mathematics
fix: exact integrals, closed-form variances, brute-force quadrature at D <= 3,
the optimal-grid fixed point (Eq. onedopt), the allocation rule's exponent
(Eqs. dh, nh), the combination formulas (Sec. 2.5) and the paper's printed
accuracies for its own examples (Sec. 2.4)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_2009_05112_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- estimates
def test_constant_integrand_is_exact(orc):
    lo, hi = np.array([0.0, 0.0, 1.0]), np.array([2.0, 0.5, 4.0])
    p = W.Params(dim=3, n_ev=3000, n_g=40, n_iter=3, lower=lo, upper=hi, seed=4)
    r = orc.Problem(p, W.const(3)).integrate()
    np.testing.assert_allclose(r["I"], 3.0, rtol=1e-12)
    # sigma is zero up to the cancellation floor of the one-pass variance
    # Omega^2 S2/n - (Omega S1/n)^2 (about sqrt(eps / N_tot) relative)
    assert np.all(r["sig"] <= 3.0 * math.sqrt(4 * 2.3e-16 / 729))


def test_gaussian_d4_closed_form(orc):
    p, f = W.cfg_small_d4()
    r = orc.Problem(p, f).integrate()
    assert abs(r["mean"] - 1.0) < 5 * r["sdev"]
    assert r["sdev"] < 1e-3
    assert r["chi2"] / r["dof"] < 3.0
    assert r["ties"] == 0


def test_diagonal_gaussians_d8(orc):
    p, f = W.cfg_diag_d8(n_ev=200_000)
    r = orc.Problem(p.with_(n_iter=8, n_discard=3), f).integrate()
    assert abs(r["mean"] - 1.0) < 5 * r["sdev"]
    assert r["sdev"] < 0.05


def test_pull_distribution(orc):
    cen = np.array([[0.3, 0.6], [0.7, 0.4]])
    f = W.Integrand("gauss_mix", 2, cen, [40.0, 60.0], [1.0, 0.5])
    exact = W.gauss_mix_exact(cen, [40.0, 60.0], [1.0, 0.5])
    pulls = []
    for seed in range(40):
        p = W.Params(dim=2, n_ev=4000, n_g=50, n_iter=6, seed=seed, n_discard=2)
        r = orc.Problem(p, f).integrate()
        pulls.append((r["mean"] - exact) / r["sdev"])
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 0.6
    assert 0.6 < pulls.std() < 1.5


def _grid_quad(fun, dim, n):
    x = (np.arange(n) + 0.5) / n
    mesh = np.meshgrid(*([x] * dim), indexing="ij")
    pts = np.stack([m.ravel() for m in mesh], axis=1)
    return fun(pts).mean()


@pytest.mark.parametrize("dim", [2, 3])
def test_bruteforce_quadrature(orc, dim):
    # non-separable peaks exp(-a|x - r|) (Eq. exponentials in low dimension)
    cen = np.array([[0.3] * dim, [0.65] * dim])
    a = np.array([12.0, 20.0])
    amps = np.array([1.0, 2.0])
    f = W.Integrand("exp_abs", dim, cen, a, amps)

    def g(x):
        return sum(amps[k] * np.exp(-a[k] * np.linalg.norm(x - cen[k], axis=1)) for k in range(2))

    quad = _grid_quad(g, dim, 2000 if dim == 2 else 240)
    p = W.Params(dim=dim, n_ev=40_000, n_g=100, n_iter=8, seed=9, n_discard=3)
    r = orc.Problem(p, f).integrate()
    assert abs(r["mean"] - quad) < 5 * r["sdev"] + 1e-5 * quad


def test_affine_variance_closed_form(orc):
    # f = x_0, identity map (alpha = 0), uniform allocation (beta = 0): each
    # hypercube's J f is uniform on an interval of width 1/N_st, so
    # E[V] = Omega (1/N_st)^2 / (12 n) and I = 1/2 (Sec. 2.1, Eq. sigest).
    p = W.Params(dim=3, n_ev=40_000, n_g=60, n_iter=1, alpha=0.0, beta=0.0, seed=2)
    pr = orc.Problem(p, W.affine([0.0, 1.0, 0.0, 0.0]))
    r = pr.integrate()
    nst, nhc = pr.n_st, pr.n_hc
    n = p.n_ev // nhc
    ev = (1.0 / nhc) * (1.0 / nst) ** 2 / (12.0 * n)
    assert abs(r["V"][0] / ev - 1.0) < 0.05
    assert abs(r["I"][0] - 0.5) < 5 * math.sqrt(ev)


# ---------------------------------------------------------------- sampling
def test_stratification_structure(orc):
    p = W.Params(dim=3, n_ev=3000, n_g=30, seed=7, hist_mode="literal")
    pr = orc.Problem(p, W.gauss_single(3, coef=10.0))
    rng = np.random.default_rng(1)
    n_h = rng.integers(2, 10, size=pr.n_hc).astype(np.int32)
    idx, t = pr.sample_indices(n_h, it=3, with_t=True)
    ns, R = pr.n_st, p.n_g / pr.n_st
    h_of = np.repeat(np.arange(pr.n_hc), n_h)
    k = np.stack([(h_of // ns ** (2 - m)) % ns for m in range(3)], axis=1)
    lo, hi = k * R, (k + 1) * R
    assert np.all(t >= lo - 1e-12) and np.all(t <= hi * (1 + 1e-15))
    assert stats.kstest(((t / R) - k).ravel(), "uniform").pvalue > 1e-3
    fmap = pr.map_init()
    out = pr.sample_range(fmap, n_h, it=3)
    # literal mode: W counts samples per increment; every axis sees all of them
    np.testing.assert_array_equal(out["W"].sum(axis=1), np.full(3, n_h.sum()))
    for m in range(3):
        np.testing.assert_array_equal(out["W"][m], np.bincount(idx[:, m], minlength=p.n_g))
    # weighted mode: each hypercube contributes n_h * (1/n_h) = 1 on every axis
    pw = orc.Problem(p.with_(hist_mode="weighted"), W.gauss_single(3, coef=10.0))
    ow = pw.sample_range(fmap, n_h, it=3)
    np.testing.assert_allclose(ow["W"].sum(axis=1), pr.n_hc, rtol=1e-12)
    hs = ow["H"].sum(axis=1)
    np.testing.assert_allclose(hs, hs[0], rtol=1e-12)


def test_identity_map_reproduces_plain_stratified_mc(orc):
    # N_g = 1: x = y exactly and J = 1, so J f is f at the stratified point
    p = W.Params(dim=2, n_ev=400, n_g=1, seed=11)
    f = W.gauss_single(2, coef=5.0)
    pr = orc.Problem(p, f)
    n_h = pr.alloc_init()
    out = pr.sample_range(pr.map_init(), n_h, it=0, records=int(n_h.sum()))
    np.testing.assert_array_equal(out["rec"]["jac"], 1.0)
    idx, t = pr.sample_indices(n_h, it=0, with_t=True)
    y = t / p.n_g
    fy = np.array([pr.f_eval(yy) for yy in y])
    np.testing.assert_allclose(out["rec"]["v"], fy, rtol=1e-15)


# ---------------------------------------------------------------- reallocation
def _sums_for_sigma(orc, pr, sig, n):
    # S1, S2 that give the hypercube standard deviations sig (Sec. 3 step 2)
    om = 1.0 / pr.n_hc
    m = 1.0
    S1 = m * n / om
    S2 = (sig ** 2 + m ** 2) * n / om ** 2
    return S1, S2


@pytest.mark.parametrize("beta", [0.5, 0.75, 1.0])
def test_allocation_exponent(orc, beta):
    p = W.Params(dim=2, n_ev=2_000_000, n_g=10, beta=beta)
    pr = orc.Problem(p, W.const(2), n_st=30)  # 900 hypercubes, ~2000 samples each
    rng = np.random.default_rng(3)
    n = np.full(pr.n_hc, 4, dtype=np.int32)
    sig = np.exp(rng.uniform(-3, 3, size=pr.n_hc))
    S1, S2 = _sums_for_sigma(orc, pr, sig, n.astype(float))
    new, ties = pr.realloc(S1, S2, n)
    assert new.min() >= 2
    assert p.n_ev - pr.n_hc <= new.sum() <= p.n_ev + 2 * pr.n_hc
    big = new >= 200
    slope = np.polyfit(np.log(sig[big]), np.log(new[big]), 1)[0]
    assert abs(slope - beta) < 0.01  # n_h proportional to sigma_h^beta


def test_beta_zero_is_uniform_and_plus2(orc):
    p = W.Params(dim=3, n_ev=10_000, n_g=10, beta=0.0)
    pr = orc.Problem(p, W.const(3))
    rng = np.random.default_rng(8)
    n = rng.integers(2, 20, size=pr.n_hc).astype(np.int32)
    S1, S2 = _sums_for_sigma(orc, pr, rng.random(pr.n_hc), n.astype(float))
    new, _ = pr.realloc(S1, S2, n)
    assert np.all(new == p.n_ev // pr.n_hc)
    p2 = orc.Problem(p.with_(beta=1.0, realloc_plus2=True), W.const(3))
    new2, _ = p2.realloc(S1, S2, n)
    assert new2.min() >= 2
    pz = orc.Problem(p.with_(beta=0.75), W.const(3))
    same, _ = pz.realloc(np.full(pr.n_hc, 5.0 * pr.n_hc), np.full(pr.n_hc, 5.0 * pr.n_hc ** 2), np.full(pr.n_hc, 5, np.int32))
    # zero variance everywhere: sum d = 0, allocation kept
    assert np.all(same == 5)


@pytest.mark.parametrize("n_ev", [6084, 24700, 65_535])
def test_single_hypercube_keeps_every_sample(orc, n_ev):
    """With one hypercube d_h equals its own sum, so the allocation is N_ev for
    any sigma: the rule must not lose a sample to rounding."""
    p = W.Params(dim=14, n_ev=n_ev, n_g=10, beta=0.75)
    pr = orc.Problem(p, W.const(14))
    assert pr.n_hc == 1
    rng = np.random.default_rng(n_ev)
    for sig in np.exp(rng.uniform(-30, 5, size=200)):
        S1, S2 = _sums_for_sigma(orc, pr, np.array([sig]), np.array([float(n_ev)]))
        new, _ = pr.realloc(S1, S2, np.array([n_ev], np.int32))
        assert new[0] == n_ev, sig


# ---------------------------------------------------------------- combination
def test_combination_fixtures(orc):
    g = json.load(open(os.path.join(GOLD, "combine_cases.json")))
    for c in g["cases"]:
        mean, sdev, chi2, dof = orc.combine(c["I"], c["sig"])
        assert mean == pytest.approx(c["mean"], rel=1e-14)
        assert sdev == pytest.approx(c["sdev"], rel=1e-14)
        assert chi2 == pytest.approx(c["chi2"], abs=1e-14)
        assert dof == c["dof"]
    d = g["discard"]
    mean, sdev, chi2, dof = orc.combine(d["I"], d["sig"], d["n_discard"])
    assert (mean, dof) == (pytest.approx(d["mean"]), d["dof"])
    assert sdev == pytest.approx(d["sdev"]) and chi2 == pytest.approx(d["chi2"])
    for c in g["unweighted"]:
        mean, sdev, chi2, dof = orc.combine(c["I"], c["sig"], c["n_discard"], "unweighted")
        assert mean == pytest.approx(c["mean"], rel=1e-14)
        assert sdev == pytest.approx(c["sdev"], rel=1e-14)
        assert (math.isnan(chi2) if c["chi2"] is None else chi2 == pytest.approx(c["chi2"], rel=1e-14))
        assert dof == c["dof"]


# ---------------------------------------------------------------- frozen phase
def test_frozen_phase_keeps_map_and_allocation(orc):
    # Sec. 2.5: after the adapting iterations the map and the allocation stop
    # changing (alpha = 0, and no reallocation), so every later iteration
    # samples the same distribution.
    f = W.gauss_single(3)
    p = W.Params(dim=3, n_ev=20_000, n_g=64, n_iter=3, seed=11)
    head = orc.Problem(p, f).integrate()
    frozen = orc.Problem(p.with_(n_iter=7, n_adapt=3), f).integrate()
    free = orc.Problem(p.with_(n_iter=7), f).integrate()
    assert np.array_equal(frozen["I"][:3], head["I"])
    assert np.array_equal(frozen["map"], head["map"])
    assert np.array_equal(frozen["n_h"], head["n_h"])
    assert not np.array_equal(free["map"], head["map"])
    assert not np.array_equal(free["n_h"], head["n_h"])
    # each frozen iteration: a fresh set of samples (new Philox iteration index)
    assert len(set(frozen["I"][3:].tolist())) == 4


def test_frozen_phase_unweighted_average_is_unbiased(orc):
    # Sec. 2.5: with the map frozen the iterations are independent, identically
    # distributed estimates; their plain average carries no weighting bias and
    # its error is the mean sigma_j over sqrt(count).  Closed form: a single
    # narrow Gaussian in D = 2, exact integral from erf.
    f = W.gauss_single(2)
    n_adapt, n_iter = 6, 46
    p = W.Params(dim=2, n_ev=4_000, n_g=50, n_iter=n_iter, seed=5, n_adapt=n_adapt, n_discard=n_adapt,
                 average="unweighted")
    r = orc.Problem(p, f).integrate()
    kept = r["I"][n_adapt:]
    assert r["mean"] == pytest.approx(kept.mean(), rel=1e-13)
    assert r["sdev"] == pytest.approx(r["sig"][n_adapt:].mean() / math.sqrt(kept.size), rel=1e-13)
    assert r["dof"] == kept.size - 1
    assert abs(r["mean"] - f.exact) < 4 * r["sdev"]
    # the spread of the frozen iterations agrees with their own sigma_j
    assert 0.5 < r["chi2"] / r["dof"] < 2.0


# ---------------------------------------------------------------- the paper's own numbers
def test_optimal_grid_fixed_point(orc):
    # Eq. (onedopt)/(invJ): the converged map for a separable Gaussian puts
    # equal probability mass in every increment: x_i = G^-1(i / N_g).
    f = W.gauss_single(2)
    p = W.Params(dim=2, n_ev=200_000, n_g=100, n_iter=15, seed=3)
    r = orc.Problem(p, f).integrate()
    s = 1 / math.sqrt(200.0)
    q = stats.truncnorm(-0.5 / s, 0.5 / s, loc=0.5, scale=s).ppf(np.arange(101) / 100)
    for mu in range(2):
        assert np.abs(r["map"][mu][10:-10] - q[10:-10]).max() < 0.006


def test_paper_ng_sensitivity(orc):
    # Sec. 2.4, Eq. (easy) with N_ev = 1e4 samples in a plain y-space Monte Carlo
    # (one hypercube): about 11% with N_g = 1 and 0.3% with N_g = 100.
    f = W.easy()
    acc = {}
    for ng in (1, 100):
        rel = []
        for seed in range(4):
            p = W.Params(dim=4, n_ev=10_000, n_g=ng, n_iter=15, seed=seed)
            r = orc.Problem(p, f, n_st=1).integrate()
            rel.append(r["sig"][-5:] / r["I"][-5:])
        acc[ng] = float(np.median(rel))
    assert 0.07 < acc[1] < 0.16
    assert 0.0015 < acc[100] < 0.006


def test_paper_balls_adaptation(orc):
    # Sec. 2.4, Eq. (balls): about 24% before the map adapts (alpha = 0.2,
    # N_ev = 1e5); sub-percent once adapted (here after 50 iterations).
    f = W.balls()
    p = W.Params(dim=4, n_ev=100_000, n_g=1000, n_iter=50, alpha=0.2, seed=0, n_discard=30)
    r = orc.Problem(p, f, n_st=1).integrate()
    rel = r["sig"] / r["I"]
    assert 0.15 < rel[0] < 0.35
    assert rel[-1] < 0.01
    assert abs(r["mean"] - f.exact) < 5 * r["sdev"]


def test_precision_split_tracks_fp64(orc):
    # FP32 map and integrand with FP64 or compensated FP32 sums: same samples up
    # to the 24-bit truncation of u, so the estimates agree far inside sigma.
    p, f = W.cfg_diag_d8(n_ev=100_000)
    out = {}
    for prec in ("fp64", "fp32_acc64", "fp32_neumaier"):
        pr = orc.Problem(p.with_(precision=prec), f)
        out[prec] = pr.iteration(pr.map_init(), pr.alloc_init(), it=0)
    ref = out["fp64"]
    for prec in ("fp32_acc64", "fp32_neumaier"):
        o = out[prec]
        assert abs(o["I"] - ref["I"]) < 0.01 * math.sqrt(ref["V"])
        assert abs(math.sqrt(o["V"]) / math.sqrt(ref["V"]) - 1) < 1e-3
    a, n = out["fp32_acc64"], out["fp32_neumaier"]
    np.testing.assert_allclose(n["S1"], a["S1"], rtol=1e-6, atol=1e-12 * np.abs(a["S1"]).max())
    np.testing.assert_allclose(n["H"], a["H"], rtol=1e-5, atol=1e-9 * a["H"].max())


def test_weighted_training_data_equal_printed_formula_at_uniform_allocation(orc):
    # Sec. 2.3 prints d_i = (1/n_i) sum J^2 f^2; with every n_h equal the
    # weighted form sum(v^2/n_h)/sum(1/n_h) reduces to it exactly.
    p = W.Params(dim=3, n_ev=20_000, n_g=40, seed=3)
    f = W.gauss_single(3, coef=20.0)
    pw = orc.Problem(p, f)
    pl = orc.Problem(p.with_(hist_mode="literal"), f)
    fmap, n_h = pw.map_init(), pw.alloc_init()
    a = pw.sample_range(fmap, n_h, 0)
    b = pl.sample_range(fmap, n_h, 0)
    dw = np.where(a["W"] > 0, a["H"] / np.where(a["W"] > 0, a["W"], 1), 0)
    dl = np.where(b["W"] > 0, b["H"] / np.where(b["W"] > 0, b["W"], 1), 0)
    np.testing.assert_allclose(dw, dl, rtol=1e-12, atol=0)


def test_weighted_training_data_unbiased_under_adapted_allocation(orc):
    # Sec. 3: the optimal map does not depend on the allocation.  Under any
    # allocation n_h, E[sum over increment i of (J f)^2 / n_h] equals N_hc times
    # the integral of (J f)^2 over the increment's slab of y, and
    # E[sum of 1 / n_h] equals N_hc / N_g, so d_i = H_i / W_i estimates N_g times
    # the slab integral of (J f)^2 -- what the map is refined on -- whatever the
    # allocation.  Closed form for a separable Gaussian on the identity map
    # (J = 1), averaged over independent iterations, with an allocation that
    # puts more samples near the peak; the count-normalised printed formula is
    # biased there.
    D, NG, a, c = 2, 16, 8.0, 0.3
    p = W.Params(dim=D, n_ev=4000, n_g=NG, seed=11)
    f = W.gauss_single(D, coef=a, c=c)
    pw = orc.Problem(p, f)
    pl = orc.Problem(p.with_(hist_mode="literal"), f)
    fmap = pw.map_init()
    nst = pw.n_st
    centres = (np.arange(nst) + 0.5) / nst
    g = np.exp(-a * (centres - c) ** 2)
    rng = np.random.default_rng(5)
    n_h = (2 + np.floor(58 * np.outer(g, g)).astype(np.int64) + rng.integers(0, 3, (nst, nst))).ravel()
    assert n_h.min() >= 2 and n_h.max() > 20 * n_h.min()
    n_h = n_h.astype(np.int32)

    def g2_int(lo, hi):  # integral of exp(-2 a (y - c)^2) over [lo, hi]
        s = math.sqrt(2 * a)
        return math.sqrt(math.pi / (8 * a)) * (math.erf(s * (hi - c)) - math.erf(s * (lo - c)))

    scale2 = f.scale ** 2
    exact = np.array([NG * g2_int(i / NG, (i + 1) / NG) * g2_int(0.0, 1.0) * scale2 for i in range(NG)])
    R = 40
    dw = np.empty((R, NG))
    dl = np.empty((R, NG))
    for it in range(R):
        A = pw.sample_range(fmap, n_h, it)
        B = pl.sample_range(fmap, n_h, it)
        dw[it] = A["H"][0] / A["W"][0]
        dl[it] = B["H"][0] / B["W"][0]
    zw = (dw.mean(0) - exact) / (dw.std(0, ddof=1) / math.sqrt(R))
    zl = (dl.mean(0) - exact) / (dl.std(0, ddof=1) / math.sqrt(R))
    print(f"weighted: max |z| {np.abs(zw).max():.2f}; printed formula: max |z| {np.abs(zl).max():.1f}")
    assert np.abs(zw).max() < 5.0
    assert np.abs(zl).max() > 10.0


@pytest.mark.parametrize("beta", [1.0, 0.5])
def test_plus2_rule_exact_counts(orc, beta):
    """Sec. 3 step 4, the alternative to Eq. nh: n_h = floor(q) + 2 with
    q = N_ev d_h / sum d.  The injected sigma_h make every q an exact
    half-integer m_h + 1/2 (far from any rounding boundary): d_h = 2 m_h + 1
    and N_ev = (sum d) / 2.  The +2 rule must give m_h + 2, the default rule
    max(2, m_h)."""
    p = W.Params(dim=2, n_ev=1000, n_g=10, beta=beta)
    pr = orc.Problem(p, W.const(2), n_st=4)   # 16 hypercubes
    m = np.array([0, 1, 2, 3, 5, 8, 13, 0, 1, 21, 34, 2, 4, 6, 7, 9])
    d = 2 * m + 1
    assert d.sum() % 2 == 0
    n_ev = int(d.sum()) // 2
    sig = d.astype(float) ** (1.0 / beta)
    n = np.full(pr.n_hc, 4, dtype=np.int32)
    S1, S2 = _sums_for_sigma(orc, pr, sig, n.astype(float))
    q = n_ev * d / d.sum()
    np.testing.assert_array_equal(q, m + 0.5)
    plus2 = orc.Problem(p.with_(n_ev=n_ev, realloc_plus2=True), W.const(2), n_st=4)
    got, ties = plus2.realloc(S1, S2, n)
    np.testing.assert_array_equal(got, m + 2)
    assert ties == 0
    plain = orc.Problem(p.with_(n_ev=n_ev), W.const(2), n_st=4)
    got0, _ = plain.realloc(S1, S2, n)
    np.testing.assert_array_equal(got0, np.maximum(2, m))


def test_sample_points_consistent(orc):
    """The per-sample view (h, j, increment indices, x, J, f) agrees with the
    index enumeration, with the recorded values v = J f of the sampling pass,
    and with the map: x lies in its increment, J is the product of N_g dx."""
    p = W.Params(dim=3, n_ev=5000, n_g=17, seed=4)
    f = W.gauss_single(3, coef=20.0)
    pr = orc.Problem(p, f)
    rng = np.random.default_rng(2)
    x0 = np.sort(rng.random((3, 16)), axis=1)
    fmap = np.concatenate([np.zeros((3, 1)), x0, np.ones((3, 1))], axis=1)
    n_h = rng.integers(2, 9, size=pr.n_hc).astype(np.int32)
    pts = pr.sample_points(fmap, n_h, it=2)
    ns = int(n_h.sum())
    np.testing.assert_array_equal(pts["h"], np.repeat(np.arange(pr.n_hc), n_h))
    np.testing.assert_array_equal(pts["j"], np.concatenate([np.arange(n) for n in n_h]))
    np.testing.assert_array_equal(pts["idx"], pr.sample_indices(n_h, it=2))
    rec = pr.sample_range(fmap, n_h, 2, records=ns)["rec"]
    np.testing.assert_array_equal(pts["jac"], rec["jac"])
    np.testing.assert_array_equal(pts["fx"], rec["fx"])
    np.testing.assert_array_equal(pts["jac"] * pts["fx"], rec["v"])
    for m in range(3):
        lo = fmap[m, pts["idx"][:, m]]
        hi = fmap[m, pts["idx"][:, m] + 1]
        assert np.all((pts["x"][:, m] >= lo) & (pts["x"][:, m] <= hi))
    dx = np.stack([fmap[m, pts["idx"][:, m] + 1] - fmap[m, pts["idx"][:, m]] for m in range(3)], axis=1)
    np.testing.assert_allclose(pts["jac"], np.prod(p.n_g * dx, axis=1), rtol=1e-14)
    np.testing.assert_allclose(pts["fx"], [pr.f_eval(x) for x in pts["x"]], rtol=1e-15)
