"""GPU parity: the HIP path against the CPU oracle, element by element.

Step-wise tests inject the GPU's state (map, allocation, iteration index)
into the oracle for every iteration and compare all outputs: per-hypercube
sums, training data, the iteration estimate, the next allocation (exactly)
and the refined map.  Literal-mode runs compare per-increment sample counts
exactly, which pins every sample's increment indices bit for bit.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2009_05112_amd import _binding as B
from paper_2009_05112_amd import workloads as W
from tests.parity import RTOL64, assert_close, step_and_compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def _pair(ctx, params, f, n_st=0):
    gp = B.Problem(ctx, params, f, n_st=n_st)
    op = oracle.Problem(params, f, n_st=gp.n_st)
    assert gp.n_hc == op.n_hc
    return gp, op


def test_initial_state_matches(ctx):
    p, f = W.cfg_small_d4()
    gp, op = _pair(ctx, p, f)
    assert gp.n_st == 12 and gp.n_hc == 12 ** 4
    np.testing.assert_array_equal(gp.map(), op.map_init())
    np.testing.assert_array_equal(gp.alloc(), op.alloc_init())


@pytest.mark.parametrize("hist_mode", ["weighted", "literal"])
def test_stepwise_cfg_small_d4(ctx, hist_mode):
    """D=4 Gaussian, N_ev=1e5, N_g=1000: ten iterations, each compared."""
    p, f = W.cfg_small_d4()
    p = p.with_(hist_mode=hist_mode)
    gp, op = _pair(ctx, p, f)
    for _ in range(p.n_iter):
        step_and_compare(gp, op, exact_counts=(hist_mode == "literal"))
    r = gp.result()
    assert abs(r["mean"] - 1.0) < 5 * r["sdev"]


def test_end_to_end_cfg_small_d4(ctx):
    """Independent runs of the whole D=4 problem agree iteration by iteration."""
    p, f = W.cfg_small_d4()
    gp, op = _pair(ctx, p, f)
    ro = op.integrate()
    gp.iterate(p.n_iter)
    rg = gp.result()
    assert ro["ties"] == 0 and rg["ties"] == 0
    assert_close(rg["I"], ro["I"], RTOL64, what="I_j")
    assert_close(rg["V"], ro["V"], RTOL64, what="V_j")
    assert_close(rg["sig"], np.sqrt(ro["V"]), RTOL64, what="sigma_j")  # returned by the library
    np.testing.assert_array_equal(rg["sig"], np.sqrt(rg["V"]))
    assert_close(rg["mean"], ro["mean"], RTOL64, what="mean")
    assert_close(rg["sdev"], ro["sdev"], RTOL64, what="sdev")
    assert_close(rg["chi2"], ro["chi2"], 1e-9, what="chi2")
    np.testing.assert_array_equal(gp.alloc(), ro["n_h"])
    assert_close(gp.map(), ro["map"], RTOL64, scale=np.ones_like(ro["map"]), what="map")
    assert rg["n_iter_done"] == p.n_iter and rg["n_evals"] >= p.n_iter * 2 * gp.n_hc


def test_stepwise_diag_d8_mid(ctx):
    """D=8 three diagonal Gaussians at N_ev=1e6 (N_st=4): adapted,
    non-uniform allocations with large hypercubes spanning many waves."""
    p, f = W.cfg_diag_d8(n_ev=1_000_000)
    gp, op = _pair(ctx, p, f)
    assert gp.map_place == "inner"  # the benchmark's layout: two innermost map axes in LDS
    for _ in range(6):
        out = step_and_compare(gp, op)
    n = out["n_new"]
    assert n.max() > 50 * n.min()  # the allocation really adapted


@pytest.mark.parametrize("dim,n_ev,place", [(4, 100_000, "lds"), (9, 300_000, "inner"), (10, 200_000, "global")])
def test_map_placements(ctx, dim, n_ev, place):
    """The three places the FP64 sampler reads the map from (N_g = 1000):
    all of it staged in LDS beside the training data (D=4), only the two
    innermost axes (D=9: 144 KB of training data leave room for two axes),
    or none (D=10), each step-wise against the oracle."""
    p = W.Params(dim=dim, n_ev=n_ev, n_g=1000, n_iter=3, seed=dim + 3)
    f = W.gauss_diag(dim, coef=50.0, cs=(0.3, 0.6))
    gp, op = _pair(ctx, p, f)
    assert gp.map_place == place and gp.hist_axes == dim
    for _ in range(3):
        step_and_compare(gp, op)


def test_stepwise_literal_d8_counts_exact(ctx):
    p, f = W.cfg_diag_d8(n_ev=500_000)
    p = p.with_(hist_mode="literal")
    gp, op = _pair(ctx, p, f)
    for _ in range(3):
        step_and_compare(gp, op, exact_counts=True)


@pytest.mark.parametrize("dim,kind", [(1, "gauss_mix"), (2, "exp_abs"), (3, "balls"), (5, "corr_gauss"),
                                      (6, "affine"), (7, "const"), (13, "corr_gauss"), (16, "gauss_mix"),
                                      (21, "corr_gauss"), (24, "gauss_mix")])
def test_integrand_kinds_and_dims(ctx, dim, kind):
    rng = np.random.default_rng(dim)
    if kind == "gauss_mix":
        f = W.Integrand("gauss_mix", dim, rng.uniform(0.3, 0.7, (2, dim)), [20.0, 40.0], [1.0, 0.5])
    elif kind == "exp_abs":
        f = W.Integrand("exp_abs", dim, rng.uniform(0.3, 0.7, (2, dim)), [10.0, 30.0], [1.0, 2.0])
    elif kind == "balls":
        f = W.Integrand("balls", dim, rng.uniform(0.3, 0.7, (2, dim)), [0.2, 0.3], [1.0, 1.0])
    elif kind == "corr_gauss":
        f = W.corr_gauss(rng, dim, s_max=0.2, cond=10.0)
    elif kind == "affine":
        f = W.affine(rng.uniform(-1, 1, dim + 1))
    else:
        f = W.const(dim, 2.5)
    n_ev = 60_000 if dim <= 8 else 200_000
    p = W.Params(dim=dim, n_ev=n_ev, n_g=64, n_iter=3, seed=dim + 17)
    gp, op = _pair(ctx, p, f)
    for _ in range(3):
        step_and_compare(gp, op)


@pytest.mark.parametrize("dim,n_ev,n_g,prec,hist", [
    (21, 300_000, 1000, "fp64", "weighted"),     # 3 slices of 7 axes, 5 chunks
    (11, 700_000, 1000, "fp64", "literal"),      # 2 slices (6 + 5 axes), counts exact
    (4, 200_000, 4096, "fp64", "weighted"),      # N_g at its maximum: 2 slices of 2 axes
    (21, 5_000, 1000, "fp64", "weighted"),       # one hypercube, one chunk
    (12, 400_000, 1000, "fp32_acc64", "weighted"),
])
def test_training_records_path(ctx, dim, n_ev, n_g, prec, hist):
    """dim * N_g too large for LDS: the sampler writes per-sample training
    records, binned per axis slice in a second pass."""
    rng = np.random.default_rng(dim)
    f = W.corr_gauss(rng, dim, s_max=0.2, cond=10.0)
    p = W.Params(dim=dim, n_ev=n_ev, n_g=n_g, n_iter=2, seed=5, precision=prec, hist_mode=hist)
    gp, op = _pair(ctx, p, f)
    for _ in range(2):
        if prec == "fp64":
            step_and_compare(gp, op, exact_counts=(hist == "literal"))
        else:
            step_and_compare(gp, op, rtol=2e-6, rtol_hist=2e-6, floor=1e-12)


def test_single_hypercube_spans_every_wave(ctx):
    p = W.Params(dim=3, n_ev=2_000_000, n_g=50, n_iter=2, seed=9)
    f = W.gauss_single(3, coef=30.0)
    gp, op = _pair(ctx, p, f, n_st=1)
    assert gp.n_hc == 1
    for _ in range(2):
        step_and_compare(gp, op)


def test_tiny_problems(ctx):
    for dim, n_ev, n_g in [(2, 4, 1), (1, 10, 3), (3, 64, 7), (2, 100, 2)]:
        p = W.Params(dim=dim, n_ev=n_ev, n_g=n_g, n_iter=3, seed=n_ev)
        f = W.gauss_single(dim, coef=3.0)
        gp, op = _pair(ctx, p, f)
        for _ in range(3):
            step_and_compare(gp, op)


def test_identity_map_ng1(ctx):
    """N_g = 1: x = y and J = 1 exactly, so the GPU reproduces plain
    stratified Monte Carlo bit for bit against the oracle's sums."""
    p = W.Params(dim=3, n_ev=50_000, n_g=1, n_iter=2, seed=1)
    f = W.gauss_single(3, coef=10.0)
    gp, op = _pair(ctx, p, f)
    for _ in range(2):
        out = step_and_compare(gp, op)
    np.testing.assert_array_equal(gp.map(), op.map_init())


def test_alpha_zero_beta_zero(ctx):
    p = W.Params(dim=4, n_ev=100_000, n_g=100, n_iter=3, alpha=0.0, beta=0.0, seed=2)
    f = W.gauss_single(4)
    gp, op = _pair(ctx, p, f)
    m0, n0 = gp.map(), gp.alloc()
    gp.iterate(3)
    np.testing.assert_array_equal(gp.map(), m0)
    np.testing.assert_array_equal(gp.alloc(), n0)


@pytest.mark.parametrize("average", ["weighted", "unweighted"])
def test_frozen_phase(ctx, average):
    """Sec. 2.5: three adapting iterations, then four in which neither the map
    nor the allocation changes; the combination over the frozen iterations,
    weighted or plain."""
    p, f = W.cfg_small_d4()
    p = p.with_(n_iter=7, n_adapt=3, n_discard=3, average=average, seed=21)
    gp, op = _pair(ctx, p, f)
    ro = op.integrate()
    for _ in range(3):
        step_and_compare(gp, op)
    m3, n3 = gp.map(), gp.alloc()
    for _ in range(4):
        step_and_compare(gp, op, check_map=False, check_alloc=False)
        np.testing.assert_array_equal(gp.map(), m3)
        np.testing.assert_array_equal(gp.alloc(), n3)
    rg = gp.result()
    np.testing.assert_array_equal(n3, ro["n_h"])
    assert_close(m3, ro["map"], RTOL64, scale=np.ones_like(m3), what="frozen map")
    assert_close(rg["I"], ro["I"], RTOL64, what="I_j")
    assert_close(rg["V"], ro["V"], RTOL64, what="V_j")
    assert_close(rg["mean"], ro["mean"], RTOL64, what="mean")
    assert_close(rg["sdev"], ro["sdev"], RTOL64, what="sdev")
    assert_close(rg["chi2"], ro["chi2"], 1e-9, what="chi2")
    assert rg["dof"] == ro["dof"] == 3
    if average == "unweighted":
        sig = np.sqrt(rg["V"][3:])
        assert rg["mean"] == pytest.approx(rg["I"][3:].mean(), rel=1e-14)
        assert rg["sdev"] == pytest.approx(sig.mean() / 2.0, rel=1e-14)


def test_constant_integrand(ctx):
    lo, hi = np.array([0.0, 0.0, 1.0]), np.array([2.0, 0.5, 4.0])
    p = W.Params(dim=3, n_ev=3000, n_g=40, n_iter=3, lower=lo, upper=hi, seed=4)
    gp, op = _pair(ctx, p, W.const(3))
    for _ in range(3):
        step_and_compare(gp, op)
    r = gp.result()
    assert abs(r["mean"] - 3.0) < 1e-12 * 3.0


def test_checkpoint_resume(ctx):
    p, f = W.cfg_small_d4()
    g1 = B.Problem(ctx, p, f)
    g1.iterate(10)
    r1 = g1.result()
    g2 = B.Problem(ctx, p, f)
    g2.iterate(5)
    blob = g2.export_state()
    g3 = B.Problem(ctx, p, f)
    g3.import_state(blob)
    assert g3.it == 5
    g3.iterate(5)
    r3 = g3.result()
    assert_close(r3["I"], r1["I"], RTOL64, what="I_j after resume")
    assert_close(r3["mean"], r1["mean"], RTOL64, what="mean after resume")
    np.testing.assert_array_equal(g3.alloc(), g1.alloc())


def test_invalid_arguments(ctx):
    f = W.gauss_single(2)
    bad = [W.Params(dim=0, n_ev=100), W.Params(dim=2, n_ev=3), W.Params(dim=2, n_ev=100, n_g=0),
           W.Params(dim=2, n_ev=100, alpha=-1.0), W.Params(dim=2, n_ev=100, beta=-0.5),
           W.Params(dim=25, n_ev=100), W.Params(dim=17, n_ev=100, precision="fp32_acc64"),
           W.Params(dim=2, n_ev=100, n_g=5000)]
    for p in bad:
        ff = W.gauss_single(max(p.dim, 1)) if p.dim != 2 else f
        with pytest.raises(B.VegaspError) as e:
            B.Problem(ctx, p, ff)
        assert e.value.status == B.VP_ERR_INVALID_ARG
    gp = B.Problem(ctx, W.Params(dim=2, n_ev=100, n_g=10), f)
    with pytest.raises(B.VegaspError):
        gp.set_alloc(np.ones(gp.n_hc, dtype=np.int32))
    too_many = np.full(gp.n_hc, 2, dtype=np.int32)
    too_many[0] = 100 + 2 * gp.n_hc  # beyond n_ev + 2 n_hc: the buffers are sized for that bound
    with pytest.raises(B.VegaspError):
        gp.set_alloc(too_many)
    m = gp.map()
    m[0, 3] = m[0, 5]
    m[0, 4] = 0.0
    with pytest.raises(B.VegaspError):
        gp.set_map(m)


def test_nonfinite_reported(ctx):
    f = W.const(2, float("inf"))
    gp = B.Problem(ctx, W.Params(dim=2, n_ev=1000, n_g=10, alpha=0.0, beta=0.0), f)
    gp.iterate(1)
    with pytest.raises(B.VegaspError) as e:
        gp.result()
    assert e.value.status == B.VP_ERR_NUMERIC
    assert gp.result(allow_nonfinite=True)["nonfinite"] > 0


@pytest.mark.parametrize("dim,n_ev,n_iter", [(4, 100_000, 6), (8, 1_000_000, 4)])
def test_stepwise_plus2_rule(ctx, dim, n_ev, n_iter):
    """The alternative allocation rule of Sec. 3 step 4, n_h = floor(q) + 2:
    every iteration compared with the oracle, the next allocation exactly."""
    if dim == 4:
        p, f = W.cfg_small_d4()
    else:
        p, f = W.cfg_diag_d8(n_ev=n_ev)
    p = p.with_(realloc_plus2=True, n_iter=n_iter, seed=31)
    gp, op = _pair(ctx, p, f)
    for _ in range(n_iter):
        out = step_and_compare(gp, op)
    n = out["n_new"]
    assert n.min() >= 2
    # the +2 rule adds two samples to every hypercube's floor(q): the total
    # exceeds N_ev by about 1.5 per hypercube, unlike the max(2, .) rule
    assert n.sum() > p.n_ev + gp.n_hc
