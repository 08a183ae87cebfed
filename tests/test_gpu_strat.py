"""GPU parity of mixed stratification (Sec. 4): per-axis counts from the
mixed rule or given per axis, hypercubes in their mixed radix, every
iteration compared with the oracle run from the same state."""
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


def _pair(ctx, params, f):
    gp = B.Problem(ctx, params, f)
    op = oracle.Problem(params, f)
    assert list(gp.n_st_axes) == list(op.n_st_axes)
    assert gp.n_hc == op.n_hc == int(np.prod(op.n_st_axes.astype(np.int64)))
    return gp, op


def test_mixed_rule_counts(ctx):
    for D, n_ev in ((6, 30_000), (8, 10 ** 6), (16, 250_000), (20, 50_000), (3, 10 ** 7)):
        p = W.Params(dim=D, n_ev=n_ev, n_g=64, strat="mixed")
        gp = B.Problem(ctx, p, W.const(D))
        want, _ = oracle.nst_mixed(D, n_ev)
        assert list(gp.n_st_axes) == list(want), (D, n_ev)
        gp.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_acc64", "fp32_neumaier"])
@pytest.mark.parametrize("hist", ["weighted", "literal"])
def test_stepwise_mixed_rule(ctx, prec, hist):
    """D=6 Gaussian mixture, counts (5, 5, 4, 4, 4, 4): three iterations."""
    f = W.gauss_diag(6, coef=30.0)
    p = W.Params(dim=6, n_ev=30_000, n_g=200, n_iter=3, seed=12, strat="mixed", precision=prec, hist_mode=hist)
    gp, op = _pair(ctx, p, f)
    assert list(gp.n_st_axes) == [5, 5, 4, 4, 4, 4]
    # the split precisions to the bound of their own parity tests (FP32 map
    # and integrand, sums near the FP32 denormal range compared absolutely)
    split = prec != "fp64"
    tol = 2e-6 if split else RTOL64
    for _ in range(3):
        step_and_compare(gp, op, exact_counts=(hist == "literal"), rtol=tol, rtol_hist=tol,
                         floor=1e-12 if split else 0.0)


@pytest.mark.parametrize("counts,n_ev,n_g,kind", [
    ([4, 3, 1, 2, 2], 3_000, 40, "gauss_mix"),
    ([1, 7, 1, 3], 50_000, 500, "exp_abs"),
    ([2, 3, 2, 3, 2, 3, 2, 3, 2, 3, 2, 3], 400_000, 1000, "gauss_mix"),  # D=12: training records
])
def test_stepwise_given_counts(ctx, counts, n_ev, n_g, kind):
    D = len(counts)
    f = W.gauss_diag(D, coef=25.0) if kind == "gauss_mix" else W.exponentials(D, a=20.0)
    p = W.Params(dim=D, n_ev=n_ev, n_g=n_g, n_iter=3, seed=len(counts), n_st_axes=np.array(counts))
    gp, op = _pair(ctx, p, f)
    for _ in range(3):
        step_and_compare(gp, op)


def test_two_structured_axes_d21(ctx):
    """The shape of the D=21 example of Sec. 6: 46 stratifications on two
    axes, none on the other 19, against the oracle, then the whole run."""
    D = 21
    s = np.array([0.03, 0.03] + [0.4] * 19)
    mu = np.array([0.4, 0.6] + [0.5] * 19)
    exact = float(np.prod([W.gauss_box_1d(1 / (2 * si * si), m) for si, m in zip(s, mu)]))
    f = W.Integrand("corr_gauss", D, mu.reshape(1, -1), [0.5], [1.0], chol=np.diag(1.0 / s), exact=exact)
    p = W.Params(dim=D, n_ev=12_000, n_g=100, n_iter=20, seed=0, n_discard=10,
                 n_st_axes=np.array([46, 46] + [1] * 19))
    gp, op = _pair(ctx, p, f)
    assert gp.n_hc == 46 * 46
    for _ in range(3):
        step_and_compare(gp, op)
    g2 = B.Problem(ctx, p, f)
    g2.iterate(p.n_iter)
    r = g2.result()
    assert abs(r["mean"] - exact) < 5 * r["sdev"]


def test_equal_counts_equal_uniform(ctx):
    """Per-axis counts that are all equal take the uniform kernel: same
    integers, same sums."""
    p, f = W.cfg_small_d4()
    a = B.Problem(ctx, p, f)
    b = B.Problem(ctx, p.with_(n_st_axes=np.array([a.n_st] * 4)), f)
    a.iterate(2)
    b.iterate(2)
    np.testing.assert_array_equal(a.alloc(), b.alloc())
    ra, rb = a.result(), b.result()
    assert_close(rb["I"], ra["I"], RTOL64, what="I_j")
    assert_close(rb["V"], ra["V"], RTOL64, what="V_j")


def test_invalid_counts(ctx):
    f = W.const(3)
    base = W.Params(dim=3, n_ev=1000, n_g=10)
    for bad in ([0, 2, 2], [10, 10, 10], [-1, 1, 1]):
        with pytest.raises(B.VegaspError) as e:
            B.Problem(ctx, base.with_(n_st_axes=np.array(bad)), f)
        assert e.value.status == B.VP_ERR_INVALID_ARG
    with pytest.raises(B.VegaspError):
        B.Problem(ctx, base.with_(strat="mixed"), f, n_st=2)
