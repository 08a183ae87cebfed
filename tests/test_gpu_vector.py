"""GPU parity of vector-valued batched integrands (Sec. 6): the components
g, g x0, g x1, g x0^2, g x0 x1 of a Gaussian density from the example
library; every iteration's estimates and covariance against the oracle from
the same state, the combination against the oracle's from the same
per-iteration values, then moments and correlated errors."""
import math

import numpy as np
import pytest

import oracle
from paper_2009_05112_amd import _binding as B
from paper_2009_05112_amd import workloads as W
from tests.parity import RTOL64, assert_close, step_and_compare

pytestmark = pytest.mark.gpu

E1 = [-1, 0, 1, 0, 0]
E2 = [-1, -1, -1, 0, 1]


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("dim,n_ev,strat", [(3, 40_000, "uniform"), (5, 200_000, "mixed"), (2, 3_000, "uniform")])
def test_vector_stepwise_against_oracle(ctx, dim, n_ev, strat):
    f = W.gauss_diag(dim, coef=30.0)
    p = W.Params(dim=dim, n_ev=n_ev, n_g=100, n_iter=4, seed=dim, strat=strat, n_discard=1)
    bf = B.example_gauss_moments(f, E1, E2)
    try:
        gp = B.Problem(ctx, p, bf)
        op = oracle.Problem(p, f)
        for it in range(4):
            m, n = gp.map(), gp.alloc()
            Io, Co, sc = op.vec_iteration(m, n, gp.it, E1, E2)
            step_and_compare(gp, op)  # component 0 drives the adaptation
            rv = gp.result_vec(5)
            assert_close(rv["I"][-1], Io, RTOL64, what="I_a")
            scale = np.sqrt(np.outer(sc, sc))
            assert_close(rv["C"][-1], Co, RTOL64, scale=scale, what="C_ab")
        mean, cov, chi2, dof = oracle.combine_vec(rv["I"], rv["C"], n_discard=1)
        sd = np.sqrt(np.abs(np.diag(cov)))
        assert_close(rv["mean"], mean, 1e-9, scale=np.maximum(np.abs(mean), sd), what="mean")
        assert_close(rv["cov"], cov, 1e-9, scale=np.outer(sd, sd), what="cov")
        assert_close(rv["chi2"], chi2, 1e-9, what="chi2")
        assert rv["dof"] == dof == (3 - 1) * 5
        r = gp.result()
        assert_close(r["I"], rv["I"][:, 0], RTOL64, what="the scalar I_j are component 0's")
        gp.close()
    finally:
        B.examples().vp_example_free_user(bf.user)


def test_vector_unweighted_and_frozen(ctx):
    f = W.gauss_single(3, coef=40.0, c=0.45)
    p = W.Params(dim=3, n_ev=40_000, n_g=100, n_iter=10, seed=5, n_adapt=4, n_discard=4, average="unweighted")
    bf = B.example_gauss_moments(f, E1, E2)
    try:
        gp = B.Problem(ctx, p, bf)
        gp.iterate(10)
        rv = gp.result_vec(5)
        mean, cov, chi2, dof = oracle.combine_vec(rv["I"], rv["C"], n_discard=4, average="unweighted")
        sd = np.sqrt(np.diag(cov))
        assert_close(rv["mean"], mean, 1e-12, scale=np.abs(mean), what="mean")
        assert_close(rv["cov"], cov, 1e-12, scale=np.outer(sd, sd), what="cov")
        assert_close(rv["chi2"], chi2, 1e-9, what="chi2")
        gp.close()
    finally:
        B.examples().vp_example_free_user(bf.user)


def test_moments_and_correlated_errors(ctx):
    """<x0> = I_1 / I_0 from one run: consistent with the closed form, its
    error through the covariance several times smaller than without."""
    from tests.test_oracle_vector import _moment_exact
    f = W.gauss_single(3, coef=40.0, c=0.45)
    p = W.Params(dim=3, n_ev=400_000, n_g=200, n_iter=10, seed=6, n_discard=4)
    bf = B.example_gauss_moments(f, E1, E2)
    try:
        gp = B.Problem(ctx, p, bf)
        gp.iterate(10)
        rv = gp.result_vec(5)
        exact = np.array([_moment_exact(f, a, b) for a, b in zip(E1, E2)])
        assert np.all(np.abs(rv["mean"] - exact) < 5 * np.sqrt(np.diag(rv["cov"])))
        r = rv["mean"][1] / rv["mean"][0]
        g = np.array([-r / rv["mean"][0], 1 / rv["mean"][0]])
        c2 = rv["cov"][:2, :2]
        sig_corr = math.sqrt(g @ c2 @ g)
        assert abs(r - exact[1] / exact[0]) < 5 * sig_corr
        assert sig_corr < 0.5 * math.sqrt(g @ np.diag(np.diag(c2)) @ g)
        gp.close()
    finally:
        B.examples().vp_example_free_user(bf.user)


def test_vector_limits(ctx):
    f = W.gauss_single(2)
    with pytest.raises(B.VegaspError) as e:
        B.example_gauss_moments(f, [-1] * 17, [-1] * 17)
    bf = B.example_gauss_moments(f, E1, E2)
    try:
        bf.n_out = 17
        with pytest.raises(B.VegaspError) as e:
            B.Problem(ctx, W.Params(dim=2, n_ev=1000, n_g=10), bf)
        assert e.value.status == B.VP_ERR_INVALID_ARG
    finally:
        B.examples().vp_example_free_user(bf.user)
    # a scalar problem reports itself as one component
    p = W.Params(dim=2, n_ev=2000, n_g=20, n_iter=3)
    gp = B.Problem(ctx, p, f)
    gp.iterate(3)
    rv, r = gp.result_vec(1), gp.result()
    assert rv["mean"][0] == r["mean"] and rv["cov"][0, 0] == pytest.approx(r["sdev"] ** 2, rel=1e-15)
    np.testing.assert_array_equal(rv["C"][:, 0, 0], r["V"])
