"""Batched integrands (VP_F_BATCH): the library writes each iteration's points
as structure-of-arrays device buffers, the user's function fills f, and the
library accumulates J f.  The example library's Gaussian mixture performs the
built-in kind's operations in the same order, so the batched path must give
the built-in path's results up to the order of the sums (the two kernels split
the samples over waves differently); step by step it is compared with the
oracle evaluating the same mixture."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2009_05112_amd import _binding as B
from paper_2009_05112_amd import workloads as W
from tests.parity import step_and_compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def _mix(dim, k, seed):
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.3, 0.7, size=(k, dim))
    coefs = rng.uniform(20.0, 80.0, size=k)
    amps = rng.uniform(0.5, 1.5, size=k)
    return W.Integrand("gauss_mix", dim, centers, coefs, amps, scale=1.7)


@pytest.mark.parametrize("dim,k,n_ev,n_g", [(4, 3, 100_000, 200), (8, 2, 400_000, 1000), (12, 1, 300_000, 1000),
                                           (8, 3, 4_000_000, 1000)])
def test_batched_equals_builtin(ctx, dim, k, n_ev, n_g):
    """Each step starts both problems from the same state (map, allocation,
    iteration): same points and values, sums in another order (the two
    kernels split the samples over waves differently).  At 4e6 samples the
    generate and accumulate kernels run on different grids."""
    f = _mix(dim, k, dim)
    p = W.Params(dim=dim, n_ev=n_ev, n_g=n_g, n_iter=4, seed=11)
    bf = B.example_gauss_mix(f)
    try:
        gb = B.Problem(ctx, p, bf)
        gf = B.Problem(ctx, p, f)
        for _ in range(p.n_iter):
            gb.set_map(gf.map())
            gb.set_alloc(gf.alloc())
            gb.set_it(gf.it)
            gb.iterate(1)
            gf.iterate(1)
            ab, af = gb.accum(), gf.accum()
            np.testing.assert_allclose(ab["S1"], af["S1"], rtol=1e-12, atol=1e-300)
            np.testing.assert_allclose(ab["S2"], af["S2"], rtol=1e-12, atol=1e-300)
            for m in range(dim):
                tot = np.abs(af["H"][m]).sum()
                assert np.abs(ab["H"][m] - af["H"][m]).max() <= 1e-12 * tot
            np.testing.assert_array_equal(gb.alloc(), gf.alloc())
            rb, rf = gb.result(), gf.result()
            assert abs(rb["I"][-1] - rf["I"][-1]) <= 1e-12 * abs(rf["I"][-1])
        gb.close()
        gf.close()
    finally:
        B.examples().vp_example_free_user(bf.user)


def test_batched_two_samples_per_hypercube(ctx):
    """n_h = 2 everywhere (the smallest allocation, Sec. 3): a lane's 16
    samples of a tile then cross eight hypercube boundaries, every one of
    those the batched modes load at the start of the tile.  Against the
    built-in path from the same state, with H and W element by element."""
    dim = 4
    f = _mix(dim, 2, 77)
    p = W.Params(dim=dim, n_ev=131_072, n_g=200, n_iter=3, seed=3)
    bf = B.example_gauss_mix(f)
    try:
        gb = B.Problem(ctx, p, bf)
        gf = B.Problem(ctx, p, f)
        assert gf.n_hc > 20_000
        two = np.full(gf.n_hc, 2, dtype=np.int32)
        for _ in range(p.n_iter):
            gf.set_alloc(two)
            gb.set_map(gf.map())
            gb.set_alloc(two)
            gb.set_it(gf.it)
            gb.iterate(1)
            gf.iterate(1)
            ab, af = gb.accum(), gf.accum()
            np.testing.assert_allclose(ab["S1"], af["S1"], rtol=1e-12, atol=1e-300)
            np.testing.assert_allclose(ab["S2"], af["S2"], rtol=1e-12, atol=1e-300)
            for key in ("H", "W"):
                for m in range(dim):
                    tot = np.abs(af[key][m]).sum()
                    assert np.abs(ab[key][m] - af[key][m]).max() <= 1e-12 * tot, (key, m)
        gb.close()
        gf.close()
    finally:
        B.examples().vp_example_free_user(bf.user)


@pytest.mark.parametrize("dim,n_ev,n_g", [(4, 50_000, 100), (11, 200_000, 1000)])
def test_batched_stepwise_against_oracle(ctx, dim, n_ev, n_g):
    """The oracle evaluates the same mixture itself; D=11 at N_g=1000 takes
    the training-record path for one axis."""
    f = _mix(dim, 3, 100 + dim)
    p = W.Params(dim=dim, n_ev=n_ev, n_g=n_g, n_iter=3, seed=5)
    bf = B.example_gauss_mix(f)
    try:
        gp = B.Problem(ctx, p, bf)
        op = oracle.Problem(p, f, n_st=gp.n_st)
        for _ in range(3):
            step_and_compare(gp, op)
        gp.close()
    finally:
        B.examples().vp_example_free_user(bf.user)


def test_batched_mixed_stratification(ctx):
    """Per-axis stratification (the mixed rule: 5, 5, 4, 4, 4, 4) in the
    generate and accumulate modes, against the oracle."""
    f = _mix(6, 2, 66)
    p = W.Params(dim=6, n_ev=30_000, n_g=100, n_iter=3, seed=6, strat="mixed")
    bf = B.example_gauss_mix(f)
    try:
        gp = B.Problem(ctx, p, bf)
        op = oracle.Problem(p, f)
        assert list(gp.n_st_axes) == list(op.n_st_axes) == [5, 5, 4, 4, 4, 4]
        for _ in range(3):
            step_and_compare(gp, op)
        gp.close()
    finally:
        B.examples().vp_example_free_user(bf.user)


def test_python_callback(ctx):
    """A batched integrand given as a Python function: it counts the calls and
    hands the device buffers to the example library's kernel."""
    f = _mix(3, 2, 7)
    p = W.Params(dim=3, n_ev=20_000, n_g=100, n_iter=3, seed=2)
    inner = B.example_gauss_mix(f)
    c_fn = B.BATCH_FN(inner.fn)
    calls = []

    def fn(user, stream, n, dim, x, out):
        calls.append((n, dim))
        return c_fn(inner.user, stream, n, dim, x, out)

    cb = B.BATCH_FN(fn)
    try:
        gp = B.Problem(ctx, p, B.BatchIntegrand(3, cb, None, scale=f.scale))
        gf = B.Problem(ctx, p, f)
        gp.iterate(p.n_iter)
        gf.iterate(p.n_iter)
        rp, rf = gp.result(), gf.result()
        assert len(calls) == p.n_iter and all(d == 3 and n > 0 for n, d in calls)
        assert rp["n_evals"] == rf["n_evals"] == sum(n for n, _ in calls)
        assert abs(rp["mean"] - rf["mean"]) <= 1e-9 * abs(rf["mean"])
        gp.close()
        gf.close()
    finally:
        B.examples().vp_example_free_user(inner.user)


def test_failing_function_is_reported(ctx):
    fn = C.cast(B.examples().vp_example_failing, C.c_void_p).value
    p = W.Params(dim=2, n_ev=1000, n_g=10, n_iter=1)
    gp = B.Problem(ctx, p, B.BatchIntegrand(2, fn, None))
    with pytest.raises(B.VegaspError) as e:
        gp.iterate(1)
    assert e.value.status == B.VP_ERR_DEVICE
    gp.close()


def test_batched_limits(ctx):
    fn = C.cast(B.examples().vp_example_failing, C.c_void_p).value
    with pytest.raises(B.VegaspError) as e:
        B.Problem(ctx, W.Params(dim=2, n_ev=1000, precision="fp32_acc64"), B.BatchIntegrand(2, fn, None))
    assert e.value.status == B.VP_ERR_INVALID_ARG
    with pytest.raises(B.VegaspError) as e:
        B.Problem(ctx, W.Params(dim=2, n_ev=1000), B.BatchIntegrand(2, 0, None))
    assert e.value.status == B.VP_ERR_INVALID_ARG
    s = B.Server(ctx)
    with pytest.raises(B.VegaspError) as e:
        s.submit(W.Params(dim=2, n_ev=1000), B.BatchIntegrand(2, fn, None))
    assert e.value.status == B.VP_ERR_INVALID_ARG
    s.close()
