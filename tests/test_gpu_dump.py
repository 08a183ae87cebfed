"""Per-sample parity through vp_debug_dump: the sampling kernel records the
samples of a range of the next iteration (hypercube h, index j, increment
index and point x on every axis, J, f(x)), and each is compared with the
oracle's own enumeration of the same samples (uniform y in each hypercube,
Sec. 3; the map of Sec. 2.2, Eqs. y and jac).  Hypercube, sample and
increment indices must match bit for bit; x and J are the same operations in
the same order on both sides and must match to the last bit in double
precision; f(x) differs only by the exponential's last bits (1e-12).  The
iteration's sums are compared as well, so the dumped run is a normal run."""
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


def _pair(ctx, params, f):
    gp = B.Problem(ctx, params, f)
    op = oracle.Problem(params, f, n_st=gp.n_st)
    assert gp.n_hc == op.n_hc
    return gp, op


def _compare(d, o, sl, what, rtol_f=1e-12, exact_x=True):
    for k in ("h", "j"):
        np.testing.assert_array_equal(d[k], o[k][sl], err_msg=f"{what}: {k}")
    np.testing.assert_array_equal(d["idx"], o["idx"][sl], err_msg=f"{what}: increment indices")
    if exact_x:
        np.testing.assert_array_equal(d["x"], o["x"][sl], err_msg=f"{what}: x")
        np.testing.assert_array_equal(d["jac"], o["jac"][sl], err_msg=f"{what}: J")
    else:
        np.testing.assert_allclose(d["x"], o["x"][sl], rtol=0, atol=1e-15, err_msg=f"{what}: x")
        np.testing.assert_allclose(d["jac"], o["jac"][sl], rtol=1e-14, err_msg=f"{what}: J")
    ofx = o["fx"][sl]
    np.testing.assert_allclose(d["fx"], ofx, rtol=rtol_f, atol=rtol_f * np.abs(ofx).max() * 1e-3,
                               err_msg=f"{what}: f(x)")


def _dump_step(gp, op, first, count, **kw):
    """Arms the dump of samples [first, first + count) of the next iteration,
    runs it (compared step-wise with the oracle) and returns the dump with the
    oracle's per-sample view of the same state."""
    fmap, n_h, it = gp.map(), gp.alloc(), gp.it
    gp.debug_dump(first, count)
    step_and_compare(gp, op, **kw)
    d = gp.debug_dump_get()
    cum = np.concatenate([[0], np.cumsum(n_h.astype(np.int64))])
    h0 = int(np.searchsorted(cum, first, side="right") - 1)
    h1 = int(np.searchsorted(cum, min(first + count, cum[-1]), side="left"))
    o = op.sample_points(fmap, n_h, it, h0, h1)
    off = first - int(cum[h0])
    return d, o, slice(off, off + len(d["h"])), int(cum[-1])


def test_dump_whole_iteration_d4(ctx):
    """D=4, N_ev=1e5 (N_st=12): every sample of iterations 0 and 3."""
    p, f = W.cfg_small_d4()
    gp, op = _pair(ctx, p, f)
    for it in range(4):
        if it in (0, 3):
            d, o, sl, n_tot = _dump_step(gp, op, 0, 400_000)
            assert len(d["h"]) == n_tot  # the dump stops at the iteration's last sample
            _compare(d, o, sl, f"iteration {it}")
        else:
            step_and_compare(gp, op)


def test_dump_ranges_d8_adapted(ctx):
    """D=8 three diagonal Gaussians at N_ev=1e6 (two innermost map axes in
    LDS, the benchmark's layout), after two adapting iterations: ranges that
    start and end inside hypercubes."""
    p, f = W.cfg_diag_d8(n_ev=1_000_000)
    gp, op = _pair(ctx, p, f)
    assert gp.map_place == "inner"
    for _ in range(2):
        step_and_compare(gp, op)
    for first, count in ((3, 50_000), (517_001, 70_000), (1_000_000, 10**6)):
        d, o, sl, n_tot = _dump_step(gp, op, first, count)
        assert len(d["h"]) == min(count, n_tot - first)
        _compare(d, o, sl, f"[{first}, +{count})")


@pytest.mark.parametrize("case", ["corr_gauss", "mixed", "fp32_acc64", "fp32_neumaier", "global_map"])
def test_dump_kernels(ctx, case):
    """The other kernel families: correlated Gaussian (D=13), mixed
    stratification (generic kernel), the two split precisions (single-
    precision x and J, compared with the oracle in the same precision), and
    the map read from global memory (D=10)."""
    rng = np.random.default_rng(5)
    kw = {}
    exact_x, rtol_f = True, 1e-12
    if case == "corr_gauss":
        f = W.corr_gauss(rng, 13, s_max=0.2, cond=10.0)
        p = W.Params(dim=13, n_ev=300_000, n_g=200, n_iter=3, seed=3)
    elif case == "mixed":
        f = W.gauss_single(6, coef=20.0)
        p = W.Params(dim=6, n_ev=200_000, n_g=300, n_iter=3, seed=4, strat="mixed")
    elif case == "global_map":
        f = W.gauss_diag(10, coef=50.0, cs=(0.3, 0.6))
        p = W.Params(dim=10, n_ev=200_000, n_g=1000, n_iter=3, seed=6)
    else:
        p, f = W.cfg_diag_d8(n_ev=400_000, precision=case)
        p = p.with_(n_iter=3, seed=8)
        kw = {"rtol": 2e-6, "rtol_hist": 2e-6, "floor": 1e-12}
        rtol_f = 2e-6
    gp, op = _pair(ctx, p, f)
    if case == "global_map":
        assert gp.map_place == "global"
    step_and_compare(gp, op, **kw)
    d, o, sl, _ = _dump_step(gp, op, 1234, 60_000, **kw)
    _compare(d, o, sl, case, rtol_f=rtol_f, exact_x=exact_x)


def test_dump_arming_rules(ctx):
    p, f = W.cfg_small_d4()
    gp = B.Problem(ctx, p, f)
    gp.debug_dump(0, 10)
    with pytest.raises(B.VegaspError) as e:
        gp.debug_dump_get()  # the iteration has not run
    assert e.value.status == B.VP_ERR_STATE
    with pytest.raises(B.VegaspError) as e:
        gp.debug_dump(-1, 10)
    assert e.value.status == B.VP_ERR_INVALID_ARG
    with pytest.raises(B.VegaspError) as e:
        gp.debug_dump(0, (1 << 24) + 1)
    assert e.value.status == B.VP_ERR_INVALID_ARG
    gp.debug_dump(0, 10)
    gp.iterate(2)  # only the first of the two iterations is dumped
    d = gp.debug_dump_get()
    assert len(d["h"]) == 10 and list(d["h"]) == [0] * 4 + [1] * 4 + [2] * 2
    gp.debug_dump(10**9, 5)  # beyond the last sample: nothing recorded
    gp.iterate(1)
    assert len(gp.debug_dump_get()["h"]) == 0
    gp.close()
