"""GPU parity of map training on given samples (Sec. 5.2, preconditioned
integrators): training data and refined map of every pass against the
oracle from the same map, then the paper's three-peak workflow."""
import numpy as np
import pytest

import oracle
from paper_2009_05112_amd import _binding as B
from paper_2009_05112_amd import workloads as W
from tests.parity import RTOL64, assert_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def _values(f, x):
    out = np.zeros(len(x))
    for k in range(f.n_terms):
        out += f.amps[k] * np.exp(-f.coefs[k] * ((x - f.centers[k]) ** 2).sum(axis=1))
    return f.scale * out


def test_training_data_by_hand(ctx):
    # maps (0, 1/4, 1) and (0, 1/2, 1); (0.1, 0.9) with f = 2 adds 1 to
    # increments (0, 1), (0.7, 0.2) with f = 1 adds 9/4 to increments (1, 0)
    p = W.Params(dim=2, n_ev=100, n_g=2, alpha=0.0)
    gp = B.Problem(ctx, p, W.const(2))
    gp.set_map(np.array([[0.0, 0.25, 1.0], [0.0, 0.5, 1.0]]))
    gp.train_map(np.array([[0.1, 0.9], [0.7, 0.2]]), np.array([2.0, 1.0]), 1, 0.0)
    acc = gp.accum()
    np.testing.assert_array_equal(acc["H"], [[1.0, 2.25], [2.25, 1.0]])
    np.testing.assert_array_equal(acc["W"], [[1.0, 1.0], [1.0, 1.0]])
    np.testing.assert_array_equal(gp.map(), [[0.0, 0.25, 1.0], [0.0, 0.5, 1.0]])  # alpha = 0


def test_training_passes_against_oracle(ctx):
    """The three-peak sample of Sec. 5.2 (3000 points, D=8, N_g=1000): every
    pass's counts exactly, its sums to 1e-12 of the axis total, its map from
    those sums; then points placed exactly on grid points."""
    f = W.gauss_diag(8, coef=1e4)
    x = W.precondition_points(3000, f.centers, 1e4, seed=1)
    fx = _values(f, x)
    p = W.Params(dim=8, n_ev=1_000_000, n_g=1000, n_iter=8, alpha=0.0, seed=2)
    gp = B.Problem(ctx, p, f)
    op = oracle.Problem(p.with_(alpha=0.5), f)
    for _ in range(10):
        m = gp.map()
        gp.train_map(x, fx, 1, 0.5)
        acc = gp.accum()
        H, Wc = op.train_hist(x, fx, m)
        np.testing.assert_array_equal(acc["W"], Wc)
        for mu in range(8):
            assert_close(acc["H"][mu], H[mu], RTOL64, scale=np.abs(H[mu]).sum(), what=f"H[{mu}]")
        assert_close(gp.map(), op.refine(acc["H"], acc["W"], m), RTOL64, scale=np.ones_like(m), what="map")
    m = gp.map()
    xg = np.stack([m[mu][(np.arange(500) * 7) % 1001] for mu in range(8)], axis=1)
    gp.train_map(xg, np.ones(500), 1, 0.0)
    _, Wc = op.train_hist(xg, np.ones(500), m)
    np.testing.assert_array_equal(gp.accum()["W"], Wc)


def test_paper_three_peaks(ctx):
    """Train 10 passes, then 8 iterations with alpha = 0 at N_ev = 1e6:
    percent-level accuracy."""
    f = W.gauss_diag(8, coef=1e4)
    x = W.precondition_points(3000, f.centers, 1e4, seed=1)
    p = W.Params(dim=8, n_ev=1_000_000, n_g=1000, n_iter=8, alpha=0.0, seed=2)
    gp = B.Problem(ctx, p, f)
    gp.train_map(x, _values(f, x), 10, 0.5)
    gp.iterate(8)
    r = gp.result()
    assert abs(r["mean"] - 1.0) < 5 * r["sdev"] and r["sdev"] < 0.05


def test_training_rejects_bad_points(ctx):
    p = W.Params(dim=2, n_ev=100, n_g=10)
    gp = B.Problem(ctx, p, W.const(2))
    for x, fx in ((np.array([[0.5, 1.5]]), np.array([1.0])), (np.array([[0.5, 0.5]]), np.array([np.nan])),
                  (np.array([[np.nan, 0.5]]), np.array([1.0]))):
        with pytest.raises(B.VegaspError) as e:
            gp.train_map(x, fx, 1, 0.5)
        assert e.value.status == B.VP_ERR_INVALID_ARG
