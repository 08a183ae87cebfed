"""Preconditioned map (Sec. 5.2): training the vegas map on given samples
{x, f(x)} before integrating.  Pinned by hand-worked training data, by the
inverse of the map, by the optimal-map fixed point (the quantiles of the
sampled density) and by the paper's three-peak example."""
import math

import numpy as np
import pytest

import oracle as orc
from paper_2009_05112_amd import workloads as W


def _values(f, x):
    """The integrand at the training points, written out for the inputs."""
    out = np.zeros(len(x))
    for k in range(f.n_terms):
        out += f.amps[k] * np.exp(-f.coefs[k] * ((x - f.centers[k]) ** 2).sum(axis=1))
    return f.scale * out


def test_training_data_by_hand():
    # D=1, N_g=2, map (0, 1/4, 1): N_g Delta = 1/2 and 3/2.  Points 0.1, 0.2
    # (f = 1) in increment 0: (J f)^2 = 1/4 each; 0.7 (f = 2): (3/2 * 2)^2 = 9.
    p = W.Params(dim=1, n_ev=100, n_g=2)
    pr = orc.Problem(p, W.const(1))
    H, Wc = pr.train_hist(np.array([[0.1], [0.2], [0.7]]), np.array([1.0, 1.0, 2.0]),
                          np.array([[0.0, 0.25, 1.0]]))
    np.testing.assert_array_equal(H, [[0.5, 9.0]])
    np.testing.assert_array_equal(Wc, [[2.0, 1.0]])
    # D=2: J is the product over both axes.  Maps (0, 1/4, 1) and (0, 1/2, 1).
    # (0.1, 0.9), f = 2: J = 1/2 * 1 -> (J f)^2 = 1, increments (0, 1);
    # (0.7, 0.2), f = 1: J = 3/2 * 1 -> 9/4, increments (1, 0).
    p = W.Params(dim=2, n_ev=100, n_g=2)
    pr = orc.Problem(p, W.const(2))
    H, Wc = pr.train_hist(np.array([[0.1, 0.9], [0.7, 0.2]]), np.array([2.0, 1.0]),
                          np.array([[0.0, 0.25, 1.0], [0.0, 0.5, 1.0]]))
    np.testing.assert_array_equal(H, [[1.0, 2.25], [2.25, 1.0]])
    np.testing.assert_array_equal(Wc, [[1.0, 1.0], [1.0, 1.0]])


def test_points_land_in_the_increment_of_their_y():
    # inverse map: x = x(y) on a random non-uniform map lies in increment
    # floor(y N_g) (one point per call; W marks its increment)
    rng = np.random.default_rng(0)
    ng = 37
    m = np.concatenate([[0.0], np.cumsum(rng.uniform(0.2, 3.0, size=ng))])
    m /= m[-1]
    m[-1] = 1.0
    p = W.Params(dim=1, n_ev=100, n_g=ng)
    pr = orc.Problem(p, W.const(1))
    for y in np.concatenate([rng.uniform(0, 1, 200), np.arange(ng) / ng]):
        t = y * ng
        i = min(int(math.floor(t)), ng - 1)
        x = m[i] + (m[i + 1] - m[i]) * (t - i)
        _, Wc = pr.train_hist(np.array([[x]]), np.array([1.0]), m[None, :])
        assert int(np.argmax(Wc[0])) == i and Wc.sum() == 1.0


def test_uniform_data_keep_the_uniform_map():
    # a constant integrand sampled anywhere: every non-empty increment has
    # d_i = f^2, so the refinement keeps the uniform map
    rng = np.random.default_rng(1)
    p = W.Params(dim=3, n_ev=100, n_g=20)
    pr = orc.Problem(p, W.const(3))
    x = rng.uniform(0, 1, size=(5000, 3))
    m0 = pr.map_init()
    m = pr.map_train(x, np.full(5000, 2.5), m0, 3, 0.5)
    assert np.abs(m - m0).max() < 1e-14


def test_training_converges_to_the_quantiles():
    # Eq. (onedopt)/(invJ): the optimal map has J f constant, i.e. equal mass
    # of f in every increment.  For a piecewise-constant density (3 on [0, 1/4),
    # 1 on [1/4, 1]; equal masses) and N_g = 10 those quantiles form a grid on
    # which f is constant in every increment, so every d_i is the same and the
    # grid is an exact fixed point of training; from the uniform map training
    # converges to it.
    rng = np.random.default_rng(4)
    n = 100_000
    n_a = rng.binomial(n, 0.5)
    x = np.concatenate([rng.uniform(0, 0.25, n_a), rng.uniform(0.25, 1.0, n - n_a)])[:, None]
    fx = np.where(x[:, 0] < 0.25, 3.0, 1.0)
    p = W.Params(dim=1, n_ev=100, n_g=10)
    pr = orc.Problem(p, W.const(1))
    q = np.concatenate([np.linspace(0, 0.25, 6), np.linspace(0.25, 1.0, 6)[1:]])[None, :]
    assert np.abs(pr.map_train(x, fx, q, 5, 0.5) - q).max() < 1e-15
    m = pr.map_train(x, fx, pr.map_init(), 60, 0.5)
    assert np.abs(m - q).max() < 1e-4


def test_paper_three_peaks():
    # Sec. 5.2: three peaks exp(-1e4 |x - r_i|^2) on the diagonal of the
    # 8-cube; a map trained for 10 passes on 3000 points drawn near the peaks,
    # then 8 iterations with alpha = 0: about percent accuracy at N_ev = 1e6,
    # where the untrained map does not find the peaks.
    f = W.gauss_diag(8, coef=1e4)
    x = W.precondition_points(3000, f.centers, 1e4, seed=1)
    p = W.Params(dim=8, n_ev=1_000_000, n_g=1000, n_iter=8, alpha=0.0, seed=2)
    pr = orc.Problem(p, f)
    m = pr.map_train(x, _values(f, x), pr.map_init(), 10, 0.5)
    r = pr.integrate(fmap=m)
    assert abs(r["mean"] - 1.0) < 5 * r["sdev"] and r["sdev"] < 0.05
    plain = orc.Problem(p.with_(n_ev=100_000, alpha=0.5), f).integrate()
    assert plain["mean"] < 0.5
