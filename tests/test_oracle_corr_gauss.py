"""Pins of the oracle's correlated Gaussian, the integrand of the served
stream: exp(-1/2 (x - m)^T Sigma^-1 (x - m)) with Sigma = Q diag(s^2) Q^T for a
random rotation Q (the rotated analogue of the oblique Gaussian of Sec. 3.1).
The oracle evaluates it from an upper-triangular factor U with U^T U =
Sigma^-1; the pins below do not use U:

* pointwise, through the whitening x = m + Q diag(s) z, for which the
  quadratic form is exactly |z|^2, and against Sigma^-1 rebuilt from Q and s;
* the integral over the box against the full-space closed form
  (2 pi)^(D/2) prod s (the box cuts off less than 1e-7 of it), within 5 sigma
  of the oracle's own error estimate, for D = 3 .. 8.
A factor read in the wrong triangle (which leaves only its diagonal), a
dropped 1/2 or a transposed rotation fails them."""
import math

import numpy as np
import pytest

from paper_2009_05112_amd import workloads as W


def _whitened_points(f, rng, n):
    z = rng.standard_normal((n, f.dim)) * 1.5
    x = f.centers[0] + z @ (f.rotation * f.sdevs).T   # m + Q diag(s) z
    return x, z


@pytest.mark.parametrize("dim", [2, 3, 5, 8, 13, 21])
def test_corr_gauss_whitened_closed_form(orc, dim):
    rng = np.random.default_rng(40 + dim)
    f = W.corr_gauss(rng, dim)
    pr = orc.Problem(W.Params(dim=dim, n_ev=1000, n_g=4), f)
    x, z = _whitened_points(f, rng, 64)
    got = np.array([pr.f_eval(xx) for xx in x])
    want = np.exp(-0.5 * np.sum(z * z, axis=1))
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=0)


@pytest.mark.parametrize("dim", [3, 6])
def test_corr_gauss_against_precision_from_rotation(orc, dim):
    rng = np.random.default_rng(7 + dim)
    f = W.corr_gauss(rng, dim)
    prec = f.rotation @ np.diag(f.sdevs ** -2.0) @ f.rotation.T
    pr = orc.Problem(W.Params(dim=dim, n_ev=1000, n_g=4), f)
    x = f.centers[0] + rng.uniform(-0.03, 0.03, size=(64, dim))
    t = x - f.centers[0]
    want = np.exp(-0.5 * np.einsum("ni,ij,nj->n", t, prec, t))
    got = np.array([pr.f_eval(xx) for xx in x])
    keep = want > 1e-250
    assert keep.sum() > 16
    np.testing.assert_allclose(got[keep], want[keep], rtol=1e-8, atol=0)


def test_wrong_triangle_is_caught(orc):
    """A factor read in its lower triangle keeps only the diagonal of U:
    the whitened check must reject it."""
    rng = np.random.default_rng(3)
    f = W.corr_gauss(rng, 5)
    bad = W.Integrand("corr_gauss", 5, f.centers, [0.5], [1.0], chol=np.diag(np.diag(f.chol)))
    pr = orc.Problem(W.Params(dim=5, n_ev=1000, n_g=4), bad)
    x, z = _whitened_points(f, rng, 64)
    got = np.array([pr.f_eval(xx) for xx in x])
    want = np.exp(-0.5 * np.sum(z * z, axis=1))
    assert np.max(np.abs(got / want - 1.0)) > 1e-3


@pytest.mark.parametrize("dim,seed", [(3, 0), (4, 1), (5, 2), (6, 0), (7, 1), (8, 2)])
def test_corr_gauss_integral_closed_form(orc, dim, seed):
    rng = np.random.default_rng(100 + dim + 10 * seed)
    f = W.corr_gauss(rng, dim)
    assert f.exact == pytest.approx((2.0 * math.pi) ** (dim / 2.0) * float(np.prod(f.sdevs)), rel=1e-14)
    # eight adapting iterations, then eight with map and allocation frozen,
    # averaged without weights (Sec. 2.5): an unbiased estimate
    p = W.Params(dim=dim, n_ev=100_000, n_g=200, n_iter=16, seed=dim + seed, n_discard=8, n_adapt=8,
                 average="unweighted")
    r = orc.Problem(p, f).integrate()
    assert r["sdev"] < 0.1 * f.exact
    assert abs(r["mean"] - f.exact) < 5.0 * r["sdev"], (r["mean"], f.exact, r["sdev"])
