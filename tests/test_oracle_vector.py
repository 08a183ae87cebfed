"""Vector-valued integrands (Sec. 6): several integrals from the same
samples, with their covariance summed over hypercubes, and the combination
of correlated estimates over iterations.  Pinned by hand-worked
combinations, the scalar special case, closed-form moments of a Gaussian
density and the consistency of the covariance with the spread of the
estimates."""
import json
import math
import os

import numpy as np
import pytest

import oracle as orc
from paper_2009_05112_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_combination_by_hand():
    # independent components: each combines as a scalar (weights 1, 1 and
    # 1/4, 1): means 2 and 0.4, variances 1/2 and 4/5;
    # chi2 = 1 + 1 + (1.6^2)/4 + 0.4^2 = 2.8 with dof (2 - 1) * 2
    I = [[1.0, 2.0], [3.0, 0.0]]
    C = [np.diag([1.0, 4.0]), np.diag([1.0, 1.0])]
    mean, cov, chi2, dof = orc.combine_vec(I, C)
    np.testing.assert_allclose(mean, [2.0, 0.4], rtol=1e-15)
    np.testing.assert_allclose(cov, np.diag([0.5, 0.8]), rtol=1e-15, atol=1e-16)
    assert chi2 == pytest.approx(2.8, rel=1e-14) and dof == 2
    # correlated, equal covariances: the plain mean, covariance C / 2,
    # chi2 = 2 * (1, 1) C^-1 (1, 1) = 2 * 4/3
    Cc = np.array([[1.0, 0.5], [0.5, 1.0]])
    mean, cov, chi2, dof = orc.combine_vec([[0.0, 0.0], [2.0, 2.0]], [Cc, Cc])
    np.testing.assert_allclose(mean, [1.0, 1.0], rtol=1e-15)
    np.testing.assert_allclose(cov, Cc / 2, rtol=1e-15)
    assert chi2 == pytest.approx(8.0 / 3.0, rel=1e-14)
    # unweighted: plain mean, covariance sum C_j / count^2
    mean, cov, chi2, dof = orc.combine_vec(I, C, average="unweighted")
    np.testing.assert_allclose(mean, [2.0, 1.0])
    np.testing.assert_allclose(cov, np.diag([0.5, 1.25]))
    # a singular covariance (a component without error): the plain mean, NaN chi2
    mean, cov, chi2, dof = orc.combine_vec([[1.0, 5.0], [3.0, 5.0]], [np.diag([1.0, 0.0])] * 2)
    np.testing.assert_allclose(mean, [2.0, 5.0])
    assert math.isnan(chi2) and dof == 2


def test_one_component_is_the_scalar_combination():
    g = json.load(open(os.path.join(GOLD, "combine_cases.json")))
    for c in g["cases"]:
        I = np.array(c["I"])[:, None]
        Cs = (np.array(c["sig"]) ** 2)[:, None, None]
        mean, cov, chi2, dof = orc.combine_vec(I, Cs)
        assert mean[0] == pytest.approx(c["mean"], rel=1e-14)
        assert math.sqrt(cov[0, 0]) == pytest.approx(c["sdev"], rel=1e-14)
        assert chi2 == pytest.approx(c["chi2"], abs=1e-14) and dof == c["dof"]


E1 = [-1, 0, 1, 0, 0]
E2 = [-1, -1, -1, 0, 1]   # components g, g x0, g x1, g x0^2, g x0 x1


def test_component_zero_is_the_scalar_iteration():
    f = W.gauss_diag(3, coef=30.0)
    p = W.Params(dim=3, n_ev=20_000, n_g=50, seed=3)
    pr = orc.Problem(p, f)
    m, n = pr.map_init(), pr.alloc_init()
    I, C, _ = pr.vec_iteration(m, n, 0, E1, E2)
    s = pr.iteration(m, n, it=0)
    assert I[0] == pytest.approx(s["I"], rel=1e-14)
    assert C[0, 0] == pytest.approx(s["V"], rel=1e-12)
    np.testing.assert_array_equal(C, C.T)
    assert np.all(np.linalg.eigvalsh(C) > -1e-12 * np.trace(C))


def _moment_exact(f, e1, e2):
    """The integral over the unit box of f (x_e1 or 1)(x_e2 or 1) for a
    Gaussian mixture, factor by factor: int x^p exp(-c (x - m)^2) dx on [0, 1]
    for p = 0, 1, 2 in closed form."""
    def one(c, m, pw):
        s = math.sqrt(c)
        g0 = 0.5 * math.sqrt(math.pi / c) * (math.erf(s * (1 - m)) + math.erf(s * m))
        e0, e1_ = math.exp(-c * m * m), math.exp(-c * (1 - m) ** 2)
        g1 = (e0 - e1_) / (2 * c)                                  # int (x - m) e^..
        g2 = (-(1 - m) * e1_ - m * e0) / (2 * c) + g0 / (2 * c)    # int (x - m)^2 e^..
        if pw == 0:
            return g0
        if pw == 1:
            return g1 + m * g0
        return g2 + 2 * m * g1 + m * m * g0
    tot = 0.0
    for k in range(f.n_terms):
        pw = np.zeros(f.dim, dtype=int)
        for e in (e1, e2):
            if e >= 0:
                pw[e] += 1
        prod = f.amps[k]
        for mu in range(f.dim):
            prod *= one(f.coefs[k], f.centers[k][mu], pw[mu])
        tot += prod
    return f.scale * tot


def test_moments_and_correlated_errors():
    # closed-form moments of a Gaussian density; the mean <x0> = I_1 / I_0 with
    # the error propagated through the covariance is consistent and several
    # times smaller than when the correlation is ignored (Sec. 6)
    f = W.gauss_single(3, coef=40.0, c=0.45)
    p = W.Params(dim=3, n_ev=40_000, n_g=100, seed=5)
    pr = orc.Problem(p, f)
    m, n = pr.map_init(), pr.alloc_init()
    Is, Cs = [], []
    for it in range(8):
        I, C, _ = pr.vec_iteration(m, n, it, E1, E2)
        s = pr.iteration(m, n, it)
        m, n = s["map"], s["n_h"]
        Is.append(I)
        Cs.append(C)
    mean, cov, chi2, dof = orc.combine_vec(Is[3:], Cs[3:])
    exact = np.array([_moment_exact(f, a, b) for a, b in zip(E1, E2)])
    err = np.sqrt(np.diag(cov))
    assert np.all(np.abs(mean - exact) < 5 * err)
    r = mean[1] / mean[0]
    g = np.array([-r / mean[0], 1 / mean[0]])
    sig_corr = math.sqrt(g @ cov[:2, :2] @ g)
    sig_nocorr = math.sqrt(g @ np.diag(np.diag(cov[:2, :2])) @ g)
    r_exact = exact[1] / exact[0]
    assert abs(r - r_exact) < 5 * sig_corr
    assert sig_corr < 0.5 * sig_nocorr


def test_covariance_matches_the_spread_of_estimates():
    # with the map and allocation held fixed, the estimates of independent
    # iterations scatter as their covariance says: chi^2 / dof near 1
    f = W.gauss_single(2, coef=20.0, c=0.5)
    p = W.Params(dim=2, n_ev=5_000, n_g=40, seed=9)
    pr = orc.Problem(p, f)
    m, n = pr.map_init(), pr.alloc_init()
    for it in range(4):  # adapt
        s = pr.iteration(m, n, it)
        m, n = s["map"], s["n_h"]
    Is, Cs = [], []
    for it in range(4, 64):
        I, C, _ = pr.vec_iteration(m, n, it, E1, E2)
        Is.append(I)
        Cs.append(C)
    mean, cov, chi2, dof = orc.combine_vec(Is, Cs)
    assert 0.7 < chi2 / dof < 1.35
