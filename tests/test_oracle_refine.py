"""Pins of the map refinement (Sec. 2.3): smoothing and normalisation
(hand-worked fixtures), compression (closed forms and limits), and the regrid
(the equal-share invariant it is built to satisfy, checked by integrating the
piecewise-constant density independently)."""
import json
import math
import os

import numpy as np
import pytest

from paper_2009_05112_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "smoothing_cases.json")


def test_smoothing_fixtures(orc):
    for c in json.load(open(GOLD))["cases"]:
        d = np.array(c["d"], dtype=float)
        st = orc.refine_stages(1.0, d, np.ones_like(d))
        assert st is not None
        np.testing.assert_array_equal(st[0], d)
        np.testing.assert_allclose(st[1], c["smooth"], rtol=0, atol=1e-15)


def test_smoothing_preserves_total(orc):
    rng = np.random.default_rng(0)
    for n in (2, 3, 7, 100, 1000):
        d = rng.exponential(size=n) * (rng.random(n) < 0.7)
        st = orc.refine_stages(0.5, d, np.ones(n))
        assert abs(st[1].sum() - 1.0) < 1e-13


def test_compression_closed_forms(orc):
    for n in (2, 4, 1000):
        for alpha in (0.0, 0.5, 1.0, 1.5):
            st = orc.refine_stages(alpha, np.ones(n), np.ones(n))
            want = ((1 - 1 / n) / math.log(n)) ** alpha
            np.testing.assert_allclose(st[2], want, rtol=1e-14)
    # monotone in d, zero maps to zero, and (1 - d)/ln(1/d) -> 1 as d -> 1
    d = np.array([0.0, 1e-9, 1e-3, 0.1, 0.5, 0.9, 0.999])
    st = orc.refine_stages(1.0, np.r_[d, 0.0, 0.0], np.ones(d.size + 2))
    c = st[2][1:d.size - 1]
    assert np.all(np.diff(c) > 0)
    z = orc.refine_stages(1.0, np.array([0.0, 0.0, 0.0, 1.0]), np.ones(4))
    assert z[2][0] == 0.0 and z[2][1] == 0.0


def _mass_at(xgrid, c, xq):
    """Cumulative mass of the piecewise-constant density c_j / dx_j at xq."""
    cum = np.r_[0.0, np.cumsum(c)]
    j = np.clip(np.searchsorted(xgrid, xq, side="right") - 1, 0, len(c) - 1)
    frac = (xq - xgrid[j]) / (xgrid[j + 1] - xgrid[j])
    return cum[j] + c[j] * frac


@pytest.mark.parametrize("n_g,alpha,seed", [(10, 0.5, 0), (1000, 0.5, 1), (1000, 1.5, 2), (64, 0.2, 3)])
def test_regrid_equal_share(orc, n_g, alpha, seed):
    rng = np.random.default_rng(seed)
    x = np.sort(np.r_[0.0, rng.random(n_g - 1), 1.0])
    H = rng.exponential(size=n_g) * (rng.random(n_g) < 0.8)
    Wt = rng.integers(1, 50, size=n_g).astype(float)
    p = W.Params(dim=1, n_ev=100, n_g=n_g, alpha=alpha)
    xn = orc.refine_axis(p, H, Wt, x)
    c = orc.refine_stages(alpha, H, Wt)[2]
    assert xn[0] == x[0] and xn[-1] == x[-1]
    assert np.all(np.diff(xn) >= 0)
    m = _mass_at(x, c, xn)
    share = c.sum() / n_g
    np.testing.assert_allclose(m, share * np.arange(n_g + 1), rtol=0, atol=1e-12 * c.sum())


def test_alpha_zero_and_degenerate_axes(orc):
    rng = np.random.default_rng(5)
    n = 50
    x = np.sort(np.r_[0.0, rng.random(n - 1), 1.0])
    H = rng.random(n)
    p0 = W.Params(dim=1, n_ev=100, n_g=n, alpha=0.0)
    assert np.array_equal(orc.refine_axis(p0, H, np.ones(n), x), x)  # alpha = 0: no refinement
    p = W.Params(dim=1, n_ev=100, n_g=n, alpha=0.5)
    assert np.array_equal(orc.refine_axis(p, np.zeros(n), np.ones(n), x), x)  # no signal
    assert np.array_equal(orc.refine_axis(p, H, np.zeros(n), x), x)  # no samples
    p1 = W.Params(dim=1, n_ev=100, n_g=1, alpha=0.5)
    assert np.array_equal(orc.refine_axis(p1, np.ones(1), np.ones(1), np.array([0.0, 1.0])),
                          np.array([0.0, 1.0]))


def test_constant_training_data_is_a_fixed_point(orc):
    # all d_i equal: the grid is already optimal (Eq. onedopt) and is kept
    n = 200
    x = np.linspace(0.0, 1.0, n + 1)
    x[1:-1] += 0.3 / n * np.sin(np.arange(1, n))
    p = W.Params(dim=1, n_ev=100, n_g=n, alpha=0.5)
    xn = orc.refine_axis(p, np.full(n, 3.0), np.full(n, 2.0), x)
    np.testing.assert_allclose(xn, x, rtol=0, atol=1e-14)


def test_map_init(orc):
    p = W.Params(dim=3, n_ev=1000, n_g=7, lower=np.array([-1.0, 0.0, 2.0]), upper=np.array([1.0, 0.5, 3.0]))
    pr = orc.Problem(p, W.const(3))
    m = pr.map_init()
    assert m.shape == (3, 8)
    np.testing.assert_array_equal(m[:, 0], p.lower)
    np.testing.assert_array_equal(m[:, -1], p.upper)
    np.testing.assert_allclose(np.diff(m, axis=1), np.repeat(((p.upper - p.lower) / 7)[:, None], 7, axis=1), rtol=1e-13)
