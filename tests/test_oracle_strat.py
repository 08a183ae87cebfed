"""Mixed stratification (Sec. 4): the rule for per-axis counts, the
mixed-radix hypercube index, and the sampling inside each hypercube, pinned
by the paper's own figures, brute force and the uniform special case."""
import itertools
import math

import numpy as np
import pytest

import oracle as orc
from paper_2009_05112_amd import workloads as W


def brute_mixed(dim, n_ev):
    """Largest d with 4 (N+1)^d N^(dim-d) <= n_ev by enumeration, N from Eq. Nst_vegasp."""
    n = 1
    while 4 * (n + 1) ** dim <= n_ev:
        n += 1
    d = max(dd for dd in range(dim + 1) if 4 * (n + 1) ** dd * n ** (dim - dd) <= n_ev or dd == 0)
    return [n + 1] * d + [n] * (dim - d), d


def test_mixed_rule_paper_figures():
    # Sec. 4: with at most 2.5e5 samples, d = 15 and N_st = 1 for D > 15 (2^15
    # hypercubes, where the uniform rule has one); with 5e4 samples, 2^13
    # hypercubes for D > 13, while the uniform rule drops from 2^13 at D = 13
    # to a single hypercube at D = 14.
    for D in (16, 20, 30, 50):
        axes, d = orc.nst_mixed(D, 250_000)
        assert d == 15 and orc.nst(D, 250_000) == 1
        assert int(np.prod(axes.astype(np.int64))) == 2 ** 15
    for D in (14, 20, 40):
        axes, d = orc.nst_mixed(D, 50_000)
        assert d == 13 and int(np.prod(axes.astype(np.int64))) == 2 ** 13
    assert orc.nst(13, 50_000) == 2 and orc.nst(14, 50_000) == 1


@pytest.mark.parametrize("seed", range(4))
def test_mixed_rule_brute_force(seed):
    rng = np.random.default_rng(seed)
    for _ in range(60):
        D = int(rng.integers(1, 11))
        n_ev = int(10 ** rng.uniform(1, 7.5))
        axes, d = orc.nst_mixed(D, n_ev)
        want, wd = brute_mixed(D, n_ev)
        assert list(axes) == want and d == wd, (D, n_ev)
        assert 4 * int(np.prod(axes.astype(np.int64))) <= n_ev or orc.nst(D, n_ev) == 1


def _digits(h, counts):
    k = []
    for c in reversed(counts):
        k.append(h % c)
        h //= c
    return k[::-1]


@pytest.mark.parametrize("prec", ["fp64", "fp32_acc64"])
def test_samples_fall_in_their_mixed_radix_cell(prec):
    # every sample of hypercube h has floor(y^mu N_st^mu) = k_mu, the digits
    # of h in the mixed radix of the counts (axis 0 most significant), so t =
    # y N_g lies in [k_mu R_mu, (k_mu + 1) R_mu]
    counts = [3, 1, 2, 4]
    p = W.Params(dim=4, n_ev=400, n_g=24, seed=3, precision=prec, n_st_axes=np.array(counts))
    pr = orc.Problem(p, W.const(4))
    assert pr.n_hc == 24 and list(pr.n_st_axes) == counts
    n_h = pr.alloc_init()
    idx, t = pr.sample_indices(n_h, it=0, with_t=True)
    hs = np.repeat(np.arange(pr.n_hc), n_h)
    for s in range(hs.size):
        k = _digits(int(hs[s]), counts)
        for mu in range(4):
            R = 24 / counts[mu]
            assert k[mu] * R <= t[s, mu] <= (k[mu] + 1) * R
            assert idx[s, mu] == min(int(math.floor(t[s, mu])), 23)
    # every cell of the product grid is visited
    cells = {tuple(_digits(int(h), counts)) for h in hs}
    assert cells == set(itertools.product(*[range(c) for c in counts]))


def test_equal_counts_are_the_uniform_path():
    # per-axis counts that are all equal reproduce the uniform stratification
    # bit for bit (same digits, same R)
    f = W.gauss_single(3)
    p = W.Params(dim=3, n_ev=5000, n_g=30, seed=8)
    a = orc.Problem(p, f)
    b = orc.Problem(p.with_(n_st_axes=np.array([a.n_st] * 3)), f)
    ra = a.iteration(a.map_init(), a.alloc_init(), it=0)
    rb = b.iteration(b.map_init(), b.alloc_init(), it=0)
    for key in ("S1", "S2", "H", "W"):
        assert np.array_equal(ra[key], rb[key])
    assert ra["I"] == rb["I"] and ra["V"] == rb["V"]


def test_mixed_stratification_integrates():
    # constant integrand: exact for any stratification; a narrow Gaussian:
    # within the error
    counts = np.array([4, 3, 1, 2, 2])
    p = W.Params(dim=5, n_ev=3000, n_g=40, n_iter=4, seed=2, n_st_axes=counts)
    r = orc.Problem(p, W.const(5)).integrate()
    assert abs(r["mean"] - 1.0) < 1e-13
    f = W.gauss_single(6, coef=20.0)
    p = W.Params(dim=6, n_ev=30_000, n_g=50, n_iter=10, seed=4, strat="mixed", n_discard=3)
    pr = orc.Problem(p, f)
    assert list(pr.n_st_axes) == [5, 5, 4, 4, 4, 4]
    r = pr.integrate()
    assert abs(r["mean"] - f.exact) < 5 * r["sdev"]


def test_stratifying_the_structured_axes_halves_the_error():
    # Sec. 6 (D = 21 fit): with too few samples for N_st = 2 on every axis,
    # 46 stratifications on each of the two sharply determined directions and
    # none on the others cut the error about in half at the same N_ev.  Here a
    # Gaussian narrow in axes 0 and 1 and broad in the other 19.
    D = 21
    s = np.array([0.03, 0.03] + [0.4] * 19)
    mu = np.array([0.4, 0.6] + [0.5] * 19)
    exact = float(np.prod([W.gauss_box_1d(1 / (2 * si * si), m) for si, m in zip(s, mu)]))
    f = W.Integrand("corr_gauss", D, mu.reshape(1, -1), [0.5], [1.0], chol=np.diag(1.0 / s), exact=exact)
    err = {}
    for name, axes in (("none", None), ("46x46", np.array([46, 46] + [1] * 19))):
        rel = []
        for seed in range(2):
            p = W.Params(dim=D, n_ev=12_000, n_g=100, n_iter=20, seed=seed, n_discard=10, n_st_axes=axes)
            pr = orc.Problem(p, f)
            assert pr.n_hc == (1 if axes is None else 46 * 46)
            r = pr.integrate()
            assert abs(r["mean"] - exact) < 5 * r["sdev"]
            rel.append(r["sdev"] / exact)
        err[name] = float(np.mean(rel))
    assert err["46x46"] < 0.7 * err["none"]
