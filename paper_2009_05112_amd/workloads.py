"""Seeded synthetic inputs: integrands, problem parameters and request mixes.

This module holds no step of the integration method.  It only builds the
integrands the method is run on (with their exact integrals where a closed
form exists) and the parameter sets of the workloads, so that the HIP library,
the CPU oracle, the tests and the benchmark all see identical inputs.

The integrands are the paper's test functions or Gaussian analogues of them:

* ``gauss_diag`` -- D=8, three Gaussians exp(-100 |x - c|^2) centred on the
  diagonal at c = 0.23, 0.39, 0.74; the Gaussian analogue of the exponential
  peaks of Sec. 3.1, Eq. (exponentials), normalised to integral 1.
* ``gauss_single`` -- D=4, one Gaussian exp(-100 |x - 1/2|^2) normalised to 1,
  the one-peak form of Sec. 2.4, Eq. (easy).
* ``easy`` -- Sec. 2.4, Eq. (easy): two Gaussians at r1, r2 of Eq. (easyr).
* ``balls`` -- Sec. 2.4, Eq. (balls): indicator of two 4-balls of radius 0.067.
* ``exponentials`` -- Sec. 3.1, Eq. (exponentials): exp(-50 |x - r_i|).
* ``served_batch`` / ``served_stream`` -- request mixes for the serving loop
  (isotropic Gaussian mixtures; correlated Gaussians with a random rotation).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

KINDS = ("gauss_mix", "corr_gauss", "exp_abs", "const", "affine", "balls")
PRECISIONS = ("fp64", "fp32_acc64", "fp32_neumaier")
HIST_MODES = ("weighted", "literal")


@dataclass
class Integrand:
    """f(x) = scale * g(x); ``kind`` selects g (see KINDS).

    gauss_mix:  g = sum_k amps[k] exp(-coefs[k] |x - centers[k]|^2)
    corr_gauss: g = exp(-1/2 |U (x - centers[0])|^2), U = chol (upper-triangular)
    exp_abs:    g = sum_k amps[k] exp(-coefs[k] |x - centers[k]|)
    const:      g = 1
    affine:     g = a_0 + sum_d a_{d+1} x_d with a = centers.ravel()
    balls:      g = sum_k amps[k] [ |x - centers[k]| < coefs[k] ]
    """

    kind: str
    dim: int
    centers: np.ndarray
    coefs: np.ndarray
    amps: np.ndarray
    chol: Optional[np.ndarray] = None
    scale: float = 1.0
    exact: Optional[float] = None  # exact integral over the box, when known
    # correlated Gaussian only: the rotation Q and standard deviations s the
    # covariance Sigma = Q diag(s^2) Q^T was built from (generator inputs)
    rotation: Optional[np.ndarray] = None
    sdevs: Optional[np.ndarray] = None

    def __post_init__(self):
        assert self.kind in KINDS, self.kind
        self.centers = np.ascontiguousarray(self.centers, dtype=np.float64)
        self.coefs = np.ascontiguousarray(self.coefs, dtype=np.float64).ravel()
        self.amps = np.ascontiguousarray(self.amps, dtype=np.float64).ravel()
        if self.chol is not None:
            self.chol = np.ascontiguousarray(self.chol, dtype=np.float64)

    @property
    def n_terms(self) -> int:
        return int(self.amps.size)


@dataclass
class Params:
    """The problem statement of the method: dimension, samples per iteration,
    map increments, damping parameters, iterations, box and generator seed."""

    dim: int
    n_ev: int
    n_g: int = 1000
    n_iter: int = 10
    alpha: float = 0.5
    beta: float = 0.75
    seed: int = 0
    precision: str = "fp64"
    hist_mode: str = "weighted"
    realloc_plus2: bool = False
    n_discard: int = 0
    n_adapt: int = 0            # > 0: iterations from this index on neither reallocate nor refine
    average: str = "weighted"   # combination of the kept iterations: "weighted" or "unweighted"
    strat: str = "uniform"      # stratifications per axis: "uniform" or "mixed" (N_st + 1 on the first axes)
    n_st_axes: Optional[np.ndarray] = None  # explicit per-axis stratifications (override strat)
    lower: Optional[np.ndarray] = None
    upper: Optional[np.ndarray] = None
    flags: int = 0              # library options: 1 device-side checks, 2 deterministic training data

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


# --------------------------------------------------------------------------
# exact integrals of the building blocks (inputs' normalisation)
# --------------------------------------------------------------------------
def gauss_box_1d(coef: float, c: float, a: float = 0.0, b: float = 1.0) -> float:
    """Integral of exp(-coef (x - c)^2) over [a, b]."""
    s = math.sqrt(coef)
    return 0.5 * math.sqrt(math.pi / coef) * (math.erf(s * (b - c)) - math.erf(s * (a - c)))


def gauss_mix_exact(centers: np.ndarray, coefs, amps) -> float:
    tot = 0.0
    for k in range(len(amps)):
        p = float(amps[k])
        for c in centers[k]:
            p *= gauss_box_1d(float(coefs[k]), float(c))
        tot += p
    return tot


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
def gauss_single(dim: int = 4, coef: float = 100.0, c: float = 0.5) -> Integrand:
    centers = np.full((1, dim), c)
    z = gauss_mix_exact(centers, [coef], [1.0])
    return Integrand("gauss_mix", dim, centers, [coef], [1.0], scale=1.0 / z, exact=1.0)


def gauss_diag(dim: int = 8, coef: float = 100.0, cs=(0.23, 0.39, 0.74)) -> Integrand:
    centers = np.array([[c] * dim for c in cs])
    amps = np.ones(len(cs))
    coefs = np.full(len(cs), coef)
    z = gauss_mix_exact(centers, coefs, amps)
    return Integrand("gauss_mix", dim, centers, coefs, amps, scale=1.0 / z, exact=1.0)


def easy() -> Integrand:
    centers = np.array([[0.33, 0.5, 0.5, 0.5], [0.67, 0.5, 0.5, 0.5]])
    z = gauss_mix_exact(centers, [100.0, 100.0], [1.0, 1.0])
    return Integrand("gauss_mix", 4, centers, [100.0, 100.0], [1.0, 1.0], exact=z)


def balls(radius: float = 0.067) -> Integrand:
    centers = np.array([[0.33, 0.5, 0.5, 0.5], [0.67, 0.5, 0.5, 0.5]])
    # both balls lie inside the unit box and do not overlap: 2 x volume of a 4-ball
    vol = 2.0 * 0.5 * math.pi ** 2 * radius ** 4
    return Integrand("balls", 4, centers, [radius, radius], [1.0, 1.0], exact=vol)


def exponentials(dim: int = 8, a: float = 50.0, cs=(0.23, 0.39, 0.74)) -> Integrand:
    centers = np.array([[c] * dim for c in cs])
    return Integrand("exp_abs", dim, centers, np.full(len(cs), a), np.ones(len(cs)))


def const(dim: int, value: float = 1.0) -> Integrand:
    return Integrand("const", dim, np.zeros((1, dim)), [0.0], [1.0], scale=value)


def affine(coeffs) -> Integrand:
    a = np.asarray(coeffs, dtype=np.float64)
    dim = a.size - 1
    return Integrand("affine", dim, a.reshape(1, -1), [0.0], [1.0])


def cfg_small_d4() -> (Params, Integrand):
    """D=4 normalised Gaussian at the centre, N_ev=1e5, 10 iterations, N_g=1000."""
    return Params(dim=4, n_ev=100_000, n_g=1000, n_iter=10, alpha=0.5, beta=0.75, seed=0), gauss_single(4)


def cfg_diag_d8(n_ev: int = 100_000_000, precision: str = "fp64") -> (Params, Integrand):
    """D=8 three diagonal Gaussians, N_ev=1e8, 20 iterations, N_g=1000."""
    return (Params(dim=8, n_ev=n_ev, n_g=1000, n_iter=20, alpha=0.5, beta=0.75, seed=0,
                   precision=precision), gauss_diag(8))


# --------------------------------------------------------------------------
# request mixes for the serving loop
# --------------------------------------------------------------------------
@dataclass
class Request:
    params: Params
    integrand: Integrand
    arrival: float = 0.0


def served_batch(n_req: int = 4096, seed: int = 0, d_range=(2, 16), nev_log=(4.0, 6.0),
                 n_iter: int = 10, n_g: int = 500) -> List[Request]:
    """Isotropic Gaussian mixtures: D ~ U{2..16}, N_ev log-uniform in [1e4, 1e6],
    K ~ U{1..4} terms with centres in [0.2, 0.8]^D and widths s in [0.05, 0.2]
    (g_k = exp(-|x - c_k|^2 / (2 s_k^2))), amplitude 1; Philox seed = index."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_req):
        dim = int(rng.integers(d_range[0], d_range[1] + 1))
        n_ev = int(round(10 ** rng.uniform(*nev_log)))
        k = int(rng.integers(1, 5))
        centers = rng.uniform(0.2, 0.8, size=(k, dim))
        widths = rng.uniform(0.05, 0.2, size=k)
        coefs = 1.0 / (2.0 * widths ** 2)
        amps = np.ones(k)
        exact = gauss_mix_exact(centers, coefs, amps)
        f = Integrand("gauss_mix", dim, centers, coefs, amps, exact=exact)
        p = Params(dim=dim, n_ev=n_ev, n_g=n_g, n_iter=n_iter, alpha=0.5, beta=0.75, seed=r)
        out.append(Request(p, f, 0.0))
    return out


def precondition_points(n: int, centers, coef: float, width: float = 1.0, seed: int = 0) -> np.ndarray:
    """Points drawn from Gaussians exp(-coef |x - c|^2) around the given
    centres (one chosen uniformly per point), widened by `width`, kept inside
    the unit box by redrawing: the kind of sample an MCMC run or a peak finder
    supplies for training a map before integrating.  [n][dim]."""
    rng = np.random.default_rng(seed)
    centers = np.asarray(centers, dtype=np.float64)
    sd = width / math.sqrt(2.0 * coef)
    out = np.empty((n, centers.shape[1]))
    have = 0
    while have < n:
        k = rng.integers(0, len(centers), size=n - have)
        x = centers[k] + sd * rng.standard_normal((n - have, centers.shape[1]))
        x = x[np.all((x >= 0.0) & (x <= 1.0), axis=1)]
        out[have:have + len(x)] = x
        have += len(x)
    return out


def haar_rotation(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Haar-random orthogonal matrix: QR of a Gaussian matrix with the signs of
    R's diagonal folded into Q (Mezzadri 2007)."""
    a = rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(a)
    return q * np.sign(np.diag(r))


def corr_gauss(rng: np.random.Generator, dim: int, s_max: float = 0.05, cond: float = 100.0,
               mu_range=(0.3, 0.7)) -> Integrand:
    """exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)), Sigma = Q diag(s^2) Q^T with s spaced
    geometrically from s_max down to s_max / sqrt(cond) (so cond(Sigma) = cond)."""
    s_min = s_max / math.sqrt(cond)
    s = np.geomspace(s_max, s_min, dim) if dim > 1 else np.array([s_max])
    q = haar_rotation(rng, dim)
    prec = q @ np.diag(1.0 / s ** 2) @ q.T
    prec = 0.5 * (prec + prec.T)
    u = np.linalg.cholesky(prec).T  # upper: U^T U = prec
    mu = rng.uniform(mu_range[0], mu_range[1], size=dim)
    exact = (2.0 * math.pi) ** (dim / 2.0) * float(np.prod(s))
    return Integrand("corr_gauss", dim, mu.reshape(1, -1), [0.5], [1.0], chol=np.triu(u), exact=exact,
                     rotation=q, sdevs=s)


def served_stream(n_req: int, rate: float, seed: int = 1, d_range=(3, 21), nev_log=(5.0, 7.0),
                  it_range=(5, 20), n_g: int = 1000) -> List[Request]:
    """Poisson arrivals at ``rate`` requests/s of correlated Gaussians: D ~ U{3..21},
    N_ev log-uniform in [1e5, 1e7], 5-20 iterations."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_req):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        dim = int(rng.integers(d_range[0], d_range[1] + 1))
        n_ev = int(round(10 ** rng.uniform(*nev_log)))
        n_it = int(rng.integers(it_range[0], it_range[1] + 1))
        f = corr_gauss(rng, dim)
        p = Params(dim=dim, n_ev=n_ev, n_g=n_g, n_iter=n_it, alpha=0.5, beta=0.75, seed=1000 + r)
        out.append(Request(p, f, t))
    return out
