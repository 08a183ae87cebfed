"""ctypes binding of the CPU oracle (oracle/vp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark; never by the library.  Every array crossing the
boundary is a contiguous numpy array; the C side follows the paper step by
step in FP64 (see the comments in vp_oracle.c for the passage of each step).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_KIND = {"gauss_mix": 1, "corr_gauss": 2, "exp_abs": 3, "const": 4, "affine": 5, "balls": 6}
_PREC = {"fp64": 0, "fp32_acc64": 1, "fp32_neumaier": 2}
_HIST = {"weighted": 0, "literal": 1}


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_ev", C.c_int64), ("n_g", C.c_int32), ("n_st", C.c_int32),
                ("alpha", C.c_double), ("beta", C.c_double), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("hist_mode", C.c_int32), ("realloc_plus2", C.c_int32),
                ("n_adapt", C.c_int32), ("n_st_axes", C.c_int32 * 64)]


class _Integrand(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("n_terms", C.c_int32),
                ("centers", C.POINTER(C.c_double)), ("coefs", C.POINTER(C.c_double)),
                ("amps", C.POINTER(C.c_double)), ("chol", C.POINTER(C.c_double)),
                ("scale", C.c_double)]


class _Rec(C.Structure):
    _fields_ = [("h", C.c_int64), ("j", C.c_int32), ("pad", C.c_int32), ("v", C.c_double),
                ("jac", C.c_double), ("fx", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(
                os.path.join(_HERE, "vp_oracle.c")):
            _build.build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.or_nst.argtypes = [C.c_int32, C.c_int64]
        L.or_nst.restype = C.c_int32
        L.or_vec_iteration.argtypes = [C.POINTER(_Params), C.POINTER(_Integrand), dp, ip, C.c_int32, C.c_int32,
                                       ip, ip, dp, dp, dp]
        L.or_vec_iteration.restype = C.c_int
        L.or_train_hist.argtypes = [C.POINTER(_Params), dp, dp, C.c_int64, dp, dp, dp]
        L.or_train_hist.restype = C.c_int
        L.or_map_train.argtypes = [C.POINTER(_Params), dp, dp, C.c_int64, dp, C.c_int32, C.c_double]
        L.or_map_train.restype = C.c_int
        L.or_nst_mixed.argtypes = [C.c_int32, C.c_int64, C.POINTER(C.c_int32)]
        L.or_nst_mixed.restype = C.c_int32
        L.or_nst_classic.argtypes = [C.c_int32, C.c_int64]
        L.or_nst_classic.restype = C.c_int32
        L.or_integrand_eval.argtypes = [C.POINTER(_Integrand), dp]
        L.or_integrand_eval.restype = C.c_double
        L.or_n_hypercubes.argtypes = [C.POINTER(_Params)]
        L.or_n_hypercubes.restype = C.c_int64
        L.or_map_init.argtypes = [C.c_int32, C.c_int32, dp, dp, dp]
        L.or_alloc_init.argtypes = [C.POINTER(_Params), ip]
        L.or_sample_range.argtypes = [C.POINTER(_Params), C.POINTER(_Integrand), dp, ip, C.c_int32,
                                      C.c_int64, C.c_int64, dp, dp, dp, dp, C.POINTER(_Rec),
                                      C.c_int64, C.POINTER(C.c_int64)]
        L.or_sample_range.restype = C.c_int
        L.or_sample_indices.argtypes = [C.POINTER(_Params), ip, C.c_int32, C.c_int64, C.c_int64,
                                        ip, dp, C.c_int64]
        L.or_sample_indices.restype = C.c_int
        L.or_sample_points.argtypes = [C.POINTER(_Params), C.POINTER(_Integrand), dp, ip, C.c_int32, C.c_int64,
                                       C.c_int64, C.POINTER(C.c_int64), ip, ip, dp, dp, dp, C.c_int64]
        L.or_sample_points.restype = C.c_int
        L.or_reduce.argtypes = [C.POINTER(_Params), ip, dp, dp, dp, dp]
        L.or_realloc.argtypes = [C.POINTER(_Params), dp, dp, ip, ip]
        L.or_realloc.restype = C.c_int64
        L.or_refine_axis.argtypes = [C.POINTER(_Params), dp, dp, dp, dp]
        L.or_refine_axis.restype = C.c_int
        L.or_refine_stages.argtypes = [C.POINTER(_Params), dp, dp, dp, dp, dp]
        L.or_refine_stages.restype = C.c_int
        L.or_refine.argtypes = [C.POINTER(_Params), dp, dp, dp]
        L.or_refine.restype = C.c_int
        L.or_combine.argtypes = [dp, dp, C.c_int32, C.c_int32, C.c_int32, dp, dp, dp, ip]
        L.or_iteration.argtypes = [C.POINTER(_Params), C.POINTER(_Integrand), dp, ip, C.c_int32,
                                   dp, dp, dp, dp, dp, dp]
        L.or_iteration.restype = C.c_int64
        L.or_integrate.argtypes = [C.POINTER(_Params), C.POINTER(_Integrand), dp, ip, C.c_int32,
                                   C.c_int32, dp, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.or_integrate.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


# ------------------------------------------------------------------ helpers
def nst(dim: int, n_ev: int) -> int:
    return int(lib().or_nst(dim, n_ev))


def nst_mixed(dim: int, n_ev: int):
    """Per-axis stratifications of the mixed rule and its d (Sec. 4)."""
    out = np.zeros(dim, dtype=np.int32)
    d = lib().or_nst_mixed(dim, n_ev, _ip(out))
    return out, int(d)


def nst_classic(dim: int, n_ev: int) -> int:
    return int(lib().or_nst_classic(dim, n_ev))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


class Problem:
    """Parameters and integrand marshalled for the C side (keeps buffers alive)."""

    def __init__(self, params, integrand, n_st: int | None = None):
        self.params = params
        self.f = integrand
        ns = n_st if n_st is not None else nst(params.dim, params.n_ev)
        axes = getattr(params, "n_st_axes", None)
        if axes is not None:
            axes = np.asarray(axes, dtype=np.int32).ravel()
        elif getattr(params, "strat", "uniform") == "mixed":
            axes, _ = nst_mixed(params.dim, params.n_ev)
        else:
            axes = np.full(params.dim, ns, dtype=np.int32)
        self.n_st_axes = axes
        ns = int(axes[0])
        self.n_st = ns
        self.p = _Params(params.dim, int(params.n_ev), params.n_g, ns, float(params.alpha),
                         float(params.beta), int(params.seed) & ((1 << 64) - 1),
                         _PREC[params.precision], _HIST[params.hist_mode],
                         1 if params.realloc_plus2 else 0, int(getattr(params, "n_adapt", 0) or 0),
                         (C.c_int32 * 64)(*[int(v) for v in axes]))
        f = integrand
        self._centers = np.ascontiguousarray(f.centers, dtype=np.float64).ravel()
        self._coefs = np.ascontiguousarray(f.coefs, dtype=np.float64)
        self._amps = np.ascontiguousarray(f.amps, dtype=np.float64)
        self._chol = (np.ascontiguousarray(f.chol, dtype=np.float64).ravel()
                      if f.chol is not None else np.zeros(1))
        self.fi = _Integrand(_KIND[f.kind], f.dim, f.n_terms, _dp(self._centers), _dp(self._coefs),
                             _dp(self._amps), _dp(self._chol), float(f.scale))
        self.n_hc = int(lib().or_n_hypercubes(C.byref(self.p)))

    # -- state
    def map_init(self):
        P = self.params
        m = np.empty((P.dim, P.n_g + 1))
        lo = None if P.lower is None else np.ascontiguousarray(P.lower, dtype=np.float64)
        hi = None if P.upper is None else np.ascontiguousarray(P.upper, dtype=np.float64)
        lib().or_map_init(P.dim, P.n_g, _dp(lo) if lo is not None else None,
                          _dp(hi) if hi is not None else None, _dp(m))
        return m

    def alloc_init(self):
        n = np.empty(self.n_hc, dtype=np.int32)
        lib().or_alloc_init(C.byref(self.p), _ip(n))
        return n

    def f_eval(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return float(lib().or_integrand_eval(C.byref(self.fi), _dp(x)))

    # -- steps
    def sample_range(self, fmap, n_h, it, h0=0, h1=None, records: int = 0):
        P = self.params
        h1 = self.n_hc if h1 is None else h1
        fmap = np.ascontiguousarray(fmap, dtype=np.float64)
        n_h = np.ascontiguousarray(n_h, dtype=np.int32)
        S1 = np.zeros(h1 - h0)
        S2 = np.zeros(h1 - h0)
        H = np.zeros((P.dim, P.n_g))
        W = np.zeros((P.dim, P.n_g))
        rec = (_Rec * records)() if records else None
        cnt = C.c_int64(0)
        rc = lib().or_sample_range(C.byref(self.p), C.byref(self.fi), _dp(fmap), _ip(n_h), it, h0, h1,
                                   _dp(S1), _dp(S2), _dp(H), _dp(W), rec, records, C.byref(cnt))
        if rc != 0:
            raise RuntimeError(f"or_sample_range failed: {rc}")
        out = {"S1": S1, "S2": S2, "H": H, "W": W, "n_samples": int(cnt.value)}
        if records:
            m = min(records, cnt.value)
            out["rec"] = {
                "h": np.array([rec[i].h for i in range(m)]),
                "j": np.array([rec[i].j for i in range(m)]),
                "v": np.array([rec[i].v for i in range(m)]),
                "jac": np.array([rec[i].jac for i in range(m)]),
                "fx": np.array([rec[i].fx for i in range(m)]),
            }
        return out

    def sample_indices(self, n_h, it, h0=0, h1=None, with_t=False):
        P = self.params
        h1 = self.n_hc if h1 is None else h1
        n_h = np.ascontiguousarray(n_h, dtype=np.int32)
        ns = int(n_h[h0:h1].astype(np.int64).sum())
        idx = np.empty((ns, P.dim), dtype=np.int32)
        t = np.empty((ns, P.dim)) if with_t else None
        rc = lib().or_sample_indices(C.byref(self.p), _ip(n_h), it, h0, h1, _ip(idx),
                                     _dp(t) if with_t else None, ns)
        if rc != 0:
            raise RuntimeError("or_sample_indices failed")
        return (idx, t) if with_t else idx

    def sample_points(self, fmap, n_h, it, h0=0, h1=None):
        """Every sample of hypercubes [h0, h1) in (h, j) order: h, j [n];
        idx, x [n][dim]; jac, fx [n]."""
        P = self.params
        h1 = self.n_hc if h1 is None else h1
        n_h = np.ascontiguousarray(n_h, dtype=np.int32)
        ns = int(n_h[h0:h1].astype(np.int64).sum())
        h = np.empty(ns, dtype=np.int64)
        j = np.empty(ns, dtype=np.int32)
        idx = np.empty((ns, P.dim), dtype=np.int32)
        x = np.empty((ns, P.dim))
        jac = np.empty(ns)
        fx = np.empty(ns)
        rc = lib().or_sample_points(C.byref(self.p), C.byref(self.fi), _dp(np.ascontiguousarray(fmap, dtype=np.float64)),
                                    _ip(n_h), it, h0, h1, h.ctypes.data_as(C.POINTER(C.c_int64)), _ip(j), _ip(idx),
                                    _dp(x), _dp(jac), _dp(fx), ns)
        if rc != 0:
            raise RuntimeError("or_sample_points failed")
        return {"h": h, "j": j, "idx": idx, "x": x, "jac": jac, "fx": fx}

    def vec_iteration(self, fmap, n_h, it, e1, e2):
        """Vector estimates of one iteration (Sec. 6) for the components
        f * (x_e1 or 1) * (x_e2 or 1): I [M], C [M][M] and the scale [M] of
        the variance terms before cancellation."""
        e1 = np.ascontiguousarray(e1, dtype=np.int32)
        e2 = np.ascontiguousarray(e2, dtype=np.int32)
        M = len(e1)
        I = np.empty(M)
        Cm = np.empty((M, M))
        sc = np.empty(M)
        rc = lib().or_vec_iteration(C.byref(self.p), C.byref(self.fi), _dp(np.ascontiguousarray(fmap)),
                                    _ip(np.ascontiguousarray(n_h, dtype=np.int32)), it, M, _ip(e1), _ip(e2),
                                    _dp(I), _dp(Cm), _dp(sc))
        if rc != 0:
            raise RuntimeError("or_vec_iteration failed")
        return I, Cm, sc

    def train_hist(self, x, fx, fmap):
        """Training data of the preconditioned map (Sec. 5.2) for points x
        [n][dim] with values fx under the map fmap: H, W [dim][n_g]."""
        P = self.params
        x = np.ascontiguousarray(x, dtype=np.float64)
        fx = np.ascontiguousarray(fx, dtype=np.float64)
        m = np.ascontiguousarray(fmap, dtype=np.float64)
        H = np.empty((P.dim, P.n_g))
        W = np.empty((P.dim, P.n_g))
        if lib().or_train_hist(C.byref(self.p), _dp(x), _dp(fx), len(fx), _dp(m), _dp(H), _dp(W)) != 0:
            raise RuntimeError("or_train_hist failed")
        return H, W

    def map_train(self, x, fx, fmap, n_iter, alpha):
        """n_iter training passes from fmap; returns the trained map."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        fx = np.ascontiguousarray(fx, dtype=np.float64)
        m = np.array(fmap, dtype=np.float64, copy=True)
        if lib().or_map_train(C.byref(self.p), _dp(x), _dp(fx), len(fx), _dp(m), n_iter, float(alpha)) != 0:
            raise RuntimeError("or_map_train failed")
        return m

    def reduce(self, n_h, S1, S2):
        I = C.c_double()
        V = C.c_double()
        lib().or_reduce(C.byref(self.p), _ip(np.ascontiguousarray(n_h, dtype=np.int32)),
                        _dp(np.ascontiguousarray(S1)), _dp(np.ascontiguousarray(S2)), C.byref(I),
                        C.byref(V))
        return I.value, V.value

    def realloc(self, S1, S2, n_h):
        n_h = np.ascontiguousarray(n_h, dtype=np.int32)
        out = np.empty_like(n_h)
        ties = lib().or_realloc(C.byref(self.p), _dp(np.ascontiguousarray(S1)),
                                _dp(np.ascontiguousarray(S2)), _ip(n_h), _ip(out))
        return out, int(ties)

    def refine(self, H, W, fmap):
        m = np.array(fmap, dtype=np.float64, copy=True, order="C")
        lib().or_refine(C.byref(self.p), _dp(np.ascontiguousarray(H)), _dp(np.ascontiguousarray(W)),
                        _dp(m))
        return m

    def iteration(self, fmap, n_h, it):
        """One full iteration from (map, n_h); returns the sums and the next state."""
        P = self.params
        m = np.array(fmap, dtype=np.float64, copy=True, order="C")
        n = np.array(n_h, dtype=np.int32, copy=True)
        S1 = np.empty(self.n_hc)
        S2 = np.empty(self.n_hc)
        H = np.empty((P.dim, P.n_g))
        W = np.empty((P.dim, P.n_g))
        I = C.c_double()
        V = C.c_double()
        ties = lib().or_iteration(C.byref(self.p), C.byref(self.fi), _dp(m), _ip(n), it, _dp(S1),
                                  _dp(S2), _dp(H), _dp(W), C.byref(I), C.byref(V))
        if ties < 0:
            raise RuntimeError("or_iteration failed")
        return {"S1": S1, "S2": S2, "H": H, "W": W, "I": I.value, "V": V.value, "map": m, "n_h": n,
                "ties": int(ties)}

    def integrate(self, n_iter=None, fmap=None, n_h=None, it0=0):
        n_iter = self.params.n_iter if n_iter is None else n_iter
        m = self.map_init() if fmap is None else np.array(fmap, dtype=np.float64, copy=True)
        n = self.alloc_init() if n_h is None else np.array(n_h, dtype=np.int32, copy=True)
        I = np.empty(n_iter)
        V = np.empty(n_iter)
        ties = C.c_int64(0)
        evals = C.c_int64(0)
        rc = lib().or_integrate(C.byref(self.p), C.byref(self.fi), _dp(m), _ip(n), it0, n_iter, _dp(I),
                                _dp(V), C.byref(ties), C.byref(evals))
        if rc != 0:
            raise RuntimeError("or_integrate failed")
        sig = np.sqrt(V)
        mean, sdev, chi2, dof = combine(I, sig, self.params.n_discard, getattr(self.params, "average", "weighted"))
        return {"I": I, "V": V, "sig": sig, "mean": mean, "sdev": sdev, "chi2": chi2, "dof": dof,
                "map": m, "n_h": n, "ties": int(ties.value), "n_evals": int(evals.value)}


def combine(I, sig, n_discard: int = 0, average: str = "weighted"):
    I = np.ascontiguousarray(I, dtype=np.float64)
    sig = np.ascontiguousarray(sig, dtype=np.float64)
    mean = C.c_double()
    sdev = C.c_double()
    chi2 = C.c_double()
    dof = C.c_int32()
    lib().or_combine(_dp(I), _dp(sig), I.size, n_discard, 1 if average == "unweighted" else 0, C.byref(mean), C.byref(sdev), C.byref(chi2),
                     C.byref(dof))
    return mean.value, sdev.value, chi2.value, int(dof.value)


def _positive_definite(A):
    """Cholesky pivots all above 1e-14 of their diagonal entries (the rule
    that decides between the weighted and the unweighted combination)."""
    m = A.shape[0]
    L = np.zeros_like(A)
    for i in range(m):
        for j in range(i + 1):
            s = A[i, j] - sum(L[i, k] * L[j, k] for k in range(j))
            if i == j:
                if not s > 1e-14 * A[i, i]:
                    return False
                L[i, i] = np.sqrt(s)
            else:
                L[i, j] = s / L[j, j]
    return True


def combine_vec(I, Cs, n_discard: int = 0, average: str = "weighted"):
    """Combination of vector estimates over iterations n_discard.. (Sec. 2.5
    for several correlated integrals, Sec. 6): with C_j^-1 weights, the mean
    (sum C_j^-1)^-1 sum C_j^-1 I_j and its covariance (sum C_j^-1)^-1; else
    (or when some C_j is not positive definite) the plain mean with covariance
    sum C_j / count^2.  chi^2 = sum (I_j - mean)^T C_j^-1 (I_j - mean), NaN
    when some C_j is not positive definite; dof = (count - 1) M."""
    I = np.asarray(I, dtype=np.float64)
    Cs = np.asarray(Cs, dtype=np.float64)
    first = max(0, n_discard)
    I, Cs = I[first:], Cs[first:]
    cnt, M = I.shape
    if cnt <= 0:
        return np.full(M, np.nan), np.full((M, M), np.nan), float("nan"), 0
    pd = all(_positive_definite(c) for c in Cs)
    if average == "weighted" and pd:
        Ws = [np.linalg.inv(c) for c in Cs]
        SW = sum(Ws)
        cov = np.linalg.inv(SW)
        mean = cov @ sum(w @ i for w, i in zip(Ws, I))
    else:
        mean = I.mean(axis=0)
        cov = Cs.sum(axis=0) / cnt ** 2
    if pd:
        chi2 = float(sum((i - mean) @ np.linalg.solve(c, i - mean) for i, c in zip(I, Cs)))
    else:
        chi2 = float("nan")
    return mean, cov, chi2, (cnt - 1) * M


def refine_axis(params, H, W, x):
    """Refine one axis (N_g = len(H)) in place on a copy; returns the new grid."""
    p = _Params(1, 1, len(H), 1, float(params.alpha), float(params.beta), 0, 0, 0, 0)
    xx = np.array(x, dtype=np.float64, copy=True)
    work = np.empty(4 * (len(H) + 1))
    lib().or_refine_axis(C.byref(p), _dp(np.ascontiguousarray(H, dtype=np.float64)),
                         _dp(np.ascontiguousarray(W, dtype=np.float64)), _dp(xx), _dp(work))
    return xx


def refine_stages(alpha, H, W):
    """(raw d, smoothed+normalised d, compressed d) of one axis, or None when
    the axis would not be refined."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    n = H.size
    p = _Params(1, 1, n, 1, float(alpha), 0.0, 0, 0, 0, 0)
    a, b, c = np.zeros(n), np.zeros(n), np.zeros(n)
    ok = lib().or_refine_stages(C.byref(p), _dp(H), _dp(W), _dp(a), _dp(b), _dp(c))
    return (a, b, c) if ok else None
