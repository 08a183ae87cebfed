"""ctypes binding of libvegasp.so (include/vegasp.h): argument marshalling only.

Every computation runs in the library's HIP kernels.  If the library is not
built, or no GPU is visible, the calls raise instead of falling back to
anything else.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvegasp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vegasp.h")

_KIND = {"gauss_mix": 1, "corr_gauss": 2, "exp_abs": 3, "const": 4, "affine": 5, "balls": 6}
_PREC = {"fp64": 0, "fp32_acc64": 1, "fp32_neumaier": 2}
_HIST = {"weighted": 0, "literal": 1}
_AVG = {"weighted": 0, "unweighted": 1}
_STRAT = {"uniform": 0, "mixed": 1}

VP_OK, VP_ERR_INVALID_ARG, VP_ERR_OOM, VP_ERR_DEVICE, VP_ERR_NUMERIC, VP_ERR_NOT_READY, \
    VP_ERR_CANCELLED, VP_ERR_STATE, VP_ERR_INVARIANT = range(9)
VP_FLAG_CHECKS, VP_FLAG_DETERMINISTIC = 1, 2
VP_CHECK_MAP_ORDER, VP_CHECK_MAP_ENDS, VP_CHECK_NH_MIN, VP_CHECK_NH_SUM = 1, 2, 4, 8


class VegaspError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


VP_F_BATCH = 100
# int fn(void* user, void* hip_stream, int64 n, int32 dim, const double* x_soa, double* f_out)
BATCH_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p)


class vp_integrand(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("n_terms", C.c_int32),
                ("centers", C.POINTER(C.c_double)), ("coefs", C.POINTER(C.c_double)),
                ("amps", C.POINTER(C.c_double)), ("chol", C.POINTER(C.c_double)),
                ("scale", C.c_double), ("fn", C.c_void_p), ("user", C.c_void_p), ("n_out", C.c_int32)]


class BatchIntegrand:
    """A batched integrand (VP_F_BATCH): ``fn`` is the address of a
    vp_batch_fn (or a BATCH_FN callback object, kept alive here), ``user``
    the pointer passed to it; the library multiplies its values by scale."""

    def __init__(self, dim: int, fn, user=None, scale: float = 1.0, n_out: int = 1):
        self.dim = dim
        self.scale = scale
        self.n_out = n_out
        self._fn_obj = fn if isinstance(fn, BATCH_FN) else None
        self.fn = C.cast(fn, C.c_void_p).value if isinstance(fn, BATCH_FN) else int(fn)
        self.user = user


class vp_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_ev", C.c_int64), ("n_g", C.c_int32), ("n_iter", C.c_int32),
                ("alpha", C.c_double), ("beta", C.c_double), ("lower", C.POINTER(C.c_double)),
                ("upper", C.POINTER(C.c_double)), ("seed", C.c_uint64), ("precision", C.c_int32),
                ("hist_mode", C.c_int32), ("realloc_plus2", C.c_int32), ("n_discard", C.c_int32),
                ("n_st", C.c_int32), ("n_adapt", C.c_int32), ("average", C.c_int32),
                ("strat", C.c_int32), ("n_st_axes", C.POINTER(C.c_int32)), ("flags", C.c_int32)]


class vp_result(C.Structure):
    _fields_ = [("mean", C.c_double), ("sdev", C.c_double), ("chi2", C.c_double), ("dof", C.c_int32),
                ("n_iter_done", C.c_int32), ("n_evals", C.c_int64), ("n_near_ties", C.c_int64),
                ("n_nonfinite", C.c_int64)]


class vp_server_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("completed", C.c_int64), ("cancelled", C.c_int64),
                ("failed", C.c_int64), ("samples", C.c_int64), ("graph_launches", C.c_int64),
                ("graph_captures", C.c_int64), ("active", C.c_int32), ("pending", C.c_int32),
                ("peak_active", C.c_int32), ("pad", C.c_int32), ("mem_in_use", C.c_int64),
                ("mem_peak", C.c_int64), ("t_admit", C.c_double), ("t_plan", C.c_double),
                ("t_step", C.c_double), ("t_retire", C.c_double)]


VP_SERVER_NO_GRAPH = 1

_lib = None


def lib():
    """Loads libvegasp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        sig = {
            "vp_status_string": ([C.c_int], C.c_char_p),
            "vp_last_error": ([], C.c_char_p),
            "vp_ctx_create": ([C.c_int, vp, C.POINTER(vp)], C.c_int),
            "vp_ctx_destroy": ([vp], C.c_int),
            "vp_ctx_info": ([vp, ip, C.POINTER(C.c_int64)], C.c_int),
            "vp_problem_create": ([vp, C.POINTER(vp_params), C.POINTER(vp_integrand), C.POINTER(vp)], C.c_int),
            "vp_problem_destroy": ([vp], C.c_int),
            "vp_problem_info": ([vp, ip, C.POINTER(C.c_int64)], C.c_int),
            "vp_problem_strat": ([vp, ip], C.c_int),
            "vp_problem_layout": ([vp, ip, ip], C.c_int),
            "vp_map_train": ([vp, C.c_int64, dp, dp, C.c_int32, C.c_double], C.c_int),
            "vp_map_train_noalloc": ([vp, C.c_int64, dp, dp, C.c_int32, C.c_double], C.c_int),
            "vp_result_vec_get": ([vp, dp, dp, dp, ip, dp, dp, C.c_int32], C.c_int),
            "vp_iterate": ([vp, C.c_int32], C.c_int),
            "vp_sync": ([vp], C.c_int),
            "vp_result_get": ([vp, C.POINTER(vp_result), dp, dp, dp, C.c_int32], C.c_int),
            "vp_map_get": ([vp, dp], C.c_int),
            "vp_check_get": ([vp, C.POINTER(C.c_uint32), ip], C.c_int),
            "vp_map_set": ([vp, dp], C.c_int),
            "vp_alloc_get": ([vp, ip], C.c_int),
            "vp_alloc_set": ([vp, ip], C.c_int),
            "vp_iteration_get": ([vp, ip], C.c_int),
            "vp_iteration_set": ([vp, C.c_int32], C.c_int),
            "vp_accum_get": ([vp, dp, dp, dp, dp], C.c_int),
            "vp_debug_dump": ([vp, C.c_int64, C.c_int64], C.c_int),
            "vp_debug_dump_get": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), ip, ip, dp, dp, dp], C.c_int),
            "vp_state_export": ([vp, vp, C.POINTER(C.c_size_t)], C.c_int),
            "vp_state_import": ([vp, vp, C.c_size_t], C.c_int),
            "vp_profile_enable": ([vp, C.c_int32], C.c_int),
            "vp_kernel_time": ([vp, C.c_int32, dp, C.POINTER(C.c_int64)], C.c_int),
            "vp_integrate": ([vp, C.POINTER(vp_params), C.POINTER(vp_integrand), C.POINTER(vp_result)], C.c_int),
            "vp_server_create": ([vp, C.c_size_t, C.c_int32, C.c_int32, C.POINTER(vp)], C.c_int),
            "vp_server_submit": ([vp, C.POINTER(vp_params), C.POINTER(vp_integrand), C.POINTER(C.c_uint64)],
                                 C.c_int),
            "vp_server_submit_many": ([vp, C.c_int32, C.POINTER(vp_params), C.POINTER(vp_integrand),
                                       C.POINTER(C.c_uint64)], C.c_int),
            "vp_server_request_bytes": ([vp, C.POINTER(vp_params), C.POINTER(vp_integrand),
                                         C.POINTER(C.c_size_t)], C.c_int),
            "vp_server_poll": ([vp, C.c_uint64, C.POINTER(vp_result)], C.c_int),
            "vp_server_wait": ([vp, C.c_uint64, C.POINTER(vp_result)], C.c_int),
            "vp_server_times": ([vp, C.c_uint64, dp, dp, dp], C.c_int),
            "vp_server_now": ([vp, dp], C.c_int),
            "vp_server_cancel": ([vp, C.c_uint64], C.c_int),
            "vp_server_stats_get": ([vp, C.POINTER(vp_server_stats)], C.c_int),
            "vp_server_destroy": ([vp], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int, what: str = ""):
    if status != VP_OK:
        msg = lib().vp_last_error().decode(errors="replace")
        raise VegaspError(status, f"{what}: {msg}" if what else msg)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Context:
    """One GPU and one HIP stream (NULL: a stream of the library's own)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.h = C.c_void_p()
        check(lib().vp_ctx_create(device, C.c_void_p(stream) if stream else None, C.byref(self.h)),
              "vp_ctx_create")

    def info(self):
        n = C.c_int32()
        lds = C.c_int64()
        check(lib().vp_ctx_info(self.h, C.byref(n), C.byref(lds)))
        return {"n_cu": n.value, "lds_bytes": lds.value}

    def close(self):
        if self.h:
            lib().vp_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        # at interpreter exit the process teardown releases device memory
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def marshal(params, integrand):
    """(vp_params, vp_integrand, keep-alive list) from workloads.Params and a
    workloads.Integrand or a BatchIntegrand."""
    keep = []
    f = integrand

    def arr(a):
        if a is None:
            return None
        x = np.ascontiguousarray(a, dtype=np.float64).ravel()
        keep.append(x)
        return _dp(x)

    if isinstance(f, BatchIntegrand):
        keep.append(f)
        fi = vp_integrand(VP_F_BATCH, f.dim, 0, None, None, None, None, float(f.scale), f.fn, f.user,
                          int(getattr(f, "n_out", 1)))
    else:
        fi = vp_integrand(_KIND[f.kind], f.dim, f.n_terms, arr(f.centers), arr(f.coefs), arr(f.amps),
                          arr(f.chol), float(f.scale), None, None, 1)
    p = params
    axes = getattr(p, "n_st_axes", None)
    if axes is not None:
        axes = np.ascontiguousarray(axes, dtype=np.int32).ravel()
        keep.append(axes)
    pp = vp_params(p.dim, int(p.n_ev), p.n_g, p.n_iter, float(p.alpha), float(p.beta), arr(p.lower),
                   arr(p.upper), int(p.seed) & ((1 << 64) - 1), _PREC[p.precision], _HIST[p.hist_mode],
                   1 if p.realloc_plus2 else 0, int(p.n_discard), int(getattr(p, "n_st", 0) or 0),
                   int(getattr(p, "n_adapt", 0) or 0), _AVG[getattr(p, "average", "weighted")],
                   _STRAT[getattr(p, "strat", "uniform")], None if axes is None else _ip(axes),
                   int(getattr(p, "flags", 0) or 0))
    return pp, fi, keep


class Problem:
    """Device state of one integration (vp_problem)."""

    def __init__(self, ctx: Context, params, integrand, n_st: int = 0):
        self.ctx = ctx
        self.params = params
        pp, fi, keep = marshal(params, integrand)
        if n_st:
            pp.n_st = n_st
        self.h = C.c_void_p()
        check(lib().vp_problem_create(ctx.h, C.byref(pp), C.byref(fi), C.byref(self.h)), "vp_problem_create")
        ns = C.c_int32()
        nh = C.c_int64()
        check(lib().vp_problem_info(self.h, C.byref(ns), C.byref(nh)))
        self.n_st, self.n_hc = ns.value, nh.value
        ax = np.empty(params.dim, dtype=np.int32)
        check(lib().vp_problem_strat(self.h, _ip(ax)))
        self.n_st_axes = ax
        mp = C.c_int32()
        ha = C.c_int32()
        check(lib().vp_problem_layout(self.h, C.byref(mp), C.byref(ha)))
        self.map_place, self.hist_axes = ("global", "lds", "inner")[mp.value], ha.value

    def iterate(self, n: int = 1):
        check(lib().vp_iterate(self.h, n), "vp_iterate")

    def sync(self):
        check(lib().vp_sync(self.h), "vp_sync")

    def result(self, cap: int | None = None, allow_nonfinite: bool = False):
        r = vp_result()
        cap = cap if cap is not None else 65536
        I = np.zeros(cap)
        V = np.zeros(cap)
        sig = np.zeros(cap)
        st = lib().vp_result_get(self.h, C.byref(r), _dp(I), _dp(sig), _dp(V), cap)
        if not (allow_nonfinite and st == VP_ERR_NUMERIC):
            check(st, "vp_result_get")
        n = r.n_iter_done
        return {"mean": r.mean, "sdev": r.sdev, "chi2": r.chi2, "dof": r.dof, "n_iter_done": n,
                "n_evals": r.n_evals, "ties": r.n_near_ties, "nonfinite": r.n_nonfinite,
                "I": I[:n].copy(), "V": V[:n].copy(), "sig": sig[:n].copy()}

    def checks(self):
        """Device-side invariant findings (vp_check_get): (flags, first iteration)."""
        fl = C.c_uint32()
        it = C.c_int32()
        check(lib().vp_check_get(self.h, C.byref(fl), C.byref(it)), "vp_check_get")
        return fl.value, it.value

    def result_vec(self, m: int, cap: int = 4096):
        """Vector results (vp_result_vec_get) of an integrand with m components."""
        mean = np.empty(m)
        cov = np.empty((m, m))
        chi2 = C.c_double()
        dof = C.c_int32()
        I = np.empty((cap, m))
        Cj = np.empty((cap, m, m))
        check(lib().vp_result_vec_get(self.h, _dp(mean), _dp(cov), C.byref(chi2), C.byref(dof), _dp(I), _dp(Cj),
                                      cap), "vp_result_vec_get")
        n = min(cap, self.it_done())
        return {"mean": mean, "cov": cov, "chi2": chi2.value, "dof": dof.value, "I": I[:n].copy(), "C": Cj[:n].copy()}

    def it_done(self):
        r = vp_result()
        st = lib().vp_result_get(self.h, C.byref(r), None, None, None, 0)
        if st not in (0, VP_ERR_NUMERIC):
            check(st, "vp_result_get")
        return r.n_iter_done

    def train_map(self, x, fx, n_iter: int, alpha: float):
        """Preconditioned map: n_iter training passes on points x [n][dim]
        with values fx (vp_map_train)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        fx = np.ascontiguousarray(fx, dtype=np.float64)
        check(lib().vp_map_train(self.h, len(fx), _dp(x), _dp(fx), int(n_iter), float(alpha)), "vp_map_train")

    def train_map_noalloc(self, x, fx, n_iter: int, alpha: float):
        """As train_map, staging the points in the library's static device
        workspace instead of allocating (vp_map_train_noalloc)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        fx = np.ascontiguousarray(fx, dtype=np.float64)
        check(lib().vp_map_train_noalloc(self.h, len(fx), _dp(x), _dp(fx), int(n_iter), float(alpha)),
              "vp_map_train_noalloc")

    def map(self):
        P = self.params
        m = np.empty((P.dim, P.n_g + 1))
        check(lib().vp_map_get(self.h, _dp(m)), "vp_map_get")
        return m

    def set_map(self, m):
        m = np.ascontiguousarray(m, dtype=np.float64)
        check(lib().vp_map_set(self.h, _dp(m)), "vp_map_set")

    def alloc(self):
        n = np.empty(self.n_hc, dtype=np.int32)
        check(lib().vp_alloc_get(self.h, _ip(n)), "vp_alloc_get")
        return n

    def set_alloc(self, n_h):
        n = np.ascontiguousarray(n_h, dtype=np.int32)
        check(lib().vp_alloc_set(self.h, _ip(n)), "vp_alloc_set")

    @property
    def it(self) -> int:
        v = C.c_int32()
        check(lib().vp_iteration_get(self.h, C.byref(v)))
        return v.value

    def set_it(self, it: int):
        check(lib().vp_iteration_set(self.h, it), "vp_iteration_set")

    def accum(self):
        P = self.params
        S1 = np.empty(self.n_hc)
        S2 = np.empty(self.n_hc)
        H = np.empty((P.dim, P.n_g))
        W = np.empty((P.dim, P.n_g))
        check(lib().vp_accum_get(self.h, _dp(S1), _dp(S2), _dp(H), _dp(W)), "vp_accum_get")
        return {"S1": S1, "S2": S2, "H": H, "W": W}

    def debug_dump(self, first: int, count: int):
        """Arms the per-sample dump of the next iteration (vp_debug_dump)."""
        check(lib().vp_debug_dump(self.h, int(first), int(count)), "vp_debug_dump")
        self._dump_count = int(count)

    def debug_dump_get(self):
        """The dumped samples (vp_debug_dump_get): h, j [n]; idx, x [n][dim]; jac, fx [n]."""
        c = self._dump_count
        D = self.params.dim
        n = C.c_int64()
        h = np.empty(c, dtype=np.int64)
        j = np.empty(c, dtype=np.int32)
        idx = np.empty(D * c, dtype=np.int32)
        x = np.empty(D * c)
        jac = np.empty(c)
        fx = np.empty(c)
        check(lib().vp_debug_dump_get(self.h, C.byref(n), h.ctypes.data_as(C.POINTER(C.c_int64)), _ip(j), _ip(idx),
                                      _dp(x), _dp(jac), _dp(fx)), "vp_debug_dump_get")
        m = n.value
        return {"h": h[:m].copy(), "j": j[:m].copy(), "idx": idx[:D * m].reshape(D, m).T.copy(),
                "x": x[:D * m].reshape(D, m).T.copy(), "jac": jac[:m].copy(), "fx": fx[:m].copy()}

    def export_state(self) -> bytes:
        n = C.c_size_t(0)
        check(lib().vp_state_export(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(lib().vp_state_export(self.h, buf, C.byref(n)), "vp_state_export")
        return buf.raw[: n.value]

    def import_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        check(lib().vp_state_import(self.h, buf, len(blob)), "vp_state_import")

    def profile(self, on: bool = True):
        check(lib().vp_profile_enable(self.h, 1 if on else 0))

    def kernel_time(self, which: int = 0):
        t = C.c_double()
        n = C.c_int64()
        check(lib().vp_kernel_time(self.h, which, C.byref(t), C.byref(n)), "vp_kernel_time")
        return t.value, n.value

    def close(self):
        if self.h:
            lib().vp_problem_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        # at interpreter exit the process teardown releases device memory
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def integrate(ctx: Context, params, integrand, prepared=None):
    """vp_integrate; prepared: the (params, integrand) structures from
    marshal(), when the caller built them beforehand."""
    pp, fi, keep = prepared if prepared is not None else marshal(params, integrand)
    r = vp_result()
    check(lib().vp_integrate(ctx.h, C.byref(pp), C.byref(fi), C.byref(r)), "vp_integrate")
    return {"mean": r.mean, "sdev": r.sdev, "chi2": r.chi2, "dof": r.dof, "n_evals": r.n_evals,
            "n_iter_done": r.n_iter_done, "ties": r.n_near_ties}


def _result_dict(r):
    return {"mean": r.mean, "sdev": r.sdev, "chi2": r.chi2, "dof": r.dof, "n_evals": r.n_evals,
            "n_iter_done": r.n_iter_done, "ties": r.n_near_ties, "nonfinite": r.n_nonfinite}


class Server:
    """Continuous-batching server (vp_server): submit integrations from any
    thread, the library's scheduler runs all admitted ones in batched steps."""

    def __init__(self, ctx: Context, mem_budget: int = 0, max_slots: int = 256, graphs: bool = True):
        self.ctx = ctx
        self.h = C.c_void_p()
        flags = 0 if graphs else VP_SERVER_NO_GRAPH
        check(lib().vp_server_create(ctx.h, int(mem_budget), int(max_slots), flags, C.byref(self.h)),
              "vp_server_create")

    def submit(self, params, integrand) -> int:
        pp, fi, keep = marshal(params, integrand)
        t = C.c_uint64()
        check(lib().vp_server_submit(self.h, C.byref(pp), C.byref(fi), C.byref(t)), "vp_server_submit")
        return t.value

    @staticmethod
    def prepare(reqs):
        """The C structures of (params, integrand) pairs, for submit_many."""
        n = len(reqs)
        P = (vp_params * n)()
        F = (vp_integrand * n)()
        keep = []
        for i, (p, f) in enumerate(reqs):
            pp, fi, k = marshal(p, f)
            P[i] = pp
            F[i] = fi
            keep.append(k)
        return n, P, F, keep

    def submit_many(self, reqs) -> list:
        """vp_server_submit_many: a list of (params, integrand) pairs, or
        what prepare() returned for one; the tickets in order."""
        n, P, F, keep = reqs if isinstance(reqs, tuple) else self.prepare(reqs)
        T = (C.c_uint64 * max(n, 1))()
        check(lib().vp_server_submit_many(self.h, n, P, F, T), "vp_server_submit_many")
        return [int(T[i]) for i in range(n)]

    def request_bytes(self, params, integrand) -> int:
        pp, fi, keep = marshal(params, integrand)
        n = C.c_size_t()
        check(lib().vp_server_request_bytes(self.h, C.byref(pp), C.byref(fi), C.byref(n)),
              "vp_server_request_bytes")
        return n.value

    def poll(self, ticket: int):
        """The result once finished, None while it runs."""
        r = vp_result()
        st = lib().vp_server_poll(self.h, ticket, C.byref(r))
        if st == VP_ERR_NOT_READY:
            return None
        check(st, "vp_server_poll")
        return _result_dict(r)

    def wait(self, ticket: int):
        r = vp_result()
        check(lib().vp_server_wait(self.h, ticket, C.byref(r)), "vp_server_wait")
        return _result_dict(r)

    def times(self, ticket: int):
        """(submitted, admitted, finished) in seconds on the server's clock."""
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        check(lib().vp_server_times(self.h, ticket, C.byref(a), C.byref(b), C.byref(c)), "vp_server_times")
        return a.value, b.value, c.value

    def now(self) -> float:
        t = C.c_double()
        check(lib().vp_server_now(self.h, C.byref(t)))
        return t.value

    def cancel(self, ticket: int):
        check(lib().vp_server_cancel(self.h, ticket), "vp_server_cancel")

    def stats(self):
        st = vp_server_stats()
        check(lib().vp_server_stats_get(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in vp_server_stats._fields_ if k != "pad"}

    def close(self):
        if self.h:
            lib().vp_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


EXAMPLES_PATH = os.path.join(HERE, "libvegasp_examples.so")
_examples = None


def examples():
    """libvegasp_examples.so (include/vegasp_examples.h): example batched
    integrands; raises if it has not been built."""
    global _examples
    if _examples is None:
        if not os.path.exists(EXAMPLES_PATH):
            raise RuntimeError(f"{EXAMPLES_PATH} is missing: build it first")
        L = C.CDLL(EXAMPLES_PATH)
        dp = C.POINTER(C.c_double)
        L.vp_example_gauss_mix_user.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, C.POINTER(C.c_void_p)]
        L.vp_example_gauss_mix_user.restype = C.c_int
        ip = C.POINTER(C.c_int32)
        L.vp_example_gauss_moments_user.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, C.c_int32, ip, ip,
                                                    C.POINTER(C.c_void_p)]
        L.vp_example_gauss_moments_user.restype = C.c_int
        L.vp_example_free_user.argtypes = [C.c_void_p]
        L.vp_example_free_user.restype = C.c_int
        _examples = L
    return _examples


def example_gauss_mix(integrand):
    """A BatchIntegrand evaluating a workloads gauss_mix Integrand through the
    example library (same operations as the built-in kind)."""
    L = examples()
    f = integrand
    c = np.ascontiguousarray(f.centers, dtype=np.float64).ravel()
    k = np.ascontiguousarray(f.coefs, dtype=np.float64)
    a = np.ascontiguousarray(f.amps, dtype=np.float64)
    user = C.c_void_p()
    rc = L.vp_example_gauss_mix_user(f.dim, f.n_terms, _dp(c), _dp(k), _dp(a), C.byref(user))
    if rc != 0:
        raise VegaspError(VP_ERR_INVALID_ARG, f"vp_example_gauss_mix_user returned {rc}")
    fn = C.cast(L.vp_example_gauss_mix, C.c_void_p).value
    return BatchIntegrand(f.dim, fn, user.value, scale=f.scale)


def example_gauss_moments(integrand, e1, e2):
    """A vector-valued BatchIntegrand: component a is the workloads gauss_mix
    density times the monomial (x_e1[a] or 1)(x_e2[a] or 1)."""
    L = examples()
    f = integrand
    c = np.ascontiguousarray(f.centers, dtype=np.float64).ravel()
    k = np.ascontiguousarray(f.coefs, dtype=np.float64)
    a = np.ascontiguousarray(f.amps, dtype=np.float64)
    i1 = np.ascontiguousarray(e1, dtype=np.int32)
    i2 = np.ascontiguousarray(e2, dtype=np.int32)
    user = C.c_void_p()
    rc = L.vp_example_gauss_moments_user(f.dim, f.n_terms, _dp(c), _dp(k), _dp(a), len(i1), _ip(i1), _ip(i2),
                                         C.byref(user))
    if rc != 0:
        raise VegaspError(VP_ERR_INVALID_ARG, f"vp_example_gauss_moments_user returned {rc}")
    fn = C.cast(L.vp_example_gauss_moments, C.c_void_p).value
    return BatchIntegrand(f.dim, fn, user.value, scale=f.scale, n_out=len(i1))


def declared_symbols(header: str = HEADER) -> list:
    """Function names declared in include/vegasp.h."""
    import re
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(vp_\w+)\s*\(", src, flags=re.M)))
