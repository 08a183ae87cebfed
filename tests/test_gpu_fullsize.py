"""GPU parity at the full D=8, N_ev=1e8 size (16.7M hypercubes), in the launch
configuration the benchmark times.  The oracle runs the whole iteration on the
host's threads (one contiguous block of hypercubes each): every hypercube's
sums and every bin of the training data are compared with it, and the
reductions, the allocation and the refinement are recomputed in full from the
GPU's sums, up to the largest size the interface accepts (1.72e9 samples).
The training data are also checked through invariants that hold at any
size.  The samples of one range of
hypercubes per iteration are dumped by the sampling kernel (vp_debug_dump) and
compared one by one with the oracle's: indices bit for bit, x and J to the
last bit."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2009_05112_amd import _binding as B
from paper_2009_05112_amd import workloads as W
from tests.parity import RTOL64, assert_close, variance_scale

pytestmark = pytest.mark.gpu


def _arm_dump(gp, n_h, h0, width=2000):
    """Dump of the samples of hypercubes [h0, h0 + width) of the next iteration."""
    first = int(n_h[:h0].astype(np.int64).sum())
    count = int(n_h[h0:h0 + width].astype(np.int64).sum())
    gp.debug_dump(first, count)
    return h0, h0 + width


def _check_dump(gp, op, fmap, n_h, it, hr, rtol_f=1e-12):
    d = gp.debug_dump_get()
    o = op.sample_points(fmap, n_h, it, hr[0], hr[1])
    assert len(d["h"]) == len(o["h"])
    for k in ("h", "j", "idx", "x", "jac"):
        np.testing.assert_array_equal(d[k], o[k], err_msg=f"dumped {k} of hypercubes {hr}")
    np.testing.assert_allclose(d["fx"], o["fx"], rtol=rtol_f, atol=rtol_f * 1e-3 * np.abs(o["fx"]).max(),
                               err_msg=f"dumped f(x) of hypercubes {hr}")


def _oracle_iteration(op, fmap, n_h, it):
    """The whole iteration from the oracle: per-hypercube sums S1, S2 and the
    training data H, W [dim][n_g], the hypercubes in one contiguous block per
    host thread (the oracle's range call releases the interpreter), the
    blocks' training data added in block order."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    n = max(1, min(n, cap) if cap > 0 else n)
    edges = [op.n_hc * t // n for t in range(n + 1)]
    with ThreadPoolExecutor(max_workers=n) as ex:
        parts = list(ex.map(lambda t: op.sample_range(fmap, n_h, it, edges[t], edges[t + 1]), range(n)))
    H = np.zeros_like(parts[0]["H"])
    W = np.zeros_like(parts[0]["W"])
    for q in parts:
        H += q["H"]
        W += q["W"]
    return np.concatenate([q["S1"] for q in parts]), np.concatenate([q["S2"] for q in parts]), H, W


def _check_iteration(gp, op, fmap, n_h, it, rtol=RTOL64, floor=0.0, rtol_hist=None):
    """Every hypercube's sums and every bin of the training data against the
    oracle's whole iteration.  rtol, floor: the per-hypercube sums' bar (the
    split precisions compare sums of single-precision values; everything
    after the sums is double precision and held to 1e-12 either way).
    rtol_hist: the training data's bar, relative to each axis's total
    (default rtol)."""
    acc = gp.accum()
    res = gp.result()
    top1, top2 = np.abs(acc["S1"]).max(), np.abs(acc["S2"]).max()
    rh = rtol if rtol_hist is None else rtol_hist
    S1o, S2o, Ho, Wo = _oracle_iteration(op, fmap, n_h, it)
    s1, s2 = acc["S1"], acc["S2"]
    sc1 = np.maximum(np.maximum(np.abs(s1), np.abs(S1o)), floor * top1 / rtol)
    sc2 = np.maximum(np.maximum(np.abs(s2), np.abs(S2o)), floor * top2 / rtol)
    assert_close(s1, S1o, rtol, scale=sc1, what="S1 (every hypercube)")
    assert_close(s2, S2o, rtol, scale=sc2, what="S2 (every hypercube)")
    del S1o, S2o, sc1, sc2
    for m in range(Ho.shape[0]):
        assert_close(acc["W"][m], Wo[m], rh, scale=np.abs(Wo[m]).sum(), what=f"W[{m}]")
        assert_close(acc["H"][m], Ho[m], rh, scale=np.abs(Ho[m]).sum(), what=f"H[{m}]")
    # invariants of the training data: every hypercube adds n_h * (1/n_h) = 1
    # to W on every axis (the compensated split weighs by the single-precision
    # 1/n_h, so n_h fl32(1/n_h)); every sample adds the same v^2/n_h to one bin
    # per axis
    if op.params.precision == "fp32_neumaier":
        n32 = n_h.astype(np.float32)
        w_tot = float(((np.float32(1.0) / n32).astype(np.float64) * n_h).sum())
    else:
        w_tot = float(gp.n_hc)
    np.testing.assert_allclose(acc["W"].sum(axis=1), w_tot, rtol=1e-12)
    hs = acc["H"].sum(axis=1)
    np.testing.assert_allclose(hs, hs[0], rtol=1e-12)
    I, V = op.reduce(n_h, acc["S1"], acc["S2"])
    assert_close(res["I"][-1], I, RTOL64, what="I_j")
    assert_close(res["V"][-1], V, RTOL64, scale=variance_scale(gp.n_hc, n_h, acc["S2"]), what="V_j")
    n_o, ties = op.realloc(acc["S1"], acc["S2"], n_h)
    n_g = gp.alloc()
    diff = np.flatnonzero(n_g != n_o)
    assert diff.size == 0, f"n_h differs at {diff.size} hypercubes (oracle near-ties {ties})"
    m_o = op.refine(acc["H"], acc["W"], fmap)
    assert_close(gp.map(), m_o, RTOL64, scale=np.ones_like(m_o), what="map")
    return res


def test_fullsize_diag_d8_two_iterations():
    ctx = B.Context(0)
    p, f = W.cfg_diag_d8()
    gp = B.Problem(ctx, p, f)
    op = oracle.Problem(p, f, n_st=gp.n_st)
    assert (gp.n_st, gp.n_hc) == (8, 8 ** 8)
    for k in range(2):
        fmap, n_h, it = gp.map(), gp.alloc(), gp.it
        hr = _arm_dump(gp, n_h, gp.n_hc // 2 if k == 0 else gp.n_hc - 2000)
        gp.iterate(1)
        res = _check_iteration(gp, op, fmap, n_h, it)
        _check_dump(gp, op, fmap, n_h, it, hr)
    assert res["n_evals"] > 1.5e8
    gp.close()
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32_acc64", "fp32_neumaier"])
def test_fullsize_split_d8_two_iterations(prec):
    """The precision split (single-precision map and integrand; double sums,
    or compensated single-precision pairs) at the same size: the sums and
    the training data against the oracle's whole iteration in the same
    precision (2e-6, as in the split's step-wise tests), the double-precision
    steps from the GPU's sums at 1e-12."""
    ctx = B.Context(0)
    p, f = W.cfg_diag_d8(precision=prec)
    gp = B.Problem(ctx, p, f)
    op = oracle.Problem(p, f, n_st=gp.n_st)
    assert gp.map_place == "inner" and gp.hist_axes == 8
    for _ in range(2):
        fmap, n_h, it = gp.map(), gp.alloc(), gp.it
        hr = _arm_dump(gp, n_h, gp.n_hc // 3)
        gp.iterate(1)
        res = _check_iteration(gp, op, fmap, n_h, it, rtol=2e-6, floor=1e-12)
        _check_dump(gp, op, fmap, n_h, it, hr, rtol_f=2e-6)
    assert res["n_evals"] > 1.5e8
    gp.close()
    ctx.close()


def test_fullsize_batched_d8_two_iterations():
    """The benchmark's batched-integrand workload: the D=8 three-Gaussian
    problem at N_ev=1e8, its points written as structure-of-arrays buffers
    and f evaluated by the example library's Gaussian mixture (a user
    function); two iterations, each against the oracle's whole iteration."""
    ctx = B.Context(0)
    p, f = W.cfg_diag_d8()
    bf = B.example_gauss_mix(f)
    try:
        gp = B.Problem(ctx, p, bf)
        op = oracle.Problem(p, f, n_st=gp.n_st)
        assert (gp.n_st, gp.n_hc) == (8, 8 ** 8)
        for _ in range(2):
            fmap, n_h, it = gp.map(), gp.alloc(), gp.it
            gp.iterate(1)
            res = _check_iteration(gp, op, fmap, n_h, it)
        assert res["n_evals"] > 1.5e8
        gp.close()
    finally:
        B.examples().vp_example_free_user(bf.user)
    ctx.close()


def test_fullsize_deterministic_d8():
    """The bitwise-deterministic mode at the benchmark's size: two runs of
    two iterations agree bit for bit in every output, and each iteration of
    the first passes the whole-iteration comparison with the oracle."""
    ctx = B.Context(0)
    p, f = W.cfg_diag_d8()
    p = p.with_(flags=B.VP_FLAG_DETERMINISTIC)
    runs = []
    for k in range(2):
        gp = B.Problem(ctx, p, f)
        op = oracle.Problem(p, f, n_st=gp.n_st) if k == 0 else None
        out = []
        for _ in range(2):
            fmap, n_h, it = gp.map(), gp.alloc(), gp.it
            gp.iterate(1)
            if op is not None:
                _check_iteration(gp, op, fmap, n_h, it)
            acc = gp.accum()
            out.append({"S1": acc["S1"], "S2": acc["S2"], "H": acc["H"], "W": acc["W"], "map": gp.map(),
                        "n_h": gp.alloc()})
        r = gp.result()
        out.append({key: np.asarray(r[key]) for key in ("mean", "sdev", "I", "V", "n_evals")})
        runs.append(out)
        gp.close()
    for k, (x, y) in enumerate(zip(*runs)):
        for key in x:
            np.testing.assert_array_equal(x[key], y[key], err_msg=f"step {k}: {key}")
    ctx.close()


def test_maxsize_d8_one_iteration():
    """The largest N_ev the interface accepts (2^31 - 1) at D=8: N_st = 12,
    N_hc = 12^8 = 429,981,696 (R = 1000/12 is not an integer), four samples per
    hypercube, 1.72e9 samples in one launch, every hypercube and bin against
    the oracle's whole iteration (about 30 GB of host memory)."""
    ctx = B.Context(0)
    p, f = W.cfg_diag_d8(n_ev=2**31 - 1)
    gp = B.Problem(ctx, p, f)
    op = oracle.Problem(p, f, n_st=gp.n_st)
    assert (gp.n_st, gp.n_hc) == (12, 12 ** 8)
    fmap, n_h, it = gp.map(), gp.alloc(), gp.it
    assert int(n_h.min()) == int(n_h.max()) == 4
    hr = _arm_dump(gp, n_h, gp.n_hc - 1000, width=1000)  # samples numbered beyond 2^31
    gp.iterate(1)
    res = _check_iteration(gp, op, fmap, n_h, it)
    _check_dump(gp, op, fmap, n_h, it, hr)
    assert res["n_evals"] == 4 * 12 ** 8
    gp.close()
    ctx.close()


@pytest.mark.parametrize("prec,dim,n_st", [("fp64", 6, 17), ("fp32_acc64", 4, 70)])
def test_fullsize_high_digits(prec, dim, n_st):
    """Digits of 16 and more (double precision, D=6) and of 64 and more (the
    split, D=4) reach the top bits of the 32-bit word in which the sampler
    joins a hypercube's digit with its axis's random bits (Sec. 3, uniform y
    within each hypercube).  About 2.4e7 hypercubes, four samples each; the
    last hypercubes (every digit at its largest) are dumped and compared
    sample by sample, the sampled sums and the steps after them as above."""
    ctx = B.Context(0)
    p = W.Params(dim=dim, n_ev=100_000_000, n_g=1000, n_iter=1, seed=6, precision=prec,
                 n_st_axes=np.full(dim, n_st, dtype=np.int32))
    f = W.gauss_single(dim, coef=20.0)
    gp = B.Problem(ctx, p, f)
    op = oracle.Problem(p, f, n_st=gp.n_st)
    assert (gp.n_st, gp.n_hc) == (n_st, n_st ** dim)
    fmap, n_h, it = gp.map(), gp.alloc(), gp.it
    assert int(n_h.min()) >= 4
    hr = _arm_dump(gp, n_h, gp.n_hc - 2000)
    gp.iterate(1)
    kw = {} if prec == "fp64" else {"rtol": 2e-6, "floor": 1e-12}
    _check_iteration(gp, op, fmap, n_h, it, **kw)
    _check_dump(gp, op, fmap, n_h, it, hr, rtol_f=1e-12 if prec == "fp64" else 2e-6)
    gp.close()
    ctx.close()
