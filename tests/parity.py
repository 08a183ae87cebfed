"""Shared helpers of the GPU parity tests: one iteration on the GPU compared
element by element with the oracle run from the same state."""
import numpy as np

import oracle
from paper_2009_05112_amd import _binding as B

# Double-precision bar: 1e-12 relative (sums per hypercube, the estimate, the
# variance); per-increment training data relative to the axis total; the map
# relative to the box width.
RTOL64 = 1e-12


def assert_close(a, b, rtol, scale=None, what=""):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if scale is None:
        scale = np.maximum(np.abs(a), np.abs(b))
    err = np.abs(a - b)
    bad = err > rtol * scale + 1e-300
    if np.any(bad):
        i = np.flatnonzero(bad.ravel())[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} differ beyond rtol={rtol}; "
                             f"first at {i}: gpu={a.ravel()[i]} oracle={b.ravel()[i]}")


def variance_scale(n_hc, n_h, S2):
    """Scale of the one-pass variance before cancellation: the per-iteration
    variance is sum_h (Omega^2 S2_h/n_h - (Omega S1_h/n_h)^2)/(n_h - 1); its
    rounding error is relative to sum_h Omega^2 S2_h / n_h / (n_h - 1)."""
    om2 = (1.0 / n_hc) ** 2
    n = np.asarray(n_h, dtype=np.float64)
    return float(np.sum(om2 * np.asarray(S2) / n / (n - 1.0)))


def step_and_compare(gp: B.Problem, op: oracle.Problem, rtol=RTOL64, rtol_hist=RTOL64,
                     exact_counts=False, check_map=True, check_alloc=True, floor=0.0):
    """Run one GPU iteration from its current state, run the oracle from the
    same (map, n_h, it), compare every output.  Returns the oracle's outputs.
    floor: per-hypercube sums are compared up to an absolute floor of
    floor * max|sum| (single-precision paths: values near the FP32 underflow
    threshold are denormal, with few significant bits, and carry no weight in
    any result)."""
    fmap = gp.map()
    n_h = gp.alloc()
    it = gp.it
    gp.iterate(1)
    acc = gp.accum()
    res = gp.result(allow_nonfinite=True)
    o = op.sample_range(fmap, n_h, it)
    sc1 = np.maximum(np.abs(acc["S1"]), np.abs(o["S1"]))
    sc2 = np.maximum(np.abs(acc["S2"]), np.abs(o["S2"]))
    assert_close(acc["S1"], o["S1"], rtol, scale=np.maximum(sc1, floor * sc1.max() / rtol), what="S1")
    assert_close(acc["S2"], o["S2"], rtol, scale=np.maximum(sc2, floor * sc2.max() / rtol), what="S2")
    for m in range(fmap.shape[0]):
        if exact_counts:
            np.testing.assert_array_equal(acc["W"][m], o["W"][m])
        else:
            assert_close(acc["W"][m], o["W"][m], rtol_hist, scale=np.abs(o["W"][m]).sum(), what=f"W[{m}]")
        assert_close(acc["H"][m], o["H"][m], rtol_hist, scale=np.abs(o["H"][m]).sum(), what=f"H[{m}]")
    I, V = op.reduce(n_h, o["S1"], o["S2"])
    assert_close(res["I"][-1], I, rtol, what="I_j")
    assert_close(res["V"][-1], V, rtol, scale=variance_scale(op.n_hc, n_h, o["S2"]), what="V_j")
    out = {"acc": acc, "oracle": o, "I": I, "V": V, "fmap": fmap, "n_h": n_h, "it": it}
    if check_alloc:
        # reallocation from the GPU's own sums (isolates the allocation rule)
        n_o, ties = op.realloc(acc["S1"], acc["S2"], n_h)
        n_g = gp.alloc()
        diff = np.flatnonzero(n_g != n_o)
        assert diff.size == 0, f"n_h differs at {diff[:10]} ({diff.size}); oracle near-ties {ties}"
        out["n_new"] = n_g
    if check_map:
        m_o = op.refine(acc["H"], acc["W"], fmap)
        m_g = gp.map()
        P = op.params
        width = (np.ones(P.dim) if P.upper is None else (np.asarray(P.upper) - np.asarray(P.lower)))
        assert_close(m_g, m_o, rtol, scale=width[:, None] * np.ones_like(m_o), what="map")
        out["map_new"] = m_g
    return out
