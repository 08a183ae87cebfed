"""Device-side invariant checks (VP_FLAG_CHECKS) and the bitwise-deterministic
mode (VP_FLAG_DETERMINISTIC).

Checks: the state each iteration starts from must have a finite, strictly
increasing map from the box's lower to its upper end on every axis (Sec. 2.2),
n_h >= 2 (Sec. 3), and a scanned total equal to sum n_h.  Clean runs in every
mode report nothing and give the results of unchecked runs; maps the host
accepts but that break an invariant (a zero-width increment, a moved end
point) are reported with the iteration at which they were seen.

Deterministic mode: two runs from the same inputs agree bit for bit in every
output (sums, training data, map, allocation, estimates), and each iteration
still matches the oracle at the usual bar (Sec. 3 steps 1-4)."""
import numpy as np
import pytest

import oracle
from paper_2009_05112_amd import _binding as B
from paper_2009_05112_amd import workloads as W
from tests.parity import RTOL64, assert_close, step_and_compare

pytestmark = pytest.mark.gpu

CHECKS, DET = B.VP_FLAG_CHECKS, B.VP_FLAG_DETERMINISTIC


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def _cases():
    p4, f4 = W.cfg_small_d4()
    p8, f8 = W.cfg_diag_d8(n_ev=1_000_000)
    return {
        "d4": (p4.with_(n_iter=4), f4),
        "d4_literal_plus2": (p4.with_(n_iter=4, hist_mode="literal", realloc_plus2=True), f4),
        "d4_frozen": (p4.with_(n_iter=5, n_adapt=2, n_discard=2, average="unweighted"), f4),
        "d6_mixed": (W.Params(dim=6, n_ev=200_000, n_g=300, n_iter=3, seed=4, strat="mixed"),
                     W.gauss_single(6, coef=20.0)),
        "d8": (p8.with_(n_iter=3), f8),
        "d8_fp32": (W.cfg_diag_d8(n_ev=1_000_000, precision="fp32_acc64")[0].with_(n_iter=3), f8),
    }


@pytest.mark.parametrize("case", list(_cases()))
def test_checks_clean_runs(ctx, case):
    p, f = _cases()[case]
    gc = B.Problem(ctx, p.with_(flags=CHECKS), f)
    gc.iterate(p.n_iter)
    rc = gc.result()  # raises on VP_ERR_INVARIANT
    assert gc.checks() == (0, -1)
    gp = B.Problem(ctx, p, f)
    gp.iterate(p.n_iter)
    rp = gp.result()
    assert rc["n_evals"] == rp["n_evals"]
    np.testing.assert_array_equal(gc.alloc(), gp.alloc())
    assert_close(rc["mean"], rp["mean"], RTOL64, what="mean")
    assert_close(rc["sdev"], rp["sdev"], RTOL64, what="sdev")
    with pytest.raises(B.VegaspError) as e:
        gp.checks()  # created without the flag
    assert e.value.status == B.VP_ERR_STATE
    gc.close()
    gp.close()


def test_checks_find_zero_width_increment(ctx):
    p, f = W.cfg_small_d4()
    gp = B.Problem(ctx, p.with_(flags=CHECKS), f)
    gp.iterate(2)
    assert gp.checks() == (0, -1)
    m = gp.map()
    m[1, 7] = m[1, 6]  # accepted by the host (non-decreasing), not strictly increasing
    gp.set_map(m)
    gp.iterate(1)
    with pytest.raises(B.VegaspError) as e:
        gp.result()
    assert e.value.status == B.VP_ERR_INVARIANT
    flags, it = gp.checks()
    assert flags == B.VP_CHECK_MAP_ORDER and it == 2
    gp.close()


def test_checks_find_moved_end_point(ctx):
    p, f = W.cfg_small_d4()
    gp = B.Problem(ctx, p.with_(flags=CHECKS), f)
    m = gp.map()
    m[3, 0] = 0.25 * m[3, 1]  # inside the box: increasing, but no longer starts at the lower end
    gp.set_map(m)
    gp.iterate(1)
    with pytest.raises(B.VegaspError) as e:
        gp.result()
    assert e.value.status == B.VP_ERR_INVARIANT
    assert gp.checks() == (B.VP_CHECK_MAP_ENDS, 0)
    gp.close()


def _run_outputs(ctx, p, f, n):
    gp = B.Problem(ctx, p, f)
    out = []
    for _ in range(n):
        gp.iterate(1)
        acc = gp.accum()
        out.append({"S1": acc["S1"], "S2": acc["S2"], "H": acc["H"], "W": acc["W"], "map": gp.map(),
                    "n_h": gp.alloc()})
    r = gp.result()
    gp.close()
    return out, r


@pytest.mark.parametrize("prec", ["fp64", "fp32_acc64"])
def test_deterministic_runs_bitwise_equal(ctx, prec):
    p, f = W.cfg_diag_d8(n_ev=1_000_000, precision=prec)
    p = p.with_(n_iter=3, flags=DET)
    a, ra = _run_outputs(ctx, p, f, 3)
    b, rb = _run_outputs(ctx, p, f, 3)
    for k, (x, y) in enumerate(zip(a, b)):
        for key in x:
            np.testing.assert_array_equal(x[key], y[key], err_msg=f"iteration {k}: {key}")
    for key in ("mean", "sdev", "chi2", "I", "V", "n_evals"):
        np.testing.assert_array_equal(ra[key], rb[key], err_msg=key)


@pytest.mark.parametrize("prec", ["fp64", "fp32_acc64"])
def test_deterministic_matches_oracle(ctx, prec):
    """Each deterministic iteration against the oracle, as every other path."""
    p, f = W.cfg_diag_d8(n_ev=400_000, precision=prec)
    gp = B.Problem(ctx, p.with_(n_iter=3, seed=8, flags=DET | CHECKS), f)
    assert gp.hist_axes == 0  # every axis through the records
    op = oracle.Problem(p.with_(n_iter=3, seed=8), f, n_st=gp.n_st)
    kw = {} if prec == "fp64" else {"rtol": 2e-6, "rtol_hist": 2e-6, "floor": 1e-12}
    for _ in range(3):
        step_and_compare(gp, op, **kw)
    assert gp.checks() == (0, -1)
    gp.close()


def test_deterministic_checkpoint_resume_bitwise(ctx):
    """A resumed deterministic run continues bit for bit (Philox is keyed by
    the iteration, the state is map, n_h, iteration and history)."""
    p, f = W.cfg_small_d4()
    p = p.with_(n_iter=6, flags=DET)
    ga = B.Problem(ctx, p, f)
    ga.iterate(3)
    blob = ga.export_state()
    ga.iterate(3)
    gb = B.Problem(ctx, p, f)
    gb.import_state(blob)
    gb.iterate(3)
    np.testing.assert_array_equal(ga.map(), gb.map())
    np.testing.assert_array_equal(ga.alloc(), gb.alloc())
    ra, rb = ga.result(), gb.result()
    for key in ("mean", "sdev", "chi2", "I", "V"):
        np.testing.assert_array_equal(ra[key], rb[key], err_msg=key)
    ga.close()
    gb.close()


def _serve(ctx, reqs):
    srv = B.Server(ctx)
    tickets = [srv.submit(pp, ff) for pp, ff in reqs]
    out = [srv.wait(t) for t in tickets]
    srv.close()
    return out


def test_deterministic_served(ctx):
    """Deterministic requests served twice, in different company and order,
    give the same bits; against the plain path (another split of the work)
    they agree to rounding."""
    p4, f4 = W.cfg_small_d4()
    p8, f8 = W.cfg_diag_d8(n_ev=300_000)
    reqs = [(p4.with_(seed=s, n_iter=3, flags=DET), f4) for s in range(3)]
    reqs.append((p8.with_(n_iter=2, flags=DET), f8))
    first = _serve(ctx, reqs)
    again = _serve(ctx, reqs[::-1] + [(p4.with_(seed=9, n_iter=4), f4)])[:len(reqs)][::-1]
    for a, b in zip(first, again):
        for key in ("mean", "sdev", "chi2", "n_evals"):
            assert a[key] == b[key], key
    for (pp, ff), rs in zip(reqs, first):
        gp = B.Problem(ctx, pp, ff)
        gp.iterate(pp.n_iter)
        r = gp.result()
        gp.close()
        assert rs["n_evals"] == r["n_evals"] or r["ties"] > 0
        if r["ties"] == 0:
            assert_close(rs["mean"], r["mean"], RTOL64, what="mean")


def test_flag_rules(ctx):
    p, f = W.cfg_small_d4()
    for bad in (p.with_(flags=4), p.with_(precision="fp32_neumaier", flags=DET)):
        with pytest.raises(B.VegaspError) as e:
            B.Problem(ctx, bad, f)
        assert e.value.status == B.VP_ERR_INVALID_ARG
