"""The precision split (single-precision map and integrand; sums in double
precision or as Neumaier-compensated single-precision pairs) against the
oracle run in the same precision, and its error against the FP64 oracle.

Tolerance: both sides do the same single-precision operations in the same
order; only expf differs (device library vs glibc, each within about one
ulp), so a sample's J f differs by at most a few units of 2^-24 relative.
Sums of such values (S1, S2, the training data, I) then agree to 2e-6
relative; the increment indices and counts are bit-exact; everything after
the sums (allocation, refinement) is double precision and held to 1e-12.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2009_05112_amd import _binding as B
from paper_2009_05112_amd import workloads as W
from tests.parity import step_and_compare

pytestmark = pytest.mark.gpu
RTOL32 = 2e-6
# per-hypercube sums below 1e-12 of the largest are compared absolutely
# (single-precision values near underflow are denormal, with few significant
# bits, so one-ulp differences there are large relative errors; such values
# weigh nothing)
FLOOR32 = 1e-12


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["fp32_acc64", "fp32_neumaier"])
@pytest.mark.parametrize("hist_mode", ["weighted", "literal"])
def test_split_stepwise_d8(ctx, prec, hist_mode):
    p, f = W.cfg_diag_d8(n_ev=1_000_000, precision=prec)
    p = p.with_(hist_mode=hist_mode)
    gp = B.Problem(ctx, p, f)
    op = oracle.Problem(p, f, n_st=gp.n_st)
    for _ in range(4):
        step_and_compare(gp, op, rtol=RTOL32, rtol_hist=RTOL32, exact_counts=(hist_mode == "literal"),
                         floor=FLOOR32)


@pytest.mark.parametrize("prec", ["fp32_acc64", "fp32_neumaier"])
def test_split_stepwise_d4(ctx, prec):
    p, f = W.cfg_small_d4()
    p = p.with_(precision=prec)
    gp = B.Problem(ctx, p, f)
    # the split kernels stage the two innermost map axes in LDS and read the others by buffer loads
    assert gp.map_place == "inner" and gp.hist_axes == 4
    op = oracle.Problem(p, f, n_st=gp.n_st)
    for _ in range(4):
        step_and_compare(gp, op, rtol=RTOL32, rtol_hist=RTOL32, floor=FLOOR32)


@pytest.mark.parametrize("prec", ["fp32_acc64", "fp32_neumaier"])
def test_split_error_vs_fp64_oracle(ctx, prec):
    """Equal stated accuracy: over a 10-iteration D=8 run the split's combined
    estimate lies within 0.1 sigma of the FP64 oracle's and its error
    estimate within 1%."""
    p, f = W.cfg_diag_d8(n_ev=400_000)
    p = p.with_(n_iter=10)
    ro = oracle.Problem(p, f).integrate()
    gp = B.Problem(ctx, p.with_(precision=prec), f)
    gp.iterate(p.n_iter)
    rs = gp.result()
    dev = abs(rs["mean"] - ro["mean"])
    print(f"{prec}: |I_split - I_fp64| = {dev:.3e} = {dev / ro['sdev']:.4f} sigma "
          f"({dev / abs(ro['mean']):.2e} relative); sigma ratio {rs['sdev'] / ro['sdev']:.6f}")
    assert dev <= 0.1 * ro["sdev"]
    assert abs(rs["sdev"] / ro["sdev"] - 1.0) < 0.01


def test_split_larger_map(ctx):
    """N_g = 1200 at D=8: 9600 increments' training data in LDS, the map read
    through buffer loads."""
    p, f = W.cfg_diag_d8(n_ev=500_000, precision="fp32_acc64")
    p = p.with_(n_g=1200)
    gp = B.Problem(ctx, p, f)
    op = oracle.Problem(p, f, n_st=gp.n_st)
    for _ in range(3):
        step_and_compare(gp, op, rtol=RTOL32, rtol_hist=RTOL32, floor=FLOOR32)
