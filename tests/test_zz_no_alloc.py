"""vp_map_train_noalloc, the training call that stages its points in the
library's static device workspace instead of allocating: its trained map
against vp_map_train's on the same inputs (Sec. 5.2), over two calls in a
row, the second with fewer points (the workspace keeps the first call's
contents beyond them), and its size limit."""
import numpy as np
import pytest

from paper_2009_05112_amd import _binding as B
from paper_2009_05112_amd import workloads as W
from tests.parity import RTOL64, assert_close

pytestmark = pytest.mark.gpu


def _values(f, x):
    out = np.zeros(len(x))
    for k in range(f.n_terms):
        out += f.amps[k] * np.exp(-f.coefs[k] * ((x - f.centers[k]) ** 2).sum(axis=1))
    return f.scale * out


def test_noalloc_training_equals_allocating_call():
    ctx = B.Context(0)
    f = W.gauss_diag(6, coef=2e3)
    p = W.Params(dim=6, n_ev=100_000, n_g=300, n_iter=4, alpha=0.0, seed=5)
    ref = B.Problem(ctx, p, f)
    gp = B.Problem(ctx, p, f)
    for n, seed in ((60_000, 1), (7_000, 2)):
        x = W.precondition_points(n, f.centers, 2e3, seed=seed)
        fx = _values(f, x)
        print(f"training call: n={n} points, D=6, N_g=300", flush=True)
        ref.train_map(x, fx, 3, 0.7)
        gp.train_map_noalloc(x, fx, 3, 0.7)
        a, b = gp.accum(), ref.accum()
        np.testing.assert_array_equal(a["W"], b["W"])  # counts of the last pass
        for mu in range(p.dim):
            assert_close(a["H"][mu], b["H"][mu], RTOL64, scale=np.abs(b["H"][mu]).sum(), what=f"H[{mu}]")
        assert_close(gp.map(), ref.map(), RTOL64, scale=np.ones((p.dim, p.n_g + 1)), what="map")
    # beyond the workspace: a clear error, nothing run
    m0 = gp.map()
    n_big = (32 << 20) // (8 * (p.dim + 1)) + 1
    xb = np.full((n_big, p.dim), 0.5)
    with pytest.raises(B.VegaspError) as e:
        gp.train_map_noalloc(xb, np.ones(n_big), 1, 0.5)
    assert e.value.status == B.VP_ERR_INVALID_ARG and "workspace" in str(e.value)
    np.testing.assert_array_equal(gp.map(), m0)
    gp.close()
    ref.close()
    ctx.close()
