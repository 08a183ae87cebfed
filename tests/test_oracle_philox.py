"""Pins of the oracle's Philox4x32-10 (the generator the paper leaves open).

* against rocRAND's independent implementation of the same published
  generator (Salmon et al., SC'11), built here for the host;
* statistical sanity of the 53-bit uniforms built from two words.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "philox_rocrand.cpp")


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", HELPER, "-o", exe], check=True, capture_output=True)

    def run(rows):
        inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return [[int(v) for v in line.split()] for line in out.strip().splitlines()]

    return run


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(123)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]]
    for _ in range(300):
        c = rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)
        c[1] %= 2 ** 30  # the reference's offset encoding
        rows.append([int(v) for v in c])
    # the counters the sampler actually uses: (sample, hypercube, iteration, block)
    for j in range(4):
        for h in (0, 1, 4095, 16777215):
            rows.append([j, h, 7, j % 4, 0, 0])
    ref = rocrand_ref(rows)
    for r, e in zip(rows, ref):
        assert orc.philox(r[:4], r[4:]) == e, r


def test_uniform_53bit_statistics(orc):
    # u = ((w_hi >> 5) 2^26 + (w_lo >> 6)) 2^-53 from the two words of one axis
    n = 20000
    u = np.empty(n)
    for s in range(n):
        w = orc.philox([s, 11, 3, 0], [5, 9])
        u[s] = (((w[0] >> 5) << 26) | (w[2] >> 6)) * 2.0 ** -53
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 0.005
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # neighbouring counters give uncorrelated words
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 4 / np.sqrt(n)


def test_key_and_counter_sensitivity(orc):
    base = orc.philox([1, 2, 3, 4], [5, 6])
    for k in range(4):
        ctr = [1, 2, 3, 4]
        ctr[k] ^= 1
        other = orc.philox(ctr, [5, 6])
        flips = sum(bin(a ^ b).count("1") for a, b in zip(base, other))
        assert 30 < flips < 98  # avalanche: about half of 128 bits change
    other = orc.philox([1, 2, 3, 4], [5, 7])
    assert sum(bin(a ^ b).count("1") for a, b in zip(base, other)) > 30
