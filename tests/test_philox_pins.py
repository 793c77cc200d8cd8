"""Pins for the oracle's counter-based probe generator."""
import os

import numpy as np
from scipy import stats

from oracle.philox import gaussian_probes, philox4x32_10

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_known_answer_vectors():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        w = [int(v, 16) for v in row]
        out = philox4x32_10([np.uint64(v) for v in w[:4]], [np.uint64(v) for v in w[4:6]])
        assert [int(v) for v in out] == w[6:]


def test_probes_are_standard_normal():
    z = gaussian_probes(4, 20001, seed=12345)
    assert z.shape == (4, 20001)
    for row in z:
        assert stats.kstest(row, "norm").pvalue > 1e-3
    # distinct probes and seeds give different streams
    assert not np.allclose(z[0], z[1])
    assert not np.allclose(gaussian_probes(1, 100, 1), gaussian_probes(1, 100, 2))
