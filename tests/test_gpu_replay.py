"""Deterministic replay: the same seed gives the same bits.

Two HODLR builds from the same Philox seed (device-generated probes) and the series solves run with them give
bitwise-identical H x and solutions, with equal iteration counts and statuses, in complex FP64 and complex FP32:
every reduction on the path from the probes to the iterates has a fixed order (split-K partials are summed in
launch order, no atomics).  The residual norms' atomic sums decide convergence only, and the counts match.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import announce, dev, host, make_op, require_gpu
from paper_2005_01372_amd import lsop, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("dtype,tol", [(lsop.C128, 1e-12), (lsop.C64, 1e-5)])
def test_same_seed_replays_bitwise(dtype, tol):
    announce(f"replay dtype={dtype}")
    w = synth.model_layered_salt(n=64, h=10.0, freq=15.0, seed=2, nsrc=4)
    tdt = torch.complex128 if dtype == lsop.C128 else torch.complex64
    x = synth.random_vectors((3, 64, 64), 9)
    runs = []
    for _ in range(2):
        op = make_op(w, dtype, 4)
        pc = lsop.Preconditioner(op, lsop.PC_HODLR, rank=20, levels=3, power_iters=1, seed=11)
        pc.build(None)
        hx = host(pc.apply(dev(x, tdt)))
        psi, info = lsop.series_solve(op, pc, op.incident(w.src_i, w.src_j), tol=tol, max_iter=60)
        runs.append((hx, host(psi), [(i.iters, i.status) for i in info]))
        del pc, op
    assert all(st == lsop.OK for _, st in runs[0][2])
    assert runs[0][2] == runs[1][2]
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
