"""GPU tests of the frequency sweep of Section 3.1 (lowest frequency first, at most 30 series iterations, rebuild
with a larger rank and restart from psi0 on failure, a larger rank for the next frequency after more than 10
iterations).  Every frequency's fields are compared with the oracle's dense-LU solution of that frequency's
problem times the source spectrum (a Ricker wavelet, written out here from its definition): FP64 <= 1e-10
(series to 1e-12), complex FP32 <= 1e-4.  The rank schedule is checked against the rule itself, from the
iteration counts and rebuilds the sweep reports."""
import numpy as np
import pytest
import torch

from gpu_helpers import announce, host, rel, require_gpu
from oracle import lsop_oracle as O
from paper_2005_01372_amd import lsop, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def ricker(f, fc):
    return 2.0 / np.sqrt(np.pi) * f ** 2 / fc ** 3 * np.exp(-(f / fc) ** 2) * np.exp(-2j * np.pi * f / fc)


def check_schedule(info, start, step, cap, above=10):
    rank = start
    for k, x in enumerate(info):
        assert x["rank"] == min(cap, rank + x["rebuilds"] * step), (k, x, rank)
        rank = x["rank"] + (step if x["iters_max"] > above else 0)
        rank = min(cap, rank)


def check_fields(psi, info, w, freqs, fc, tol):
    for k, f in enumerate(freqs):
        prob = O.Problem(w.vel, w.h, f, w.c0)
        ref = O.solve_direct(prob, ricker(f, fc) * prob.incident(w.src_i, w.src_j))
        assert info[k]["status"] == lsop.OK, info[k]
        assert rel(host(psi[k]), ref) <= tol, (f, rel(host(psi[k]), ref))


def test_sweep_simple_preconditioner_fp64():
    announce("sweep simple fp64")
    w = synth.model_smooth_inclusion(n=48, h=10.0 * 64 / 48, freq=10.0, seed=1)
    w.src_i, w.src_j = np.array([24, 8]), np.array([0, 0])
    freqs = [1.0, 2.0, 4.0, 6.0, 8.0, 10.0, 12.0]
    op = lsop.Operator(48, 48, lsop.C128, 4)
    psi, info = lsop.sweep(op, w.vel, w.h, w.c0, freqs, w.src_i, w.src_j, kind=lsop.PC_LOWRANK, rank=4,
                           rank_step=12, tol=1e-12, max_iter=30, seed=3, ricker_fc=10.0)
    announce(f"ranks {[x['rank'] for x in info]}, iterations {[x['iters_max'] for x in info]}, "
             f"rebuilds {[x['rebuilds'] for x in info]}")
    check_schedule(info, 4, 12, 256)
    check_fields(psi, info, w, freqs, 10.0, 1e-10)
    assert info[-1]["rank"] > 4                         # the rank grew with frequency


def test_sweep_rebuilds_a_diverging_preconditioner():
    """Rank 1 at 12 Hz diverges: the sweep rebuilds with larger ranks until the series converges."""
    announce("sweep rebuild")
    w = synth.model_smooth_inclusion(n=48, h=10.0 * 64 / 48, freq=12.0, seed=1)
    op = lsop.Operator(48, 48, lsop.C128, 4)
    psi, info = lsop.sweep(op, w.vel, w.h, w.c0, [12.0], w.src_i, w.src_j, kind=lsop.PC_LOWRANK, rank=1,
                           rank_step=16, tol=1e-12, max_iter=30, seed=5, ricker_fc=8.0)
    assert info[0]["rebuilds"] >= 1 and info[0]["status"] == lsop.OK
    check_schedule(info, 1, 16, 256)
    check_fields(psi, info, w, [12.0], 8.0, 1e-10)


def test_sweep_hodlr_fp32():
    announce("sweep hodlr fp32")
    w = synth.model_layered_salt(n=64, h=10.0, freq=15.0, seed=2, nsrc=3)
    freqs = [3.0, 6.0, 9.0, 12.0, 15.0]
    op = lsop.Operator(64, 64, lsop.C64, 4)
    psi, info = lsop.sweep(op, w.vel, w.h, w.c0, freqs, w.src_i, w.src_j, kind=lsop.PC_HODLR, rank=4, levels=3,
                           power_iters=1, rank_step=4, tol=1e-6, max_iter=30, seed=7, ricker_fc=10.0)
    announce(f"ranks {[x['rank'] for x in info]}, iterations {[x['iters_max'] for x in info]}")
    check_schedule(info, 4, 4, 256)
    check_fields(psi, info, w, freqs, 10.0, 1e-4)


def test_sweep_rejects_bad_arguments():
    announce("sweep invalid")
    w = synth.model_smooth_inclusion(n=32, h=20.0, freq=10.0, seed=1)
    op = lsop.Operator(32, 32, lsop.C128, 2)
    for kw in (dict(freqs=[5.0, 4.0]), dict(freqs=[0.0, 4.0]), dict(kind=lsop.PC_SCALAR), dict(rank=0)):
        args = dict(freqs=[2.0, 4.0], kind=lsop.PC_LOWRANK, rank=4)
        args.update(kw)
        with pytest.raises(lsop.LsopError) as e:
            lsop.sweep(op, w.vel, w.h, w.c0, args.pop("freqs"), w.src_i, w.src_j, **args)
        assert e.value.status == lsop.EINVAL
