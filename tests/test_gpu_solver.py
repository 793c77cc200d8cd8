"""GPU parity of the randomized preconditioner (Alg. 2, eq. 12) and the series (eqs. 10-14).

Solutions are compared with the oracle's dense-LU solution (eq. 6) as a
relative L2 error over all cells, per source: complex double <= 1e-10 (solved
to a residual of 1e-13, since the error is at most ||A^-1|| times the
residual); FP32 + FP64 refinement <= 1e-10; plain FP32 series to 1e-6 <= 1e-4.
The preconditioner itself is compared through H x (U and W are unique only up
to a unitary factor).
"""
import numpy as np
import pytest
import torch

from gpu_helpers import announce, dev, host, make_op, rel, require_gpu
from oracle import lsop_oracle as O
from oracle.philox import gaussian_probes as philox_probes
from paper_2005_01372_amd import lsop, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def cfg1(n=64):
    return synth.model_smooth_inclusion(n=n, h=10.0 * 64 / n, freq=10.0, seed=1)


@pytest.mark.parametrize("dtype,q,tol", [(lsop.C128, 0, 1e-11), (lsop.C128, 1, 1e-11), (lsop.C64, 0, 2e-5)])
def test_precond_apply_matches_oracle(dtype, q, tol):
    announce(f"precond apply dtype={dtype} q={q}")
    w = cfg1(48)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    r = 24
    om = synth.gaussian_probes(prob.n, r, 5)
    H = O.LowRankPreconditioner.build(prob, om.reshape(r, 48, 48), q=q)
    op = make_op(w, dtype, 8)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=r, power_iters=q)
    pc.build(torch.as_tensor(om).cuda())
    assert pc.info()[0] == r
    x = synth.random_vectors((5, 48, 48), 9)
    tdt = torch.complex128 if dtype == lsop.C128 else torch.complex64
    assert rel(host(pc.apply(dev(x, tdt))), H.apply(x)) <= tol


def test_precond_fp32_odd_cell_count_matches_oracle():
    """45 x 45 = 2025 cells: the complex-FP32 products cannot take their 16-byte operand loads (odd row
    length), so this covers their element-wise path; rank 72 spans two orthonormalisation blocks."""
    announce("precond apply fp32 odd n")
    w = cfg1(45)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    r = 72
    om = synth.gaussian_probes(prob.n, r, 11)
    H = O.LowRankPreconditioner.build(prob, om.reshape(r, 45, 45))
    op = make_op(w, lsop.C64, 4)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=r)
    pc.build(torch.as_tensor(om).cuda())
    assert pc.info()[0] == r
    x = synth.random_vectors((3, 45, 45), 2)
    assert rel(host(pc.apply(dev(x, torch.complex64))), H.apply(x)) <= 2e-5


def test_precond_fp32_many_vectors_matches_oracle():
    """Complex FP32 at rank 96 applied to 40 vectors: the build's first 64-column block and the apply's U Z(.)
    take the tile-form update (more than 32 vectors), the projection of the second block and W^H x the inner
    product's 64-wide vector tile, both in the 3M form (three real products per complex one)."""
    announce("precond apply fp32 rank 96, 40 vectors")
    w = cfg1(48)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    r = 96
    om = synth.gaussian_probes(prob.n, r, 13)
    H = O.LowRankPreconditioner.build(prob, om.reshape(r, 48, 48))
    op = make_op(w, lsop.C64, 8)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=r)
    pc.build(torch.as_tensor(om).cuda())
    assert pc.info()[0] == r
    x = synth.random_vectors((40, 48, 48), 6)
    assert rel(host(pc.apply(dev(x, torch.complex64))), H.apply(x)) <= 2e-5


@pytest.mark.parametrize("dtype", [lsop.C64, lsop.C128])
def test_profiler_counts_gemm_flops_of_each_form(dtype):
    """The library's profiler, whose counts the bench's roofline divides by kernel time, counts 6 real flops per
    complex multiply-add for the complex-FP32 GEMMs (Gauss's 3M form: three real products per complex one) and 8
    for complex FP64 (real and imaginary chains): W^H x and U (Z .) of a rank-96 preconditioner on 40 vectors."""
    announce(f"profiler gemm flops dtype={dtype}")
    w = cfg1(48)
    r, nv, n = 96, 40, 48 * 48
    om = synth.gaussian_probes(n, r, 13)
    op = make_op(w, dtype, 8)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=r)
    pc.build(torch.as_tensor(om).cuda())
    tdt = torch.complex64 if dtype == lsop.C64 else torch.complex128
    x = dev(synth.random_vectors((nv, 48, 48), 6), tdt)
    torch.cuda.synchronize()
    lsop.profile_reset()
    lsop.profile_enable(True)
    try:
        pc.apply(x)
        torch.cuda.synchronize()
        ks = lsop.profile_read(by_kernel=True)
    finally:
        lsop.profile_enable(False)
    per = (6.0 if dtype == lsop.C64 else 8.0) * r * nv * n
    t = "float" if dtype == lsop.C64 else "double"
    ahb = ks[f"k_gemm_ah_b_mfma<{t}>"]
    assert ahb["launches"] == 1 and ahb["flops"] == per, ahb
    upd = "k_gemm_update_tile<double>" if dtype == lsop.C64 else "k_gemm_update_mfma<double, double, 4, 4, 3>"
    assert ks[upd]["launches"] == 1 and ks[upd]["flops"] == per, (upd, sorted(ks))


def test_precond_rank_above_128_matches_oracle():
    """Z = (I - W^H U)^{-1} of more than 128 probes takes the pivoted Gauss-Jordan in global memory, whose
    thread layout (one column per thread, fewer threads than 2 * rank) differs from the small-block kernel."""
    announce("precond apply rank 160")
    w = cfg1(48)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    r = 160
    om = synth.gaussian_probes(prob.n, r, 7)
    H = O.LowRankPreconditioner.build(prob, om.reshape(r, 48, 48))
    op = make_op(w, lsop.C128, 4)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=r)
    pc.build(torch.as_tensor(om).cuda())
    assert pc.info()[0] == r
    x = synth.random_vectors((3, 48, 48), 4)
    assert rel(host(pc.apply(dev(x))), H.apply(x)) <= 1e-10


def test_device_philox_probes_match_oracle():
    """A preconditioner drawn on the device (Philox4x32-10 + Box-Muller) equals one built from the oracle's draw."""
    announce("philox")
    w = cfg1(40)
    op = make_op(w, lsop.C128, 8)
    seed = 0x1234567890ABCDEF
    pa = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=16, seed=seed)
    pa.build(None)
    pb = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=16)
    pb.build(torch.as_tensor(philox_probes(16, 40 * 40, seed)).cuda())
    x = synth.random_vectors((2, 40, 40), 1)
    assert rel(host(pa.apply(dev(x))), host(pb.apply(dev(x)))) <= 1e-12


def test_series_fp64_matches_lu_and_iteration_count():
    """Configuration 1 (64^2, 10 Hz, smooth +-10 % plus a 3000 m/s disk; rank 64, q = 0) to residual 1e-13."""
    announce("series fp64 cfg1")
    w = cfg1(64)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)
    ref = O.solve_direct(prob, psi0)
    om = synth.gaussian_probes(prob.n, 64, 11)
    Ho = O.LowRankPreconditioner.build(prob, om.reshape(64, 64, 64))
    _, it_o, _, st_o = O.series_solve(prob, Ho.apply, psi0[0], 1e-13, 60)
    op = make_op(w, lsop.C128, 8)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=64)
    pc.build(torch.as_tensor(om).cuda())
    rhs = op.incident(w.src_i, w.src_j)
    assert rel(host(rhs), psi0) <= 1e-14
    psi, info = lsop.series_solve(op, pc, rhs, tol=1e-13, max_iter=60)
    assert info[0].status == lsop.OK and st_o == O.OK
    assert abs(info[0].iters - it_o) <= 1
    assert rel(host(psi), ref) <= 1e-10
    # residual reported = residual recomputed by the oracle
    assert abs(info[0].rel_residual - O.relative_residual(prob, host(psi)[0], psi0[0])) <= 1e-15


def test_born_series_weak_contrast():
    announce("born")
    w = synth.weak_contrast(n=48)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)
    op = make_op(w, lsop.C128, 4)
    psi, info = lsop.series_solve(op, None, op.incident(w.src_i, w.src_j), tol=1e-13, max_iter=200)
    assert info[0].status == lsop.OK
    assert rel(host(psi), O.solve_direct(prob, psi0)) <= 1e-10
    # a fixed number of Born steps equals the oracle's Born iterate
    psi7, info7 = lsop.series_solve(op, None, op.incident(w.src_i, w.src_j), tol=1e-300, max_iter=7)
    assert info7[0].status == lsop.NOT_CONVERGED and info7[0].iters == 7
    assert rel(host(psi7)[0], O.born(prob, psi0[0], 7)) <= 1e-13


def test_zero_contrast_gives_identity():
    announce("zero contrast")
    n = 40
    w = synth.Workload("zero", np.full((n, n), 2000.0), 10.0, 10.0, 2000.0, np.array([5, 30]), np.array([0, 7]))
    op = make_op(w, lsop.C128, 4)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=8, seed=3)
    pc.build(None)
    assert pc.info()[0] == 0  # every column dropped: H = I
    rhs = op.incident(w.src_i, w.src_j)
    psi, info = lsop.series_solve(op, pc, rhs, tol=1e-12)
    assert all(i.iters == 0 and i.status == lsop.OK for i in info)
    assert torch.equal(psi, rhs)
    assert torch.isfinite(torch.view_as_real(psi)).all()


def test_full_rank_probe_block_solves_in_zero_iterations():
    """Inclusion-only model: chi is non-zero on m disk cells, so l >= m probes give H = A^-1."""
    announce("full rank")
    n = 32
    w = synth.model_smooth_inclusion(n=n, h=20.0, freq=10.0, seed=1, with_background=False)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    m = int(np.count_nonzero(prob.chi))
    op = make_op(w, lsop.C128, 4)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=m + 8, seed=9)
    pc.build(None)
    assert pc.info()[0] == m
    psi, info = lsop.series_solve(op, pc, op.incident(w.src_i, w.src_j), tol=1e-11)
    assert info[0].iters == 0 and info[0].status == lsop.OK
    assert rel(host(psi), O.solve_direct(prob, prob.incident(w.src_i, w.src_j))) <= 1e-10


def test_reciprocity_on_gpu():
    announce("reciprocity")
    w = synth.model_layered_salt(n=48, h=10.0, freq=8.0, seed=5, nsrc=2)
    si, sj = np.array([3, 40]), np.array([0, 21])
    op = make_op(w, lsop.C128, 4)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=96, seed=1)
    pc.build(None)
    psi, info = lsop.series_solve(op, pc, op.incident(si, sj), tol=1e-13, max_iter=200)
    assert all(i.status == lsop.OK for i in info)
    p = host(psi)
    assert abs(p[0][si[1], sj[1]] - p[1][si[0], sj[0]]) <= 1e-10 * abs(p[0][si[1], sj[1]])


def test_mixed_precision_refinement_matches_fp64():
    """FP32 inner series with FP64 residual refinement reaches the FP64 solution (1e-10)."""
    announce("mixed refinement")
    w = cfg1(64)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    si, sj = np.array([32, 5, 60]), np.array([32, 0, 10])
    ref = O.solve_direct(prob, prob.incident(si, sj))
    op = make_op(w, lsop.MIXED, 8)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=64, seed=7)
    pc.build(None)
    psi, info = lsop.series_solve(op, pc, op.incident(si, sj), tol=1e-12, max_iter=30, inner_tol=1e-5)
    assert all(i.status == lsop.OK for i in info), [i.status_name for i in info]
    assert all(i.refine_steps >= 2 for i in info)
    assert rel(host(psi), ref) <= 1e-10


def test_fp32_series():
    announce("fp32 series")
    w = cfg1(64)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    ref = O.solve_direct(prob, prob.incident(w.src_i, w.src_j))
    op = make_op(w, lsop.C64, 8)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=64, seed=7)
    pc.build(None)
    psi, info = lsop.series_solve(op, pc, op.incident(w.src_i, w.src_j), tol=1e-6)
    assert info[0].status == lsop.OK and info[0].rel_residual <= 1e-6
    assert rel(host(psi), ref) <= 1e-4


def test_fp32_series_many_sources_low_rank():
    """Complex-FP32 series with the low-rank preconditioner on 40 sources: the update psi -= U Z W^H r covers
    more than 32 vectors (the 64 x 64 tile form of the update GEMM), reads the residual through the active-set
    index list and subtracts it as its second addend, and the set shrinks as sources converge at different
    iterations.  Every solution matches dense LU to 1e-4 (FP32 series to a residual of 1e-6)."""
    announce("fp32 series, 40 sources, low rank")
    w = synth.model_smooth_inclusion(n=48, h=13.0, freq=10.0, seed=2)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    rng = np.random.default_rng(11)
    si, sj = rng.integers(0, 48, 40), rng.integers(0, 48, 40)
    amp = rng.uniform(0.5, 2.0, 40) * np.exp(2j * np.pi * rng.uniform(size=40))
    ref = O.solve_direct(prob, prob.incident(si, sj, amp))
    op = make_op(w, lsop.C64, 40)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=32, seed=4)
    pc.build(None)
    psi, info = lsop.series_solve(op, pc, op.incident(si, sj, amp), tol=1e-6, max_iter=80)
    assert all(i.status == lsop.OK for i in info)
    iters = sorted({i.iters for i in info})
    announce(f"iteration counts {iters}")
    assert len(iters) > 1
    out = host(psi)
    for k in range(len(si)):
        assert rel(out[k], ref[k]) <= 1e-4


def test_many_sources_converge_independently():
    """Sources converge at different iterations; each stops on its own and matches the LU solution."""
    announce("many sources")
    w = synth.model_smooth_inclusion(n=48, h=13.0, freq=10.0, seed=2)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    si = np.array([2, 10, 24, 33, 40, 47, 20])
    sj = np.array([0, 5, 24, 40, 2, 47, 30])
    amp = np.array([1, 1j, -2, 0.5, 3 - 1j, 1, 1e-3])
    ref = O.solve_direct(prob, prob.incident(si, sj, amp))
    op = make_op(w, lsop.C128, 3)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=32, seed=4)
    pc.build(None)
    psi, info = lsop.series_solve(op, pc, op.incident(si, sj, amp), tol=1e-13, max_iter=80)
    assert all(i.status == lsop.OK for i in info)
    for k in range(len(si)):
        assert rel(host(psi)[k], ref[k]) <= 1e-10


def test_failure_statuses():
    announce("failure statuses")
    # strong contrast, Born: diverges
    w = synth.model_layered_salt(n=64, h=10.0, freq=15.0, seed=2, nsrc=2)
    op = make_op(w, lsop.C128, 4)
    psi, info = lsop.series_solve(op, None, op.incident(w.src_i, w.src_j), tol=1e-10, max_iter=30)
    assert all(i.status == lsop.DIVERGED for i in info)
    # a tiny iteration cap: not converged, iterate and residual still reported
    w1 = cfg1(32)
    op1 = make_op(w1, lsop.C128, 4)
    psi, info = lsop.series_solve(op1, None, op1.incident(w1.src_i, w1.src_j), tol=1e-14, max_iter=1)
    assert info[0].status in (lsop.NOT_CONVERGED, lsop.DIVERGED) and np.isfinite(info[0].rel_residual)
    with pytest.raises(lsop.LsopError):
        lsop.series_solve(op1, None, op1.incident(w1.src_i, w1.src_j), tol=-1.0)


def test_warm_start_reaches_same_fixed_point():
    """Any initial guess converges to the same psi (eqs. 7-9)."""
    announce("warm start")
    w = cfg1(40)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    ref = O.solve_direct(prob, prob.incident(w.src_i, w.src_j))
    op = make_op(w, lsop.C128, 4)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=40, seed=2)
    pc.build(None)
    guess = dev(synth.random_vectors((1, 40, 40), 3))
    psi, info = lsop.series_solve(op, pc, op.incident(w.src_i, w.src_j), psi=guess, init="user", tol=1e-13,
                                  max_iter=80)
    assert info[0].status == lsop.OK
    assert rel(host(psi), ref) <= 1e-10


@pytest.mark.parametrize("init", ["h_rhs", "zero"])
def test_series_output_buffer_contents_are_ignored(init):
    """psi is an output for these starts: NaN left in it by earlier use must not leak into the result."""
    announce(f"garbage psi init={init}")
    w = synth.weak_contrast(32)
    op = make_op(w, lsop.C128, 4)
    rhs = op.incident(w.src_i, w.src_j)
    psi = torch.full_like(rhs, float("nan"))
    psi, res = lsop.series_solve(op, None, rhs, psi=psi, tol=1e-12, max_iter=60, init=init)
    assert res[0].status == lsop.OK
    assert not torch.isnan(psi).any()
