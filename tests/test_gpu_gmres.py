"""GPU parity of restarted GMRES (Section 3.2.3's comparison method), right-preconditioned by the library's H.

Unpreconditioned GMRES(m) is compared with scipy's GMRES(m) on the oracle's FFT operator (the same Krylov
spaces in exact arithmetic): iteration counts within 1 and solutions within 1e-10 (FP64, solved to a relative
residual of 1e-13).  Preconditioned runs are compared with the oracle's dense-LU solution (1e-10, FP64);
GMRES converges where the series cannot (rho(I - H A) >= 1), and its solution equals the series' fixed point
(Section 2.2: the fixed point does not depend on H).
"""
import numpy as np
import pytest
import torch
from scipy.sparse.linalg import LinearOperator, gmres

from gpu_helpers import announce, dev, golden_layered_salt, host, make_op, rel, require_gpu
from oracle import lsop_oracle as O
from paper_2005_01372_amd import lsop, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def scipy_gmres(prob, b, restart, tol):
    shp = (prob.nx, prob.nz)
    A = LinearOperator((prob.n, prob.n), dtype=np.complex128,
                       matvec=lambda v: prob.apply(v.reshape(shp), "A").reshape(-1))
    its = [0]

    def cb(_):
        its[0] += 1
    x, info = gmres(A, b.reshape(-1), rtol=tol, atol=0.0, restart=restart, maxiter=200, callback=cb,
                    callback_type="pr_norm")
    assert info == 0
    return x.reshape(shp), its[0]


@pytest.mark.parametrize("n,restart,model", [(48, 20, "inclusion"), (64, 10, "weak"), (40, 5, "inclusion")])
def test_unpreconditioned_gmres_matches_scipy(n, restart, model):
    announce(f"gmres vs scipy n={n} restart={restart} {model}")
    w = synth.model_smooth_inclusion(n=n, h=10.0 * 64 / n, freq=10.0, seed=1) if model == "inclusion" \
        else synth.weak_contrast(n=n, freq=12.0)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)
    ref, its = scipy_gmres(prob, psi0[0], restart, 1e-12)
    op = make_op(w, lsop.C128, 4)
    psi, res = lsop.gmres_solve(op, None, op.incident(w.src_i, w.src_j), tol=1e-12, restart=restart, max_iter=2000)
    assert res[0].status == lsop.OK and res[0].rel_residual <= 1e-12
    assert abs(res[0].iters - its) <= 2, (res[0].iters, its)
    assert rel(host(psi)[0], ref) <= 1e-10


@pytest.mark.parametrize("kind", ["lowrank", "hodlr", "scalar"])
def test_preconditioned_gmres_matches_dense_lu(kind):
    announce(f"preconditioned gmres {kind}")
    w = synth.model_layered_salt(n=64, h=10.0, freq=15.0, seed=2, nsrc=5)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    lu = O.solve_direct(prob, prob.incident(w.src_i, w.src_j))
    op = make_op(w, lsop.C128, 8)
    if kind == "lowrank":
        pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=24, seed=3)
    elif kind == "hodlr":
        pc = lsop.Preconditioner(op, lsop.PC_HODLR, rank=16, levels=3, power_iters=1, seed=3)
    else:
        pc = lsop.Preconditioner(op, lsop.PC_SCALAR, alpha=0.5)
    pc.build()
    # GMRES(30) stagnates on this medium whatever H (scipy on the oracle's operator too: 1e-4 unpreconditioned,
    # 2e-7 with the rank-24 H after 3000 iterations); a 200-vector cycle converges in one cycle
    psi, res = lsop.gmres_solve(op, pc, op.incident(w.src_i, w.src_j), tol=1e-13, restart=200, max_iter=1000,
                                init="h_rhs" if kind != "scalar" else "zero")
    assert all(r.status == lsop.OK for r in res), [(r.status_name, r.rel_residual) for r in res]
    for v in range(5):
        assert rel(host(psi)[v], lu[v]) <= 1e-10


def test_gmres_converges_where_the_series_diverges_fp64_and_mixed():
    """256^2 layered + salt, 15 Hz, 32 top-row sources.  With a HODLR H of rank 40 (5 levels, q = 1) the series
    diverges (rho(I - H A) > 1); GMRES with the same H reaches 1e-10 in FP64, and in complex FP32 with FP64
    refinement.  Both equal the fixed point of the series run with the stronger rank-80 H (Section 2.2: the
    fixed point does not depend on H) within 1e-8, and the oracle's own solution of this workload (its
    matrix-free HODLR series to 1e-13, stored at 512 cells of 4 sources) within 1e-8 at those cells.  (The simple rank-40 + 10 H of this workload's
    configuration is too weak for GMRES(200) as well: 3000 iterations do not reach 1e-10.)"""
    announce("gmres at 256^2 with HODLR rank 40")
    w = synth.model_layered_salt(n=256, h=10.0, freq=15.0, seed=2, nsrc=32)
    out = {}
    for dt in (lsop.C128, lsop.MIXED):
        op = make_op(w, dt, 32)
        pc = lsop.Preconditioner(op, lsop.PC_HODLR, rank=40, levels=5, power_iters=1, seed=4)
        pc.build()
        rhs = op.incident(w.src_i, w.src_j)
        _, rs = lsop.series_solve(op, pc, rhs, tol=1e-10, max_iter=30)
        assert all(r.status != lsop.OK for r in rs)
        psi, res = lsop.gmres_solve(op, pc, rhs, tol=1e-10, restart=50, max_iter=500, init="h_rhs")
        announce(f"dtype {dt}: iterations {min(r.iters for r in res)}..{max(r.iters for r in res)}")
        assert all(r.status == lsop.OK and r.rel_residual <= 1e-10 for r in res), dt
        out[dt] = host(psi)
        del pc, op
    op = make_op(w, lsop.C128, 32)
    pc = lsop.Preconditioner(op, lsop.PC_HODLR, rank=80, levels=5, power_iters=1, seed=4)
    pc.build()
    psi_s, rs = lsop.series_solve(op, pc, op.incident(w.src_i, w.src_j), tol=1e-10, max_iter=30)
    assert all(r.status == lsop.OK for r in rs)
    ref = host(psi_s)
    assert rel(out[lsop.C128], ref) <= 1e-8
    assert rel(out[lsop.MIXED], ref) <= 1e-8
    _, cells = golden_layered_salt()
    for dt in (lsop.C128, lsop.MIXED):
        for s, vals in cells.items():
            got = np.array([out[dt][s, i, j] for i, j, _ in vals])
            want = np.array([v for *_, v in vals])
            assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-8, (dt, s)


def test_gmres_fp32_and_ragged_active_set():
    """Complex FP32 with sources of very different difficulty (the zero right-hand side converges at once and
    leaves the active set; the others run cycles of different length), against dense LU within 1e-4."""
    announce("gmres fp32 ragged")
    w = synth.model_smooth_inclusion(n=48, h=10.0 * 64 / 48, freq=10.0, seed=1)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    si, sj = np.array([24, 3, 40]), np.array([24, 0, 47])
    psi0 = prob.incident(si, sj)
    psi0[1] = 0.0
    lu = O.solve_direct(prob, psi0)
    op = make_op(w, lsop.C64, 4)
    psi, res = lsop.gmres_solve(op, None, dev(psi0, torch.complex64), tol=1e-6, restart=7, max_iter=500)
    assert all(r.status == lsop.OK for r in res)
    assert res[1].iters == 0
    got = host(psi)
    assert np.all(got[1] == 0)
    for v in (0, 2):
        assert rel(got[v], lu[v]) <= 1e-4
