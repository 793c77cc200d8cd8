"""GPU parity of the 3D operator (the paper's extension to 3D) against the 3D oracle (oracle/lsop3d.py): the
ball-integrated kernel table, the four modes against the direct sums (FP64 <= 1e-12, FP32 <= 1e-5) and the FFT
product at 64^3, incident fields, the series with the randomized preconditioner and GMRES against dense LU
(FP64 <= 1e-10), and the exact solution for a homogeneous ball (within the grid's discretisation error)."""
import os

import numpy as np
import pytest
import torch

from gpu_helpers import announce, dev, host, rel, require_gpu
from oracle import lsop3d as O3
from oracle import lsop_oracle as O
from paper_2005_01372_amd import lsop

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def medium(shape, spread=0.3, seed=0):
    rng = np.random.default_rng(seed)
    return 2000.0 * (1.0 + spread * rng.uniform(-1, 1, shape))


def op3(vel, h, f, dtype=lsop.C128, max_vec=4):
    op = lsop.Operator3D(*vel.shape, dtype, max_vec)
    op.set_problem(torch.as_tensor(vel).cuda(), h, f, 2000.0)
    return op


def rvec(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.mark.parametrize("shape", [(9, 12, 10), (20, 17, 33), (40, 3, 70)])
def test_kernel_table_3d(shape):
    announce(f"3d table {shape}")
    op = op3(medium(shape), 10.0, 15.0)
    ref = O3.cell_kernel3(*shape, 10.0, O.wavenumber(15.0, 2000.0))
    assert np.max(np.abs(host(op.kernel_table()) - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", [(9, 12, 10), (13, 7, 21), (5, 33, 6)])
@pytest.mark.parametrize("dtype,tol", [(lsop.C128, 1e-12), (lsop.C64, 1e-5)])
@pytest.mark.parametrize("mode", ["A", "G0V", "AH", "VHG0H"])
def test_apply_3d_vs_direct(shape, dtype, tol, mode):
    announce(f"3d apply {shape} {dtype} {mode}")
    vel = medium(shape, 0.4, seed=sum(shape))
    P = O3.Problem3(vel, 10.0, 15.0, 2000.0)
    x = rvec((3,) + shape, 5)
    ref = P.apply_direct(x, mode)
    op = op3(vel, 10.0, 15.0, dtype, max_vec=2)      # 3 vectors in chunks of 2
    tdt = torch.complex128 if dtype == lsop.C128 else torch.complex64
    assert rel(host(op.apply(dev(x, tdt), mode)), ref) <= tol


@pytest.mark.parametrize("dtype,tol", [(lsop.C128, 1e-12), (lsop.C64, 1e-5)])
def test_apply_3d_64_cubed_vs_oracle_fft(dtype, tol):
    announce(f"3d apply 64^3 {dtype}")
    vel = medium((64, 64, 64), 0.5, seed=3)
    P = O3.Problem3(vel, 5.0, 25.0, 2000.0)
    P.workers = os.cpu_count()
    x = rvec((2, 64, 64, 64), 7)
    op = op3(vel, 5.0, 25.0, dtype, max_vec=2)
    tdt = torch.complex128 if dtype == lsop.C128 else torch.complex64
    for mode in ("A", "VHG0H"):
        assert rel(host(op.apply(dev(x, tdt), mode)), P.apply(x, mode)) <= tol


def test_incident_and_residual_3d():
    announce("3d incident")
    shape = (16, 12, 20)
    vel = medium(shape, 0.3, seed=4)
    P = O3.Problem3(vel, 10.0, 12.0, 2000.0)
    op = op3(vel, 10.0, 12.0)
    src = [(8, 6, 0), (0, 11, 19), (3, 2, 10)]
    ref = P.incident(src, [1.0, 2 - 1j, 0.5j])
    got = host(op.incident(src, [1.0, 2 - 1j, 0.5j]))
    assert rel(got, ref) <= 1e-14
    psi = rvec((3,) + shape, 1)
    r, nrm = op.residual(dev(psi), dev(ref))
    rr = P.apply(psi) - ref
    assert rel(host(r), rr) <= 1e-12
    np.testing.assert_allclose(nrm.cpu().numpy(), np.sum(np.abs(rr) ** 2, axis=(1, 2, 3)), rtol=1e-12)


def test_series_and_gmres_3d_match_dense_lu():
    """12 x 14 x 13 cells, 20 Hz, +-40% velocity: the randomized preconditioner's series and GMRES both reach the
    dense-LU solution; fixed point independent of H (Section 2.2)."""
    announce("3d series and gmres")
    shape = (12, 14, 13)
    vel = medium(shape, 0.4, seed=6)
    P = O3.Problem3(vel, 10.0, 20.0, 2000.0)
    src = [(6, 7, 0), (2, 3, 12)]
    lu = O3.solve_direct3(P, P.incident(src))
    op = op3(vel, 10.0, 20.0)
    rhs = op.incident(src)
    pc = lsop.Preconditioner(op, lsop.PC_LOWRANK, rank=64, seed=2)
    pc.build()
    psi, res = lsop.series_solve(op, pc, rhs, tol=1e-13, max_iter=200)
    assert all(r.status == lsop.OK for r in res), [r.status_name for r in res]
    assert rel(host(psi), lu) <= 1e-10
    psi, res = lsop.gmres_solve(op, None, rhs, tol=1e-13, restart=60, max_iter=600)
    assert all(r.status == lsop.OK for r in res)
    assert rel(host(psi), lu) <= 1e-10


def test_ball_scattering_3d():
    """A 60 m ball of 2600 m/s in 2000 m/s at 15 Hz, point source 90 m from its centre on its axis, h = 6 m
    (40^3 cells), complex FP32 GMRES to 1e-6: within 5% of the exact series solution away from the ball surface
    and the source (the grid's own discretisation error, as for the oracle's grid solution)."""
    announce("3d ball scattering")
    R, rs, f, c0, c1, h, L = 60.0, 90.0, 15.0, 2000.0, 2600.0, 6.0, 240.0
    n = int(round(L / h))
    ctr = (np.arange(n) + 0.5) * h - L / 2
    X, Y, Z = np.meshgrid(ctr, ctr, ctr, indexing="ij")
    src = (int(np.argmin(np.abs(ctr))), int(np.argmin(np.abs(ctr))), int(np.argmin(np.abs(ctr - rs))))
    sx, sz = ctr[src[0]], ctr[src[2]]
    vel = np.where((X - sx) ** 2 + (Y - sx) ** 2 + Z ** 2 <= R ** 2, c1, c0)
    op = op3(vel, h, f, lsop.C64, 1)
    psi, res = lsop.gmres_solve(op, None, op.incident([src]), tol=1e-6, restart=40, max_iter=400)
    assert res[0].status == lsop.OK
    pts = np.stack([X.reshape(-1) - sx, Y.reshape(-1) - sx, Z.reshape(-1)], 1)
    rr = np.linalg.norm(pts, axis=1)
    ds = np.linalg.norm(pts - np.array([0.0, 0.0, sz]), axis=1)
    keep = (rr > R + 2 * h) & (ds > 3 * h)
    inc, sc = O3.sphere_scattering(O.wavenumber(f, c0), O.wavenumber(f, c1), R, sz, pts[keep])
    got = host(psi)[0].reshape(-1)[keep]
    assert np.linalg.norm(got - inc - sc) / np.linalg.norm(inc + sc) < 0.05


def test_3d_guards():
    announce("3d guards")
    op = op3(medium((8, 8, 8)), 10.0, 10.0)
    with pytest.raises(lsop.LsopError):
        lsop.Preconditioner(op, lsop.PC_HODLR, rank=8, levels=1)
    with pytest.raises(lsop.LsopError):
        lsop.Batch([op])
    with pytest.raises(lsop.LsopError):
        lsop.load_library()
        lsop._check(op.lib.lsop_set_problem(op.handle, lsop._ptr(op._vel), 10.0, 10.0, 2000.0, lsop._stream()))
