"""Pins of the 3D oracle (oracle/lsop3d.py): the ball-integrated kernel against quadrature, the FFT product
against the direct sum, the adjoint identity, and the grid solution against the exact series solution for a
point source and a homogeneous ball (it approaches it as the grid is refined)."""
import numpy as np
import pytest
import scipy.integrate as integrate

from oracle import lsop3d as O3
from oracle import lsop_oracle as O


def test_self_term_quadrature():
    h, k0 = 10.0, O.wavenumber(15.0, 2000.0)
    a = O3.ball_radius(h)
    re = integrate.quad(lambda r: np.cos(k0 * r) * r, 0, a, epsabs=1e-15)[0]     # 4 pi r^2 e^{ikr} / (4 pi r)
    im = integrate.quad(lambda r: np.sin(k0 * r) * r, 0, a, epsabs=1e-15)[0]
    K = O3.cell_kernel3(1, 1, 1, h, k0)
    assert abs(K[0, 0, 0] - complex(re, im)) <= 1e-12 * abs(K[0, 0, 0])


@pytest.mark.parametrize("lag", [(1, 0, 0), (1, 1, 0), (2, 1, 3)])
def test_offdiag_quadrature(lag):
    """K at a lag equals the integral of e^{ik|x - y|} / (4 pi |x - y|) over the ball around the lag's centre
    (spherical coordinates, 3D quadrature)."""
    h, k0 = 10.0, O.wavenumber(25.0, 2000.0)
    a = O3.ball_radius(h)
    c = h * np.array(lag, np.float64)

    def g(ph, th, r, part):
        y = c + r * np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
        d = np.linalg.norm(y)
        v = np.exp(1j * k0 * d) / (4 * np.pi * d) * r * r * np.sin(th)
        return v.real if part == 0 else v.imag
    opts = dict(epsabs=1e-13, epsrel=1e-11)
    re = integrate.tplquad(lambda ph, th, r: g(ph, th, r, 0), 0, a, 0, np.pi, 0, 2 * np.pi, **opts)[0]
    im = integrate.tplquad(lambda ph, th, r: g(ph, th, r, 1), 0, a, 0, np.pi, 0, 2 * np.pi, **opts)[0]
    K = O3.cell_kernel3(*(l + 1 for l in lag), h, k0)
    assert abs(K[lag] - complex(re, im)) <= 1e-9 * abs(K[lag])


def _medium(n, seed=0):
    rng = np.random.default_rng(seed)
    return 2000.0 * (1.0 + 0.3 * rng.uniform(-1, 1, (n, n + 1, n - 1)))


@pytest.mark.parametrize("mode", ["A", "G0V", "AH", "VHG0H"])
def test_fft_equals_direct(mode):
    vel = _medium(7)
    P = O3.Problem3(vel, 10.0, 15.0, 2000.0)
    x = np.random.default_rng(1).standard_normal((2,) + vel.shape) + 0j
    assert np.allclose(P.apply(x, mode), P.apply_direct(x, mode), rtol=0, atol=1e-13 * np.abs(P.apply_direct(x, mode)).max())


def test_adjoint_identity():
    vel = _medium(6, 2)
    P = O3.Problem3(vel, 10.0, 12.0, 2000.0)
    r = np.random.default_rng(3)
    x = r.standard_normal(vel.shape) + 1j * r.standard_normal(vel.shape)
    y = r.standard_normal(vel.shape) + 1j * r.standard_normal(vel.shape)
    for fwd, adj in (("A", "AH"), ("G0V", "VHG0H")):
        lhs = np.vdot(y, P.apply(x, fwd))
        rhs = np.vdot(P.apply(y, adj), x)
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_ball_scattering_closed_form():
    """A ball of radius 60 m and 2600 m/s in a 2000 m/s background, 15 Hz, point source 90 m from its centre on
    its axis: the grid solution (scipy GMRES on the oracle's FFT operator, to 1e-10) matches the exact series
    solution at cells away from the ball surface and the source within 5%, and its scattered part moves towards
    the exact scattered field as h goes from 12 m to 8 m (staircase ball and cell averages)."""
    from scipy.sparse.linalg import LinearOperator, gmres
    R, rs, f, c0, c1 = 60.0, 90.0, 15.0, 2000.0, 2600.0
    k0, k1 = O.wavenumber(f, c0), O.wavenumber(f, c1)
    tot, scat = [], []
    for h in (12.0, 8.0):
        L = 240.0
        n = int(round(L / h))
        ctr = (np.arange(n) + 0.5) * h - L / 2
        X, Y, Z = np.meshgrid(ctr, ctr, ctr, indexing="ij")
        src = (int(np.argmin(np.abs(ctr))), int(np.argmin(np.abs(ctr))), int(np.argmin(np.abs(ctr - rs))))
        sx, sz = ctr[src[0]], ctr[src[2]]
        vel = np.where((X - sx) ** 2 + (Y - sx) ** 2 + Z ** 2 <= R ** 2, c1, c0)   # ball on the source's axis
        P = O3.Problem3(vel, h, f, c0)
        b = P.incident([src])[0].reshape(-1)
        A = LinearOperator((P.n, P.n), dtype=complex, matvec=lambda v: P.apply(v.reshape(vel.shape)).reshape(-1))
        x, info = gmres(A, b, rtol=1e-10, atol=0.0, restart=100, maxiter=50)
        assert info == 0
        pts = np.stack([X.reshape(-1) - sx, Y.reshape(-1) - sx, Z.reshape(-1)], 1)
        rr = np.linalg.norm(pts, axis=1)
        ds = np.linalg.norm(pts - np.array([0.0, 0.0, sz]), axis=1)
        keep = (rr > R + 2 * h) & (ds > 3 * h)
        inc, sc = O3.sphere_scattering(k0, k1, R, sz, pts[keep])
        got = x[keep]
        tot.append(np.linalg.norm(got - inc - sc) / np.linalg.norm(inc + sc))
        scat.append(np.linalg.norm(got - inc - sc) / np.linalg.norm(sc))
    assert max(tot) < 0.05, tot
    assert scat[1] < scat[0], scat
