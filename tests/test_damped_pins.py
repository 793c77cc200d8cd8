"""Pins of the convergent Born series oracle (oracle/damped.py; Section 2.2's review of the series with a
dissipative background): quadrature of the complex-wavenumber kernel, continuity at zero dissipation, the
convergence condition eps >= max |chi| stated in Section 2.2 (spectral radius of M below 1 where the Born series
diverges), the converged series against dense LU, and absorbing layers bringing the solution towards the
undissipated one."""
import numpy as np
import pytest
import scipy.integrate as integrate
import scipy.special as sp

from oracle import damped as D
from oracle import lsop_oracle as O
from paper_2005_01372_amd import synth


def _k(freq=10.0, c0=2000.0, eps=4e-4):
    return D.damped_wavenumber(O.wavenumber(freq, c0), eps)


def test_damped_wavenumber_branch():
    k = _k()
    assert k.real > 0 and k.imag > 0
    assert abs(k * k - (O.wavenumber(10.0, 2000.0) ** 2 + 4e-4j)) < 1e-18


def test_damped_self_term_quadrature():
    """K(0,0) equals the integral of (i/4) H0^(1)(k r) over the equal-area disk, complex k (radial quadrature)."""
    h, k = 10.0, _k()
    a = h / np.sqrt(np.pi)
    f = lambda r, part: (0.25j * sp.hankel1(0, k * r) * 2 * np.pi * r).real if part == 0 else \
        (0.25j * sp.hankel1(0, k * r) * 2 * np.pi * r).imag
    re = integrate.quad(lambda r: f(r, 0), 0, a, limit=200, epsabs=1e-15)[0]
    im = integrate.quad(lambda r: f(r, 1), 0, a, limit=200, epsabs=1e-15)[0]
    K = D.damped_kernel(1, 1, h, k)
    assert abs(K[0, 0] - complex(re, im)) <= 1e-10 * abs(K[0, 0])


@pytest.mark.parametrize("p,q", [(1, 0), (2, 3), (7, 5)])
def test_damped_offdiag_quadrature(p, q):
    """K(p,q) equals the 2D quadrature of (i/4) H0^(1)(k |x|) over the disk cell at lag (p,q), complex k."""
    h, k = 10.0, _k(eps=1.5e-3)
    a = h / np.sqrt(np.pi)
    cx, cz = p * h, q * h

    def g(th, r, part):
        v = 0.25j * sp.hankel1(0, k * np.hypot(cx + r * np.cos(th), cz + r * np.sin(th))) * r
        return v.real if part == 0 else v.imag
    re = integrate.dblquad(lambda th, r: g(th, r, 0), 0, a, 0, 2 * np.pi, epsabs=1e-14)[0]
    im = integrate.dblquad(lambda th, r: g(th, r, 1), 0, a, 0, 2 * np.pi, epsabs=1e-14)[0]
    K = D.damped_kernel(p + 1, q + 1, h, k)
    assert abs(K[p, q] - complex(re, im)) <= 1e-9 * abs(K[p, q])


def test_continuous_at_zero_dissipation():
    k0 = O.wavenumber(12.0, 2000.0)
    Kd = D.damped_kernel(9, 7, 10.0, D.damped_wavenumber(k0, 1e-14))
    K = O.cell_kernel(9, 7, 10.0, k0)
    assert np.max(np.abs(Kd - K)) <= 1e-9 * np.max(np.abs(K))


def _medium(n, freq, pert, seed=1):
    rng = np.random.default_rng(seed)
    return 2000.0 * (1.0 + pert * synth.smoothed_field((n, n), 3.0, rng)), freq


@pytest.mark.parametrize("n,freq,pert", [(32, 15.0, 0.5), (24, 10.0, 0.3)])
def test_contraction_for_eps_at_least_max_contrast(n, freq, pert):
    """Section 2.2: with eps >= max |chi| the series converges: rho(M) < 1 (here even ||M||_2 < 1) for
    M = I - gamma A_eps, also on media where the Born series diverges."""
    vel, f = _medium(n, freq, pert)
    P = O.Problem(vel, 10.0, f, 2000.0)
    born_rho = np.abs(np.linalg.eigvals(np.eye(P.n) - P.dense())).max()
    eps = np.abs(P.chi).max()
    Dp = D.DampedProblem(vel, 10.0, f, 2000.0, eps)
    M = np.eye(Dp.n) - (1j * Dp.V.reshape(-1) / eps)[:, None] * Dp.dense()
    assert np.linalg.norm(M, 2) < 1.0
    if n == 32:
        assert born_rho > 1.0      # the plain Born series diverges on this medium


def test_converged_series_equals_dense_solution():
    vel, f = _medium(24, 15.0, 0.5, seed=3)
    eps = 1.2 * np.abs(O.contrast(vel, f, 2000.0)).max()
    Dp = D.DampedProblem(vel, 10.0, f, 2000.0, eps, absorb=4)
    psi0 = Dp.incident([12], [12])[0]
    ref = np.linalg.solve(Dp.dense(), psi0.reshape(-1)).reshape(psi0.shape)
    psi, it, res, st = O.series_solve(Dp, Dp.gamma, psi0, 1e-12, max_iter=5000)
    assert st == O.OK
    assert np.linalg.norm(psi - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.allclose(Dp.apply(psi0[None]), Dp.apply_direct(psi0[None]), rtol=0, atol=1e-13 * np.abs(psi0).max())


def test_absorbing_layers_approach_the_undissipated_solution():
    """The medium padded with background cells that form the absorbing layer: the solution on the original cells
    moves towards the undissipated LS solution (dense LU) as the layer widens."""
    n0, h, f = 24, 10.0, 10.0
    rng = np.random.default_rng(2)
    core = 2000.0 * (1.0 + 0.3 * synth.smoothed_field((n0, n0), 3.0, rng))
    diffs = []
    for pad in (6, 12):
        n = n0 + 2 * pad
        vel = np.full((n, n), 2000.0)
        vel[pad:pad + n0, pad:pad + n0] = core
        P = O.Problem(vel, h, f, 2000.0)
        ref = O.solve_direct(P, P.incident([n // 2], [n // 2]))[0][pad:pad + n0, pad:pad + n0]
        Dp = D.DampedProblem(vel, h, f, 2000.0, 2.0 * np.abs(P.chi).max(), absorb=pad)
        psi = np.linalg.solve(Dp.dense(), Dp.incident([n // 2], [n // 2])[0].reshape(-1)).reshape(n, n)
        diffs.append(np.linalg.norm(psi[pad:pad + n0, pad:pad + n0] - ref) / np.linalg.norm(ref))
    assert diffs[1] < diffs[0] and diffs[1] < 0.1
