"""Pins for the FP64 oracle against facts the paper and the mathematics fix.

None of these tests retypes an oracle formula: each compares the oracle with
an independent route (quadrature, a printed table, mpmath, dense LAPACK, an
identity or a closed form) chosen so that a dropped term, a wrong sign or a
transposed operand in the oracle fails at least one of them.
"""
import os

import numpy as np
import pytest
from scipy import integrate
from scipy import special as sp

from oracle import lsop_oracle as O
from oracle.inclusion import inclusion_field
from paper_2005_01372_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


# ---------------------------------------------------------------- kernel table
def test_bessel_printed_table():
    """FP64 Bessel values used by the kernel table match the printed A&S Table 9.1 values."""
    fn = {"J0": lambda x: sp.jv(0, x), "J1": lambda x: sp.jv(1, x),
          "Y0": lambda x: sp.yv(0, x), "Y1": lambda x: sp.yv(1, x)}
    with open(os.path.join(GOLDEN, "bessel_unit_argument.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    for name, x, v in rows:
        assert abs(fn[name](float(x)) - float(v)) <= 1e-15 * max(1.0, abs(float(v)))


def test_hankel_against_mpmath():
    """H0^(1), H1^(1), J1 in the table agree with mpmath's arbitrary-precision values."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    for x in [0.05, 0.1, 0.3, 1.0, 3.7, 12.0, 40.0, 155.5, 700.0]:
        for nu in (0, 1):
            ref = complex(mp.hankel1(nu, x))
            got = sp.hankel1(nu, x)
            assert abs(got - ref) <= 1e-13 * abs(ref), (nu, x)


@pytest.mark.parametrize("h,freq", [(10.0, 10.0), (5.0, 25.0), (15.0, 20.0)])
def test_self_term_quadrature(h, freq):
    """K(0,0) equals the integral of (i/4) H0^(1)(k0 r) over the equal-area disk (quadrature)."""
    k0 = O.wavenumber(freq, 2000.0)
    a = h / np.sqrt(np.pi)
    re = integrate.quad(lambda r: -0.25 * sp.y0(k0 * r) * 2 * np.pi * r, 0, a, limit=200, epsabs=1e-14)[0]
    im = integrate.quad(lambda r: 0.25 * sp.j0(k0 * r) * 2 * np.pi * r, 0, a, limit=200, epsabs=1e-14)[0]
    K = O.cell_kernel(2, 2, h, k0)
    assert abs(K[0, 0] - (re + 1j * im)) <= 1e-12 * abs(K[0, 0])


@pytest.mark.parametrize("p,q", [(1, 0), (1, 1), (3, 2)])
def test_offdiag_quadrature(p, q):
    """K(p,q) equals the 2D quadrature of (i/4) H0^(1) over the disk cell at lag (p,q)."""
    h, k0 = 10.0, O.wavenumber(12.0, 2000.0)
    a = h / np.sqrt(np.pi)
    rho = h * np.hypot(p, q)

    def g(th, r, part):
        d = k0 * np.hypot(rho - r * np.cos(th), r * np.sin(th))
        return (-0.25 * sp.y0(d) if part == 0 else 0.25 * sp.j0(d)) * r

    re = integrate.dblquad(lambda th, r: g(th, r, 0), 0, a, 0, 2 * np.pi, epsabs=1e-13)[0]
    im = integrate.dblquad(lambda th, r: g(th, r, 1), 0, a, 0, 2 * np.pi, epsabs=1e-13)[0]
    K = O.cell_kernel(4, 4, h, k0)
    assert abs(K[p, q] - (re + 1j * im)) <= 1e-11 * abs(K[p, q])


def test_disk_cell_close_to_square_cell():
    """The disk-equivalent cell integral is within O((k0 h)^2) of the square-cell integral."""
    h, k0 = 10.0, O.wavenumber(10.0, 2000.0)
    K = O.cell_kernel(3, 3, h, k0)
    sq = integrate.dblquad(lambda z, x: 0.25 * sp.j0(k0 * np.hypot(h + x, z)), -h / 2, h / 2, -h / 2, h / 2)[0]
    sq_im = integrate.dblquad(lambda z, x: -0.25 * sp.y0(k0 * np.hypot(h + x, z)), -h / 2, h / 2, -h / 2, h / 2)[0]
    ref = sq_im + 1j * sq   # (i/4)H0 = -Y0/4 + i J0/4
    assert abs(K[1, 0] - ref) / abs(ref) < (k0 * h) ** 2


# ------------------------------------------------------------------- operator
@pytest.mark.parametrize("nx,nz", [(5, 7), (12, 12), (9, 4), (1, 6)])
@pytest.mark.parametrize("mode", O.MODES)
def test_fft_equals_direct(nx, nz, mode):
    """P1: the circulant-embedded FFT product equals the direct O(n^2) sum."""
    rng = np.random.default_rng(nx * 100 + nz)
    vel = 2000.0 * (1 + 0.3 * rng.uniform(-1, 1, (nx, nz)))
    prob = O.Problem(vel, 10.0, 12.0, 2000.0)
    x = synth.random_vectors((3, nx, nz), 5)
    assert rel(prob.apply(x, mode), O.apply_direct(prob.K, prob.chi, x, mode)) < 1e-13


def test_adjoint_identity():
    """P2: <A x, y> = <x, A^H y> and <G0V x, y> = <x, V^H G0^H y>."""
    w = synth.model_layered_salt(n=24, h=10.0, freq=15.0, seed=3, nsrc=2)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    x = synth.random_vectors((prob.nx, prob.nz), 1)
    y = synth.random_vectors((prob.nx, prob.nz), 2)
    for fwd, adj in (("A", "AH"), ("G0V", "VHG0H")):
        lhs = np.vdot(y, prob.apply(x, fwd))
        rhs = np.vdot(prob.apply(y, adj), x)
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_greens_matrix_complex_symmetric():
    w = synth.weak_contrast(n=8)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    G = O.greens_matrix(prob.K)
    assert np.array_equal(G, G.T)


# ------------------------------------------------------------------ solutions
def small_inclusion(n=32):
    return synth.model_smooth_inclusion(n=n, h=10.0 * 64 / n, freq=10.0, seed=1)


def test_series_matches_lu():
    """P3: the preconditioned series converges to the dense-LU solution (eq. 6)."""
    w = small_inclusion(32)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)[0]
    ref = O.solve_direct(prob, psi0)
    om = synth.gaussian_probes(prob.n, 32, 11).reshape(32, prob.nx, prob.nz)
    H = O.LowRankPreconditioner.build(prob, om)
    psi, it, r, st = O.series_solve(prob, H.apply, psi0, 1e-13, 60)
    assert st == O.OK and r <= 1e-13
    assert rel(psi, ref) < 1e-10
    assert 1 <= it <= 30


def test_zero_contrast():
    """P4: chi = 0 gives W = 0, H = I, psi = psi0 after zero iterations, no NaN."""
    n = 16
    w = synth.Workload("zero", np.full((n, n), 2000.0), 10.0, 10.0, 2000.0,
                       np.array([3]), np.array([0]))
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)[0]
    om = synth.gaussian_probes(prob.n, 8, 3).reshape(8, n, n)
    H = O.LowRankPreconditioner.build(prob, om)
    assert np.all(np.isfinite(H.U)) and np.all(H.W == 0)
    psi, it, r, st = O.series_solve(prob, H.apply, psi0, 1e-12, 30)
    assert it == 0 and st == O.OK and np.array_equal(psi, psi0)


def test_reciprocity():
    """P5: psi_{s1}(x_{s2}) = psi_{s2}(x_{s1}) for the discrete system (A^{-1} G0 is complex symmetric)."""
    w = synth.model_layered_salt(n=24, h=10.0, freq=15.0, seed=5, nsrc=2)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    si, sj = np.array([3, 17]), np.array([0, 9])
    psi = O.solve_direct(prob, prob.incident(si, sj))
    a = psi[0][si[1], sj[1]]
    b = psi[1][si[0], sj[0]]
    assert abs(a - b) <= 1e-12 * abs(a)


def test_smw_identity():
    """P6: H (I - U W^H) x = x for H = I + U (I - W^H U)^{-1} W^H (eq. 12)."""
    rng = np.random.default_rng(4)
    n, r = 200, 12
    U = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    W = 0.1 * (rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r)))
    H = O.LowRankPreconditioner(U, W)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = H.apply(x - U @ (W.conj().T @ x))
    assert rel(y, x) < 1e-13


def test_full_rank_probe_block_inverts():
    """P7: with l >= rank(G0 V), U W^H = G0 V, H = A^{-1}, and H psi0 already solves eq. (5)."""
    n = 32
    w = synth.model_smooth_inclusion(n=n, h=20.0, freq=10.0, seed=1, with_background=False)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    m = int(np.count_nonzero(prob.chi))
    l = m + 8
    om = synth.gaussian_probes(prob.n, l, 9).reshape(l, n, n)
    H = O.LowRankPreconditioner.build(prob, om)
    G0V = O.greens_matrix(prob.K) * prob.chi.reshape(-1)[None, :]
    assert rel(H.approx_g0v(), G0V) < 1e-12
    psi0 = prob.incident(w.src_i, w.src_j)[0]
    psi, it, r, st = O.series_solve(prob, H.apply, psi0, 1e-11, 30)
    assert it == 0 and st == O.OK


def test_halko_bound():
    """P8: ||G0V - U W^H||_2 <= [1 + 9 sqrt(k+p) sqrt(n)] sigma_{k+1} (Halko et al., w.p. >= 1 - 3 p^-p)."""
    w = synth.model_layered_salt(n=16, h=10.0, freq=15.0, seed=2, nsrc=1)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    k, p = 10, 6
    om = synth.gaussian_probes(prob.n, k + p, 21).reshape(k + p, 16, 16)
    U, W = O.range_finder_g0v(prob, om)
    G0V = O.greens_matrix(prob.K) * prob.chi.reshape(-1)[None, :]
    s = np.linalg.svd(G0V, compute_uv=False)
    err = np.linalg.norm(G0V - U @ W.conj().T, 2)
    assert err <= (1 + 9 * np.sqrt(k + p) * np.sqrt(prob.n)) * s[k]
    assert err >= s[k + p] * (1 - 1e-12)     # no rank-(k+p) factorization beats the SVD
    # q = 1 power iteration (Alg. 2 step 4) does not make the error worse than the bound either
    U1, W1 = O.range_finder_g0v(prob, om, q=1)
    assert np.linalg.norm(G0V - U1 @ W1.conj().T, 2) <= (1 + 9 * np.sqrt(k + p) * np.sqrt(prob.n)) * s[k]


def test_oversampled_truncation_is_rank_k():
    """Oversampling l = k + p with SVD truncation yields exactly rank-k factors of the same range."""
    w = synth.model_layered_salt(n=16, h=10.0, freq=15.0, seed=2, nsrc=1)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    om = synth.gaussian_probes(prob.n, 14, 5).reshape(14, 16, 16)
    U, W = O.range_finder_g0v(prob, om, rank=10)
    assert U.shape == (prob.n, 10) and W.shape == (prob.n, 10)
    Q, Wf = O.range_finder_g0v(prob, om)
    Af = Q @ Wf.conj().T
    s = np.linalg.svd(Af, compute_uv=False)
    assert abs(np.linalg.norm(Af - U @ W.conj().T, 2) - s[10]) <= 1e-10 * s[0]


def test_born_equals_neumann_sum():
    """P10: the Born iterate psi_j equals sum_{n<=j} (G0 V)^n psi0 and converges to the LU solution."""
    w = synth.weak_contrast(n=16)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)[0]
    G0V = O.greens_matrix(prob.K) * prob.chi.reshape(-1)[None, :]
    acc, term = psi0.reshape(-1).copy(), psi0.reshape(-1).copy()
    for _ in range(6):
        term = G0V @ term
        acc = acc + term
    assert rel(O.born(prob, psi0, 6).reshape(-1), acc) < 1e-13
    assert np.abs(prob.chi).max() * np.abs(O.circulant_table(prob.K)).sum() < 1
    assert rel(O.born(prob, psi0, 40), O.solve_direct(prob, psi0)) < 1e-12


def test_series_with_identity_is_born():
    """H = I turns eq. (11) into the Born recursion (Section 2.2)."""
    w = synth.weak_contrast(n=16)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)[0]
    psi, it, r, st = O.series_solve(prob, O.identity_preconditioner, psi0, 1e-300, 7)
    assert st == O.NOT_CONVERGED
    assert rel(psi, O.born(prob, psi0, 7)) < 1e-14


def test_block_inverse_identity():
    """P11: the 2x2 block inverse (Section 2.4) with top-right block -A^{-1} B S^{-1}."""
    rng = np.random.default_rng(8)
    a, d = 7, 5
    M = rng.standard_normal((a + d, a + d)) + 1j * rng.standard_normal((a + d, a + d)) + 4 * np.eye(a + d)
    A, B, C, D = M[:a, :a], M[:a, a:], M[a:, :a], M[a:, a:]
    assert rel(O.block_inverse(A, B, C, D), np.linalg.inv(M)) < 1e-13


def test_printed_block_inverse_reading_is_wrong():
    """The printed top-right block -B A^{-1} S^{-1} is not the inverse for square non-commuting blocks."""
    rng = np.random.default_rng(9)
    M = rng.standard_normal((8, 8)) + 5 * np.eye(8)
    A, B, C, D = M[:4, :4], M[:4, 4:], M[4:, :4], M[4:, 4:]
    Ai = np.linalg.inv(A)
    Si = np.linalg.inv(D - C @ Ai @ B)
    assert np.linalg.norm(-B @ Ai @ Si - np.linalg.inv(M)[:4, 4:]) > 1e-3


def test_printed_update_reading_is_wrong():
    """Eq. (14) taken literally (psi_j = a + U Z W^H a) does not converge to the solution."""
    w = small_inclusion(16)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)[0]
    om = synth.gaussian_probes(prob.n, 32, 11).reshape(32, 16, 16)
    H = O.LowRankPreconditioner.build(prob, om)
    psi = H.apply(psi0)
    for _ in range(20):
        psi = H.apply(prob.apply(psi, "A") - psi0)
    assert O.relative_residual(prob, psi, psi0) > 1e-3


def test_fixed_point_independent_of_h_and_start():
    """P14: different preconditioners and initial guesses reach the same fixed point (eqs. 7-9)."""
    w = small_inclusion(24)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)[0]
    ref = O.solve_direct(prob, psi0)
    outs = []
    for l, seed in ((24, 1), (48, 2)):
        om = synth.gaussian_probes(prob.n, l, seed).reshape(l, 24, 24)
        H = O.LowRankPreconditioner.build(prob, om)
        for phi0 in (None, synth.random_vectors((24, 24), seed)):
            psi, it, r, st = O.series_solve(prob, H.apply, psi0, 1e-13, 80, phi0=phi0)
            assert st == O.OK
            outs.append(psi)
    for p in outs:
        assert rel(p, ref) < 1e-10


def test_gmres_agrees_with_lu():
    w = small_inclusion(24)
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    psi0 = prob.incident(w.src_i, w.src_j)
    assert rel(O.gmres_solve(prob, psi0), O.solve_direct(prob, psi0)) < 1e-11


@pytest.mark.slow
def test_inclusion_closed_form_convergence():
    """P12: the discrete LS field approaches the Bessel-series field as h decreases (factor-3 refinement)."""
    L, f, c0, c1, R = 480.0, 8.0, 2000.0, 2500.0, 100.0
    centre = (300.0, 240.0)
    k0, k1 = 2 * np.pi * f / c0, 2 * np.pi * f / c1
    errs = []
    for n, (si, sj) in ((24, (5, 12)), (72, (16, 37))):
        h = L / n
        xc = (np.arange(n) + 0.5) * h
        X, Z = np.meshgrid(xc, xc, indexing="ij")
        vel = np.where(np.hypot(X - centre[0], Z - centre[1]) <= R, c1, c0)
        prob = O.Problem(vel, h, f, c0)
        psi0 = prob.incident([si], [sj])
        psi = O.gmres_solve(prob, psi0, tol=1e-12)[0]
        src = ((si + 0.5) * h, (sj + 0.5) * h)
        exact = inclusion_field(X, Z, centre, R, k0, k1, src)
        # compare on the coarse-grid cell centres away from the interface and the source
        hc = L / 24
        sel = (np.abs(np.hypot(X - centre[0], Z - centre[1]) - R) > 2 * hc) & \
              (np.hypot(X - src[0], Z - src[1]) > 2 * hc)
        coarse = np.isclose(np.mod(X / hc - 0.5, 1.0), 0) & np.isclose(np.mod(Z / hc - 0.5, 1.0), 0)
        m = sel & coarse
        errs.append(np.linalg.norm(psi[m] - exact[m]) / np.linalg.norm(exact[m]))
    assert errs[0] < 0.1
    assert errs[1] < 0.6 * errs[0], errs
