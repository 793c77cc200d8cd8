"""Plain FP64 CPU oracle for the preconditioned Lippmann-Schwinger solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this module.  The
product path (the HIP library and its Python binding) never does, and shares
no code with it: the only common module is the seeded input generator, which
holds none of the solver's arithmetic.

Everything here is written from Eikrem, Naevdal & Jakobsen, "Iterative
solution of the Lippmann-Schwinger equation in strongly scattering acoustic
media by randomized construction of preconditioners" (arXiv 2005.01372), in
complex128 with numpy / scipy, with no blocking, fusion or reordering beyond
what the paper states.

Readings of points the paper leaves open (each pinned by a test):

* The background Green's function of the 2D Helmholtz operator with the
  paper's sign convention (Section 2.1: right-hand sides -S and -delta) is
  G0(r) = (i/4) H0^(1)(k0 r), outgoing for an exp(-i omega t) time factor.
* The value of G0 per pair of grid cells (Section 2.1, eq. 4): the product G0 * dv
  of the matrix G0 V is taken as the integral of G0 over the source cell,
  with the square cell replaced by the disk of equal area (radius
  a = h / sqrt(pi)).  Integrating (i/4) H0^(1) over that disk gives, by
  Graf's addition theorem, K(p,q) = (i pi a / (2 k0)) J1(k0 a) H0^(1)(k0 h rho)
  for a cell at lag (p,q), rho = sqrt(p^2+q^2) > 0, and the closed form
  K(0,0) = (i pi a / (2 k0)) H1^(1)(k0 a) - 1/k0^2 for the singular self cell.
  (G0 V)_{mn} = K(m - n) chi_n.
* The extension of G0's first row for the FFT (Section 2.2, after eq. 11) is the symmetric
  circulant embedding into a P_x x P_z array with P >= 2N - 1 (here P = 2N),
  lag -p stored at index P - p.  This makes the FFT product exact on the grid.
* Every transpose in Alg. 1 / Alg. 2 is the conjugate transpose (Section 2.3
  defines its transposes that way), so
  W = V^H G0^H Q.
* Eq. (14) as printed cannot be the update (its fixed point is psi = 0); it is
  read as psi_j = psi_{j-1} - (a_{j-1} + U Z W^H a_{j-1}) = psi_{j-1} - H a_{j-1},
  which is eq. (11) with the low-rank H of eq. (12).
* The stopping rule is the relative residual ||A psi - psi0|| / ||psi0|| per
  source; the returned iterate is the one whose residual passed.
* A point source of amplitude ``amp`` in cell s has density amp / dv in that
  cell, so psi0_m = amp * K(m - s) / dv.

Grid: cell (i, j) with i horizontal, j depth, centre ((i+1/2) h, (j+1/2) h);
vectors are flattened with n = i * nz + j (column-wise ordering, Section 2.4).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.special as sp

# status codes shared by definition (not by code) with the C ABI
OK, NOT_CONVERGED, DIVERGED = 0, 4, 5


# --------------------------------------------------------------------------
# Section 2.1: physics and discretization
# --------------------------------------------------------------------------
def angular(freq_hz):
    return 2.0 * np.pi * freq_hz


def wavenumber(freq_hz, c0):
    return angular(freq_hz) / c0


def contrast(vel, freq_hz, c0):
    """Eq. (1): omega^2 / c(x)^2 = omega^2 / c0^2 + chi(x)."""
    w = angular(freq_hz)
    return w * w * (1.0 / np.asarray(vel, np.float64) ** 2 - 1.0 / c0 ** 2)


def cell_kernel(nx, nz, h, k0):
    """K[p, q] = integral of (i/4) H0^(1)(k0 |x|) over the cell at lag (p, q) (disk-equivalent).

    Returns the lags p in [0, nx), q in [0, nz); K is even in each lag.
    """
    a = h / np.sqrt(np.pi)
    c = 1j * np.pi * a / (2.0 * k0)
    p = np.arange(nx, dtype=np.float64)[:, None]
    q = np.arange(nz, dtype=np.float64)[None, :]
    rho = np.sqrt(p * p + q * q)
    rho[0, 0] = 1.0  # placeholder, overwritten below
    K = c * sp.jv(1, k0 * a) * sp.hankel1(0, k0 * h * rho)
    K[0, 0] = c * sp.hankel1(1, k0 * a) - 1.0 / k0 ** 2
    return K


def greens_matrix(K):
    """Dense n x n matrix with entries K(m - n) (G0 times dv), n = i * nz + j."""
    nx, nz = K.shape
    i = np.repeat(np.arange(nx), nz)
    j = np.tile(np.arange(nz), nx)
    return K[np.abs(i[:, None] - i[None, :]), np.abs(j[:, None] - j[None, :])]


def operator_matrix(K, chi):
    """Dense I - G0 V of eq. (5) (small grids only)."""
    G = greens_matrix(K)
    return np.eye(G.shape[0]) - G * chi.reshape(-1)[None, :]


# --------------------------------------------------------------------------
# Section 2.2: the operator by direct summation and by FFT
# --------------------------------------------------------------------------
MODES = ("A", "G0V", "AH", "VHG0H")


def apply_direct(K, chi, x, mode="A"):
    """Direct O(n^2) evaluation of the four operator modes on a batch x[..., nx, nz]."""
    nx, nz = K.shape
    G = greens_matrix(K)
    c = chi.reshape(-1)
    xb = np.asarray(x, np.complex128).reshape(-1, nx * nz)
    if mode == "A":
        y = xb - (G @ (c[:, None] * xb.T)).T
    elif mode == "G0V":
        y = (G @ (c[:, None] * xb.T)).T
    elif mode == "AH":
        y = xb - (np.conj(c)[:, None] * (G.conj().T @ xb.T)).T
    elif mode == "VHG0H":
        y = (np.conj(c)[:, None] * (G.conj().T @ xb.T)).T
    else:
        raise ValueError(mode)
    return y.reshape(np.shape(x))


def circulant_table(K):
    """Symmetric circulant embedding of the lag table into a (2 nx) x (2 nz) array.

    Index p holds lag min(p, P - p); the lag of magnitude N (index N) is zero.
    """
    nx, nz = K.shape
    px, pz = 2 * nx, 2 * nz
    lx = np.minimum(np.arange(px), px - np.arange(px))
    lz = np.minimum(np.arange(pz), pz - np.arange(pz))
    mx, mz = lx < nx, lz < nz
    Kt = np.zeros((px, pz), np.complex128)
    Kt[np.ix_(mx, mz)] = K[np.ix_(lx[mx], lz[mz])]
    return Kt


def spectrum(K):
    """F(G0~): 2D FFT of the circulant embedding."""
    return sfft.fft2(circulant_table(K))


def conv_fft(Ghat, u, workers=None):
    """F^-1(Ghat . F(u zero-extended)), cropped back to the grid, for u[..., nx, nz]."""
    px, pz = Ghat.shape
    nx, nz = u.shape[-2:]
    U = sfft.fft2(np.asarray(u, np.complex128), s=(px, pz), axes=(-2, -1), workers=workers)
    return sfft.ifft2(U * Ghat, axes=(-2, -1), workers=workers)[..., :nx, :nz]


def apply_fft(Ghat, chi, x, mode="A", workers=None):
    """The four operator modes through the FFT product (G0 is symmetric, so G0^H uses conj(Ghat))."""
    if mode == "A":
        return x - conv_fft(Ghat, chi * x, workers)
    if mode == "G0V":
        return conv_fft(Ghat, chi * x, workers)
    if mode == "AH":
        return x - np.conj(chi) * conv_fft(np.conj(Ghat), x, workers)
    if mode == "VHG0H":
        return np.conj(chi) * conv_fft(np.conj(Ghat), x, workers)
    raise ValueError(mode)


class Problem:
    """A discretized LS problem: contrast, kernel table and spectrum."""

    def __init__(self, vel, h, freq_hz, c0):
        self.vel = np.asarray(vel, np.float64)
        self.nx, self.nz = self.vel.shape
        self.h, self.freq, self.c0 = float(h), float(freq_hz), float(c0)
        self.k0 = wavenumber(freq_hz, c0)
        self.chi = contrast(self.vel, freq_hz, c0)
        self.K = cell_kernel(self.nx, self.nz, self.h, self.k0)
        self.Ghat = spectrum(self.K)
        self.workers = None

    @property
    def n(self):
        return self.nx * self.nz

    def apply(self, x, mode="A"):
        return apply_fft(self.Ghat, self.chi, x, mode, self.workers)

    def incident(self, src_i, src_j, amp=None):
        """psi0[s] = amp_s K(m - s) / dv for point sources at cells (src_i, src_j)."""
        src_i = np.atleast_1d(src_i)
        src_j = np.atleast_1d(src_j)
        amp = np.ones(len(src_i), np.complex128) if amp is None else np.atleast_1d(amp)
        i = np.arange(self.nx)[:, None]
        j = np.arange(self.nz)[None, :]
        out = np.empty((len(src_i), self.nx, self.nz), np.complex128)
        for s, (a, b) in enumerate(zip(src_i, src_j)):
            out[s] = amp[s] * self.K[np.abs(i - a), np.abs(j - b)] / self.h ** 2
        return out

    def dense(self):
        return operator_matrix(self.K, self.chi)


# --------------------------------------------------------------------------
# Eq. (6): direct solve, and the Born series (Section 2.2)
# --------------------------------------------------------------------------
def solve_direct(prob, psi0):
    """psi = (I - G0 V)^{-1} psi0 by dense LU (n up to a few thousand)."""
    A = prob.dense()
    lu = sla.lu_factor(A)
    b = np.asarray(psi0).reshape(-1, prob.n).T
    return sla.lu_solve(lu, b).T.reshape(np.shape(psi0))


def born(prob, psi0, n_terms):
    """psi_j = G0 V psi_{j-1} + psi0 with psi_0 = psi0; returns psi_{n_terms}."""
    psi = np.array(psi0, np.complex128)
    for _ in range(n_terms):
        psi = prob.apply(psi, "G0V") + psi0
    return psi


def gmres_solve(prob, psi0, tol=1e-13, restart=200, maxiter=50):
    """Independent Krylov solve of eq. (5) through the FFT operator (scipy GMRES)."""
    from scipy.sparse.linalg import LinearOperator, gmres
    shp = (prob.nx, prob.nz)
    op = LinearOperator((prob.n, prob.n), dtype=np.complex128,
                        matvec=lambda v: prob.apply(v.reshape(shp), "A").reshape(-1))
    out = []
    for b in np.asarray(psi0).reshape(-1, prob.n):
        x, info = gmres(op, b, rtol=tol, atol=0.0, restart=restart, maxiter=maxiter)
        out.append(x)
    return np.array(out).reshape(np.shape(psi0))


# --------------------------------------------------------------------------
# Eqs. (7)-(11): the homotopy / preconditioned scattering series
# --------------------------------------------------------------------------
def relative_residual(prob, psi, psi0):
    r = prob.apply(psi, "A") - psi0
    ax = tuple(range(r.ndim - 2, r.ndim))
    return np.sqrt(np.sum(np.abs(r) ** 2, axis=ax) / np.sum(np.abs(psi0) ** 2, axis=ax))


def series_solve(prob, apply_H, psi0, tol, max_iter=30, phi0=None, diverge_window=5):
    """Eq. (11) for one source: psi_j = psi_{j-1} - H (psi_{j-1} - G0 V psi_{j-1} - psi0).

    Starts from psi_0 = H psi0 (the paper's choice of phi0) unless ``phi0`` is
    given.  Returns (psi, iterations, relative residual, status) for the last
    iterate whose residual was evaluated: the first one with relative
    residual <= tol (OK), the one at max_iter (NOT_CONVERGED), or the one at
    which the residual was non-finite or had risen ``diverge_window`` times in
    a row (DIVERGED).
    """
    psi0 = np.asarray(psi0, np.complex128)
    nb = np.linalg.norm(psi0)
    psi = apply_H(psi0) if phi0 is None else np.array(phi0, np.complex128)
    rising = 0
    prev = np.inf
    it = 0
    while True:
        a = prob.apply(psi, "A") - psi0          # eq. (13)
        rel = np.linalg.norm(a) / nb if nb > 0 else np.linalg.norm(a)
        if not np.isfinite(rel):
            return psi, it, rel, DIVERGED
        if rel <= tol:
            return psi, it, rel, OK
        rising = rising + 1 if rel > prev else 0
        prev = rel
        if rising >= diverge_window:
            return psi, it, rel, DIVERGED
        if it == max_iter:
            return psi, it, rel, NOT_CONVERGED
        psi = psi - apply_H(a)                   # eq. (11) / (14) as read
        it += 1


# --------------------------------------------------------------------------
# Section 2.3: randomized low-rank approximation and the SMW preconditioner
# --------------------------------------------------------------------------
def orth(Y):
    """Orthonormal basis of the columns of Y (n x l) by Householder QR (LAPACK)."""
    Q, _ = np.linalg.qr(Y, mode="reduced")
    return Q


def range_finder_generic(A, omega, q=0):
    """Alg. 1 for an explicit matrix A (m x n) with a given Gaussian block omega (n x r).

    Returns (Q_q, Y~_{q+1}) with A ~= Q_q Y~_{q+1}^H.
    """
    Q = orth(A @ omega)
    for _ in range(q):
        Qt = orth(A.conj().T @ Q)
        Q = orth(A @ Qt)
    return Q, A.conj().T @ Q


def range_finder_g0v(prob, omega, q=0, rank=None):
    """Alg. 2: U, W with G0 V ~= U W^H from the probe block omega[l, nx, nz] (real).

    With ``rank`` < l, the l-column factorization is truncated to ``rank``
    columns through an l x l SVD (oversampling; not in the paper).
    """
    l = omega.shape[0]
    n = prob.n
    shp = (l, prob.nx, prob.nz)
    Y = prob.apply(np.asarray(omega, np.complex128).reshape(shp), "G0V").reshape(l, n).T
    Q = orth(Y)
    for _ in range(q):
        Yt = prob.apply(Q.T.reshape(shp), "VHG0H").reshape(l, n).T
        Qt = orth(Yt)
        Y = prob.apply(Qt.T.reshape(shp), "G0V").reshape(l, n).T
        Q = orth(Y)
    W = prob.apply(Q.T.reshape(shp), "VHG0H").reshape(l, n).T
    if rank is not None and rank < l:
        Q2, R2 = np.linalg.qr(W, mode="reduced")
        Ub, s, Vbh = np.linalg.svd(R2.conj().T)
        U = Q @ (Ub[:, :rank] * s[:rank])
        W = Q2 @ Vbh.conj().T[:, :rank]
        return U, W
    return Q, W


def smw_core(U, W):
    """Z = (I_r - W^H U)^{-1} of eq. (12)."""
    r = U.shape[1]
    return np.linalg.inv(np.eye(r) - W.conj().T @ U)


class LowRankPreconditioner:
    """H = I + U Z W^H (eq. 12), applied as three factors (eqs. 13-14)."""

    def __init__(self, U, W):
        self.U, self.W = U, W
        self.Z = smw_core(U, W)

    @classmethod
    def build(cls, prob, omega, q=0, rank=None):
        U, W = range_finder_g0v(prob, omega, q, rank)
        return cls(U, W)

    def apply(self, x):
        x = np.asarray(x, np.complex128)
        shp = x.shape
        xb = x.reshape(-1, self.U.shape[0]).T
        y = xb + self.U @ (self.Z @ (self.W.conj().T @ xb))
        return y.T.reshape(shp)

    def approx_g0v(self):
        return self.U @ self.W.conj().T


def identity_preconditioner(x):
    return np.array(x, np.complex128)


# --------------------------------------------------------------------------
# Section 2.4: the 2x2 block inverse used recursively for hierarchical matrices
# --------------------------------------------------------------------------
def block_inverse(A, B, C, D):
    """Inverse of [[A, B], [C, D]] via the Schur complement S = D - C A^{-1} B.

    The top-right block is -A^{-1} B S^{-1} (the printed order -B A^{-1} S^{-1}
    is read as a typo: it is not defined for non-square B).
    """
    Ai = np.linalg.inv(A)
    S = D - C @ Ai @ B
    Si = np.linalg.inv(S)
    return np.block([[Ai + Ai @ B @ Si @ C @ Ai, -Ai @ B @ Si],
                     [-Si @ C @ Ai, Si]])
