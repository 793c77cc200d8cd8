"""Plain FP64 oracle of the Lippmann-Schwinger operator in 3D.

TEST INFRASTRUCTURE ONLY (see ``oracle/lsop_oracle.py``).

The paper works the method out in 2D and notes that the same construction
carries over to 3D (Section 1 and the conclusions).  The 3D form used here
keeps every reading of the 2D oracle and changes only what the dimension
changes:

* Green's function of the 3D Helmholtz operator with the paper's sign
  convention (right-hand side -S): G0(r) = exp(i k0 r) / (4 pi r), outgoing
  for an exp(-i omega t) time factor.
* Cell integral over the ball of equal volume, radius a = h (3 / (4 pi))^(1/3).
  For a cell at lag (p, q, s) != 0 (distance r = h |(p, q, s)| >= h > a) the
  mean-value property of Helmholtz solutions over spheres gives
  K = (sin(k0 a) - k0 a cos(k0 a)) / k0^3 * exp(i k0 r) / r; the self cell
  integrates to K(0) = ((1 - i k0 a) exp(i k0 a) - 1) / k0^2.
  (G0 V)_{mn} = K(m - n) chi_n with chi of eq. (1), dv = h^3.
* Cells (i, j, l) with l fastest, n = (i ny + j) nz + l; vectors [.., nx, ny, nz].
* The circulant embedding, point sources (density amp / dv) and the four
  operator modes are those of the 2D oracle, one axis more.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

from .lsop_oracle import contrast, wavenumber


def ball_radius(h):
    return h * (3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)


def cell_kernel3(nx, ny, nz, h, k0):
    """K[p, q, s]: integral of exp(i k0 |x|) / (4 pi |x|) over the equal-volume ball at lag (p, q, s)."""
    a = ball_radius(h)
    ka = k0 * a
    p = np.arange(nx, dtype=np.float64)[:, None, None]
    q = np.arange(ny, dtype=np.float64)[None, :, None]
    s = np.arange(nz, dtype=np.float64)[None, None, :]
    r = h * np.sqrt(p * p + q * q + s * s)
    r[0, 0, 0] = 1.0
    K = (np.sin(ka) - ka * np.cos(ka)) / k0 ** 3 * np.exp(1j * k0 * r) / r
    K[0, 0, 0] = ((1.0 - 1j * ka) * np.exp(1j * ka) - 1.0) / k0 ** 2
    return K


def greens_matrix3(K):
    nx, ny, nz = K.shape
    i, j, l = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    i, j, l = i.reshape(-1), j.reshape(-1), l.reshape(-1)
    return K[np.abs(i[:, None] - i[None, :]), np.abs(j[:, None] - j[None, :]), np.abs(l[:, None] - l[None, :])]


def apply_direct3(K, chi, x, mode="A"):
    """Direct O(n^2) evaluation of the four modes on x[..., nx, ny, nz]."""
    G = greens_matrix3(K)
    c = chi.reshape(-1)
    n = c.size
    xb = np.asarray(x, np.complex128).reshape(-1, n)
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


def circulant_table3(K):
    """Symmetric circulant embedding into (2 nx) x (2 ny) x (2 nz); index p holds lag min(p, P - p), lag N is 0."""
    shp = K.shape
    idx = []
    for N in shp:
        P = 2 * N
        lag = np.minimum(np.arange(P), P - np.arange(P))
        idx.append(lag)
    out = np.zeros(tuple(2 * N for N in shp), np.complex128)
    m = [lag < N for lag, N in zip(idx, shp)]
    out[np.ix_(*m)] = K[np.ix_(*[lag[mm] for lag, mm in zip(idx, m)])]
    return out


def conv_fft3(Ghat, u, workers=None):
    P = Ghat.shape
    n = u.shape[-3:]
    U = sfft.fftn(np.asarray(u, np.complex128), s=P, axes=(-3, -2, -1), workers=workers)
    return sfft.ifftn(U * Ghat, axes=(-3, -2, -1), workers=workers)[..., :n[0], :n[1], :n[2]]


class Problem3:
    """The 3D grid problem: velocity [nx, ny, nz], cell size h, frequency, background c0."""

    def __init__(self, vel, h, freq_hz, c0):
        self.vel = np.asarray(vel, np.float64)
        self.nx, self.ny, self.nz = self.vel.shape
        self.h, self.freq, self.c0 = float(h), float(freq_hz), float(c0)
        self.k0 = wavenumber(freq_hz, c0)
        self.chi = contrast(self.vel, freq_hz, c0)
        self.K = cell_kernel3(self.nx, self.ny, self.nz, self.h, self.k0)
        self.Ghat = sfft.fftn(circulant_table3(self.K))
        self.workers = None

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def apply(self, x, mode="A"):
        chi = self.chi
        if mode == "A":
            return x - conv_fft3(self.Ghat, chi * x, self.workers)
        if mode == "G0V":
            return conv_fft3(self.Ghat, chi * x, self.workers)
        if mode == "AH":
            return x - np.conj(chi) * conv_fft3(np.conj(self.Ghat), x, self.workers)
        if mode == "VHG0H":
            return np.conj(chi) * conv_fft3(np.conj(self.Ghat), x, self.workers)
        raise ValueError(mode)

    def apply_direct(self, x, mode="A"):
        return apply_direct3(self.K, self.chi, x, mode)

    def incident(self, src, amp=None):
        """psi0 of point sources src[k] = (i, j, l) with amplitude amp[k] (density amp / h^3)."""
        amp = np.ones(len(src)) if amp is None else np.asarray(amp)
        i, j, l = np.meshgrid(np.arange(self.nx), np.arange(self.ny), np.arange(self.nz), indexing="ij")
        out = np.empty((len(src), self.nx, self.ny, self.nz), np.complex128)
        for k, (si, sj, sl) in enumerate(src):
            out[k] = amp[k] * self.K[np.abs(i - si), np.abs(j - sj), np.abs(l - sl)] / self.h ** 3
        return out

    def dense(self):
        G = greens_matrix3(self.K)
        return np.eye(self.n) - G * self.chi.reshape(-1)[None, :]


def solve_direct3(prob, psi0):
    lu = sla.lu_factor(prob.dense())
    b = np.asarray(psi0).reshape(-1, prob.n).T
    return sla.lu_solve(lu, b).T.reshape(np.shape(psi0))


def sphere_scattering(k0, k1, R, rs, r_obs, nmax=None):
    """Exact field of a point source (density delta, exp(-i omega t), G0 = e^{ikr}/(4 pi r)) at distance rs from
    the centre of a homogeneous ball of radius R and wavenumber k1 in a background k0, at observation points
    r_obs [m, 3] outside the ball, source on the +z axis.  Expansion in spherical harmonics (Legendre
    polynomials about the source axis): the incident field is
    i k0 sum_l (2l+1) j_l(k0 r<) h_l(k0 r>) P_l(cos theta) / (4 pi); the scattered field outside is
    sum_l b_l h_l(k0 r) P_l(cos theta) with b_l from continuity of the field and its radial derivative."""
    import scipy.special as sp
    if nmax is None:
        nmax = int(k0 * max(R, rs) + 25)
    r_obs = np.asarray(r_obs, np.float64)
    r = np.linalg.norm(r_obs, axis=1)
    ct = r_obs[:, 2] / r
    out_inc = np.zeros(len(r), np.complex128)
    out_sc = np.zeros(len(r), np.complex128)

    def h1(l, x, d=False):
        return sp.spherical_jn(l, x, d) + 1j * sp.spherical_yn(l, x, d)
    for l in range(nmax + 1):
        Pl = sp.eval_legendre(l, ct)
        c = 1j * k0 * (2 * l + 1) / (4 * np.pi)
        alpha = c * h1(l, k0 * rs)                       # incident: alpha j_l(k0 r) P_l for r < rs
        num = k1 * sp.spherical_jn(l, k1 * R, True) * sp.spherical_jn(l, k0 * R) - \
            k0 * sp.spherical_jn(l, k1 * R) * sp.spherical_jn(l, k0 * R, True)
        den = k0 * sp.spherical_jn(l, k1 * R) * h1(l, k0 * R, True) - k1 * sp.spherical_jn(l, k1 * R, True) * h1(l, k0 * R)
        b = alpha * num / den
        rl, rg = np.minimum(r, rs), np.maximum(r, rs)
        out_inc += c * sp.spherical_jn(l, k0 * rl) * h1(l, k0 * rg) * Pl
        out_sc += b * h1(l, k0 * r) * Pl
    return out_inc, out_sc
