"""Convergent Born series (the series of Osnabrugge et al. that Section 2.2 reviews): plain FP64 oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/lsop_oracle.py``).

Section 2.2 describes it as the homotopy series of eq. (9) with the
preconditioner H = gamma = i V / eps, where the background Green's function is
made dissipative and a gain i eps added to V so that the equation itself is
unchanged, and states that the series converges when eps is at least
omega^2 max |1/c^2 - 1/c0^2| = max |chi|.

Readings (the paper gives the construction in words only):

* Time convention exp(-i omega t) with outgoing (i/4) H0^(1) (as the rest of
  this oracle): the dissipative background is k_eps^2 = k0^2 + i eps, with
  k_eps the root of positive real and imaginary part, and the Helmholtz
  equation with k^2 = k0^2 + chi becomes
  (Laplacian + k_eps^2) psi = -S - (chi - i eps) psi, i.e.
  psi = psi0_eps + G_eps V_eps psi with V_eps = chi - i eps (the paper writes
  chi + i eps for the opposite time convention).
* G_eps is discretised exactly as G0 (cell integral over the equal-area
  disk, Graf's addition theorem), with k0 replaced by k_eps:
  K(p,q) = (i pi a / (2 k)) J1(k a) H0^(1)(k h rho), K(0,0) = (i pi a / (2 k))
  H1^(1)(k a) - 1/k^2.
* Outside the grid V_eps = 0: the exterior is the dissipative background, an
  absorbing exterior.  Optional absorbing layer of `absorb` cells at the grid
  edges: the compensation -i eps is scaled by r(d) = 1 - (1 - d / absorb) / 2
  for d < absorb cells from the edge (r = 1/2 on the edge cells), so the
  medium turns lossy gradually.
* gamma = i V_eps / eps pointwise; the series is eq. (11) with H = gamma and
  psi_0 = gamma psi0_eps (the paper: phi_0 = gamma psi0).
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

from .lsop_oracle import apply_direct, apply_fft, contrast, greens_matrix, spectrum, wavenumber


def damped_wavenumber(k0, eps):
    """k_eps with k_eps^2 = k0^2 + i eps, Re k_eps > 0, Im k_eps >= 0."""
    return np.sqrt(complex(k0) ** 2 + 1j * eps)


def damped_kernel(nx, nz, h, k):
    """Cell-integrated kernel of the dissipative Green's function (i/4) H0^(1)(k |x|), complex k."""
    a = h / np.sqrt(np.pi)
    c = 1j * np.pi * a / (2.0 * k)
    p = np.arange(nx, dtype=np.float64)[:, None]
    q = np.arange(nz, dtype=np.float64)[None, :]
    rho = np.sqrt(p * p + q * q)
    rho[0, 0] = 1.0
    K = c * sp.jv(1, k * a) * sp.hankel1(0, k * h * rho)
    K[0, 0] = c * sp.hankel1(1, k * a) - 1.0 / k ** 2
    return K


def compensation(nx, nz, absorb):
    """Fraction r of the gain i eps kept per cell: 1 inside, 1/2 .. 1 across an absorbing layer."""
    if absorb <= 0:
        return np.ones((nx, nz))
    i = np.arange(nx)[:, None]
    j = np.arange(nz)[None, :]
    d = np.minimum(np.minimum(i, j), np.minimum(nx - 1 - i, nz - 1 - j)).astype(np.float64)
    return 1.0 - 0.5 * np.maximum(0.0, 1.0 - d / absorb)


class DampedProblem:
    """The grid problem of the convergent Born series: operator I - G_eps V_eps, incident field G_eps S."""

    def __init__(self, vel, h, freq_hz, c0, eps, absorb=0):
        self.vel = np.asarray(vel, np.float64)
        self.nx, self.nz = self.vel.shape
        self.h, self.freq, self.c0, self.eps = float(h), float(freq_hz), float(c0), float(eps)
        self.k0 = wavenumber(freq_hz, c0)
        self.k = damped_wavenumber(self.k0, eps)
        self.chi = contrast(self.vel, freq_hz, c0)
        self.V = self.chi - 1j * self.eps * compensation(self.nx, self.nz, absorb)
        self.K = damped_kernel(self.nx, self.nz, self.h, self.k)
        self.Ghat = spectrum(self.K)
        self.workers = None

    @property
    def n(self):
        return self.nx * self.nz

    def apply(self, x, mode="A"):
        return apply_fft(self.Ghat, self.V, x, mode, self.workers)

    def apply_direct(self, x, mode="A"):
        return apply_direct(self.K, self.V, x, mode)

    def incident(self, src_i, src_j, amp=None):
        amp = np.ones(len(src_i)) if amp is None else np.asarray(amp)
        out = np.empty((len(src_i), self.nx, self.nz), np.complex128)
        i = np.arange(self.nx)[:, None]
        j = np.arange(self.nz)[None, :]
        for s, (si, sj) in enumerate(zip(src_i, src_j)):
            out[s] = amp[s] * self.K[np.abs(i - si), np.abs(j - sj)] / self.h ** 2
        return out

    def dense(self):
        G = greens_matrix(self.K)
        return np.eye(self.n) - G * self.V.reshape(-1)[None, :]

    def gamma(self, x):
        """H = gamma = i V_eps / eps, pointwise."""
        return (1j * self.V / self.eps) * np.asarray(x, np.complex128)
