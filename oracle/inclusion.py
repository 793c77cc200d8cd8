"""Closed-form field of a line source near a homogeneous circular inclusion (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/lsop_oracle.py``).

This is the continuous problem of Section 2.1 for the simplest non-trivial
medium: background wavenumber k0 everywhere except inside a disk of radius R
with wavenumber k1, constant density, and a unit line source
S = delta(x - x_s) outside the disk, so that the incident field is
psi0 = (i/4) H0^(1)(k0 |x - x_s|).  Separation of variables in polar
coordinates about the disk centre, with psi and its radial derivative
continuous at r = R, gives

* incident, expanded by Graf's theorem for r < r_s:
  sum_n alpha_n J_n(k0 r) e^{i n (theta - theta_s)}, alpha_n = (i/4) H_n^(1)(k0 r_s)
* scattered field outside:  sum_n b_n H_n^(1)(k0 r) e^{i n (theta - theta_s)}
* field inside:             sum_n c_n J_n(k1 r)     e^{i n (theta - theta_s)}

with
  b_n = alpha_n [k1 J_n'(k1 R) J_n(k0 R) - k0 J_n(k1 R) J_n'(k0 R)]
        / [k0 J_n(k1 R) H_n'(k0 R) - k1 J_n'(k1 R) H_n(k0 R)]
and c_n from either matching condition.  The discrete LS solution converges
to this field as the grid is refined (staircased disk, cell-averaged kernel).
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp


def inclusion_coefficients(k0, k1, R, r_s, nmax):
    n = np.arange(-nmax, nmax + 1)
    alpha = 0.25j * sp.hankel1(n, k0 * r_s)
    J0R, J1R = sp.jv(n, k0 * R), sp.jv(n, k1 * R)
    dJ0R, dJ1R = sp.jvp(n, k0 * R), sp.jvp(n, k1 * R)
    H0R, dH0R = sp.hankel1(n, k0 * R), sp.h1vp(n, k0 * R)
    b = alpha * (k1 * dJ1R * J0R - k0 * J1R * dJ0R) / (k0 * J1R * dH0R - k1 * dJ1R * H0R)
    # c_n from the continuity of psi, or of d psi / dr where J_n(k1 R) is tiny
    use_val = np.abs(J1R) >= np.abs(dJ1R)
    c_val = (alpha * J0R + b * H0R) / np.where(use_val, J1R, 1.0)
    c_der = (alpha * k0 * dJ0R + b * k0 * dH0R) / np.where(use_val, 1.0, k1 * dJ1R)
    c = np.where(use_val, c_val, c_der)
    return n, alpha, b, c


def inclusion_field(px, pz, centre, R, k0, k1, src, amp=1.0):
    """Total field at points (px, pz) (arrays, metres) for a source at ``src`` outside the disk."""
    px = np.asarray(px, np.float64)
    pz = np.asarray(pz, np.float64)
    xs, zs = src
    xc, zc = centre
    r_s = np.hypot(xs - xc, zs - zc)
    th_s = np.arctan2(zs - zc, xs - xc)
    if r_s <= R:
        raise ValueError("source must lie outside the inclusion")
    nmax = int(np.ceil(max(k0, k1) * max(R, r_s))) + 20
    n, alpha, b, c = inclusion_coefficients(k0, k1, R, r_s, nmax)
    r = np.hypot(px - xc, pz - zc)
    th = np.arctan2(pz - zc, px - xc)
    ph = np.exp(1j * n[None, :] * (th.reshape(-1)[:, None] - th_s))
    rr = r.reshape(-1)[:, None]
    inside = (r.reshape(-1) < R)
    out = np.empty(r.size, np.complex128)
    rin = np.where(inside[:, None], rr, 0.0)
    out_in = np.sum(c[None, :] * sp.jv(n[None, :], k1 * rin) * ph, axis=1)
    rout = np.where(inside[:, None], R, rr)
    scat = np.sum(b[None, :] * sp.hankel1(n[None, :], k0 * rout) * ph, axis=1)
    dist = np.hypot(px.reshape(-1) - xs, pz.reshape(-1) - zs)
    inc = 0.25j * sp.hankel1(0, k0 * np.where(dist > 0, dist, 1.0))
    out[:] = np.where(inside, out_in, inc + scat)
    return (amp * out).reshape(r.shape)
