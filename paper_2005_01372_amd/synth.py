"""Seeded synthetic inputs: velocity models, source positions and Gaussian probes.

This module holds no arithmetic of the solver itself. It only draws the
inputs that both the HIP path and the FP64 oracle consume, so that the two
see identical problems. The paper's own models (a resampled Marmousi2 subset
and the 2D SEG/EAGE salt model, Section 3) are not available; the workloads
below are synthetic stand-ins with the velocity ranges, grid spacings and
source geometry of the benchmark configurations.

Grid convention (Section 2.4, column-wise ordering): arrays are indexed
``[ix, iz]`` with ``ix`` the horizontal cell index and ``iz`` the depth index
(``iz = 0`` is the top row); ``iz`` is the fastest-varying index in memory.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

C0_DEFAULT = 2000.0  # background velocity used in both of the paper's experiments (Section 3)


@dataclass
class Workload:
    """One Helmholtz problem: velocity grid, frequency, spacing and point sources."""
    name: str
    vel: np.ndarray            # [nx, nz] float64, m/s
    h: float                   # cell size, m
    freq: float                # Hz
    c0: float                  # background velocity, m/s
    src_i: np.ndarray          # [nsrc] int32 horizontal cell index
    src_j: np.ndarray          # [nsrc] int32 depth cell index
    amp: np.ndarray = field(default=None)   # [nsrc] complex128 source amplitudes

    def __post_init__(self):
        if self.amp is None:
            self.amp = np.ones(len(self.src_i), np.complex128)

    @property
    def nx(self):
        return self.vel.shape[0]

    @property
    def nz(self):
        return self.vel.shape[1]

    @property
    def nsrc(self):
        return len(self.src_i)


def smoothed_field(shape, sigma, rng):
    """Gaussian-filtered iid N(0,1) field (reflect boundary) scaled to max |s| = 1."""
    s = ndimage.gaussian_filter(rng.standard_normal(shape), sigma, mode="reflect")
    return s / np.abs(s).max()


def disk_mask(nx, nz, ci, cj, radius):
    """Cells whose centres lie within ``radius`` cells of cell centre (ci, cj)."""
    i = np.arange(nx)[:, None]
    j = np.arange(nz)[None, :]
    return (i - ci) ** 2 + (j - cj) ** 2 <= radius ** 2


def model_smooth_inclusion(n=64, h=10.0, freq=10.0, seed=1, with_background=True):
    """Smooth +-10 % perturbation of 2000 m/s plus a 3000 m/s disk of radius 8 cells.

    With ``with_background=False`` the background is exactly c0, so the contrast
    is non-zero only inside the disk (the inclusion-only variant).
    """
    rng = np.random.default_rng(seed)
    s = smoothed_field((n, n), 4.0 * n / 64, rng)
    vel = C0_DEFAULT * (1.0 + 0.1 * s) if with_background else np.full((n, n), C0_DEFAULT)
    ci, cj, rad = 44 * n // 64, 32 * n // 64, 8 * n / 64
    vel = np.where(disk_mask(n, n, ci, cj, rad), 3000.0, vel)
    si = np.array([n // 2], np.int32)
    sj = np.array([n // 2], np.int32)
    return Workload(f"smooth+inclusion {n}x{n}", vel, h, freq, C0_DEFAULT, si, sj)


def model_layered_salt(n=256, h=10.0, freq=15.0, seed=2, nsrc=32):
    """Eight layers 1500-4500 m/s with two rectangular 4500 m/s salt-like blocks."""
    rng = np.random.default_rng(seed)
    sc = n / 256
    ifc = np.sort(rng.integers(int(16 * sc), int(240 * sc) + 1, 7))
    vlay = np.clip(np.linspace(1500.0, 4500.0, 8) + rng.uniform(-100.0, 100.0, 8), 1500.0, 4500.0)
    layer = np.searchsorted(ifc, np.arange(n), side="right")
    vel = np.repeat(vlay[layer][None, :], n, axis=0).astype(np.float64)
    for _ in range(2):
        w = max(1, int(rng.integers(30, 71) * sc))
        hh = max(1, int(rng.integers(15, 36) * sc))
        i0 = int(rng.integers(0, n - w + 1))
        j0 = int(rng.integers(int(64 * sc), max(int(64 * sc) + 1, int(224 * sc) - hh + 1)))
        vel[i0:i0 + w, j0:j0 + hh] = 4500.0
    step = max(1, n // nsrc)
    si = (step // 2 + step * np.arange(nsrc)).astype(np.int32) % n
    sj = np.zeros(nsrc, np.int32)
    return Workload(f"layered+salt {n}x{n}", vel, h, freq, C0_DEFAULT, si, sj)


def model_random_ellipses(n=1024, h=5.0, freq=25.0, seed=3, nsrc=128, vmin=1500.0, vmax=5000.0):
    """Smoothed random field mapped to [vmin, vmax] plus six random elliptical inclusions."""
    rng = np.random.default_rng(seed)
    s = smoothed_field((n, n), 24.0 * n / 1024, rng)
    vel = vmin + (s - s.min()) / (s.max() - s.min()) * (vmax - vmin)
    i = np.arange(n)[:, None] + 0.5
    j = np.arange(n)[None, :] + 0.5
    sc = n / 1024
    for _ in range(6):
        ci, cj = rng.uniform(0.1, 0.9, 2) * n
        a, b = rng.integers(15, 81, 2) * sc
        th = rng.uniform(0.0, np.pi)
        v = rng.uniform(vmin, vmax)
        u = (i - ci) * np.cos(th) + (j - cj) * np.sin(th)
        w = -(i - ci) * np.sin(th) + (j - cj) * np.cos(th)
        vel = np.where((u / max(a, 1)) ** 2 + (w / max(b, 1)) ** 2 <= 1.0, v, vel)
    step = max(1, n // nsrc)
    si = (step // 2 + step * np.arange(nsrc)).astype(np.int32) % n
    sj = np.zeros(nsrc, np.int32)
    return Workload(f"smooth random+ellipses {n}x{n}", vel, h, freq, C0_DEFAULT, si, sj)


def model_uneven_batch(count=64, seed0=4, sizes=(128, 192, 256, 384, 512), fmin=5.0, fmax=30.0, h=5.0):
    """Independent instances of uneven grid size, frequency and source count."""
    out = []
    for t in range(count):
        rng = np.random.default_rng(seed0 + t)
        n = int(rng.choice(sizes))
        f = float(rng.uniform(fmin, fmax))
        s = smoothed_field((n, n), n / 32.0, rng)
        vel = 1500.0 + (s - s.min()) / (s.max() - s.min()) * 3000.0
        ns = int(rng.integers(1, 17))
        si = ((np.arange(ns) + 0.5) * n / ns).astype(np.int32)
        out.append(Workload(f"instance {t} {n}x{n}", vel, h, f, C0_DEFAULT, si, np.zeros(ns, np.int32)))
    return out


def weak_contrast(n=32, h=10.0, freq=5.0, seed=7, pert=0.02):
    """Small grid with a weak smooth perturbation, where the Born series converges."""
    rng = np.random.default_rng(seed)
    vel = C0_DEFAULT * (1.0 + pert * smoothed_field((n, n), 3.0, rng))
    return Workload(f"weak {n}x{n}", vel, h, freq, C0_DEFAULT,
                    np.array([n // 2], np.int32), np.array([0], np.int32))


def gaussian_probes(n_cells, nprobe, seed):
    """Real standard-normal probe block, shape [nprobe, n_cells] (one probe per row)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nprobe, n_cells))


def random_vectors(shape, seed, dtype=np.complex128):
    """Complex vectors with iid N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return v.astype(dtype)
