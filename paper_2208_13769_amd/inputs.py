"""Seeded synthetic workloads for the Lagrangian solid LBM.

This module only draws and shapes initial fields and plate parameters. It
holds none of the method's arithmetic, so the FP64 oracle and the HIP path
can both be fed from it. Every array is float64 in physical units, laid out
as ``[component, y, x]`` with x fastest; node (x, y) sits at X = (x dX, y dX).

Workloads (all units physical, dX = rho0 = 1 unless stated):

* ``shear_wave``: u0 = 0 and v0_y = amp sin(2 pi x / wavelength), v0_x = 0 --
  a small-strain standing shear wave on a periodic grid.
* ``filtered_random_velocity``: i.i.d. N(0, 1) per site and component from
  numpy's PCG64 with the given seed, Gaussian-filtered over the periodic grid
  in Fourier space (standard deviation ``sigma`` cells, mean removed), then
  scaled so that the largest |v| component equals ``peak``.
* ``plate_batch``: plates for a batched run -- side N = round(64 * 16**U),
  U ~ U[0, 1) (log-uniform over 64..1024), lam ~ U[0.05, 0.2],
  mu ~ U[0.02, 0.1], all from one seeded PCG64 stream.
* ``top_pulse``: a downward velocity pulse at the top edge of a plate of N
  rows and Nx columns, v_y = -amp exp(-(d / w)^2) (1 - cos(2 pi x / Nx)) / 2
  with d the distance in cells from the top node row and w = max(2, N / 32).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def shear_wave(nx: int, ny: int, amp: float, wavelength: float):
    x = np.arange(nx, dtype=np.float64)
    u0 = np.zeros((2, ny, nx))
    v0 = np.zeros((2, ny, nx))
    v0[1] = amp * np.sin(2.0 * np.pi * x / wavelength)[None, :]
    return u0, v0


def longitudinal_wave(nx: int, ny: int, amp: float, wavelength: float):
    """u0 = 0 and v0_x = amp sin(2 pi x / wavelength): a compression wave."""
    x = np.arange(nx, dtype=np.float64)
    u0 = np.zeros((2, ny, nx))
    v0 = np.zeros((2, ny, nx))
    v0[0] = amp * np.sin(2.0 * np.pi * x / wavelength)[None, :]
    return u0, v0


def filtered_random_velocity(nx: int, ny: int, sigma: float, seed: int, peak: float):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((2, ny, nx))
    kx = np.fft.fftfreq(nx) * 2.0 * np.pi
    ky = np.fft.fftfreq(ny) * 2.0 * np.pi
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    filt = np.exp(-0.5 * sigma * sigma * k2)
    filt[0, 0] = 0.0
    v = np.real(np.fft.ifft2(np.fft.fft2(g, axes=(1, 2)) * filt[None], axes=(1, 2)))
    v *= peak / np.max(np.abs(v))
    return np.zeros((2, ny, nx)), np.ascontiguousarray(v)


def random_field(nx: int, ny: int, seed: int, scale: float):
    """Unfiltered i.i.d. N(0, scale^2) values per site and component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal((2, ny, nx))


@dataclass
class Plate:
    n: int
    lam: float
    mu: float


def plate_batch(count: int, seed: int, n_min: int = 64, n_max: int = 1024):
    rng = np.random.Generator(np.random.PCG64(seed))
    ratio = n_max / n_min
    plates = []
    for _ in range(count):
        u = rng.random()
        n = int(round(n_min * ratio ** u))
        lam = 0.05 + 0.15 * rng.random()
        mu = 0.02 + 0.08 * rng.random()
        plates.append(Plate(n=n, lam=lam, mu=mu))
    return plates


def top_pulse(n: int, amp: float, nx: int | None = None):
    """Plate of n rows (and nx columns, default n) with the pulse at its top."""
    nx = n if nx is None else nx
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(n, dtype=np.float64)
    d = (n - 1) - y
    w = max(2.0, n / 32.0)
    prof = np.exp(-(d / w) ** 2)[:, None] * (0.5 * (1.0 - np.cos(2.0 * np.pi * x / nx)))[None, :]
    u0 = np.zeros((2, n, nx))
    v0 = np.zeros((2, n, nx))
    v0[1] = -amp * prof
    return u0, v0
