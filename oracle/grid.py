"""Equidistant periodic grid, inner product and FFT derivatives (oracle).

Sec. 2.2: all functions live on a 3D equidistant grid and derivatives are
taken with FFTs.  Sec. 3.1: a spinor has V = nx*ny*nz*2 components.

Readings (the paper does not spell these out):
* grid points x_i = i*dx, i = 0..n-1, box L = n*dx, dV = dx^3;
* wave numbers k = 2 pi m / L with m in FFT order (0..n/2-1, -n/2..-1);
* derivative of a complex spinor component keeps the Nyquist mode
  (multiplier i*k with k = -pi/dx there), so D^2 = -k^2 everywhere;
* derivative of a real field zeroes the Nyquist mode so the result stays real;
* the Laplacian of a real field multiplies by -|k|^2 (Nyquist kept: it is
  real and even, so the result stays real);
* twisted boundary conditions (Sec. 1 names twist-averaged boundary
  conditions as the remedy for finite-volume effects): a state obeys
  psi(r + L e_m) = exp(i theta_m) psi(r).  It is stored as its periodic part
  u = exp(-i theta.r/L) psi, so every derivative of a state becomes
  d_m + i theta_m/L, i.e. the multiplier i(k_m + theta_m/L).  Densities and
  mean fields are periodic, so derivatives of real fields are untouched.

Arrays are indexed [..., z, y, x]; ``axis`` 0/1/2 means x/y/z.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np
import scipy.fft as sfft

# threads of scipy.fft (SKY_ORACLE_THREADS, default: every core of the process)
_WORKERS = int(os.environ.get("SKY_ORACLE_THREADS", "0")) or -1


@dataclasses.dataclass(frozen=True)
class Grid:
    n: int
    dx: float
    # Bloch phase per axis (x, y, z) in radians; (0, 0, 0) = periodic
    twist: tuple = (0.0, 0.0, 0.0)

    def with_twist(self, theta) -> "Grid":
        return Grid(self.n, self.dx, tuple(float(t) for t in theta))

    @property
    def L(self) -> float:
        return self.n * self.dx

    @property
    def dV(self) -> float:
        return self.dx ** 3

    def k(self) -> np.ndarray:
        """Wave numbers in FFT order, Nyquist at index n/2 (= -pi/dx)."""
        return 2.0 * math.pi * np.fft.fftfreq(self.n, d=self.dx)

    def k_real(self) -> np.ndarray:
        """Wave numbers with the Nyquist mode zeroed (for real fields)."""
        k = self.k()
        if self.n % 2 == 0:
            k[self.n // 2] = 0.0
        return k

    def k2(self) -> np.ndarray:
        """|k|^2 on the 3D grid, indexed [z, y, x] (real fields, no twist)."""
        k = self.k()
        return (k[:, None, None] ** 2 + k[None, :, None] ** 2
                + k[None, None, :] ** 2)

    def k_psi(self, axis: int) -> np.ndarray:
        """Wave numbers seen by a state along ``axis``: k + theta_axis / L."""
        return self.k() + self.twist[axis] / self.L

    def k2_psi(self) -> np.ndarray:
        """|k + theta/L|^2 on the 3D grid, indexed [z, y, x]."""
        kx, ky, kz = self.k_psi(0), self.k_psi(1), self.k_psi(2)
        return (kz[:, None, None] ** 2 + ky[None, :, None] ** 2
                + kx[None, None, :] ** 2)


def _array_axis(axis: int) -> int:
    # axis 0 = x is the last array axis, 1 = y, 2 = z
    return -1 - axis


def _bcast(vec: np.ndarray, axis: int, ndim: int) -> np.ndarray:
    shape = [1] * ndim
    shape[_array_axis(axis)] = vec.size
    return vec.reshape(shape)


def deriv(f: np.ndarray, g: Grid, axis: int) -> np.ndarray:
    """Spectral derivative of a state array along ``axis`` (Nyquist kept),
    including the grid's twist: multiplier i (k + theta_axis / L)."""
    ax = _array_axis(axis)
    fk = sfft.fft(f, axis=ax, workers=_WORKERS)
    fk *= 1j * _bcast(g.k_psi(axis), axis, f.ndim)
    return sfft.ifft(fk, axis=ax, workers=_WORKERS)


def deriv_real(f: np.ndarray, g: Grid, axis: int) -> np.ndarray:
    """Spectral derivative of a real field along ``axis`` (Nyquist zeroed)."""
    ax = _array_axis(axis)
    fk = sfft.fft(f, axis=ax, workers=_WORKERS)
    fk *= 1j * _bcast(g.k_real(), axis, f.ndim)
    return sfft.ifft(fk, axis=ax, workers=_WORKERS).real


def laplacian_real(f: np.ndarray, g: Grid) -> np.ndarray:
    """Laplacian of a real field: multiply by -|k|^2 in Fourier space."""
    fk = sfft.fftn(f, axes=(-3, -2, -1), workers=_WORKERS)
    fk *= -g.k2()
    return sfft.ifftn(fk, axes=(-3, -2, -1), workers=_WORKERS).real

