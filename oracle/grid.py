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
  real and even, so the result stays real).

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
        """|k|^2 on the 3D grid, indexed [z, y, x]."""
        k = self.k()
        return (k[:, None, None] ** 2 + k[None, :, None] ** 2
                + k[None, None, :] ** 2)


def _array_axis(axis: int) -> int:
    # axis 0 = x is the last array axis, 1 = y, 2 = z
    return -1 - axis


def _bcast(vec: np.ndarray, axis: int, ndim: int) -> np.ndarray:
    shape = [1] * ndim
    shape[_array_axis(axis)] = vec.size
    return vec.reshape(shape)


def deriv(f: np.ndarray, g: Grid, axis: int) -> np.ndarray:
    """Spectral derivative of a complex array along ``axis`` (Nyquist kept)."""
    ax = _array_axis(axis)
    fk = sfft.fft(f, axis=ax, workers=_WORKERS)
    fk *= 1j * _bcast(g.k(), axis, f.ndim)
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


def inner(a: np.ndarray, b: np.ndarray, g: Grid) -> complex:
    """<a|b> = dV * sum over points and spin of conj(a) b (Sec. 3.1's psi(V))."""
    return g.dV * np.vdot(a.ravel(), b.ravel())
