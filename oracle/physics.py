"""Densities, Skyrme energy functional, mean field and h*psi (oracle).

Sec. 2.1 gives the densities rho, J, tau (Eqs. rho, curr, tau) and a
schematic Skyrme functional (Eq. Skyrme); Sec. 2.2 states that h is the
kinetic energy plus the Skyrme mean field plus Coulomb, with FFT derivatives
and Coulomb solved in momentum space.

Readings:
* Eq. Skyrme is taken as the standard Skyrme functional in b-coefficient
  form with isospin-coupled terms (the per-species terms of Eq. Skyrme are
  its like-particle part), time-even only, no J^2 tensor terms;
* J is the real part of Eq. curr, i.e. J_k = Im sum psi^dag eps_klm sigma_m
  d_l psi (exactly real for time-reversal symmetric states, Sec. 2.1);
* Coulomb is the direct term of the proton density with the k = 0 mode
  dropped (neutralising electron background, Sec. 1), exchange off;
* h is the exact derivative of the *discrete* functional,
  h psi = (1/dV) dE/dpsi^*, which makes it Hermitian on the grid.

Spinor arrays are [state][spin][z][y][x]; fields are [z][y][x].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Tuple

import numpy as np
import scipy.fft as sfft

from .grid import _WORKERS, Grid, deriv, deriv_real, laplacian_real

# Pauli matrices sigma_x, sigma_y, sigma_z
SIGMA = np.array([[[0, 1], [1, 0]],
                  [[0, -1j], [1j, 0]],
                  [[1, 0], [0, -1]]], dtype=np.complex128)

# Levi-Civita symbol eps[k, l, m]
EPS = np.zeros((3, 3, 3))
for _k, _l, _m in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    EPS[_k, _l, _m] = 1.0
    EPS[_k, _m, _l] = -1.0


@dataclasses.dataclass
class Densities:
    """Local densities of one species (Eqs. rho, curr, tau) + derived fields."""
    rho: np.ndarray          # number density
    tau: np.ndarray          # kinetic density
    J: np.ndarray            # spin-orbit density, [3][z][y][x]
    s: np.ndarray            # spin density (diagnostic), [3][z][y][x]
    j: np.ndarray            # current density (diagnostic), [3][z][y][x]


def densities(psi: np.ndarray, g: Grid, nocc: int = None) -> Densities:
    """rho, tau, J of one species (Eqs. rho, curr, tau).

    Occupations (Sec. 2.1): v^2 = 1 for the first ``nocc`` states and 0 for
    the rest (all states when ``nocc`` is None).  The solver keeps its states
    in ascending order of their subspace eigenvalues, so the first ``nocc``
    are the occupied ones of the aufbau principle.  Derivatives of the states
    carry the grid's twist.
    """
    if nocc is not None:
        psi = psi[:nocc]
    shape = psi.shape[2:]
    rho = np.zeros(shape)
    tau = np.zeros(shape)
    J = np.zeros((3,) + shape)
    s = np.zeros((3,) + shape)
    j = np.zeros((3,) + shape)
    chunk = max(1, int(2 ** 25 // max(1, int(np.prod(psi.shape[1:])))))
    for a0 in range(0, psi.shape[0], chunk):
        p = psi[a0:a0 + chunk]                       # [a][spin][z][y][x]
        rho += (np.abs(p) ** 2).sum(axis=(0, 1))
        for m in range(3):
            sp = np.einsum("asxyz,st,atxyz->xyz", p.conj(), SIGMA[m], p)
            s[m] += sp.real
        for l in range(3):
            dp = deriv(p, g, l)
            tau += (np.abs(dp) ** 2).sum(axis=(0, 1))
            j[l] += (p.conj() * dp).sum(axis=(0, 1)).imag
            for m in range(3):
                z = np.einsum("asxyz,st,atxyz->xyz", p.conj(), SIGMA[m], dp)
                for k in range(3):
                    if EPS[k, l, m] != 0.0:
                        J[k] += EPS[k, l, m] * z.imag
    return Densities(rho, tau, J, s, j)


def average(ds) -> Densities:
    """Twist average of the densities of one species (equal weights): the
    mean field of twist-averaged boundary conditions is built from it."""
    t = len(ds)
    return Densities(*[sum(getattr(d, f) for d in ds) / t
                       for f in ("rho", "tau", "J", "s", "j")])


def skyrme_b(p: Dict[str, float]) -> Dict[str, float]:
    """b-coefficients of the Skyrme functional from t0..t3, x0..x3, W0."""
    t0, t1, t2, t3 = p["t0"], p["t1"], p["t2"], p["t3"]
    x0, x1, x2, x3 = p["x0"], p["x1"], p["x2"], p["x3"]
    return dict(
        b0=t0 * (1 + x0 / 2), b0p=t0 * (0.5 + x0),
        b1=(t1 * (1 + x1 / 2) + t2 * (1 + x2 / 2)) / 4,
        b1p=(t1 * (0.5 + x1) - t2 * (0.5 + x2)) / 4,
        b2=(3 * t1 * (1 + x1 / 2) - t2 * (1 + x2 / 2)) / 8,
        b2p=(3 * t1 * (0.5 + x1) + t2 * (0.5 + x2)) / 8,
        b3=t3 * (1 + x3 / 2) / 4, b3p=t3 * (0.5 + x3) / 4,
        b4=p["W0"] / 2, b4p=p["W0"] / 2,
    )


def coulomb(rho_p: np.ndarray, g: Grid, e2: float) -> np.ndarray:
    """Direct Coulomb potential solved in momentum space (Sec. 2.2).

    V_C(k) = 4 pi e^2 rho_p(k) / |k|^2 for k != 0, and 0 at k = 0.
    """
    k2 = g.k2()
    fk = sfft.fftn(rho_p, workers=_WORKERS)
    with np.errstate(divide="ignore", invalid="ignore"):
        mult = np.where(k2 > 0.0, 4.0 * math.pi * e2 / np.where(k2 > 0, k2, 1.0),
                        0.0)
    return sfft.ifftn(fk * mult, workers=_WORKERS).real


@dataclasses.dataclass
class MeanField:
    """Mean field of one species: h = U - sum D B D + spin-orbit(W)."""
    U: np.ndarray
    B: np.ndarray
    W: np.ndarray            # [3][z][y][x]
    hb2m: float              # bare hbar^2/2m (used by the damping operator)


def _derived(d: Densities, g: Grid) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Laplacian of rho, gradient of rho, divergence of J (real fields)."""
    lap = laplacian_real(d.rho, g)
    grad = np.stack([deriv_real(d.rho, g, m) for m in range(3)])
    divJ = sum(deriv_real(d.J[m], g, m) for m in range(3))
    return lap, grad, divJ


def mean_field(dn: Densities, dp: Densities, g: Grid, p: Dict[str, float]
               ) -> Tuple[MeanField, MeanField, np.ndarray]:
    """U_q, B_q, W_q of both species and the Coulomb potential.

    Exact derivatives of ``energy`` with respect to rho_q, tau_q, J_q.
    The term rho^(alpha-1) sum rho_q^2 is evaluated as
    rho^alpha * (sum rho_q^2 / rho) with rho floored at 1e-30.
    """
    b = skyrme_b(p)
    al = p["alpha"]
    rho = dn.rho + dp.rho
    tau = dn.tau + dp.tau
    lap_n, grad_n, divJ_n = _derived(dn, g)
    lap_p, grad_p, divJ_p = _derived(dp, g)
    lap = lap_n + lap_p
    grad = grad_n + grad_p
    divJ = divJ_n + divJ_p
    rho_safe = np.maximum(rho, 1e-30)
    rho_al = rho_safe ** al
    sum_q2 = dn.rho ** 2 + dp.rho ** 2
    vc = coulomb(dp.rho, g, p["e2"]) if p["e2"] != 0.0 else np.zeros_like(rho)
    out = []
    for q, (d, lap_q, grad_q, divJ_q) in enumerate(
            ((dn, lap_n, grad_n, divJ_n), (dp, lap_p, grad_p, divJ_p))):
        U = (b["b0"] * rho - b["b0p"] * d.rho
             + b["b1"] * tau - b["b1p"] * d.tau
             - b["b2"] * lap + b["b2p"] * lap_q
             - b["b4"] * divJ - b["b4p"] * divJ_q
             + b["b3"] / 3 * (al + 2) * rho_safe ** (al + 1)
             - b["b3p"] / 3 * (al * rho_al * (sum_q2 / rho_safe)
                               + 2 * rho_al * d.rho))
        if q == 1:
            U = U + vc
        hb2m = p["hb2m_n"] if q == 0 else p["hb2m_p"]
        B = hb2m + b["b1"] * rho - b["b1p"] * d.rho
        W = b["b4"] * grad + b["b4p"] * grad_q
        out.append(MeanField(U, B, W, hb2m))
    return out[0], out[1], vc


def energy(dn: Densities, dp: Densities, g: Grid, p: Dict[str, float],
           vc: np.ndarray) -> Dict[str, float]:
    """Total energy: kinetic + Skyrme (Eq. Skyrme, b-form) + Coulomb direct."""
    b = skyrme_b(p)
    al = p["alpha"]
    rho = dn.rho + dp.rho
    tau = dn.tau + dp.tau
    lap_n, _, divJ_n = _derived(dn, g)
    lap_p, _, divJ_p = _derived(dp, g)
    lap = lap_n + lap_p
    divJ = divJ_n + divJ_p
    rho_safe = np.maximum(rho, 1e-30)
    kin = p["hb2m_n"] * dn.tau + p["hb2m_p"] * dp.tau
    e_rho = b["b0"] / 2 * rho ** 2 - b["b0p"] / 2 * (dn.rho ** 2 + dp.rho ** 2)
    e_3 = (b["b3"] / 3 * rho_safe ** (al + 2)
           - b["b3p"] / 3 * rho_safe ** al * (dn.rho ** 2 + dp.rho ** 2))
    e_tau = b["b1"] * rho * tau - b["b1p"] * (dn.rho * dn.tau + dp.rho * dp.tau)
    e_lap = -b["b2"] / 2 * rho * lap + b["b2p"] / 2 * (dn.rho * lap_n
                                                        + dp.rho * lap_p)
    e_so = -b["b4"] * rho * divJ - b["b4p"] * (dn.rho * divJ_n + dp.rho * divJ_p)
    e_c = 0.5 * dp.rho * vc
    parts = dict(kin=kin, rho=e_rho, rho3=e_3, tau=e_tau, lap=e_lap, so=e_so,
                 coul=e_c)
    out = {k: float(g.dV * v.sum()) for k, v in parts.items()}
    out["total"] = float(sum(out[k] for k in parts))
    return out


def so_matrix(W: np.ndarray, m: int) -> np.ndarray:
    """A_m = (W x sigma)_m as a 2x2 matrix field [2][2][z][y][x]."""
    A = np.zeros((2, 2) + W.shape[1:], dtype=np.complex128)
    for k in range(3):
        for l in range(3):
            if EPS[m, k, l] != 0.0:
                A += EPS[m, k, l] * W[k][None, None] * SIGMA[l][:, :, None, None,
                                                                 None]
    return A


def _mat_spinor(A: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(A psi)_s = sum_t A_st psi_t for spinor arrays [a][spin][z][y][x]."""
    return np.einsum("stxyz,atxyz->asxyz", A, psi)


def apply_h(psi: np.ndarray, mf: MeanField, g: Grid) -> np.ndarray:
    """h psi = U psi - sum_m D_m(B D_m psi)
               + (i/2) sum_m [A_m D_m psi + D_m(A_m psi)],  A_m = (W x sigma)_m.

    This is (1/dV) dE/dpsi^* of the discrete functional in ``energy``.
    """
    out = mf.U[None, None] * psi
    for m in range(3):
        A = so_matrix(mf.W, m)
        dpsi = deriv(psi, g, m)
        out -= deriv(mf.B[None, None] * dpsi, g, m)
        out += 0.5j * (_mat_spinor(A, dpsi) + deriv(_mat_spinor(A, psi), g, m))
    return out
