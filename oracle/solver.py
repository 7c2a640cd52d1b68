"""Damped-gradient iteration with subspace orthonormalisation (oracle).

Follows Fig. 1 of the paper (steps 1-6), the damped gradient step
(Eq. dampstep), the convergence measure (Eq. convergence), the overlap and
Hamiltonian matrices (Eqs. normmatrix, hammatrix), and the diagonalisation +
orthonormalisation of Sec. 3.3.2-3.3.3.

Readings:
* Eq. dampstep's operator delta/(T + E0) is applied in Fourier space as
  x0 / (E0 + hb2m_q |k|^2) with the bare hbar^2/2m of the species, and
  <h> is the real part of the Rayleigh quotient;
* h is applied twice per iteration: to psi for the gradient step and to the
  stepped phi for the subspace Hamiltonian (Fig. 1 step 2);
* the combined update of Sec. 3.3.3 is taken in its exact generalised
  Rayleigh-Ritz form: I = L L^H (Cholesky), C = L^-H, H' = C^H H C = Z Lam Z^H
  with ascending eigenvalues, psi = phi (C Z).  This is the same I^3 + I^2 V
  cost and the same fixed point as the paper's C^T Z^H product;
* Delta-eps (Eq. convergence) uses the identity <h^2> - <h>^2 = ||h psi -
  <h> psi||^2 for normalised psi and sums over both species;
* initial orthonormalisation is Loewdin's C = I^(-1/2) (Eqs. Loewedin,
  orthmatvec).

State arrays are [state][spin][z][y][x] complex128.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np
import scipy.fft as sfft

from .grid import _WORKERS, Grid
from .physics import (Densities, MeanField, apply_h, densities, energy,
                      mean_field)


def _rows(x: np.ndarray) -> np.ndarray:
    """[state][spinor components] view (also for an empty species)."""
    return x.reshape(x.shape[0], int(np.prod(x.shape[1:])))


def overlap(a: np.ndarray, b: np.ndarray, g: Grid) -> np.ndarray:
    """M[alpha, beta] = <a_alpha | b_beta> (Eqs. normmatrix/hammatrix)."""
    af = _rows(a)
    bf = _rows(b)
    return g.dV * (af.conj() @ bf.T)


def combine(phi: np.ndarray, U: np.ndarray) -> np.ndarray:
    """psi_beta = sum_alpha phi_alpha U[alpha, beta] (Sec. 3.3.3, step 3e)."""
    pf = _rows(phi)
    return (U.T @ pf).reshape((U.shape[1],) + phi.shape[1:])


def loewdin(phi: np.ndarray, g: Grid) -> np.ndarray:
    """Loewdin orthonormalisation: C = I^(-1/2) = X Lam^(-1/2) X^H."""
    I = overlap(phi, phi, g)
    I = 0.5 * (I + I.conj().T)
    lam, X = np.linalg.eigh(I)
    C = (X * lam ** -0.5) @ X.conj().T
    return combine(phi, C)


def rayleigh_ritz(I: np.ndarray, H: np.ndarray):
    """U with U^H I U = 1 and U^H H U = diag(lam), lam ascending.

    Cholesky of the overlap, then the Hermitian eigenproblem of
    H' = L^-1 H L^-H (Sec. 3.3.2 diagonalisation + orthonormalisation).
    """
    I = 0.5 * (I + I.conj().T)
    H = 0.5 * (H + H.conj().T)
    L = np.linalg.cholesky(I)
    Linv = np.linalg.inv(L)
    Hp = Linv @ H @ Linv.conj().T
    Hp = 0.5 * (Hp + Hp.conj().T)
    lam, Z = np.linalg.eigh(Hp)
    return Linv.conj().T @ Z, lam


def damping(r: np.ndarray, g: Grid, hb2m: float, x0: float, e0: float
            ) -> np.ndarray:
    """x0 * F^-1[ F(r) / (E0 + hb2m |k|^2) ] per spinor component (Eq. dampstep)."""
    fk = sfft.fftn(r, axes=(-3, -2, -1), workers=_WORKERS)
    fk *= x0 / (e0 + hb2m * g.k2())
    return sfft.ifftn(fk, axes=(-3, -2, -1), workers=_WORKERS)


def rayleigh_and_residual(psi: np.ndarray, hpsi: np.ndarray, g: Grid):
    """eps_a = Re <psi_a|h psi_a>, r_a = h psi_a - eps_a psi_a, ||r_a||^2."""
    pf = _rows(psi)
    hf = _rows(hpsi)
    eps = g.dV * np.einsum("av,av->a", pf.conj(), hf).real
    r = hpsi - eps[:, None, None, None, None] * psi
    rf = _rows(r)
    r2 = g.dV * (np.abs(rf) ** 2).sum(axis=1)
    return eps, r, r2


@dataclasses.dataclass
class State:
    """Orthonormal states of both species plus the mean field built from them."""
    g: Grid
    params: Dict[str, float]
    x0: float
    e0: float
    psi: List[np.ndarray]                 # [neutrons, protons]
    dens: Optional[List[Densities]] = None
    mf: Optional[List[MeanField]] = None
    vc: Optional[np.ndarray] = None
    E: Optional[Dict[str, float]] = None

    def update_fields(self) -> None:
        """Fig. 1 steps 4a/4b/5: densities -> mean field -> energy."""
        self.dens = [densities(p, self.g) for p in self.psi]
        mn, mp, vc = mean_field(self.dens[0], self.dens[1], self.g, self.params)
        self.mf, self.vc = [mn, mp], vc
        self.E = energy(self.dens[0], self.dens[1], self.g, self.params, vc)


def initial_state(raw_n: np.ndarray, raw_p: np.ndarray, g: Grid,
                  params: Dict[str, float], x0: float, e0: float) -> State:
    """Fig. 1 step 1: Loewdin-orthonormalised trial states and their mean field."""
    st = State(g, params, x0, e0, [loewdin(raw_n, g), loewdin(raw_p, g)])
    st.update_fields()
    return st


@dataclasses.dataclass
class StepReport:
    de: float                  # Delta-eps of the states entering the step (MeV)
    eps: List[np.ndarray]      # Rayleigh quotients entering the step
    ritz: List[np.ndarray]     # subspace eigenvalues after the step
    E: Dict[str, float]        # energy after the step


def iterate(st: State, self_consistent: bool = True) -> StepReport:
    """One damped-gradient iteration, Fig. 1 steps 2-5, both species.

    With ``self_consistent=False`` the mean field is held fixed (step 4 is
    skipped), which turns the iteration into an eigensolver for a given h.
    """
    g = st.g
    eps_all, r2_all, new_psi, ritz = [], [], [], []
    for q in range(2):
        psi, mf = st.psi[q], st.mf[q]
        if psi.shape[0] == 0:
            eps_all.append(np.zeros(0)); r2_all.append(np.zeros(0))
            new_psi.append(psi); ritz.append(np.zeros(0))
            continue
        hpsi = apply_h(psi, mf, g)
        eps, r, r2 = rayleigh_and_residual(psi, hpsi, g)
        phi = psi - damping(r, g, mf.hb2m, st.x0, st.e0)
        hphi = apply_h(phi, mf, g)
        I = overlap(phi, phi, g)
        H = overlap(phi, hphi, g)
        U, lam = rayleigh_ritz(I, H)
        new_psi.append(combine(phi, U))
        eps_all.append(eps); r2_all.append(r2); ritz.append(lam)
    r2 = np.concatenate(r2_all)
    de = float(np.sqrt(r2.sum() / max(1, r2.size)))
    st.psi = new_psi
    if self_consistent:
        st.update_fields()
    return StepReport(de, eps_all, ritz, dict(st.E or {}))


def residual(st: State) -> float:
    """Delta-eps (Eq. convergence) of the current states with their own h."""
    r2 = []
    for q in range(2):
        if st.psi[q].shape[0] == 0:
            continue
        hpsi = apply_h(st.psi[q], st.mf[q], st.g)
        r2.append(rayleigh_and_residual(st.psi[q], hpsi, st.g)[2])
    r2 = np.concatenate(r2)
    return float(np.sqrt(r2.sum() / max(1, r2.size)))
