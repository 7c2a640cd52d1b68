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

Options beyond that reading, each off by default:
* occupations (Sec. 2.1: v^2 in {0, 1}, more wave functions than particles
  allowed): a species may carry extra states; the first N_q states in
  ascending subspace-eigenvalue order are occupied (aufbau) and only they
  enter the densities and Delta-eps;
* twist-averaged boundary conditions (Sec. 1): a set of twists theta; every
  twist carries its own states of both species, the derivatives of those
  states carry i theta/L, and all twists share one mean field built from
  the twist-averaged densities;
* the paper-literal combined update (Sec. 3.3.3): Z from the eigenvectors
  of H alone (step 3b), C = I^-1/2 from I alone (step 3c), combined as
  psi = phi Z C (step 3d), an approximation whose error vanishes with
  I - 1 at convergence when Z is taken in the gauge closest to the
  identity;
* one h application per iteration (Sec. 3.4 keeps h psi in hampsi for
  step 3a): h psi of the new states is taken as (h phi) U, the previous
  mean field's Hamiltonian on the new states, so the next gradient step uses
  a Hamiltonian one iteration behind.

State arrays are [state][spin][z][y][x] complex128.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.fft as sfft

from .grid import _WORKERS, Grid
from .physics import (Densities, MeanField, apply_h, average, densities,
                      energy, mean_field)


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


# Eigenvalues of H closer than this (MeV) form one cluster of the gauge of Z
PAPER_CLUSTER_TOL = 1e-3


def paper_gauge(lam: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """Eigenvectors Z of H (columns, ascending lam) in the gauge closest to
    the identity.  Within each cluster of eigenvalues (consecutive gaps below
    PAPER_CLUSTER_TOL) the eigenvectors may be rotated freely; the rotation Q
    that makes the cluster's diagonal block Z_cc Q Hermitian positive
    semi-definite (the polar factor, Q = V W^H for Z_cc = W S V^H) is the one
    closest to the identity.  A cluster of one state reduces to the phase
    that makes Z_bb real and positive."""
    Z = Z.copy()
    m = lam.size
    a = 0
    while a < m:
        b = a + 1
        while b < m and lam[b] - lam[b - 1] < PAPER_CLUSTER_TOL:
            b += 1
        W, _, Vh = np.linalg.svd(Z[a:b, a:b])
        Z[:, a:b] = Z[:, a:b] @ (Vh.conj().T @ W.conj().T)
        a = b
    return Z


def paper_update(I: np.ndarray, H: np.ndarray):
    """The paper-literal combined update of Sec. 3.3.3: U = Z C.

    Step 3b diagonalises H alone (H Z = Z Lam, ascending), step 3c takes
    Loewdin's C = I^-1/2 from I alone, and step 3d combines them into one
    transform applied to phi.  The paper writes the update as the product
    C^T Z^H acting on the column of states; with the eigenvectors in the
    columns of Z (psi_a = sum_b Z_ba phi_b diagonalises H) that is
    psi = phi Z C.  C was computed for phi, not for phi Z, which is the small
    error the paper notes.  It vanishes with I - 1 only if Z tends to the
    identity as phi becomes diagonal, so Z is taken in the gauge closest to
    the identity (paper_gauge): with an arbitrary rotation inside the
    (Kramers-)degenerate pairs of eigenvalues the orthonormality error of
    psi = phi Z C does not vanish and the iteration levels off.
    """
    I = 0.5 * (I + I.conj().T)
    H = 0.5 * (H + H.conj().T)
    lam, Z = np.linalg.eigh(H)
    Z = paper_gauge(lam, Z)
    w, X = np.linalg.eigh(I)
    C = (X * w ** -0.5) @ X.conj().T
    return Z @ C, lam


def damping(r: np.ndarray, g: Grid, hb2m: float, x0: float, e0: float
            ) -> np.ndarray:
    """x0 * F^-1[ F(r) / (E0 + hb2m |k|^2) ] per spinor component (Eq. dampstep).

    |k|^2 is the kinetic spectrum of a state, |k + theta/L|^2 under a twist.
    """
    fk = sfft.fftn(r, axes=(-3, -2, -1), workers=_WORKERS)
    fk *= x0 / (e0 + hb2m * g.k2_psi())
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
    """Orthonormal states plus the mean field built from them.

    ``psi`` holds one array per state set: set 2 t + q is species q (0 = n,
    1 = p) under twist t.  Without twists there are two sets.  ``nocc``
    gives the occupied states per species (None: every state occupied);
    ``twists`` the Bloch phases (None: one untwisted set per species).
    """
    g: Grid
    params: Dict[str, float]
    x0: float
    e0: float
    psi: List[np.ndarray]
    dens: Optional[List[Densities]] = None
    mf: Optional[List[MeanField]] = None
    vc: Optional[np.ndarray] = None
    E: Optional[Dict[str, float]] = None
    nocc: Optional[Tuple[int, int]] = None
    twists: Optional[Sequence[Sequence[float]]] = None
    rr: str = "exact"                       # "exact" | "paper"
    one_h: bool = False
    hpsi_lag: Optional[List[np.ndarray]] = None

    def ntwist(self) -> int:
        return 1 if self.twists is None else len(self.twists)

    def grid_of(self, s: int) -> Grid:
        """Grid (with the twist) of state set s."""
        if self.twists is None:
            return self.g
        return self.g.with_twist(self.twists[s // 2])

    def occ(self, s: int) -> int:
        q = s % 2
        return self.psi[s].shape[0] if self.nocc is None else self.nocc[q]

    def update_fields(self) -> None:
        """Fig. 1 steps 4a/4b/5: densities -> mean field -> energy.

        Each species' densities are summed over its occupied states and
        averaged over the twists."""
        t = self.ntwist()
        dq = []
        for q in range(2):
            ds = [densities(self.psi[2 * k + q], self.grid_of(2 * k + q),
                            self.occ(2 * k + q)) for k in range(t)]
            dq.append(ds[0] if t == 1 else average(ds))
        self.dens = dq
        mn, mp, vc = mean_field(self.dens[0], self.dens[1], self.g, self.params)
        self.mf, self.vc = [mn, mp], vc
        self.E = energy(self.dens[0], self.dens[1], self.g, self.params, vc)


def initial_state(raw_n: np.ndarray, raw_p: np.ndarray, g: Grid,
                  params: Dict[str, float], x0: float, e0: float,
                  nocc: Optional[Tuple[int, int]] = None,
                  twists: Optional[Sequence[Sequence[float]]] = None,
                  rr: str = "exact", one_h: bool = False) -> State:
    """Fig. 1 step 1: Loewdin-orthonormalised trial states and their mean field.

    With twists every twist starts from the same trial states."""
    t = 1 if twists is None else len(twists)
    psi = []
    for _ in range(t):
        psi += [loewdin(raw_n, g), loewdin(raw_p, g)]
    st = State(g, params, x0, e0, psi, nocc=nocc, twists=twists, rr=rr,
               one_h=one_h)
    st.update_fields()
    return st


@dataclasses.dataclass
class StepReport:
    de: float                  # Delta-eps of the states entering the step (MeV)
    eps: List[np.ndarray]      # Rayleigh quotients entering the step, per set
    ritz: List[np.ndarray]     # subspace eigenvalues after the step, per set
    E: Dict[str, float]        # energy after the step


def iterate(st: State, self_consistent: bool = True) -> StepReport:
    """One damped-gradient iteration, Fig. 1 steps 2-5, every state set.

    With ``self_consistent=False`` the mean field is held fixed (step 4 is
    skipped), which turns the iteration into an eigensolver for a given h.
    Delta-eps runs over the occupied states of every set.
    """
    eps_all, r2_occ, new_psi, ritz, new_lag = [], [], [], [], []
    for s, psi in enumerate(st.psi):
        g, mf = st.grid_of(s), st.mf[s % 2]
        if psi.shape[0] == 0:
            eps_all.append(np.zeros(0)); new_psi.append(psi)
            ritz.append(np.zeros(0)); new_lag.append(psi)
            continue
        if st.one_h and st.hpsi_lag is not None:
            hpsi = st.hpsi_lag[s]        # h of the previous mean field
        else:
            hpsi = apply_h(psi, mf, g)
        eps, r, r2 = rayleigh_and_residual(psi, hpsi, g)
        phi = psi - damping(r, g, mf.hb2m, st.x0, st.e0)
        hphi = apply_h(phi, mf, g)
        I = overlap(phi, phi, g)
        H = overlap(phi, hphi, g)
        if st.rr == "paper":
            U, lam = paper_update(I, H)
        else:
            U, lam = rayleigh_ritz(I, H)
        new_psi.append(combine(phi, U))
        new_lag.append(combine(hphi, U) if st.one_h else None)
        eps_all.append(eps); r2_occ.append(r2[:st.occ(s)]); ritz.append(lam)
    r2 = np.concatenate(r2_occ) if r2_occ else np.zeros(0)
    de = float(np.sqrt(r2.sum() / max(1, r2.size)))
    st.psi = new_psi
    st.hpsi_lag = new_lag if st.one_h else None
    if self_consistent:
        st.update_fields()
    return StepReport(de, eps_all, ritz, dict(st.E or {}))


def residual(st: State) -> float:
    """Delta-eps (Eq. convergence) of the current occupied states with their
    own self-consistent h."""
    r2 = []
    for s, psi in enumerate(st.psi):
        if psi.shape[0] == 0:
            continue
        g = st.grid_of(s)
        hpsi = apply_h(psi, st.mf[s % 2], g)
        r2.append(rayleigh_and_residual(psi, hpsi, g)[2][:st.occ(s)])
    r2 = np.concatenate(r2)
    return float(np.sqrt(r2.sum() / max(1, r2.size)))
