"""Seeded synthetic workloads for the damped-gradient Skyrme solver.

This module only *describes and draws inputs*: box geometry, the Skyrme
parameter set, and the raw (non-orthonormal) trial spinors.  It contains none
of the solver's arithmetic (no derivatives, densities, mean fields,
orthonormalisation or damping); both the FP64 oracle and the HIP library take
what this module produces and do all of that themselves.

Trial states follow the paper's initialisation for periodic systems
(Sec. 2.2: plane waves for periodic boxes), modulated by a seed-drawn density
perturbation (slab or rod shaped, the pasta geometries named in Sec. 1) and,
for the small box, complex Gaussian noise.

Layout of every state array: ``[state][spin][z][y][x]`` complex, x fastest,
spin 0 = up, spin 1 = down.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np

# SLy4 (Chabanat et al., Nucl. Phys. A 635 (1998) 231; literature values).
# Units: t0 MeV fm^3, t1/t2 MeV fm^5, t3 MeV fm^(3+3 alpha), W0 MeV fm^5,
# hbar^2/2m MeV fm^2, e^2 MeV fm.
SLY4: Dict[str, float] = dict(
    t0=-2488.91, t1=486.82, t2=-546.39, t3=13777.0,
    x0=0.834, x1=-0.344, x2=-1.0, x3=1.354,
    alpha=1.0 / 6.0, W0=123.0,
    hb2m_n=20.73553, hb2m_p=20.73553, e2=1.439964,
)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic box: geometry, particle numbers, force and trial state."""
    name: str
    n: int                     # grid points per axis (cubic box)
    dx: float                  # spacing in fm (same on every axis)
    n_neutrons: int
    n_protons: int
    init: str                  # "plain" | "slab" | "rod" | "random"
    seed: int
    amp: float = 0.3           # perturbation amplitude of the density shape f
    noise: float = 0.0         # amplitude of the complex Gaussian noise
    damp_x0: float = 0.45      # damping step delta of the gradient step
    damp_e0: float = 100.0     # damping energy E0 in MeV
    force: Tuple[Tuple[str, float], ...] = tuple(SLY4.items())
    extra_n: int = 0           # unoccupied (v^2 = 0) states carried beyond the
    extra_p: int = 0           # particles of each species (Sec. 2.1)

    @property
    def params(self) -> Dict[str, float]:
        return dict(self.force)

    @property
    def states_n(self) -> int:
        return self.n_neutrons + self.extra_n

    @property
    def states_p(self) -> int:
        return self.n_protons + self.extra_p

    @property
    def box(self) -> float:
        return self.n * self.dx

    @property
    def n_states(self) -> int:
        return self.n_neutrons + self.n_protons


# The synthetic workloads.  Densities follow the pasta regime of the paper's
# experiments (Sec. 5.1: ~1 fm spacing, 0.02-0.14 fm^-3 mean density) at the
# sizes the solver is measured on.
WORKLOADS: Dict[str, Workload] = {
    # 16 fm box, 8 n + 8 p, lowest plane waves plus noise 0.1, 200 iterations.
    "fermi16": Workload("fermi16", 16, 1.0, 8, 8, "plain", seed=0, amp=0.0,
                        noise=0.1),
    # 32 fm pasta box, 640 n + 160 p, slab perturbation along z.
    "slab32": Workload("slab32", 32, 1.0, 640, 160, "slab", seed=1),
    # 48 fm pasta box, 1600 n + 400 p, rod perturbation (cylinders along z).
    "rod48": Workload("rod48", 48, 1.0, 1600, 400, "rod", seed=2),
    # Saturation-density boxes (closed plane-wave shells, weak slab, small
    # noise): uniform matter there is stable, so the iteration converges
    # (Delta-eps 1e-6 and below).  24 fm, 1030 n + 1030 p (shells
    # |n|^2 <= 25), 0.149 fm^-3, on a 24^3 grid at 1 fm or a 48^3 grid at
    # 0.5 fm; 8 fm, 38 n + 38 p, 0.148 fm^-3.
    "sat24": Workload("sat24", 24, 1.0, 1030, 1030, "slab", seed=4, amp=0.1, noise=0.02),
    "sat48": Workload("sat48", 48, 0.5, 1030, 1030, "slab", seed=4, amp=0.1, noise=0.02),
    "sat8": Workload("sat8", 8, 1.0, 38, 38, "slab", seed=22, amp=0.1, noise=0.02),
}


def plane_wave_labels(n: int, count: int) -> np.ndarray:
    """First ``count`` plane-wave spinor labels ``(nx, ny, nz, spin)``.

    Order: |n|^2 ascending, then nx, ny, nz ascending, spin up before down.
    Integer wave numbers run over the FFT range -n/2 .. n/2-1 on each axis.
    """
    half = n // 2
    rng = np.arange(-half, half)
    nz, ny, nx = np.meshgrid(rng, rng, rng, indexing="ij")
    lab = np.stack([nx.ravel(), ny.ravel(), nz.ravel()], axis=1)
    n2 = (lab ** 2).sum(axis=1)
    order = np.lexsort((lab[:, 2], lab[:, 1], lab[:, 0], n2))
    lab = lab[order]
    need = (count + 1) // 2
    if need > lab.shape[0]:
        raise ValueError("more states than plane waves on the grid")
    out = np.empty((2 * need, 4), dtype=np.int64)
    out[0::2, :3] = lab[:need]
    out[1::2, :3] = lab[:need]
    out[0::2, 3] = 0
    out[1::2, 3] = 1
    return out[:count]


def _shape_field(w: Workload, rng: np.random.Generator) -> np.ndarray:
    """Density shape f(r) >= 0.05 on the grid, indexed [z][y][x]."""
    n = w.n
    t = 2.0 * math.pi * np.arange(n) / n          # 2 pi x / L on the grid
    f = np.ones((n, n, n))
    if w.init == "plain":
        return f
    if w.init == "slab":
        ph = rng.uniform(0.0, 2.0 * math.pi)
        f = f + w.amp * np.cos(t + ph)[:, None, None]
    elif w.init == "rod":
        phx, phy = rng.uniform(0.0, 2.0 * math.pi, size=2)
        f = f + 0.5 * w.amp * (np.cos(t + phx)[None, None, :]
                               + np.cos(t + phy)[None, :, None])
    elif w.init == "random":
        # smooth random field from the |m| <= 2 Fourier modes, max-normalised
        acc = np.zeros((n, n, n))
        zz, yy, xx = np.meshgrid(t, t, t, indexing="ij")
        for mz in range(-2, 3):
            for my in range(-2, 3):
                for mx in range(-2, 3):
                    m2 = mx * mx + my * my + mz * mz
                    if m2 == 0 or m2 > 4:
                        continue
                    a, ph = rng.standard_normal(), rng.uniform(0, 2 * math.pi)
                    acc += a * np.cos(mx * xx + my * yy + mz * zz + ph)
        f = f + w.amp * acc / np.abs(acc).max()
    else:
        raise ValueError(f"unknown init kind {w.init!r}")
    return np.maximum(f, 0.05)


def raw_states(w: Workload) -> Tuple[np.ndarray, np.ndarray]:
    """Raw trial spinors (neutrons, protons), complex128, not orthonormal:
    the particles' states followed by the extra states of each species.

    psi[alpha, s] = sqrt(f) * exp(i k.r) delta_{s, s_alpha} / sqrt(L^3)
                    (+ noise * (g1 + i g2) / sqrt(2) / sqrt(L^3)),
    with k = 2 pi n / L.  Random numbers come from numpy's PCG64 seeded with
    ``w.seed``: first the shape phases, then the noise, neutrons before
    protons, each drawn in array order with the real part before the
    imaginary part.
    """
    rng = np.random.default_rng(w.seed)
    n = w.n
    sqrt_f = np.sqrt(_shape_field(w, rng))
    norm = 1.0 / math.sqrt(w.box ** 3)
    phase1d = np.exp(2j * math.pi * np.outer(np.arange(-(n // 2), n // 2),
                                             np.arange(n)) / n)
    out = []
    for count in (w.states_n, w.states_p):
        lab = plane_wave_labels(n, count)
        psi = np.zeros((count, 2, n, n, n), dtype=np.complex128)
        for a, (kx, ky, kz, s) in enumerate(lab):
            ex = phase1d[kx + n // 2]
            ey = phase1d[ky + n // 2]
            ez = phase1d[kz + n // 2]
            psi[a, s] = (ez[:, None, None] * ey[None, :, None]
                         * ex[None, None, :]) * (sqrt_f * norm)
        if w.noise > 0.0:
            g = rng.standard_normal((count, 2, n, n, n, 2))
            psi += (w.noise * norm / math.sqrt(2.0)) * (g[..., 0] + 1j * g[..., 1])
        out.append(psi)
    return out[0], out[1]


def small_workload(name: str, n: int, n_neutrons: int, n_protons: int,
                   init: str = "plain", seed: int = 7, noise: float = 0.1,
                   amp: float = 0.3, dx: float = 1.0, extra_n: int = 0,
                   extra_p: int = 0) -> Workload:
    """A reduced box for fast tests (same force and damping as the others)."""
    return Workload(name, n, dx, n_neutrons, n_protons, init, seed=seed,
                    amp=amp if init != "plain" else 0.0, noise=noise,
                    extra_n=extra_n, extra_p=extra_p)


def special_twists(k: int = 2) -> List[Tuple[float, float, float]]:
    """A k x k x k grid of Bloch phases theta_m = pi (2 j + 1 - k) / k,
    j = 0..k-1 per axis, symmetric about zero (k = 2: the eight corners
    (+-pi/2, +-pi/2, +-pi/2)): the twists of a twist-averaged box."""
    th = [math.pi * (2 * j + 1 - k) / k for j in range(k)]
    return [(tx, ty, tz) for tz in th for ty in th for tx in th]


def batch_workloads(count: int = 64, seed: int = 3) -> List[Workload]:
    """Independent uneven boxes: grid from {16, 24, 32}^3 at 1 fm spacing,
    mean density uniform in [0.02, 0.06] fm^-3, nucleon number
    A = round(density * L^3) clamped to [64, 512], proton fraction uniform in
    [0.1, 0.5] (Z = round(fraction * A), at least 1), initial shape slab, rod
    or random with equal odds, a seed of its own per box.  All draws come
    from numpy's PCG64 seeded with ``seed``, box by box in the order grid,
    density, fraction, shape, box seed."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice([16, 24, 32]))
        rho = float(rng.uniform(0.02, 0.06))
        frac = float(rng.uniform(0.1, 0.5))
        init = str(rng.choice(["slab", "rod", "random"]))
        bseed = int(rng.integers(0, 2 ** 31 - 1))
        a = int(min(512, max(64, round(rho * n ** 3))))
        z = max(1, int(round(frac * a)))
        out.append(Workload(f"b{i:02d}_{n}_{a - z}n{z}p", n, 1.0, a - z, z, init, seed=bseed,
                            noise=0.02))
    return out
