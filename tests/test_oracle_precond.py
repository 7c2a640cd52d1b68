"""Pins of the learned-damping oracle (oracle/precond.py).

Checked against things other than the oracle itself: exhaustive nearest-
bfloat16 search, central finite differences of the loss, Parseval's
identity, the plain damping routine (all gains 1), the closed-form Newton
gain of a free plane-wave residual, and numpy's least-squares solver.
"""
import math

import numpy as np
import pytest

from oracle import Grid
from oracle import physics as ph
from oracle import precond as pc
from oracle import solver as so


def _nearest_bf16(x: float) -> float:
    """Nearest bfloat16 by search over the neighbours of x (ties to even)."""
    x32 = np.float32(x)
    bits = int(np.array([x32]).view(np.uint32)[0])
    lo = bits & 0xFFFF0000
    cands = [lo, lo + 0x10000]
    vals = [float(np.array([c], dtype=np.uint32).view(np.float32)[0]) for c in cands]
    d = [abs(v - float(x32)) for v in vals]
    if d[0] < d[1]:
        return vals[0]
    if d[1] < d[0]:
        return vals[1]
    return vals[0] if ((cands[0] >> 16) & 1) == 0 else vals[1]


def test_bf16_round_matches_nearest_search():
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 8, 2000),
                         [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8,
                          1.0 + 2 ** -8 + 2 ** -20, 0.0, 3.0e38]]).astype(np.float32)
    got = pc.bf16_round(xs)
    want = np.array([_nearest_bf16(float(v)) for v in xs])
    assert np.array_equal(got, want)
    # ties go to the even neighbour
    assert got[-7 + 1] == 1.0 and got[-7 + 2] == 1.0 + 2 ** -6


def _rows(rng, B):
    rows = np.zeros((B, 6))
    rows[:, 0] = rng.uniform(0, 1, B)
    rows[:, 1] = rng.uniform(-2, 0.5, B)
    rows[:, 2] = rng.uniform(-1, 1, B)
    rows[:, 3] = rng.uniform(0, 6, B)
    rows[:, 4] = rng.uniform(0, 4, B)
    rows[:, 5] = rng.uniform(0, 1, B)
    return rows


def _params(rng):
    P = pc.init_params(7).astype(np.float64)
    P += 0.05 * rng.standard_normal(P.shape)   # away from the initial symmetric biases
    return P.astype(np.float32)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(11)
    rows = _rows(rng, 37)
    P = _params(rng)
    L, G = pc.loss_and_grad(P, rows)
    Pr = pc.bf16_round(P)
    assert L == pytest.approx(pc.loss(Pr, rows), rel=1e-14)
    # every block of the layout: W1, b1, W2, b2, W3, b3, W4, b4
    off = np.cumsum([0, 512, 128, 16384, 128, 16384, 128, 128])
    idx = []
    for k in range(7):
        idx += list(rng.integers(off[k], off[k + 1], 6))
    idx.append(pc.NPAR - 1)
    h = 1e-6
    for i in idx:
        e = np.zeros(pc.NPAR)
        e[i] = h
        fd = (pc.loss(Pr + e, rows) - pc.loss(Pr - e, rows)) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * (1e-3 + abs(G).max()), (i, fd, G[i])


def test_adam_descends():
    rng = np.random.default_rng(12)
    rows = _rows(rng, 64)
    P = _params(rng).astype(np.float64)
    M = np.zeros_like(P)
    V = np.zeros_like(P)
    L0, _ = pc.loss_and_grad(P, rows)
    for step in range(1, 61):
        _, G = pc.loss_and_grad(P, rows)
        P, M, V = pc.adam(P, G, M, V, step, 3e-3)
    L1, _ = pc.loss_and_grad(P, rows)
    assert L1 < 0.5 * L0


def test_initial_gain_is_one():
    P = pc.init_params(0)
    p = pc.unpack(P)
    assert pc.gains_of(np.array([p["b4"]]))[0] == pytest.approx(1.0, rel=1e-6)
    rows = _rows(np.random.default_rng(1), 50)
    g = pc.gains_of(pc.forward(pc.bf16_round(P), rows)[0])
    assert np.all(np.abs(g - 1.0) < 0.2)


@pytest.mark.parametrize("n", [8, 16, 24, 48])
def test_shells_match_float_radius_away_from_edges(n):
    """Shell = floor(S |k| / |k|max) capped at S - 1, from the float radius
    wherever the radius is not within 1e-9 of a shell edge."""
    sh = pc.shell_of_modes(n)
    m = pc.mode_indices(n)
    r = np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2) \
        / (math.sqrt(3.0) * n / 2) * pc.S
    ok = np.abs(r - np.round(r)) > 1e-9
    want = np.minimum(np.floor(r), pc.S - 1).astype(int)
    assert np.array_equal(sh[ok], want[ok])
    # exact edges: |k| = |k|max / 8 at m = (n/16)(1, 1, 1) belongs to shell 1
    if n % 16 == 0:
        j = n // 16
        assert sh[j, j, j] == 1
    assert sh[n // 2, n // 2, n // 2] == pc.S - 1 and sh[0, 0, 0] == 0
    assert set(np.unique(sh)) == set(range(pc.S))


def test_shell_power_parseval():
    g = Grid(16, 1.0)
    rng = np.random.default_rng(3)
    r = rng.standard_normal((3, 2, 16, 16, 16)) + 1j * rng.standard_normal((3, 2, 16, 16, 16))
    P = pc.shell_power(r, g)
    want = 16 ** 3 * (np.abs(r) ** 2).reshape(3, -1).sum(axis=1)
    assert np.allclose(P.sum(axis=1), want, rtol=1e-12)


def test_unit_gains_are_the_plain_damping():
    g = Grid(16, 0.9)
    rng = np.random.default_rng(4)
    r = rng.standard_normal((2, 2, 16, 16, 16)) + 1j * rng.standard_normal((2, 2, 16, 16, 16))
    a = pc.gained_damping(r, np.ones((2, pc.S)), g, 20.7, 0.45, 100.0)
    b = so.damping(r, g, 20.7, 0.45, 100.0)
    assert np.allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())
    # the shell-restricted steps add up to the plain step
    d = pc.shell_steps(r, g, 20.7, 0.45, 100.0)
    assert np.allclose(d.sum(axis=0), b, rtol=0, atol=1e-13 * np.abs(b).max())


def _free_field(g, hb2m):
    z = np.zeros((g.n,) * 3)
    return ph.MeanField(U=z.copy(), B=np.full_like(z, hb2m), W=np.zeros((3,) + z.shape),
                        hb2m=hb2m)


def test_target_gain_is_newton_gain_of_free_plane_waves():
    """Free particles, residual of one plane wave per shell: (h - <h>) d_s =
    (T_k - <h>) x0 r_k / (E0 + T_k), so the exact minimiser is
    g_s = (E0 + T_k) / (x0 (T_k - <h>)) in each shell (others get 0)."""
    n, dx, hb2m, x0, e0 = 16, 1.0, 20.7, 0.45, 100.0
    g = Grid(n, dx)
    mf = _free_field(g, hb2m)
    ku = 2 * math.pi / g.L
    zz, yy, xx = np.meshgrid(*(np.arange(n) * dx,) * 3, indexing="ij")
    # psi = k=0 constant plus small plane waves; <h> = Rayleigh quotient
    modes = [(3, 0, 0), (4, 2, 0), (5, 3, 2)]
    psi = np.ones((1, 2, n, n, n), dtype=complex)
    amps = [0.05, 0.03, 0.02]
    for (a, b, c), amp in zip(modes, amps):
        psi[0, 0] += amp * np.exp(1j * ku * (a * xx + b * yy + c * zz))
    psi /= math.sqrt(so.overlap(psi, psi, g)[0, 0].real)
    hpsi = ph.apply_h(psi, mf, g)
    eps, r, _ = so.rayleigh_and_residual(psi, hpsi, g)
    got = pc.target_gains(psi, hpsi, eps, mf, g, hb2m, x0, e0)[0]
    sh = pc.shell_of_modes(n)
    want = np.zeros(pc.S)
    for (a, b, c) in modes:
        T = hb2m * ku ** 2 * (a * a + b * b + c * c)
        want[sh[c, b, a]] = np.clip((e0 + T) / (x0 * (T - eps[0])), 0, pc.GMAX)
    assert np.allclose(got, want, rtol=1e-5, atol=1e-8), (got, want)
    assert np.count_nonzero(want) == 3


def test_target_gains_match_lstsq():
    """General mean field: the normal-equation gains agree with numpy's
    least-squares solution of the stacked real system (ridge is 1e-6)."""
    n = 8
    g = Grid(n, 1.1)
    rng = np.random.default_rng(9)
    mf = ph.MeanField(U=-40 + 10 * rng.standard_normal((n,) * 3),
                      B=20 + rng.uniform(0, 3, (n,) * 3),
                      W=0.5 * rng.standard_normal((3,) + (n,) * 3), hb2m=20.7)
    psi = rng.standard_normal((3, 2, n, n, n)) + 1j * rng.standard_normal((3, 2, n, n, n))
    psi = so.loewdin(psi, g)
    hpsi = ph.apply_h(psi, mf, g)
    eps, r, _ = so.rayleigh_and_residual(psi, hpsi, g)
    got = pc.target_gains(psi, hpsi, eps, mf, g, 20.7, 0.45, 100.0, clip=False)
    d = pc.shell_steps(r, g, 20.7, 0.45, 100.0)
    for a in range(3):
        W = np.stack([(ph.apply_h(d[s, a:a + 1], mf, g) - eps[a] * d[s, a:a + 1]).ravel()
                      for s in range(pc.S)], axis=1)
        A = np.concatenate([W.real, W.imag])
        y = np.concatenate([r[a].ravel().real, r[a].ravel().imag])
        want = np.linalg.lstsq(A, y, rcond=None)[0]
        assert np.allclose(got[a], want, rtol=1e-3, atol=1e-4), (got[a], want)
