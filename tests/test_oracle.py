"""Pins of the FP64 oracle against closed forms, textbook limits and brute force.

Each test checks the oracle against something other than itself: analytic
derivatives of grid harmonics, the textbook Skyrme energy of uniform
symmetric and pure-neutron matter, SLy4's published saturation point,
scipy's generalised eigensolver, finite differences of the energy, symmetry,
and dense diagonalisation of h on an 8^3 grid.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import Grid
from oracle import physics as ph
from oracle import solver as so
from oracle.grid import deriv, deriv_real, laplacian_real
from paper_1610_07522_amd import inputs

SLY4 = inputs.SLY4


def _free(params=None):
    p = dict(params or SLY4)
    for k in ("t0", "t1", "t2", "t3", "W0", "e2"):
        p[k] = 0.0
    return p


def _plane_states(g, count, rng=None, noise=0.0):
    w = inputs.Workload("t", g.n, g.dx, count, 0, "plain", seed=3, amp=0.0,
                        noise=noise)
    return inputs.raw_states(w)[0]


# ---------------------------------------------------------------- derivatives
@pytest.mark.parametrize("n", [8, 12, 16, 24])
def test_derivative_of_grid_harmonics(n):
    """T1: D e^{ikx} = ik e^{ikx} (Nyquist kept); D_real cos = -k sin."""
    g = Grid(n, 0.8)
    x = np.arange(n) * g.dx
    for m in range(-n // 2, n // 2):
        k = 2 * math.pi * m / g.L
        for axis in range(3):
            shape = [1, 1, 1]
            shape[2 - axis] = n
            f = np.broadcast_to(np.exp(1j * k * x).reshape(shape), (n, n, n))
            d = deriv(f, g, axis)
            np.testing.assert_allclose(d, 1j * k * f, atol=1e-12 * (1 + abs(k)))
            if abs(m) < n // 2:
                c = np.cos(k * x).reshape(shape) * np.ones((n, n, n))
                dr = deriv_real(c, g, axis)
                np.testing.assert_allclose(dr, -k * np.sin(k * x).reshape(shape)
                                           * np.ones((n, n, n)), atol=1e-12)
    # Nyquist of a real field is dropped: the result stays real and is zero
    c = np.cos(math.pi * x / g.dx).reshape(1, 1, n) * np.ones((n, n, n))
    assert np.abs(deriv_real(c, g, 0)).max() < 1e-12
    # Laplacian keeps it: -(pi/dx)^2 cos
    np.testing.assert_allclose(laplacian_real(c, g), -(math.pi / g.dx) ** 2 * c,
                               atol=1e-10)


def test_parseval():
    """T2: sum |f|^2 = n^-3 sum |F f|^2 for the FFT convention used."""
    rng = np.random.default_rng(0)
    f = rng.standard_normal((8, 8, 8)) + 1j * rng.standard_normal((8, 8, 8))
    F = np.fft.fftn(f)
    assert abs((abs(f) ** 2).sum() - (abs(F) ** 2).sum() / 512) < 1e-12 * 512


# ---------------------------------------------------------------- operators
def _random_fields(g, rng, w_scale=1.0):
    """Smooth non-uniform U, B > 0, W built from a few random Fourier modes."""
    n = g.n
    t = 2 * math.pi * np.arange(n) / n
    zz, yy, xx = np.meshgrid(t, t, t, indexing="ij")

    def smooth():
        f = np.zeros((n, n, n))
        for _ in range(4):
            m = rng.integers(-2, 3, size=3)
            f += rng.standard_normal() * np.cos(m[0] * xx + m[1] * yy
                                                + m[2] * zz + rng.uniform(0, 6))
        return f
    U = -40 + 10 * smooth()
    B = 20 + 3 * smooth()
    W = w_scale * np.stack([smooth() for _ in range(3)])
    return ph.MeanField(U, B, W, 20.0)


def test_h_hermitian():
    """T3: <a|h b> = conj(<b|h a>) with U, B and spin-orbit all non-uniform."""
    rng = np.random.default_rng(1)
    g = Grid(12, 1.0)
    mf = _random_fields(g, rng)
    a = rng.standard_normal((3, 2, 12, 12, 12)) + 1j * rng.standard_normal(
        (3, 2, 12, 12, 12))
    ha = ph.apply_h(a, mf, g)
    M = so.overlap(a, ha, g)
    np.testing.assert_allclose(M, M.conj().T, rtol=0, atol=1e-12 * abs(M).max())


def test_h_on_plane_wave_constant_fields():
    """h e^{ik.r} chi = (U + B k^2) e^{ik.r} chi - k.(W x sigma) e^{ik.r} chi
    for constant U, B, W (closed form of the kinetic and spin-orbit terms)."""
    g = Grid(8, 1.0)
    n = g.n
    U0, B0, W0 = -30.0, 18.0, np.array([0.7, -1.3, 2.1])
    mf = ph.MeanField(np.full((n, n, n), U0), np.full((n, n, n), B0),
                      W0[:, None, None, None] * np.ones((3, n, n, n)), 18.0)
    r = np.arange(n) * g.dx
    zz, yy, xx = np.meshgrid(r, r, r, indexing="ij")
    sig = ph.SIGMA
    for m in [(1, 0, 0), (0, -2, 1), (3, 1, -4)]:
        k = 2 * math.pi * np.array(m) / g.L
        pw = np.exp(1j * (k[0] * xx + k[1] * yy + k[2] * zz))
        chi = np.array([0.6, 0.8j])
        psi = (chi[:, None, None, None] * pw)[None]
        hpsi = ph.apply_h(psi, mf, g)
        # (W x sigma)_m k_m = sum eps_mab W_a sigma_b k_m
        so_mat = sum(np.cross(W0, np.eye(3)[b])[mm] * k[mm] * sig[b]
                     for mm in range(3) for b in range(3))
        # so_mat = sum_m k_m (W x sigma)_m with (W x sigma)_m = eps_mab W_a sig_b
        M = (U0 + B0 * k @ k) * np.eye(2) - so_mat
        expect = (M @ chi)[:, None, None, None] * pw
        np.testing.assert_allclose(hpsi[0], expect, atol=1e-11)


def test_h_variable_effective_mass():
    """-d/dz(B(z) d/dz) on e^{ikz} with B = b0 + b1 cos(qz): closed form."""
    g = Grid(16, 1.0)
    n = g.n
    z = np.arange(n) * g.dx
    k = 2 * math.pi * 2 / g.L
    q = 2 * math.pi * 1 / g.L
    b0, b1 = 20.0, 3.0
    Bz = b0 + b1 * np.cos(q * z)
    mf = ph.MeanField(np.zeros((n, n, n)), Bz[:, None, None] * np.ones((n, n, n)),
                      np.zeros((3, n, n, n)), 20.0)
    psi = np.zeros((1, 2, n, n, n), dtype=complex)
    psi[0, 0] = np.exp(1j * k * z)[:, None, None]
    hpsi = ph.apply_h(psi, mf, g)[0, 0]
    # -(B psi')' = B k^2 psi - i k B' psi,  B' = -b1 q sin(qz)
    expect = (Bz * k * k + 1j * k * b1 * q * np.sin(q * z)) * np.exp(1j * k * z)
    np.testing.assert_allclose(hpsi, expect[:, None, None] * np.ones((n, n, n)),
                               atol=1e-10)


# ---------------------------------------------------------------- functional
def _uniform(g, rho_n, rho_p, tau_n, tau_p):
    sh = (g.n,) * 3
    z3 = np.zeros((3,) + sh)
    mk = lambda r, t: ph.Densities(np.full(sh, r), np.full(sh, t), z3, z3, z3)
    return mk(rho_n, tau_n), mk(rho_p, tau_p)


def _textbook_symmetric(p, rho, tau):
    """Skyrme energy density of spin-saturated symmetric matter (t-form)."""
    return (p["hb2m_n"] * tau + 3 / 8 * p["t0"] * rho ** 2
            + p["t3"] / 16 * rho ** (p["alpha"] + 2)
            + (3 * p["t1"] + p["t2"] * (5 + 4 * p["x2"])) / 16 * rho * tau)


def _textbook_neutron(p, rho, tau):
    """Skyrme energy density of pure neutron matter (t-form)."""
    return (p["hb2m_n"] * tau + p["t0"] * (1 - p["x0"]) / 4 * rho ** 2
            + p["t3"] * (1 - p["x3"]) / 24 * rho ** (p["alpha"] + 2)
            + (p["t1"] * (1 - p["x1"]) + 3 * p["t2"] * (1 + p["x2"])) / 8
            * rho * tau)


@pytest.mark.parametrize("rho,tau", [(0.16, 0.36), (0.05, 0.04), (0.01, 0.004)])
def test_uniform_matter_textbook(rho, tau):
    """T5a: the functional reduces to the textbook symmetric / neutron matter."""
    g = Grid(4, 1.0)
    dn, dp = _uniform(g, rho / 2, rho / 2, tau / 2, tau / 2)
    E = ph.energy(dn, dp, g, SLY4, np.zeros((4, 4, 4)))["total"]
    assert E == pytest.approx(g.L ** 3 * _textbook_symmetric(SLY4, rho, tau),
                              rel=1e-13)
    dn, dp = _uniform(g, rho, 0.0, tau, 0.0)
    E = ph.energy(dn, dp, g, SLY4, np.zeros((4, 4, 4)))["total"]
    assert E == pytest.approx(g.L ** 3 * _textbook_neutron(SLY4, rho, tau),
                              rel=1e-13)


def test_sly4_saturation_point():
    """T14: SLy4 symmetric matter saturates at ~0.160 fm^-3, E/A ~ -15.97 MeV
    (published properties of the force) with the continuum Fermi-gas tau."""
    g = Grid(2, 1.0)

    def e_per_a(rho):
        kf = (1.5 * math.pi ** 2 * rho) ** (1 / 3)
        tau = 0.6 * kf ** 2 * rho
        dn, dp = _uniform(g, rho / 2, rho / 2, tau / 2, tau / 2)
        return ph.energy(dn, dp, g, SLY4, np.zeros((2, 2, 2)))["total"] / (
            g.L ** 3 * rho)
    res = scipy.optimize.minimize_scalar(e_per_a, bounds=(0.1, 0.22),
                                         method="bounded",
                                         options=dict(xatol=1e-7))
    assert res.x == pytest.approx(0.160, abs=0.002)
    assert res.fun == pytest.approx(-15.97, abs=0.05)


def test_mean_field_is_energy_derivative_uniform():
    """eps = dE/drho_q + k^2 dE/dtau_q in uniform matter: the potentials U_q
    and B_q equal finite differences of the energy density."""
    g = Grid(4, 1.0)
    base = (0.05, 0.02, 0.06, 0.015)
    dn, dp = _uniform(g, *base)
    mn, mp, _ = ph.mean_field(dn, dp, g, SLY4)
    V = g.L ** 3

    def edens(v):
        a, b = _uniform(g, *v)
        return ph.energy(a, b, g, SLY4, np.zeros((4, 4, 4)))["total"] / V
    h = 1e-6
    for idx, want in ((0, mn.U), (1, mp.U), (2, mn.B), (3, mp.B)):
        vp = list(base); vm = list(base)
        vp[idx] += h; vm[idx] -= h
        fd = (edens(vp) - edens(vm)) / (2 * h)
        assert fd == pytest.approx(want.flat[0], rel=1e-7)


def test_uniform_plane_waves_fixed_point():
    """T5b: closed-shell plane waves in a box are an exact fixed point of the
    full Skyrme h; eps = U_q + B_q k^2 with textbook uniform-matter values."""
    g = Grid(8, 1.0)
    psi = _plane_states(g, 14)
    st = so.State(g, SLY4, 0.45, 100.0, [psi.copy(), psi.copy()])
    st.update_fields()
    rho = 28 / g.L ** 3
    k1 = 2 * math.pi / g.L
    tau = 2 * 12 * k1 ** 2 / g.L ** 3
    assert st.E["total"] == pytest.approx(
        g.L ** 3 * _textbook_symmetric({**SLY4, "e2": 0}, rho, tau), rel=1e-12)
    # U and B of symmetric matter from d/d(rho), d/d(tau) of the textbook form
    h = 1e-7
    U = (_textbook_symmetric(SLY4, rho + h, tau)
         - _textbook_symmetric(SLY4, rho - h, tau)) / (2 * h)
    B = (_textbook_symmetric(SLY4, rho, tau + h)
         - _textbook_symmetric(SLY4, rho, tau - h)) / (2 * h)
    assert st.mf[0].U.flat[0] == pytest.approx(U, rel=1e-7)
    assert st.mf[0].B.flat[0] == pytest.approx(B, rel=1e-7)
    assert so.residual(st) < 1e-10
    rep = so.iterate(st)
    lab = inputs.plane_wave_labels(8, 14)
    k2 = (lab[:, :3] ** 2).sum(1) * k1 ** 2
    np.testing.assert_allclose(np.sort(rep.ritz[0]),
                               np.sort(st.mf[0].U.flat[0] + st.mf[0].B.flat[0]
                                       * k2), atol=1e-9)


def test_coulomb_single_mode():
    """Poisson in k-space: rho_p = c cos(qz) gives V = 4 pi e2 c cos(qz)/q^2."""
    g = Grid(16, 1.0)
    z = np.arange(16.0)
    q = 2 * math.pi * 3 / g.L
    rho = 0.02 + 0.01 * np.cos(q * z)[:, None, None] * np.ones((16, 16, 16))
    V = ph.coulomb(rho, g, 1.44)
    np.testing.assert_allclose(V, 4 * math.pi * 1.44 * 0.01 * np.cos(q * z)[
        :, None, None] / q ** 2 * np.ones((16, 16, 16)), atol=1e-12)


def test_gradient_terms_closed_form():
    """E_lap and E_so for a single modulated spinor in closed form.

    psi = A (1 + c cos qz) e^{i kx x} chi_up: rho = A^2 (1 + c cos)^2,
    int rho Lap rho = -A^4 L^3 q^2 (2 c^2 + c^4 / 2);
    J_y = -kx rho, J_x = J_z = 0 so div J = 0 and E_so = 0.
    """
    g = Grid(16, 1.0)
    n = g.n
    z = np.arange(n) * g.dx
    x = np.arange(n) * g.dx
    q = 2 * math.pi / g.L
    kx = 2 * math.pi * 2 / g.L
    c = 0.4
    amp = (1 + c * np.cos(q * z))[:, None, None] * np.exp(1j * kx * x)[None, None]
    psi = np.zeros((1, 2, n, n, n), dtype=complex)
    psi[0, 0] = amp * np.ones((n, n, n))
    A2 = 1.0 / (g.dV * (abs(psi) ** 2).sum())
    psi *= math.sqrt(A2)
    d = ph.densities(psi, g)
    np.testing.assert_allclose(d.J[1], -kx * d.rho, atol=1e-12)
    assert abs(d.J[0]).max() < 1e-12 and abs(d.J[2]).max() < 1e-12
    np.testing.assert_allclose(d.s[2], d.rho, atol=1e-12)
    np.testing.assert_allclose(d.j[0], kx * d.rho, atol=1e-12)
    lap = ph._derived(d, g)[0]
    integral = g.dV * (d.rho * lap).sum()
    assert integral == pytest.approx(
        -A2 ** 2 * g.L ** 3 * q ** 2 * (2 * c ** 2 + c ** 4 / 2), rel=1e-12)
    # tau = |d psi|^2 = A^2 [c^2 q^2 sin^2 + kx^2 (1 + c cos)^2]
    tau = A2 * (c ** 2 * q ** 2 * np.sin(q * z) ** 2 + kx ** 2 * (1 + c * np.cos(
        q * z)) ** 2)
    np.testing.assert_allclose(d.tau, tau[:, None, None] * np.ones((n, n, n)),
                               atol=1e-12)


def test_variational_consistency():
    """T6: dE/d(eta) along a random direction equals 2 Re sum <dpsi|h psi>."""
    rng = np.random.default_rng(5)
    g = Grid(8, 1.0)
    w = inputs.small_workload("v", 8, 4, 3, init="rod", seed=11, noise=0.3)
    rn, rp = inputs.raw_states(w)
    st = so.initial_state(rn, rp, g, SLY4, 0.45, 100.0)
    dpsi = [rng.standard_normal(p.shape) + 1j * rng.standard_normal(p.shape)
            for p in st.psi]
    dpsi = [0.01 * d / math.sqrt(g.dV * (abs(d) ** 2).sum()) for d in dpsi]
    lin = sum(2 * so.overlap(d, ph.apply_h(p, m, g), g).trace().real
              for d, p, m in zip(dpsi, st.psi, st.mf))

    def E_at(eta):
        s2 = so.State(g, SLY4, 0.45, 100.0,
                      [p + eta * d for p, d in zip(st.psi, dpsi)])
        s2.update_fields()
        return s2.E["total"]
    eta = 1e-3
    fd = (E_at(eta) - E_at(-eta)) / (2 * eta)
    assert fd == pytest.approx(lin, rel=1e-6)


# ---------------------------------------------------------------- solver
def test_damping_plane_wave_closed_form():
    """Damping of a plane wave multiplies it by x0 / (E0 + hb2m k^2)."""
    g = Grid(8, 1.0)
    x = np.arange(8.0)
    for m in (0, 1, 3, -4):
        k = 2 * math.pi * m / g.L
        f = np.exp(1j * k * x)[None, None, None, None, :] * np.ones((1, 2, 8, 8, 8))
        out = so.damping(f, g, 20.0, 0.45, 100.0)
        np.testing.assert_allclose(out, 0.45 / (100.0 + 20.0 * k * k) * f,
                                   atol=1e-14)


def test_residual_two_plane_waves():
    """Eq. convergence: <h^2> - <h>^2 for a superposition of two free plane
    waves equals |a|^2 e1^2 + |b|^2 e2^2 - eps^2."""
    g = Grid(8, 1.0)
    n = 8
    x = np.arange(n) * 1.0
    hb = 20.0
    mf = ph.MeanField(np.zeros((n,) * 3), np.full((n,) * 3, hb),
                      np.zeros((3,) + (n,) * 3), hb)
    k1, k2 = 2 * math.pi / g.L, 2 * math.pi * 2 / g.L
    a, b = 0.6, 0.8j
    psi = np.zeros((1, 2, n, n, n), dtype=complex)
    psi[0, 0] = (a * np.exp(1j * k1 * x) + b * np.exp(1j * k2 * x)) / math.sqrt(
        g.L ** 3)
    hpsi = ph.apply_h(psi, mf, g)
    eps, r, r2 = so.rayleigh_and_residual(psi, hpsi, g)
    e1, e2 = hb * k1 ** 2, hb * k2 ** 2
    want = abs(a) ** 2 * e1 + abs(b) ** 2 * e2
    assert eps[0] == pytest.approx(want, rel=1e-13)
    assert r2[0] == pytest.approx(abs(a) ** 2 * e1 ** 2 + abs(b) ** 2 * e2 ** 2
                                  - want ** 2, rel=1e-12)


def test_rayleigh_ritz_vs_generalised_eigh():
    """T8: U^H I U = 1, U^H H U = diag(lam); lam = scipy's eigh(H, I)."""
    rng = np.random.default_rng(2)
    for n in (1, 5, 37):
        X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        I = np.eye(n) + 0.05 * (X @ X.conj().T) / n
        Y = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        H = Y + Y.conj().T
        U, lam = so.rayleigh_ritz(I, H)
        np.testing.assert_allclose(U.conj().T @ I @ U, np.eye(n), atol=1e-12)
        np.testing.assert_allclose(U.conj().T @ H @ U, np.diag(lam), atol=1e-11)
        np.testing.assert_allclose(lam, scipy.linalg.eigh(H, I,
                                                          eigvals_only=True),
                                   atol=1e-11)
        assert np.all(np.diff(lam) >= 0)


def test_loewdin_orthonormal_and_particle_number():
    """T7/T8: Loewdin states are orthonormal and integrate rho to N."""
    w = inputs.small_workload("l", 8, 10, 6, init="slab", seed=4, noise=0.2)
    rn, rp = inputs.raw_states(w)
    g = Grid(8, 1.0)
    for raw in (rn, rp):
        psi = so.loewdin(raw, g)
        np.testing.assert_allclose(so.overlap(psi, psi, g), np.eye(len(psi)),
                                   atol=1e-12)
        d = ph.densities(psi, g)
        assert g.dV * d.rho.sum() == pytest.approx(len(psi), rel=1e-12)


def test_loewdin_is_closest_orthonormal_set():
    """Loewdin's set minimises sum ||psi_a - phi_a||^2 among orthonormal sets
    (its defining property, Sec. 3.3.2): compare with the polar factor."""
    rng = np.random.default_rng(9)
    g = Grid(4, 1.0)
    phi = rng.standard_normal((5, 2, 4, 4, 4)) + 1j * rng.standard_normal(
        (5, 2, 4, 4, 4))
    psi = so.loewdin(phi, g)
    # polar decomposition of the weighted matrix sqrt(dV) Phi^T
    A = math.sqrt(g.dV) * phi.reshape(5, -1).T
    Uw, _, Vh = np.linalg.svd(A, full_matrices=False)
    polar = (Uw @ Vh).T.reshape(phi.shape) / math.sqrt(g.dV)
    np.testing.assert_allclose(psi, polar, atol=1e-12)


def test_span_invariance_loewdin_vs_cholesky():
    """T10: densities depend only on the span of the occupied states."""
    w = inputs.small_workload("s", 8, 7, 5, init="rod", seed=6, noise=0.2)
    rn, _ = inputs.raw_states(w)
    g = Grid(8, 1.0)
    a = so.loewdin(rn, g)
    I = so.overlap(rn, rn, g)
    L = np.linalg.cholesky(I)
    b = so.combine(rn, np.linalg.inv(L).conj().T)
    da, db = ph.densities(a, g), ph.densities(b, g)
    for f in ("rho", "tau", "J"):
        np.testing.assert_allclose(getattr(da, f), getattr(db, f), atol=1e-12)


def test_translation_and_axis_permutation_invariance():
    """T11: E is unchanged by a grid translation and by swapping x and y."""
    w = inputs.small_workload("t", 8, 6, 4, init="rod", seed=8, noise=0.3)
    rn, rp = inputs.raw_states(w)
    g = Grid(8, 1.0)
    st = so.initial_state(rn, rp, g, SLY4, 0.45, 100.0)
    E0 = st.E["total"]
    moved = [np.roll(p, (1, 3, 2), axis=(2, 3, 4)) for p in st.psi]
    s2 = so.State(g, SLY4, 0.45, 100.0, moved)
    s2.update_fields()
    assert s2.E["total"] == pytest.approx(E0, rel=1e-12)
    # 120 degree rotation about (1,1,1): e_x -> e_y -> e_z -> e_x, a proper
    # rotation that maps the grid onto itself without reflections; spinors
    # rotate with exp(-i theta/2 n.sigma).  psi'(x,y,z) = U psi(y,z,x).
    Us = 0.5 * np.eye(2) - 0.5j * (ph.SIGMA[0] + ph.SIGMA[1] + ph.SIGMA[2])
    rot = [np.einsum("st,atxyz->asxyz", Us, np.transpose(p, (0, 1, 3, 4, 2)))
           for p in st.psi]
    s3 = so.State(g, SLY4, 0.45, 100.0, rot)
    s3.update_fields()
    assert s3.E["total"] == pytest.approx(E0, rel=1e-12)
    # rotating space without the spin changes the spin-orbit energy
    bare = [np.transpose(p, (0, 1, 3, 4, 2)) for p in st.psi]
    s4 = so.State(g, SLY4, 0.45, 100.0, bare)
    s4.update_fields()
    assert abs(s4.E["so"] - st.E["so"]) > 1e-6 * abs(st.E["so"])


def test_time_even_start_stays_time_even():
    """T12: Kramers-paired closed shells keep s = 0 and j ~ 0 through iterations.

    s vanishes to rounding.  j vanishes only up to the Nyquist mode: the first
    derivative keeps the Nyquist multiplier (so D^2 = -k^2 there), which does
    not commute with complex conjugation, so h is time-reversal symmetric only
    up to the states' Nyquist content.  A genuine time-reversal error (a wrong
    sign or factor i in the spin-orbit term) gives j ~ rho*k, far above the
    bound used here.
    """
    g = Grid(8, 1.0)
    w = inputs.small_workload("te", 8, 14, 2, init="slab", seed=12, noise=0.0)
    rn, rp = inputs.raw_states(w)
    st = so.initial_state(rn, rp, g, SLY4, 0.45, 100.0)
    for _ in range(3):
        so.iterate(st)
    k1 = 2 * math.pi / g.L
    for d in st.dens:
        assert abs(d.s).max() < 1e-13
        assert abs(d.j).max() < 1e-3 * d.rho.max() * k1


def test_free_fermi_gas_converges_to_closed_form():
    """T4: Skyrme and Coulomb off, 14 + 2 states from a noisy start converge
    to the closed-shell free-gas energy sum hb2m k^2."""
    g = Grid(8, 1.0)
    w = inputs.small_workload("ff", 8, 14, 2, seed=13, noise=0.3)
    rn, rp = inputs.raw_states(w)
    p = _free()
    st = so.initial_state(rn, rp, g, p, 0.45, 20.0)
    k1 = 2 * math.pi / g.L
    want = p["hb2m_n"] * 12 * k1 ** 2
    for _ in range(600):
        rep = so.iterate(st)
        if rep.de < 1e-9:
            break
    assert rep.de < 1e-8
    assert st.E["total"] == pytest.approx(want, rel=1e-10)
    np.testing.assert_allclose(rep.ritz[0], np.r_[0, 0, [p["hb2m_n"] * k1 ** 2]
                                                  * 12], atol=1e-8)


def test_dense_h_8cubed_aufbau():
    """T9: dense 1024x1024 h on an 8^3 grid, built by applying h to unit
    vectors, is Hermitian; with that (non-uniform, spin-orbit on) mean field
    held fixed, the damped-gradient iteration converges to its lowest N
    eigenvalues and to eigenvectors spanning the same space."""
    rng = np.random.default_rng(21)
    g = Grid(8, 1.0)
    mf = _random_fields(g, rng)
    eye = np.eye(1024, dtype=complex).reshape(1024, 2, 8, 8, 8)
    Hd = ph.apply_h(eye, mf, g).reshape(1024, 1024).T
    assert abs(Hd - Hd.conj().T).max() < 1e-12 * abs(Hd).max()
    ev, vec = np.linalg.eigh(0.5 * (Hd + Hd.conj().T))
    gaps = np.diff(ev[:24])
    nq = int(np.argmax(gaps[3:]) + 4)          # occupy below the widest gap
    assert gaps[nq - 1] > 2.0
    assert gaps[1] > 2.0                       # the lowest pair is isolated too
    w = inputs.small_workload("d", 8, nq, 2, init="rod", seed=14, noise=0.2)
    rn, rp = inputs.raw_states(w)
    st = so.State(g, SLY4, 0.45, 20.0, [so.loewdin(rn, g), so.loewdin(rp, g)])
    st.mf = [mf, mf]
    for _ in range(1000):
        rep = so.iterate(st, self_consistent=False)
        if rep.de < 1e-10:
            break
    assert rep.de < 1e-9
    np.testing.assert_allclose(rep.ritz[0], ev[:nq], atol=1e-9)
    np.testing.assert_allclose(rep.ritz[1], ev[:2], atol=1e-9)
    # same span: projector onto the solver's states equals the exact one
    P = st.psi[0].reshape(nq, -1).T * math.sqrt(g.dV)
    Q = vec[:, :nq]
    np.testing.assert_allclose(P @ P.conj().T, Q @ Q.conj().T, atol=1e-7)


@pytest.mark.parametrize("name", ["sat8", "sat24"])
def test_saturation_box_ground_state_energy(name):
    """The closed-shell plane-wave determinant of the saturation boxes (the
    state their iterations converge to: uniform matter there is stable) has
    the textbook symmetric-matter energy with the box's discrete tau."""
    import dataclasses
    w = inputs.WORKLOADS[name]
    wp = dataclasses.replace(w, init="plain", amp=0.0, noise=0.0)
    raw = inputs.raw_states(wp)
    g = Grid(w.n, w.dx)
    st = so.initial_state(raw[0], raw[1], g, w.params, w.damp_x0, w.damp_e0)
    L = w.n * w.dx
    lab = inputs.plane_wave_labels(w.n, w.n_neutrons)
    k2 = ((2 * math.pi / L) ** 2 * (lab[:, :3] ** 2).sum(axis=1)).sum()
    rho = (w.n_neutrons + w.n_protons) / L ** 3
    tau = 2 * k2 / L ** 3
    p = dict(w.params)
    assert st.E["total"] == pytest.approx(L ** 3 * _textbook_symmetric(p, rho, tau), rel=1e-12)
