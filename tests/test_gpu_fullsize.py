"""Full-size checks in the launch configuration bench.py times (48^3 grid,
1600 neutron + 400 proton states, complex128).

Where the oracle can produce sampled outputs one by one it does (mean field
from a few states, h*psi and the damped step of sampled states, sampled
overlap entries); elsewhere the checks are properties that hold at any size:
orthonormality, the polar-decomposition property of Loewdin's states,
U^H I U = 1 and U^H H U = diag(ritz), and a decreasing energy.
"""
import numpy as np
import pytest

from oracle import Grid
from oracle import physics as ph
from oracle import solver as so
from paper_1610_07522_amd import inputs

from gpu_util import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

W = inputs.WORKLOADS["rod48"]
NS = 6           # states per species that carry the density in the field test


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def raw():
    return inputs.raw_states(W)


@pytest.fixture(scope="module")
def box(torch_mod):
    from paper_1610_07522_amd import sky
    b = sky.Box(sky.desc_from_workload(W))
    yield b
    b.close()


def _eye(torch, m):
    return torch.eye(m, dtype=torch.complex128, device="cuda:0")


def test_fullsize_kernels_vs_oracle(torch_mod, box, raw):
    torch = torch_mod
    g = Grid(W.n, W.dx)
    rng = np.random.default_rng(5)
    # densities from NS states per species (the rest zero), all kernels at full size
    for q in range(2):
        psi = box.view("psi", q)
        psi.zero_()
        psi[:NS].copy_(to_dev(raw[q][:NS]))
    box.densities()
    box.sync()
    sub = [raw[0][:NS], raw[1][:NS]]
    dens = [ph.densities(s, g) for s in sub]
    mn, mp, vc = ph.mean_field(dens[0], dens[1], g, W.params)
    for q, m in ((0, mn), (1, mp)):
        gm = to_host(box.view("meanfield", q))
        for i, ref in enumerate([m.U, m.B, m.W[0], m.W[1], m.W[2]]):
            assert np.abs(gm[i] - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max()), (q, i)
    # h psi and the damped step over every state of the species, sampled output
    for q, mf in ((0, mn), (1, mp)):
        m = raw[q].shape[0]
        psi, hpsi, phi = box.view("psi", q), box.view("hpsi", q), box.view("phi", q)
        psi.copy_(to_dev(raw[q]))
        eps = torch.zeros(m, dtype=torch.float64, device="cuda:0")
        r2 = torch.zeros(m, dtype=torch.float64, device="cuda:0")
        box.apply_h(q, psi, hpsi, m, eps)
        box.damped_step(q, psi, hpsi, eps, phi, m, r2)
        box.sync()
        pick = np.sort(rng.choice(m, 6, replace=False))
        pick = np.unique(np.r_[pick, m - 1])
        h_ref = ph.apply_h(raw[q][pick], mf, g)
        e_ref, r_ref, r2_ref = so.rayleigh_and_residual(raw[q][pick], h_ref, g)
        phi_ref = raw[q][pick] - so.damping(r_ref, g, mf.hb2m, W.damp_x0, W.damp_e0)
        idx = torch.as_tensor(pick, device="cuda:0")
        assert rel_err(to_host(hpsi[idx]), h_ref) <= 1e-11, q
        assert rel_err(to_host(eps[idx]), e_ref) <= 1e-10, q
        assert rel_err(to_host(r2[idx]), r2_ref) <= 1e-9, q
        assert rel_err(to_host(phi[idx]), phi_ref) <= 1e-11, q


def test_fullsize_loewdin(torch_mod, box, raw):
    """Overlap GEMM on sampled entries; Loewdin states orthonormal and the
    polar factor of the trial set (<psi|raw> Hermitian positive definite)."""
    torch = torch_mod
    rng = np.random.default_rng(6)
    dV = W.dx ** 3
    for q in range(2):
        m = raw[q].shape[0]
        rd = to_dev(raw[q])
        out = torch.empty_like(rd)
        box.orthonormalize(q, rd, None, out)
        I = to_host(box.view("overlap", q))
        rf = raw[q].reshape(m, -1)
        err = 0.0
        for _ in range(200):
            a, b = rng.integers(0, m, 2)
            err = max(err, abs(I[a, b] - dV * np.vdot(rf[a], rf[b])))
        assert err <= 1e-12, q
        o = out.reshape(m, -1)
        G = dV * (o.conj() @ o.T.contiguous())
        assert (G - _eye(torch, m)).abs().max().item() <= 1e-11, q
        M = dV * (o.conj() @ rd.reshape(m, -1).T.contiguous())
        assert (M - M.conj().T).abs().max().item() <= 1e-11, q
        assert torch.linalg.eigvalsh(0.5 * (M + M.conj().T)).min().item() > 0.0, q
        del rd, out, o, G, M


def test_fullsize_iterations(torch_mod, box, raw):
    """Init + 3 iterations at full size: orthonormal states, exact
    Rayleigh-Ritz identities, ascending Ritz values, decreasing energy; from
    the second iteration on the eigenvector refinement converges without
    falling back to Jacobi."""
    torch = torch_mod
    dV = W.dx ** 3
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    E = [to_host(box.view("energy"))[7]]
    for it in range(3):
        rep = box.iterate(1)
        assert np.isfinite(rep["residual"])
        # after the first Rayleigh-Ritz step (far from diagonal: the blocked
        # Jacobi solver takes it) the eigenvector refinement finishes alone
        if it > 0:
            assert rep["eig_fallbacks"] == 0, rep
        E.append(rep["energy"])
        for q in range(2):
            m = raw[q].shape[0]
            p = box.view("psi", q).reshape(m, -1)
            G = dV * (p.conj() @ p.T.contiguous())
            assert (G - _eye(torch, m)).abs().max().item() <= 1e-11, q
    assert all(E[i + 1] < E[i] for i in range(3)), E
    # last species (protons) of the last iteration: RR identities
    m = raw[1].shape[0]
    I, H, U = box.view("overlap", 1), box.view("hsub", 1), box.view("umat", 1)
    lam = box.view("ritz", 1)
    assert (U.conj().T @ I @ U - _eye(torch, m)).abs().max().item() <= 1e-11
    D = torch.diag(lam).to(torch.complex128)
    assert (U.conj().T @ H @ U - D).abs().max().item() <= 1e-10 * max(1.0, lam.abs().max().item())
    assert bool((lam[1:] >= lam[:-1]).all())
