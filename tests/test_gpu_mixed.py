"""Mixed-precision form (complex64 states, FP32 FFT and h*psi, split-FP16
MFMA products with FP32 accumulation folded into FP64, FP64 subspace solve)
against the FP64 oracle.

The oracle gets the same complex64-rounded inputs, widened exactly to
complex128, so each bar measures only the mixed arithmetic.  Bars derive from
the FP32 unit roundoff u = 2^-24 ~ 6e-8:
* split-FP16 products (x = h + l, |x - h - l| <= 2^-22 |x| = 4u|x| under
  a power-of-two scale; h h' + h l' + l h', the dropped l l' <= 4u) accumulate
  in FP32 over 256 elements before folding into FP64: relative error about
  ten u of the largest entry -> 1e-6;
* an FP32 spectral derivative loses ~log2(n) u -> h*psi, densities and the
  damped step within 2e-5 of their max-norm (two derivatives per direction,
  three directions, FP32 pointwise algebra);
* the energy is a difference of kinetic and potential parts ~50x larger
  than the total in a pasta box, so per-iteration energy error is bounded by
  a few hundred u times the sum of |parts|.
"""
import json
from pathlib import Path

import numpy as np
import pytest

from oracle import Grid
from oracle import physics as ph
from oracle import solver as so
from paper_1610_07522_amd import inputs

from gpu_util import CASES, rel_err, to_dev, to_host

ROOT = Path(__file__).resolve().parents[1]

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
MIXED_CASES = ["n16_8p8", "n24_13p7_rod", "n32_70p33_slab", "n24_200p50_rod"]


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _box(w, ladder_tol=0.0):
    from paper_1610_07522_amd import sky
    return sky.Box(sky.desc_from_workload(w, precision=sky.SKY_MIXED, ladder_tol=ladder_tol))


def _c64(x):
    return x.astype(np.complex64)


@pytest.mark.parametrize("case", MIXED_CASES)
def test_mixed_overlap_and_loewdin(torch_mod, case):
    torch = torch_mod
    w = CASES[case]
    raw = [_c64(r) for r in inputs.raw_states(w)]
    g = Grid(w.n, w.dx)
    box = _box(w)
    for q in range(2):
        m = raw[q].shape[0]
        out = torch.empty(raw[q].shape, dtype=torch.complex64, device="cuda:0")
        box.orthonormalize(q, to_dev(raw[q]), None, out)
        ref64 = raw[q].astype(np.complex128)
        I_ref = so.overlap(ref64, ref64, g)
        assert rel_err(to_host(box.view("overlap", q)), I_ref) <= 1e-6, (case, q)
        o = to_host(out).astype(np.complex128)
        G = so.overlap(o, o, g)
        assert np.abs(G - np.eye(m)).max() <= 2e-6, (case, q)
        assert rel_err(o, so.loewdin(ref64, g)) <= 2e-5, (case, q)


@pytest.mark.parametrize("case", MIXED_CASES)
def test_mixed_fields_h_and_damping(torch_mod, case):
    torch = torch_mod
    w = CASES[case]
    raw = [_c64(r) for r in inputs.raw_states(w)]
    ref = [r.astype(np.complex128) for r in raw]
    g = Grid(w.n, w.dx)
    box = _box(w)
    for q in range(2):
        box.view("psi", q).copy_(to_dev(raw[q]))
    box.densities()
    box.sync()
    dn, dp = ph.densities(ref[0], g), ph.densities(ref[1], g)
    mn, mp, vc = ph.mean_field(dn, dp, g, w.params)
    E = ph.energy(dn, dp, g, w.params, vc)
    for q, d in ((0, dn), (1, dp)):
        gd = to_host(box.view("dens", q))
        assert rel_err(gd[0], d.rho) <= 2e-6, (case, q)
        assert rel_err(gd[1], d.tau) <= 2e-5, (case, q)
    parts = sum(abs(E[k]) for k in ("kin", "rho", "rho3", "tau", "lap", "so", "coul"))
    assert abs(to_host(box.view("energy"))[7] - E["total"]) <= 300 * U32 * parts, case
    for q, mf in ((0, mn), (1, mp)):
        m = raw[q].shape[0]
        psi, hpsi, phi = box.view("psi", q), box.view("hpsi", q), box.view("phi", q)
        eps = torch.zeros(m, dtype=torch.float64, device="cuda:0")
        r2 = torch.zeros(m, dtype=torch.float64, device="cuda:0")
        box.apply_h(q, psi, hpsi, m, eps)
        box.damped_step(q, psi, hpsi, eps, phi, m, r2)
        box.sync()
        h_ref = ph.apply_h(ref[q], mf, g)
        e_ref, r_ref, r2_ref = so.rayleigh_and_residual(ref[q], h_ref, g)
        phi_ref = ref[q] - so.damping(r_ref, g, mf.hb2m, w.damp_x0, w.damp_e0)
        assert rel_err(to_host(hpsi), h_ref) <= 2e-5, (case, q)
        assert rel_err(to_host(eps), e_ref) <= 2e-5, (case, q)
        assert rel_err(to_host(phi), phi_ref) <= 2e-6, (case, q)


@pytest.mark.parametrize("case", ["n16_8p8", "n24_200p50_rod"])
def test_mixed_trajectory_tracks_fp64(torch_mod, case):
    """Mixed iterations stay within FP32-level distance of the FP64 oracle
    trajectory started from the same raw states."""
    w = CASES[case]
    raw = inputs.raw_states(w)
    g = Grid(w.n, w.dx)
    st = so.initial_state(*raw, g, w.params, w.damp_x0, w.damp_e0)
    box = _box(w)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    for it in range(5):
        rep = box.iterate(1)
        ro = so.iterate(st)
        assert rep["precision"] == 1
        parts = sum(abs(st.E[k]) for k in ("kin", "rho", "rho3", "tau", "lap", "so", "coul"))
        assert abs(rep["energy"] - st.E["total"]) <= 1000 * U32 * parts * (it + 1), (case, it)
        assert abs(rep["residual"] - ro.de) <= 1e-4 * max(1.0, ro.de), (case, it)
        for q in range(2):
            assert rel_err(to_host(box.view("ritz", q)), ro.ritz[q]) <= 1e-5, (case, it, q)


def test_precision_ladder_switches_to_fp64(torch_mod):
    """With ladder_tol above the starting residual the context switches to
    FP64 after the first iteration, and then tracks the FP64 oracle at the
    FP64 bar relative to where it switched."""
    w = CASES["n16_8p8"]
    raw = inputs.raw_states(w)
    g = Grid(w.n, w.dx)
    box = _box(w, ladder_tol=1e3)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    assert box.precision() == 1
    rep = box.iterate(1)
    assert rep["precision"] == 0 and box.precision() == 0
    assert box.view("psi", 0).dtype.itemsize == 16
    st = so.initial_state(*raw, g, w.params, w.damp_x0, w.damp_e0)
    so.iterate(st)
    e1 = rep["energy"]
    # the FP64 continuation from the mixed first iterate stays close to the oracle
    rep = box.iterate(5)
    for _ in range(5):
        so.iterate(st)
    parts = sum(abs(st.E[k]) for k in ("kin", "rho", "rho3", "tau", "lap", "so", "coul"))
    assert abs(rep["energy"] - st.E["total"]) <= 1000 * U32 * parts, (e1, rep, st.E)


@pytest.mark.parametrize("waves", [8, 4])
def test_mixed_overlap_and_combine_fullsize(torch_mod, tmp_path, waves):
    """48^3 x 1600 neutrons, the bench configuration, in both wave layouts of
    the plane products (forced through the committed tuning cache with the
    layout keys overridden): sampled rows of the
    split-FP16 overlap (FP32 accumulation over each split-K chunk of the
    221184-long contraction, chunks summed in FP64) against the oracle's
    overlap of the same complex64 states (widened to complex128), at the 1e-6
    bar; then sampled output states of the split-FP16 recombination
    psi' = psi U (U the Rayleigh-Ritz transform of the states with their own
    h, a rotation far from the identity; from the planes of U^T and psi^T)
    against the oracle's combination of the same states and the same U, at
    the same bar."""
    torch = torch_mod
    w = inputs.WORKLOADS["rod48"]
    rn, rp = inputs.raw_states(w)
    box = _box(w)
    box.init_box(to_dev(rn), to_dev(rp))
    keys = json.loads((ROOT / "paper_1610_07522_amd" / "tuning_mi355x.json").read_text())
    for m in (w.n_neutrons, w.n_protons):
        for kind in ("overlap", "combine"):
            keys[f"plane_waves_{kind}/m{m}/k{2 * w.n ** 3}"] = waves
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps(keys))
    t = box.autotune(str(cache))
    assert t["overlap_waves"] == [waves, waves] and t["combine_waves"] == [waves, waves]
    box.init_box(to_dev(rn), to_dev(rp))
    del rn, rp
    q = 0
    psi = box.view("psi", q)
    hpsi = box.view("hpsi", q)
    m = psi.shape[0]
    box.apply_h(q, psi, hpsi, m)
    out = torch.empty_like(psi)
    box.orthonormalize(q, psi, hpsi, out)
    box.sync()
    g = Grid(w.n, w.dx)
    P = to_host(psi).astype(np.complex128)            # the states both sides use
    I_gpu = to_host(box.view("overlap", q))
    worst = 0.0
    for r in range(0, m, 97):
        ref = so.overlap(P[r:r + 1], P, g)[0]
        worst = max(worst, np.abs(I_gpu[r] - ref).max() / np.abs(ref).max())
    assert worst <= 1e-6, ("overlap", worst)
    U = to_host(box.view("umat", q))
    assert np.abs(U - np.diag(np.diag(U))).max() > 0.1      # a real rotation
    o = to_host(out)
    worst = 0.0
    for b in list(range(0, m, 211)) + [m - 1]:
        ref = so.combine(P, U[:, b:b + 1])[0]
        worst = max(worst, np.abs(o[b] - ref).max() / np.abs(ref).max())
    assert worst <= 1e-6, ("combine", worst)


@pytest.mark.parametrize("ladder", [1e-4, 0.0])
def test_mixed_matches_oracle_at_convergence(torch_mod, ladder):
    """A saturation-density box (8^3, 38 n + 38 p) that converges: the mixed
    form (with the precision ladder, to Delta-eps 1e-9; without it, 600
    iterations, where its residual has levelled off) against the FP64 oracle
    converged to Delta-eps 1e-9: total energy within 1e-6 relative, every
    single-particle energy within 1e-5 MeV."""
    w = inputs.WORKLOADS["sat8"]
    raw = inputs.raw_states(w)
    box = _box(w, ladder_tol=ladder)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    rep = box.iterate(3000, 1e-9) if ladder > 0 else box.iterate(600)
    if ladder > 0:
        assert rep["converged"] and rep["precision"] == 0
    else:
        assert rep["precision"] == 1 and rep["residual"] < 1e-3
    e_ref, ritz_ref = _sat8_converged()
    assert abs(rep["energy"] - e_ref) <= 1e-6 * abs(e_ref), (rep, e_ref)
    for q in range(2):
        got = np.sort(to_host(box.view("ritz", q)))
        want = np.sort(ritz_ref[q])
        assert np.abs(got - want).max() <= 1e-5, (q, np.abs(got - want).max())


_SAT8 = {}


def _sat8_converged():
    """FP64 oracle on the saturation box, iterated to Delta-eps 1e-9 (once)."""
    if not _SAT8:
        w = inputs.WORKLOADS["sat8"]
        raw = inputs.raw_states(w)
        st = so.initial_state(*raw, Grid(w.n, w.dx), w.params, w.damp_x0, w.damp_e0)
        for _ in range(3000):
            ro = so.iterate(st)
            if ro.de <= 1e-9:
                break
        assert ro.de <= 1e-9
        _SAT8["E"], _SAT8["ritz"] = st.E["total"], ro.ritz
    return _SAT8["E"], _SAT8["ritz"]


@pytest.mark.parametrize("mixed", [False, True])
def test_refinement_orthonormality_target(torch_mod, mixed):
    """The subspace eigenvectors Z of H' after refined Rayleigh-Ritz solves
    are orthonormal to the form's target: 1e-13 in FP64, 2^-30 in the mixed
    form (whose U = C Z is then rounded to the 2^-22 of the split planes).
    Z is checked in FP64 on the host (the device tests the same bound on its
    own product Z^H Z); the protons are the last set solved, so their Z is
    the one the context holds."""
    from paper_1610_07522_amd import sky
    w = CASES["n32_70p33_slab"]
    prec = sky.SKY_MIXED if mixed else sky.SKY_FP64
    box = sky.Box(sky.desc_from_workload(w, precision=prec))
    raw = inputs.raw_states(w)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    box.iterate(2)
    rep = box.iterate(1)
    assert rep["eig_fallbacks"] == 0   # the refinement, not the Jacobi fallback
    Z = to_host(box.view("evec", 1)).astype(np.complex128)
    assert Z.shape == (w.n_protons, w.n_protons)
    dev = np.abs(Z.conj().T @ Z - np.eye(Z.shape[0])).max()
    bound = 2.0 ** -30 if mixed else 1e-13
    assert dev <= bound * 1.01 + 1e-14, (dev, bound)
