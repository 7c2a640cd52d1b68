"""Autotuner (launch shapes of the h passes and of the split-K products):
tuned shapes compute the same iteration as the defaults, come from the
candidate lists, and round-trip through the JSON cache."""
import json

import numpy as np
import pytest

from paper_1610_07522_amd import inputs

from gpu_util import CASES, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _box(w, precision):
    from paper_1610_07522_amd import sky
    return sky.Box(sky.desc_from_workload(w, precision=precision))


@pytest.mark.parametrize("case,precision,tol", [("n24_200p50_rod", 0, 1e-10),
                                                ("n32_70p33_slab", 1, 2e-6)])
def test_autotune_parity_and_cache(torch_mod, tmp_path, case, precision, tol):
    w = CASES[case]
    raw = inputs.raw_states(w)
    cache = tmp_path / "tune.json"
    ref = _box(w, precision)
    ref.init_box(to_dev(raw[0]), to_dev(raw[1]))
    r_ref = ref.iterate(3)
    rho_ref = to_host(ref.view("dens", 0))[0]
    ritz_ref = to_host(ref.view("ritz", 0))

    box = _box(w, precision)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    t = box.autotune(str(cache))
    assert not t["from_cache"]
    stored = json.loads(cache.read_text())
    prec = "mixed" if precision else "fp64"
    assert stored[f"h_lines/n{w.n}/{prec}"] == t["h_lines"]
    assert stored[f"overlap_split/m{w.n_neutrons}/k{2 * w.n ** 3}/{prec}"] == t["overlap_split"][0]
    assert t["h_lines"] in (-1, 16, 32, 64, 128) and all(s >= 1 for s in t["square_split"])
    assert t["damp_xy"] in (-1, 0, 1)
    r = box.iterate(3)
    assert abs(r["energy"] - r_ref["energy"]) <= tol * abs(r_ref["energy"]), (r, r_ref)
    assert rel_err(to_host(box.view("dens", 0))[0], rho_ref) <= tol
    assert rel_err(to_host(box.view("ritz", 0)), ritz_ref) <= tol

    again = _box(w, precision)
    again.init_box(to_dev(raw[0]), to_dev(raw[1]))
    t2 = again.autotune(str(cache))
    assert t2["from_cache"]
    assert {k: v for k, v in t2.items() if k != "from_cache"} == \
        {k: v for k, v in t.items() if k != "from_cache"}


@pytest.mark.parametrize("case,precision", [("n24_13p7_rod", 0), ("n32_70p33_slab", 0),
                                            ("n16_8p8", 1), ("n24_13p7_rod", 1),
                                            ("n48_6p3", 1)])
@pytest.mark.parametrize("h_lines,damp_xy", [(-1, 1), (0, 0)])
def test_slice_and_pencil_variants_match_oracle(torch_mod, tmp_path, case, precision,
                                                h_lines, damp_xy):
    """h psi, <h> and the damped step in both layouts (x and y on LDS z-slices,
    or three line passes), forced through the tuning cache, against the
    oracle (FP64 1e-11; complex64 inputs 2e-5 on h psi, 2e-6 on the step)."""
    import torch
    from oracle import Grid
    from oracle import physics as ph
    from oracle import solver as so
    w = CASES[case] if case in CASES else inputs.small_workload(case, 48, 6, 3, init="rod",
                                                                 seed=34, noise=0.05)
    raw = inputs.raw_states(w)
    box = _box(w, precision)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    prec = "mixed" if precision else "fp64"
    lines = h_lines if h_lines else {8: 64, 16: 64, 24: 32, 32: 32, 48: 32}[w.n]
    cache = tmp_path / "force.json"
    cache.write_text(json.dumps({f"h_lines/n{w.n}/{prec}": lines,
                                 f"damp_xy/n{w.n}/{prec}": damp_xy}))
    t = box.autotune(str(cache))
    assert t["h_lines"] == lines and t["damp_xy"] == damp_xy
    g = Grid(w.n, w.dx)
    q = 0
    m = w.n_neutrons
    # inputs: the raw states rounded to the working precision, fields from them
    cdt = torch.complex64 if precision else torch.complex128
    for s in range(2):
        box.view("psi", s).copy_(to_dev(raw[s]).to(cdt))
    box.densities()
    xs = [to_host(box.view("psi", s)).astype(np.complex128) for s in range(2)]
    dens = [ph.densities(xs[0], g), ph.densities(xs[1], g)]
    mf = ph.mean_field(dens[0], dens[1], g, w.params)[q]
    psi, hpsi, phi = box.view("psi", q), box.view("hpsi", q), box.view("phi", q)
    eps = torch.empty(m, dtype=torch.float64, device=psi.device)
    box.apply_h(q, psi, hpsi, m, eps)
    box.damped_step(q, psi, hpsi, eps, phi, m)
    torch.cuda.synchronize()
    x = xs[q]
    h_ref = ph.apply_h(x, mf, g)
    e_ref, r_ref, _ = so.rayleigh_and_residual(x, h_ref, g)
    phi_ref = x - so.damping(r_ref, g, mf.hb2m, w.damp_x0, w.damp_e0)
    th, tp = (2e-5, 2e-6) if precision else (1e-11, 1e-11)
    assert rel_err(to_host(hpsi), h_ref) <= th
    assert rel_err(to_host(eps), e_ref) <= th
    assert rel_err(to_host(phi), phi_ref) <= tp


@pytest.mark.parametrize("n,nn,np_,precision", [(48, 6, 3, 0), (64, 4, 2, 1)])
@pytest.mark.parametrize("damp_xy", [1, 0])
def test_damped_step_slices_large_grids(torch_mod, tmp_path, n, nn, np_, precision, damp_xy):
    """The damped step's slice kernels where only they fit in LDS with the
    in-place FFT exchange (48^3 FP64, 64^3 complex64), and the line passes,
    forced through the tuning cache, against the oracle (FP64 1e-11;
    complex64 inputs 2e-6)."""
    import torch
    from oracle import Grid
    from oracle import physics as ph
    from oracle import solver as so
    w = inputs.small_workload(f"n{n}_{nn}p{np_}", n, nn, np_, init="rod", seed=35, noise=0.05)
    raw = inputs.raw_states(w)
    box = _box(w, precision)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    prec = "mixed" if precision else "fp64"
    lines = box.tuning()["h_lines"]
    cache = tmp_path / "force.json"
    cache.write_text(json.dumps({f"h_lines/n{n}/{prec}": lines, f"damp_xy/n{n}/{prec}": damp_xy}))
    t = box.autotune(str(cache))
    assert t["damp_xy"] == damp_xy
    g = Grid(w.n, w.dx)
    cdt = torch.complex64 if precision else torch.complex128
    for s in range(2):
        box.view("psi", s).copy_(to_dev(raw[s]).to(cdt))
    box.densities()
    xs = [to_host(box.view("psi", s)).astype(np.complex128) for s in range(2)]
    dens = [ph.densities(xs[0], g), ph.densities(xs[1], g)]
    mf = ph.mean_field(dens[0], dens[1], g, w.params)[0]
    psi, hpsi, phi = box.view("psi", 0), box.view("hpsi", 0), box.view("phi", 0)
    eps = torch.empty(nn, dtype=torch.float64, device=psi.device)
    box.apply_h(0, psi, hpsi, nn, eps)
    # the step from the oracle's h psi rounded to the working precision
    x = xs[0]
    h_ref = ph.apply_h(x, mf, g)
    hpsi.copy_(to_dev(h_ref).to(cdt))
    hr = to_host(hpsi).astype(np.complex128)
    e_ref, r_ref, _ = so.rayleigh_and_residual(x, hr, g)
    eps.copy_(to_dev(e_ref))
    box.damped_step(0, psi, hpsi, eps, phi, nn)
    torch.cuda.synchronize()
    phi_ref = x - so.damping(r_ref, g, mf.hb2m, w.damp_x0, w.damp_e0)
    assert rel_err(to_host(phi), phi_ref) <= (2e-6 if precision else 1e-11)


@pytest.mark.parametrize("case", ["n32_70p33_slab", "n24_200p50_rod"])
def test_plane_product_wave_layouts(torch_mod, tmp_path, case):
    """The split-FP16 overlap and recombination in both wave layouts of a
    128 x 128 tile (8 waves of 32 x 64, 4 waves of 64 x 64), forced through
    the tuning cache: the overlap against the oracle's overlap of the same
    complex64 states (1e-6), the Rayleigh-Ritz combination against the
    oracle's combination with the same U (1e-6), and the energies of three
    iterations of the two layouts against each other (the other launch
    shapes the tuner times may differ between the two boxes, and raw states
    depend on eigenvector phases, so only span-invariant results are
    compared)."""
    import torch
    from oracle import Grid
    from oracle import solver as so
    from paper_1610_07522_amd import sky
    w = CASES[case]
    raw = inputs.raw_states(w)
    g = Grid(w.n, w.dx)
    outs = {}
    for waves in (8, 4):
        box = _box(w, sky.SKY_MIXED)
        box.init_box(to_dev(raw[0]), to_dev(raw[1]))
        cache = tmp_path / f"w{waves}.json"
        keys = {}
        for q, m in ((0, w.n_neutrons), (1, w.n_protons)):
            keys[f"plane_waves_overlap/m{m}/k{2 * w.n ** 3}"] = waves
            keys[f"plane_waves_combine/m{m}/k{2 * w.n ** 3}"] = waves
        cache.write_text(json.dumps(keys))
        t = box.autotune(str(cache))
        assert t["overlap_waves"] == [waves, waves] and t["combine_waves"] == [waves, waves]
        box.init_box(to_dev(raw[0]), to_dev(raw[1]))
        psi, hpsi = box.view("psi", 0), box.view("hpsi", 0)
        m = psi.shape[0]
        box.apply_h(0, psi, hpsi, m)
        out = torch.empty_like(psi)
        box.orthonormalize(0, psi, hpsi, out)
        box.sync()
        P = to_host(psi).astype(np.complex128)
        I_ref = so.overlap(P, P, g)
        I_gpu = to_host(box.view("overlap", 0))
        assert rel_err(I_gpu, I_ref) <= 1e-6, (waves, "overlap")
        U = to_host(box.view("umat", 0))
        assert rel_err(to_host(out), so.combine(P, U)) <= 1e-6, (waves, "combine")
        rep = box.iterate(3)
        outs[waves] = rep["energy"]
    assert abs(outs[4] - outs[8]) <= 2e-6 * abs(outs[8])


def test_ladder_switch_takes_the_cached_fp64_shapes(torch_mod, tmp_path):
    """A mixed box tuned against a cache that also holds the box's FP64
    entries runs the precision ladder's FP64 iterations with those shapes."""
    from paper_1610_07522_amd import sky
    w = CASES["n32_70p33_slab"]
    raw = inputs.raw_states(w)
    cache = tmp_path / "tune.json"
    b64 = _box(w, 0)
    b64.init_box(to_dev(raw[0]), to_dev(raw[1]))
    t64 = b64.autotune(str(cache))
    mixed = sky.Box(sky.desc_from_workload(w, precision=sky.SKY_MIXED, ladder_tol=10.0))
    mixed.init_box(to_dev(raw[0]), to_dev(raw[1]))
    tm = mixed.autotune(str(cache))
    assert not tm["from_cache"]   # the mixed shapes were timed
    rep = mixed.iterate(2)
    assert rep["precision"] == 0   # the ladder switched to FP64
    t = mixed.tuning()
    for key in ("h_lines", "damp_xy", "overlap_split"):
        assert t[key] == t64[key], (key, t[key], t64[key])
