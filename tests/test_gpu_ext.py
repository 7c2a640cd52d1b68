"""HIP library vs FP64 oracle for the optional iteration forms, state I/O and
error paths, through the C ABI.

* occupations with extra (v^2 = 0) states (Sec. 2.1);
* twist-averaged boundary conditions (Sec. 1): h psi and the damped step
  under a twist element by element, trajectories of several twists sharing
  one mean field;
* the paper-literal combined update (Sec. 3.3.3) and one h application per
  iteration (Sec. 3.4, hampsi);
* checkpoint and resume (Fig. 1 step 6): the resumed FP64 trajectory is the
  uninterrupted one bit for bit;
* loading a trained network into another context;
* a NaN in the states and a duplicated state end with the documented errors.

FP64 bar as in the other parity tests: 1e-10 relative on energies, fields and
eigenvalues, 1e-11 of the max-norm on h psi and the damped step.
"""
import numpy as np
import pytest

from oracle import Grid
from oracle import physics as ph
from oracle import solver as so
from paper_1610_07522_amd import inputs

from gpu_util import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-10
TWISTS = [(0.5, -1.3, 2.1), (-2.4, 0.8, -0.3), (1.7, 1.7, -2.9)]

EXTRA_CASES = {
    # 16^3, 8 + 8 nucleons carried by 12 + 10 states
    "n16_8p8_x4x2": inputs.small_workload("x16", 16, 8, 8, seed=41, noise=0.1,
                                         extra_n=4, extra_p=2),
    # 24^3 rod, ragged counts, extras not a multiple of any tile
    "n24_13p7_rod_x5x3": inputs.small_workload("x24", 24, 13, 7, init="rod", seed=42,
                                              noise=0.05, extra_n=5, extra_p=3),
}


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _box(w, stream=None, **kw):
    from paper_1610_07522_amd import sky
    return sky.Box(sky.desc_from_workload(w, **kw), stream=stream)


def _compare_iterate(box, st, w, iters, tag, ritz_sets=None):
    g = Grid(w.n, w.dx)
    done = 0
    for target in iters:
        rep_o = None
        for _ in range(target - done):
            rep_o = so.iterate(st)
        rep = box.iterate(target - done)
        done = target
        E = st.E["total"]
        assert abs(rep["energy"] - E) <= TOL * max(1.0, abs(E)), (tag, target, rep["energy"], E)
        assert abs(rep["residual"] - rep_o.de) <= 1e-8 * max(1.0, rep_o.de), (tag, target)
        for q in range(2):
            gd = to_host(box.view("dens", q))
            assert rel_err(gd[0], st.dens[q].rho) <= TOL, (tag, target, q)
            assert rel_err(gd[1], st.dens[q].tau) <= TOL, (tag, target, q)
            assert rel_err(gd[2:5], st.dens[q].J) <= 1e-9, (tag, target, q)
        for s in (ritz_sets if ritz_sets is not None else range(len(st.psi))):
            if st.psi[s].shape[0]:
                assert rel_err(to_host(box.view("ritz", s)), rep_o.ritz[s]) <= TOL, (tag, target, s)
    del g


# ------------------------------------------------------------ extra states
@pytest.mark.parametrize("case", list(EXTRA_CASES))
def test_extra_states_trajectory(torch_mod, case):
    """Occupied + extra states: energy, densities of the occupied states,
    Delta-eps over the occupied states and the Ritz values of every state
    follow the oracle's trajectory."""
    w = EXTRA_CASES[case]
    raw = inputs.raw_states(w)
    assert raw[0].shape[0] == w.n_neutrons + w.extra_n
    g = Grid(w.n, w.dx)
    st = so.initial_state(*raw, g, w.params, w.damp_x0, w.damp_e0,
                          nocc=(w.n_neutrons, w.n_protons))
    box = _box(w)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    ge = to_host(box.view("energy"))
    assert abs(ge[7] - st.E["total"]) <= TOL * max(1.0, abs(st.E["total"]))
    _compare_iterate(box, st, w, (1, 5, 20), case)
    for q, nq in enumerate((w.n_neutrons, w.n_protons)):
        rho = to_host(box.view("dens", q))[0]
        assert abs(rho.sum() * w.dx ** 3 - nq) <= 1e-10 * nq


def test_extra_states_mixed_tracks_oracle(torch_mod):
    """Mixed precision with extra states stays within FP32-level distance of
    the FP64 oracle (bars of the mixed-form tests)."""
    from paper_1610_07522_amd import sky
    w = EXTRA_CASES["n16_8p8_x4x2"]
    raw = inputs.raw_states(w)
    g = Grid(w.n, w.dx)
    st = so.initial_state(*raw, g, w.params, w.damp_x0, w.damp_e0, nocc=(8, 8))
    box = _box(w, precision=sky.SKY_MIXED)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    u32 = 2.0 ** -24
    for it in range(5):
        rep = box.iterate(1)
        ro = so.iterate(st)
        parts = sum(abs(st.E[k]) for k in ("kin", "rho", "rho3", "tau", "lap", "so", "coul"))
        assert abs(rep["energy"] - st.E["total"]) <= 1000 * u32 * parts * (it + 1), it
        assert abs(rep["residual"] - ro.de) <= 1e-4 * max(1.0, ro.de), it
        for q in range(2):
            assert rel_err(to_host(box.view("ritz", q)), ro.ritz[q]) <= 1e-5, (it, q)


# ------------------------------------------------------------ twists
def test_twisted_h_and_damped_step(torch_mod):
    """h psi, <psi|h psi>, ||r||^2 and the damped step under each twist
    (set 2 t + q), element by element against the oracle with the twisted
    grid."""
    torch = torch_mod
    w = inputs.small_workload("tw24", 24, 13, 7, init="rod", seed=43, noise=0.1)
    raw = inputs.raw_states(w)
    box = _box(w, twists=TWISTS)
    for s in range(2 * len(TWISTS)):
        box.view("psi", s).copy_(to_dev(raw[s % 2]))
    box.densities()
    g = Grid(w.n, w.dx)
    ds = []
    for q in range(2):
        ds.append(ph.average([ph.densities(raw[q], g.with_twist(t)) for t in TWISTS]))
    mn, mp, vc = ph.mean_field(ds[0], ds[1], g, w.params)
    mfs = [mn, mp]
    for q in range(2):
        gd = to_host(box.view("dens", q))
        assert rel_err(gd[0], ds[q].rho) <= TOL and rel_err(gd[1], ds[q].tau) <= TOL, q
        assert rel_err(gd[2:5], ds[q].J) <= 1e-9, q
        assert rel_err(gd[8:11], ds[q].j) <= 1e-9, q
    for s in range(2 * len(TWISTS)):
        q, gt = s % 2, g.with_twist(TWISTS[s // 2])
        m = raw[q].shape[0]
        psi, hpsi, phi = box.view("psi", s), box.view("hpsi", s), box.view("phi", s)
        eps = torch.zeros(m, dtype=torch.float64, device="cuda:0")
        r2 = torch.zeros(m, dtype=torch.float64, device="cuda:0")
        box.apply_h(s, psi, hpsi, m, eps)
        box.damped_step(s, psi, hpsi, eps, phi, m, r2)
        box.sync()
        h_ref = ph.apply_h(raw[q], mfs[q], gt)
        e_ref, r_ref, r2_ref = so.rayleigh_and_residual(raw[q], h_ref, gt)
        phi_ref = raw[q] - so.damping(r_ref, gt, mfs[q].hb2m, w.damp_x0, w.damp_e0)
        assert rel_err(to_host(hpsi), h_ref) <= 1e-11, s
        assert rel_err(to_host(eps), e_ref) <= TOL, s
        assert rel_err(to_host(r2), r2_ref) <= 1e-9, s
        assert rel_err(to_host(phi), phi_ref) <= 1e-11, s


@pytest.mark.parametrize("extra", [0, 3])
def test_twist_averaged_trajectory(torch_mod, extra):
    """Three twists sharing the mean field of the twist-averaged densities
    (with and without extra states): energy, averaged densities, Delta-eps
    and every set's Ritz values follow the oracle's trajectory."""
    w = inputs.small_workload("ta16", 16, 8, 6, init="slab", seed=44, noise=0.1,
                              extra_n=extra, extra_p=extra)
    raw = inputs.raw_states(w)
    g = Grid(w.n, w.dx)
    st = so.initial_state(*raw, g, w.params, w.damp_x0, w.damp_e0, twists=TWISTS,
                          nocc=(w.n_neutrons, w.n_protons))
    box = _box(w, twists=TWISTS)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    ge = to_host(box.view("energy"))
    assert abs(ge[7] - st.E["total"]) <= TOL * max(1.0, abs(st.E["total"]))
    _compare_iterate(box, st, w, (1, 4, 12), f"twist{extra}")


def test_twist_averaged_mixed_tracks_oracle(torch_mod):
    from paper_1610_07522_amd import sky
    w = inputs.small_workload("tm16", 16, 8, 6, init="slab", seed=44, noise=0.1)
    raw = inputs.raw_states(w)
    g = Grid(w.n, w.dx)
    st = so.initial_state(*raw, g, w.params, w.damp_x0, w.damp_e0, twists=TWISTS[:2])
    box = _box(w, twists=TWISTS[:2], precision=sky.SKY_MIXED)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    u32 = 2.0 ** -24
    for it in range(4):
        rep = box.iterate(1)
        ro = so.iterate(st)
        parts = sum(abs(st.E[k]) for k in ("kin", "rho", "rho3", "tau", "lap", "so", "coul"))
        assert abs(rep["energy"] - st.E["total"]) <= 1000 * u32 * parts * (it + 1), it
        for s in range(4):
            assert rel_err(to_host(box.view("ritz", s)), ro.ritz[s]) <= 1e-5, (it, s)


# ------------------------------------------------------------ update forms
@pytest.mark.parametrize("case", ["n16", "n24rod"])
def test_paper_update_trajectory(torch_mod, case):
    """Sec. 3.3.3 as printed (Z of H alone, C = I^-1/2 of I alone,
    psi = phi Z C, Z in its identity-closest gauge) against the oracle's
    same update, from noisy starts."""
    from paper_1610_07522_amd import sky
    w = (inputs.small_workload("pu16", 16, 8, 8, seed=45, noise=0.1) if case == "n16" else
         inputs.small_workload("pu24", 24, 13, 7, init="rod", seed=46, noise=0.05))
    raw = inputs.raw_states(w)
    g = Grid(w.n, w.dx)
    st = so.initial_state(*raw, g, w.params, w.damp_x0, w.damp_e0, rr="paper")
    box = _box(w, update=sky.SKY_UPDATE_PAPER)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    _compare_iterate(box, st, w, (1, 3, 8), "paper " + case)
    # the states are orthonormal only to O(||I - 1||): the update is approximate
    for q in range(2):
        p = to_host(box.view("psi", q))
        dev = np.abs(so.overlap(p, p, g) - np.eye(p.shape[0])).max()
        dev_o = np.abs(so.overlap(st.psi[q], st.psi[q], g) - np.eye(p.shape[0])).max()
        assert abs(dev - dev_o) <= 1e-9 + 1e-6 * dev_o, (q, dev, dev_o)


@pytest.mark.parametrize("prec", [0, 1])
def test_one_h_trajectory(torch_mod, prec):
    """One h application per iteration (h psi_new = (h phi) U, <psi|h psi>
    from the subspace eigenvalues) against the oracle's same form: FP64 at
    the FP64 bar, mixed at FP32-level bars."""
    from paper_1610_07522_amd import sky
    w = inputs.small_workload("oh16", 16, 8, 8, seed=47, noise=0.1)
    raw = inputs.raw_states(w)
    g = Grid(w.n, w.dx)
    st = so.initial_state(*raw, g, w.params, w.damp_x0, w.damp_e0, one_h=True)
    box = _box(w, one_h=True, precision=prec)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    if prec == 0:
        _compare_iterate(box, st, w, (1, 2, 6, 20), "one_h")
        # the carried h psi: its matrix with the states and its norm are
        # independent of the eigenvectors' phases (raw states are not)
        for q in range(2):
            p, hp = to_host(box.view("psi", q)), to_host(box.view("hpsi", q))
            M, M_ref = so.overlap(p, hp, g), so.overlap(st.psi[q], st.hpsi_lag[q], g)
            assert rel_err(M, M_ref) <= 1e-10, q
            n2 = so.overlap(hp, hp, g).trace().real
            n2_ref = so.overlap(st.hpsi_lag[q], st.hpsi_lag[q], g).trace().real
            assert abs(n2 - n2_ref) <= 1e-10 * n2_ref, q
        return
    u32 = 2.0 ** -24
    for it in range(6):
        rep = box.iterate(1)
        ro = so.iterate(st)
        parts = sum(abs(st.E[k]) for k in ("kin", "rho", "rho3", "tau", "lap", "so", "coul"))
        assert abs(rep["energy"] - st.E["total"]) <= 1000 * u32 * parts * (it + 1), it
        assert abs(rep["residual"] - ro.de) <= 1e-4 * max(1.0, ro.de), it


# ------------------------------------------------------------ checkpoint / resume
@pytest.mark.parametrize("graphs", [False, True])
def test_resume_reproduces_trajectory_bitwise(torch_mod, graphs):
    """Fig. 1 step 6 and back: states and iteration counter written after 6
    FP64 iterations and read into a fresh context, which rebuilds its mean
    field from them, continue exactly as the uninterrupted run (bitwise
    states and energy after 6 more iterations)."""
    torch = torch_mod
    w = inputs.small_workload("rs24", 24, 13, 7, init="rod", seed=48, noise=0.05,
                              extra_n=2, extra_p=1)
    raw = inputs.raw_states(w)
    a = _box(w, stream=torch.cuda.Stream() if graphs else None)
    a.init_box(to_dev(raw[0]), to_dev(raw[1]))
    if graphs:
        a.set_graphs(True)
    a.iterate(6)
    ckpt = []
    for q in range(2):
        t = torch.empty_like(a.view("psi", q))
        a.get_states(q, t)
        a.sync()
        ckpt.append(t.cpu())
    it6 = a.iteration()
    assert it6 == 6
    rep_a = a.iterate(6)
    b = _box(w, stream=torch.cuda.Stream() if graphs else None)
    b.init_box(to_dev(raw[0]), to_dev(raw[1]))     # any states: overwritten below
    if graphs:
        b.set_graphs(True)
    dev = [c.to("cuda:0") for c in ckpt]
    torch.cuda.synchronize()
    for q in range(2):
        b.set_states(q, dev[q])
    b.set_iteration(it6)
    b.densities()
    rep_b = b.iterate(6)
    assert b.iteration() == 12
    assert rep_b["energy"] == rep_a["energy"], (rep_a, rep_b)
    assert rep_b["residual"] == rep_a["residual"]
    for q in range(2):
        assert torch.equal(a.view("psi", q), b.view("psi", q)), q
        assert torch.equal(a.view("dens", q), b.view("dens", q)), q


def test_state_io_precision_conversion(torch_mod):
    """sky_get_states / sky_set_states round a complex128 context's states to
    complex64 and widen them back exactly as complex64 -> complex128."""
    torch = torch_mod
    w = inputs.small_workload("io8", 8, 5, 3, init="slab", seed=49, noise=0.2)
    raw = inputs.raw_states(w)
    a = _box(w)
    a.init_box(to_dev(raw[0]), to_dev(raw[1]))
    lo = torch.empty(a.view("psi", 0).shape, dtype=torch.complex64, device="cuda:0")
    a.get_states(0, lo)
    a.sync()
    assert torch.equal(lo, a.view("psi", 0).to(torch.complex64))
    a.set_states(0, lo)
    a.sync()
    assert torch.equal(a.view("psi", 0), lo.to(torch.complex128))


# ------------------------------------------------------------ preconditioner hand-off
def test_set_preconditioner_carries_a_network(torch_mod):
    """A network trained in one context and loaded into another
    (sky_set_preconditioner) gives the same learned step there: same gains
    and the same energy after one learned iteration from the same states."""
    torch = torch_mod
    w = inputs.small_workload("pc24", 24, 13, 7, init="rod", seed=50, noise=0.05)
    raw = inputs.raw_states(w)
    a = _box(w)
    a.init_box(to_dev(raw[0]), to_dev(raw[1]))
    a.iterate(3)
    for q in range(2):
        a.precond_collect(q)
    a.precond_train(30, 1e-3)
    params = a.view("pc_params").clone()
    b = _box(w)
    b.init_box(to_dev(raw[0]), to_dev(raw[1]))
    with pytest.raises(Exception):
        b.precond_use(True)                    # untrained
    b.set_preconditioner(params)
    assert torch.equal(b.view("pc_params"), params)
    for q in range(2):
        st = torch.empty_like(a.view("psi", q))
        a.get_states(q, st)
        b.set_states(q, st)
    b.set_iteration(a.iteration())
    b.densities()
    a.precond_use(True, rise_tol=-1.0)
    b.precond_use(True, rise_tol=-1.0)
    ra, rb = a.iterate(1), b.iterate(1)
    assert ra["precond_iters"] == 1 and rb["precond_iters"] == 1
    assert torch.equal(a.view("pc_gains", 0), b.view("pc_gains", 0))
    assert rb["energy"] == pytest.approx(ra["energy"], rel=1e-12)


# ------------------------------------------------------------ error paths
def test_nan_in_states_reports_nan(torch_mod):
    """A NaN in one state: sky_iterate stops with SKY_ERR_NAN (the overlap
    norm is checked on the host before any eigensolver loop)."""
    from paper_1610_07522_amd import sky
    w = inputs.small_workload("nan8", 8, 5, 3, init="slab", seed=51, noise=0.2)
    raw = inputs.raw_states(w)
    box = _box(w)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    bad = raw[0].copy()
    bad[2, 0, 3, 4, 5] = np.nan
    box.set_states(0, to_dev(bad))
    with pytest.raises(sky.SkyError) as e:
        box.iterate(1)
    assert e.value.code == sky.SKY_ERR_NAN


def test_duplicated_state_reports_not_positive_definite(torch_mod):
    """Two equal states make the overlap singular: the Cholesky pivot floor
    reports SKY_ERR_NOT_POSITIVE_DEFINITE."""
    from paper_1610_07522_amd import sky
    w = inputs.small_workload("dup8", 8, 5, 3, init="slab", seed=52, noise=0.2)
    raw = inputs.raw_states(w)
    box = _box(w)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    psi = box.view("psi", 0).clone()
    psi[1] = psi[0]
    box.set_states(0, psi)
    box.densities()
    with pytest.raises(sky.SkyError) as e:
        box.iterate(1)
    assert e.value.code == sky.SKY_ERR_NOT_POSITIVE_DEFINITE
    # a duplicated trial state at initialisation is reported the same way
    raw_dup = raw[0].copy()
    raw_dup[1] = raw_dup[0]
    box2 = _box(w)
    with pytest.raises(sky.SkyError) as e2:
        box2.init_box(to_dev(raw_dup), to_dev(raw[1]))
    assert e2.value.code == sky.SKY_ERR_NOT_POSITIVE_DEFINITE
