"""Edge cases of the iteration against the FP64 oracle: an empty species
(pure neutron matter), one state per species, the largest grid (64^3) and
a grid spacing other than 1 fm (0.5 fm).
FP64 bar: 1e-10 relative on the energy, 1e-8 on Delta-eps; the mixed form
within 2e-5 relative of the FP64 oracle's energy after one iteration
(complex64 states, FP32 h psi)."""
import numpy as np
import pytest

from oracle import Grid
from oracle import solver as so
from paper_1610_07522_amd import inputs

from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


EDGE = {
    "empty_protons_n16": inputs.small_workload("e0", 16, 10, 0, init="slab", seed=4, noise=0.05),
    "empty_neutrons_n16": inputs.small_workload("e1", 16, 0, 7, init="rod", seed=6, noise=0.05),
    "one_state_each_n8": inputs.small_workload("e2", 8, 1, 1, init="slab", seed=7, noise=0.1),
    "largest_grid_n64": inputs.small_workload("e3", 64, 4, 2, init="rod", seed=5, noise=0.05),
    "half_fm_spacing_n16": inputs.small_workload("e4", 16, 6, 4, init="slab", seed=8, noise=0.05,
                                                 dx=0.5),
}


def _run(w, precision, iters):
    from paper_1610_07522_amd import sky
    raw = inputs.raw_states(w)
    box = sky.Box(sky.desc_from_workload(w, precision=precision))
    box.init_box(to_dev(raw[0]) if raw[0].shape[0] else None,
                 to_dev(raw[1]) if raw[1].shape[0] else None)
    rep = box.iterate(iters)
    st = so.initial_state(raw[0], raw[1], Grid(w.n, w.dx), w.params, w.damp_x0, w.damp_e0)
    for _ in range(iters):
        ro = so.iterate(st)
    return box, rep, st, ro


@pytest.mark.parametrize("case", list(EDGE))
def test_edge_trajectory_fp64(torch_mod, case):
    w = EDGE[case]
    iters = 1 if w.n == 64 else 3
    box, rep, st, ro = _run(w, 0, iters)
    assert rep["energy"] == pytest.approx(st.E["total"], rel=1e-10, abs=1e-9), case
    assert rep["residual"] == pytest.approx(ro.de, rel=1e-8), case
    # orthonormal states of each non-empty species
    for q in range(2):
        if (w.n_neutrons, w.n_protons)[q] == 0:
            continue
        psi = to_host(box.view("psi", q)).reshape((w.n_neutrons, w.n_protons)[q], -1)
        ov = (psi.conj() @ psi.T) * w.dx ** 3
        assert np.abs(ov - np.eye(ov.shape[0])).max() <= 1e-12


@pytest.mark.parametrize("case", ["empty_protons_n16", "largest_grid_n64", "half_fm_spacing_n16"])
def test_edge_mixed(torch_mod, case):
    w = EDGE[case]
    box, rep, st, ro = _run(w, 1, 1)
    assert rep["energy"] == pytest.approx(st.E["total"], rel=2e-5), case


def test_empty_species_learned_and_batched(torch_mod):
    """The learned step and the batched driver with an empty species."""
    from paper_1610_07522_amd import sky
    w = EDGE["empty_protons_n16"]
    raw = inputs.raw_states(w)
    box = sky.Box(sky.desc_from_workload(w))
    box.init_box(to_dev(raw[0]), None)
    box.iterate(2)
    assert box.precond_collect(0) == 10 * 8
    assert box.precond_collect(1) == 10 * 8   # nothing to collect from an empty species
    box.precond_train(10, 1e-3)
    box.precond_use(True, -1.0, 0)
    r = box.iterate(2)
    assert r["precond_iters"] == 2 and np.isfinite(r["energy"])
    other = sky.Box(sky.desc_from_workload(EDGE["empty_neutrons_n16"]))
    raw1 = inputs.raw_states(EDGE["empty_neutrons_n16"])
    other.init_box(None, to_dev(raw1[1]))
    reps = sky.batch_iterate([box, other], 2, 2)
    assert all(np.isfinite(x["energy"]) and x["iters"] == 2 for x in reps)
