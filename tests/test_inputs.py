"""Host checks of the workload descriptions (no GPU, no solver arithmetic):
the saturation-density boxes hold closed plane-wave shells at the stated
density, and the 24^3 and 48^3 versions describe the same physical box."""
import numpy as np
import pytest

from paper_1610_07522_amd import inputs


@pytest.mark.parametrize("name,shell", [("sat24", 25), ("sat48", 25), ("sat8", 2)])
def test_saturation_boxes_are_closed_shells(name, shell):
    w = inputs.WORKLOADS[name]
    L = w.n * w.dx
    assert w.n_neutrons == w.n_protons
    assert 0.14 <= (w.n_neutrons + w.n_protons) / L ** 3 <= 0.16
    lab = inputs.plane_wave_labels(w.n, w.n_neutrons)
    n2 = (lab[:, :3] ** 2).sum(axis=1)
    # every plane wave with |n|^2 <= shell, both spins, and nothing beyond
    assert n2.max() == shell
    half = w.n // 2
    r = np.arange(-half, half)
    all_n2 = (r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2).ravel()
    assert w.n_neutrons == 2 * int((all_n2 <= shell).sum())


def test_sat48_is_sat24_on_a_finer_grid():
    a, b = inputs.WORKLOADS["sat24"], inputs.WORKLOADS["sat48"]
    assert a.n * a.dx == b.n * b.dx
    assert (a.n_neutrons, a.n_protons, a.init, a.seed, a.amp, a.noise) == \
        (b.n_neutrons, b.n_protons, b.init, b.seed, b.amp, b.noise)
    assert np.array_equal(inputs.plane_wave_labels(a.n, a.n_neutrons),
                          inputs.plane_wave_labels(b.n, b.n_neutrons))


def test_small_workload_spacing():
    w = inputs.small_workload("t", 16, 6, 4, init="slab", seed=8, noise=0.05, dx=0.5)
    assert w.dx == 0.5 and w.n == 16 and w.n_states == 10
